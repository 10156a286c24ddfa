// Gram and FGS kernels (single-system and batched) for basis widths s = 25..32
// (see gram_impl.h, fgs_core.h, batched_impl.h).
#include "batched_impl.h"

namespace sstep {

hipError_t gram_launch_25_32(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 25:
        return a.fp32 ? gram_launch_s<float, 25>(a, st) : gram_launch_s<double, 25>(a, st);
    case 26:
        return a.fp32 ? gram_launch_s<float, 26>(a, st) : gram_launch_s<double, 26>(a, st);
    case 27:
        return a.fp32 ? gram_launch_s<float, 27>(a, st) : gram_launch_s<double, 27>(a, st);
    case 28:
        return a.fp32 ? gram_launch_s<float, 28>(a, st) : gram_launch_s<double, 28>(a, st);
    case 29:
        return a.fp32 ? gram_launch_s<float, 29>(a, st) : gram_launch_s<double, 29>(a, st);
    case 30:
        return a.fp32 ? gram_launch_s<float, 30>(a, st) : gram_launch_s<double, 30>(a, st);
    case 31:
        return a.fp32 ? gram_launch_s<float, 31>(a, st) : gram_launch_s<double, 31>(a, st);
    case 32:
        return a.fp32 ? gram_launch_s<float, 32>(a, st) : gram_launch_s<double, 32>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t fgs_launch_25_32(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 25:
        return fgs_launch_s<25>(a, st);
    case 26:
        return fgs_launch_s<26>(a, st);
    case 27:
        return fgs_launch_s<27>(a, st);
    case 28:
        return fgs_launch_s<28>(a, st);
    case 29:
        return fgs_launch_s<29>(a, st);
    case 30:
        return fgs_launch_s<30>(a, st);
    case 31:
        return fgs_launch_s<31>(a, st);
    case 32:
        return fgs_launch_s<32>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bgram_launch_25_32(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 25:
        return a.fp32 ? bgram_launch_s<float, 25>(a, st) : bgram_launch_s<double, 25>(a, st);
    case 26:
        return a.fp32 ? bgram_launch_s<float, 26>(a, st) : bgram_launch_s<double, 26>(a, st);
    case 27:
        return a.fp32 ? bgram_launch_s<float, 27>(a, st) : bgram_launch_s<double, 27>(a, st);
    case 28:
        return a.fp32 ? bgram_launch_s<float, 28>(a, st) : bgram_launch_s<double, 28>(a, st);
    case 29:
        return a.fp32 ? bgram_launch_s<float, 29>(a, st) : bgram_launch_s<double, 29>(a, st);
    case 30:
        return a.fp32 ? bgram_launch_s<float, 30>(a, st) : bgram_launch_s<double, 30>(a, st);
    case 31:
        return a.fp32 ? bgram_launch_s<float, 31>(a, st) : bgram_launch_s<double, 31>(a, st);
    case 32:
        return a.fp32 ? bgram_launch_s<float, 32>(a, st) : bgram_launch_s<double, 32>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bfgs_launch_25_32(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 25:
        return bfgs_launch_s<25>(a, st);
    case 26:
        return bfgs_launch_s<26>(a, st);
    case 27:
        return bfgs_launch_s<27>(a, st);
    case 28:
        return bfgs_launch_s<28>(a, st);
    case 29:
        return bfgs_launch_s<29>(a, st);
    case 30:
        return bfgs_launch_s<30>(a, st);
    case 31:
        return bfgs_launch_s<31>(a, st);
    case 32:
        return bfgs_launch_s<32>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace sstep
