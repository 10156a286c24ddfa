// Gram and FGS kernels (single-system and batched) for basis widths s = 9..16
// (see gram_impl.h, fgs_core.h, batched_impl.h).
#include "batched_impl.h"

namespace sstep {

hipError_t gram_launch_9_16(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 9:
        return a.fp32 ? gram_launch_s<float, 9>(a, st) : gram_launch_s<double, 9>(a, st);
    case 10:
        return a.fp32 ? gram_launch_s<float, 10>(a, st) : gram_launch_s<double, 10>(a, st);
    case 11:
        return a.fp32 ? gram_launch_s<float, 11>(a, st) : gram_launch_s<double, 11>(a, st);
    case 12:
        return a.fp32 ? gram_launch_s<float, 12>(a, st) : gram_launch_s<double, 12>(a, st);
    case 13:
        return a.fp32 ? gram_launch_s<float, 13>(a, st) : gram_launch_s<double, 13>(a, st);
    case 14:
        return a.fp32 ? gram_launch_s<float, 14>(a, st) : gram_launch_s<double, 14>(a, st);
    case 15:
        return a.fp32 ? gram_launch_s<float, 15>(a, st) : gram_launch_s<double, 15>(a, st);
    case 16:
        return a.fp32 ? gram_launch_s<float, 16>(a, st) : gram_launch_s<double, 16>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t fgs_launch_9_16(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 9:
        return fgs_launch_s<9>(a, st);
    case 10:
        return fgs_launch_s<10>(a, st);
    case 11:
        return fgs_launch_s<11>(a, st);
    case 12:
        return fgs_launch_s<12>(a, st);
    case 13:
        return fgs_launch_s<13>(a, st);
    case 14:
        return fgs_launch_s<14>(a, st);
    case 15:
        return fgs_launch_s<15>(a, st);
    case 16:
        return fgs_launch_s<16>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bgram_launch_9_16(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 9:
        return a.fp32 ? bgram_launch_s<float, 9>(a, st) : bgram_launch_s<double, 9>(a, st);
    case 10:
        return a.fp32 ? bgram_launch_s<float, 10>(a, st) : bgram_launch_s<double, 10>(a, st);
    case 11:
        return a.fp32 ? bgram_launch_s<float, 11>(a, st) : bgram_launch_s<double, 11>(a, st);
    case 12:
        return a.fp32 ? bgram_launch_s<float, 12>(a, st) : bgram_launch_s<double, 12>(a, st);
    case 13:
        return a.fp32 ? bgram_launch_s<float, 13>(a, st) : bgram_launch_s<double, 13>(a, st);
    case 14:
        return a.fp32 ? bgram_launch_s<float, 14>(a, st) : bgram_launch_s<double, 14>(a, st);
    case 15:
        return a.fp32 ? bgram_launch_s<float, 15>(a, st) : bgram_launch_s<double, 15>(a, st);
    case 16:
        return a.fp32 ? bgram_launch_s<float, 16>(a, st) : bgram_launch_s<double, 16>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bfgs_launch_9_16(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 9:
        return bfgs_launch_s<9>(a, st);
    case 10:
        return bfgs_launch_s<10>(a, st);
    case 11:
        return bfgs_launch_s<11>(a, st);
    case 12:
        return bfgs_launch_s<12>(a, st);
    case 13:
        return bfgs_launch_s<13>(a, st);
    case 14:
        return bfgs_launch_s<14>(a, st);
    case 15:
        return bfgs_launch_s<15>(a, st);
    case 16:
        return bfgs_launch_s<16>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace sstep
