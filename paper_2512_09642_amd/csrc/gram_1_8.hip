// Gram and FGS kernels (single-system and batched) for basis widths s = 1..8
// (see gram_impl.h, fgs_core.h, batched_impl.h).
#include "batched_impl.h"

namespace sstep {

hipError_t gram_launch_1_8(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 1:
        return a.fp32 ? gram_launch_s<float, 1>(a, st) : gram_launch_s<double, 1>(a, st);
    case 2:
        return a.fp32 ? gram_launch_s<float, 2>(a, st) : gram_launch_s<double, 2>(a, st);
    case 3:
        return a.fp32 ? gram_launch_s<float, 3>(a, st) : gram_launch_s<double, 3>(a, st);
    case 4:
        return a.fp32 ? gram_launch_s<float, 4>(a, st) : gram_launch_s<double, 4>(a, st);
    case 5:
        return a.fp32 ? gram_launch_s<float, 5>(a, st) : gram_launch_s<double, 5>(a, st);
    case 6:
        return a.fp32 ? gram_launch_s<float, 6>(a, st) : gram_launch_s<double, 6>(a, st);
    case 7:
        return a.fp32 ? gram_launch_s<float, 7>(a, st) : gram_launch_s<double, 7>(a, st);
    case 8:
        return a.fp32 ? gram_launch_s<float, 8>(a, st) : gram_launch_s<double, 8>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t fgs_launch_1_8(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 1:
        return fgs_launch_s<1>(a, st);
    case 2:
        return fgs_launch_s<2>(a, st);
    case 3:
        return fgs_launch_s<3>(a, st);
    case 4:
        return fgs_launch_s<4>(a, st);
    case 5:
        return fgs_launch_s<5>(a, st);
    case 6:
        return fgs_launch_s<6>(a, st);
    case 7:
        return fgs_launch_s<7>(a, st);
    case 8:
        return fgs_launch_s<8>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bgram_launch_1_8(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 1:
        return a.fp32 ? bgram_launch_s<float, 1>(a, st) : bgram_launch_s<double, 1>(a, st);
    case 2:
        return a.fp32 ? bgram_launch_s<float, 2>(a, st) : bgram_launch_s<double, 2>(a, st);
    case 3:
        return a.fp32 ? bgram_launch_s<float, 3>(a, st) : bgram_launch_s<double, 3>(a, st);
    case 4:
        return a.fp32 ? bgram_launch_s<float, 4>(a, st) : bgram_launch_s<double, 4>(a, st);
    case 5:
        return a.fp32 ? bgram_launch_s<float, 5>(a, st) : bgram_launch_s<double, 5>(a, st);
    case 6:
        return a.fp32 ? bgram_launch_s<float, 6>(a, st) : bgram_launch_s<double, 6>(a, st);
    case 7:
        return a.fp32 ? bgram_launch_s<float, 7>(a, st) : bgram_launch_s<double, 7>(a, st);
    case 8:
        return a.fp32 ? bgram_launch_s<float, 8>(a, st) : bgram_launch_s<double, 8>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bfgs_launch_1_8(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 1:
        return bfgs_launch_s<1>(a, st);
    case 2:
        return bfgs_launch_s<2>(a, st);
    case 3:
        return bfgs_launch_s<3>(a, st);
    case 4:
        return bfgs_launch_s<4>(a, st);
    case 5:
        return bfgs_launch_s<5>(a, st);
    case 6:
        return bfgs_launch_s<6>(a, st);
    case 7:
        return bfgs_launch_s<7>(a, st);
    case 8:
        return bfgs_launch_s<8>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace sstep
