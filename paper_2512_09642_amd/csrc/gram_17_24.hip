// Gram and FGS kernels (single-system and batched) for basis widths s = 17..24
// (see gram_impl.h, fgs_core.h, batched_impl.h).
#include "batched_impl.h"

namespace sstep {

hipError_t gram_launch_17_24(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 17:
        return a.fp32 ? gram_launch_s<float, 17>(a, st) : gram_launch_s<double, 17>(a, st);
    case 18:
        return a.fp32 ? gram_launch_s<float, 18>(a, st) : gram_launch_s<double, 18>(a, st);
    case 19:
        return a.fp32 ? gram_launch_s<float, 19>(a, st) : gram_launch_s<double, 19>(a, st);
    case 20:
        return a.fp32 ? gram_launch_s<float, 20>(a, st) : gram_launch_s<double, 20>(a, st);
    case 21:
        return a.fp32 ? gram_launch_s<float, 21>(a, st) : gram_launch_s<double, 21>(a, st);
    case 22:
        return a.fp32 ? gram_launch_s<float, 22>(a, st) : gram_launch_s<double, 22>(a, st);
    case 23:
        return a.fp32 ? gram_launch_s<float, 23>(a, st) : gram_launch_s<double, 23>(a, st);
    case 24:
        return a.fp32 ? gram_launch_s<float, 24>(a, st) : gram_launch_s<double, 24>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t fgs_launch_17_24(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 17:
        return fgs_launch_s<17>(a, st);
    case 18:
        return fgs_launch_s<18>(a, st);
    case 19:
        return fgs_launch_s<19>(a, st);
    case 20:
        return fgs_launch_s<20>(a, st);
    case 21:
        return fgs_launch_s<21>(a, st);
    case 22:
        return fgs_launch_s<22>(a, st);
    case 23:
        return fgs_launch_s<23>(a, st);
    case 24:
        return fgs_launch_s<24>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bgram_launch_17_24(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 17:
        return a.fp32 ? bgram_launch_s<float, 17>(a, st) : bgram_launch_s<double, 17>(a, st);
    case 18:
        return a.fp32 ? bgram_launch_s<float, 18>(a, st) : bgram_launch_s<double, 18>(a, st);
    case 19:
        return a.fp32 ? bgram_launch_s<float, 19>(a, st) : bgram_launch_s<double, 19>(a, st);
    case 20:
        return a.fp32 ? bgram_launch_s<float, 20>(a, st) : bgram_launch_s<double, 20>(a, st);
    case 21:
        return a.fp32 ? bgram_launch_s<float, 21>(a, st) : bgram_launch_s<double, 21>(a, st);
    case 22:
        return a.fp32 ? bgram_launch_s<float, 22>(a, st) : bgram_launch_s<double, 22>(a, st);
    case 23:
        return a.fp32 ? bgram_launch_s<float, 23>(a, st) : bgram_launch_s<double, 23>(a, st);
    case 24:
        return a.fp32 ? bgram_launch_s<float, 24>(a, st) : bgram_launch_s<double, 24>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t bfgs_launch_17_24(const BatchArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 17:
        return bfgs_launch_s<17>(a, st);
    case 18:
        return bfgs_launch_s<18>(a, st);
    case 19:
        return bfgs_launch_s<19>(a, st);
    case 20:
        return bfgs_launch_s<20>(a, st);
    case 21:
        return bfgs_launch_s<21>(a, st);
    case 22:
        return bfgs_launch_s<22>(a, st);
    case 23:
        return bfgs_launch_s<23>(a, st);
    case 24:
        return bfgs_launch_s<24>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace sstep
