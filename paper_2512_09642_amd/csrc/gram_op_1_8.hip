// Gram kernels that apply the stencil operator on the fly, basis widths
// s = 1..8 (see gram_op_impl.h).
#include "gram_op_impl.h"

namespace sstep {

hipError_t gram_op_launch_1_8(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 1:
        return a.fp32 ? gram_op_launch_s<float, 1>(a, st) : gram_op_launch_s<double, 1>(a, st);
    case 2:
        return a.fp32 ? gram_op_launch_s<float, 2>(a, st) : gram_op_launch_s<double, 2>(a, st);
    case 3:
        return a.fp32 ? gram_op_launch_s<float, 3>(a, st) : gram_op_launch_s<double, 3>(a, st);
    case 4:
        return a.fp32 ? gram_op_launch_s<float, 4>(a, st) : gram_op_launch_s<double, 4>(a, st);
    case 5:
        return a.fp32 ? gram_op_launch_s<float, 5>(a, st) : gram_op_launch_s<double, 5>(a, st);
    case 6:
        return a.fp32 ? gram_op_launch_s<float, 6>(a, st) : gram_op_launch_s<double, 6>(a, st);
    case 7:
        return a.fp32 ? gram_op_launch_s<float, 7>(a, st) : gram_op_launch_s<double, 7>(a, st);
    case 8:
        return a.fp32 ? gram_op_launch_s<float, 8>(a, st) : gram_op_launch_s<double, 8>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace sstep
