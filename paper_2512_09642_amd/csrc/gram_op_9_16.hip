// Gram kernels that apply the stencil operator on the fly, basis widths
// s = 9..16 (see gram_op_impl.h).
#include "gram_op_impl.h"

namespace sstep {

hipError_t gram_op_launch_9_16(const IterArgs &a, hipStream_t st)
{
    switch (a.s) {
    case 9:
        return a.fp32 ? gram_op_launch_s<float, 9>(a, st) : gram_op_launch_s<double, 9>(a, st);
    case 10:
        return a.fp32 ? gram_op_launch_s<float, 10>(a, st) : gram_op_launch_s<double, 10>(a, st);
    case 11:
        return a.fp32 ? gram_op_launch_s<float, 11>(a, st) : gram_op_launch_s<double, 11>(a, st);
    case 12:
        return a.fp32 ? gram_op_launch_s<float, 12>(a, st) : gram_op_launch_s<double, 12>(a, st);
    case 13:
        return a.fp32 ? gram_op_launch_s<float, 13>(a, st) : gram_op_launch_s<double, 13>(a, st);
    case 14:
        return a.fp32 ? gram_op_launch_s<float, 14>(a, st) : gram_op_launch_s<double, 14>(a, st);
    case 15:
        return a.fp32 ? gram_op_launch_s<float, 15>(a, st) : gram_op_launch_s<double, 15>(a, st);
    case 16:
        return a.fp32 ? gram_op_launch_s<float, 16>(a, st) : gram_op_launch_s<double, 16>(a, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace sstep
