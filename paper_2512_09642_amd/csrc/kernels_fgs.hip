// Dispatch of the Gram and FGS launches to the translation unit that holds
// the instantiation for the basis width s.
#include "batched_impl.h"
#include "gram_op_impl.h"

namespace sstep {

hipError_t launch_gram(const IterArgs &a, hipStream_t st)
{
    if (a.gram_op)
        return a.s <= 8 ? gram_op_launch_1_8(a, st) : gram_op_launch_9_16(a, st);
    if (a.s <= 8)
        return gram_launch_1_8(a, st);
    if (a.s <= 16)
        return gram_launch_9_16(a, st);
    if (a.s <= 24)
        return gram_launch_17_24(a, st);
    return gram_launch_25_32(a, st);
}

hipError_t launch_fgs(const IterArgs &a, hipStream_t st)
{
    if (a.s <= 8)
        return fgs_launch_1_8(a, st);
    if (a.s <= 16)
        return fgs_launch_9_16(a, st);
    if (a.s <= 24)
        return fgs_launch_17_24(a, st);
    return fgs_launch_25_32(a, st);
}

hipError_t launch_bgram(const BatchArgs &a, hipStream_t st)
{
    if (a.s <= 8)
        return bgram_launch_1_8(a, st);
    if (a.s <= 16)
        return bgram_launch_9_16(a, st);
    if (a.s <= 24)
        return bgram_launch_17_24(a, st);
    return bgram_launch_25_32(a, st);
}

hipError_t launch_bfgs(const BatchArgs &a, hipStream_t st)
{
    if (a.s <= 8)
        return bfgs_launch_1_8(a, st);
    if (a.s <= 16)
        return bfgs_launch_9_16(a, st);
    if (a.s <= 24)
        return bfgs_launch_17_24(a, st);
    return bfgs_launch_25_32(a, st);
}

}  // namespace sstep
