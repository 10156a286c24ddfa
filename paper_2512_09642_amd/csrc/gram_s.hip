// Explicit instantiations of the Gram, FGS and batched launchers for one basis
// width S = SSTEP_S (the build compiles this file once per S in 1..32); the
// operator-applying Gram kernel exists for S <= kGoMaxS.
#include "batched_impl.h"
#include "dispatch.h"
#include "gram_op_impl.h"
#include "gram_sym_impl.h"

#ifndef SSTEP_S
#error "compile with -DSSTEP_S=<basis width>"
#endif
// the recurrence kind needs the Gram of s + 1 columns, so it stops one short
// of the widest basis
#define SSTEP_REC_MAX_S 31

namespace sstep {

static_assert(SSTEP_S >= 1 && SSTEP_S <= kMaxS, "basis width out of range");

template hipError_t gram_launch_s<double, SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t gram_launch_s<float, SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t fgs_launch_s<SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t bgram_launch_s<double, SSTEP_S>(const BatchArgs &, hipStream_t);
template hipError_t bgram_launch_s<float, SSTEP_S>(const BatchArgs &, hipStream_t);
template hipError_t bfgs_launch_s<SSTEP_S>(const BatchArgs &, hipStream_t);
#if SSTEP_S <= SSTEP_REC_MAX_S
template hipError_t gram_sym_launch_s<double, SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t gram_sym_launch_s<float, SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t fgs_rec_launch_s<SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t fgs_mom_launch_s<SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t bgram_sym_launch_s<double, SSTEP_S>(const BatchArgs &, hipStream_t);
template hipError_t bgram_sym_launch_s<float, SSTEP_S>(const BatchArgs &, hipStream_t);
template hipError_t bfgs_rec_launch_s<SSTEP_S>(const BatchArgs &, hipStream_t);
template hipError_t bfgs_mom_launch_s<SSTEP_S>(const BatchArgs &, hipStream_t);
#endif
#if SSTEP_S <= 16
static_assert(SSTEP_S <= kGoMaxS, "operator-applying Gram width");
template hipError_t gram_op_launch_s<double, SSTEP_S>(const IterArgs &, hipStream_t);
template hipError_t gram_op_launch_s<float, SSTEP_S>(const IterArgs &, hipStream_t);
#endif

}  // namespace sstep
