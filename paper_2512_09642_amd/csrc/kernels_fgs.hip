// Dispatch of the Gram, FGS and batched launches to the instantiation for the
// basis width s (one object per width, see dispatch.h).
#include "dispatch.h"
#include "stop.h"

namespace sstep {

namespace {
// Moments kind: the basis kernels leave, per logical block, the M inner
// products d_i = <p_i, M p_i> (slot 2i, i = 0..s) and e_i = <p_i, M p_{i-1}>
// (slot 2i - 1, i = 1..s); slot k holds cnt[k] block partials at
// part + k * stride.  One block per slot sums them in a fixed order (as
// k_partial_sums does).
__global__ __launch_bounds__(kSumThreads) void k_mom_sums(const DevState *__restrict__ st,
                                                          const double *__restrict__ part,
                                                          const int32_t *__restrict__ cnt, int64_t stride,
                                                          double *__restrict__ sums)
{
    __shared__ double wpart[kSumThreads / kWave];
    if (st->done)
        return;
    const int k = blockIdx.x;
    const double *src = part + static_cast<int64_t>(k) * stride;
    const int nb = cnt[k];
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += kSumThreads)
        acc += src[q];
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0)
        wpart[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < kSumThreads / kWave; ++w)
            v += wpart[w];
        sums[k] = v;
    }
}

}  // namespace

hipError_t launch_mom_sums(const IterArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_mom_sums, dim3(2 * a.s + 1), dim3(kSumThreads), 0, st, a.st, a.mpart, a.mcnt, a.mstride,
                       a.gsum);
    return hipGetLastError();
}

#define SSTEP_CASES_1_16(F) \
    F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16)
#define SSTEP_CASES_17_32(F) \
    F(17) F(18) F(19) F(20) F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30) F(31) F(32)

#define SSTEP_CASES_17_31(F) \
    F(17) F(18) F(19) F(20) F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30) F(31)

hipError_t launch_gram(const IterArgs &a, hipStream_t st)
{
    if (a.gram_mom)  // the basis kernels formed the products: only their sums remain
        return launch_mom_sums(a, st);
    if (a.gram_rec) {
#define SSTEP_GS(S)                                                                          \
    case S:                                                                                  \
        return a.fp32 ? gram_sym_launch_s<float, S>(a, st) : gram_sym_launch_s<double, S>(a, st);
        switch (a.s) { SSTEP_CASES_1_16(SSTEP_GS) SSTEP_CASES_17_31(SSTEP_GS) default: return hipErrorInvalidValue; }
#undef SSTEP_GS
    }
    if (a.gram_op) {
#define SSTEP_GO(S)                                                                          \
    case S:                                                                                  \
        return a.fp32 ? gram_op_launch_s<float, S>(a, st) : gram_op_launch_s<double, S>(a, st);
        switch (a.s) { SSTEP_CASES_1_16(SSTEP_GO) default: return hipErrorInvalidValue; }
#undef SSTEP_GO
    }
#define SSTEP_G(S)                                                                           \
    case S:                                                                                  \
        return a.fp32 ? gram_launch_s<float, S>(a, st) : gram_launch_s<double, S>(a, st);
    switch (a.s) { SSTEP_CASES_1_16(SSTEP_G) SSTEP_CASES_17_32(SSTEP_G) default: return hipErrorInvalidValue; }
#undef SSTEP_G
}

hipError_t launch_fgs(const IterArgs &a, hipStream_t st)
{
    if (a.gram_mom) {
#define SSTEP_FM(S) \
    case S:         \
        return fgs_mom_launch_s<S>(a, st);
        switch (a.s) { SSTEP_CASES_1_16(SSTEP_FM) SSTEP_CASES_17_31(SSTEP_FM) default: return hipErrorInvalidValue; }
#undef SSTEP_FM
    }
    if (a.gram_rec) {
#define SSTEP_FR(S) \
    case S:         \
        return fgs_rec_launch_s<S>(a, st);
        switch (a.s) { SSTEP_CASES_1_16(SSTEP_FR) SSTEP_CASES_17_31(SSTEP_FR) default: return hipErrorInvalidValue; }
#undef SSTEP_FR
    }
#define SSTEP_F(S) \
    case S:        \
        return fgs_launch_s<S>(a, st);
    switch (a.s) { SSTEP_CASES_1_16(SSTEP_F) SSTEP_CASES_17_32(SSTEP_F) default: return hipErrorInvalidValue; }
#undef SSTEP_F
}

hipError_t launch_bgram(const BatchArgs &a, hipStream_t st)
{
    if (a.mom)  // the two-step basis formed the products
        return hipSuccess;
    if (a.rec) {
#define SSTEP_BGS(S)                                                                         \
    case S:                                                                                  \
        return a.fp32 ? bgram_sym_launch_s<float, S>(a, st) : bgram_sym_launch_s<double, S>(a, st);
        switch (a.s) { SSTEP_CASES_1_16(SSTEP_BGS) SSTEP_CASES_17_31(SSTEP_BGS) default: return hipErrorInvalidValue; }
#undef SSTEP_BGS
    }
#define SSTEP_BG(S)                                                                          \
    case S:                                                                                  \
        return a.fp32 ? bgram_launch_s<float, S>(a, st) : bgram_launch_s<double, S>(a, st);
    switch (a.s) { SSTEP_CASES_1_16(SSTEP_BG) SSTEP_CASES_17_32(SSTEP_BG) default: return hipErrorInvalidValue; }
#undef SSTEP_BG
}

hipError_t launch_bfgs(const BatchArgs &a, hipStream_t st)
{
    if (a.mom) {
#define SSTEP_BFM(S) \
    case S:          \
        return bfgs_mom_launch_s<S>(a, st);
        switch (a.s) { SSTEP_CASES_1_16(SSTEP_BFM) SSTEP_CASES_17_31(SSTEP_BFM) default: return hipErrorInvalidValue; }
#undef SSTEP_BFM
    }
    if (a.rec) {
#define SSTEP_BFR(S) \
    case S:          \
        return bfgs_rec_launch_s<S>(a, st);
        switch (a.s) { SSTEP_CASES_1_16(SSTEP_BFR) SSTEP_CASES_17_31(SSTEP_BFR) default: return hipErrorInvalidValue; }
#undef SSTEP_BFR
    }
#define SSTEP_BF(S) \
    case S:         \
        return bfgs_launch_s<S>(a, st);
    switch (a.s) { SSTEP_CASES_1_16(SSTEP_BF) SSTEP_CASES_17_32(SSTEP_BF) default: return hipErrorInvalidValue; }
#undef SSTEP_BF
}

}  // namespace sstep
