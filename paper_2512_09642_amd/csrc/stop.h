// Stopping test of the outer iteration (Sec. 8: stop at the first k with
// ||r_k|| < tol ||r_0||, strict, on the true residual), run right after the
// residual kernel and before any basis or Gram work of iteration k.
#pragma once

#include "common.h"

namespace sstep {

constexpr int kSumThreads = 256;

// One thread.  rho2 = ||b - A x_k||^2.  Records rho_0 on the first call of a
// solve, then stops the solve (done = 1) when rho_k < tol rho_0, at max_outer
// (SSTEP_E_NOCONV) or on a non-finite norm (SSTEP_E_NONFINITE).  A no_stop
// state (single-step and timing entry points) stops only on a zero initial
// or a non-finite norm.  Writes rho_k to *dbg_rho (may be NULL) and
// rho_k / rho_0 to hist[k] when k < hist_cap.  Returns 1 when the solve is
// (now) stopped.
__device__ inline int stop_test(DevState *__restrict__ st, double rho2, double *__restrict__ dbg_rho,
                                double *__restrict__ hist, int hist_cap)
{
    const double rho = sqrt(rho2);
    const int first = st->first;
    const double rho0 = first ? rho : st->rho0;
    const int k = st->iter;
    int stop = 0, status = 0;
    double relres = 0.0;
    if (first && rho0 == 0.0) {
        stop = 1;
    } else if (!isfinite(rho)) {
        stop = 1;
        status = 6;  // SSTEP_E_NONFINITE
        relres = rho;
    } else {
        relres = rho / rho0;
        if (!st->no_stop) {
            if (rho < st->tol * rho0)
                stop = 1;
            else if (k >= st->max_outer) {
                stop = 1;
                status = 5;  // SSTEP_E_NOCONV
            }
        }
    }
    st->first = 0;
    st->rho0 = rho0;
    st->rho = rho;
    st->relres = relres;
    if (k < hist_cap)
        hist[k] = relres;
    if (dbg_rho)
        *dbg_rho = rho;
    if (stop) {
        st->status = status;
        st->done = 1;
    }
    return stop;
}

// Sum of part[0..cnt) in a fixed order by the first kSumThreads threads of a
// block (thread t takes t, t + 256, ..., the waves combine by butterfly and
// the four wave sums are added in order).  Returns the total in thread 0
// (other threads: unspecified).  Every thread of the block must call it.
__device__ inline double fixed_order_sum(const double *part, int cnt)
{
    __shared__ double wsum[kSumThreads / kWave];
    double acc = 0.0;
    if (threadIdx.x < kSumThreads) {
#pragma unroll 4
        for (int q = threadIdx.x; q < cnt; q += kSumThreads)
            acc += part[q];
    }
    acc = wave_sum(acc);
    if (threadIdx.x < kSumThreads && threadIdx.x % kWave == 0)
        wsum[threadIdx.x / kWave] = acc;
    __syncthreads();
    double v = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kSumThreads / kWave; ++w)
            v += wsum[w];
    return v;
}

}  // namespace sstep
