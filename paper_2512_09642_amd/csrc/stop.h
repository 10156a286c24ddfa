// Stopping test of the outer iteration (Sec. 8: stop at the first k with
// ||r_k|| < tol ||r_0||, strict, on the true residual), and the "last block"
// hand-off that lets the kernel forming the residual norm's partial sums run
// the test itself, before any basis or Gram work of iteration k is started.
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
// the four wave sums are added in order).  The caller has made the partials
// of other blocks visible (last_block).  Returns the total in thread 0 (other
// threads: unspecified).  Every thread of the block must call it.
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

// Called by every thread of every block of a grid after thread 0 of the block
// has stored the block's partial sum: true in exactly one block, the last to
// arrive, once every partial is visible to it.  Thread 0 releases the
// block's partial (device-scope fence: the XCD's L2 is written back) and
// takes a ticket; the last block acquires (device-scope fence: its L2 lines
// are invalidated, so the other XCDs' partials are read from memory) and
// resets the ticket for the next launch.
__device__ inline bool last_block(uint32_t *ticket, uint32_t nblocks)
{
    __shared__ int is_last;
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t t = atomicAdd(ticket, 1u);
        is_last = t + 1 == nblocks;
    }
    __syncthreads();
    if (!is_last)
        return false;
    __threadfence();
    if (threadIdx.x == 0)
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// The tail of a residual kernel: hand the partial sums of ||r||^2 to the last
// block, which sums them in the fixed order and runs the stopping test.
__device__ inline void residual_stop_tail(DevState *__restrict__ st, const double *rpart, int nparts,
                                          double *__restrict__ dbg_rho, double *__restrict__ hist, int hist_cap)
{
    if (!last_block(&st->ticket, static_cast<uint32_t>(nparts)))
        return;
    const double rho2 = fixed_order_sum(rpart, nparts);
    if (threadIdx.x == 0)
        stop_test(st, rho2, dbg_rho, hist, hist_cap);
}

}  // namespace sstep
