// Gram and FGS kernels of the batched outer iteration, instantiated per basis
// width next to the single-system ones.
#pragma once

#include "fgs_core.h"
#include "gram_sym_impl.h"

namespace sstep {

// A pair has stopped: counted once, by one thread.
__device__ __forceinline__ void pair_stopped(BGlob *gl, const BSys &Q)
{
    atomicAdd(&gl->ndone, 1);
    atomicAdd(&gl->bdone, Q.nbl);
}

// Gram partials of every active pair: tile (q, chunk, r) reduces rows
// [chunk*gchunk, (chunk+1)*gchunk) of pair (q, r)'s basis (column stride
// nrhs*ld, zero padding past n) into gpart[gofs + r*E*nch + e*nch + chunk].
template <typename T, int S, bool WD>
__global__ __launch_bounds__(kWave * GramPlan<S>::NG) void k_bgram(const BGlob *__restrict__ gl,
                                                                   const BSys *__restrict__ sys,
                                                                   const GTile *__restrict__ tiles, int ntiles,
                                                                   const DevState *__restrict__ pairs, int nrhs,
                                                                   const T *__restrict__ P, const T *__restrict__ AP,
                                                                   double *__restrict__ gpart)
{
    constexpr int E = S * (S + 1) / 2 + S;
    if (gl->ndone == gl->npairs)
        return;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const GTile tl = tiles[t];
        const BSys &Q = sys[tl.q];
        if (pairs[Q.pair0 + tl.r].done)
            continue;
        const int64_t off = Q.pofs + static_cast<int64_t>(tl.r) * Q.ld;
        const int64_t cs = static_cast<int64_t>(nrhs) * Q.ld;
        const int64_t beg = static_cast<int64_t>(tl.chunk) * Q.gchunk;
        const int64_t end = beg + Q.gchunk < Q.ld ? beg + Q.gchunk : Q.ld;
        const T *dv = nullptr;
        if constexpr (WD)
            dv = reinterpret_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(Q.dvec)
                                                             : static_cast<const void *>(Q.dvec32));
        gram_tile<T, S, gram_rpl<T, S>(), WD>(P + off, AP + off, dv, cs, beg, end, end - beg, end - beg + 1,
                                               gpart + Q.gofs + static_cast<int64_t>(tl.r) * E * Q.nch, Q.nch,
                                               tl.chunk);
    }
}

template <typename T, int S>
hipError_t bgram_launch_s(const BatchArgs &a, hipStream_t st)
{
    const dim3 block(kWave * GramPlan<S>::NG);
    const T *P = static_cast<const T *>(a.P);
    const T *AP = static_cast<const T *>(a.AP);
    if (a.wdvec)
        hipLaunchKernelGGL((k_bgram<T, S, true>), dim3(a.grid_gt), block, 0, st, a.gl, a.sys, a.gtiles, a.ngt,
                           a.pairs, a.nrhs, P, AP, a.gpart);
    else
        hipLaunchKernelGGL((k_bgram<T, S, false>), dim3(a.grid_gt), block, 0, st, a.gl, a.sys, a.gtiles, a.ngt,
                           a.pairs, a.nrhs, P, AP, a.gpart);
    return hipGetLastError();
}

// Recurrence Gram kind: tile (q, chunk, r) forms the partial of
// H = P^T M P over p_0 .. p_s and of c' for rows [chunk*gchunk,
// (chunk+1)*gchunk) of pair (q, r) on the matrix cores (gram_sym_rows), into
// gpart[gofs + r*E1*nch + e*nch + chunk].
template <typename T, int S1, bool WAP, bool WD>
__global__ __launch_bounds__(kGsThreads) void k_bgram_sym(const BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                           const GTile *__restrict__ tiles, int ntiles,
                                                           const DevState *__restrict__ pairs, int nrhs,
                                                           const T *__restrict__ P, double *__restrict__ gpart)
{
    constexpr int E1 = S1 * (S1 + 1) / 2 + S1;
    if (gl->ndone == gl->npairs)
        return;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const GTile tl = tiles[t];
        const BSys &Q = sys[tl.q];
        if (pairs[Q.pair0 + tl.r].done)
            continue;  // the whole block: gram_sym_rows has barriers
        const int64_t off = Q.pofs + static_cast<int64_t>(tl.r) * Q.ld;
        const int64_t cs = static_cast<int64_t>(nrhs) * Q.ld;
        const int64_t beg = static_cast<int64_t>(tl.chunk) * Q.gchunk;
        const int64_t end = beg + Q.gchunk < Q.ld ? beg + Q.gchunk : Q.ld;
        const T *dv = reinterpret_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(Q.dvec)
                                                                 : static_cast<const void *>(Q.dvec32));
        gram_sym_rows<T, S1, WAP, WD>(P + off, cs, dv, beg, end,
                                      gpart + Q.gofs + static_cast<int64_t>(tl.r) * E1 * Q.nch, Q.nch, tl.chunk);
    }
}

template <typename T, int S>
hipError_t bgram_sym_launch_s(const BatchArgs &a, hipStream_t st)
{
    constexpr int S1 = S + 1;
    const T *P = static_cast<const T *>(a.P);
    const dim3 grid(a.grid_gt), block(kGsThreads);
    if (a.rec_wap && a.wdvec)
        hipLaunchKernelGGL((k_bgram_sym<T, S1, true, true>), grid, block, 0, st, a.gl, a.sys, a.gtiles, a.ngt, a.pairs,
                           a.nrhs, P, a.gpart);
    else if (a.rec_wap)
        hipLaunchKernelGGL((k_bgram_sym<T, S1, true, false>), grid, block, 0, st, a.gl, a.sys, a.gtiles, a.ngt,
                           a.pairs, a.nrhs, P, a.gpart);
    else if (a.wdvec)
        hipLaunchKernelGGL((k_bgram_sym<T, S1, false, true>), grid, block, 0, st, a.gl, a.sys, a.gtiles, a.ngt,
                           a.pairs, a.nrhs, P, a.gpart);
    else
        hipLaunchKernelGGL((k_bgram_sym<T, S1, false, false>), grid, block, 0, st, a.gl, a.sys, a.gtiles, a.ngt,
                           a.pairs, a.nrhs, P, a.gpart);
    return hipGetLastError();
}

// One block (four waves) per pair: fixed-order sums of the pair's partials,
// then wave 0 runs the stopping test, scaling and FGS; a pair that stops is
// counted in the global done counter.
constexpr int kBFgsThreads = 256;

template <int S>
__global__ __launch_bounds__(kBFgsThreads) void k_bfgs(BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                       DevState *__restrict__ pairs, int nrhs,
                                                       const double *__restrict__ rpart,
                                                       const double *__restrict__ gpart, int nu, double cscale,
                                                       int fp32, double *__restrict__ dbg)
{
    constexpr int E = S * (S + 1) / 2 + S;
    const int p = blockIdx.x;
    DevState *ps = pairs + p;
    if (ps->done)
        return;
    const BSys &Q = sys[p / nrhs];
    const int r = p % nrhs;
    __shared__ double sg[E + 1];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const double *gp = gpart + Q.gofs + static_cast<int64_t>(r) * E * Q.nch;
    const double *rp = rpart + Q.rofs + static_cast<int64_t>(r) * Q.nch;
    for (int t = wave; t <= E; t += kBFgsThreads / kWave) {
        const double *src = t < E ? gp + static_cast<int64_t>(t) * Q.nch : rp;
        double a0 = 0.0, a1 = 0.0;
        int q = lane;
        for (; q + kWave < Q.nch; q += 2 * kWave) {
            a0 += src[q];
            a1 += src[q + kWave];
        }
        for (; q < Q.nch; q += kWave)
            a0 += src[q];
        const double acc = wave_sum(a0 + a1);
        if (lane == 0)
            sg[t] = acc;
    }
    __shared__ int stopped;
    __syncthreads();
    double *pdbg = dbg + static_cast<int64_t>(p) * dbg_size(S);
    if (threadIdx.x == 0)
        stopped = stop_test(ps, sg[E], pdbg + dbg_rho(S), nullptr, 0);
    __syncthreads();
    if (wave != 0)
        return;
    int now = stopped;
    if (!now)
        now = fgs_wave<S>(ps, sg, nu, cscale, fp32, Q.inv_sqrt_n, pdbg, nullptr, 0);
    if (now && lane == 0)
        pair_stopped(gl, Q);
}

template <int S>
hipError_t bfgs_launch_s(const BatchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_bfgs<S>, dim3(a.npairs), dim3(kBFgsThreads), 0, st, a.gl, a.sys, a.pairs, a.nrhs, a.rpart,
                       a.gpart, a.nu, a.cscale, a.fp32, a.dbg);
    return hipGetLastError();
}

// H (LDS, the recurrence kind's layout) mapped onto G_raw = P^T A P with the
// system's theta, sigma (as k_fgs_rec does), then the FGS wave.
template <int S>
__device__ __forceinline__ void bfgs_map_sweep(BGlob *__restrict__ gl, DevState *__restrict__ ps, const BSys &Q,
                                               const double *h, double *sg, int nu, double cscale, int fp32,
                                               double hscale, double *__restrict__ pdbg)
{
    constexpr int S1 = S + 1;
    constexpr int T0 = S * (S + 1) / 2;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const double theta = Q.theta, sigma = Q.sigma;
    auto H = [&](int a, int b) { return a >= b ? h[tri_index(a, b)] : h[tri_index(b, a)]; };
    for (int e = threadIdx.x; e < T0; e += kBFgsThreads) {
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= e)
            ++i;
        const int j = e - i * (i + 1) / 2;
        const double g = j == 0 ? H(i, 1) / theta + sigma * H(i, 0)
                                : (H(i, j + 1) + H(i, j - 1)) / (2.0 * theta) + sigma * H(i, j);
        sg[e] = hscale * g;
    }
    for (int i = threadIdx.x; i < S; i += kBFgsThreads)
        sg[T0 + i] = h[S1 * (S1 + 1) / 2 + i];
    __syncthreads();
    if (wave != 0)
        return;
    const int now = fgs_wave<S>(ps, sg, nu, cscale, fp32, Q.inv_sqrt_n, pdbg, nullptr, 0);
    if (now && lane == 0)
        pair_stopped(gl, Q);
}

// Recurrence Gram kind: the pair's sums of H and c', the stopping test, then
// H mapped onto G_raw = P^T A P with the system's theta, sigma (as k_fgs_rec
// does) and the FGS wave.
template <int S>
__global__ __launch_bounds__(kBFgsThreads) void k_bfgs_rec(BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                           DevState *__restrict__ pairs, int nrhs,
                                                           const double *__restrict__ rpart,
                                                           const double *__restrict__ bpart,
                                                           const double *__restrict__ gpart, int nu, double cscale,
                                                           int fp32, double hscale, double *__restrict__ dbg)
{
    constexpr int S1 = S + 1;
    constexpr int E1 = S1 * (S1 + 1) / 2 + S1;
    constexpr int T0 = S * (S + 1) / 2;
    // ||r||^2: one partial per band (bpart, k_bres_f2, one slot per
    // right-hand side) or per chunk tile (rpart, k_bresidual)
    const int p = blockIdx.x;
    DevState *ps = pairs + p;
    if (ps->done)
        return;
    const BSys &Q = sys[p / nrhs];
    const int r = p % nrhs;
    __shared__ double h[E1 + 1];
    __shared__ double sg[T0 + S];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const double *gp = gpart + Q.gofs + static_cast<int64_t>(r) * E1 * Q.nch;
    const double *rp = bpart ? bpart + Q.mofs + static_cast<int64_t>(r) * Q.nf2q
                             : rpart + Q.rofs + static_cast<int64_t>(r) * Q.nch;
    for (int t = wave; t <= E1; t += kBFgsThreads / kWave) {
        const double *src = t < E1 ? gp + static_cast<int64_t>(t) * Q.nch : rp;
        const int cnt = t < E1 || !bpart ? Q.nch : Q.nf2q;
        double a0 = 0.0, a1 = 0.0;
        int q = lane;
        for (; q + kWave < cnt; q += 2 * kWave) {
            a0 += src[q];
            a1 += src[q + kWave];
        }
        for (; q < cnt; q += kWave)
            a0 += src[q];
        const double acc = wave_sum(a0 + a1);
        if (lane == 0)
            h[t] = acc;
    }
    __shared__ int stopped;
    __syncthreads();
    double *pdbg = dbg + static_cast<int64_t>(p) * dbg_size(S);
    if (threadIdx.x == 0)
        stopped = stop_test(ps, h[E1], pdbg + dbg_rho(S), nullptr, 0);
    __syncthreads();
    if (stopped) {
        if (threadIdx.x == 0)
            pair_stopped(gl, Q);
        return;
    }
    bfgs_map_sweep<S>(gl, ps, Q, h, sg, nu, cscale, fp32, hscale, pdbg);
}

template <int S>
hipError_t bfgs_rec_launch_s(const BatchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_bfgs_rec<S>, dim3(a.npairs), dim3(kBFgsThreads), 0, st, a.gl, a.sys, a.pairs, a.nrhs,
                       a.rpart, a.bres && !a.mom ? a.mpart : nullptr, a.gpart, a.nu, a.cscale, a.fp32,
                       a.rec_hscale, a.dbg);
    return hipGetLastError();
}

// Moments kind: per pair, the sums of its 2S + 1 product slots (one partial
// per band of its system, written by the two-step basis) and of its residual
// partials, the stopping test, then the moments, H (as k_fgs_mom forms them)
// and the recurrence mapping with the FGS wave.
template <int S>
__global__ __launch_bounds__(kBFgsThreads) void k_bfgs_mom(BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                           DevState *__restrict__ pairs, int nrhs,
                                                           const double *__restrict__ mpart, int nu, double cscale,
                                                           int fp32, double hscale, double *__restrict__ dbg)
{
    constexpr int S1 = S + 1;
    constexpr int E1 = S1 * (S1 + 1) / 2 + S1;
    constexpr int T0 = S * (S + 1) / 2;
    constexpr int NS = 2 * S + 1;
    const int p = blockIdx.x;
    DevState *ps = pairs + p;
    if (ps->done)
        return;
    const BSys &Q = sys[p / nrhs];
    const int r = p % nrhs;
    __shared__ double m[NS + 1];
    __shared__ double mu[NS];
    __shared__ double h[E1];
    __shared__ double sg[T0 + S];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // slots 0 .. NS - 1: the products; slot NS: ||r||^2 (k_bres_f2)
    const double *mp = mpart + Q.mofs + static_cast<int64_t>(r) * bmom_slots(S) * Q.nf2q;
    for (int t = wave; t <= NS; t += kBFgsThreads / kWave) {
        const double *src = mp + static_cast<int64_t>(t) * Q.nf2q;
        const int cnt = Q.nf2q;
        double a0 = 0.0, a1 = 0.0;
        int q = lane;
        for (; q + kWave < cnt; q += 2 * kWave) {
            a0 += src[q];
            a1 += src[q + kWave];
        }
        for (; q < cnt; q += kWave)
            a0 += src[q];
        const double acc = wave_sum(a0 + a1);
        if (lane == 0)
            m[t] = acc;
    }
    __shared__ int stopped;
    __syncthreads();
    double *pdbg = dbg + static_cast<int64_t>(p) * dbg_size(S);
    if (threadIdx.x == 0)
        stopped = stop_test(ps, m[NS], pdbg + dbg_rho(S), nullptr, 0);
    __syncthreads();
    if (stopped) {
        if (threadIdx.x == 0)
            pair_stopped(gl, Q);
        return;
    }
    for (int k = threadIdx.x; k < NS; k += kBFgsThreads)
        mu[k] = k <= 1 ? m[k] : 2.0 * m[k] - m[k % 2];
    __syncthreads();
    for (int e = threadIdx.x; e < S1 * (S1 + 1) / 2; e += kBFgsThreads) {
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= e)
            ++i;
        const int j = e - i * (i + 1) / 2;
        h[e] = 0.5 * (mu[i + j] + mu[i - j]);
    }
    for (int i = threadIdx.x; i < S1; i += kBFgsThreads)
        h[S1 * (S1 + 1) / 2 + i] = mu[i];
    __syncthreads();
    bfgs_map_sweep<S>(gl, ps, Q, h, sg, nu, cscale, fp32, hscale, pdbg);
}

template <int S>
hipError_t bfgs_mom_launch_s(const BatchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_bfgs_mom<S>, dim3(a.npairs), dim3(kBFgsThreads), 0, st, a.gl, a.sys, a.pairs, a.nrhs,
                       a.mpart, a.nu, a.cscale, a.fp32, a.rec_hscale, a.dbg);
    return hipGetLastError();
}

}  // namespace sstep
