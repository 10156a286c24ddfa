// Tall-skinny Gram reduction G_raw = P^T (A P) (lower triangle) and
// c' = P^T W with W = p_0 or M p_0, as per-block partial sums (Sec. 1: the
// Gram system of each outer iteration; Sec. 2: G = P^T A P and P^T r).
//
// Design: the lower triangle plus the right-hand side has E = s(s+1)/2 + s
// entries.  Rows i of G (row i owns entries (i, 0..i) and c_i) are split into
// NG groups with nearly equal entry counts, fixed at compile time; wave w of a
// block owns group w and keeps its entries in registers as FP accumulators
// (vector FMA: the reduction does ~0.6 flop per byte, so it is HBM-bound and
// matrix cores would not help).  All waves of a block stream the same 64-row
// slabs of P and AP, lane = row, so every global load of a column is a
// contiguous 512-byte (FP64) segment; columns shared by several groups are
// served from L1/L2.  At the end each wave reduces its accumulators across the
// 64 lanes with a fixed butterfly and stores one partial per entry and block:
// gpart[e * nbg + block].  The second stage (fixed-order sum over blocks) runs
// in the FGS kernel, so the result is bitwise reproducible.
#pragma once

#include "launch.h"

namespace sstep {

template <int S>
struct GramPlan {
    static constexpr int NG = S <= 6 ? 1 : S <= 10 ? 2 : S <= 16 ? 4 : S <= 24 ? 8 : 16;
    int grp[S];   // group of G-row i
    int off[S];   // first accumulator of row i within its group
    int cnt[NG];  // accumulators of a group
    int jmax[NG]; // largest G-row of a group (AP columns 0..jmax are loaded)

    constexpr GramPlan() : grp(), off(), cnt(), jmax()
    {
        int load[NG] = {};
        for (int i = S - 1; i >= 0; --i) {  // heaviest rows first, into the lightest group
            int best = 0;
            for (int g = 1; g < NG; ++g)
                if (load[g] < load[best])
                    best = g;
            grp[i] = best;
            load[best] += i + 2;
        }
        for (int g = 0; g < NG; ++g) {
            cnt[g] = 0;
            jmax[g] = -1;
        }
        for (int i = 0; i < S; ++i) {
            off[i] = cnt[grp[i]];
            cnt[grp[i]] += i + 2;
            if (i > jmax[grp[i]])
                jmax[grp[i]] = i;
        }
    }
};

// Canonical entry index: (i, j <= i) -> i(i+1)/2 + j; c_i -> s(s+1)/2 + i.
__host__ __device__ constexpr int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }

template <typename T, int S, int G, bool WD>
__device__ __forceinline__ void gram_group(const T *__restrict__ P, const T *__restrict__ AP,
                                           const T *__restrict__ dvec, int64_t ld, int64_t beg, int64_t end,
                                           double *__restrict__ gpart, int nbg, int blk)
{
    constexpr GramPlan<S> pl{};
    constexpr int NA = pl.cnt[G];
    constexpr int JM = pl.jmax[G];
    if constexpr (NA == 0) {
        return;
    } else {
        const int lane = threadIdx.x % kWave;
        T acc[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a)
            acc[a] = T(0);
        for (int64_t base = beg; base < end; base += kWave) {
            const int64_t m = base + lane;
            const bool ok = m < end;
            T ap[JM + 1];
#pragma unroll
            for (int j = 0; j <= JM; ++j)
                ap[j] = ok ? AP[j * ld + m] : T(0);
            T w = ok ? P[m] : T(0);
            if constexpr (WD)
                w *= ok ? dvec[m] : T(0);
#pragma unroll
            for (int i = 0; i < S; ++i) {
                if (pl.grp[i] == G) {
                    const T p = ok ? P[i * ld + m] : T(0);
#pragma unroll
                    for (int j = 0; j <= i; ++j)
                        acc[pl.off[i] + j] += p * ap[j];
                    acc[pl.off[i] + i + 1] += p * w;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (pl.grp[i] == G) {
#pragma unroll
                for (int j = 0; j <= i + 1; ++j) {
                    const T v = wave_sum(acc[pl.off[i] + j]);
                    const int e = j <= i ? tri_index(i, j) : S * (S + 1) / 2 + i;
                    if (lane == (pl.off[i] + j) % kWave)
                        gpart[static_cast<int64_t>(e) * nbg + blk] = static_cast<double>(v);
                }
            }
        }
    }
}

template <typename T, int S, bool WD, int G>
__device__ __forceinline__ void gram_dispatch(int w, const T *P, const T *AP, const T *dvec, int64_t ld, int64_t beg,
                                              int64_t end, double *gpart, int nbg, int blk)
{
    if constexpr (G < GramPlan<S>::NG) {
        if (w == G)
            gram_group<T, S, G, WD>(P, AP, dvec, ld, beg, end, gpart, nbg, blk);
        else
            gram_dispatch<T, S, WD, G + 1>(w, P, AP, dvec, ld, beg, end, gpart, nbg, blk);
    }
}

template <typename T, int S, bool WD>
__global__ __launch_bounds__(kWave * GramPlan<S>::NG) void k_gram(const DevState *__restrict__ st,
                                                                  const T *__restrict__ P, const T *__restrict__ AP,
                                                                  const T *__restrict__ dvec, int64_t ld, int64_t n,
                                                                  int64_t chunk, double *__restrict__ gpart, int nbg)
{
    if (st->done)
        return;
    const int blk = blockIdx.x;
    const int64_t beg = static_cast<int64_t>(blk) * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    const int w = threadIdx.x / kWave;
    gram_dispatch<T, S, WD, 0>(w, P, AP, dvec, ld, beg, end, gpart, nbg, blk);
}

template <typename T, int S>
hipError_t gram_launch_s(const IterArgs &a, hipStream_t st)
{
    const dim3 block(kWave * GramPlan<S>::NG);
    const T *P = static_cast<const T *>(a.P);
    const T *AP = static_cast<const T *>(a.AP);
    const T *dv = nullptr;
    if (a.wdvec)
        dv = reinterpret_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(a.op.dvec)
                                                         : static_cast<const void *>(a.op.dvec32));
    if (a.wdvec)
        hipLaunchKernelGGL((k_gram<T, S, true>), dim3(a.nbg), block, 0, st, a.st, P, AP, dv, a.ld, a.op.n, a.gchunk,
                           a.gpart, a.nbg);
    else
        hipLaunchKernelGGL((k_gram<T, S, false>), dim3(a.nbg), block, 0, st, a.st, P, AP, dv, a.ld, a.op.n,
                           a.gchunk, a.gpart, a.nbg);
    return hipGetLastError();
}

// Launchers for a range of s, one translation unit per range.
hipError_t gram_launch_1_8(const IterArgs &a, hipStream_t st);
hipError_t gram_launch_9_16(const IterArgs &a, hipStream_t st);
hipError_t gram_launch_17_24(const IterArgs &a, hipStream_t st);
hipError_t gram_launch_25_32(const IterArgs &a, hipStream_t st);

}  // namespace sstep
