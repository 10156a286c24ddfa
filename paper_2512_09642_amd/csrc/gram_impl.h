// Tall-skinny Gram reduction G_raw = P^T (A P) (lower triangle) and
// c' = P^T W with W = p_0 or M p_0, as per-block partial sums (Sec. 1: the
// Gram system of each outer iteration; Sec. 2: G = P^T A P and P^T r).
//
// Design (gfx950, wave64, vector FMA -- the reduction does ~0.6 flop per byte,
// so it is HBM-bound and matrix cores would not help):
//  * The s columns are cut into H = ceil(s/8) blocks of B <= 8 columns.  A
//    diagonal block pair (I, I) -- a triangle plus its right-hand-side entries
//    c_i -- is one group; an off-diagonal pair (I, J), I > J, is split by rows
//    into two groups.  So there are NG = H^2 groups of at most B(B+1)/2 + B
//    entries, each needing at most 2B + 1 columns; wave g of a block owns group g
//    and keeps its entries in registers.
//  * Lane = row group of RPL consecutive rows, read with one 8/16-byte load per
//    column: a wave streams 64*RPL rows of a column as one contiguous segment.
//  * Column buffers are zero-padded to a multiple of 256 rows, so the loops
//    have no tail guards (padding rows contribute 0).
//  * Two schedules, picked by the autotuner: contiguous (block b owns one
//    contiguous chunk of rows) and strided (block b owns slabs b, b + nbg, ...).
//  * Each wave reduces its accumulators over the 64 lanes with a fixed
//    butterfly and stores entry e of its block at gpart[e * estride + slot];
//    the second stage sums the partials in a fixed order, so the result is
//    bitwise reproducible.
#pragma once

#include "launch.h"

namespace sstep {

template <int S>
struct GramPlan {
    static constexpr int H = (S + 7) / 8;
    static constexpr int B = (S + H - 1) / H;
    static constexpr int NG = H * H;
    int r0[NG], r1[NG], c0[NG], c1[NG], hasc[NG], cnt[NG];

    constexpr GramPlan() : r0(), r1(), c0(), c1(), hasc(), cnt()
    {
        int g = 0;
        for (int I = 0; I < H; ++I) {
            const int lo = I * B, hi = (I + 1) * B < S ? (I + 1) * B : S;
            r0[g] = lo, r1[g] = hi, c0[g] = lo, c1[g] = hi, hasc[g] = 1;
            ++g;
        }
        for (int I = 0; I < H; ++I)
            for (int J = 0; J < I; ++J) {
                const int lo = I * B, hi = (I + 1) * B < S ? (I + 1) * B : S;
                const int mid = (lo + hi) / 2;
                r0[g] = lo, r1[g] = mid, c0[g] = J * B, c1[g] = (J + 1) * B, hasc[g] = 0;
                ++g;
                r0[g] = mid, r1[g] = hi, c0[g] = J * B, c1[g] = (J + 1) * B, hasc[g] = 0;
                ++g;
            }
        for (int q = 0; q < NG; ++q) {
            int c = 0;
            for (int i = r0[q]; i < r1[q]; ++i)
                for (int j = c0[q]; j < c1[q]; ++j)
                    if (j <= i)
                        ++c;
            cnt[q] = c + (hasc[q] ? r1[q] - r0[q] : 0);
        }
    }
};

// Canonical entry index: (i, j <= i) -> i(i+1)/2 + j; c_i -> s(s+1)/2 + i.
__host__ __device__ constexpr int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }

template <typename T, int RPL>
struct VecT;
template <>
struct VecT<double, 1> {
    using t = double;
};
template <>
struct VecT<double, 2> {
    using t = double2;
};
template <>
struct VecT<float, 2> {
    using t = float2;
};
template <>
struct VecT<float, 4> {
    using t = float4;
};

// Non-temporal load of RPL consecutive values (data read once per launch).
template <typename T, int RPL>
__device__ __forceinline__ typename VecT<T, RPL>::t nt_load(const T *p)
{
    if constexpr (RPL == 1) {
        return __builtin_nontemporal_load(p);
    } else {
        using NV = T __attribute__((ext_vector_type(RPL)));
        const NV v = __builtin_nontemporal_load(reinterpret_cast<const NV *>(p));
        typename VecT<T, RPL>::t r;
        r.x = v[0];
        r.y = v[1];
        if constexpr (RPL == 4) {
            r.z = v[2];
            r.w = v[3];
        }
        return r;
    }
}

template <typename T, int RPL>
__device__ __forceinline__ T lanepart(const typename VecT<T, RPL>::t &v, int r)
{
    if constexpr (RPL == 1)
        return v;
    else if constexpr (RPL == 2)
        return r == 0 ? v.x : v.y;
    else
        return r == 0 ? v.x : r == 1 ? v.y : r == 2 ? v.z : v.w;
}

// Rows SPL of group G for the RPL rows starting at m (no guard: rows past the
// end of the matrix are zero padding).
template <typename T, int S, int G, int RPL, bool WD>
__device__ __forceinline__ void gram_rows(const T *__restrict__ P, const T *__restrict__ AP,
                                          const T *__restrict__ dvec, int64_t cs, int64_t m, T *acc)
{
    constexpr GramPlan<S> pl{};
    using V = typename VecT<T, RPL>::t;
    constexpr int R0 = pl.r0[G], R1 = pl.r1[G], C0 = pl.c0[G], C1 = pl.c1[G];
    constexpr bool HC = pl.hasc[G];
    V ap[C1 - C0];
#pragma unroll
    for (int j = C0; j < C1; ++j)  // P and AP are read once per launch: non-temporal loads
        ap[j - C0] = nt_load<T, RPL>(AP + j * cs + m);
    V w{};
    if constexpr (HC) {
        w = *reinterpret_cast<const V *>(P + m);
        if constexpr (WD) {
            const V dv = *reinterpret_cast<const V *>(dvec + m);
            if constexpr (RPL == 1) {
                w *= dv;
            } else {
                w.x *= dv.x;
                w.y *= dv.y;
                if constexpr (RPL == 4) {
                    w.z *= dv.z;
                    w.w *= dv.w;
                }
            }
        }
    }
    int a = 0;
#pragma unroll
    for (int i = R0; i < R1; ++i) {
        const V p = nt_load<T, RPL>(P + i * cs + m);
#pragma unroll
        for (int j = C0; j < C1; ++j) {
            if (j <= i) {
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    acc[a] += lanepart<T, RPL>(p, r) * lanepart<T, RPL>(ap[j - C0], r);
                ++a;
            }
        }
        if constexpr (HC) {
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                acc[a] += lanepart<T, RPL>(p, r) * lanepart<T, RPL>(w, r);
            ++a;
        }
    }
}

// Wave reduction of the group's accumulators and store of one partial each.
template <typename T, int S, int G>
__device__ __forceinline__ void gram_store(const T *acc, double *__restrict__ gpart, int64_t estride, int64_t slot)
{
    constexpr GramPlan<S> pl{};
    const int lane = threadIdx.x % kWave;
    int a = 0;
#pragma unroll
    for (int i = pl.r0[G]; i < pl.r1[G]; ++i) {
#pragma unroll
        for (int j = pl.c0[G]; j < pl.c1[G]; ++j) {
            if (j <= i) {
                const T v = wave_sum(acc[a]);
                if (lane == a % kWave)
                    gpart[static_cast<int64_t>(tri_index(i, j)) * estride + slot] = static_cast<double>(v);
                ++a;
            }
        }
        if (pl.hasc[G]) {
            const T v = wave_sum(acc[a]);
            if (lane == a % kWave)
                gpart[static_cast<int64_t>(S * (S + 1) / 2 + i) * estride + slot] = static_cast<double>(v);
            ++a;
        }
    }
}

// Group G over rows [beg, end) in slabs of SL rows taken every `stride`
// rows (contiguous schedule: one slab, SL = end - beg).  beg, SL and stride
// are multiples of 64 * RPL.
template <typename T, int S, int G, int RPL, bool WD>
__device__ __forceinline__ void gram_group(const T *__restrict__ P, const T *__restrict__ AP,
                                           const T *__restrict__ dvec, int64_t cs, int64_t beg, int64_t end,
                                           int64_t SL, int64_t stride, double *__restrict__ gpart, int64_t estride,
                                           int64_t slot)
{
    constexpr GramPlan<S> pl{};
    constexpr int NA = pl.cnt[G];
    const int lane = threadIdx.x % kWave;
    T acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
        acc[a] = T(0);
    constexpr int STEP = kWave * RPL;
    for (int64_t s0 = beg; s0 < end; s0 += stride) {
        const int64_t e0 = s0 + SL < end ? s0 + SL : end;
        for (int64_t base = s0; base < e0; base += STEP)
            gram_rows<T, S, G, RPL, WD>(P, AP, dvec, cs, base + lane * RPL, acc);
    }
    gram_store<T, S, G>(acc, gpart, estride, slot);
}

template <typename T, int S, int RPL, bool WD, int G>
__device__ __forceinline__ void gram_dispatch(int w, const T *P, const T *AP, const T *dvec, int64_t cs, int64_t beg,
                                              int64_t end, int64_t SL, int64_t stride, double *gpart,
                                              int64_t estride, int64_t slot)
{
    if constexpr (G < GramPlan<S>::NG) {
        if (w == G)
            gram_group<T, S, G, RPL, WD>(P, AP, dvec, cs, beg, end, SL, stride, gpart, estride, slot);
        else
            gram_dispatch<T, S, RPL, WD, G + 1>(w, P, AP, dvec, cs, beg, end, SL, stride, gpart, estride, slot);
    }
}

// The whole block's share (wave w owns group w).
template <typename T, int S, int RPL, bool WD>
__device__ __forceinline__ void gram_tile(const T *P, const T *AP, const T *dvec, int64_t cs, int64_t beg,
                                          int64_t end, int64_t SL, int64_t stride, double *gpart, int64_t estride,
                                          int64_t slot)
{
    gram_dispatch<T, S, RPL, WD, 0>(static_cast<int>(threadIdx.x / kWave), P, AP, dvec, cs, beg, end, SL, stride,
                                    gpart, estride, slot);
}

// Rows per lane: 16-byte loads, except FP64 with 16 waves per block (s > 24),
// whose 128-register budget per lane leaves room for single-row loads only.
template <typename T, int S>
constexpr int gram_rpl()
{
    return sizeof(T) == 8 ? (GramPlan<S>::NG <= 9 ? 2 : 1) : 4;
}

// Single system: rows [0, rows) with rows a multiple of 256 (zero padding).
//   contiguous: block b owns [b*chunk, (b+1)*chunk)
//   strided:    block b owns slabs [b*SL + q*nbg*SL, ... + SL)
template <typename T, int S, bool WD>
__global__ __launch_bounds__(kWave * GramPlan<S>::NG) void k_gram(const DevState *__restrict__ st,
                                                                  const T *__restrict__ P, const T *__restrict__ AP,
                                                                  const T *__restrict__ dvec, int64_t ld,
                                                                  int64_t rows, int64_t chunk, int64_t slab,
                                                                  double *__restrict__ gpart, int nbg)
{
    if (st->done)
        return;
    const int64_t b = blockIdx.x;
    if (slab > 0) {  // strided
        gram_tile<T, S, gram_rpl<T, S>(), WD>(P, AP, dvec, ld, b * slab, rows, slab, int64_t(nbg) * slab, gpart, nbg,
                                           b);
    } else {  // contiguous
        const int64_t beg = b * chunk;
        const int64_t end = beg + chunk < rows ? beg + chunk : rows;
        gram_tile<T, S, gram_rpl<T, S>(), WD>(P, AP, dvec, ld, beg, end, end - beg, end - beg + 1, gpart, nbg, b);
    }
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
        hipLaunchKernelGGL((k_gram<T, S, true>), dim3(a.nbg), block, 0, st, a.st, P, AP, dv, a.ld, a.ld, a.gchunk,
                           a.gslab, a.gpart, a.nbg);
    else
        hipLaunchKernelGGL((k_gram<T, S, false>), dim3(a.nbg), block, 0, st, a.st, P, AP, dv, a.ld, a.ld, a.gchunk,
                           a.gslab, a.gpart, a.nbg);
    return hipGetLastError();
}

}  // namespace sstep
