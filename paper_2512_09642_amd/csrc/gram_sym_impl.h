// M-weighted Gram of the s + 1 basis columns for the recurrence Gram kind,
// s <= 31:  H = P^T M P over p_0 .. p_s (lower triangle) and the right-hand
// side entries c'_i = p_i^T W (W = M p_0 or p_0), as per-block partials.  The
// FGS kernel turns H into G_raw = P^T (A P) through the basis recurrence
// (fgs_core.h, k_fgs_rec).
//
// Design (gfx950, wave64): H is a sum of outer products p p^T over the rows,
// which is what the 16 x 16 x 4 matrix-core step computes when lane l feeds
// A[l % 16][l / 16] = p_c(row) and B[l / 16][l % 16] = w(row) p_c(row) with
// c = l % 16: the same value in both operands, so each lane loads one column
// at its rows and nothing is transposed.  Lane l holds column c at 4
// consecutive rows (two 16-byte loads; the 4 lanes of a column cover one
// 128-byte line), i.e. a wave covers 16 rows of the first 16 columns per
// step, and four matrix-core steps consume them.  Column 16 (p_s at s = 16)
// and the right-hand side accumulate with vector FMAs; p_0 at a row comes
// from the column-0 lane of the same 16-lane row by a DPP broadcast.  No LDS
// and no barrier in the main loop and few registers, so many waves per SIMD
// keep many loads in flight: the kernel streams s + 1 columns (plus the M
// diagonal for non-constant diagonals) once.
#pragma once

#include "gram_op_impl.h"

namespace sstep {

constexpr int kGsThreads = 256;
constexpr int kGsRowsPerWave = 16;  // rows per wave per step
constexpr int kGsRowsPerStep = kGsRowsPerWave * (kGsThreads / kWave);

template <typename T>
struct Vec4 {
    T v[4];
};

// Four consecutive values at p (16-byte aligned: row offsets are multiples of
// 4 and columns start on 256-row boundaries), non-temporal: read once.
template <typename T>
__device__ __forceinline__ Vec4<T> ld4(const T *p)
{
    Vec4<T> r;
    if constexpr (sizeof(T) == 8) {
        using V2 = double __attribute__((ext_vector_type(2)));
        const V2 a = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(p));
        const V2 b = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(p) + 1);
        r.v[0] = a[0], r.v[1] = a[1], r.v[2] = b[0], r.v[3] = b[1];
    } else {
        using V4 = float __attribute__((ext_vector_type(4)));
        const V4 a = __builtin_nontemporal_load(reinterpret_cast<const V4 *>(p));
        r.v[0] = a[0], r.v[1] = a[1], r.v[2] = a[2], r.v[3] = a[3];
    }
    return r;
}

// S1 = s + 1 <= 32 columns: block A = columns 0..15 on the matrix cores; for
// S1 = 17 column 16 with vector FMAs; for S1 >= 18 block B = columns 16..S1-1
// as a second lane column (lane c also loads p_{16+c}) with two more
// matrix-core products per step, H[B][A] and H[B][B].  WAP: weight the second
// operand by the M diagonal array (non-constant diagonal); WD: the
// right-hand side uses W = M p_0.
//
// One block's share: rows [beg, end) of the columns P + j cs (j = 0..S1-1,
// 16-byte aligned, rows multiples of 4, zero past the system), the block's
// partial of entry e written to out[e * estride + slot].  Ends with a
// barrier, so a block may call it again for another range.
template <typename T, int S1, bool WAP, bool WD>
__device__ __forceinline__ void gram_sym_rows(const T *__restrict__ P, int64_t cs, const T *__restrict__ dvec,
                                              int64_t beg, int64_t end, double *__restrict__ out, int64_t estride,
                                              int64_t slot)
{
    static_assert(S1 >= 2 && S1 <= 32, "recurrence Gram: s + 1 <= 32 columns");
    constexpr int SM = S1 < 16 ? S1 : 16;  // columns of block A
    constexpr bool XC = S1 == 17;          // column 16 with vector FMAs
    constexpr bool TWO = S1 > 17;          // block B on the matrix cores
    constexpr int SB = TWO ? S1 - 16 : 0;
    constexpr int E = S1 * (S1 + 1) / 2 + S1;
    constexpr int T0 = S1 * (S1 + 1) / 2;
    using M = GoMfma<T>;
    __shared__ double red[kGsThreads / kWave][E];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int c = lane & 15, gq = lane >> 4;
    const bool ccol = c < SM, bcol = c < SB;
    const T *colp = P + static_cast<int64_t>(ccol ? c : 0) * cs;
    const T *colb = P + static_cast<int64_t>(16 + (bcol ? c : 0)) * cs;  // dereferenced only for S1 >= 18
    const T *xcol = P + 16 * cs;                                         // dereferenced only for S1 == 17

    typename M::acc_t gacc = {}, bacc = {}, bbacc = {};
    T cacc = T(0), cbacc = T(0), hx = T(0), hxx = T(0), cx = T(0);
    for (int64_t r0 = beg + wv * kGsRowsPerWave; r0 < end; r0 += kGsRowsPerStep) {
        const int64_t row = r0 + 4 * gq;
        const Vec4<T> p = ccol ? ld4(colp + row) : Vec4<T>{};
        Vec4<T> w{}, px{}, pb{};
        if constexpr (WAP || WD)
            w = ld4(dvec + row);
        if constexpr (XC)
            px = ld4(xcol + row);
        if constexpr (TWO)
            pb = bcol ? ld4(colb + row) : Vec4<T>{};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const T a = p.v[t];
            T b = a;
            if constexpr (WAP)
                b *= w.v[t];
            gacc = M::step(a, b, gacc);  // H[A][A]
            T w0 = go_row_bcast0(a);     // p_0 at this row
            if constexpr (WD)
                w0 *= w.v[t];
            cacc += a * w0;
            if constexpr (TWO) {
                const T ab = pb.v[t];
                T bb = ab;
                if constexpr (WAP)
                    bb *= w.v[t];
                bacc = M::step(ab, b, bacc);    // H[B][A]
                bbacc = M::step(ab, bb, bbacc);  // H[B][B]
                cbacc += ab * w0;
            }
            if constexpr (XC) {
                T xw = px.v[t];
                if constexpr (WAP)
                    xw *= w.v[t];
                hx += a * xw;  // H[16][c]
                if (c == 0) {
                    hxx += px.v[t] * xw;  // H[16][16]
                    cx += px.v[t] * w0;   // c'_16
                }
            }
        }
    }

    // per wave: the H blocks, c', column 16 into LDS; then the block's fixed-order sum
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = M::row(lane, r);
        if (i < SM && c <= i)
            red[wv][tri_index(i, c)] = static_cast<double>(gacc[r]);
        if constexpr (TWO) {
            if (i < SB) {
                red[wv][tri_index(16 + i, c)] = static_cast<double>(bacc[r]);
                if (c <= i)
                    red[wv][tri_index(16 + i, 16 + c)] = static_cast<double>(bbacc[r]);
            }
        }
    }
    auto quad = [&](T v) {  // sum over the four lanes c, c + 16, c + 32, c + 48
        v += __shfl_xor(v, 16, kWave);
        v += __shfl_xor(v, 32, kWave);
        return v;
    };
    const T csum = quad(cacc);
    if (lane < SM)
        red[wv][T0 + lane] = static_cast<double>(csum);
    if constexpr (TWO) {
        const T cb = quad(cbacc);
        if (lane < SB)
            red[wv][T0 + 16 + lane] = static_cast<double>(cb);
    }
    if constexpr (XC) {
        const T hs = quad(hx), hxs = quad(hxx), cxs = quad(cx);
        if (lane < 16)
            red[wv][tri_index(16, lane)] = static_cast<double>(hs);
        if (lane == 0) {
            red[wv][tri_index(16, 16)] = static_cast<double>(hxs);
            red[wv][T0 + 16] = static_cast<double>(cxs);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < E; e += kGsThreads)
        out[static_cast<int64_t>(e) * estride + slot] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    __syncthreads();
}

template <typename T, int S1, bool WAP, bool WD>
__global__ __launch_bounds__(kGsThreads) void k_gram_sym(const DevState *__restrict__ st, const T *__restrict__ P,
                                                          int64_t ld, const T *__restrict__ dvec, int64_t chunk,
                                                          double *__restrict__ gpart, int estride)
{
    if (st->done)
        return;
    const int64_t beg = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t end = beg + chunk < ld ? beg + chunk : ld;
    gram_sym_rows<T, S1, WAP, WD>(P, ld, dvec, beg, end, gpart, estride, blockIdx.x);
}

template <typename T, int S>
hipError_t gram_sym_launch_s(const IterArgs &a, hipStream_t st)
{
    constexpr int S1 = S + 1;
    const T *P = static_cast<const T *>(a.P);
    const T *dv = reinterpret_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(a.op.dvec)
                                                             : static_cast<const void *>(a.op.dvec32));
    const dim3 grid(static_cast<uint32_t>(a.nbg)), block(kGsThreads);
    if (a.rec_wap && a.wdvec)
        hipLaunchKernelGGL((k_gram_sym<T, S1, true, true>), grid, block, 0, st, a.st, P, a.ld, dv, a.gchunk, a.gpart,
                           a.nbg);
    else if (a.rec_wap)
        hipLaunchKernelGGL((k_gram_sym<T, S1, true, false>), grid, block, 0, st, a.st, P, a.ld, dv, a.gchunk,
                           a.gpart, a.nbg);
    else if (a.wdvec)
        hipLaunchKernelGGL((k_gram_sym<T, S1, false, true>), grid, block, 0, st, a.st, P, a.ld, dv, a.gchunk,
                           a.gpart, a.nbg);
    else
        hipLaunchKernelGGL((k_gram_sym<T, S1, false, false>), grid, block, 0, st, a.st, P, a.ld, dv, a.gchunk,
                           a.gpart, a.nbg);
    return hipGetLastError();
}

}  // namespace sstep
