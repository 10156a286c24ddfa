// Gram reduction for 7-point stencil operators that applies the operator on
// the fly: G_raw = P^T (A P) (lower triangle) and c' = P^T W, with the
// products A p_j formed from P inside the kernel instead of being read from a
// stored AP (Sec. 2: G = P^T A P).  The basis steps then write only P, and
// the last basis product (A p_{s-1}) is not launched at all, so one outer
// iteration moves w(5s - 3) + 32 bytes per unknown instead of w(7s - 2) + 32.
//
// Design (gfx950, wave64, FP64 or FP32, s <= 16):
//  * A block owns work items (in-plane tile, z-range): a tile of TX x TY =
//    32 x 8 grid points (thread = point) marched upwards through the
//    planes of the range.  Planes z-1, z and z+1 of every column of the
//    thread's point are kept in registers, so the interior of each plane of P
//    is read from HBM once per range (plus two planes of priming).
//  * Each z-step is branch-free: at its start every thread issues the loads
//    of plane z+1 of its point for all columns and its share of the tile's
//    halo ring of plane z (the 2(TX + TY) in-plane neighbours outside the
//    tile, zero outside the grid); addresses are clamped in range and unused
//    values selected away.  Then (1) the plane-z interior and halo ring go to a
//    padded (TX + 2) x (TY + 2) LDS tile per column; (2) every thread forms
//    y_j = (A p_j)(z) from the LDS tile and its registers and writes it to LDS;
//    (3) each wave accumulates its Gram group (the block decomposition of
//    gram_impl.h) over the 256 points from LDS.
//  * s <= 8 has a single group: every wave takes it over its own 64 points
//    and stores its own partial (four slots per block).  9 <= s <= 16 has four
//    groups, one per wave, each over all 256 points.
//  * The per-wave body is a template on the group, entered once through a
//    wave-uniform branch; every wave executes the same number of barriers.
//  * Partials are reduced in a fixed order by the FGS kernel, as for the
//    stored-AP Gram, so results are bitwise reproducible from run to run.
#pragma once

#include "gram_impl.h"

namespace sstep {

constexpr int kGoThreads = 256;  // points per tile = threads per block
constexpr int kGoTxl = 5;                          // tile width log2
constexpr int kGoTx = 1 << kGoTxl;                 // 32
constexpr int kGoTy = kGoThreads >> kGoTxl;        // 8
constexpr int kGoTx2 = kGoTx + 2;                  // padded row pitch
constexpr int kGoPitch = kGoTx2 * (kGoTy + 2);     // padded tile: 340 points
constexpr int kGoRing = 2 * (kGoTx + kGoTy);       // halo ring: 80 points

// 7-point constant Poisson: (A p)_c = 6 p_c - sum of the six neighbours, in
// the same order of operations as the basis kernels.
template <typename T>
struct GoPoisson {
    struct Coef {};
    __device__ __forceinline__ Coef load(const Grid3 &, uint32_t, uint32_t, int64_t) const { return {}; }
    __device__ __forceinline__ static T y(const Coef &, T pc, T w, T e, T s, T n, T b, T t)
    {
        return T(6) * pc - (((((w + e) + s) + n) + b) + t);
    }
};

// 7-point face-coefficient operator: (A p)_c = sum_f k_f (p_c - p_q), same
// order as the basis kernels.  Face arrays as in the operator description:
// kx (nx+1) x ny x nz, ky nx x (ny+1) x nz, kz nx x ny x (nz+1), x fastest.
template <typename T>
struct GoFaces {
    const T *__restrict__ kx;
    const T *__restrict__ ky;
    const T *__restrict__ kz;
    struct Coef {
        T fw, fe, fs, fn, fb, ft;
    };
    // Point c = i + nx*j + nxy*k with row index r = j + ny*k.
    __device__ __forceinline__ Coef load(const Grid3 &g, uint32_t r, uint32_t k, int64_t c) const
    {
        const int64_t fx = c + r;
        const int64_t fy = c + static_cast<int64_t>(k) * g.nx;
        return Coef{kx[fx], kx[fx + 1], ky[fy], ky[fy + g.nx], kz[c], kz[c + g.nxy]};
    }
    __device__ __forceinline__ static T y(const Coef &f, T pc, T w, T e, T s, T n, T b, T t)
    {
        return f.fw * (pc - w) + f.fe * (pc - e) + f.fs * (pc - s) + f.fn * (pc - n) + f.fb * (pc - b) +
               f.ft * (pc - t);
    }
};

// Launch geometry: 32 x 8 tiles, nzb z-ranges of zr planes; items =
// tiles_x * tiles_y * nzb, distributed over the blocks item = blockIdx.x +
// k * gridDim.x.
struct GoGeom {
    int32_t tiles_x, tiles_y;
    int32_t zr, nzb;
    int32_t items;
};

// Load at a wave-uniform base plus a 32-bit per-lane byte offset, which maps
// to the scalar-base addressing mode and keeps 64-bit addresses out of the
// vector registers (each column is under 4 GiB).
template <typename T>
__device__ __forceinline__ T go_ld(const T *base, uint32_t byte_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// 16 x 16 x 4 matrix-core step, D += A B: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; result register r (0..3) of lane l holds D[row][l % 16]
// with row = 4 r + l / 16 for FP64 (four groups of one row) and
// row = 4 (l / 16) + r for FP32 (one group of four rows).
template <typename T>
struct GoMfma;
template <>
struct GoMfma<double> {
    using acc_t = __attribute__((ext_vector_type(4))) double;
    __device__ __forceinline__ static acc_t step(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct GoMfma<float> {
    using acc_t = __attribute__((ext_vector_type(4))) float;
    __device__ __forceinline__ static acc_t step(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <class Rule, typename T, int S, bool WD>
__global__ __launch_bounds__(kGoThreads) void k_gram_op(const DevState *__restrict__ st, Grid3 g, Rule rule,
                                                        const T *__restrict__ P, int64_t ld,
                                                        const T *__restrict__ dvec, GoGeom geo,
                                                        double *__restrict__ gpart, int estride)
{
    static_assert(S >= 1 && S <= kGoMaxS, "the 16 x 16 matrix-core tile holds at most 16 columns");
    constexpr int E = S * (S + 1) / 2 + S;                             // Gram entries + right-hand side
    constexpr int NH = (kGoRing * S + kGoThreads - 1) / kGoThreads;  // halo entries per thread
    constexpr uint32_t W = sizeof(T);
    constexpr int txw = kGoTx, tyh = kGoTy, tx2 = kGoTx2, pitch = kGoPitch, ring = kGoRing;
    using M = GoMfma<T>;
    __shared__ T Pt[S * kGoPitch];
    __shared__ T APt[S][kGoThreads];
    static_assert(sizeof(APt) >= sizeof(double) * (kGoThreads / kWave) * E, "reduction buffer fits in APt");
    if (st->done)
        return;
    const int t = threadIdx.x;
    const int lane = t % kWave, wv = t / kWave;
    const int lx = t & (txw - 1), ly = t >> kGoTxl;
    const int pos = (ly + 1) * tx2 + lx + 1;  // this thread's point in the padded tile
    const uint32_t pb = static_cast<uint32_t>(g.nxy) * W;  // bytes per plane
    // matrix-core operands of this lane: column mc of P / AP at point 4 kc + lane / 16
    const int mc = lane & 15;
    const bool mcol = mc < S;

    typename M::acc_t gacc = {};  // this wave's share of G_raw
    T cacc[S];                    // this thread's share of c' = P^T W
#pragma unroll
    for (int c = 0; c < S; ++c)
        cacc[c] = T(0);

    const int tiles = geo.tiles_x * geo.tiles_y;
    for (int item = blockIdx.x; item < geo.items; item += gridDim.x) {
        const int tile = item % tiles, zb = item / tiles;
        const int i0 = (tile % geo.tiles_x) * txw, j0 = (tile / geo.tiles_x) * tyh;
        const uint32_t i = static_cast<uint32_t>(i0 + lx), j = static_cast<uint32_t>(j0 + ly);
        const bool valid = i < static_cast<uint32_t>(g.nx) && j < static_cast<uint32_t>(g.ny);
        const int z0 = zb * geo.zr;
        const int z1 = z0 + geo.zr < g.nz ? z0 + geo.zr : g.nz;
        // points outside the grid address point (0, 0, k): in range, values unused
        const uint32_t q = valid ? i + static_cast<uint32_t>(g.nx) * j : 0u;
        const uint32_t jr = valid ? j : 0u;

        // Loads for z-step kk, issued one step ahead: plane kk+1 of the point
        // (zp), the halo ring of plane kk (hv; entry h < ring * S of the
        // block: column h / ring, ring position h % ring = bottom row, top
        // row, left column, right column), the operator coefficients (f) and
        // the M-diagonal (dv) of the point.
        T zm[S], zc[S], zp[S];
        T hv[NH];
        typename Rule::Coef f{};
        T dv = T(0);
        auto issue = [&](int kk) {
            const int64_t cidx = static_cast<int64_t>(q) + static_cast<int64_t>(kk) * g.nxy;
            const uint32_t o = static_cast<uint32_t>(cidx) * W;
            const uint32_t op = valid && kk + 1 < g.nz ? o + pb : o;
#pragma unroll
            for (int m = 0; m < NH; ++m) {
                const int h = t + m * kGoThreads;
                const int c = h / ring, r = h - c * ring;
                const int hx = r < txw ? r : r < 2 * txw ? r - txw : r < 2 * txw + tyh ? -1 : txw;
                const int hy = r < txw ? -1 : r < 2 * txw ? tyh : r < 2 * txw + tyh ? r - 2 * txw : r - 2 * txw - tyh;
                const int gi = i0 + hx, gj = j0 + hy;
                const bool in = c < S && gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
                const int64_t e = in ? static_cast<int64_t>(c) * ld + gi + static_cast<int64_t>(g.nx) * gj +
                                           static_cast<int64_t>(kk) * g.nxy
                                     : 0;
                hv[m] = P[e];
            }
            // keep the halo loads first: loads complete in issue order, so the
            // halo can be stored while the plane loads are still in flight
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < S; ++c)
                zp[c] = go_ld(P + c * ld, op);
            f = rule.load(g, jr + static_cast<uint32_t>(g.ny) * static_cast<uint32_t>(kk), static_cast<uint32_t>(kk),
                          cidx);
            if constexpr (WD)
                dv = go_ld(dvec, o);
        };
        {
            const uint32_t o = (q + static_cast<uint32_t>(z0) * static_cast<uint32_t>(g.nxy)) * W;
            const uint32_t om = valid && z0 > 0 ? o - pb : o;
#pragma unroll
            for (int c = 0; c < S; ++c) {
                const T *col = P + c * ld;
                const T vm = go_ld(col, om), vc = go_ld(col, o);
                zm[c] = valid && z0 > 0 ? vm : T(0);
                zc[c] = valid ? vc : T(0);
            }
        }
        issue(z0);
        for (int k = z0; k < z1; ++k) {
            const bool ht = valid && k + 1 < g.nz;
            // (1) plane k: interior and halo ring into the padded tiles.
#pragma unroll
            for (int c = 0; c < S; ++c)
                Pt[c * pitch + pos] = zc[c];
#pragma unroll
            for (int m = 0; m < NH; ++m) {
                const int h = t + m * kGoThreads;
                const int c = h / ring, r = h - c * ring;
                const int hx = r < txw ? r : r < 2 * txw ? r - txw : r < 2 * txw + tyh ? -1 : txw;
                const int hy = r < txw ? -1 : r < 2 * txw ? tyh : r < 2 * txw + tyh ? r - 2 * txw : r - 2 * txw - tyh;
                const int gi = i0 + hx, gj = j0 + hy;
                const bool in = gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
                if (c < S)
                    Pt[c * pitch + (hy + 1) * tx2 + hx + 1] = in ? hv[m] : T(0);
            }
            __syncthreads();
            // (2) right-hand side c'_i += p_i w at this point, products
            // y_j = (A p_j)(k) into LDS, then the loads of step k + 1.
            const T w = WD ? zc[0] * dv : zc[0];
            const typename Rule::Coef fk = f;
#pragma unroll
            for (int c = 0; c < S; ++c) {
                cacc[c] += zc[c] * w;
                const T *L = Pt + c * pitch + pos;
                const T zpv = ht ? zp[c] : T(0);
                const T y = Rule::y(fk, zc[c], L[-1], L[1], L[-tx2], L[tx2], zm[c], zpv);
                APt[c][t] = valid ? y : T(0);
                zm[c] = zc[c];
                zc[c] = zpv;
                if ((c & 3) == 3)
                    __builtin_amdgcn_sched_barrier(0);  // bounds the LDS reads in flight (registers)
            }
            if (k + 1 < z1)
                issue(k + 1);
            __syncthreads();
            // (3) G_raw += P^T (A P) over this wave's 64 points, 4 at a time.
#pragma unroll 4
            for (int kc = 0; kc < kWave / 4; ++kc) {
                const int pt = wv * kWave + 4 * kc + (lane >> 4);
                const int ppos = ((pt >> kGoTxl) + 1) * tx2 + (pt & (txw - 1)) + 1;
                const int cc = mcol ? mc : 0;
                const T a = Pt[cc * pitch + ppos];
                const T b = APt[cc][pt];
                gacc = M::step(mcol ? a : T(0), mcol ? b : T(0), gacc);
            }
            __syncthreads();
        }
    }

    // Block reduction in a fixed order: wave partials into LDS (reusing APt),
    // then entry e of the block = sum over the four waves.
    double *red = reinterpret_cast<double *>(&APt[0][0]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = M::row(lane, r), n = mc;
        if (m < S && n <= m)
            red[wv * E + tri_index(m, n)] = static_cast<double>(gacc[r]);
    }
#pragma unroll
    for (int c = 0; c < S; ++c) {
        const T v = wave_sum(cacc[c]);
        if (lane == c)
            red[wv * E + S * (S + 1) / 2 + c] = static_cast<double>(v);
    }
    __syncthreads();
    for (int e = t; e < E; e += kGoThreads)
        gpart[static_cast<int64_t>(e) * estride + blockIdx.x] = ((red[e] + red[E + e]) + red[2 * E + e]) + red[3 * E + e];
}

template <typename T, int S>
hipError_t gram_op_launch_s(const IterArgs &a, hipStream_t st)
{
    const GoGeom geo{a.go_tiles_x, a.go_tiles_y, a.go_zr, a.go_nzb, a.go_items};
    const dim3 grid(static_cast<uint32_t>(a.go_blocks)), block(kGoThreads);
    const T *P = static_cast<const T *>(a.P);
    const int estride = a.nbg;
    if (a.op.kind == kOpPoisson) {
        hipLaunchKernelGGL((k_gram_op<GoPoisson<T>, T, S, false>), grid, block, 0, st, a.st, a.op.g, GoPoisson<T>{},
                           P, a.ld, static_cast<const T *>(nullptr), geo, a.gpart, estride);
    } else {
        GoFaces<T> rule;
        const T *dv;
        if constexpr (sizeof(T) == 8) {
            rule = GoFaces<T>{a.op.kx, a.op.ky, a.op.kz};
            dv = a.op.dvec;
        } else {
            rule = GoFaces<T>{a.op.kx32, a.op.ky32, a.op.kz32};
            dv = a.op.dvec32;
        }
        if (a.wdvec)
            hipLaunchKernelGGL((k_gram_op<GoFaces<T>, T, S, true>), grid, block, 0, st, a.st, a.op.g, rule, P, a.ld,
                               dv, geo, a.gpart, estride);
        else
            hipLaunchKernelGGL((k_gram_op<GoFaces<T>, T, S, false>), grid, block, 0, st, a.st, a.op.g, rule, P, a.ld,
                               dv, geo, a.gpart, estride);
    }
    return hipGetLastError();
}

hipError_t gram_op_launch_1_8(const IterArgs &a, hipStream_t st);
hipError_t gram_op_launch_9_16(const IterArgs &a, hipStream_t st);

}  // namespace sstep
