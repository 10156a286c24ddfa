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
//  * Lane l of a wave owns column l % 16 at 16 points of the tile and keeps
//    planes z-1, z (and z+1, loaded one step ahead into alternating buffers)
//    of those points in registers.  Each z-step: (1) plane z of every column
//    (lane points plus the tile's halo ring, the 2(TX + TY) in-plane
//    neighbours outside the tile, zero outside the grid) goes into a padded
//    (TX + 2) x (TY + 2) LDS tile; (2) each lane forms (A p_n)(z) at its points
//    from the tile and its registers and feeds p_n and (A p_n) to the 16 x 16
//    x 4 matrix-core step, which accumulates the wave's P^T (A P) over its 64
//    points; c'_n = p_n^T W accumulates with vector FMAs.  A lane's points
//    come in vertical pairs, so one y-neighbour is in its own registers, and
//    p_0 at a point comes from the column-0 lane of the same row by a DPP
//    broadcast: three LDS reads per point.  No branch surrounds the loads, so
//    the compiler's waits for them are exact.
//  * Full tiles and edge tiles go to two launches; the full-tile kernel has no
//    per-point selects and fits two waves per SIMD.  Blocks take tiles in an
//    XCD-contiguous order, so neighbouring tiles share an L2.
//  * The four wave partials are summed in a fixed order in LDS, one slot per
//    block, and the slots in a fixed order by the partial-sum kernel that
//    precedes the FGS solve, so results are bitwise reproducible from run to
//    run.
#pragma once

#include "gram_impl.h"

namespace sstep {

constexpr int kGoThreads = 256;  // points per tile = threads per block
constexpr int kGoTxl = 5;                          // tile width log2
constexpr int kGoTx = 1 << kGoTxl;                 // 32
constexpr int kGoTy = kGoThreads >> kGoTxl;        // 8
constexpr int kGoTx2 = kGoTx + 2;                  // padded row pitch
constexpr int kGoPitch = kGoTx2 * (kGoTy + 2);     // padded tile: 340 points

// 7-point constant Poisson: (A p)_c = 6 p_c - sum of the six neighbours, in
// the same order of operations as the basis kernels.
template <typename T>
struct GoPoisson {
    static constexpr bool kHasCoef = false;
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
    static constexpr bool kHasCoef = true;
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

// Launch geometry.  The 32 x 8 tiles of a plane split into the full tiles
// (tx < fx, ty < fy with fx = nx / 32, fy = ny / 8), taken by one launch,
// and the edge tiles (the column strip tx = fx when nx % 32 != 0, then the
// row strip ty = fy, tx < fx, when ny % 8 != 0), taken by another.  nzb
// z-ranges of zr planes; items = tiles * nzb (tile fastest), distributed over
// the logical blocks item = lb + k * blocks; partial slots slot0 + lb.
struct GoGeom {
    int32_t fx, fy;        // full tiles per row / column
    int32_t tiles_y;       // tile rows (full and edge)
    int32_t rx, ry;        // 1 when the column / row edge strip exists
    int32_t tiles;         // tiles of this launch
    int32_t zr, nzb;
    int32_t items;
    int32_t blocks;  // logical blocks (partial slots)
    int32_t per;     // logical blocks per XCD
    int32_t slot0;   // first partial slot of this launch
};

// Load at a wave-uniform base plus a 32-bit per-lane byte offset, which maps
// to the scalar-base addressing mode and keeps 64-bit addresses out of the
// vector registers (each column is under 4 GiB).
template <typename T>
__device__ __forceinline__ T go_ld(const T *base, uint32_t byte_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Value of lane 16 (l / 16) (the first lane of l's row of 16), by a DPP row
// broadcast: two 32-bit moves for a double, no LDS traffic.
constexpr int kDppRowNewBcast0 = 0x150;  // DPP control: row_newbcast:0
__device__ __forceinline__ float go_row_bcast0(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), kDppRowNewBcast0, 0xf, 0xf,
                                                              true));
}
__device__ __forceinline__ double go_row_bcast0(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<uint32_t>(u)), kDppRowNewBcast0, 0xf, 0xf, true));
    const uint32_t hi = static_cast<uint32_t>(
        __builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<uint32_t>(u >> 32)), kDppRowNewBcast0, 0xf, 0xf, true));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
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

// FULL: the launch over the full tiles; without the edge-tile selects its
// registers fit two waves per SIMD (constant Poisson, or FP32), which lets
// the two blocks on a CU hide each other's memory waits.  Otherwise the edge
// tiles, and FP64 face operators (their per-point coefficients would spill).
template <class Rule, typename T, int S, bool WD, bool FULL>
constexpr int go_waves_per_simd()
{
    return FULL && (sizeof(T) == 4 || !Rule::kHasCoef) ? 2 : 1;
}

template <class Rule, typename T, int S, bool WD, bool FULL>
__global__ __launch_bounds__(kGoThreads, (go_waves_per_simd<Rule, T, S, WD, FULL>())) void k_gram_op(
    const DevState *__restrict__ st, Grid3 g, Rule rule,
                                                        const T *__restrict__ P, int64_t ld,
                                                        const T *__restrict__ dvec, GoGeom geo,
                                                        double *__restrict__ gpart, int estride)
{
    static_assert(S >= 1 && S <= kGoMaxS, "the 16 x 16 matrix-core tile holds at most 16 columns");
    constexpr int E = S * (S + 1) / 2 + S;                             // Gram entries + right-hand side
    constexpr int KC = kWave / 4;                                      // points per lane per plane
    constexpr uint32_t W = sizeof(T);
    constexpr int txw = kGoTx, tyh = kGoTy, tx2 = kGoTx2;
    constexpr int CS = kGoPitch + 1;  // LDS stride of a column's padded tile (odd: spreads the banks)
    constexpr bool HAS_COEF = Rule::kHasCoef;
    using M = GoMfma<T>;
    using Coef = typename Rule::Coef;
    __shared__ T Pt[S * CS];
    __shared__ T Dt[WD ? kGoThreads : 1];
    __shared__ Coef Ct[HAS_COEF ? kGoThreads : 1];
    __shared__ double red[kGoThreads / kWave][E];
    if (st->done)
        return;
    // Logical block: each XCD takes a contiguous range, so the tiles next to
    // a tile (same z-range, item numbers +-1 and +-tiles_x) run at the same
    // time on the same XCD and its halo lines are hits in that XCD's L2.
    const int lb = static_cast<int>(xcd_block(blockIdx.x, static_cast<uint32_t>(geo.per)));
    if (lb >= geo.blocks)
        return;
    const int t = threadIdx.x;
    const int lane = t % kWave, wv = t / kWave;
    // Thread t as a grid point (halo, diagonal and coefficient staging).
    const int tlx = t & (txw - 1), tly = t >> kGoTxl;
    // Lane as matrix-core operand: column n at the points p(kc) = 64 wv + 4 kc + gq,
    // kc = 0..15, i.e. tile row 2 wv + kc / 8, tile column 4 (kc % 8) + gq.
    const int n = lane & 15, gq = lane >> 4;
    const bool ncol = n < S;
    const int nc = ncol ? n : 0;  // column actually read (unused lanes reread column 0)
    const uint32_t pb = static_cast<uint32_t>(g.nxy) * W;  // bytes per plane

    typename M::acc_t gacc = {};  // this wave's share of G_raw
    T cacc = T(0);                // this lane's share of c'_n

    const int tiles = geo.tiles;
    for (int item = lb; item < geo.items; item += geo.blocks) {
        const int tile = item % tiles, zb = item / tiles;
        int tx_, ty_;
        if constexpr (FULL) {
            tx_ = tile % geo.fx, ty_ = tile / geo.fx;
        } else if (geo.rx && tile < geo.tiles_y) {
            tx_ = geo.fx, ty_ = tile;
        } else {
            tx_ = tile - (geo.rx ? geo.tiles_y : 0), ty_ = geo.fy;
        }
        const int i0 = tx_ * txw, j0 = ty_ * tyh;
        const int z0 = zb * geo.zr;
        const int z1 = z0 + geo.zr < g.nz ? z0 + geo.zr : g.nz;
        // this thread's staging point
        const uint32_t ti = static_cast<uint32_t>(i0 + tlx), tj = static_cast<uint32_t>(j0 + tly);
        const bool tvalid = ti < static_cast<uint32_t>(g.nx) && tj < static_cast<uint32_t>(g.ny);
        const uint32_t tq = tvalid ? ti + static_cast<uint32_t>(g.nx) * tj : 0u;
        const uint32_t tjr = tvalid ? tj : 0u;
        // this lane's points: validity mask and in-plane offset of point kc = 0
        const int li = i0 + gq, lj = j0 + 2 * wv;
        uint32_t vmask = 0;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
            if (li + 4 * (kc % 8) < g.nx && lj + kc / 8 < g.ny)
                vmask |= 1u << kc;
        const uint32_t lq = static_cast<uint32_t>(li + g.nx * lj);
        const uint32_t rowb = static_cast<uint32_t>(g.nx) * W;  // bytes per grid row
        auto lofsb = [&](int kc) -> uint32_t {  // in-plane byte offset of point kc (valid points)
            return (lq + static_cast<uint32_t>(4 * (kc % 8))) * W + (kc / 8 ? rowb : 0u);
        };
        const int pbase = (2 * wv + 1) * tx2 + gq + 1;  // padded-tile index of point kc = 0
        const T *colp = P + nc * ld;

        // Halo ring of the tile: wave wv loads columns 4 wv .. 4 wv + 3.
        // Entries m = 0..3: column 4 wv + m, lane < 32 the row below the tile,
        // lane >= 32 the row above, x = lane % 32.  Entry 4: column
        // 4 wv + lane / 16, the column left (lane % 16 < 8) or right of the
        // tile, y = lane % 8.  Offsets without the plane term, the in-grid
        // flags and LDS indices do not change along z.
        int64_t hoff[5];
        int hpos[5];
        uint32_t hin = 0;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const int c = m < 4 ? 4 * wv + m : 4 * wv + (lane >> 4);
            const int hx = m < 4 ? (lane & 31) : (((lane >> 3) & 1) ? txw : -1);
            const int hy = m < 4 ? ((lane >> 5) ? tyh : -1) : (lane & 7);
            const int gi = i0 + hx, gj = j0 + hy;
            const bool in = c < S && gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
            hin |= in ? (1u << m) : 0u;
            hoff[m] = in ? static_cast<int64_t>(c) * ld + gi + static_cast<int64_t>(g.nx) * gj : 0;
            hpos[m] = c < S ? c * CS + (hy + 1) * tx2 + hx + 1 : -1;
        }

        // FULL (tile inside the grid in x and y) drops the per-point validity
        // selects.
        auto run = [&]() {
            auto pv = [&](int kc) -> bool { return FULL || ((vmask >> kc) & 1u); };
            // Loads for z-step kk, issued one step ahead (before the products
            // of step kk - 1): the halo ring of plane kk, plane kk+1 at the
            // lane's points, the coefficients and M-diagonal of the staging
            // point.  kk may run one plane past the range (the second step of
            // the last pair): addresses are then clamped and values unused.
            T zm[KC], zc[KC], qa[KC], qb[KC];
            T hv[5];
            Coef f{};
            T dv = T(0);
            auto issue = [&](int kk_, T(&dst)[KC]) {
                const int kk = kk_ < g.nz ? kk_ : g.nz - 1;
                const int64_t poff = static_cast<int64_t>(kk) * g.nxy;
#pragma unroll
                for (int m = 0; m < 5; ++m)
                    hv[m] = P[hoff[m] + ((hin >> m) & 1u ? poff : 0)];
                // keep the halo loads first: loads complete in issue order, so
                // the halo can be stored while the plane loads are in flight
                __builtin_amdgcn_sched_barrier(0);
                const uint32_t base = static_cast<uint32_t>(kk) * static_cast<uint32_t>(g.nxy) * W;
                const uint32_t up = kk + 1 < g.nz ? pb : 0u;
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
                    dst[kc] = go_ld(colp, base + (pv(kc) ? lofsb(kc) + up : 0u));
                const int64_t tc = static_cast<int64_t>(tq) + poff;
                if constexpr (HAS_COEF)
                    f = rule.load(g, tjr + static_cast<uint32_t>(g.ny) * static_cast<uint32_t>(kk),
                                  static_cast<uint32_t>(kk), tc);
                if constexpr (WD)
                    dv = go_ld(dvec, static_cast<uint32_t>(tc) * W);
            };
            // One z-step k: zq holds plane k+1 of the lane's points (loaded one
            // step earlier), zl receives plane k+2.  A step past the range
            // (k >= z1) adds nothing.  No branch surrounds the loads, so the
            // waits for them are exact.
            auto zstep = [&](int k, T(&zq)[KC], T(&zl)[KC]) {
                const bool ht = k + 1 < g.nz;
                const bool active = k < z1;
                // (1) plane k into the padded tiles: the lane's points of
                // column n, the halo ring, the staging point's diagonal and
                // coefficients.
                if (ncol) {
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc)
                        Pt[n * CS + pbase + (kc / 8) * tx2 + 4 * (kc % 8)] = zc[kc];
                }
#pragma unroll
                for (int m = 0; m < 5; ++m)
                    if (hpos[m] >= 0)
                        Pt[hpos[m]] = (hin >> m) & 1u ? hv[m] : T(0);
                if constexpr (WD)
                    Dt[t] = tvalid ? dv : T(0);
                if constexpr (HAS_COEF)
                    Ct[t] = f;
                __syncthreads();
                // loads of step k + 1, in flight during the products of step k
                issue(k + 1, zl);
                // the plane above the grid is zero
                if (!ht) {
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc)
                        zq[kc] = T(0);
                }
                // (2) per point: y = (A p_n)(k) from the tile and the
                // z-registers, G_raw += p y^T on the matrix cores,
                // c'_n += p_n w.  Skipped past the range (block-uniform; the
                // loads in flight are the same on both sides).
                if (active) {
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    const int pp = pbase + (kc / 8) * tx2 + 4 * (kc % 8);
                    const T *L = Pt + nc * CS + pp;
                    Coef fk{};
                    if constexpr (HAS_COEF)
                        fk = Ct[64 * wv + 4 * kc + gq];
                    const T zpv = pv(kc) ? zq[kc] : T(0);  // zero outside the grid
                    // the lane's points kc and kc + 8 are vertical neighbours:
                    // one of the two y-neighbours comes from the registers
                    const T ys = kc >= 8 ? zc[kc - 8] : L[-tx2];
                    const T yn = kc < 8 ? zc[kc + 8] : L[tx2];
                    const T y = Rule::y(fk, zc[kc], L[-1], L[1], ys, yn, zm[kc], zpv);
                    // p_0 at the point: held by the column-0 lane of this row
                    T w = go_row_bcast0(zc[kc]);
                    if constexpr (WD)
                        w *= Dt[64 * wv + 4 * kc + gq];
                    const bool v = ncol && pv(kc);
                    const T a = (S == 16 && FULL) || v ? zc[kc] : T(0);
                    gacc = M::step(a, (S == 16 && FULL) || v ? y : T(0), gacc);
                    cacc += a * w;
                    if ((kc & 3) == 3)
                        __builtin_amdgcn_sched_barrier(0);  // bounds the LDS reads in flight (registers)
                }
                // planes move down once every point has used its neighbours
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    zm[kc] = zc[kc];
                    zc[kc] = pv(kc) ? zq[kc] : T(0);
                }
                }
                __syncthreads();
            };
            {
                const uint32_t base = static_cast<uint32_t>(z0) * static_cast<uint32_t>(g.nxy) * W;
                const bool down = z0 > 0;
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    const uint32_t o = base + (pv(kc) ? lofsb(kc) : 0u);
                    const T a = go_ld(colp, down && pv(kc) ? o - pb : o), b = go_ld(colp, o);
                    zm[kc] = down && pv(kc) ? a : T(0);
                    zc[kc] = pv(kc) ? b : T(0);
                }
            }
            issue(z0, qa);
            // the two next-plane buffers alternate, so no in-flight value is copied
            for (int k = z0; k < z1; k += 2) {
                zstep(k, qa, qb);
                zstep(k + 1, qb, qa);
            }
        };
        run();
    }

    // Block reduction in a fixed order: wave partials into LDS, then entry e
    // of the block = sum over the four waves.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = M::row(lane, r);
        if (m < S && n <= m)
            red[wv][tri_index(m, n)] = static_cast<double>(gacc[r]);
    }
    {
        // c'_n of the wave: the four lanes n, n + 16, n + 32, n + 48
        T v = cacc + __shfl_xor(cacc, 16, kWave);
        v += __shfl_xor(v, 32, kWave);
        if (lane < S)
            red[wv][S * (S + 1) / 2 + lane] = static_cast<double>(v);
    }
    __syncthreads();
    for (int e = t; e < E; e += kGoThreads)
        gpart[static_cast<int64_t>(e) * estride + geo.slot0 + lb] =
            ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

template <class Rule, typename T, int S, bool WD>
void gram_op_launch_rule(const IterArgs &a, const Rule &rule, const T *dv, hipStream_t st)
{
    const T *P = static_cast<const T *>(a.P);
    int slot0 = 0;
    for (int part = 0; part < 2; ++part) {
        const int blocks = a.go_blocks[part];
        if (blocks == 0)
            continue;
        const int per = (blocks + static_cast<int>(kNumXcd) - 1) / static_cast<int>(kNumXcd);
        const GoGeom geo{a.go_fx, a.go_fy, a.go_tiles_y, a.go_rx,  a.go_ry,  a.go_tiles[part],
                         a.go_zr, a.go_nzb, a.go_items[part], blocks, per, slot0};
        const dim3 grid(static_cast<uint32_t>(per) * kNumXcd), block(kGoThreads);
        if (part == 0)
            hipLaunchKernelGGL((k_gram_op<Rule, T, S, WD, true>), grid, block, 0, st, a.st, a.op.g, rule, P, a.ld, dv,
                               geo, a.gpart, a.nbg);
        else
            hipLaunchKernelGGL((k_gram_op<Rule, T, S, WD, false>), grid, block, 0, st, a.st, a.op.g, rule, P, a.ld,
                               dv, geo, a.gpart, a.nbg);
        slot0 += blocks;
    }
}

template <typename T, int S>
hipError_t gram_op_launch_s(const IterArgs &a, hipStream_t st)
{
    if (a.op.kind == kOpPoisson) {
        gram_op_launch_rule<GoPoisson<T>, T, S, false>(a, GoPoisson<T>{}, static_cast<const T *>(nullptr), st);
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
            gram_op_launch_rule<GoFaces<T>, T, S, true>(a, rule, dv, st);
        else
            gram_op_launch_rule<GoFaces<T>, T, S, false>(a, rule, dv, st);
    }
    return hipGetLastError();
}

}  // namespace sstep
