// Two steps of the Chebyshev basis recurrence (Sec. 2, Definition) in one pass
// over memory, for the constant-coefficient 7-point operator with a constant
// Jacobi weight (Sec. 8 model problem):
//   q       = p_{j+1} = 2 theta (M^{-1} A p_j - sigma p_j) - p_{j-1}
//                       (theta (M^{-1} A p_0 - sigma p_0) when j = 0)
//   p_{j+2}           = 2 theta (M^{-1} A q - sigma q) - p_j
// Each value is formed with the same operations, in the same order, as by one
// single step (the 7-point sum W, E, S, N, below, above), so the pair equals
// two single steps bit for bit.
//
// Layout of the work: a block of 64 x EY threads owns an in-plane tile of
// TXI x (EY - 2) points (TXI <= 62) and a range of kz planes, and marches the
// range in z.
// Every thread forms q at one point of the tile or of the one-point ring
// around it, so the second step finds all its in-plane neighbours inside the
// block.  The current plane of p_j and of q sits in LDS (double-buffered, one
// barrier per plane); the planes above and below come from registers.
// Neighbours of ring points that lie outside the tile are read from global
// memory.  HBM traffic per point: p_{j-1} and p_j read, q and p_{j+2}
// written, 4 vectors for two columns against 6 for two single steps; the
// ring and the two extra planes of each range are re-reads served mostly by
// L2.  A 56-point interior keeps every FP64 row store 64-byte aligned; the
// store policy per precision is at buf_store_out.
#pragma once

#include "common.h"

namespace sstep {

constexpr int kF2Lanes = 64;  // extended tile width: one wave per tile row

struct F2Plan {
    uint32_t tiles_x, tiles_y, ranges;  // tiles along x / along y, z-ranges
    int kz;                             // planes per range
    uint32_t nbl, per;                  // logical blocks, logical blocks per XCD
    int zfast;                          // 1: z-range fastest in the block numbering
};

template <int EY, int TXI>
inline F2Plan plan_f2(const Grid3 &g, int kz, int zfast)
{
    F2Plan p;
    p.tiles_x = static_cast<uint32_t>((g.nx + TXI - 1) / TXI);
    p.tiles_y = static_cast<uint32_t>((g.ny + EY - 3) / (EY - 2));
    p.kz = kz;
    p.ranges = static_cast<uint32_t>((g.nz + kz - 1) / kz);
    p.nbl = p.tiles_x * p.tiles_y * p.ranges;
    p.per = (p.nbl + kNumXcd - 1) / kNumXcd;
    p.zfast = zfast;
    return p;
}

// Barrier for LDS traffic only: its fences order LDS accesses, so global
// loads issued before it stay in flight (the fence of __syncthreads makes
// every wave wait for all of its outstanding global loads at each barrier).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Raw buffer access through a resource that covers one window of a vector:
// an offset at or beyond the window's size reads 0 and drops a store, so the
// kernel predicates its memory accesses on the offset alone and every load
// and store is issued unconditionally (no branch around a memory access, and
// no select on a loaded value, which the compiler would turn back into a
// branch): the compiler can then count the loads in flight and keeps them
// in flight across the barriers.
constexpr uint32_t kOutside = 0x80000000u;  // beyond every window (windows stay below 2 GiB)
constexpr int32_t kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)
constexpr int kNonTemporal = 2;             // cache-policy bit of a buffer access: non-temporal
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_window(const T *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base), 0, static_cast<int>(bytes), kRsrcWord3);
}

__device__ __forceinline__ double buf_load(double, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float buf_load(float, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// FP64 results are stored non-temporally, FP32 ones through the caches: the
// 248-byte FP32 row pieces end mid-line, and L2 merges such partial lines
// only for cached stores (FP32 pair 47 us cached against 62 us
// non-temporal, FP64 84 us non-temporal against 87 us cached, in the
// solve's setting at 224^3).
__device__ __forceinline__ void buf_store_out(double v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), r, off, 0, kNonTemporal);
}
__device__ __forceinline__ void buf_store_out(float v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}

// Largest plane window one block addresses: kz + 4 planes (two below the
// range, one above it, and the range's own kz + 1 for q's top plane).  The
// launch checks that it stays below 2 GiB.
inline int64_t f2_window_bytes(const Grid3 &g, int kz, int elem)
{
    return static_cast<int64_t>(kz + 4) * g.nxy * elem;
}

// D: planes by which the global loads run ahead of their use (a ring of D
// register slots per loaded stream, the loop unrolled by D so that every
// slot index is a constant).
// MW: waves per SIMD the register allocation must allow (8 = two blocks of
// 1024 threads per CU).  TXI: interior points of a tile row.
// MOM (moments Gram kind): the block also sums, over the points it stores,
// <q, p_j>, <q, q>, <p_{j+2}, q>, <p_{j+2}, p_{j+2}> (and <p_0, p_0> first
// when FIRST), unweighted (the constant diagonal is applied afterwards), and
// writes them to consecutive slots of mpart, stride mstride, at its logical
// block index.
template <typename T, int EY, bool FIRST, int D, int MW, int TXI, bool MOM>
__global__ __launch_bounds__(kF2Lanes *EY, MW) void k_basis_f2(const DevState *__restrict__ st, Grid3 g, T minv,
                                                            const T *__restrict__ pprev, const T *__restrict__ pj,
                                                            T *__restrict__ qout, T *__restrict__ p2out, T theta,
                                                            T sigma, F2Plan plan, double *__restrict__ mpart,
                                                            int64_t mstride)
{
    constexpr int NT = kF2Lanes * EY;
    constexpr uint32_t ES = sizeof(T);
    __shared__ T ps[2][NT];
    __shared__ T qs[2][NT];
    if (st->done)
        return;
    const uint32_t lb = xcd_block(blockIdx.x, plan.per);
    if (lb >= plan.nbl)
        return;  // whole block: no barrier is skipped by part of it
    const uint32_t ntile = plan.tiles_x * plan.tiles_y;
    uint32_t tile, zr;
    if (plan.zfast) {
        zr = lb % plan.ranges;
        tile = lb / plan.ranges;
    } else {
        tile = lb % ntile;
        zr = lb / ntile;
    }
    const uint32_t ty = tile / plan.tiles_x, tx = tile - ty * plan.tiles_x;
    const int tid = threadIdx.x;
    const int lane = tid % kF2Lanes, row = tid / kF2Lanes;
    const int gi = static_cast<int>(tx) * TXI - 1 + lane;
    const int gj = static_cast<int>(ty) * (EY - 2) - 1 + row;
    const bool in_dom = lane <= TXI + 1 && gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
    const bool interior = in_dom && lane >= 1 && lane <= TXI && row >= 1 && row <= EY - 2;
    const int k0 = static_cast<int>(zr) * plan.kz;
    const int k1 = k0 + plan.kz < g.nz ? k0 + plan.kz : g.nz;
    // the block's window: planes kb .. ke - 1 of every vector (p_j is read
    // from two planes below the range to one plane above it)
    const int kb = k0 - 2 > 0 ? k0 - 2 : 0;
    const int ke = k1 + 2 < g.nz ? k1 + 2 : g.nz;
    const uint32_t wbytes = static_cast<uint32_t>(ke - kb) * static_cast<uint32_t>(g.nxy) * ES;
    const int64_t wbase = static_cast<int64_t>(kb) * g.nxy;
    const __amdgpu_buffer_rsrc_t rj = make_window(pj + wbase, wbytes);
    const __amdgpu_buffer_rsrc_t rv = make_window(FIRST ? pj + wbase : pprev + wbase, wbytes);
    const __amdgpu_buffer_rsrc_t rq = make_window(qout + wbase, wbytes);
    const __amdgpu_buffer_rsrc_t r2 = make_window(p2out + wbase, wbytes);
    const uint32_t pl = static_cast<uint32_t>(in_dom ? gj * g.nx + gi : 0);  // in-plane index
    const uint32_t plane = static_cast<uint32_t>(g.nxy) * ES;
    // byte offset of the thread's point (+ d in-plane) on plane k, or
    // kOutside when the point is outside the grid or k outside [klo, khi]
    auto at = [&](int k, int d, bool ok, int klo, int khi) -> uint32_t {
        return ok && in_dom && k >= klo && k <= khi
                   ? static_cast<uint32_t>(k - kb) * plane + static_cast<uint32_t>(static_cast<int>(pl) + d) * ES
                   : kOutside;
    };
    // A ring point reads its one neighbour outside the tile from global
    // memory: west (lane 0), east (lane TXI + 1), south (row 0) or north
    // (last row); lanes beyond TXI + 1 hold no point; it reads 0 where that neighbour is outside the grid.  The four
    // corners of the ring are no neighbour of any tile point, so their q is
    // never used and they read nothing.
    const bool edge_x = lane == 0 || lane == TXI + 1, edge_y = row == 0 || row == EY - 1;
    const int off_r = edge_x ? (lane == 0 ? -1 : 1) : (row == 0 ? -g.nx : g.nx);
    const bool ring = edge_x != edge_y && (edge_x ? (lane == 0 ? gi > 0 : gi + 1 < g.nx)
                                                  : (row == 0 ? gj > 0 : gj + 1 < g.ny));
    const int kj_hi = ke - 1;                       // last plane of p_j the range reads
    const int kv_hi = k1 < g.nz ? k1 : g.nz - 1;    // last plane of p_{j-1} and ring values
    const T two_theta = T(2) * theta;
    T pm = buf_load(T(), rj, at(k0 - 2, 0, true, 0, kj_hi));  // p_j one plane below the current one
    T p0 = buf_load(T(), rj, at(k0 - 1, 0, true, 0, kj_hi));  // p_j on the current plane
    T qb = T(0), qc = T(0);  // q two planes and one plane below the current one
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;  // products (MOM)
    // slot u holds, for plane kq = k0 - 1 + u (mod D): p_j on plane kq + 1,
    // p_{j-1} on plane kq and the ring neighbours on plane kq
    T pjs[D], pps[D], rgs[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const int kq = k0 - 1 + u;
        pjs[u] = buf_load(T(), rj, at(kq + 1, 0, true, 0, kj_hi));
        pps[u] = FIRST ? T(0) : buf_load(T(), rv, at(kq, 0, true, 0, kv_hi));
        rgs[u] = buf_load(T(), rj, at(kq, off_r, ring, 0, kv_hi));
    }
    // planes k0 - 1 .. k1, padded to a multiple of D: a padding step loads
    // nothing (its offsets lie outside the window) and stores nothing
    const int nstep = (k1 - k0 + 2 + D - 1) / D * D;
    for (int base = k0 - 1; base < k0 - 1 + nstep; base += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int kq = base + u;
            const int buf = kq & 1;
            const T pp = pjs[u], pv = pps[u], rg = rgs[u];
            ps[buf][tid] = p0;
            lds_barrier();
            T q = T(0);
            if (in_dom && kq >= 0 && kq <= k1 && kq < g.nz) {
                const T w = lane > 0 ? ps[buf][tid - 1] : rg;
                const T e = lane < TXI + 1 ? ps[buf][tid + 1] : rg;
                const T s = row > 0 ? ps[buf][tid - kF2Lanes] : rg;
                const T n = row < EY - 1 ? ps[buf][tid + kF2Lanes] : rg;
                const T y = T(6) * p0 - (((((w + e) + s) + n) + pm) + pp);
                if constexpr (FIRST)
                    q = theta * (minv * y - sigma * p0);
                else
                    q = two_theta * (minv * y - sigma * p0) - pv;
            }
            buf_store_out(q, rq, at(kq, 0, interior, k0, k1 - 1));
            qs[buf][tid] = q;
            // the second step on the plane below: q there is in qs[buf ^ 1]
            // (stored before this plane's barrier), q below it in qb, above in q
            T p2 = T(0);
            if (interior) {
                const T *qp = qs[buf ^ 1];
                const T y = T(6) * qc - (((((qp[tid - 1] + qp[tid + 1]) + qp[tid - kF2Lanes]) + qp[tid + kF2Lanes]) + qb) + q);
                p2 = two_theta * (minv * y - sigma * qc) - pm;
            }
            buf_store_out(p2, r2, at(kq - 1, 0, interior, k0, k1 - 1));
            if constexpr (MOM) {
                // the plane just stored: p_j, q and p_{j+2} of plane kq - 1
                const bool own = interior && kq - 1 >= k0 && kq - 1 < k1;
                const double a = own ? static_cast<double>(pm) : 0.0;
                const double b = own ? static_cast<double>(qc) : 0.0;
                const double c2 = own ? static_cast<double>(p2) : 0.0;
                if constexpr (FIRST)
                    m0 += a * a;
                m1 += b * a;
                m2 += b * b;
                m3 += c2 * b;
                m4 += c2 * c2;
            }
            qb = qc;
            qc = q;
            pm = p0;
            p0 = pp;
            // refill the slot for plane kq + D once its values are used, so
            // that the load writes the slot's own registers
            const int kn = kq + D;
            pjs[u] = buf_load(T(), rj, at(kn + 1, 0, true, 0, kj_hi));
            if constexpr (!FIRST)
                pps[u] = buf_load(T(), rv, at(kn, 0, true, 0, kv_hi));
            rgs[u] = buf_load(T(), rj, at(kn, off_r, ring, 0, kv_hi));
        }
    }
    if constexpr (MOM) {
        double *out = mpart + lb;
        if constexpr (FIRST) {
            const double v[5] = {m0, m1, m2, m3, m4};
            block_partials<5, kF2Lanes * EY>(v, out, mstride);
        } else {
            const double v[4] = {m1, m2, m3, m4};
            block_partials<4, kF2Lanes * EY>(v, out, mstride);
        }
    }
}

}  // namespace sstep
