// Streaming kernels of the outer iteration: residual + basis start, the fused
// SpMV/Jacobi/Chebyshev basis step, the update x += P alpha, and helpers.
// All of them are bound by HBM bandwidth (well under one flop per byte).
#include <algorithm>

#include "basis_f2.h"
#include "launch.h"
#include "opsel.h"
#include "stop.h"

namespace sstep {
namespace {

struct Launch1D {
    uint32_t nbl;   // logical blocks
    uint32_t per;   // logical blocks per XCD
    uint32_t grid;  // hardware blocks (multiple of 8)
};

inline uint32_t blocks_for(int64_t n) { return static_cast<uint32_t>((n + kBlock - 1) / kBlock); }

Launch1D plan_points(int64_t n)
{
    Launch1D l;
    l.nbl = static_cast<uint32_t>((n + kBlock - 1) / kBlock);
    l.per = (l.nbl + kNumXcd - 1) / kNumXcd;
    l.grid = l.per * kNumXcd;
    return l;
}

template <typename T>
__device__ __forceinline__ void block_sum_store(T v, T *out)
{
    __shared__ T part[kBlock / kWave];
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0)
        part[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = part[0];
#pragma unroll
        for (int q = 1; q < kBlock / kWave; ++q)
            acc += part[q];
        *out = acc;
    }
}

// The stopping test of iteration k, one block after the residual kernel: the
// fixed-order sum of its partials of ||r||^2, then stop_test (stop.h), so
// that every later kernel of a converged iteration returns at once.
__global__ __launch_bounds__(kSumThreads) void k_stop(DevState *__restrict__ st, const double *__restrict__ rpart,
                                                      int nbr, double *__restrict__ dbg_rho,
                                                      double *__restrict__ hist, int hist_cap)
{
    if (st->done)
        return;
    const double rho2 = fixed_order_sum(rpart, nbr);
    if (threadIdx.x == 0)
        stop_test(st, rho2, dbg_rho, hist, hist_cap);
}

// r = b - A x in FP64, partial sums of r^2 per logical block, and the basis
// start p_0 = p0scale * (M^{-1} r or r) written as column 0 of P.
template <class Op, typename TP>
__global__ __launch_bounds__(kBlock) void k_residual(const DevState *__restrict__ st, Op op, TP *__restrict__ p0,
                                                     double *__restrict__ rpart, int64_t n, int64_t chunk,
                                                     uint32_t per, uint32_t nbl, int p0_mode, int write_p0)
{
    if (st->done)
        return;
    const uint32_t lb = xcd_block(blockIdx.x, per);
    if (lb >= nbl)
        return;
    const double *__restrict__ b = st->b;
    const double *__restrict__ x = st->x;
    const double scale = st->p0scale;
    const int64_t beg = static_cast<int64_t>(lb) * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
        double pc, y, dinv;
        op.apply(x, c, pc, y, dinv);
        const double r = __builtin_nontemporal_load(b + c) - y;  // b is read once
        acc += r * r;
        if (write_p0)
            p0[c] = static_cast<TP>(scale * (p0_mode ? r : dinv * r));
    }
    block_sum_store(acc, rpart + lb);
}

// The residual for the constant Poisson operator in FP64 (nx even) in the
// basis kernel's shape: two x-points and kP2Kz planes per thread, 1024-thread
// blocks, +-z neighbours of x from registers, b read once (non-temporal).
// One partial sum of r^2 per block, blocks numbered blockIdx.x + gridDim.x *
// blockIdx.y (the launch keeps their number within the partial buffer).
template <typename TP>
__global__ __launch_bounds__(1024) void k_residual_p2(const DevState *__restrict__ st, Grid3 g, double minv,
                                                      TP *__restrict__ p0, double *__restrict__ rpart, int p0_mode,
                                                      int write_p0)
{
    constexpr int KZ = 8;
    __shared__ double part[1024 / kWave];
    if (st->done)
        return;
    const double *__restrict__ x = st->x;
    const double *__restrict__ b = st->b;
    const double scale = st->p0scale;
    const uint32_t pl = (blockIdx.x * 1024 + threadIdx.x) * 2;  // in-plane index of the pair
    double acc = 0.0;
    if (pl < static_cast<uint32_t>(g.nxy)) {
        const uint32_t j = fdiv(pl, g.dx);
        const uint32_t i = pl - j * g.nx;
        const int k0 = blockIdx.y * KZ;
        const double2 z = {0.0, 0.0};
        int64_t c = pl + static_cast<int64_t>(k0) * g.nxy;
        double2 below = k0 > 0 ? *reinterpret_cast<const double2 *>(x + c - g.nxy) : z;
        double2 ctr = *reinterpret_cast<const double2 *>(x + c);
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            const int k = k0 + kk;
            if (k >= g.nz)
                break;
            const double2 above = k + 1 < g.nz ? *reinterpret_cast<const double2 *>(x + c + g.nxy) : z;
            const double w = i > 0 ? x[c - 1] : 0.0;
            const double e = i + 2 < static_cast<uint32_t>(g.nx) ? x[c + 2] : 0.0;
            const double2 s = j > 0 ? *reinterpret_cast<const double2 *>(x + c - g.nx) : z;
            const double2 nn = j + 1 < static_cast<uint32_t>(g.ny) ? *reinterpret_cast<const double2 *>(x + c + g.nx) : z;
            const double bx = __builtin_nontemporal_load(b + c), by = __builtin_nontemporal_load(b + c + 1);
            const double yx = 6.0 * ctr.x - (((((w + ctr.y) + s.x) + nn.x) + below.x) + above.x);
            const double yy = 6.0 * ctr.y - (((((ctr.x + e) + s.y) + nn.y) + below.y) + above.y);
            const double rx = bx - yx, ry = by - yy;
            acc += rx * rx;
            acc += ry * ry;
            if (write_p0) {
                p0[c] = static_cast<TP>(scale * (p0_mode ? rx : minv * rx));
                p0[c + 1] = static_cast<TP>(scale * (p0_mode ? ry : minv * ry));
            }
            below = ctr;
            ctr = above;
            c += g.nxy;
        }
    }
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0)
        part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < 1024 / kWave; ++w)
            sum += part[w];
        rpart[blockIdx.x + gridDim.x * blockIdx.y] = sum;
    }
}

// One step of the Chebyshev recurrence fused with the operator apply
// (Sec. 2, Definition), for column j of the basis:
//   y = A p_j                                   -> AP[:, j]
//   p_1     = theta (M^{-1} y - sigma p_0)            (STEP 0, j = 0)
//   p_{j+1} = 2 theta (M^{-1} y - sigma p_j) - p_{j-1} (STEP 1, 0 < j < s-1)
//   nothing more for j = s-1                          (STEP 2)
template <class Op, typename T, int STEP>
__global__ __launch_bounds__(kBlock) void k_basis(const DevState *__restrict__ st, Op op, const T *__restrict__ pj,
                                                  const T *__restrict__ pprev, T *__restrict__ apj,
                                                  T *__restrict__ pnext, T theta, T sigma, int64_t n, uint32_t per,
                                                  uint32_t nbl)
{
    if (st->done)
        return;
    const uint32_t lb = xcd_block(blockIdx.x, per);
    if (lb >= nbl)
        return;
    const int64_t c = static_cast<int64_t>(lb) * kBlock + threadIdx.x;
    if (c >= n)
        return;
    T pc, y, dinv;
    op.apply(pj, c, pc, y, dinv);
    if (apj)
        __builtin_nontemporal_store(y, apj + c);
    if constexpr (STEP == 0) {
        pnext[c] = theta * (dinv * y - sigma * pc);
    } else if constexpr (STEP == 1) {
        const T two_theta = T(2) * theta;
        pnext[c] = two_theta * (dinv * y - sigma * pc) - __builtin_nontemporal_load(pprev + c);
    }
}

// The same step for the moments Gram kind (no AP): besides p_{j+1}, block
// partials of the M inner products that fix the Gram matrix (fgs_core.h,
// k_fgs_mom): <p_{j+1}, M p_j> and <p_{j+1}, M p_{j+1}>, and <p_0, M p_0>
// first when j = 0, written to consecutive slots of mpart (stride mstride),
// one value per logical block.  The threads past n take part in the block
// sums with weight 0.
template <class Op, typename T, int STEP>
__global__ __launch_bounds__(kBlock) void k_basis_mom(const DevState *__restrict__ st, Op op,
                                                      const T *__restrict__ pj, const T *__restrict__ pprev,
                                                      T *__restrict__ pnext, T theta, T sigma, int64_t n,
                                                      uint32_t per, uint32_t nbl, double *__restrict__ mpart,
                                                      int64_t mstride)
{
    static_assert(STEP == 0 || STEP == 1, "the moments kind forms every column");
    if (st->done)
        return;
    const uint32_t lb = xcd_block(blockIdx.x, per);
    if (lb >= nbl)
        return;  // whole block
    const int64_t c = static_cast<int64_t>(lb) * kBlock + threadIdx.x;
    const bool valid = c < n;
    const int64_t cc = valid ? c : n - 1;
    T pc, y, dinv, wt;
    op.apply_w(pj, cc, pc, y, dinv, wt);
    T pn;
    if constexpr (STEP == 0)
        pn = theta * (dinv * y - sigma * pc);
    else
        pn = T(2) * theta * (dinv * y - sigma * pc) - __builtin_nontemporal_load(pprev + cc);
    if (valid)
        pnext[c] = pn;
    const double w = valid ? static_cast<double>(wt) : 0.0;
    const double a = static_cast<double>(pn), b = static_cast<double>(pc);
    if constexpr (STEP == 0) {
        const double v[3] = {w * b * b, w * a * b, w * a * a};
        block_partials<3, kBlock>(v, mpart + lb, mstride);
    } else {
        const double v[2] = {w * a * b, w * a * a};
        block_partials<2, kBlock>(v, mpart + lb, mstride);
    }
}

// The same step for the constant Poisson operator in FP64 (nx even): a thread
// owns two consecutive x-points and KZ = 8 consecutive z-planes, so the +-z
// neighbours come from registers (one 16-byte load per plane instead of
// three); south/north/centre/previous column are read as 16-byte pairs,
// west/east of the pair as single values, AP and p_{j+1} written as pairs.
// p_{j-1} is read once and not reused: non-temporal loads.  1024-thread
// blocks are numbered in-plane fastest (x-y pairs, then plane groups), so a
// block spans several grid rows and its +-y neighbours are mostly its own
// loads; each XCD takes a contiguous range of those numbers, so the rows
// and planes a block shares with its neighbours are mostly L2 hits.  Shape
// measured fastest on MI355X among 1/2/4 points x 1..16 planes x 128..1024
// threads (224^3, in the solve's column rotation).
constexpr int kP2Kz = 8;
constexpr int kP2Block = 1024;
template <int STEP>
__global__ __launch_bounds__(kP2Block) void k_basis_p2(const DevState *__restrict__ st, Grid3 g, double minv,
                                                       const double *__restrict__ pj, const double *__restrict__ pprev,
                                                       double *__restrict__ apj, double *__restrict__ pnext,
                                                       double theta, double sigma, uint32_t gx, uint32_t per,
                                                       uint32_t nbl)
{
    constexpr int KZ = kP2Kz;
    if (st->done)
        return;
    // logical block (in-plane fastest) in XCD-contiguous order: the blocks
    // holding a block's +-y rows and +-z planes run on the same XCD
    const uint32_t lb = xcd_block(blockIdx.x, per);
    if (lb >= nbl)
        return;
    const uint32_t bz = lb / gx, bx = lb - bz * gx;
    const uint32_t pl = (bx * kP2Block + threadIdx.x) * 2;  // in-plane index of the pair
    if (pl >= static_cast<uint32_t>(g.nxy))
        return;
    const uint32_t j = fdiv(pl, g.dx);
    const uint32_t i = pl - j * g.nx;
    const int k0 = static_cast<int>(bz) * KZ;
    const double2 z = {0.0, 0.0};
    int64_t c = pl + static_cast<int64_t>(k0) * g.nxy;
    double2 below = k0 > 0 ? *reinterpret_cast<const double2 *>(pj + c - g.nxy) : z;
    double2 ctr = *reinterpret_cast<const double2 *>(pj + c);
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) {
        const int k = k0 + kk;
        if (k >= g.nz)
            break;
        const double2 above = k + 1 < g.nz ? *reinterpret_cast<const double2 *>(pj + c + g.nxy) : z;
        const double w = i > 0 ? pj[c - 1] : 0.0;
        const double e = i + 2 < static_cast<uint32_t>(g.nx) ? pj[c + 2] : 0.0;
        const double2 s = j > 0 ? *reinterpret_cast<const double2 *>(pj + c - g.nx) : z;
        const double2 nn = j + 1 < static_cast<uint32_t>(g.ny) ? *reinterpret_cast<const double2 *>(pj + c + g.nx) : z;
        double2 y;
        y.x = 6.0 * ctr.x - (((((w + ctr.y) + s.x) + nn.x) + below.x) + above.x);
        y.y = 6.0 * ctr.y - (((((ctr.x + e) + s.y) + nn.y) + below.y) + above.y);
        if (apj) {
            __builtin_nontemporal_store(y.x, apj + c);
            __builtin_nontemporal_store(y.y, apj + c + 1);
        }
        if constexpr (STEP == 0) {
            double2 pn;
            pn.x = theta * (minv * y.x - sigma * ctr.x);
            pn.y = theta * (minv * y.y - sigma * ctr.y);
            *reinterpret_cast<double2 *>(pnext + c) = pn;
        } else if constexpr (STEP == 1) {
            double2 pp;
            pp.x = __builtin_nontemporal_load(pprev + c);
            pp.y = __builtin_nontemporal_load(pprev + c + 1);
            const double two_theta = 2.0 * theta;
            double2 pn;
            pn.x = two_theta * (minv * y.x - sigma * ctr.x) - pp.x;
            pn.y = two_theta * (minv * y.y - sigma * ctr.y) - pp.y;
            *reinterpret_cast<double2 *>(pnext + c) = pn;
        }
        below = ctr;
        ctr = above;
        c += g.nxy;
    }
}

// CSR step with the block's rows staged: a block owns kBlock consecutive rows;
// their column indices and values (when they fit in LDS) are first copied into
// LDS with coalesced loads, then each thread forms its row's product from LDS.
template <typename T, int STEP>
__global__ __launch_bounds__(kBlock) void k_basis_csr(const DevState *__restrict__ st, OpCsr<T> op,
                                                      const T *__restrict__ pj, const T *__restrict__ pprev,
                                                      T *__restrict__ apj, T *__restrict__ pnext, T theta, T sigma,
                                                      int64_t n)
{
    constexpr int kCap = kBlock * 8;  // staged entries (up to 8 per row on average)
    __shared__ T sv[kCap];
    __shared__ int32_t sc[kCap];
    if (st->done)
        return;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kBlock;
    const int64_t r1 = r0 + kBlock < n ? r0 + kBlock : n;
    const int32_t kb = op.rp[r0], ke = op.rp[r1];
    const bool staged = ke - kb <= kCap;
    if (staged)
        for (int32_t t = threadIdx.x; t < ke - kb; t += kBlock) {
            sv[t] = op.val[kb + t];
            sc[t] = op.ci[kb + t];
        }
    __syncthreads();
    const int64_t c = r0 + threadIdx.x;
    if (c >= n)
        return;
    T acc = T(0);
    const int32_t a = op.rp[c], b = op.rp[c + 1];
    if (staged) {
        for (int32_t k = a; k < b; ++k)
            acc += sv[k - kb] * pj[sc[k - kb]];
    } else {
        for (int32_t k = a; k < b; ++k)
            acc += op.val[k] * pj[op.ci[k]];
    }
    const T pc = pj[c];
    const T dinv = op.invd[c];
    if (apj)  // AP is not kept by the recurrence Gram kind
        __builtin_nontemporal_store(acc, apj + c);
    if constexpr (STEP == 0) {
        pnext[c] = theta * (dinv * acc - sigma * pc);
    } else if constexpr (STEP == 1) {
        const T two_theta = T(2) * theta;
        pnext[c] = two_theta * (dinv * acc - sigma * pc) - pprev[c];
    }
}

// x += P alpha, alpha = S atil from the FGS kernel (FP64; P in FP64 or FP32).
// P is read once: non-temporal loads, plain block order (both measured
// faster on MI355X than cached loads and an XCD-contiguous order).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(const DevState *__restrict__ st, const T *__restrict__ P,
                                                   int64_t ld, int s, int64_t n)
{
    if (st->done)
        return;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= n)
        return;
    double *__restrict__ x = st->x;
    double acc = 0.0;
    int i = 0;
    for (; i + 4 <= s; i += 4) {
        const T v0 = __builtin_nontemporal_load(P + (i + 0) * ld + c);
        const T v1 = __builtin_nontemporal_load(P + (i + 1) * ld + c);
        const T v2 = __builtin_nontemporal_load(P + (i + 2) * ld + c);
        const T v3 = __builtin_nontemporal_load(P + (i + 3) * ld + c);
        acc += static_cast<double>(v0) * st->alpha[i + 0];
        acc += static_cast<double>(v1) * st->alpha[i + 1];
        acc += static_cast<double>(v2) * st->alpha[i + 2];
        acc += static_cast<double>(v3) * st->alpha[i + 3];
    }
    for (; i < s; ++i)
        acc += static_cast<double>(__builtin_nontemporal_load(P + i * ld + c)) * st->alpha[i];
    x[c] += acc;
}

// FP32+IR only: p0scale = 2^-e with e the exponent of ||r_0|| / sqrt(n), so
// that p_0 has entries of order one; the scaling is exact and the column
// scaling of the Gram matrix absorbs it.  Reads the residual partials of a
// norm-only residual pass.
__global__ __launch_bounds__(kBlock) void k_p0scale(DevState *st, const double *__restrict__ rpart, int nbr,
                                                    double inv_sqrt_n)
{
    if (st->done)
        return;
    double acc = 0.0;
    for (int q = threadIdx.x; q < nbr; q += kBlock)
        acc += rpart[q];
    __shared__ double tot;
    block_sum_store(acc, &tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double rms = sqrt(tot) * inv_sqrt_n;
        st->p0scale = (rms > 0.0 && isfinite(rms)) ? ldexp(1.0, -ilogb(rms)) : 1.0;
    }
}

template <class Op>
__global__ __launch_bounds__(kBlock) void k_apply(Op op, const double *__restrict__ x, double *__restrict__ y,
                                                  int64_t n, uint32_t per, uint32_t nbl)
{
    const uint32_t lb = xcd_block(blockIdx.x, per);
    if (lb >= nbl)
        return;
    const int64_t c = static_cast<int64_t>(lb) * kBlock + threadIdx.x;
    if (c >= n)
        return;
    double pc, yy, dinv;
    op.apply(x, c, pc, yy, dinv);
    y[c] = yy;
}

// dA = -lam x^T on the CSR pattern.
__global__ __launch_bounds__(kBlock) void k_grad_csr(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                     const double *__restrict__ lam, const double *__restrict__ x,
                                                     double *__restrict__ dA, int64_t n, int accumulate)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double li = lam[i];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const double g = -li * x[ci[k]];
        dA[k] = accumulate ? dA[k] + g : g;
    }
}

// Face gradient for one face array.  Faces along axis a are indexed
// (c0, c1, c2) with c_a in [0, N_a] (N_a + 1 faces) and the other two
// coordinates over the grid; face f separates cells f-1 and f along a.
// interior: -(lam_p - lam_q)(x_p - x_q); boundary: -lam_p x_p.
__global__ __launch_bounds__(kBlock) void k_grad_faces(const double *__restrict__ lam, const double *__restrict__ x,
                                                       double *__restrict__ dk, int nx, int ny, int nz, int axis,
                                                       int accumulate)
{
    const int fx = nx + (axis == 0), fy = ny + (axis == 1), fz = nz + (axis == 2);
    const int64_t nf = static_cast<int64_t>(fx) * fy * fz;
    const int64_t f = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (f >= nf)
        return;
    const int i = static_cast<int>(f % fx);
    const int64_t q = f / fx;
    const int j = static_cast<int>(q % fy);
    const int k = static_cast<int>(q / fy);
    const int64_t nxy = static_cast<int64_t>(nx) * ny;
    int pos, lim;
    int64_t stride;
    if (axis == 0) {
        pos = i, lim = nx, stride = 1;
    } else if (axis == 1) {
        pos = j, lim = ny, stride = nx;
    } else {
        pos = k, lim = nz, stride = nxy;
    }
    // cell on the high side of the face (coordinate pos along the axis)
    const int ci0 = axis == 0 ? (i < nx ? i : nx - 1) : i;
    const int cj0 = axis == 1 ? (j < ny ? j : ny - 1) : j;
    const int ck0 = axis == 2 ? (k < nz ? k : nz - 1) : k;
    const int64_t cell = ci0 + nx * (static_cast<int64_t>(cj0) + static_cast<int64_t>(ny) * ck0);
    double g;
    if (pos == 0) {
        g = -lam[cell] * x[cell];
    } else if (pos == lim) {
        g = -lam[cell] * x[cell];  // clamped to the last cell: the boundary face's own cell
    } else {
        const int64_t lo = cell - stride;
        g = -(lam[lo] - lam[cell]) * (x[lo] - x[cell]);
    }
    dk[f] = accumulate ? dk[f] + g : g;
}

__global__ __launch_bounds__(kBlock) void k_convert(const float *__restrict__ src, double *__restrict__ dst, int64_t n)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c < n)
        dst[c] = static_cast<double>(src[c]);
}

__global__ __launch_bounds__(kBlock) void k_to_fp32(const double *__restrict__ src, float *__restrict__ dst, int64_t n)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c < n)
        dst[c] = static_cast<float>(src[c]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_cols(const T *__restrict__ src, int64_t ld, int s, int64_t n,
                                                      double *__restrict__ dst)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= n)
        return;
    for (int j = 0; j < s; ++j)
        dst[j * n + c] = static_cast<double>(src[j * ld + c]);
}

// Diagonal of the face operator, summed in the order west, east, south,
// north, bottom, top.
// Flags a non-positive or non-finite diagonal.
__global__ __launch_bounds__(kBlock) void k_diag_faces(Grid3 g, const double *__restrict__ kx,
                                                       const double *__restrict__ ky, const double *__restrict__ kz,
                                                       double *__restrict__ dvec, int *__restrict__ bad, int64_t n)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= n)
        return;
    const uint32_t q = fdiv(static_cast<uint32_t>(c), g.dx);
    const uint32_t k = fdiv(q, g.dy);
    const int64_t fx = c + q;
    const int64_t fy = c + static_cast<int64_t>(k) * g.nx;
    const double d = ((((kx[fx] + kx[fx + 1]) + ky[fy]) + ky[fy + g.nx]) + kz[c]) + kz[c + g.nxy];
    dvec[c] = d;
    if (!(d > 0.0) || !isfinite(d))
        atomicOr(bad, 1);
}

// Diagonal of a CSR matrix; flags a missing, non-positive or non-finite entry.
__global__ __launch_bounds__(kBlock) void k_diag_csr(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                     const double *__restrict__ val, double *__restrict__ dvec,
                                                     int *__restrict__ bad, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n)
        return;
    double d = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i)
            d = val[k];
    dvec[i] = d;
    if (!(d > 0.0) || !isfinite(d))
        atomicOr(bad, 1);
}

__global__ __launch_bounds__(kBlock) void k_invert(const double *__restrict__ src, double *__restrict__ dst,
                                                   int64_t n, int precond)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c < n)
        dst[c] = precond ? 1.0 / src[c] : 1.0;
}



template <class Op, typename TP>
hipError_t residual_for(const IterArgs &a, const Op &op, hipStream_t st, bool write_p0)
{
    const uint32_t per = (static_cast<uint32_t>(a.nbr) + kNumXcd - 1) / kNumXcd;
    hipLaunchKernelGGL((k_residual<Op, TP>), dim3(per * kNumXcd), dim3(kBlock), 0, st, a.st, op,
                       static_cast<TP *>(a.P), a.rpart, a.op.n, a.rchunk, per, static_cast<uint32_t>(a.nbr),
                       a.p0_mode, write_p0 ? 1 : 0);
    return hipGetLastError();
}

template <typename TP>
hipError_t residual_t(const IterArgs &a, hipStream_t st, bool write_p0)
{
    switch (a.op.kind) {
    case kOpPoisson:
        if (a.res_p2) {
            const dim3 grid(static_cast<uint32_t>((a.op.g.nxy / 2 + 1023) / 1024),
                            static_cast<uint32_t>((a.op.g.nz + 7) / 8));
            hipLaunchKernelGGL(k_residual_p2<TP>, grid, dim3(1024), 0, st, a.st, a.op.g,
                               a.op.precond ? 1.0 / 6.0 : 1.0, static_cast<TP *>(a.P), a.rpart, a.p0_mode,
                               write_p0 ? 1 : 0);
            return hipGetLastError();
        }
        return residual_for<OpPoisson7<double>, TP>(a, make_poisson<double>(a.op), st, write_p0);
    case kOpFaces:
        return residual_for<OpFaces7<double>, TP>(a, Ops<double>::faces(a.op), st, write_p0);
    case kOpPoisson27:
        return residual_for<OpPoisson27<double>, TP>(a, make_poisson27<double>(a.op), st, write_p0);
    default:
        if (a.op.ell_col)
            return residual_for<OpEll<double>, TP>(a, Ops<double>::ell(a.op), st, write_p0);
        return residual_for<OpCsr<double>, TP>(a, Ops<double>::csr(a.op), st, write_p0);
    }
}

template <class Op, typename T>
hipError_t basis_for(const IterArgs &a, const Op &op, int j, int step, hipStream_t st)
{
    const Launch1D l = plan_points(a.op.n);
    T *P = static_cast<T *>(a.P);
    T *AP = static_cast<T *>(a.AP);
    const T *pj = P + j * a.ld;
    const T *pprev = j > 0 ? P + (j - 1) * a.ld : nullptr;
    T *apj = AP ? AP + j * a.ld : nullptr;
    T *pnext = j + 1 < a.s || a.gram_rec ? P + (j + 1) * a.ld : nullptr;
    const T theta = static_cast<T>(a.theta), sigma = static_cast<T>(a.sigma);
    if (a.gram_mom) {
        if (step == 2)
            return hipErrorInvalidValue;
        double *mp = a.mpart + static_cast<int64_t>(mom_slot(j)) * a.mstride;
        if (step == 0)
            hipLaunchKernelGGL((k_basis_mom<Op, T, 0>), dim3(l.grid), dim3(kBlock), 0, st, a.st, op, pj, pprev,
                               pnext, theta, sigma, a.op.n, l.per, l.nbl, mp, a.mstride);
        else
            hipLaunchKernelGGL((k_basis_mom<Op, T, 1>), dim3(l.grid), dim3(kBlock), 0, st, a.st, op, pj, pprev,
                               pnext, theta, sigma, a.op.n, l.per, l.nbl, mp, a.mstride);
        return hipGetLastError();
    }
    if (step == 2)
        hipLaunchKernelGGL((k_basis<Op, T, 2>), dim3(l.grid), dim3(kBlock), 0, st, a.st, op, pj, pprev, apj, pnext,
                           theta, sigma, a.op.n, l.per, l.nbl);
    else if (step == 0)
        hipLaunchKernelGGL((k_basis<Op, T, 0>), dim3(l.grid), dim3(kBlock), 0, st, a.st, op, pj, pprev, apj, pnext,
                           theta, sigma, a.op.n, l.per, l.nbl);
    else
        hipLaunchKernelGGL((k_basis<Op, T, 1>), dim3(l.grid), dim3(kBlock), 0, st, a.st, op, pj, pprev, apj, pnext,
                           theta, sigma, a.op.n, l.per, l.nbl);
    return hipGetLastError();
}

// FP64 constant Poisson with an even x-extent: pairs of points, two planes.
hipError_t basis_poisson_pairs(const IterArgs &a, int j, int step, hipStream_t st)
{
    const uint32_t gx = static_cast<uint32_t>((a.op.g.nxy / 2 + kP2Block - 1) / kP2Block);
    const uint32_t nbl = gx * static_cast<uint32_t>((a.op.g.nz + kP2Kz - 1) / kP2Kz);
    const uint32_t per = (nbl + kNumXcd - 1) / kNumXcd;
    const dim3 grid(per * kNumXcd);
    double *P = static_cast<double *>(a.P);
    double *AP = static_cast<double *>(a.AP);
    const double *pj = P + j * a.ld;
    const double *pprev = j > 0 ? P + (j - 1) * a.ld : nullptr;
    double *apj = AP ? AP + j * a.ld : nullptr;
    double *pnext = j + 1 < a.s || a.gram_rec ? P + (j + 1) * a.ld : nullptr;
    const double minv = a.op.precond ? 1.0 / 6.0 : 1.0;
    if (step == 2)
        hipLaunchKernelGGL(k_basis_p2<2>, grid, dim3(kP2Block), 0, st, a.st, a.op.g, minv, pj, pprev, apj, pnext,
                           a.theta, a.sigma, gx, per, nbl);
    else if (step == 0)
        hipLaunchKernelGGL(k_basis_p2<0>, grid, dim3(kP2Block), 0, st, a.st, a.op.g, minv, pj, pprev, apj, pnext,
                           a.theta, a.sigma, gx, per, nbl);
    else
        hipLaunchKernelGGL(k_basis_p2<1>, grid, dim3(kP2Block), 0, st, a.st, a.op.g, minv, pj, pprev, apj, pnext,
                           a.theta, a.sigma, gx, per, nbl);
    return hipGetLastError();
}

template <typename T>
hipError_t basis_csr(const IterArgs &a, int j, int step, hipStream_t st)
{
    const uint32_t nb = blocks_for(a.op.n);
    T *P = static_cast<T *>(a.P);
    T *AP = static_cast<T *>(a.AP);
    const T *pj = P + j * a.ld;
    const T *pprev = j > 0 ? P + (j - 1) * a.ld : nullptr;
    T *apj = AP ? AP + j * a.ld : nullptr;
    T *pnext = j + 1 < a.s || a.gram_rec ? P + (j + 1) * a.ld : nullptr;
    const T theta = static_cast<T>(a.theta), sigma = static_cast<T>(a.sigma);
    const OpCsr<T> op = Ops<T>::csr(a.op);
    if (step == 2)
        hipLaunchKernelGGL((k_basis_csr<T, 2>), dim3(nb), dim3(kBlock), 0, st, a.st, op, pj, pprev, apj, pnext, theta,
                           sigma, a.op.n);
    else if (step == 0)
        hipLaunchKernelGGL((k_basis_csr<T, 0>), dim3(nb), dim3(kBlock), 0, st, a.st, op, pj, pprev, apj, pnext, theta,
                           sigma, a.op.n);
    else
        hipLaunchKernelGGL((k_basis_csr<T, 1>), dim3(nb), dim3(kBlock), 0, st, a.st, op, pj, pprev, apj, pnext, theta,
                           sigma, a.op.n);
    return hipGetLastError();
}

// step 0: p_1 from p_0; 1: p_{j+1} from p_j, p_{j-1}; 2: the product A p_j only.
template <typename T>
hipError_t basis_t(const IterArgs &a, int j, int step, hipStream_t st)
{
    switch (a.op.kind) {
    case kOpPoisson:
        if constexpr (sizeof(T) == 8)
            if (a.op.g.nx % 2 == 0 && !a.gram_mom)
                return basis_poisson_pairs(a, j, step, st);
        return basis_for<OpPoisson7<T>, T>(a, make_poisson<T>(a.op), j, step, st);
    case kOpFaces:
        return basis_for<OpFaces7<T>, T>(a, Ops<T>::faces(a.op), j, step, st);
    case kOpPoisson27:
        return basis_for<OpPoisson27<T>, T>(a, make_poisson27<T>(a.op), j, step, st);
    default:
        if (a.op.ell_col)
            return basis_for<OpEll<T>, T>(a, Ops<T>::ell(a.op), j, step, st);
        return basis_csr<T>(a, j, step, st);
    }
}

// Two basis steps per launch (basis_f2.h) for the constant 7-point operator,
// shapes measured fastest on MI355X at 224^3: FP64 56-point tile rows
// (64-byte aligned stores), 3 planes of loads in flight; FP32 62-point rows,
// 6 planes.  With the moments Gram kind the products' FP64 accumulators take
// registers, and DM planes in flight (2 and 3) are the most that keep the
// kernel within 64 registers without spilling.  Ranges of 28 planes give 2 blocks per CU in one wave there;
// smaller grids take thinner ranges to keep some 512 blocks.
constexpr int kF2Rows = 16;
template <typename T>
struct F2Shape;
template <>
struct F2Shape<double> {
    static constexpr int D = 3, TXI = 56, DM = 2;
};
template <>
struct F2Shape<float> {
    static constexpr int D = 6, TXI = 62, DM = 3;
};

template <typename T>
F2Plan f2_plan(const Grid3 &g)
{
    constexpr int TXI = F2Shape<T>::TXI;
    const int64_t tiles = ((g.nx + TXI - 1) / TXI) * ((g.ny + kF2Rows - 3) / (kF2Rows - 2));
    int kz = 28;
    if (tiles * ((g.nz + kz - 1) / kz) < 512)
        kz = static_cast<int>(std::max<int64_t>(4, std::min<int64_t>(28, g.nz * tiles / 512)));
    return plan_f2<kF2Rows, TXI>(g, kz, 0);
}

template <typename T>
bool f2_fits(const IterArgs &a)
{
    return f2_window_bytes(a.op.g, f2_plan<T>(a.op.g).kz, sizeof(T)) < (int64_t(1) << 31);
}

// The two-step kernel serves the Chebyshev basis of the constant 7-point
// operator when AP is not stored (recurrence and operator-applying Gram kinds).
bool basis_pairs_apply(const IterArgs &a)
{
    if (a.op.kind != kOpPoisson || a.AP || a.monomial || a.one_step)
        return false;
    return a.fp32 ? f2_fits<float>(a) : f2_fits<double>(a);
}

// Columns p_1 .. p_m a basis forms: m = s - 1 when the Gram kernel applies the
// operator itself, else s (with AP stored, the last launch forms A p_{s-1}
// only; the recurrence kind forms p_s).
int basis_columns(const IterArgs &a) { return a.gram_op ? a.s - 1 : a.s; }

template <typename T>
hipError_t basis_pair(const IterArgs &a, int j, hipStream_t st)
{
    constexpr int D = F2Shape<T>::D, TXI = F2Shape<T>::TXI, DM = F2Shape<T>::DM;
    const F2Plan plan = f2_plan<T>(a.op.g);
    T *P = static_cast<T *>(a.P);
    const T *pprev = j > 0 ? P + (j - 1) * a.ld : nullptr;
    const T *pj = P + j * a.ld;
    T *q = P + (j + 1) * a.ld, *p2 = P + (j + 2) * a.ld;
    const T minv = a.op.precond ? T(1) / T(6) : T(1);
    const T theta = static_cast<T>(a.theta), sigma = static_cast<T>(a.sigma);
    const dim3 grid(plan.per * kNumXcd), block(kF2Lanes * kF2Rows);
    double *mp = a.gram_mom ? a.mpart + static_cast<int64_t>(mom_slot(j)) * a.mstride : nullptr;
    if (a.gram_mom) {
        if (j == 0)
            hipLaunchKernelGGL((k_basis_f2<T, kF2Rows, true, DM, 8, TXI, true>), grid, block, 0, st, a.st, a.op.g,
                               minv, pprev, pj, q, p2, theta, sigma, plan, mp, a.mstride);
        else
            hipLaunchKernelGGL((k_basis_f2<T, kF2Rows, false, DM, 8, TXI, true>), grid, block, 0, st, a.st, a.op.g,
                               minv, pprev, pj, q, p2, theta, sigma, plan, mp, a.mstride);
    } else if (j == 0) {
        hipLaunchKernelGGL((k_basis_f2<T, kF2Rows, true, D, 8, TXI, false>), grid, block, 0, st, a.st, a.op.g, minv,
                           pprev, pj, q, p2, theta, sigma, plan, mp, a.mstride);
    } else {
        hipLaunchKernelGGL((k_basis_f2<T, kF2Rows, false, D, 8, TXI, false>), grid, block, 0, st, a.st, a.op.g,
                           minv, pprev, pj, q, p2, theta, sigma, plan, mp, a.mstride);
    }
    return hipGetLastError();
}

// Sliced ELL from CSR (OpEll, common.h): one thread per row slot of every
// slice (rows at or beyond n are all padding).
__global__ __launch_bounds__(kBlock) void k_ell_fill_col(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                        const int64_t *__restrict__ off, int64_t n, int64_t nslice,
                                                        int32_t *__restrict__ col)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (r >= nslice * kEllSlice)
        return;
    const int64_t q = r / kEllSlice;
    const int64_t b = off[q] + (r - q * kEllSlice);
    const int w = static_cast<int>((off[q + 1] - off[q]) / kEllSlice);
    const int32_t k0 = r < n ? rp[r] : 0;
    const int len = r < n ? rp[r + 1] - k0 : 0;
    for (int k = 0; k < w; ++k)
        col[b + int64_t(k) * kEllSlice] = k < len ? ci[k0 + k] : -1;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ell_fill_val(const int32_t *__restrict__ rp, const T *__restrict__ val,
                                                        const int64_t *__restrict__ off, int64_t n, int64_t nslice,
                                                        T *__restrict__ ev)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (r >= nslice * kEllSlice)
        return;
    const int64_t q = r / kEllSlice;
    const int64_t b = off[q] + (r - q * kEllSlice);
    const int w = static_cast<int>((off[q + 1] - off[q]) / kEllSlice);
    const int32_t k0 = r < n ? rp[r] : 0;
    const int len = r < n ? rp[r + 1] - k0 : 0;
    for (int k = 0; k < w; ++k)
        ev[b + int64_t(k) * kEllSlice] = k < len ? val[k0 + k] : T(0);
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(uint64_t *__restrict__ p, int64_t words)
{
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < words;
         q += static_cast<int64_t>(gridDim.x) * kBlock)
        p[q] = 0;
}

__global__ void k_init_state(DevState *__restrict__ s, const double *b, double *x, double tol, int max_outer)
{
    if (threadIdx.x != 0)
        return;
    DevState h{};
    h.b = b;
    h.x = x;
    h.tol = tol;
    h.p0scale = 1.0;
    h.first = 1;
    h.max_outer = max_outer;
    *s = h;
}

// Row pointers of a CSR pattern: rp[0] = 0, rp[n] = nnz, non-decreasing.
__global__ __launch_bounds__(kBlock) void k_check_csr_rows(const int32_t *__restrict__ rp, int64_t n, int64_t nnz,
                                                           int *__restrict__ bad)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i > n)
        return;
    bool ok = true;
    if (i == 0)
        ok = rp[0] == 0;
    else
        ok = rp[i] >= rp[i - 1] && rp[i] <= nnz;
    if (i == n)
        ok = ok && rp[n] == nnz;
    if (!ok)
        atomicOr(bad, 1);
}

// Columns of a CSR pattern whose row pointers passed k_check_csr_rows: in
// [0, n) and strictly ascending within each row.
__global__ __launch_bounds__(kBlock) void k_check_csr_cols(const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci, int64_t n,
                                                           int *__restrict__ bad)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n)
        return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] < 0 || ci[k] >= n || (k > rp[i] && ci[k] <= ci[k - 1])) {
            atomicOr(bad, 1);
            return;
        }
}

}  // namespace

hipError_t launch_ell_fill_col(const OpDev &op, int32_t *col, hipStream_t st)
{
    const uint32_t grid = blocks_for(op.ell_nslice * kEllSlice);
    hipLaunchKernelGGL(k_ell_fill_col, dim3(grid), dim3(kBlock), 0, st, op.rp, op.ci, op.ell_off, op.n,
                       op.ell_nslice, col);
    return hipGetLastError();
}

hipError_t launch_ell_fill_val(const OpDev &op, const double *val, double *ev, hipStream_t st)
{
    const uint32_t grid = blocks_for(op.ell_nslice * kEllSlice);
    hipLaunchKernelGGL(k_ell_fill_val<double>, dim3(grid), dim3(kBlock), 0, st, op.rp, val, op.ell_off, op.n,
                       op.ell_nslice, ev);
    return hipGetLastError();
}

hipError_t launch_ell_fill_val(const OpDev &op, const float *val, float *ev, hipStream_t st)
{
    const uint32_t grid = blocks_for(op.ell_nslice * kEllSlice);
    hipLaunchKernelGGL(k_ell_fill_val<float>, dim3(grid), dim3(kBlock), 0, st, op.rp, val, op.ell_off, op.n,
                       op.ell_nslice, ev);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st)
{
    const int64_t words = static_cast<int64_t>(bytes / 8);
    if (words == 0)
        return hipSuccess;
    const uint32_t grid = static_cast<uint32_t>(std::min<int64_t>((words + kBlock - 1) / kBlock, 4096));
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(kBlock), 0, st, static_cast<uint64_t *>(p), words);
    return hipGetLastError();
}

hipError_t launch_init_state(DevState *s, const double *b, double *x, double tol, int max_outer, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(kWave), 0, st, s, b, x, tol, max_outer);
    return hipGetLastError();
}

hipError_t launch_check_csr_rows(const int32_t *rp, int64_t n, int64_t nnz, int *bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_csr_rows, dim3(blocks_for(n + 1)), dim3(kBlock), 0, st, rp, n, nnz, bad);
    return hipGetLastError();
}

hipError_t launch_check_csr_cols(const int32_t *rp, const int32_t *ci, int64_t n, int *bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_csr_cols, dim3(blocks_for(n)), dim3(kBlock), 0, st, rp, ci, n, bad);
    return hipGetLastError();
}

hipError_t launch_residual(const IterArgs &a, hipStream_t st, bool write_p0)
{
    const hipError_t e = a.fp32 ? residual_t<float>(a, st, write_p0) : residual_t<double>(a, st, write_p0);
    if (e != hipSuccess || !write_p0)
        return e;  // the norm-only pass of FP32+IR runs no stopping test
    hipLaunchKernelGGL(k_stop, dim3(1), dim3(kSumThreads), 0, st, a.st, a.rpart, a.nbr, a.dbg + dbg_rho(a.s), a.hist,
                       a.hist_cap);
    return hipGetLastError();
}

hipError_t launch_p0scale(const IterArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_p0scale, dim3(1), dim3(kBlock), 0, st, a.st, a.rpart, a.nbr, a.inv_sqrt_n);
    return hipGetLastError();
}

hipError_t launch_basis(const IterArgs &a, int j, hipStream_t st)
{
    // the last launch forms only A p_{s-1} (stored AP), or p_s (recurrence kind)
    const bool last_product = j + 1 >= a.s && !a.gram_rec;
    if (a.monomial) {
        // p_{j+1} = theta (M^{-1} A p_j - sigma p_j) with theta = 1, sigma = 0
        IterArgs m = a;
        m.theta = 1.0;
        m.sigma = 0.0;
        const int step = last_product ? 2 : 0;
        return a.fp32 ? basis_t<float>(m, j, step, st) : basis_t<double>(m, j, step, st);
    }
    const int step = last_product ? 2 : (j == 0 ? 0 : 1);
    return a.fp32 ? basis_t<float>(a, j, step, st) : basis_t<double>(a, j, step, st);
}

int basis_kernel_count(const IterArgs &a, int *pairs)
{
    const int m = basis_columns(a);
    if (!basis_pairs_apply(a)) {
        if (pairs)
            *pairs = 0;
        return a.gram_op ? a.s - 1 : a.s;
    }
    if (pairs)
        *pairs = m / 2;
    return m / 2 + m % 2;
}

hipError_t launch_basis_all(const IterArgs &a, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (!basis_pairs_apply(a)) {
        for (int j = 0; j < basis_kernel_count(a, nullptr) && e == hipSuccess; ++j)
            e = launch_basis(a, j, st);
        return e;
    }
    const int m = basis_columns(a);
    int j = 0;
    for (; j + 2 <= m && e == hipSuccess; j += 2)
        e = a.fp32 ? basis_pair<float>(a, j, st) : basis_pair<double>(a, j, st);
    if (j < m && e == hipSuccess)
        e = launch_basis(a, j, st);  // an odd count: the last column alone
    return e;
}

void mom_layout(const IterArgs &a, int32_t *cnt, int64_t *stride)
{
    const int m = basis_columns(a);
    int64_t mx = 0;
    auto put = [&](int j, int ncols, int64_t nbl) {
        const int first = mom_slot(j);
        const int nslot = (j == 0 ? 1 : 0) + 2 * ncols;
        for (int k = first; k < first + nslot; ++k)
            cnt[k] = static_cast<int32_t>(nbl);
        mx = std::max(mx, nbl);
    };
    int j = 0;
    if (basis_pairs_apply(a)) {
        const int64_t nbl = a.fp32 ? f2_plan<float>(a.op.g).nbl : f2_plan<double>(a.op.g).nbl;
        for (; j + 2 <= m; j += 2)
            put(j, 2, nbl);
    }
    for (; j < m; ++j)
        put(j, 1, plan_points(a.op.n).nbl);
    *stride = mx;
}

hipError_t launch_product(const IterArgs &a, int j, hipStream_t st)
{
    IterArgs p = a;  // A p_j alone: no products for the moments kind
    p.gram_mom = 0;
    return a.fp32 ? basis_t<float>(p, j, 2, st) : basis_t<double>(p, j, 2, st);
}

hipError_t launch_update(const IterArgs &a, hipStream_t st)
{
    const dim3 grid(blocks_for(a.op.n));
    if (a.fp32)
        hipLaunchKernelGGL(k_update<float>, grid, dim3(kBlock), 0, st, a.st, static_cast<const float *>(a.P), a.ld,
                           a.s, a.op.n);
    else
        hipLaunchKernelGGL(k_update<double>, grid, dim3(kBlock), 0, st, a.st, static_cast<const double *>(a.P), a.ld,
                           a.s, a.op.n);
    return hipGetLastError();
}

hipError_t launch_apply(const OpDev &op, const double *x, double *y, hipStream_t st)
{
    const Launch1D l = plan_points(op.n);
    switch (op.kind) {
    case kOpPoisson:
        hipLaunchKernelGGL(k_apply<OpPoisson7<double>>, dim3(l.grid), dim3(kBlock), 0, st, make_poisson<double>(op),
                           x, y, op.n, l.per, l.nbl);
        break;
    case kOpFaces:
        hipLaunchKernelGGL(k_apply<OpFaces7<double>>, dim3(l.grid), dim3(kBlock), 0, st, Ops<double>::faces(op), x,
                           y, op.n, l.per, l.nbl);
        break;
    case kOpPoisson27:
        hipLaunchKernelGGL(k_apply<OpPoisson27<double>>, dim3(l.grid), dim3(kBlock), 0, st,
                           make_poisson27<double>(op), x, y, op.n, l.per, l.nbl);
        break;
    default:
        if (op.ell_col)
            hipLaunchKernelGGL(k_apply<OpEll<double>>, dim3(l.grid), dim3(kBlock), 0, st, Ops<double>::ell(op), x,
                               y, op.n, l.per, l.nbl);
        else
            hipLaunchKernelGGL(k_apply<OpCsr<double>>, dim3(l.grid), dim3(kBlock), 0, st, Ops<double>::csr(op), x,
                               y, op.n, l.per, l.nbl);
    }
    return hipGetLastError();
}

hipError_t launch_grad(const OpDev &op, const double *lam, const double *x, double *dA, int accumulate,
                       hipStream_t st)
{
    if (op.kind == kOpPoisson27)
        return hipErrorInvalidValue;  // no coefficients to differentiate
    if (op.kind == kOpCsr) {
        hipLaunchKernelGGL(k_grad_csr, dim3(blocks_for(op.n)), dim3(kBlock), 0, st, op.rp, op.ci, lam, x, dA, op.n,
                           accumulate);
        return hipGetLastError();
    }
    const int nx = op.g.nx, ny = op.g.ny, nz = op.g.nz;
    const int64_t nfx = static_cast<int64_t>(nx + 1) * ny * nz;
    const int64_t nfy = static_cast<int64_t>(nx) * (ny + 1) * nz;
    const int64_t nfz = static_cast<int64_t>(nx) * ny * (nz + 1);
    hipLaunchKernelGGL(k_grad_faces, dim3(blocks_for(nfx)), dim3(kBlock), 0, st, lam, x, dA, nx, ny, nz, 0,
                       accumulate);
    hipLaunchKernelGGL(k_grad_faces, dim3(blocks_for(nfy)), dim3(kBlock), 0, st, lam, x, dA + nfx, nx, ny, nz, 1,
                       accumulate);
    hipLaunchKernelGGL(k_grad_faces, dim3(blocks_for(nfz)), dim3(kBlock), 0, st, lam, x, dA + nfx + nfy, nx, ny, nz,
                       2, accumulate);
    return hipGetLastError();
}

hipError_t launch_convert(const float *src, double *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_convert, dim3(blocks_for(n)), dim3(kBlock), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_copy_cols(const void *src, int64_t ld, int fp32, int s, int64_t n, double *dst, hipStream_t st)
{
    if (fp32)
        hipLaunchKernelGGL(k_copy_cols<float>, dim3(blocks_for(n)), dim3(kBlock), 0, st,
                           static_cast<const float *>(src), ld, s, n, dst);
    else
        hipLaunchKernelGGL(k_copy_cols<double>, dim3(blocks_for(n)), dim3(kBlock), 0, st,
                           static_cast<const double *>(src), ld, s, n, dst);
    return hipGetLastError();
}

hipError_t launch_diag_from_faces(const OpDev &op, double *dvec, int *bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_faces, dim3(blocks_for(op.n)), dim3(kBlock), 0, st, op.g, op.kx, op.ky, op.kz, dvec,
                       bad, op.n);
    return hipGetLastError();
}

hipError_t launch_diag_from_csr(const OpDev &op, double *dvec, int *bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_csr, dim3(blocks_for(op.n)), dim3(kBlock), 0, st, op.rp, op.ci, op.val, dvec, bad,
                       op.n);
    return hipGetLastError();
}

hipError_t launch_to_fp32(const double *src, float *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_fp32, dim3(blocks_for(n)), dim3(kBlock), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_invert(const double *src, double *dst, int64_t n, int precond, hipStream_t st)
{
    hipLaunchKernelGGL(k_invert, dim3(blocks_for(n)), dim3(kBlock), 0, st, src, dst, n, precond);
    return hipGetLastError();
}

}  // namespace sstep
