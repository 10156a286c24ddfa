// Spectrum bounds for the Chebyshev basis by Lanczos (Sec. 8, setup of the
// experiments): a few Lanczos steps on M^{-1}A give Ritz values that
// approximate its extreme eigenvalues from inside.
//
// M^{-1}A is self-adjoint in the M-inner product <u, v>_M = u^T M v, so the
// recurrence runs on M-orthonormal vectors z_j (no reorthogonalisation):
//     z_0 = u / ||u||_M,  beta_0 = 0,
//     y = A z_j,  alpha_j = z_j^T y,
//     w = M^{-1} y - alpha_j z_j - beta_j z_{j-1},
//     beta_{j+1} = ||w||_M,  z_{j+1} = w / beta_{j+1},
// stopping early (m = j + 1 steps) when beta_{j+1} is not above
// 1e-13 max_{i<=j} |alpha_i| or not finite.  The Ritz values are the
// eigenvalues of the m x m tridiagonal T_m = tridiag(beta; alpha; beta),
// found on the device by bisection on Sturm counts, one lane per eigenvalue.
//
// Every pass is a streaming kernel over row chunks (one partial sum per
// block, kSumThreads-thread fixed-order sums), HBM-bound like the basis
// kernels; the whole estimate is a setup cost of a few passes per step.
#include "launch.h"
#include "opsel.h"
#include "stop.h"

namespace sstep {
namespace {

// M diagonal and its inverse at a point: constant (Poisson, or no
// preconditioner) or from the library's diagonal arrays.
struct Diag {
    const double *d;     // M diagonal, or null for the constant dconst
    const double *dinv;  // M^{-1} diagonal (CSR), or null: 1/d
    double dconst;

    __device__ __forceinline__ void at(int64_t c, double &dd, double &di) const
    {
        if (d) {
            dd = d[c];
            di = dinv ? dinv[c] : 1.0 / dd;
        } else {
            dd = dconst;
            di = 1.0 / dconst;
        }
    }
};

__device__ __forceinline__ void block_partial(double v, double *out)
{
    __shared__ double part[kBlock / kWave];
    v = wave_sum(v);
    if (threadIdx.x % kWave == 0)
        part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = part[0];
#pragma unroll
        for (int q = 1; q < kBlock / kWave; ++q)
            acc += part[q];
        *out = acc;
    }
}

// Partial sums of ||u||_M^2 = sum d u^2.
__global__ __launch_bounds__(kBlock) void k_lz_norm0(const LzState *__restrict__ ls, Diag dg,
                                                     const double *__restrict__ u, double *__restrict__ part,
                                                     int64_t n, int64_t chunk)
{
    const int64_t beg = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
        double d, di;
        dg.at(c, d, di);
        acc += d * u[c] * u[c];
    }
    block_partial(acc, part + blockIdx.x);
}

// z = v / ls->scale (the start vector, or w with scale = beta_{j+1}).
__global__ __launch_bounds__(kBlock) void k_lz_scale(const LzState *__restrict__ ls, const double *__restrict__ v,
                                                     double *__restrict__ z, int64_t n)
{
    if (ls->stopped)
        return;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c < n)
        z[c] = v[c] / ls->scale;
}

// y = A z_j and partial sums of z_j^T y.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_lz_apply(const LzState *__restrict__ ls, Op op,
                                                     const double *__restrict__ z, double *__restrict__ y,
                                                     double *__restrict__ part, int64_t n, int64_t chunk)
{
    if (ls->stopped)
        return;
    const int64_t beg = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
        double pc, yy, dinv;
        op.apply(z, c, pc, yy, dinv);
        y[c] = yy;
        acc += pc * yy;
    }
    block_partial(acc, part + blockIdx.x);
}

// w = M^{-1} y - alpha_j z_j - beta_j z_{j-1} (in place of y) and partial
// sums of ||w||_M^2.
__global__ __launch_bounds__(kBlock) void k_lz_orth(const LzState *__restrict__ ls, Diag dg,
                                                    double *__restrict__ y, const double *__restrict__ z,
                                                    const double *__restrict__ zprev, const double *__restrict__ ab,
                                                    int j, int steps, double *__restrict__ part, int64_t n,
                                                    int64_t chunk)
{
    if (ls->stopped)
        return;
    const double aj = ab[j];
    const double bj = j > 0 ? ab[steps + j - 1] : 0.0;
    const int64_t beg = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
        double d, di;
        dg.at(c, d, di);
        const double zp = j > 0 ? zprev[c] : 0.0;
        const double w = di * y[c] - aj * z[c] - bj * zp;
        y[c] = w;
        acc += d * w * w;
    }
    block_partial(acc, part + blockIdx.x);
}

// The fixed-order sum of the block partials and what follows from it:
//   kind 0: ||u||_M (start vector): scale = it, stop with m = 0 unless > 0;
//   kind 1: alpha_j = the sum, amax = max(amax, |alpha_j|);
//   kind 2: beta_{j+1} = sqrt(sum), scale = beta_{j+1}, m = j + 1, stop when
//           beta_{j+1} <= 1e-13 amax or not finite.
__global__ __launch_bounds__(kSumThreads) void k_lz_sum(LzState *__restrict__ ls, const double *__restrict__ part,
                                                        int cnt, int kind, int j, int steps,
                                                        double *__restrict__ ab)
{
    if (ls->stopped)
        return;
    const double v = fixed_order_sum(part, cnt);
    if (threadIdx.x != 0)
        return;
    if (kind == 0) {
        const double un = sqrt(v);
        ls->scale = un;
        ls->m = 0;
        ls->amax = 0.0;
        if (!(un > 0.0) || !isfinite(un))
            ls->stopped = 1;
    } else if (kind == 1) {
        ab[j] = v;
        ls->amax = fmax(ls->amax, fabs(v));
    } else {
        const double bn = sqrt(v);
        ab[steps + j] = bn;
        ls->scale = bn;
        ls->m = j + 1;
        if (!(bn > 1e-13 * ls->amax) || !isfinite(bn))
            ls->stopped = 1;
    }
}

// Number of eigenvalues of T_m below x (Sturm count: negative pivots of the
// LDL^T factorisation of T_m - x I).
__device__ int sturm_count(const double *al, const double *be, int m, double x, double pivmin)
{
    int cnt = 0;
    double d = al[0] - x;
    if (fabs(d) < pivmin)
        d = -pivmin;
    cnt += d < 0.0;
    for (int i = 1; i < m; ++i) {
        d = (al[i] - x) - be[i - 1] * be[i - 1] / d;
        if (fabs(d) < pivmin)
            d = -pivmin;
        cnt += d < 0.0;
    }
    return cnt;
}

// Ritz values of T_m, ascending: lane k bisects for the k-th smallest
// eigenvalue inside the Gershgorin interval of T_m until the interval can
// no longer be halved in FP64.
__global__ __launch_bounds__(kWave) void k_lz_ritz(const LzState *__restrict__ ls, const double *__restrict__ ab,
                                                   int steps, double *__restrict__ ritz)
{
    __shared__ double al[kMaxLanczos], be[kMaxLanczos];
    const int m = ls->m;
    for (int i = threadIdx.x; i < m; i += kWave) {
        al[i] = ab[i];
        be[i] = ab[steps + i];
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k >= m)
        return;
    double lo = al[0], hi = al[0], tmax = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < m ? fabs(be[i]) : 0.0);
        lo = fmin(lo, al[i] - r);
        hi = fmax(hi, al[i] + r);
        tmax = fmax(tmax, fabs(al[i]) + r);
    }
    const double pivmin = 1e-300 + 4.0 * 2.2250738585072014e-308 * fmax(1.0, tmax * tmax);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        if (sturm_count(al, be, m, mid, pivmin) <= k)
            lo = mid;
        else
            hi = mid;
    }
    ritz[k] = 0.5 * (lo + hi);
}

Diag diag_of(const OpDev &op)
{
    if (!op.precond)
        return Diag{nullptr, nullptr, 1.0};
    if (op.kind == kOpPoisson)
        return Diag{nullptr, nullptr, 6.0};
    if (op.kind == kOpPoisson27)
        return Diag{nullptr, nullptr, 26.0};
    if (op.kind == kOpFaces)
        return Diag{op.dvec, nullptr, 1.0};
    return Diag{op.dvec, op.invd, 1.0};
}

template <class Op>
hipError_t apply_step(const LzArgs &l, const Op &op, const double *z, double *y, hipStream_t st)
{
    hipLaunchKernelGGL((k_lz_apply<Op>), dim3(l.nb), dim3(kBlock), 0, st, l.ls, op, z, y, l.part, l.n, l.chunk);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lanczos(const LzArgs &l, const OpDev &op, const double *u, int steps, hipStream_t st)
{
    const Diag dg = diag_of(op);
    const uint32_t pts = static_cast<uint32_t>((l.n + kBlock - 1) / kBlock);
    double *zprev = l.v[0], *z = l.v[1], *y = l.v[2];
    hipLaunchKernelGGL(k_lz_norm0, dim3(l.nb), dim3(kBlock), 0, st, l.ls, dg, u, l.part, l.n, l.chunk);
    hipLaunchKernelGGL(k_lz_sum, dim3(1), dim3(kSumThreads), 0, st, l.ls, l.part, l.nb, 0, 0, steps, l.ab);
    hipLaunchKernelGGL(k_lz_scale, dim3(pts), dim3(kBlock), 0, st, l.ls, u, z, l.n);
    for (int j = 0; j < steps; ++j) {
        hipError_t e;
        if (op.kind == kOpPoisson)
            e = apply_step(l, make_poisson<double>(op), z, y, st);
        else if (op.kind == kOpPoisson27)
            e = apply_step(l, make_poisson27<double>(op), z, y, st);
        else if (op.kind == kOpFaces)
            e = apply_step(l, Ops<double>::faces(op), z, y, st);
        else if (op.ell_col)
            e = apply_step(l, Ops<double>::ell(op), z, y, st);
        else
            e = apply_step(l, Ops<double>::csr(op), z, y, st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_lz_sum, dim3(1), dim3(kSumThreads), 0, st, l.ls, l.part, l.nb, 1, j, steps, l.ab);
        hipLaunchKernelGGL(k_lz_orth, dim3(l.nb), dim3(kBlock), 0, st, l.ls, dg, y, z, zprev, l.ab, j, steps,
                           l.part, l.n, l.chunk);
        hipLaunchKernelGGL(k_lz_sum, dim3(1), dim3(kSumThreads), 0, st, l.ls, l.part, l.nb, 2, j, steps, l.ab);
        if (j + 1 < steps) {
            // z_{j+1} = w / beta_{j+1} into the buffer of z_{j-1}; rotate
            hipLaunchKernelGGL(k_lz_scale, dim3(pts), dim3(kBlock), 0, st, l.ls, y, zprev, l.n);
            double *t = zprev;
            zprev = z;
            z = t;
        }
    }
    hipLaunchKernelGGL(k_lz_ritz, dim3(1), dim3(kWave), 0, st, l.ls, l.ab, steps, l.ab + 2 * steps);
    return hipGetLastError();
}

}  // namespace sstep
