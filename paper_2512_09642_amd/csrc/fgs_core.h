// Stopping test, column scaling and forward Gauss-Seidel on the reduced Gram
// system, executed by one wave.  Shared by the single-system and the batched
// outer iterations.
#pragma once

#include "gram_impl.h"
#include "stop.h"

namespace sstep {

// Value of v held by lane l (l uniform across the wave), as scalar registers.
__device__ __forceinline__ double readlane(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// sg holds the reduced sums: Gram entries in canonical order (lower triangle
// row by row, then the right-hand side).  The stopping test of iteration k
// has already run (stop.h), and st->rho holds ||r_k||.
// 1. Column scaling (Sec. 2): d_i = G_raw,ii^{-1/2}; G = S G_raw S with the
//    diagonal set to one and each off-diagonal pair scaled once from the lower
//    triangle, so G is exactly symmetric; ctil = S c.  A diagonal entry that is
//    not positive and finite is a breakdown.
// 2. nu forward Gauss-Seidel sweeps from atil = 0 (Sec. 2, FGS iteration;
//    Sec. 3), j = 0..s-1 in order, in residual form: lane i keeps row i of G
//    and rho_i = ctil_i - (G atil)_i; visiting j adds rho_j to atil_j and
//    subtracts G_ij rho_j from every rho_i -- the same update as
//    atil_j <- ctil_j - sum_{i != j} G_ji atil_i since G_jj = 1.
// 3. alpha = S atil for the update kernel; delta = ||ctil - G atil|| / ||ctil||
//    (the Gram-solve accuracy of Sec. 7), ||L||_F of the strictly lower part
//    of G (Sec. 4) and their histories.
// The basis width s is a template parameter so that the nu*s dependent steps of
// the sweeps carry no bound checks.  Returns 1 on a breakdown (the solve is
// stopped).
template <int s>
__device__ __forceinline__ int fgs_wave(DevState *__restrict__ st, const double *__restrict__ sg, int nu,
                                        double cscale, int fp32, double inv_sqrt_n, double *__restrict__ dbg,
                                        double *__restrict__ hist, int hist_cap)
{
    const int lane = threadIdx.x % kWave;
    constexpr int T0 = s * (s + 1) / 2;
    const int k = st->iter;
    const double rho = st->rho;

    // ---- column scaling -----------------------------------------------------
    const int i = lane;
    const bool own = i < s;
    const double gii = own ? sg[tri_index(i, i)] : 1.0;
    const bool bad = own && !(gii > 0.0 && isfinite(gii));
    if (__any(bad)) {
        if (lane == 0) {
            st->status = 4;  // SSTEP_E_BREAKDOWN
            st->done = 1;
        }
        return 1;
    }
    // c = P^T r: the reduction formed P^T (M p_0) (times cscale for a constant
    // M) with p_0 = p0scale * M^{-1} r, so divide the scale back out.
    const double d = own ? 1.0 / sqrt(gii) : 0.0;
    const double ct = own ? d * (sg[T0 + i] * cscale / st->p0scale) : 0.0;
    double grow[s];
#pragma unroll
    for (int j = 0; j < s; ++j) {
        double g = 0.0;
        {
            const double dj = readlane(d, j);
            if (own) {
                if (i == j)
                    g = 1.0;
                else if (i > j)
                    g = (d * sg[tri_index(i, j)]) * dj;
                else
                    g = (dj * sg[tri_index(j, i)]) * d;
            }
        }
        grow[j] = g;
    }

    // ---- forward Gauss-Seidel, residual form ---------------------------------
    double rv = ct, a = 0.0;
    for (int sweep = 0; sweep < nu; ++sweep) {
#pragma unroll
        for (int j = 0; j < s; ++j) {
            const double delta = readlane(rv, j);
            if (i == j)
                a += delta;
            rv -= grow[j] * delta;
        }
    }

    // ---- outputs --------------------------------------------------------------
    double res = ct;
#pragma unroll
    for (int j = 0; j < s; ++j)
        res -= grow[j] * readlane(a, j);
    const double num = wave_sum(res * res);
    const double den = wave_sum(ct * ct);
    const double delta = den > 0.0 ? sqrt(num / den) : 0.0;
    double lsq = 0.0;
#pragma unroll
    for (int j = 0; j < s; ++j)
        if (j < i)
            lsq += grow[j] * grow[j];
    const double lnorm = sqrt(wave_sum(lsq));
    if (own) {
        st->alpha[i] = d * a;
        dbg[dbg_ctil(s) + i] = ct;
        dbg[dbg_atil(s) + i] = a;
        dbg[dbg_d(s) + i] = d;
#pragma unroll
        for (int j = 0; j < s; ++j)
            dbg[i * s + j] = grow[j];
    }
    if (lane == 0) {
        st->delta = delta;
        st->lnorm = lnorm;
        if (k < hist_cap) {
            hist[hist_cap + k] = delta;
            hist[2 * hist_cap + k] = lnorm;
        }
        st->iter = k + 1;
        if (fp32) {
            const double rms = rho * inv_sqrt_n;
            st->p0scale = (rms > 0.0 && isfinite(rms)) ? ldexp(1.0, -ilogb(rms)) : 1.0;
        }
    }
    return 0;
}

constexpr int kFgsThreads = 256;

// Sum of the block partials of one Gram entry e (one block per entry), in a
// fixed order: thread t takes partials t, t + 256, ..., the waves combine by
// butterfly and the four wave sums in order.  One block per entry keeps every
// partial load of the reduction in flight at once across the chip.
template <int s>
__global__ __launch_bounds__(kSumThreads) void k_partial_sums(const DevState *__restrict__ st,
                                                              const double *__restrict__ gpart, int nbg,
                                                              double *__restrict__ sums)
{
    __shared__ double part[kSumThreads / kWave];
    if (st->done)
        return;
    const int e = blockIdx.x;
    const double *src = gpart + static_cast<int64_t>(e) * nbg;
    double acc = 0.0;
    for (int q = threadIdx.x; q < nbg; q += kSumThreads)
        acc += src[q];
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0)
        part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < kSumThreads / kWave; ++w)
            v += part[w];
        sums[e] = v;
    }
}

// One outer iteration's Gram solve for a single system: the block loads the
// totals of the E Gram entries and of ||r||^2 (k_partial_sums) into LDS, then
// wave 0 runs fgs_wave.
template <int s>
__global__ __launch_bounds__(kFgsThreads) void k_fgs(DevState *__restrict__ st, const double *__restrict__ sums, int nu,
                                                     double cscale, int fp32, double inv_sqrt_n,
                                                     double *__restrict__ dbg, double *__restrict__ hist,
                                                     int hist_cap)
{
    if (st->done)
        return;
    __shared__ double sg[s * (s + 1) / 2 + s];
    constexpr int E = s * (s + 1) / 2 + s;
    const int wave = threadIdx.x / kWave;
    for (int t = threadIdx.x; t < E; t += kFgsThreads)
        sg[t] = sums[t];
    __syncthreads();
    if (wave != 0)
        return;
    fgs_wave<s>(st, sg, nu, cscale, fp32, inv_sqrt_n, dbg, hist, hist_cap);
}

// The recurrence kind: the sums hold the M-weighted Gram H = P^T M P of the
// s + 1 columns p_0 .. p_s (lower triangle, canonical order) and c'_i (s + 1
// entries).  The Chebyshev recurrence of the basis (Sec. 2, Definition) gives
//     M^{-1} A p_0 = p_1 / theta + sigma p_0,
//     M^{-1} A p_j = (p_{j+1} + p_{j-1}) / (2 theta) + sigma p_j,   j >= 1,
// (the monomial basis: M^{-1} A p_j = p_{j+1}), hence
//     G_raw,ij = p_i^T A p_j = H_i1 / theta + sigma H_i0                (j = 0)
//              = (H_i,j+1 + H_i,j-1) / (2 theta) + sigma H_ij          (j >= 1),
// the same matrix P^T (A P) without applying A.  hscale is the constant M
// diagonal (6, 26 or 1) when the kernel did not weight by M itself.  The
// block writes G_raw (lower triangle) and c' for the s columns into LDS in
// the layout of k_fgs, then wave 0 runs fgs_wave.
// The block's part after h (LDS, the layout above) is filled and synchronised.
template <int s>
__device__ __forceinline__ void fgs_rec_from_h(DevState *__restrict__ st, const double *h, int nu, double cscale,
                                               int fp32, double inv_sqrt_n, double *__restrict__ dbg,
                                               double *__restrict__ hist, int hist_cap, double theta, double sigma,
                                               double hscale, int monomial)
{
    constexpr int S1 = s + 1;
    constexpr int T0 = s * (s + 1) / 2;
    __shared__ double sg[T0 + s];
    auto H = [&](int a, int b) { return a >= b ? h[tri_index(a, b)] : h[tri_index(b, a)]; };
    for (int e = threadIdx.x; e < T0; e += kFgsThreads) {
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= e)
            ++i;
        const int j = e - i * (i + 1) / 2;
        double g;
        if (monomial)
            g = H(i, j + 1);
        else if (j == 0)
            g = H(i, 1) / theta + sigma * H(i, 0);
        else
            g = (H(i, j + 1) + H(i, j - 1)) / (2.0 * theta) + sigma * H(i, j);
        sg[e] = hscale * g;
    }
    for (int i = threadIdx.x; i < s; i += kFgsThreads)
        sg[T0 + i] = h[S1 * (S1 + 1) / 2 + i];
    __syncthreads();
    if (threadIdx.x / kWave != 0)
        return;
    fgs_wave<s>(st, sg, nu, cscale, fp32, inv_sqrt_n, dbg, hist, hist_cap);
}

template <int s>
__global__ __launch_bounds__(kFgsThreads) void k_fgs_rec(DevState *__restrict__ st, const double *__restrict__ sums,
                                                         int nu, double cscale, int fp32, double inv_sqrt_n,
                                                         double *__restrict__ dbg, double *__restrict__ hist,
                                                         int hist_cap, double theta, double sigma, double hscale,
                                                         int monomial)
{
    if (st->done)
        return;
    constexpr int S1 = s + 1;
    constexpr int E1 = S1 * (S1 + 1) / 2 + S1;
    __shared__ double h[E1];
    for (int t = threadIdx.x; t < E1; t += kFgsThreads)
        h[t] = sums[t];
    __syncthreads();
    fgs_rec_from_h<s>(st, h, nu, cscale, fp32, inv_sqrt_n, dbg, hist, hist_cap, theta, sigma, hscale, monomial);
}

// The Gram matrix of the Chebyshev basis from its moments.  With
// X = theta (M^{-1} A - sigma I), p_i = T_i(X) p_0 (Sec. 2, Definition) and M X
// symmetric, the product rule of Chebyshev polynomials, T_i T_j =
// (T_{i+j} + T_{|i-j|}) / 2, gives
//     H_ij = <p_i, M p_j> = (mu_{i+j} + mu_{|i-j|}) / 2,  mu_k = <p_0, M T_k(X) p_0>,
// and taking (i, j) = (i, i) and (i, i-1):
//     mu_0 = d_0, mu_1 = e_1, mu_2i = 2 d_i - mu_0, mu_{2i-1} = 2 e_i - mu_1,
// so the 2s + 1 products d_i, e_i fix all of H (p_0 .. p_s), and the
// right-hand side c'_i = <p_i, M p_0> = mu_i.  The block forms h in the
// recurrence kind's layout and continues as k_fgs_rec.
template <int s>
__global__ __launch_bounds__(kFgsThreads) void k_fgs_mom(DevState *__restrict__ st, const double *__restrict__ sums,
                                                         int nu, double cscale, int fp32, double inv_sqrt_n,
                                                         double *__restrict__ dbg, double *__restrict__ hist,
                                                         int hist_cap, double theta, double sigma, double hscale)
{
    if (st->done)
        return;
    constexpr int S1 = s + 1;
    constexpr int E1 = S1 * (S1 + 1) / 2 + S1;
    __shared__ double mu[2 * s + 1];
    __shared__ double h[E1];
    for (int k = threadIdx.x; k <= 2 * s; k += kFgsThreads) {
        double m;
        if (k <= 1)
            m = sums[k];
        else if (k % 2 == 0)
            m = 2.0 * sums[k] - sums[0];
        else
            m = 2.0 * sums[k] - sums[1];
        mu[k] = m;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < S1 * (S1 + 1) / 2; e += kFgsThreads) {
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= e)
            ++i;
        const int j = e - i * (i + 1) / 2;
        h[e] = 0.5 * (mu[i + j] + mu[i - j]);
    }
    for (int i = threadIdx.x; i < S1; i += kFgsThreads)
        h[S1 * (S1 + 1) / 2 + i] = mu[i];
    __syncthreads();
    fgs_rec_from_h<s>(st, h, nu, cscale, fp32, inv_sqrt_n, dbg, hist, hist_cap, theta, sigma, hscale, 0);
}

template <int s>
hipError_t fgs_rec_launch_s(const IterArgs &a, hipStream_t st)
{
    constexpr int S1 = s + 1;
    constexpr int E1 = S1 * (S1 + 1) / 2 + S1;
    hipLaunchKernelGGL(k_partial_sums<S1>, dim3(E1), dim3(kSumThreads), 0, st, a.st, a.gpart, a.nbg, a.gsum);
    hipLaunchKernelGGL(k_fgs_rec<s>, dim3(1), dim3(kFgsThreads), 0, st, a.st, a.gsum, a.nu, a.cscale, a.fp32,
                       a.inv_sqrt_n, a.dbg, a.hist, a.hist_cap, a.theta, a.sigma, a.rec_hscale, a.monomial);
    return hipGetLastError();
}

template <int s>
hipError_t fgs_mom_launch_s(const IterArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_fgs_mom<s>, dim3(1), dim3(kFgsThreads), 0, st, a.st, a.gsum, a.nu, a.cscale, a.fp32,
                       a.inv_sqrt_n, a.dbg, a.hist, a.hist_cap, a.theta, a.sigma, a.rec_hscale);
    return hipGetLastError();
}

template <int s>
hipError_t fgs_launch_s(const IterArgs &a, hipStream_t st)
{
    constexpr int E = s * (s + 1) / 2 + s;
    hipLaunchKernelGGL(k_partial_sums<s>, dim3(E), dim3(kSumThreads), 0, st, a.st, a.gpart, a.nbg, a.gsum);
    hipLaunchKernelGGL(k_fgs<s>, dim3(1), dim3(kFgsThreads), 0, st, a.st, a.gsum, a.nu, a.cscale, a.fp32,
                       a.inv_sqrt_n, a.dbg, a.hist, a.hist_cap);
    return hipGetLastError();
}

}  // namespace sstep
