// Batched outer iteration over many stencil systems and right-hand sides:
// residual + basis start, basis step, update and the FP32 scaling pre-pass.
// Each kernel is persistent: a fixed grid walks a table of tiles, and the work
// of pairs whose solve has stopped is skipped.  The Gram and FGS kernels of
// the batched iteration live with the single-system ones (batched_impl.h).
#include "launch.h"

namespace sstep {
namespace {

// Stencil at one point of one system, its face coefficients loaded once and
// reused for every right-hand side.
template <typename T, bool FACES>
struct PointStencil {
    int64_t c, nx, nxy;
    bool hw, he, hs, hn, hb, ht;
    T fw, fe, fs, fn, fb, ft, dinv;

    __device__ __forceinline__ void init(const BSys &S, int64_t cc, int precond, const T *kx, const T *ky,
                                         const T *kz)
    {
        c = cc;
        nx = S.g.nx;
        nxy = S.g.nxy;
        const uint32_t q = fdiv(static_cast<uint32_t>(c), S.g.dx);
        const uint32_t i = static_cast<uint32_t>(c) - q * S.g.nx;
        const uint32_t k = fdiv(q, S.g.dy);
        const uint32_t j = q - k * S.g.ny;
        hw = i > 0, he = i + 1 < static_cast<uint32_t>(S.g.nx);
        hs = j > 0, hn = j + 1 < static_cast<uint32_t>(S.g.ny);
        hb = k > 0, ht = k + 1 < static_cast<uint32_t>(S.g.nz);
        if constexpr (FACES) {
            const int64_t fx = c + q, fy = c + static_cast<int64_t>(k) * S.g.nx;
            fw = kx[fx], fe = kx[fx + 1], fs = ky[fy], fn = ky[fy + S.g.nx], fb = kz[c], ft = kz[c + S.g.nxy];
            dinv = precond ? T(1) / (((((fw + fe) + fs) + fn) + fb) + ft) : T(1);
        } else {
            dinv = precond ? T(1) / T(6) : T(1);
        }
    }

    __device__ __forceinline__ T apply(const T *__restrict__ p, T &pc) const
    {
        pc = p[c];
        const T w = hw ? p[c - 1] : T(0), e = he ? p[c + 1] : T(0);
        const T s = hs ? p[c - nx] : T(0), n = hn ? p[c + nx] : T(0);
        const T b = hb ? p[c - nxy] : T(0), t = ht ? p[c + nxy] : T(0);
        if constexpr (FACES)
            return fw * (pc - w) + fe * (pc - e) + fs * (pc - s) + fn * (pc - n) + fb * (pc - b) + ft * (pc - t);
        else
            return T(6) * pc - (((((w + e) + s) + n) + b) + t);
    }
};

template <typename T>
__device__ __forceinline__ T block_sum(T v)
{
    __shared__ T part[kBlock / kWave];
    v = wave_sum(v);
    if (threadIdx.x % kWave == 0)
        part[threadIdx.x / kWave] = v;
    __syncthreads();
    T acc = part[0];
#pragma unroll
    for (int q = 1; q < kBlock / kWave; ++q)
        acc += part[q];
    __syncthreads();
    return acc;
}

// r = b - A x (FP64) per pair over a chunk, ||r||^2 partial per (pair, chunk),
// p_0 = p0scale * (M^{-1} r or r) as column 0 of the pair's basis.  The
// right-hand sides go in groups of kRhsGroup: a point's coefficients are
// loaded once for the group, and each pair's partial is summed in the same
// order as one pair at a time would.
constexpr int kRhsGroup = 8;
template <typename TP, bool FACES>
__global__ __launch_bounds__(kBlock) void k_bresidual(const BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                      const BTile *__restrict__ tiles, int ntiles,
                                                      const DevState *__restrict__ pairs, int nrhs, int precond,
                                                      int p0_mode, int write_p0, TP *__restrict__ P,
                                                      double *__restrict__ rpart)
{
    if (gl->ndone == gl->npairs)
        return;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BSys &S = sys[tl.q];
        const int64_t beg = static_cast<int64_t>(tl.chunk) * S.gchunk;
        const int64_t end = beg + S.gchunk < S.n ? beg + S.gchunk : S.n;
        for (int r0 = 0; r0 < nrhs; r0 += kRhsGroup) {
            bool act[kRhsGroup];
            bool any = false;
#pragma unroll
            for (int u = 0; u < kRhsGroup; ++u) {
                act[u] = r0 + u < nrhs && !pairs[S.pair0 + r0 + u].done;
                any = any || act[u];
            }
            if (!any)
                continue;  // the same for the whole block
            double acc[kRhsGroup];
#pragma unroll
            for (int u = 0; u < kRhsGroup; ++u)
                acc[u] = 0.0;
            for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
                PointStencil<double, FACES> op;
                op.init(S, c, precond, S.kx, S.ky, S.kz);
#pragma unroll
                for (int u = 0; u < kRhsGroup; ++u) {
                    if (!act[u])
                        continue;
                    const DevState &ps = pairs[S.pair0 + r0 + u];
                    double pc;
                    const double rr = ps.b[c] - op.apply(ps.x, pc);
                    acc[u] += rr * rr;
                    if (write_p0)
                        P[S.pofs + static_cast<int64_t>(r0 + u) * S.ld + c] =
                            static_cast<TP>(ps.p0scale * (p0_mode ? rr : op.dinv * rr));
                }
            }
#pragma unroll
            for (int u = 0; u < kRhsGroup; ++u) {
                if (!act[u])
                    continue;  // act is the same in every thread
                const double sum = block_sum(acc[u]);
                if (threadIdx.x == 0)
                    rpart[S.rofs + static_cast<int64_t>(r0 + u) * S.nch + tl.chunk] = sum;
            }
        }
    }
}

// FP32+IR pre-pass: p0scale of each pair from its residual partials.
__global__ __launch_bounds__(kBlock) void k_bp0scale(const BSys *__restrict__ sys, DevState *__restrict__ pairs,
                                                     int npairs, int nrhs, const double *__restrict__ rpart)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npairs || pairs[p].done)
        return;
    const BSys &S = sys[p / nrhs];
    const int r = p % nrhs;
    double acc = 0.0;
    for (int q = 0; q < S.nch; ++q)
        acc += rpart[S.rofs + static_cast<int64_t>(r) * S.nch + q];
    const double rms = sqrt(acc) * S.inv_sqrt_n;
    pairs[p].p0scale = (rms > 0.0 && isfinite(rms)) ? ldexp(1.0, -ilogb(rms)) : 1.0;
}

// Basis step j for every active pair (Sec. 2, Definition): y = A p_j -> AP
// (when AP is kept), p_{j+1} from the three-term recurrence.
template <typename T, bool FACES, int STEP>
__global__ __launch_bounds__(kBlock) void k_bbasis(const BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                   const PTile *__restrict__ tiles, int ntiles,
                                                   const DevState *__restrict__ pairs, int nrhs, int precond, int j,
                                                   T *__restrict__ P, T *__restrict__ AP)
{
    if (gl->ndone == gl->npairs)
        return;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const PTile tl = tiles[t];
        const BSys &S = sys[tl.q];
        const int64_t c = static_cast<int64_t>(tl.blk) * kBlock + threadIdx.x;
        if (c >= S.n)
            continue;
        const T *kx = nullptr, *ky = nullptr, *kz = nullptr;
        if constexpr (FACES) {
            if constexpr (sizeof(T) == 8)
                kx = reinterpret_cast<const T *>(S.kx), ky = reinterpret_cast<const T *>(S.ky),
                kz = reinterpret_cast<const T *>(S.kz);
            else
                kx = reinterpret_cast<const T *>(S.kx32), ky = reinterpret_cast<const T *>(S.ky32),
                kz = reinterpret_cast<const T *>(S.kz32);
        }
        PointStencil<T, FACES> op;
        op.init(S, c, precond, kx, ky, kz);
        const T theta = static_cast<T>(S.theta), sigma = static_cast<T>(S.sigma);
        const int64_t step = static_cast<int64_t>(nrhs) * S.ld;
        // Right-hand sides in groups of kRg: every load of a group is issued
        // before its stores (P is read and written through one pointer, so
        // the compiler keeps loads after earlier stores).
        constexpr int kRg = 4;
        for (int r0 = 0; r0 < nrhs; r0 += kRg) {
            T y[kRg], pc[kRg], pp[kRg];
            bool act[kRg];
#pragma unroll
            for (int u = 0; u < kRg; ++u) {
                const int r = r0 + u;
                act[u] = r < nrhs && !pairs[S.pair0 + r].done;
                y[u] = pc[u] = pp[u] = T(0);
                if (act[u]) {
                    const int64_t col = S.pofs + (static_cast<int64_t>(j) * nrhs + r) * S.ld;
                    y[u] = op.apply(P + col, pc[u]);
                    if constexpr (STEP == 1)
                        pp[u] = P[col - step + c];
                }
            }
#pragma unroll
            for (int u = 0; u < kRg; ++u) {
                if (!act[u])
                    continue;
                const int64_t col = S.pofs + (static_cast<int64_t>(j) * nrhs + r0 + u) * S.ld;
                if (AP)  // not kept by the recurrence Gram kind
                    __builtin_nontemporal_store(y[u], AP + col + c);
                if constexpr (STEP == 0) {
                    P[col + step + c] = theta * (op.dinv * y[u] - sigma * pc[u]);
                } else if constexpr (STEP == 1) {
                    const T two_theta = T(2) * theta;
                    P[col + step + c] = two_theta * (op.dinv * y[u] - sigma * pc[u]) - pp[u];
                }
            }
        }
    }
}

// x += P alpha for every pair whose solve continues.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bupdate(const BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                    const BTile *__restrict__ tiles, int ntiles,
                                                    const DevState *__restrict__ pairs, int nrhs, int s,
                                                    const T *__restrict__ P)
{
    if (gl->ndone == gl->npairs)
        return;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BTile tl = tiles[t];
        const BSys &S = sys[tl.q];
        const int64_t beg = static_cast<int64_t>(tl.chunk) * S.gchunk;
        const int64_t end = beg + S.gchunk < S.n ? beg + S.gchunk : S.n;
        for (int r = 0; r < nrhs; ++r) {
            const DevState &ps = pairs[S.pair0 + r];
            if (ps.done)
                continue;
            double *__restrict__ x = ps.x;
            const T *Pr = P + S.pofs + static_cast<int64_t>(r) * S.ld;
            const int64_t step = static_cast<int64_t>(nrhs) * S.ld;
            for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
                // P is read once: non-temporal loads, eight columns in flight
                // at a time, summed in column order
                double acc = 0.0;
                int i = 0;
                for (; i + 8 <= s; i += 8) {
                    T v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        v[u] = __builtin_nontemporal_load(Pr + (i + u) * step + c);
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        acc += static_cast<double>(v[u]) * ps.alpha[i + u];
                }
                for (; i < s; ++i)
                    acc += static_cast<double>(__builtin_nontemporal_load(Pr + i * step + c)) * ps.alpha[i];
                x[c] += acc;
            }
        }
    }
}

}  // namespace

hipError_t launch_bresidual(const BatchArgs &a, hipStream_t st, bool write_p0)
{
    const int w = write_p0 ? 1 : 0;
    if (a.fp32) {
        if (a.faces)
            hipLaunchKernelGGL((k_bresidual<float, true>), dim3(a.grid_bt), dim3(kBlock), 0, st, a.gl, a.sys,
                               a.btiles, a.nbt, a.pairs, a.nrhs, a.precond, a.p0_mode, w,
                               static_cast<float *>(a.P), a.rpart);
        else
            hipLaunchKernelGGL((k_bresidual<float, false>), dim3(a.grid_bt), dim3(kBlock), 0, st, a.gl, a.sys,
                               a.btiles, a.nbt, a.pairs, a.nrhs, a.precond, a.p0_mode, w,
                               static_cast<float *>(a.P), a.rpart);
    } else {
        if (a.faces)
            hipLaunchKernelGGL((k_bresidual<double, true>), dim3(a.grid_bt), dim3(kBlock), 0, st, a.gl, a.sys,
                               a.btiles, a.nbt, a.pairs, a.nrhs, a.precond, a.p0_mode, w,
                               static_cast<double *>(a.P), a.rpart);
        else
            hipLaunchKernelGGL((k_bresidual<double, false>), dim3(a.grid_bt), dim3(kBlock), 0, st, a.gl, a.sys,
                               a.btiles, a.nbt, a.pairs, a.nrhs, a.precond, a.p0_mode, w,
                               static_cast<double *>(a.P), a.rpart);
    }
    return hipGetLastError();
}

hipError_t launch_bp0scale(const BatchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_bp0scale, dim3((a.npairs + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a.sys, a.pairs,
                       a.npairs, a.nrhs, a.rpart);
    return hipGetLastError();
}

namespace {
template <typename T, bool FACES>
hipError_t bbasis_t(const BatchArgs &a, int j, hipStream_t st)
{
    T *P = static_cast<T *>(a.P), *AP = static_cast<T *>(a.AP);
    if (j + 1 >= a.s && !a.rec)  // the last step forms A p_{s-1} only, unless p_s is kept
        hipLaunchKernelGGL((k_bbasis<T, FACES, 2>), dim3(a.grid_pt), dim3(kBlock), 0, st, a.gl, a.sys, a.ptiles,
                           a.npt, a.pairs, a.nrhs, a.precond, j, P, AP);
    else if (j == 0)
        hipLaunchKernelGGL((k_bbasis<T, FACES, 0>), dim3(a.grid_pt), dim3(kBlock), 0, st, a.gl, a.sys, a.ptiles,
                           a.npt, a.pairs, a.nrhs, a.precond, j, P, AP);
    else
        hipLaunchKernelGGL((k_bbasis<T, FACES, 1>), dim3(a.grid_pt), dim3(kBlock), 0, st, a.gl, a.sys, a.ptiles,
                           a.npt, a.pairs, a.nrhs, a.precond, j, P, AP);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_bbasis(const BatchArgs &a, int j, hipStream_t st)
{
    if (a.fp32)
        return a.faces ? bbasis_t<float, true>(a, j, st) : bbasis_t<float, false>(a, j, st);
    return a.faces ? bbasis_t<double, true>(a, j, st) : bbasis_t<double, false>(a, j, st);
}

hipError_t launch_bupdate(const BatchArgs &a, hipStream_t st)
{
    if (a.fp32)
        hipLaunchKernelGGL(k_bupdate<float>, dim3(a.grid_bt), dim3(kBlock), 0, st, a.gl, a.sys, a.btiles, a.nbt,
                           a.pairs, a.nrhs, a.s, static_cast<const float *>(a.P));
    else
        hipLaunchKernelGGL(k_bupdate<double>, dim3(a.grid_bt), dim3(kBlock), 0, st, a.gl, a.sys, a.btiles, a.nbt,
                           a.pairs, a.nrhs, a.s, static_cast<const double *>(a.P));
    return hipGetLastError();
}

}  // namespace sstep
