// Shared device-side definitions of the s-step CG library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sstep {

constexpr int kMaxS = 32;             // largest basis width
constexpr int kMaxE = kMaxS * (kMaxS + 1) / 2 + kMaxS;  // Gram lower triangle + right-hand side
constexpr int kBlock = 256;           // threads per block of the streaming kernels
constexpr int kWave = 64;
constexpr unsigned kNumXcd = 8;       // MI355X: 8 XCDs, each with its own L2

// State of one solve, resident in device memory.  Every kernel of the outer
// iteration reads `done` first and returns at once when it is set, so graph
// replays issued after convergence do no work.
struct DevState {
    const double *b;   // right-hand side of the current solve
    double *x;         // iterate, updated in place
    double tol;        // relative residual tolerance
    double rho0;       // ||b - A x_0||
    double rho;        // ||b - A x_k|| of the last residual
    double relres;     // rho / rho0
    double p0scale;    // power-of-two factor applied to p_0 (FP32+IR); 1 in FP64
    double delta;      // ||ctil - G atil|| / ||ctil|| of the last Gram solve
    double lnorm;      // ||L||_F, L the strictly lower part of the last scaled Gram matrix
    int32_t done;      // 1 once the solve has stopped
    int32_t status;    // sstep_status value
    int32_t iter;      // completed outer updates
    int32_t max_outer;
    int32_t first;     // 1 until rho0 has been recorded
    int32_t no_stop;   // 1 = never stop (single-step and timing entry points)
    int32_t hist_cap;  // capacity of the device history (0 = off)
    int32_t pad;
    double alpha[kMaxS];  // coefficients of the unscaled basis, x += P alpha
};

// Division of 32-bit unsigned n < 2^31 by an invariant divisor d >= 1 with a
// multiply-high and a shift (Granlund & Montgomery, PLDI 1994, round-up
// variant): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// n / d = (n + mulhi(m, n)) >> l.
struct FastDiv {
    uint32_t d, m, l;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d)
        ++l;
    const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return FastDiv{d, static_cast<uint32_t>(m), l};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    const uint32_t t = __umulhi(f.m, n);
    return static_cast<uint32_t>((static_cast<uint64_t>(t) + n) >> f.l);
}

// Grid of a 3D stencil operator, x fastest.
struct Grid3 {
    int32_t nx, ny, nz;
    int64_t nxy;
    FastDiv dx, dy;
};

// Logical block index that gives each XCD a contiguous range of blocks:
// hardware block b runs on XCD b % 8, so XCD x processes logical blocks
// [x * per, (x + 1) * per) in ascending order and the stencil neighbours of a
// block (one plane away) are mostly resident in that XCD's own L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t per)
{
    return (b % kNumXcd) * per + b / kNumXcd;
}

// Butterfly sum over the 64 lanes of a wave; every lane gets the total and the
// order of the additions is fixed, so the result is reproducible.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
}

// Block sums of NV per-thread values in a fixed order (each wave by
// butterfly, then the waves in order); value u goes to out[u * stride].
// Every thread of the block must call it.
template <int NV, int NT>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double *__restrict__ out, int64_t stride)
{
    constexpr int NW = NT / kWave;
    __shared__ double part[NW][NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const double t = wave_sum(v[u]);
        if (threadIdx.x % kWave == 0)
            part[threadIdx.x / kWave][u] = t;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double acc = 0.0;
        for (int w = 0; w < NW; ++w)
            acc += part[w][threadIdx.x];
        out[threadIdx.x * stride] = acc;
    }
}

// ---------------------------------------------------------------------------
// Operators.  apply() returns the centre value p_c, y = (A p)_c and the
// Jacobi factor M^{-1}_cc (1 without preconditioning); apply_w() also the
// weight of the M inner product at c: the diagonal a_cc with Jacobi, 1
// without, and 1 for the constant-coefficient stencils, whose constant
// diagonal the caller applies afterwards.
// ---------------------------------------------------------------------------

// Constant-coefficient 7-point Poisson operator: diagonal 6, off-diagonal -1.
template <typename T>
struct OpPoisson7 {
    Grid3 g;
    T minv;  // 1/6 with Jacobi, 1 without

    __device__ __forceinline__ void apply_w(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv, T &wt) const
    {
        apply(p, c, pc, y, dinv);
        wt = T(1);
    }
    __device__ __forceinline__ void apply(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv) const
    {
        const uint32_t q = fdiv(static_cast<uint32_t>(c), g.dx);  // j + ny*k
        const uint32_t i = static_cast<uint32_t>(c) - q * g.nx;
        const uint32_t k = fdiv(q, g.dy);
        const uint32_t j = q - k * g.ny;
        pc = p[c];
        const T w = i > 0 ? p[c - 1] : T(0);
        const T e = i + 1 < static_cast<uint32_t>(g.nx) ? p[c + 1] : T(0);
        const T s = j > 0 ? p[c - g.nx] : T(0);
        const T n = j + 1 < static_cast<uint32_t>(g.ny) ? p[c + g.nx] : T(0);
        const T b = k > 0 ? p[c - g.nxy] : T(0);
        const T t = k + 1 < static_cast<uint32_t>(g.nz) ? p[c + g.nxy] : T(0);
        y = T(6) * pc - (((((w + e) + s) + n) + b) + t);
        dinv = minv;
    }
};

// Constant-coefficient 27-point operator (Sec. 8): diagonal 26, -1 on the 26
// other points of the 3 x 3 x 3 box, so (A p)_c = 27 p_c - (sum of p over the
// box); neighbours outside the grid are 0.
template <typename T>
struct OpPoisson27 {
    Grid3 g;
    T minv;  // 1/26 with Jacobi, 1 without

    __device__ __forceinline__ void apply_w(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv, T &wt) const
    {
        apply(p, c, pc, y, dinv);
        wt = T(1);
    }
    __device__ __forceinline__ void apply(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv) const
    {
        const uint32_t q = fdiv(static_cast<uint32_t>(c), g.dx);
        const uint32_t i = static_cast<uint32_t>(c) - q * g.nx;
        const uint32_t k = fdiv(q, g.dy);
        const uint32_t j = q - k * g.ny;
        const bool has_w = i > 0, has_e = i + 1 < static_cast<uint32_t>(g.nx);
        const bool has_s = j > 0, has_n = j + 1 < static_cast<uint32_t>(g.ny);
        const bool has_b = k > 0, has_t = k + 1 < static_cast<uint32_t>(g.nz);
        pc = p[c];
        T box = T(0);
#pragma unroll
        for (int dk = -1; dk <= 1; ++dk) {
            if ((dk < 0 && !has_b) || (dk > 0 && !has_t))
                continue;
            T plane = T(0);
#pragma unroll
            for (int dj = -1; dj <= 1; ++dj) {
                if ((dj < 0 && !has_s) || (dj > 0 && !has_n))
                    continue;
                const int64_t r = c + dj * static_cast<int64_t>(g.nx) + dk * g.nxy;
                T row = p[r];
                if (has_w)
                    row += p[r - 1];
                if (has_e)
                    row += p[r + 1];
                plane += row;
            }
            box += plane;
        }
        y = T(27) * pc - box;
        dinv = minv;
    }
};

// Variable-coefficient 7-point operator from face coefficients (boundary
// faces included): (A p)_c = sum_f k_f (p_c - p_q), p_q = 0 outside.
template <typename T>
struct OpFaces7 {
    Grid3 g;
    const T *__restrict__ kx;
    const T *__restrict__ ky;
    const T *__restrict__ kz;
    int precond;

    __device__ __forceinline__ void apply(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv) const
    {
        T wt;
        apply_w(p, c, pc, y, dinv, wt);
    }
    __device__ __forceinline__ void apply_w(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv, T &wt) const
    {
        const uint32_t q = fdiv(static_cast<uint32_t>(c), g.dx);
        const uint32_t i = static_cast<uint32_t>(c) - q * g.nx;
        const uint32_t k = fdiv(q, g.dy);
        const uint32_t j = q - k * g.ny;
        const int64_t fx = c + q;                          // (k*ny + j)*(nx+1) + i
        const int64_t fy = c + static_cast<int64_t>(k) * g.nx;  // (k*(ny+1) + j)*nx + i
        const T fw = kx[fx], fe = kx[fx + 1];
        const T fs = ky[fy], fn = ky[fy + g.nx];
        const T fb = kz[c], ft = kz[c + g.nxy];
        pc = p[c];
        const T w = i > 0 ? p[c - 1] : T(0);
        const T e = i + 1 < static_cast<uint32_t>(g.nx) ? p[c + 1] : T(0);
        const T s = j > 0 ? p[c - g.nx] : T(0);
        const T n = j + 1 < static_cast<uint32_t>(g.ny) ? p[c + g.nx] : T(0);
        const T b = k > 0 ? p[c - g.nxy] : T(0);
        const T t = k + 1 < static_cast<uint32_t>(g.nz) ? p[c + g.nxy] : T(0);
        y = fw * (pc - w) + fe * (pc - e) + fs * (pc - s) + fn * (pc - n) + fb * (pc - b) + ft * (pc - t);
        const T d = ((((fw + fe) + fs) + fn) + fb) + ft;
        dinv = precond ? T(1) / d : T(1);
        wt = precond ? d : T(1);
    }
};

// General CSR matrix, one row per thread.
template <typename T>
struct OpCsr {
    const int32_t *__restrict__ rp;
    const int32_t *__restrict__ ci;
    const T *__restrict__ val;
    const T *__restrict__ invd;  // M^{-1} diagonal (all ones without preconditioning)

    __device__ __forceinline__ void apply_w(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv, T &wt) const
    {
        apply(p, c, pc, y, dinv);
        wt = T(1) / dinv;
    }
    __device__ __forceinline__ void apply(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv) const
    {
        const int32_t k0 = rp[c], k1 = rp[c + 1];
        T acc = T(0);
        for (int32_t k = k0; k < k1; ++k)
            acc += val[k] * p[ci[k]];
        pc = p[c];
        y = acc;
        dinv = invd[c];
    }
};

// The same CSR operator stored as sliced ELL: rows in slices of kEllSlice
// consecutive rows; slice q holds w_q = (off[q+1] - off[q]) / kEllSlice
// entries per row (the longest row of the slice), column-major inside the
// slice, so entry k of row r = q kEllSlice + l sits at off[q] + k kEllSlice +
// l and the lanes of a wave that takes one slice read each entry index with
// one coalesced load.  A row keeps its CSR entries in their order; the
// padding has column -1 and is skipped, so the sum is formed with the same
// operations in the same order as by OpCsr.
constexpr int kEllSlice = 64;
//
// In FP64 the Jacobi weight is formed from the row's own diagonal entry,
// precond ? 1 / a_cc : 1 (the value the M^{-1} vector holds, to the bit),
// which saves reading that vector; FP32 reads its rounded copy.
template <typename T>
struct OpEll {
    const int32_t *__restrict__ col;
    const T *__restrict__ val;
    const int64_t *__restrict__ off;
    const T *__restrict__ invd;  // M^{-1} diagonal (all ones without preconditioning); FP32 only
    int precond;

    __device__ __forceinline__ void apply(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv) const
    {
        T wt;
        apply_w(p, c, pc, y, dinv, wt);
    }
    __device__ __forceinline__ void apply_w(const T *__restrict__ p, int64_t c, T &pc, T &y, T &dinv, T &wt) const
    {
        const int64_t q = c / kEllSlice;
        const int64_t o0 = off[q];
        const int w = static_cast<int>((off[q + 1] - o0) / kEllSlice);
        const int64_t b = o0 + (c - q * kEllSlice);
        T acc = T(0), diag = T(1);
        constexpr int U = 8;  // entries whose loads are issued together
        for (int k0 = 0; k0 < w; k0 += U) {
            int32_t j[U];
            T v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k0 + u < w) {  // read once per product: non-temporal
                    j[u] = __builtin_nontemporal_load(col + b + int64_t(k0 + u) * kEllSlice);
                    v[u] = __builtin_nontemporal_load(val + b + int64_t(k0 + u) * kEllSlice);
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k0 + u < w && j[u] >= 0) {
                    acc += v[u] * p[j[u]];
                    if (j[u] == c)
                        diag = v[u];
                }
        }
        pc = p[c];
        y = acc;
        if constexpr (sizeof(T) == 8)
            dinv = precond ? T(1) / diag : T(1);
        else
            dinv = invd[c];
        wt = precond ? diag : T(1);
    }
};

}  // namespace sstep
