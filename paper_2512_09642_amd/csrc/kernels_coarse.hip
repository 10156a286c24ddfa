// Coarse-grid solve of a two-level hierarchy (Sec. 6, Proposition "AMG
// Convergence" and the streaming remark after it; Sec. 8, "AMG and
// performance"): A_c = P^T A_f P with the trilinear prolongation P from an
// ncx x ncy x ncz coarse grid to the (2nc+1)-point fine grid, and nu forward
// Gauss-Seidel sweeps on A_c u = f from u = 0, unknowns in natural order.
//
// Two ways, both exactly the natural-order sweep:
//  * streamed (A_c never formed): the fine vector v = P u is kept, and the
//    update of coarse unknown j is
//        u_j += (f_j - p_j^T A_f v) / a_jj,   v += (that step) p_j,
//    with p_j^T A_f v formed on the fly from the 27 fine points of p_j's
//    support (A_f applied there from the face coefficients); only the
//    diagonal a_jj (n_c values) is stored;
//  * formed: the 27 entries of each row of A_c are computed once on the
//    device (27 n_c values), then u_j = (f_j - sum_{i != j} a_ji u_i) / a_jj.
// Parallel schedule: unknown (I, J, K) belongs to wavefront t = I + 2J + 4K.
// Two unknowns of one wavefront are never A_c-neighbours (their offsets would
// need dI + 2dJ + 4dK = 0 with |d| <= 1), and every neighbour with a lower
// index has a lower t, so processing the wavefronts in order, the unknowns of
// one wavefront in parallel, sees exactly the values of the sequential sweep.
// One workgroup runs the sweeps (one wave per unknown, a barrier between
// wavefronts); the whole solve is latency-bound (ν (ncx + 2ncy + 4ncz)
// dependent steps), the data (v, u, f, coefficients) are L2-resident.
#include <algorithm>

#include "launch.h"

namespace sstep {
namespace {

constexpr int kCoarseThreads = 1024;
constexpr int kCoarseWaves = kCoarseThreads / kWave;

// 1D hat of the trilinear basis: 1 at fine distance 0, 1/2 at 1, else 0.
__device__ __forceinline__ double hat(int d) { return d == 0 ? 1.0 : (d == 1 || d == -1 ? 0.5 : 0.0); }

// (A_f v)(x, y, z) = sum over the six faces of k_f (v_m - v_q), v_q = 0
// outside the fine grid; kx == null means every k_f = 1.
struct FineOp {
    int nx, ny, nz;
    int64_t nxy;
    const double *kx, *ky, *kz;

    __device__ __forceinline__ double face(const double *k, int64_t idx) const { return kx ? k[idx] : 1.0; }

    template <class V>
    __device__ __forceinline__ double apply(const V &v, int x, int y, int z) const
    {
        const int64_t c = x + nx * (static_cast<int64_t>(y) + static_cast<int64_t>(ny) * z);
        const int64_t fx = (static_cast<int64_t>(z) * ny + y) * (nx + 1) + x;
        const int64_t fy = (static_cast<int64_t>(z) * (ny + 1) + y) * nx + x;
        const int64_t fz = (static_cast<int64_t>(z) * ny + y) * nx + x;
        const double vm = v(c, x, y, z);
        const double vw = x > 0 ? v(c - 1, x - 1, y, z) : 0.0;
        const double ve = x + 1 < nx ? v(c + 1, x + 1, y, z) : 0.0;
        const double vs = y > 0 ? v(c - nx, x, y - 1, z) : 0.0;
        const double vn = y + 1 < ny ? v(c + nx, x, y + 1, z) : 0.0;
        const double vb = z > 0 ? v(c - nxy, x, y, z - 1) : 0.0;
        const double vt = z + 1 < nz ? v(c + nxy, x, y, z + 1) : 0.0;
        return face(kx, fx) * (vm - vw) + face(kx, fx + 1) * (vm - ve) + face(ky, fy) * (vm - vs) +
               face(ky, fy + nx) * (vm - vn) + face(kz, fz) * (vm - vb) + face(kz, fz + nxy) * (vm - vt);
    }
};

// The trilinear basis function of coarse unknown (I, J, K), centred on fine
// point (2I+1, 2J+1, 2K+1), as a fine-grid vector.
struct Hat {
    int cx, cy, cz;
    __device__ __forceinline__ double operator()(int64_t, int x, int y, int z) const
    {
        return hat(x - cx) * hat(y - cy) * hat(z - cz);
    }
};

// A fine vector in memory.
struct Mem {
    const double *v;
    __device__ __forceinline__ double operator()(int64_t c, int, int, int) const { return v[c]; }
};

__device__ __forceinline__ void coarse_ijk(int j, int ncx, int ncy, int &I, int &J, int &K)
{
    I = j % ncx;
    const int q = j / ncx;
    J = q % ncy;
    K = q / ncy;
}

// a_jj = p_j^T A_f p_j over the 27 fine points of p_j's support.
__global__ __launch_bounds__(kBlock) void k_coarse_diag(FineOp op, int ncx, int ncy, int ncz, double *__restrict__ diag)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= ncx * ncy * ncz)
        return;
    int I, J, K;
    coarse_ijk(j, ncx, ncy, I, J, K);
    const Hat p{2 * I + 1, 2 * J + 1, 2 * K + 1};
    double acc = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = p.cx + dx, y = p.cy + dy, z = p.cz + dz;
                acc += p(0, x, y, z) * op.apply(p, x, y, z);
            }
    diag[j] = acc;
}

// Row j of A_c: rows[27 j + o] = p_j^T A_f p_i for the neighbour i at offset
// o = (dI + 1) + 3 (dJ + 1) + 9 (dK + 1), 0 where i is outside the coarse grid.
__global__ __launch_bounds__(kBlock) void k_coarse_rows(FineOp op, int ncx, int ncy, int ncz, double *__restrict__ rows)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int nc = ncx * ncy * ncz;
    if (t >= static_cast<int64_t>(nc) * 27)
        return;
    const int j = static_cast<int>(t / 27), o = static_cast<int>(t % 27);
    int I, J, K;
    coarse_ijk(j, ncx, ncy, I, J, K);
    const int I2 = I + o % 3 - 1, J2 = J + (o / 3) % 3 - 1, K2 = K + o / 9 - 1;
    double acc = 0.0;
    if (I2 >= 0 && I2 < ncx && J2 >= 0 && J2 < ncy && K2 >= 0 && K2 < ncz) {
        const Hat pj{2 * I + 1, 2 * J + 1, 2 * K + 1};
        const Hat pi{2 * I2 + 1, 2 * J2 + 1, 2 * K2 + 1};
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int x = pj.cx + dx, y = pj.cy + dy, z = pj.cz + dz;
                    acc += pj(0, x, y, z) * op.apply(pi, x, y, z);
                }
    }
    rows[t] = acc;
}

__global__ __launch_bounds__(kBlock) void k_coarse_zero(double *__restrict__ a, int64_t n)
{
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < n;
         q += static_cast<int64_t>(gridDim.x) * kBlock)
        a[q] = 0.0;
}

// The sweeps, streamed: lane l < 27 of the wave that updates unknown j owns
// fine point (2I + l%3, 2J + (l/3)%3, 2K + l/9) of p_j's support.
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_fgs_streamed(
    FineOp op, int ncx, int ncy, const double *__restrict__ diag, const double *__restrict__ f,
    double *__restrict__ u, double *__restrict__ v, const int32_t *__restrict__ order,
    const int32_t *__restrict__ wf, int nwf, int nu)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const Mem vm{v};
    for (int sweep = 0; sweep < nu; ++sweep)
        for (int t = 0; t < nwf; ++t) {
            for (int q = wf[t] + wave; q < wf[t + 1]; q += kCoarseWaves) {
                const int j = order[q];
                int I, J, K;
                coarse_ijk(j, ncx, ncy, I, J, K);
                double w = 0.0, contrib = 0.0;
                int64_t c = 0;
                if (lane < 27) {
                    const int dx = lane % 3, dy = (lane / 3) % 3, dz = lane / 9;
                    const int x = 2 * I + dx, y = 2 * J + dy, z = 2 * K + dz;
                    w = hat(dx - 1) * hat(dy - 1) * hat(dz - 1);
                    c = x + op.nx * (static_cast<int64_t>(y) + static_cast<int64_t>(op.ny) * z);
                    contrib = w * op.apply(vm, x, y, z);
                }
                const double ajv = wave_sum(contrib);  // (A_c u)_j = p_j^T A_f v
                const double step = (f[j] - ajv) / diag[j];
                if (lane == 0)
                    u[j] += step;
                if (lane < 27)
                    v[c] += step * w;
            }
            __syncthreads();
        }
}

// The sweeps with A_c formed: lane o < 27 holds entry o of row j.
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_fgs_formed(
    int ncx, int ncy, int ncz, const double *__restrict__ rows, const double *__restrict__ f, double *__restrict__ u,
    const int32_t *__restrict__ order, const int32_t *__restrict__ wf, int nwf, int nu)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int sweep = 0; sweep < nu; ++sweep)
        for (int t = 0; t < nwf; ++t) {
            for (int q = wf[t] + wave; q < wf[t + 1]; q += kCoarseWaves) {
                const int j = order[q];
                int I, J, K;
                coarse_ijk(j, ncx, ncy, I, J, K);
                double contrib = 0.0;
                if (lane < 27 && lane != 13) {
                    const int I2 = I + lane % 3 - 1, J2 = J + (lane / 3) % 3 - 1, K2 = K + lane / 9 - 1;
                    if (I2 >= 0 && I2 < ncx && J2 >= 0 && J2 < ncy && K2 >= 0 && K2 < ncz)
                        contrib = rows[static_cast<int64_t>(j) * 27 + lane] * u[I2 + ncx * (J2 + ncy * K2)];
                }
                const double off = wave_sum(contrib);
                if (lane == 0)
                    u[j] = (f[j] - off) / rows[static_cast<int64_t>(j) * 27 + 13];
            }
            __syncthreads();
        }
}

FineOp fine_op(const CoarseArgs &c)
{
    return FineOp{c.nfx, c.nfy, c.nfz, static_cast<int64_t>(c.nfx) * c.nfy, c.kx, c.ky, c.kz};
}

}  // namespace

hipError_t launch_coarse_prepare(const CoarseArgs &c, hipStream_t st)
{
    const int nc = c.ncx * c.ncy * c.ncz;
    hipLaunchKernelGGL(k_coarse_diag, dim3((nc + kBlock - 1) / kBlock), dim3(kBlock), 0, st, fine_op(c), c.ncx,
                       c.ncy, c.ncz, c.diag);
    if (c.rows) {
        const int64_t total = static_cast<int64_t>(nc) * 27;
        hipLaunchKernelGGL(k_coarse_rows, dim3(static_cast<uint32_t>((total + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, st, fine_op(c), c.ncx, c.ncy, c.ncz, c.rows);
    }
    return hipGetLastError();
}

hipError_t launch_coarse_fgs(const CoarseArgs &c, const double *f, double *u, int nu, hipStream_t st)
{
    const int64_t nc = static_cast<int64_t>(c.ncx) * c.ncy * c.ncz;
    hipLaunchKernelGGL(k_coarse_zero, dim3(static_cast<uint32_t>(std::min<int64_t>((nc + kBlock - 1) / kBlock, 1024))),
                       dim3(kBlock), 0, st, u, nc);
    if (c.rows) {
        hipLaunchKernelGGL(k_coarse_fgs_formed, dim3(1), dim3(kCoarseThreads), 0, st, c.ncx, c.ncy, c.ncz, c.rows, f,
                           u, c.order, c.wf, c.nwf, nu);
    } else {
        const int64_t nf = static_cast<int64_t>(c.nfx) * c.nfy * c.nfz;
        hipLaunchKernelGGL(k_coarse_zero, dim3(static_cast<uint32_t>(std::min<int64_t>((nf + kBlock - 1) / kBlock, 1024))),
                           dim3(kBlock), 0, st, c.v, nf);
        hipLaunchKernelGGL(k_coarse_fgs_streamed, dim3(1), dim3(kCoarseThreads), 0, st, fine_op(c), c.ncx, c.ncy,
                           c.diag, f, u, c.v, c.order, c.wf, c.nwf, nu);
    }
    return hipGetLastError();
}

}  // namespace sstep
