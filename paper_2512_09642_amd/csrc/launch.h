// Host-side launch interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bands.h"
#include "common.h"

namespace sstep {

enum OpKind { kOpCsr = 0, kOpPoisson = 1, kOpFaces = 2, kOpPoisson27 = 3 };

// Column padding of the basis buffers and of the M-diagonal arrays (rows).
constexpr int64_t kPad = 256;
// Largest Gram partial-block count a schedule may use.
constexpr int kMaxGramBlocks = 2048;
// Widest basis served by the Gram kernel that applies a stencil operator itself.
constexpr int kGoMaxS = 16;
// Widest basis of the recurrence Gram kind (it needs the Gram of s + 1 columns).
constexpr int kRecMaxS = 31;
// Smallest row chunk of a batched tile; the tile tables and partial buffers
// are sized for it.
constexpr int64_t kMinBatchChunk = 2048;

// Device copy of the operator in both precisions (the FP32 arrays exist only
// in FP32+IR mode).
struct OpDev {
    int kind = kOpPoisson;
    int precond = 1;
    int64_t n = 0;
    int64_t nnz = 0;
    Grid3 g{};
    const int32_t *rp = nullptr;
    const int32_t *ci = nullptr;
    const double *val = nullptr;
    const float *val32 = nullptr;
    const double *kx = nullptr, *ky = nullptr, *kz = nullptr;
    const float *kx32 = nullptr, *ky32 = nullptr, *kz32 = nullptr;
    const double *invd = nullptr;  // CSR: M^{-1} diagonal
    const float *invd32 = nullptr;
    const double *dvec = nullptr;  // M diagonal (Jacobi, non-constant diagonal)
    const float *dvec32 = nullptr;
    // CSR also stored as sliced ELL (OpEll, common.h) when ell_col is set
    const int32_t *ell_col = nullptr;
    const double *ell_val = nullptr;
    const float *ell_val32 = nullptr;
    const int64_t *ell_off = nullptr;  // [nslice + 1]
    int64_t ell_nslice = 0;
};

// Everything one outer iteration needs; all pointers are device memory.
struct IterArgs {
    DevState *st = nullptr;
    OpDev op;
    int fp32 = 0;     // 1 = FP32 basis / SpMV / Gram
    int p0_mode = 0;  // 0: p_0 = M^{-1} r, 1: p_0 = r
    int monomial = 0; // 1: monomial basis p_{j+1} = M^{-1} A p_j instead of Chebyshev
    int one_step = 0; // 1: one basis step per launch even where two fit
    int s = 0, nu = 0;
    double theta = 0, sigma = 0;
    void *P = nullptr;   // n x s, column-major, leading dimension ld
    void *AP = nullptr;  // n x s
    int64_t ld = 0;      // multiple of kPad; rows n..ld-1 of every column stay zero
    double *rpart = nullptr;  // residual-norm partial sums [nbr]
    int nbr = 0;
    int64_t rchunk = 0;
    int res_p2 = 0;  // constant Poisson, nx even: residual in the basis kernel's shape (nbr = its blocks)
    double *gpart = nullptr;  // Gram partial sums [E][nbg]
    double *gsum = nullptr;   // totals: the E Gram entries, then ||r||^2 (E + 1 doubles)
    int nbg = 0;
    int64_t gchunk = 0;  // contiguous schedule: rows per block
    int64_t gslab = 0;   // strided schedule: rows per slab (0 = contiguous schedule)
    int wdvec = 0;        // Gram right-hand side uses M-diagonal * p_0 (else p_0)
    double cscale = 1.0;  // constant factor applied to c = P^T (W) in the FGS kernel
    double *dbg = nullptr;   // G (s*s), ctil (s), atil (s), d (s), rho: written by the FGS kernel
    double *hist = nullptr;  // [3 * hist_cap]: relres, delta, ||L||_F
    int hist_cap = 0;
    double inv_sqrt_n = 1.0;
    // Gram kernel that applies the stencil operator itself (AP not stored;
    // the basis steps skip the AP write and the last product):
    int gram_op = 0;
    int go_fx = 0, go_fy = 0;           // full 32 x 8 tiles per row / column of tiles
    int go_tiles_y = 0;                 // tile rows, full and edge
    int go_rx = 0, go_ry = 0;           // column / row strip of edge tiles present
    int go_zr = 0, go_nzb = 0;          // planes per z-range, z-ranges
    int go_tiles[2] = {0, 0};           // tiles of the full-tile and edge-tile launches
    int go_items[2] = {0, 0};           // work items (tile, z-range) of each launch
    int go_blocks[2] = {0, 0};          // blocks (= partial slots) of each launch
    // Recurrence kind (G_raw from the M-weighted Gram of p_0 .. p_s): the basis
    // makes s launches, the last writing p_s into column s of P:
    int gram_rec = 0;
    int rec_wap = 0;          // the Gram kernel weights by the M diagonal array
    double rec_hscale = 1.0;  // constant M diagonal applied by the FGS kernel otherwise
    // Moments kind (also gram_rec): no Gram kernel; the basis kernels write
    // block partials of <p_i, M p_i> (slot 2i) and <p_i, M p_{i-1}> (slot
    // 2i - 1), slot k at mpart + k * mstride with mcnt[k] of them
    int gram_mom = 0;
    double *mpart = nullptr;
    int32_t *mcnt = nullptr;
    int64_t mstride = 0;
};

// Debug block layout written by the FGS kernel.
__host__ __device__ inline int64_t dbg_G(int) { return 0; }
__host__ __device__ inline int64_t dbg_ctil(int s) { return int64_t(s) * s; }
__host__ __device__ inline int64_t dbg_atil(int s) { return int64_t(s) * s + s; }
__host__ __device__ inline int64_t dbg_d(int s) { return int64_t(s) * s + 2 * s; }
__host__ __device__ inline int64_t dbg_rho(int s) { return int64_t(s) * s + 3 * s; }
__host__ __device__ inline int64_t dbg_size(int s) { return int64_t(s) * s + 3 * s + 1; }

__host__ __device__ inline int gram_entries(int s) { return s * (s + 1) / 2 + s; }

// ---------------------------------------------------------------------------
// Batched solves: nsys stencil systems x nrhs right-hand sides ("pairs").
// System q's basis block is laid out [s][nrhs][ld_q] at element offset pofs:
// column j of pair (q, r) starts at pofs + (j*nrhs + r)*ld_q.
// ---------------------------------------------------------------------------
// Per-band partial slots of a batched pair in the moments kind: the 2s + 1
// basis products (slots 0 .. 2s) and ||r||^2 (slot 2s + 1).
__host__ __device__ inline int bmom_slots(int s) { return 2 * s + 2; }

struct BSys {
    Grid3 g;
    int64_t n, ld, pofs;
    const double *kx, *ky, *kz;      // face coefficients (null: constant Poisson)
    const float *kx32, *ky32, *kz32;
    const double *dvec;              // M diagonal, zero-padded to ld
    const float *dvec32;
    const double *dinv;              // Jacobi weights 1 / diag (1 without Jacobi), faces only
    const float *dinv32;             // the same from the FP32 faces (FP32+IR)
    double theta, sigma, inv_sqrt_n;
    int64_t gchunk;                  // rows per chunk tile (multiple of kPad)
    int64_t gofs;                    // Gram partials of pair (q, r): gofs + r*E*nch
    int64_t rofs;                    // residual partials of pair (q, r): rofs + r*nch
    int32_t pair0, nch;
    // two steps per launch: this system's bands are entries f2first ..
    // f2first + nf2q - 1 of the band table; slot k of pair (q, r) holds one
    // partial per band at mofs + (r slots + k) nf2q (slots: bres_slots)
    int64_t mofs;
    int32_t f2first, nf2q;
    // bands of this system in the band table of the whole batch: what a pair
    // of it adds to BGlob::bdone when it stops
    int32_t nbl, pad;
};
struct BTile {  // chunk of one system, all right-hand sides
    int32_t q, chunk;
};
struct PTile {  // kBlock points of one system (basis)
    int32_t q, blk;
};
struct GTile {  // chunk of one pair (Gram)
    int32_t q, chunk, r, pad;
};
// ndone: pairs that have stopped; bdone: the band-table blocks of the whole
// batch's two-step basis those pairs no longer start (the host reads both
// after each graph replay)
struct BGlob {
    int32_t ndone, npairs, bdone, pad;
};

struct BatchArgs {
    BGlob *gl = nullptr;
    const BSys *sys = nullptr;
    int nsys = 0, nrhs = 0, npairs = 0;
    int s = 0, nu = 0, fp32 = 0, p0_mode = 0, precond = 1, faces = 0;
    void *P = nullptr, *AP = nullptr;
    const BTile *btiles = nullptr;
    const PTile *ptiles = nullptr;
    const GTile *gtiles = nullptr;
    int nbt = 0, npt = 0, ngt = 0;
    int grid_bt = 0, grid_pt = 0, grid_gt = 0;  // persistent grid sizes
    DevState *pairs = nullptr;
    double *rpart = nullptr, *gpart = nullptr, *dbg = nullptr;
    double cscale = 1.0;
    int wdvec = 0;
    // recurrence Gram kind: P holds p_0..p_s per pair, no AP; the Gram kernel
    // forms H = P^T M P (rec_wap: M from the diagonal arrays, else
    // rec_hscale M = const), the FGS kernel maps H onto P^T A P
    int rec = 0, rec_wap = 0;
    double rec_hscale = 1.0;
    // two basis steps per launch (f2 = 1): nf2 bands x nrhs logical blocks
    // (band e, right-hand side r: e * nrhs + r); hardware block b of the
    // f2grid runs logical block f2map[b] (none if it is nf2 * nrhs or more)
    int f2 = 0, nf2 = 0;
    uint32_t f2grid = 0;
    const uint32_t *f2map = nullptr;
    const BF2Tile *f2tiles = nullptr;
    // moments Gram kind (also rec): the two-step basis writes the products
    // and k_bres_f2 ||r||^2, per band; k_bfgs_mom sums them; no Gram kernel
    int mom = 0;
    double *mpart = nullptr;
    // residual over the band table (k_bres_f2; every context with f2): its
    // ||r||^2 per band in slot bres_slot of bres_slots per right-hand side of
    // mpart (the moments kind: bmom_slots(s), 2s + 1; the recurrence kind: 1, 0)
    int bres = 0, bres_slots = 0, bres_slot = 0;
};

hipError_t launch_bresidual(const BatchArgs &a, hipStream_t st, bool write_p0);
hipError_t launch_bp0scale(const BatchArgs &a, hipStream_t st);
hipError_t launch_bbasis(const BatchArgs &a, int j, hipStream_t st);
hipError_t launch_bres_f2(const BatchArgs &a, hipStream_t st);
hipError_t launch_bbasis_pair(const BatchArgs &a, int j, hipStream_t st);
hipError_t launch_bdinv(const BSys &S, int precond, int fp32, double *dinv, float *dinv32, hipStream_t st);
hipError_t launch_bgram(const BatchArgs &a, hipStream_t st);
hipError_t launch_bfgs(const BatchArgs &a, hipStream_t st);
hipError_t launch_bupdate(const BatchArgs &a, hipStream_t st);

// Lanczos spectrum estimate (kernels_lanczos.hip).
constexpr int kMaxLanczos = 64;  // largest number of Lanczos steps
struct LzState {
    double scale;  // ||u||_M, then the last beta_{j+1}
    double amax;   // max |alpha_i| so far
    int32_t m;     // completed steps
    int32_t stopped;
};
struct LzArgs {
    LzState *ls = nullptr;
    double *v[3] = {nullptr, nullptr, nullptr};  // z_{j-1}, z_j, y / w: n doubles each
    double *part = nullptr;                      // block partials [nb]
    double *ab = nullptr;                        // alpha [steps], beta [steps], Ritz values [steps]
    int64_t n = 0, chunk = 0;
    int nb = 0;
};
// Enqueues steps Lanczos steps from u (n doubles) and the Ritz values of T_m;
// results in l.ab and l.ls once the stream reaches them.
hipError_t launch_lanczos(const LzArgs &l, const OpDev &op, const double *u, int steps, hipStream_t st);

// Helpers of the allocation-free solve: zero bytes (a multiple of 8) at p;
// the initial solve state; two-phase device checks of a CSR pattern (row
// pointers first, then columns), setting *bad on a violation.
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_init_state(DevState *s, const double *b, double *x, double tol, int max_outer, hipStream_t st);
hipError_t launch_check_csr_rows(const int32_t *rp, int64_t n, int64_t nnz, int *bad, hipStream_t st);
hipError_t launch_check_csr_cols(const int32_t *rp, const int32_t *ci, int64_t n, int *bad, hipStream_t st);

// Two-level coarse solve (kernels_coarse.hip).
struct CoarseArgs {
    int ncx = 0, ncy = 0, ncz = 0;       // coarse grid
    int nfx = 0, nfy = 0, nfz = 0;       // fine grid, 2 nc + 1 per axis
    const double *kx = nullptr, *ky = nullptr, *kz = nullptr;  // fine face coefficients (null: all 1)
    double *diag = nullptr;               // a_jj [n_c]
    double *rows = nullptr;               // formed A_c rows [27 n_c], or null (streamed)
    double *v = nullptr;                  // streamed: the fine vector P u [n_f]
    const int32_t *order = nullptr;       // coarse unknowns by wavefront [n_c]
    const int32_t *wf = nullptr;          // wavefront starts [nwf + 1]
    int nwf = 0;
};
// a_jj and, when formed, the rows of A_c.
hipError_t launch_coarse_prepare(const CoarseArgs &c, hipStream_t st);
// u = nu forward Gauss-Seidel sweeps on A_c u = f from u = 0.
hipError_t launch_coarse_fgs(const CoarseArgs &c, const double *f, double *u, int nu, hipStream_t st);

hipError_t launch_residual(const IterArgs &a, hipStream_t st, bool write_p0);
hipError_t launch_p0scale(const IterArgs &a, hipStream_t st);
hipError_t launch_basis(const IterArgs &a, int j, hipStream_t st);
// Sliced ELL copy of a CSR operator: the columns (pattern) and the values in
// FP64 or FP32 (from the CSR arrays rp, ci, val of the same precision).
hipError_t launch_ell_fill_col(const OpDev &op, int32_t *col, hipStream_t st);
hipError_t launch_ell_fill_val(const OpDev &op, const double *val, double *ev, hipStream_t st);
hipError_t launch_ell_fill_val(const OpDev &op, const float *val, float *ev, hipStream_t st);
// The whole basis p_1 .. p_m of one outer iteration: two steps per launch
// for the constant 7-point operator without stored AP, else one per launch.
hipError_t launch_basis_all(const IterArgs &a, hipStream_t st);
// Moments kind: the basis launch that starts at column j writes its products
// from slot 0 (j = 0: <p_0,Mp_0>, <p_1,Mp_0>, <p_1,Mp_1>, ...) or from slot
// 2j + 1 (<p_{j+1},Mp_j>, <p_{j+1},Mp_{j+1}>, ...).  mom_layout gives the
// block count each of the 2s + 1 slots receives from the launches
// launch_basis_all makes, and the largest.
inline int mom_slot(int j) { return j == 0 ? 0 : 2 * j + 1; }
void mom_layout(const IterArgs &a, int32_t *cnt, int64_t *stride);
hipError_t launch_mom_sums(const IterArgs &a, hipStream_t st);
// Launches launch_basis_all makes, and (if pairs is not NULL) how many of
// them form two columns.
int basis_kernel_count(const IterArgs &a, int *pairs);
// AP[:, j] = A p_j alone (into a.AP, which must be set).
hipError_t launch_product(const IterArgs &a, int j, hipStream_t st);
hipError_t launch_gram(const IterArgs &a, hipStream_t st);
hipError_t launch_fgs(const IterArgs &a, hipStream_t st);
hipError_t launch_update(const IterArgs &a, hipStream_t st);
hipError_t launch_apply(const OpDev &op, const double *x, double *y, hipStream_t st);
hipError_t launch_grad(const OpDev &op, const double *lam, const double *x, double *dA, int accumulate,
                       hipStream_t st);
hipError_t launch_convert(const float *src, double *dst, int64_t n, hipStream_t st);
hipError_t launch_copy_cols(const void *src, int64_t ld, int fp32, int s, int64_t n, double *dst, hipStream_t st);
hipError_t launch_diag_from_faces(const OpDev &op, double *dvec, int *bad, hipStream_t st);
hipError_t launch_diag_from_csr(const OpDev &op, double *dvec, int *bad, hipStream_t st);
hipError_t launch_to_fp32(const double *src, float *dst, int64_t n, hipStream_t st);
hipError_t launch_invert(const double *src, double *dst, int64_t n, int precond, hipStream_t st);

}  // namespace sstep
