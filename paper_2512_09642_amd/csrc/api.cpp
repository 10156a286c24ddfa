// C ABI of the s-step CG library: argument checking, device copies of the
// operator, workspace, the captured outer-iteration graph and the solve loop.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "launch.h"
#include "sstep.h"
#include "tune_cache.h"

using namespace sstep;

namespace {
thread_local std::string g_setup_error;  // message of a failed setup (no context yet)
}


struct sstep_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t user = nullptr;
    hipEvent_t ev_in = nullptr;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    IterArgs it;
    sstep_options opt{};
    std::vector<void *> dev_allocs;
    DevState *st_host = nullptr;  // pinned host mirror of the device state
    int32_t *poll_host = nullptr; // pinned [2][4]: done, status, iter of the last replays
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int chunk = 4;
    int64_t grad_size = 0;
    int *bad_flag = nullptr;       // device flag of the diagonal check
    char *ap_step = nullptr;       // A P of sstep_step when AP is not kept (allocated on first use)
    LzArgs lz;                     // Lanczos workspace (vectors: P's storage, or allocated on first use)
    double *lz_vecs = nullptr;
    struct Batched *batch = nullptr;  // set for contexts made by sstep_setup_batched
    CoarseArgs *coarse = nullptr;     // set for contexts made by sstep_coarse_setup
    int64_t coarse_bytes = 0;
    std::string err;
};

// State of a batched context (see sstep_setup_batched).
struct Batched {
    BatchArgs ba;
    std::vector<BSys> sys;
    std::vector<int64_t> n;
    BSys *dsys = nullptr;
    BTile *dbt = nullptr;
    PTile *dpt = nullptr;
    GTile *dgt = nullptr;
    BF2Tile *df2 = nullptr;
    // the two-step basis over ranges of kBf2MinPlanes planes, for the end of
    // a solve when too few pairs are left to fill the chip with the longer
    // ranges of df2: its band table, its systems (their moment partials laid
    // out for it) and a second graph
    BF2Tile *df2_tail = nullptr;
    BSys *dsys_tail = nullptr;
    int nf2_tail = 0;
    uint32_t *dmap = nullptr, *dmap_tail = nullptr;  // dispatch orders of the two tables
    uint32_t grid_tail = 0;
    struct BandLayout {
        int64_t mofs;
        int32_t f2first, nf2q;
    };
    std::vector<BandLayout> tail_bands;
    hipGraph_t graph_tail = nullptr;
    hipGraphExec_t gexec_tail = nullptr;
    int32_t tail_replays = 0;        // replays of the last solve on the short ranges
    int64_t gchunk = kMinBatchChunk;
    int grid_factor = 4;
    int cus = 256;
    DevState *pairs_host = nullptr;  // pinned
    BGlob *gl_host = nullptr;        // pinned
    int64_t total_n = 0;
};

namespace {

sstep_status fail(sstep_ctx *ctx, sstep_status code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_setup_error = msg;
    return code;
}

sstep_status hip_fail(sstep_ctx *ctx, const char *what, hipError_t e)
{
    return fail(ctx, e == hipErrorOutOfMemory ? SSTEP_E_NOMEM : SSTEP_E_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                 \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess)                             \
            return hip_fail((ctx), #call, e_);            \
    } while (0)

template <typename T>
sstep_status dalloc(sstep_ctx *ctx, T **p, size_t count)
{
    void *v = nullptr;
    const size_t bytes = count * sizeof(T) > 0 ? count * sizeof(T) : 256;
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess)
        return hip_fail(ctx, "hipMalloc", e);
    ctx->dev_allocs.push_back(v);
    *p = static_cast<T *>(v);
    return SSTEP_OK;
}

#define OKCHK(call)                          \
    do {                                     \
        sstep_status s_ = (call);            \
        if (s_ != SSTEP_OK)                  \
            return s_;                       \
    } while (0)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Copies count elements from host or device memory into a fresh device buffer.
template <typename T>
sstep_status to_device(sstep_ctx *ctx, T **dst, const T *src, size_t count, int ptr_space)
{
    OKCHK(dalloc(ctx, dst, count));
    HIPCHK(ctx, hipMemcpy(*dst, src, count * sizeof(T), ptr_space ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    return SSTEP_OK;
}

template <typename T>
sstep_status overwrite_device(sstep_ctx *ctx, T *dst, const T *src, size_t count, int ptr_space)
{
    HIPCHK(ctx, hipMemcpy(dst, src, count * sizeof(T), ptr_space ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    return SSTEP_OK;
}

template <typename T>
std::vector<T> to_host(const T *src, size_t count, int ptr_space, hipError_t *err)
{
    std::vector<T> h(count);
    *err = hipSuccess;
    if (count == 0)
        return h;
    if (ptr_space)
        *err = hipMemcpy(h.data(), src, count * sizeof(T), hipMemcpyDeviceToHost);
    else
        std::memcpy(h.data(), src, count * sizeof(T));
    return h;
}

int64_t faces_x(const sstep_operator *A) { return int64_t(A->nx + 1) * A->ny * A->nz; }
int64_t faces_y(const sstep_operator *A) { return int64_t(A->nx) * (A->ny + 1) * A->nz; }
int64_t faces_z(const sstep_operator *A) { return int64_t(A->nx) * A->ny * (A->nz + 1); }

sstep_status check_operator(sstep_ctx *ctx, const sstep_operator *A)
{
    if (!A)
        return fail(ctx, SSTEP_E_ARG, "operator is NULL");
    if (A->ptr_space != 0 && A->ptr_space != 1)
        return fail(ctx, SSTEP_E_ARG, "ptr_space must be 0 (host) or 1 (device)");
    if (A->kind == SSTEP_OP_STENCIL7) {
        if (A->nx < 1 || A->ny < 1 || A->nz < 1)
            return fail(ctx, SSTEP_E_ARG, "stencil grid sizes must be >= 1");
        const int64_t n = int64_t(A->nx) * A->ny * A->nz;
        if (n >= (int64_t(1) << 31) || faces_x(A) >= (int64_t(1) << 31) || faces_y(A) >= (int64_t(1) << 31) ||
            faces_z(A) >= (int64_t(1) << 31))
            return fail(ctx, SSTEP_E_ARG, "stencil grid too large (n must be < 2^31)");
        const int given = (A->kx != nullptr) + (A->ky != nullptr) + (A->kz != nullptr);
        if (given != 0 && given != 3)
            return fail(ctx, SSTEP_E_ARG, "give all three face arrays kx, ky, kz or none");
        return SSTEP_OK;
    }
    if (A->kind == SSTEP_OP_STENCIL27) {
        if (A->nx < 1 || A->ny < 1 || A->nz < 1)
            return fail(ctx, SSTEP_E_ARG, "stencil grid sizes must be >= 1");
        if (int64_t(A->nx) * A->ny * A->nz >= (int64_t(1) << 31))
            return fail(ctx, SSTEP_E_ARG, "stencil grid too large (n must be < 2^31)");
        if (A->kx || A->ky || A->kz)
            return fail(ctx, SSTEP_E_ARG, "the 27-point operator takes no coefficient arrays");
        return SSTEP_OK;
    }
    if (A->kind == SSTEP_OP_CSR) {
        if (A->n < 1 || A->n >= (int64_t(1) << 31))
            return fail(ctx, SSTEP_E_ARG, "CSR n must be in [1, 2^31)");
        if (A->nnz < 1 || A->nnz >= (int64_t(1) << 31))
            return fail(ctx, SSTEP_E_ARG, "CSR nnz must be in [1, 2^31)");
        if (!A->row_ptr || !A->col_idx || !A->val)
            return fail(ctx, SSTEP_E_ARG, "CSR arrays must not be NULL");
        return SSTEP_OK;
    }
    return fail(ctx, SSTEP_E_ARG, "unknown operator kind");
}

// CSR pattern check on the host: row_ptr[0] = 0, monotone, row_ptr[n] = nnz,
// columns in range and strictly ascending within a row.
sstep_status check_csr_pattern(sstep_ctx *ctx, const sstep_operator *A)
{
    hipError_t e1, e2;
    std::vector<int32_t> rp = to_host(A->row_ptr, size_t(A->n + 1), A->ptr_space, &e1);
    std::vector<int32_t> ci = to_host(A->col_idx, size_t(A->nnz), A->ptr_space, &e2);
    if (e1 != hipSuccess)
        return hip_fail(ctx, "hipMemcpy(row_ptr)", e1);
    if (e2 != hipSuccess)
        return hip_fail(ctx, "hipMemcpy(col_idx)", e2);
    if (rp[0] != 0 || rp[size_t(A->n)] != A->nnz)
        return fail(ctx, SSTEP_E_ARG, "malformed CSR: row_ptr[0] != 0 or row_ptr[n] != nnz");
    for (int64_t i = 0; i < A->n; ++i) {
        if (rp[i + 1] < rp[i])
            return fail(ctx, SSTEP_E_ARG, "malformed CSR: row_ptr not monotone at row " + std::to_string(i));
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= A->n)
                return fail(ctx, SSTEP_E_ARG, "malformed CSR: column out of range in row " + std::to_string(i));
            if (k > rp[i] && ci[k] <= ci[k - 1])
                return fail(ctx, SSTEP_E_ARG, "malformed CSR: columns not strictly ascending in row " +
                                                  std::to_string(i));
        }
    }
    return SSTEP_OK;
}

// The sliced ELL copy of a CSR pattern (OpEll): slice widths from the
// (validated) row pointers, slice offsets uploaded, columns filled on the
// device; the values are filled by load_coefficients.
sstep_status setup_ell(sstep_ctx *ctx, const sstep_operator *A)
{
    OpDev &op = ctx->it.op;
    hipError_t e = hipSuccess;
    const std::vector<int32_t> rp = to_host(A->row_ptr, size_t(A->n + 1), A->ptr_space, &e);
    if (e != hipSuccess)
        return hip_fail(ctx, "hipMemcpy(row_ptr)", e);
    const int64_t nslice = (op.n + kEllSlice - 1) / kEllSlice;
    std::vector<int64_t> off(size_t(nslice) + 1, 0);
    for (int64_t q = 0; q < nslice; ++q) {
        int32_t w = 0;
        for (int64_t r = q * kEllSlice; r < std::min<int64_t>(op.n, (q + 1) * kEllSlice); ++r)
            w = std::max(w, rp[size_t(r) + 1] - rp[size_t(r)]);
        off[size_t(q) + 1] = off[size_t(q)] + int64_t(w) * kEllSlice;
    }
    const size_t total = size_t(off[size_t(nslice)]);
    int64_t *doff = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    OKCHK(dalloc(ctx, &doff, size_t(nslice) + 1));
    OKCHK(dalloc(ctx, &col, total));
    OKCHK(dalloc(ctx, &val, total));
    HIPCHK(ctx, hipMemcpyAsync(doff, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    op.ell_off = doff;
    op.ell_nslice = nslice;
    op.ell_col = col;
    op.ell_val = val;
    HIPCHK(ctx, launch_ell_fill_col(op, col, ctx->stream));
    if (ctx->it.fp32) {
        float *val32 = nullptr;
        OKCHK(dalloc(ctx, &val32, total));
        op.ell_val32 = val32;
    }
    // off must stay alive until the copy has run
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SSTEP_OK;
}

// Loads (or reloads) the operator's coefficients and everything derived from
// them: M diagonal, its inverse, FP32 copies.
sstep_status load_coefficients(sstep_ctx *ctx, const sstep_operator *A, bool first)
{
    OpDev &op = ctx->it.op;
    const int fp32 = ctx->it.fp32;
    hipStream_t s = ctx->stream;
    if (first)
        OKCHK(dalloc(ctx, &ctx->bad_flag, 1));
    int *bad = ctx->bad_flag;
    HIPCHK(ctx, hipMemsetAsync(bad, 0, sizeof(int), s));
    if (op.kind == kOpCsr) {
        double *val = const_cast<double *>(op.val);
        double *dvec = const_cast<double *>(op.dvec);
        double *invd = const_cast<double *>(op.invd);
        if (first) {
            OKCHK(to_device(ctx, &val, A->val, size_t(op.nnz), A->ptr_space));
            OKCHK(dalloc(ctx, &dvec, size_t(ctx->it.ld)));
            OKCHK(dalloc(ctx, &invd, size_t(op.n)));
            HIPCHK(ctx, hipMemsetAsync(dvec, 0, size_t(ctx->it.ld) * sizeof(double), s));
            op.val = val;
            op.dvec = dvec;
            op.invd = invd;
        } else {
            OKCHK(overwrite_device(ctx, val, A->val, size_t(op.nnz), A->ptr_space));
        }
        HIPCHK(ctx, launch_diag_from_csr(op, dvec, bad, s));
        HIPCHK(ctx, launch_invert(dvec, invd, op.n, op.precond, s));
        if (op.ell_col)
            HIPCHK(ctx, launch_ell_fill_val(op, op.val, const_cast<double *>(op.ell_val), s));
        if (fp32) {
            float *val32 = const_cast<float *>(op.val32), *invd32 = const_cast<float *>(op.invd32);
            float *dvec32 = const_cast<float *>(op.dvec32);
            if (first) {
                OKCHK(dalloc(ctx, &val32, size_t(op.nnz)));
                OKCHK(dalloc(ctx, &invd32, size_t(op.n)));
                OKCHK(dalloc(ctx, &dvec32, size_t(ctx->it.ld)));
                HIPCHK(ctx, hipMemsetAsync(dvec32, 0, size_t(ctx->it.ld) * sizeof(float), s));
                op.val32 = val32;
                op.invd32 = invd32;
                op.dvec32 = dvec32;
            }
            HIPCHK(ctx, launch_to_fp32(val, val32, op.nnz, s));
            HIPCHK(ctx, launch_to_fp32(invd, invd32, op.n, s));
            HIPCHK(ctx, launch_to_fp32(dvec, dvec32, op.n, s));
            if (op.ell_val32)
                HIPCHK(ctx, launch_ell_fill_val(op, op.val32, const_cast<float *>(op.ell_val32), s));
        }
    } else if (op.kind == kOpFaces) {
        const int64_t nfx = faces_x(A), nfy = faces_y(A), nfz = faces_z(A);
        double *k = const_cast<double *>(op.kx);
        double *dvec = const_cast<double *>(op.dvec);
        if (first) {
            OKCHK(dalloc(ctx, &k, size_t(nfx + nfy + nfz)));
            OKCHK(dalloc(ctx, &dvec, size_t(ctx->it.ld)));
            HIPCHK(ctx, hipMemsetAsync(dvec, 0, size_t(ctx->it.ld) * sizeof(double), s));
            op.kx = k;
            op.ky = k + nfx;
            op.kz = k + nfx + nfy;
            op.dvec = dvec;
        }
        OKCHK(overwrite_device(ctx, k, A->kx, size_t(nfx), A->ptr_space));
        OKCHK(overwrite_device(ctx, k + nfx, A->ky, size_t(nfy), A->ptr_space));
        OKCHK(overwrite_device(ctx, k + nfx + nfy, A->kz, size_t(nfz), A->ptr_space));
        HIPCHK(ctx, launch_diag_from_faces(op, dvec, bad, s));
        if (fp32) {
            float *k32 = const_cast<float *>(op.kx32), *dvec32 = const_cast<float *>(op.dvec32);
            if (first) {
                OKCHK(dalloc(ctx, &k32, size_t(nfx + nfy + nfz)));
                OKCHK(dalloc(ctx, &dvec32, size_t(ctx->it.ld)));
                HIPCHK(ctx, hipMemsetAsync(dvec32, 0, size_t(ctx->it.ld) * sizeof(float), s));
                op.kx32 = k32;
                op.ky32 = k32 + nfx;
                op.kz32 = k32 + nfx + nfy;
                op.dvec32 = dvec32;
            }
            HIPCHK(ctx, launch_to_fp32(k, k32, nfx + nfy + nfz, s));
            HIPCHK(ctx, launch_to_fp32(dvec, dvec32, op.n, s));
        }
    }
    int hbad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (hbad)
        return fail(ctx, SSTEP_E_ARG, "matrix has a missing, non-positive or non-finite diagonal entry");
    return SSTEP_OK;
}

// The operator-applying Gram kernel: 7-point stencil operators, s <= 16,
// columns under 4 GiB (32-bit byte offsets); by default for FP64 only (in
// FP32+IR the stored-AP kernel is as fast).
// The moments kind needs the Chebyshev basis and c = P^T r expressible in the
// same M inner product as H: r = M p_0 (p_0 = M^{-1} r) or M = I; and FP64:
// an FP32 basis departs from the polynomial identities by about 1e-8, which
// under loose bounds can exceed the small diagonal entries p_i^T A p_i formed
// from H (a batched FP32+IR solve broke down so).
bool moments_fit(int s, const sstep_options &o)
{
    return s <= kRecMaxS && o.basis == 0 && (o.p0_mode == 0 || o.precond == 0) && o.precision == SSTEP_FP64;
}

sstep_status choose_gram_kind(sstep_ctx *ctx, const sstep_operator *A, int s, const sstep_options &o, int *kind,
                              bool allow_moments)
{
    if (o.gram == SSTEP_GRAM_MOMENTS) {
        if (!allow_moments || !moments_fit(s, o))
            return fail(ctx, SSTEP_E_UNSUPPORTED,
                        "the moments Gram kind needs FP64, the Chebyshev basis, s <= 31, p_0 = M^{-1} r or no "
                        "preconditioner, and a context that may allocate");
        *kind = SSTEP_GRAM_MOMENTS;
        return SSTEP_OK;
    }
    // AUTO: the moments kind where it applies (FP64)
    if (o.gram == SSTEP_GRAM_AUTO && allow_moments && moments_fit(s, o)) {
        *kind = SSTEP_GRAM_MOMENTS;
        return SSTEP_OK;
    }
    if (o.gram == SSTEP_GRAM_RECURRENCE) {
        if (s > kRecMaxS)
            return fail(ctx, SSTEP_E_UNSUPPORTED, "the recurrence Gram kind needs s <= 31");
        *kind = SSTEP_GRAM_RECURRENCE;
        return SSTEP_OK;
    }
    const int64_t n = A->kind == SSTEP_OP_CSR ? A->n : int64_t(A->nx) * A->ny * A->nz;
    const uint64_t wbytes = o.precision == SSTEP_FP32_IR ? sizeof(float) : sizeof(double);
    const bool op_ok = A->kind == SSTEP_OP_STENCIL7 && s <= kGoMaxS &&
                       uint64_t(round_up(n, kPad)) * wbytes < (uint64_t(1) << 32);
    if (o.gram == SSTEP_GRAM_APPLY_OP && !op_ok)
        return fail(ctx, SSTEP_E_UNSUPPORTED,
                    "the operator-applying Gram kernel needs a 7-point stencil operator, s <= 16 and columns "
                    "under 4 GiB");
    if (o.gram == SSTEP_GRAM_APPLY_OP)
        *kind = SSTEP_GRAM_APPLY_OP;
    else if (o.gram == SSTEP_GRAM_STORED_AP)
        *kind = SSTEP_GRAM_STORED_AP;
    else  // AUTO: the recurrence kind was measured fastest for every operator, precision and s <= 31
        *kind = s <= kRecMaxS ? SSTEP_GRAM_RECURRENCE : (op_ok && o.precision == SSTEP_FP64 ? SSTEP_GRAM_APPLY_OP
                                                                                               : SSTEP_GRAM_STORED_AP);
    return SSTEP_OK;
}

// The Gram kind's launch arguments.  Recurrence kind: the Gram kernel weights
// its second operand by the M diagonal array when M is not a constant
// multiple of I, else the FGS kernel applies the constant (6, 26, or 1 without
// preconditioning).
void set_gram_kind(IterArgs &it, int kind, int precond, bool const_diag)
{
    it.gram_op = kind == SSTEP_GRAM_APPLY_OP;
    it.gram_rec = kind == SSTEP_GRAM_RECURRENCE || kind == SSTEP_GRAM_MOMENTS;
    it.gram_mom = kind == SSTEP_GRAM_MOMENTS;
    it.rec_wap = it.gram_rec && precond && !const_diag;
    it.rec_hscale = (it.gram_rec && precond && const_diag) ? (it.op.kind == kOpPoisson27 ? 26.0 : 6.0) : 1.0;
}

// Residual kernel schedule: at most 1024 row chunks (one partial each), or
// for the constant Poisson operator with an even x-extent the 1024-thread
// blocks of 2 x-points x 8 planes when they number at most 1024.
void set_residual_schedule(IterArgs &it)
{
    const OpDev &op = it.op;
    const int64_t n = op.n;
    it.nbr = int(std::min<int64_t>(1024, (n + kBlock - 1) / kBlock));
    it.rchunk = round_up((n + it.nbr - 1) / it.nbr, kBlock);
    it.res_p2 = 0;
    if (op.kind == kOpPoisson && op.g.nx % 2 == 0) {
        const int64_t blocks = ((op.g.nxy / 2 + 1023) / 1024) * ((op.g.nz + 7) / 8);
        if (blocks <= 1024) {
            it.res_p2 = 1;
            it.nbr = int(blocks);
        }
    }
}

// Enqueues one outer iteration: residual + p_0, the basis steps, Gram
// partials, FGS, update.
hipError_t enqueue_iteration(const IterArgs &a, hipStream_t s)
{
    hipError_t e;
    if ((e = launch_residual(a, s, true)) != hipSuccess)
        return e;
    if ((e = launch_basis_all(a, s)) != hipSuccess)
        return e;
    if ((e = launch_gram(a, s)) != hipSuccess)
        return e;
    if ((e = launch_fgs(a, s)) != hipSuccess)
        return e;
    return launch_update(a, s);
}

// Initial device state for a solve (or a single step) on b, x.
sstep_status start_state(sstep_ctx *ctx, const double *b, double *x, double tol, int no_stop)
{
    DevState &h = *ctx->st_host;
    std::memset(&h, 0, sizeof(DevState));
    h.b = b;
    h.x = x;
    h.tol = tol;
    h.p0scale = 1.0;
    h.first = 1;
    h.no_stop = no_stop;
    h.max_outer = no_stop ? (1 << 30) : ctx->opt.max_outer;
    h.hist_cap = ctx->it.hist_cap;
    HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    HIPCHK(ctx, hipMemcpyAsync(ctx->it.st, &h, sizeof(DevState), hipMemcpyHostToDevice, ctx->stream));
    if (ctx->it.fp32) {
        HIPCHK(ctx, launch_residual(ctx->it, ctx->stream, false));
        HIPCHK(ctx, launch_p0scale(ctx->it, ctx->stream));
    }
    return SSTEP_OK;
}


// ---------------------------------------------------------------------------
// Gram schedule and its autotuner.
// ---------------------------------------------------------------------------
// nbg: stored-AP kernel: partial blocks; operator-applying kernel: block cap.
// slab: stored-AP kernel: 0 contiguous chunks, > 0 strided slabs of this many rows.
using GramSchedule = TuneEntry;

GramSchedule default_gram_schedule(const IterArgs &it)
{
    // Measured on MI355X at 224^3, s = 16: FP64 prefers one contiguous chunk
    // per CU, FP32 prefers grid-strided 2048-row slabs.
    if (it.gram_op)
        return GramSchedule{1024, 0, 0.0};
    if (it.gram_rec)
        return GramSchedule{kMaxGramBlocks, 0, 0.0};  // matrix-core Gram: many small blocks, contiguous rows
    return it.fp32 ? GramSchedule{256, 2048, 0.0} : GramSchedule{256, 0, 0.0};
}

// Geometry of the operator-applying Gram kernel: 32 x 8 in-plane tiles, the
// full ones taken by one launch and the edge ones (partial in x or y) by a
// second; the z-extent cut into even ranges so that the (tile, range) items
// number about `cap`; one block per item up to the cap (a block loops over
// several items beyond that).  One partial slot per block, the edge launch's
// after the full launch's.
void set_go_geometry(IterArgs &it, int cap)
{
    const Grid3 &g = it.op.g;
    const int64_t tx = 32, ty = 8;
    cap = std::max(2, std::min(cap, kMaxGramBlocks));
    const int64_t tiles_x = (g.nx + tx - 1) / tx, tiles_y = (g.ny + ty - 1) / ty;
    const int64_t tiles = tiles_x * tiles_y;
    it.go_fx = int(g.nx / tx);
    it.go_fy = int(g.ny / ty);
    it.go_tiles_y = int(tiles_y);
    it.go_rx = g.nx % tx != 0;
    it.go_ry = g.ny % ty != 0;
    const int64_t nzb_t = std::max<int64_t>(1, std::min<int64_t>(g.nz, cap / tiles));
    const int64_t zr = round_up((g.nz + nzb_t - 1) / nzb_t, 2);  // even: the kernel runs z-steps in pairs
    const int64_t nzb = (g.nz + zr - 1) / zr;
    it.go_zr = int(zr);
    it.go_nzb = int(nzb);
    const int64_t tf = int64_t(it.go_fx) * it.go_fy;
    const int64_t te = tiles - tf;  // = rx * tiles_y + ry * fx
    it.go_tiles[0] = int(tf);
    it.go_tiles[1] = int(te);
    it.go_items[0] = int(tf * nzb);
    it.go_items[1] = int(te * nzb);
    // blocks in proportion to the items, within the cap in total
    const int64_t items = tiles * nzb;
    int64_t bf = std::min<int64_t>(tf * nzb, std::max<int64_t>(tf > 0, (int64_t(cap) * tf * nzb) / items));
    int64_t be = std::min<int64_t>(te * nzb, std::max<int64_t>(te > 0, int64_t(cap) - bf));
    it.go_blocks[0] = int(bf);
    it.go_blocks[1] = int(be);
    it.nbg = int(bf + be);
}

void set_gram_schedule(IterArgs &it, const GramSchedule &g)
{
    if (it.gram_op) {
        set_go_geometry(it, g.nbg);
        return;
    }
    const int64_t blocks_needed = (it.ld + kPad - 1) / kPad;
    it.nbg = int(std::max<int64_t>(1, std::min<int64_t>(std::min(g.nbg, kMaxGramBlocks), blocks_needed)));
    it.gslab = g.slab;
    it.gchunk = round_up((it.ld + it.nbg - 1) / it.nbg, kPad);
}

std::string tune_cache_path()
{
    if (const char *p = std::getenv("SSTEP_TUNE_CACHE"))
        return p;
    const char *home = std::getenv("HOME");
    if (!home)
        return "";
    std::string dir = std::string(home) + "/.cache";
    mkdir(dir.c_str(), 0755);
    dir += "/sstep";
    mkdir(dir.c_str(), 0755);
    return dir + "/tune.json";
}

std::string tune_key(const IterArgs &it)
{
    std::ostringstream k;
    k << kTuneSchema << " gfx950 gram s=" << it.s << " prec=" << (it.fp32 ? "fp32" : "fp64") << " rows=" << it.ld
      << " wd=" << it.wdvec;
    if (it.gram_op)
        k << " op2=" << it.op.kind << " grid=" << it.op.g.nx << "x" << it.op.g.ny << "x" << it.op.g.nz;
    if (it.gram_rec)
        k << " rec wap=" << it.rec_wap;
    return k.str();
}

// Times each candidate Gram schedule on the context's own buffers (the values
// do not matter for the timing) and keeps the fastest; the result is cached
// on disk per device, basis width, precision, row count and right-hand-side mode.
sstep_status tune_gram(sstep_ctx *ctx)
{
    IterArgs &it = ctx->it;
    const std::string path = tune_cache_path();
    const std::string key = tune_key(it);
    std::map<std::string, GramSchedule> cache;
    if (!path.empty()) {
        cache = read_tune_cache(path);
        auto f = cache.find(key);
        if (f != cache.end() && gram_entry_ok(f->second, kMaxGramBlocks, kPad)) {
            set_gram_schedule(it, f->second);
            return SSTEP_OK;
        }
    }
    std::vector<GramSchedule> cand;
    if (it.gram_op) {
        // at most 1024 partial slots: the FGS kernel's reduction of the
        // partials grows with their number and is not part of this timing
        for (int cap : {256, 384, 512, 768, 1024})
            cand.push_back({cap, 0, 0.0});
    } else if (it.gram_rec) {
        for (int nbg : {512, 1024, 1536, 2048})  // contiguous row chunks only
            cand.push_back({nbg, 0, 0.0});
    } else {
        for (int nbg : {256, 384, 512, 1024, 2048})
            cand.push_back({nbg, 0, 0.0});
        for (int64_t slab : {int64_t(1024), int64_t(2048), int64_t(4096)})
            for (int nbg : {256, 512, 1024, 2048})
                cand.push_back({nbg, slab, 0.0});
    }
    GramSchedule best = default_gram_schedule(it);
    best.us = 1e30;
    for (GramSchedule &c : cand) {
        set_gram_schedule(it, c);
        HIPCHK(ctx, launch_gram(it, ctx->stream));  // warm-up
        HIPCHK(ctx, hipEventRecord(ctx->ev_t0, ctx->stream));
        const int reps = 3;
        for (int r = 0; r < reps; ++r)
            HIPCHK(ctx, launch_gram(it, ctx->stream));
        HIPCHK(ctx, hipEventRecord(ctx->ev_t1, ctx->stream));
        HIPCHK(ctx, hipEventSynchronize(ctx->ev_t1));
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
        c.us = 1e3 * ms / reps;
        if (c.us < best.us)
            best = c;
    }
    set_gram_schedule(it, best);
    if (!path.empty()) {
        cache[key] = best;
        write_tune_cache(path, cache);
    }
    return SSTEP_OK;
}

sstep_status capture_graph(sstep_ctx *ctx)
{
    HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int c = 0; c < ctx->chunk && e == hipSuccess; ++c)
        e = enqueue_iteration(ctx->it, ctx->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
    if (e != hipSuccess)
        return hip_fail(ctx, "kernel launch during graph capture", e);
    if (e2 != hipSuccess)
        return hip_fail(ctx, "hipStreamEndCapture", e2);
    ctx->graph = g;
    HIPCHK(ctx, hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
    return SSTEP_OK;
}

sstep_status run_solve(sstep_ctx *ctx, const double *b, double *x, double tol, sstep_stats *stats)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (ctx->batch)
        return fail(ctx, SSTEP_E_ARG, "this context was made by sstep_setup_batched: use sstep_solve_batched");
    if (!b || !x)
        return fail(ctx, SSTEP_E_ARG, "b and x must not be NULL");
    if (!(tol > 0.0) || !(tol < 1.0))
        return fail(ctx, SSTEP_E_ARG, "tol must be in (0, 1)");
    OKCHK(start_state(ctx, b, x, tol, 0));
    const int max_replays = (ctx->opt.max_outer + 1 + ctx->chunk - 1) / ctx->chunk + 1;
    int launched = 0, checked = 0;
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = hipGraphLaunch(ctx->gexec, ctx->stream);
        if (e != hipSuccess)
            return e;
        int32_t *slot = ctx->poll_host + 4 * (launched % 2);
        e = hipMemcpyAsync(slot, &ctx->it.st->done, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
        if (e != hipSuccess)
            return e;
        e = hipEventRecord(ctx->ev_poll[launched % 2], ctx->stream);
        ++launched;
        return e;
    };
    HIPCHK(ctx, enqueue());
    for (;;) {
        if (launched < max_replays)
            HIPCHK(ctx, enqueue());  // keep one replay queued behind the one being checked
        HIPCHK(ctx, hipEventSynchronize(ctx->ev_poll[checked % 2]));
        const int32_t done = ctx->poll_host[4 * (checked % 2)];
        ++checked;
        if (done)
            break;
        if (checked >= launched) {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            return fail(ctx, SSTEP_E_HIP, "solve did not stop within the replay bound");
        }
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    DevState h;
    HIPCHK(ctx, hipMemcpy(&h, ctx->it.st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (stats) {
        stats->outer_iters = h.iter;
        stats->status = h.status;
        stats->rel_res = h.relres;
        stats->res0 = h.rho0;
        if (stats->hist_cap > 0 && ctx->it.hist_cap > 0) {
            const int nr = std::min(std::min(stats->hist_cap, ctx->it.hist_cap), h.iter + 1);
            const int nd = std::min(std::min(stats->hist_cap, ctx->it.hist_cap), h.iter);
            if (stats->hist_relres && nr > 0)
                HIPCHK(ctx, hipMemcpy(stats->hist_relres, ctx->it.hist, nr * sizeof(double), hipMemcpyDeviceToHost));
            if (stats->hist_delta && nd > 0)
                HIPCHK(ctx, hipMemcpy(stats->hist_delta, ctx->it.hist + ctx->it.hist_cap, nd * sizeof(double),
                                      hipMemcpyDeviceToHost));
            if (stats->hist_lnorm && nd > 0)
                HIPCHK(ctx, hipMemcpy(stats->hist_lnorm, ctx->it.hist + 2 * ctx->it.hist_cap, nd * sizeof(double),
                                      hipMemcpyDeviceToHost));
        }
    }
    const sstep_status code = static_cast<sstep_status>(h.status);
    if (code != SSTEP_OK)
        return fail(ctx, code, std::string("solve stopped: ") + sstep_status_string(code));
    return SSTEP_OK;
}

}  // namespace

extern "C" {

void sstep_default_options(sstep_options *opt)
{
    if (!opt)
        return;
    opt->precision = SSTEP_FP64;
    opt->precond = 1;
    opt->p0_mode = 0;
    opt->max_outer = 10000;
    opt->graph_chunk = 4;
    opt->record_history = 0;
    opt->autotune = 1;
    opt->gram = SSTEP_GRAM_AUTO;
    opt->basis = 0;
    opt->basis_steps = 0;
    opt->stream = nullptr;
}

const char *sstep_status_string(sstep_status s)
{
    switch (s) {
    case SSTEP_OK:
        return "SSTEP_OK";
    case SSTEP_E_ARG:
        return "SSTEP_E_ARG";
    case SSTEP_E_HIP:
        return "SSTEP_E_HIP";
    case SSTEP_E_NOMEM:
        return "SSTEP_E_NOMEM";
    case SSTEP_E_BREAKDOWN:
        return "SSTEP_E_BREAKDOWN";
    case SSTEP_E_NOCONV:
        return "SSTEP_E_NOCONV";
    case SSTEP_E_NONFINITE:
        return "SSTEP_E_NONFINITE";
    case SSTEP_E_UNSUPPORTED:
        return "SSTEP_E_UNSUPPORTED";
    }
    return "unknown status";
}

const char *sstep_last_error(const sstep_ctx *ctx) { return ctx ? ctx->err.c_str() : g_setup_error.c_str(); }

void sstep_destroy(sstep_ctx *ctx)
{
    if (!ctx)
        return;
    if (ctx->stream)
        (void)hipStreamSynchronize(ctx->stream);
    if (ctx->gexec)
        (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph)
        (void)hipGraphDestroy(ctx->graph);
    for (void *p : ctx->dev_allocs)
        (void)hipFree(p);
    if (ctx->st_host)
        (void)hipHostFree(ctx->st_host);
    if (ctx->poll_host)
        (void)hipHostFree(ctx->poll_host);
    for (hipEvent_t e : {ctx->ev_in, ctx->ev_poll[0], ctx->ev_poll[1], ctx->ev_t0, ctx->ev_t1})
        if (e)
            (void)hipEventDestroy(e);
    if (ctx->stream)
        (void)hipStreamDestroy(ctx->stream);
    delete ctx->coarse;
    if (ctx->batch) {
        if (ctx->batch->gexec_tail)
            (void)hipGraphExecDestroy(ctx->batch->gexec_tail);
        if (ctx->batch->graph_tail)
            (void)hipGraphDestroy(ctx->batch->graph_tail);
        if (ctx->batch->pairs_host)
            (void)hipHostFree(ctx->batch->pairs_host);
        if (ctx->batch->gl_host)
            (void)hipHostFree(ctx->batch->gl_host);
        delete ctx->batch;
    }
    delete ctx;
}

static sstep_status setup_impl(sstep_ctx *ctx, const sstep_operator *A, int32_t s, int32_t nu, double lmin,
                               double lmax, const sstep_options *opt)
{
    if (opt)
        ctx->opt = *opt;
    else
        sstep_default_options(&ctx->opt);
    sstep_options &o = ctx->opt;
    if (s < 1 || s > kMaxS)
        return fail(ctx, SSTEP_E_ARG, "s must be in [1, 32]");
    if (nu < 1)
        return fail(ctx, SSTEP_E_ARG, "nu must be >= 1");
    if (!std::isfinite(lmin) || !std::isfinite(lmax) || lmin < 0.0 || !(lmax > lmin))
        return fail(ctx, SSTEP_E_ARG, "bounds must be finite with 0 <= lambda_min < lambda_max");
    if (o.precision != SSTEP_FP64 && o.precision != SSTEP_FP32_IR)
        return fail(ctx, SSTEP_E_ARG, "unknown precision");
    if (o.precond != 0 && o.precond != 1)
        return fail(ctx, SSTEP_E_ARG, "precond must be 0 or 1");
    if (o.p0_mode != 0 && o.p0_mode != 1)
        return fail(ctx, SSTEP_E_ARG, "p0_mode must be 0 or 1");
    if (o.max_outer < 0)
        return fail(ctx, SSTEP_E_ARG, "max_outer must be >= 0");
    if (o.basis != 0 && o.basis != 1)
        return fail(ctx, SSTEP_E_ARG, "basis must be 0 (Chebyshev) or 1 (monomial)");
    if (o.basis_steps != 0 && o.basis_steps != 1)
        return fail(ctx, SSTEP_E_ARG, "basis_steps must be 0 or 1");
    if (o.graph_chunk <= 0)
        o.graph_chunk = 4;
    OKCHK(check_operator(ctx, A));
    if (A->kind == SSTEP_OP_CSR)
        OKCHK(check_csr_pattern(ctx, A));
    if (o.gram < SSTEP_GRAM_AUTO || o.gram > SSTEP_GRAM_MOMENTS)
        return fail(ctx, SSTEP_E_ARG, "unknown gram kind");
    int gram_kind = SSTEP_GRAM_STORED_AP;
    OKCHK(choose_gram_kind(ctx, A, s, o, &gram_kind, true));

    HIPCHK(ctx, hipGetDevice(&ctx->device));
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    ctx->user = static_cast<hipStream_t>(o.stream);
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_poll[0], hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_poll[1], hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreate(&ctx->ev_t0));
    HIPCHK(ctx, hipEventCreate(&ctx->ev_t1));
    {
        void *p = nullptr;
        HIPCHK(ctx, hipHostMalloc(&p, sizeof(DevState), hipHostMallocDefault));
        ctx->st_host = static_cast<DevState *>(p);
        HIPCHK(ctx, hipHostMalloc(&p, 8 * sizeof(int32_t), hipHostMallocDefault));
        ctx->poll_host = static_cast<int32_t *>(p);
    }

    IterArgs &it = ctx->it;
    OpDev &op = it.op;
    it.fp32 = o.precision == SSTEP_FP32_IR;
    it.p0_mode = o.p0_mode;
    it.monomial = o.basis;
    it.one_step = o.basis_steps;
    it.s = s;
    it.nu = nu;
    it.theta = 2.0 / (lmax - lmin);
    it.sigma = (lmax + lmin) / 2.0;
    op.precond = o.precond;
    if (A->kind == SSTEP_OP_STENCIL7 || A->kind == SSTEP_OP_STENCIL27) {
        op.kind = A->kind == SSTEP_OP_STENCIL27 ? kOpPoisson27 : (A->kx ? kOpFaces : kOpPoisson);
        op.n = int64_t(A->nx) * A->ny * A->nz;
        op.g.nx = A->nx;
        op.g.ny = A->ny;
        op.g.nz = A->nz;
        op.g.nxy = int64_t(A->nx) * A->ny;
        op.g.dx = make_fastdiv(uint32_t(A->nx));
        op.g.dy = make_fastdiv(uint32_t(A->ny));
        ctx->grad_size = op.kind == kOpPoisson27 ? 0 : faces_x(A) + faces_y(A) + faces_z(A);
    } else {
        op.kind = kOpCsr;
        op.n = A->n;
        op.nnz = A->nnz;
        int32_t *rp = nullptr, *ci = nullptr;
        OKCHK(to_device(ctx, &rp, A->row_ptr, size_t(A->n + 1), A->ptr_space));
        OKCHK(to_device(ctx, &ci, A->col_idx, size_t(A->nnz), A->ptr_space));
        op.rp = rp;
        op.ci = ci;
        ctx->grad_size = A->nnz;
        OKCHK(setup_ell(ctx, A));
    }
    it.ld = round_up(op.n, kPad);
    OKCHK(load_coefficients(ctx, A, true));

    // right-hand side of the Gram system: c = P^T r with r = M p_0 (p0_mode 0)
    // or r = p_0 (p0_mode 1 or no preconditioner)
    const bool jac_p0 = o.precond == 1 && o.p0_mode == 0;
    const bool const_diag = op.kind == kOpPoisson || op.kind == kOpPoisson27;
    it.wdvec = jac_p0 && !const_diag;
    it.cscale = (jac_p0 && const_diag) ? (op.kind == kOpPoisson27 ? 26.0 : 6.0) : 1.0;

    // workspace: P and AP zero-filled, so the padding rows n..ld-1 read as 0;
    // stencil operators with s <= 16 use the Gram kernel that applies the
    // operator itself, and AP is not kept
    const int64_t n = op.n;
    const size_t w = it.fp32 ? sizeof(float) : sizeof(double);
    set_gram_kind(it, gram_kind, o.precond, const_diag);
    {
        // the recurrence kind keeps one more column, p_s
        const int pcols = s + it.gram_rec;
        char *P = nullptr, *AP = nullptr;
        OKCHK(dalloc(ctx, &P, size_t(it.ld) * pcols * w));
        HIPCHK(ctx, hipMemsetAsync(P, 0, size_t(it.ld) * pcols * w, ctx->stream));
        if (!it.gram_op && !it.gram_rec) {
            OKCHK(dalloc(ctx, &AP, size_t(it.ld) * s * w));
            HIPCHK(ctx, hipMemsetAsync(AP, 0, size_t(it.ld) * s * w, ctx->stream));
        }
        it.P = P;
        it.AP = AP;
    }
    set_residual_schedule(it);
    OKCHK(dalloc(ctx, &it.rpart, size_t(it.nbr)));
    if (it.gram_mom) {
        std::vector<int32_t> cnt(size_t(2 * s + 1), 0);
        mom_layout(it, cnt.data(), &it.mstride);
        OKCHK(dalloc(ctx, &it.mpart, size_t(2 * s + 1) * size_t(it.mstride)));
        OKCHK(dalloc(ctx, &it.mcnt, cnt.size()));
        HIPCHK(ctx, hipMemcpy(it.mcnt, cnt.data(), cnt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    } else {
        OKCHK(dalloc(ctx, &it.gpart, size_t(gram_entries(s + it.gram_rec)) * kMaxGramBlocks));
    }
    OKCHK(dalloc(ctx, &it.gsum, size_t(gram_entries(s + it.gram_rec)) + 1));
    OKCHK(dalloc(ctx, &it.st, 1));
    OKCHK(dalloc(ctx, &it.dbg, size_t(dbg_size(s))));
    it.hist_cap = o.record_history ? o.max_outer + 1 : 0;
    OKCHK(dalloc(ctx, &it.hist, size_t(3 * std::max(it.hist_cap, 1))));
    it.inv_sqrt_n = 1.0 / std::sqrt(double(n));
    {
        LzArgs &l = ctx->lz;
        l.n = n;
        l.nb = int(std::min<int64_t>(1024, (n + kBlock - 1) / kBlock));
        l.chunk = round_up((n + l.nb - 1) / l.nb, kBlock);
        OKCHK(dalloc(ctx, &l.part, size_t(l.nb)));
        OKCHK(dalloc(ctx, &l.ab, size_t(3 * kMaxLanczos)));
        OKCHK(dalloc(ctx, &l.ls, 1));
    }
    HIPCHK(ctx, hipMemsetAsync(it.st, 0, sizeof(DevState), ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    set_gram_schedule(it, default_gram_schedule(it));
    if (o.autotune && n >= (int64_t(1) << 20) && !it.gram_mom)  // the moments kind has no Gram kernel
        OKCHK(tune_gram(ctx));

    ctx->chunk = o.graph_chunk;
    OKCHK(capture_graph(ctx));
    return SSTEP_OK;
}

sstep_status sstep_setup(sstep_ctx **out, const sstep_operator *A, int32_t s, int32_t nu, double lambda_min,
                         double lambda_max, const sstep_options *opt)
{
    if (!out)
        return fail(nullptr, SSTEP_E_ARG, "out is NULL");
    *out = nullptr;
    sstep_ctx *ctx = new (std::nothrow) sstep_ctx();
    if (!ctx)
        return fail(nullptr, SSTEP_E_NOMEM, "out of host memory");
    const sstep_status st = setup_impl(ctx, A, s, nu, lambda_min, lambda_max, opt);
    if (st != SSTEP_OK) {
        g_setup_error = ctx->err;
        sstep_destroy(ctx);
        return st;
    }
    *out = ctx;
    return SSTEP_OK;
}

sstep_status sstep_update_coefficients(sstep_ctx *ctx, const sstep_operator *A)
{
    if (!ctx)
        return SSTEP_E_ARG;
    OKCHK(check_operator(ctx, A));
    const OpDev &op = ctx->it.op;
    if (op.kind == kOpCsr) {
        if (A->kind != SSTEP_OP_CSR || A->n != op.n || A->nnz != op.nnz)
            return fail(ctx, SSTEP_E_ARG, "operator kind or sizes differ from setup");
    } else {
        const int kind = op.kind == kOpPoisson27 ? SSTEP_OP_STENCIL27 : SSTEP_OP_STENCIL7;
        if (A->kind != kind || A->nx != op.g.nx || A->ny != op.g.ny || A->nz != op.g.nz)
            return fail(ctx, SSTEP_E_ARG, "operator kind or grid differ from setup");
        if ((op.kind == kOpFaces) != (A->kx != nullptr))
            return fail(ctx, SSTEP_E_ARG, "constant and face-coefficient stencils cannot be swapped");
        if (op.kind == kOpPoisson || op.kind == kOpPoisson27)
            return SSTEP_OK;  // no coefficients
    }
    return load_coefficients(ctx, A, false);
}

int64_t sstep_n(const sstep_ctx *ctx) { return ctx ? (ctx->batch ? ctx->batch->total_n : ctx->it.op.n) : 0; }

int64_t sstep_grad_size(const sstep_ctx *ctx) { return ctx ? ctx->grad_size : 0; }

sstep_status sstep_apply(sstep_ctx *ctx, const double *x, double *y)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (!x || !y || x == y)
        return fail(ctx, SSTEP_E_ARG, "x and y must be distinct non-NULL device pointers");
    HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    HIPCHK(ctx, launch_apply(ctx->it.op, x, y, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SSTEP_OK;
}

int32_t sstep_gram_mode(const sstep_ctx *ctx)
{
    if (!ctx)
        return -1;
    if (ctx->batch)
        return ctx->batch->ba.mom ? SSTEP_GRAM_MOMENTS
                                  : (ctx->batch->ba.rec ? SSTEP_GRAM_RECURRENCE : SSTEP_GRAM_STORED_AP);
    if (ctx->it.gram_mom)
        return SSTEP_GRAM_MOMENTS;
    return ctx->it.gram_rec ? SSTEP_GRAM_RECURRENCE : (ctx->it.gram_op ? SSTEP_GRAM_APPLY_OP : SSTEP_GRAM_STORED_AP);
}

sstep_status sstep_batched_tiles(const sstep_ctx *ctx, int64_t *rows_per_tile, int32_t *grid_factor)
{
    if (!ctx || !ctx->batch)
        return SSTEP_E_ARG;
    if (rows_per_tile)
        *rows_per_tile = ctx->batch->gchunk;
    if (grid_factor)
        *grid_factor = ctx->batch->grid_factor;
    return SSTEP_OK;
}

sstep_status sstep_batched_bands(const sstep_ctx *ctx, int32_t *bands, int32_t *tail_bands, int32_t *tail_replays)
{
    if (!ctx || !ctx->batch)
        return SSTEP_E_ARG;
    const Batched &B = *ctx->batch;
    if (bands)
        *bands = B.ba.f2 ? B.ba.nf2 : 0;
    if (tail_bands)
        *tail_bands = B.nf2_tail;
    if (tail_replays)
        *tail_replays = B.tail_replays;
    return SSTEP_OK;
}

int32_t sstep_basis_launches(const sstep_ctx *ctx, int32_t *pairs)
{
    if (!ctx)
        return -1;
    int np = 0, n = 0;
    if (ctx->batch) {
        const BatchArgs &a = ctx->batch->ba;
        np = a.f2 ? a.s / 2 : 0;
        n = a.s - np;
    } else {
        n = basis_kernel_count(ctx->it, &np);
    }
    if (pairs)
        *pairs = np;
    return n;
}

sstep_status sstep_solve(sstep_ctx *ctx, const double *b, double *x, double tol, sstep_stats *st)
{
    return run_solve(ctx, b, x, tol, st);
}

sstep_status sstep_solve_adjoint(sstep_ctx *ctx, const double *g, double *lam, double tol, sstep_stats *st)
{
    // A is symmetric positive definite, so A^T lam = g is the same system.
    return run_solve(ctx, g, lam, tol, st);
}

sstep_status sstep_grad_operator(sstep_ctx *ctx, const double *lam, const double *x, double *dA, int32_t accumulate)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (!lam || !x || !dA)
        return fail(ctx, SSTEP_E_ARG, "lam, x and dA must not be NULL");
    if (ctx->it.op.kind == kOpPoisson27)
        return fail(ctx, SSTEP_E_UNSUPPORTED, "the 27-point operator has no coefficients to differentiate");
    HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    HIPCHK(ctx, launch_grad(ctx->it.op, lam, x, dA, accumulate ? 1 : 0, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SSTEP_OK;
}

sstep_status sstep_step(sstep_ctx *ctx, const double *b, double *x, double *alpha_tilde, double *G, double *ctil,
                        double *rnorm, double *P_out, double *AP_out)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (!b || !x)
        return fail(ctx, SSTEP_E_ARG, "b and x must not be NULL");
    const IterArgs &it = ctx->it;
    const int s = it.s;
    HIPCHK(ctx, hipMemsetAsync(it.dbg, 0, size_t(dbg_size(s)) * sizeof(double), ctx->stream));
    OKCHK(start_state(ctx, b, x, 0.5, 1));
    HIPCHK(ctx, enqueue_iteration(it, ctx->stream));
    if (P_out)
        HIPCHK(ctx, launch_copy_cols(it.P, it.ld, it.fp32, s, it.op.n, P_out, ctx->stream));
    if (AP_out) {
        if (!it.AP) {
            // AP is not kept: form A p_j with the basis kernels' product step
            // into a buffer allocated on first use.
            if (!ctx->ap_step) {
                char *buf = nullptr;
                const size_t bytes = size_t(it.ld) * s * (it.fp32 ? sizeof(float) : sizeof(double));
                OKCHK(dalloc(ctx, &buf, bytes));
                HIPCHK(ctx, hipMemsetAsync(buf, 0, bytes, ctx->stream));
                ctx->ap_step = buf;
            }
            IterArgs t = it;
            t.AP = ctx->ap_step;
            for (int j = 0; j < s; ++j)
                HIPCHK(ctx, launch_product(t, j, ctx->stream));
            HIPCHK(ctx, launch_copy_cols(t.AP, it.ld, it.fp32, s, it.op.n, AP_out, ctx->stream));
        } else {
            HIPCHK(ctx, launch_copy_cols(it.AP, it.ld, it.fp32, s, it.op.n, AP_out, ctx->stream));
        }
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<double> dbg(size_t(dbg_size(s)));
    HIPCHK(ctx, hipMemcpy(dbg.data(), it.dbg, dbg.size() * sizeof(double), hipMemcpyDeviceToHost));
    DevState h;
    HIPCHK(ctx, hipMemcpy(&h, it.st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (alpha_tilde)
        std::memcpy(alpha_tilde, dbg.data() + dbg_atil(s), s * sizeof(double));
    if (G)
        std::memcpy(G, dbg.data() + dbg_G(s), size_t(s) * s * sizeof(double));
    if (ctil)
        std::memcpy(ctil, dbg.data() + dbg_ctil(s), s * sizeof(double));
    if (rnorm)
        *rnorm = dbg[size_t(dbg_rho(s))];
    if (h.status != SSTEP_OK)
        return fail(ctx, static_cast<sstep_status>(h.status), "step stopped");
    return SSTEP_OK;
}

sstep_status sstep_lanczos(sstep_ctx *ctx, const double *u, int32_t steps, double *alpha, double *beta,
                           double *ritz, int32_t *m_out)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (ctx->batch)
        return fail(ctx, SSTEP_E_ARG, "not available for a batched context");
    if (!u)
        return fail(ctx, SSTEP_E_ARG, "u must not be NULL");
    if (steps < 1 || steps > kMaxLanczos)
        return fail(ctx, SSTEP_E_ARG, "steps must be in [1, 64]");
    LzArgs &l = ctx->lz;
    const IterArgs &it = ctx->it;
    const size_t need = size_t(3) * size_t(it.ld) * sizeof(double);
    const size_t pbytes = size_t(it.ld) * it.s * (it.fp32 ? sizeof(float) : sizeof(double));
    if (pbytes >= need) {
        // the basis storage is scratch between solves
        double *P = static_cast<double *>(it.P);
        l.v[0] = P, l.v[1] = P + it.ld, l.v[2] = P + 2 * it.ld;
    } else {
        if (!ctx->lz_vecs)
            OKCHK(dalloc(ctx, &ctx->lz_vecs, size_t(3) * size_t(it.ld)));
        l.v[0] = ctx->lz_vecs, l.v[1] = ctx->lz_vecs + it.ld, l.v[2] = ctx->lz_vecs + 2 * it.ld;
    }
    HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    HIPCHK(ctx, hipMemsetAsync(l.ls, 0, sizeof(LzState), ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(l.ab, 0, size_t(3 * kMaxLanczos) * sizeof(double), ctx->stream));
    HIPCHK(ctx, launch_lanczos(l, it.op, u, steps, ctx->stream));
    std::vector<double> ab(size_t(3) * steps);
    LzState h;
    HIPCHK(ctx, hipMemcpyAsync(ab.data(), l.ab, ab.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(&h, l.ls, sizeof(LzState), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const int m = h.m;
    if (m_out)
        *m_out = m;
    for (int i = 0; i < steps; ++i) {
        if (alpha)
            alpha[i] = i < m ? ab[size_t(i)] : 0.0;
        if (beta)
            beta[i] = i < m ? ab[size_t(steps + i)] : 0.0;
        if (ritz)
            ritz[i] = i < m ? ab[size_t(2 * steps + i)] : 0.0;
    }
    if (m < 1)
        return fail(ctx, SSTEP_E_ARG, "the start vector has zero M-norm");
    return SSTEP_OK;
}

sstep_status sstep_set_bounds(sstep_ctx *ctx, double lambda_min, double lambda_max)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (ctx->batch)
        return fail(ctx, SSTEP_E_ARG, "a batched context takes its bounds at setup");
    if (!std::isfinite(lambda_min) || !std::isfinite(lambda_max) || lambda_min < 0.0 || !(lambda_max > lambda_min))
        return fail(ctx, SSTEP_E_ARG, "bounds must be finite with 0 <= lambda_min < lambda_max");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->it.theta = 2.0 / (lambda_max - lambda_min);
    ctx->it.sigma = (lambda_max + lambda_min) / 2.0;
    // the basis kernels take theta and sigma as arguments: capture the graph again
    if (ctx->gexec)
        HIPCHK(ctx, hipGraphExecDestroy(ctx->gexec));
    ctx->gexec = nullptr;
    if (ctx->graph)
        HIPCHK(ctx, hipGraphDestroy(ctx->graph));
    ctx->graph = nullptr;
    return capture_graph(ctx);
}

sstep_status sstep_lanczos_bounds(sstep_ctx *ctx, const double *u, int32_t steps, double margin,
                                  double *lambda_min, double *lambda_max)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (!(margin >= 0.0) || !(margin < 1.0))
        return fail(ctx, SSTEP_E_ARG, "margin must be in [0, 1)");
    std::vector<double> ritz(size_t(std::max(steps, 1)));
    int32_t m = 0;
    OKCHK(sstep_lanczos(ctx, u, steps, nullptr, nullptr, ritz.data(), &m));
    const double lo = std::max(0.0, (1.0 - margin) * ritz[0]);
    const double hi = (1.0 + margin) * ritz[size_t(m - 1)];
    if (!(hi > lo))
        return fail(ctx, SSTEP_E_BREAKDOWN, "Lanczos gave a degenerate interval (one Ritz value and no margin)");
    OKCHK(sstep_set_bounds(ctx, lo, hi));
    if (lambda_min)
        *lambda_min = lo;
    if (lambda_max)
        *lambda_max = hi;
    return SSTEP_OK;
}

sstep_status sstep_last_iteration(sstep_ctx *ctx, double *rnorm, double *delta, double *lnorm)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (ctx->batch)
        return fail(ctx, SSTEP_E_ARG, "not available for a batched context");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    DevState h;
    HIPCHK(ctx, hipMemcpy(&h, ctx->it.st, sizeof(DevState), hipMemcpyDeviceToHost));
    if (rnorm)
        *rnorm = h.rho;
    if (delta)
        *delta = h.delta;
    if (lnorm)
        *lnorm = h.lnorm;
    return SSTEP_OK;
}

sstep_status sstep_kernel_times(sstep_ctx *ctx, const double *b, double *x, int32_t reps, double *ms_out)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (!b || !x || !ms_out || reps < 1)
        return fail(ctx, SSTEP_E_ARG, "b, x, ms_out must not be NULL and reps >= 1");
    const IterArgs &it = ctx->it;
    hipStream_t s = ctx->stream;
    OKCHK(start_state(ctx, b, x, 0.5, 1));
    HIPCHK(ctx, enqueue_iteration(it, s));  // warm-up, leaves a valid basis and alpha behind
    for (int cls = 0; cls < SSTEP_KT_COUNT; ++cls) {
        HIPCHK(ctx, hipEventRecord(ctx->ev_t0, s));
        for (int r = 0; r < reps; ++r) {
            switch (cls) {
            case SSTEP_KT_RESIDUAL:
                HIPCHK(ctx, launch_residual(it, s, true));
                break;
            case SSTEP_KT_BASIS:
                HIPCHK(ctx, launch_basis_all(it, s));
                break;
            case SSTEP_KT_GRAM:
                HIPCHK(ctx, launch_gram(it, s));
                break;
            case SSTEP_KT_FGS:
                HIPCHK(ctx, launch_fgs(it, s));
                break;
            default:
                HIPCHK(ctx, launch_update(it, s));
            }
        }
        HIPCHK(ctx, hipEventRecord(ctx->ev_t1, s));
        HIPCHK(ctx, hipEventSynchronize(ctx->ev_t1));
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
        const int per = cls == SSTEP_KT_BASIS ? basis_kernel_count(it, nullptr) : 1;
        ms_out[cls] = per > 0 ? double(ms) / (double(reps) * per) : 0.0;
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    return SSTEP_OK;
}

static sstep_status batched_tiles(sstep_ctx *ctx, int64_t gchunk, int factor, bool upload)
{
    if (gchunk < kMinBatchChunk || gchunk % kPad != 0 || factor < 1)
        return fail(ctx, SSTEP_E_ARG, "batched tile schedule out of range");
    Batched &B = *ctx->batch;
    BatchArgs &a = B.ba;
    const int E = gram_entries(a.s + a.rec);
    std::vector<BTile> bt;
    std::vector<PTile> pt;
    std::vector<GTile> gt;
    int64_t rofs = 0, gofs = 0;
    for (int q = 0; q < a.nsys; ++q) {
        BSys &S = B.sys[size_t(q)];
        S.gchunk = gchunk;
        S.nch = int32_t((S.ld + gchunk - 1) / gchunk);
        S.rofs = rofs;
        S.gofs = gofs;
        rofs += int64_t(a.nrhs) * S.nch;
        gofs += int64_t(a.nrhs) * E * S.nch;
        for (int c = 0; c < S.nch; ++c) {
            bt.push_back({q, c});
            for (int r = 0; r < a.nrhs; ++r)
                gt.push_back({q, c, r, 0});
        }
        for (int64_t b = 0; b < (S.n + kBlock - 1) / kBlock; ++b)
            pt.push_back({q, int32_t(b)});
    }
    a.nbt = int(bt.size());
    a.npt = int(pt.size());
    a.ngt = int(gt.size());
    a.grid_bt = std::max(1, std::min(a.nbt, B.cus * factor));
    a.grid_pt = std::max(1, std::min(a.npt, B.cus * factor));
    a.grid_gt = std::max(1, std::min(a.ngt, B.cus * 2));
    if (upload) {
        HIPCHK(ctx, hipMemcpy(B.dsys, B.sys.data(), B.sys.size() * sizeof(BSys), hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(B.dbt, bt.data(), bt.size() * sizeof(BTile), hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(B.dpt, pt.data(), pt.size() * sizeof(PTile), hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(B.dgt, gt.data(), gt.size() * sizeof(GTile), hipMemcpyHostToDevice));
    }
    B.gchunk = gchunk;
    B.grid_factor = factor;
    return SSTEP_OK;
}

static hipError_t enqueue_batched_iteration(const BatchArgs &a, hipStream_t s)
{
    hipError_t e;
    // with two basis steps per launch the residual runs over the band table,
    // its ||r||^2 per band (beside the basis products in the moments kind)
    if ((e = a.bres ? launch_bres_f2(a, s) : launch_bresidual(a, s, true)) != hipSuccess)
        return e;
    int j = 0;
    if (a.f2)  // two steps per launch, an odd last step alone
        for (; j + 2 <= a.s; j += 2)
            if ((e = launch_bbasis_pair(a, j, s)) != hipSuccess)
                return e;
    for (; j < a.s; ++j)
        if ((e = launch_bbasis(a, j, s)) != hipSuccess)
            return e;
    if ((e = launch_bgram(a, s)) != hipSuccess)
        return e;
    if ((e = launch_bfgs(a, s)) != hipSuccess)
        return e;
    return launch_bupdate(a, s);
}

// Times the launches of an outer iteration that the tile schedule sets (the
// residual outside the moments kind, the single-step basis and the Gram
// reduction when they run, the update) for each tile size and persistent-grid factor; keeps the
// fastest pair, cached like the single-system Gram schedule.  The residual
// and the update run on zeroed scratch right-hand sides and iterates with
// zero step lengths (x stays zero), freed before returning; without device
// memory for them the default schedule stays.
static sstep_status tune_batched(sstep_ctx *ctx)
{
    Batched &B = *ctx->batch;
    BatchArgs &a = B.ba;
    std::ostringstream key;
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : B.n)
        h = (h ^ uint64_t(v)) * 1099511628211ull;
    key << kTuneSchema << " gfx950 batched s=" << a.s << " prec=" << (a.fp32 ? "fp32" : "fp64") << " nrhs=" << a.nrhs
        << " nsys=" << a.nsys << " faces=" << a.faces << " rec=" << a.rec << " mom=" << a.mom << " f2=" << a.f2
        << " timed=iteration sizes=" << std::hex << h;
    const std::string path = tune_cache_path();
    std::map<std::string, GramSchedule> cache;
    if (!path.empty()) {
        cache = read_tune_cache(path);
        auto f = cache.find(key.str());
        if (f != cache.end() && batched_entry_ok(f->second, kPad, kMinBatchChunk))
            return batched_tiles(ctx, f->second.slab, f->second.nbg, true);
    }
    struct Scratch {
        double *p = nullptr;
        ~Scratch()
        {
            if (p)
                (void)hipFree(p);
        }
    } xb;
    const size_t nb = size_t(B.total_n) * size_t(a.nrhs);
    if (hipMalloc(&xb.p, 2 * nb * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();  // no room for the scratch: keep the default schedule
        xb.p = nullptr;
        return SSTEP_OK;
    }
    HIPCHK(ctx, hipMemsetAsync(xb.p, 0, 2 * nb * sizeof(double), ctx->stream));
    {
        std::vector<DevState> ps(size_t(a.npairs));
        size_t off = 0;
        for (int q = 0; q < a.nsys; ++q)
            for (int r = 0; r < a.nrhs; ++r) {
                DevState &d = ps[size_t(q * a.nrhs + r)];
                std::memset(&d, 0, sizeof(DevState));
                d.x = xb.p + off;
                d.b = xb.p + nb + off;
                d.p0scale = 1.0;
                off += size_t(B.n[size_t(q)]);
            }
        HIPCHK(ctx, hipMemcpyAsync(a.pairs, ps.data(), sizeof(DevState) * ps.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    auto iteration = [&]() -> hipError_t {
        hipError_t e;
        if (!a.bres && (e = launch_bresidual(a, ctx->stream, true)) != hipSuccess)
            return e;
        if (!a.f2 && (e = launch_bbasis(a, 1 < a.s ? 1 : 0, ctx->stream)) != hipSuccess)
            return e;
        if ((e = launch_bgram(a, ctx->stream)) != hipSuccess)
            return e;
        return launch_bupdate(a, ctx->stream);
    };
    int64_t best_chunk = B.gchunk;
    int best_factor = B.grid_factor;
    double best = 1e30;
    for (int64_t gchunk : {int64_t(2048), int64_t(8192), int64_t(32768)}) {
        for (int factor : {2, 4, 8}) {
            OKCHK(batched_tiles(ctx, gchunk, factor, true));
            HIPCHK(ctx, iteration());
            HIPCHK(ctx, hipEventRecord(ctx->ev_t0, ctx->stream));
            for (int r = 0; r < 2; ++r)
                HIPCHK(ctx, iteration());
            HIPCHK(ctx, hipEventRecord(ctx->ev_t1, ctx->stream));
            HIPCHK(ctx, hipEventSynchronize(ctx->ev_t1));
            float ms = 0.f;
            HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
            if (ms < best) {
                best = ms;
                best_chunk = gchunk;
                best_factor = factor;
            }
        }
    }
    HIPCHK(ctx, hipMemsetAsync(a.pairs, 0, sizeof(DevState) * size_t(a.npairs), ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    OKCHK(batched_tiles(ctx, best_chunk, best_factor, true));
    if (!path.empty()) {
        cache[key.str()] = GramSchedule{best_factor, best_chunk, 1e3 * best / 2};
        write_tune_cache(path, cache);
    }
    return SSTEP_OK;
}

static sstep_status setup_batched_impl(sstep_ctx *ctx, int32_t nsys, const sstep_operator *A, int32_t nrhs,
                                       int32_t s, int32_t nu, const double *lmin, const double *lmax,
                                       const sstep_options *opt)
{
    if (opt)
        ctx->opt = *opt;
    else
        sstep_default_options(&ctx->opt);
    sstep_options &o = ctx->opt;
    if (nsys < 1 || !A || !lmin || !lmax)
        return fail(ctx, SSTEP_E_ARG, "nsys >= 1 operators and bounds are required");
    if (nrhs < 1 || nrhs > 64)
        return fail(ctx, SSTEP_E_ARG, "nrhs must be in [1, 64]");
    if (s < 1 || s > kMaxS)
        return fail(ctx, SSTEP_E_ARG, "s must be in [1, 32]");
    if (nu < 1)
        return fail(ctx, SSTEP_E_ARG, "nu must be >= 1");
    if (o.precision != SSTEP_FP64 && o.precision != SSTEP_FP32_IR)
        return fail(ctx, SSTEP_E_ARG, "unknown precision");
    if ((o.precond != 0 && o.precond != 1) || (o.p0_mode != 0 && o.p0_mode != 1) || o.max_outer < 0 ||
        (o.basis_steps != 0 && o.basis_steps != 1))
        return fail(ctx, SSTEP_E_ARG, "invalid options");
    if (o.basis != 0)
        return fail(ctx, SSTEP_E_UNSUPPORTED, "batched solves use the Chebyshev basis");
    if (o.gram < SSTEP_GRAM_AUTO || o.gram > SSTEP_GRAM_MOMENTS)
        return fail(ctx, SSTEP_E_ARG, "unknown gram kind");
    if (o.gram == SSTEP_GRAM_APPLY_OP)
        return fail(ctx, SSTEP_E_UNSUPPORTED, "batched solves take the moments, recurrence or stored-AP Gram kind");
    // the moments kind in batched solves: FP64, two basis steps per launch
    // with no single step left (even s), c = P^T r in the M inner product
    const bool mom_fit = o.precision == SSTEP_FP64 && s % 2 == 0 && s <= kRecMaxS && o.basis_steps == 0 &&
                         (o.p0_mode == 0 || o.precond == 0);
    if (o.gram == SSTEP_GRAM_MOMENTS && !mom_fit)
        return fail(ctx, SSTEP_E_UNSUPPORTED,
                    "the batched moments Gram kind needs FP64, an even s <= 31, two basis steps per launch and "
                    "p_0 = M^{-1} r or no preconditioner");
    if (o.gram == SSTEP_GRAM_RECURRENCE && s > kRecMaxS)
        return fail(ctx, SSTEP_E_UNSUPPORTED, "the recurrence Gram kind needs s <= 31");
    if (o.graph_chunk <= 0)
        o.graph_chunk = 4;
    for (int q = 0; q < nsys; ++q) {
        OKCHK(check_operator(ctx, &A[q]));
        if (A[q].kind != SSTEP_OP_STENCIL7)
            return fail(ctx, SSTEP_E_UNSUPPORTED, "batched solves take 7-point stencil operators");
        if ((A[q].kx != nullptr) != (A[0].kx != nullptr))
            return fail(ctx, SSTEP_E_ARG, "all batched systems must have face coefficients, or none");
        if (!std::isfinite(lmin[q]) || !std::isfinite(lmax[q]) || lmin[q] < 0.0 || !(lmax[q] > lmin[q]))
            return fail(ctx, SSTEP_E_ARG, "bounds must be finite with 0 <= lambda_min < lambda_max");
    }
    HIPCHK(ctx, hipGetDevice(&ctx->device));
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    ctx->user = static_cast<hipStream_t>(o.stream);
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_poll[0], hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_poll[1], hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreate(&ctx->ev_t0));
    HIPCHK(ctx, hipEventCreate(&ctx->ev_t1));
    ctx->batch = new (std::nothrow) Batched();
    if (!ctx->batch)
        return fail(ctx, SSTEP_E_NOMEM, "out of host memory");
    Batched &B = *ctx->batch;
    BatchArgs &a = B.ba;
    {
        int cus = 0;
        HIPCHK(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        B.cus = cus > 0 ? cus : 256;
        void *p = nullptr;
        HIPCHK(ctx, hipHostMalloc(&p, sizeof(DevState) * size_t(nsys) * nrhs, hipHostMallocDefault));
        B.pairs_host = static_cast<DevState *>(p);
        HIPCHK(ctx, hipHostMalloc(&p, sizeof(BGlob), hipHostMallocDefault));
        B.gl_host = static_cast<BGlob *>(p);
        HIPCHK(ctx, hipHostMalloc(&p, 8 * sizeof(int32_t), hipHostMallocDefault));
        ctx->poll_host = static_cast<int32_t *>(p);
    }
    a.nsys = nsys;
    a.nrhs = nrhs;
    a.npairs = nsys * nrhs;
    a.s = s;
    a.nu = nu;
    a.fp32 = o.precision == SSTEP_FP32_IR;
    a.p0_mode = o.p0_mode;
    a.precond = o.precond;
    a.faces = A[0].kx != nullptr;
    const bool jac_p0 = o.precond == 1 && o.p0_mode == 0;
    a.wdvec = jac_p0 && a.faces;
    a.cscale = (jac_p0 && !a.faces) ? 6.0 : 1.0;
    // recurrence kind by default for s <= 31: H = P^T M P with M the face
    // diagonals, or 6 I (constant Poisson with Jacobi), or I (no Jacobi)
    a.rec = o.gram == SSTEP_GRAM_RECURRENCE || o.gram == SSTEP_GRAM_MOMENTS ||
            (o.gram == SSTEP_GRAM_AUTO && s <= kRecMaxS);
    a.rec_wap = a.rec && o.precond == 1 && a.faces;
    a.rec_hscale = (a.rec && o.precond == 1 && !a.faces) ? 6.0 : 1.0;
    OKCHK(dalloc(ctx, &ctx->bad_flag, 1));
    HIPCHK(ctx, hipMemsetAsync(ctx->bad_flag, 0, sizeof(int), ctx->stream));
    const size_t w = a.fp32 ? sizeof(float) : sizeof(double);
    int64_t pofs = 0;
    for (int q = 0; q < nsys; ++q) {
        const sstep_operator &Aq = A[q];
        BSys S{};
        S.g.nx = Aq.nx;
        S.g.ny = Aq.ny;
        S.g.nz = Aq.nz;
        S.g.nxy = int64_t(Aq.nx) * Aq.ny;
        S.g.dx = make_fastdiv(uint32_t(Aq.nx));
        S.g.dy = make_fastdiv(uint32_t(Aq.ny));
        S.n = S.g.nxy * Aq.nz;
        S.ld = round_up(S.n, kPad);
        S.pofs = pofs;
        pofs += int64_t(s + a.rec) * nrhs * S.ld;  // p_0 .. p_{s-1} (and p_s with the recurrence kind)
        S.theta = 2.0 / (lmax[q] - lmin[q]);
        S.sigma = (lmax[q] + lmin[q]) / 2.0;
        S.inv_sqrt_n = 1.0 / std::sqrt(double(S.n));
        S.pair0 = q * nrhs;
        if (a.faces) {
            const int64_t nfx = faces_x(&Aq), nfy = faces_y(&Aq), nfz = faces_z(&Aq);
            double *k = nullptr, *dv = nullptr;
            OKCHK(dalloc(ctx, &k, size_t(nfx + nfy + nfz)));
            OKCHK(overwrite_device(ctx, k, Aq.kx, size_t(nfx), Aq.ptr_space));
            OKCHK(overwrite_device(ctx, k + nfx, Aq.ky, size_t(nfy), Aq.ptr_space));
            OKCHK(overwrite_device(ctx, k + nfx + nfy, Aq.kz, size_t(nfz), Aq.ptr_space));
            OKCHK(dalloc(ctx, &dv, size_t(S.ld)));
            HIPCHK(ctx, hipMemsetAsync(dv, 0, size_t(S.ld) * sizeof(double), ctx->stream));
            S.kx = k, S.ky = k + nfx, S.kz = k + nfx + nfy, S.dvec = dv;
            OpDev od;
            od.kind = kOpFaces;
            od.n = S.n;
            od.g = S.g;
            od.kx = S.kx, od.ky = S.ky, od.kz = S.kz;
            HIPCHK(ctx, launch_diag_from_faces(od, dv, ctx->bad_flag, ctx->stream));
            if (a.fp32) {
                float *k32 = nullptr, *dv32 = nullptr;
                OKCHK(dalloc(ctx, &k32, size_t(nfx + nfy + nfz)));
                OKCHK(dalloc(ctx, &dv32, size_t(S.ld)));
                HIPCHK(ctx, hipMemsetAsync(dv32, 0, size_t(S.ld) * sizeof(float), ctx->stream));
                HIPCHK(ctx, launch_to_fp32(k, k32, nfx + nfy + nfz, ctx->stream));
                HIPCHK(ctx, launch_to_fp32(dv, dv32, S.n, ctx->stream));
                S.kx32 = k32, S.ky32 = k32 + nfx, S.kz32 = k32 + nfx + nfy, S.dvec32 = dv32;
            }
            if (a.rec && o.basis_steps == 0) {  // Jacobi weights for the two-step basis
                double *di = nullptr;
                float *di32 = nullptr;
                OKCHK(dalloc(ctx, &di, size_t(S.ld)));
                if (a.fp32)
                    OKCHK(dalloc(ctx, &di32, size_t(S.ld)));
                S.dinv = di;
                S.dinv32 = di32;
                HIPCHK(ctx, launch_bdinv(S, o.precond, a.fp32, di, di32, ctx->stream));
            }
        }
        B.sys.push_back(S);
        B.n.push_back(S.n);
        B.total_n += S.n;
    }
    {
        int hbad = 0;
        HIPCHK(ctx, hipMemcpyAsync(&hbad, ctx->bad_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (hbad)
            return fail(ctx, SSTEP_E_ARG, "a face operator has a non-positive or non-finite diagonal");
    }
    {
        char *P = nullptr, *AP = nullptr;
        OKCHK(dalloc(ctx, &P, size_t(pofs) * w));
        HIPCHK(ctx, hipMemsetAsync(P, 0, size_t(pofs) * w, ctx->stream));
        if (!a.rec) {
            OKCHK(dalloc(ctx, &AP, size_t(pofs) * w));
            HIPCHK(ctx, hipMemsetAsync(AP, 0, size_t(pofs) * w, ctx->stream));
        }
        a.P = P;
        a.AP = AP;
    }
    // tables and partials sized for the smallest tile (kMinBatchChunk rows)
    int64_t max_nch = 0, max_pt = 0;
    for (const BSys &S : B.sys) {
        max_nch += (S.ld + kMinBatchChunk - 1) / kMinBatchChunk;
        max_pt += (S.n + kBlock - 1) / kBlock;
    }
    OKCHK(dalloc(ctx, &B.dsys, size_t(nsys)));
    OKCHK(dalloc(ctx, &B.dbt, size_t(max_nch)));
    OKCHK(dalloc(ctx, &B.dpt, size_t(max_pt)));
    OKCHK(dalloc(ctx, &B.dgt, size_t(max_nch) * nrhs));
    OKCHK(dalloc(ctx, &a.rpart, size_t(max_nch) * nrhs));
    OKCHK(dalloc(ctx, &a.gpart, size_t(max_nch) * nrhs * gram_entries(s + a.rec)));
    OKCHK(dalloc(ctx, &a.pairs, size_t(a.npairs)));
    OKCHK(dalloc(ctx, &a.gl, 1));
    OKCHK(dalloc(ctx, &a.dbg, size_t(a.npairs) * dbg_size(s)));
    HIPCHK(ctx, hipMemsetAsync(a.pairs, 0, sizeof(DevState) * size_t(a.npairs), ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(a.gl, 0, sizeof(BGlob), ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    a.sys = B.dsys;
    a.btiles = B.dbt;
    a.ptiles = B.dpt;
    a.gtiles = B.dgt;
    if (a.rec && o.basis_steps == 0) {
        std::vector<BandGrid> grids;
        for (const BSys &S : B.sys)
            grids.push_back({S.g.nx, S.g.ny, S.g.nz});
        const std::vector<BF2Tile> f2 = bf2_bands(grids, w, a.faces, kBf2Threads, a.nrhs, B.cus);
        std::vector<BF2Tile> f2s;
        if (!f2.empty()) {
            OKCHK(dalloc(ctx, &B.df2, f2.size()));
            HIPCHK(ctx, hipMemcpy(B.df2, f2.data(), f2.size() * sizeof(BF2Tile), hipMemcpyHostToDevice));
            a.f2 = 1;
            a.nf2 = int(f2.size());
            a.f2tiles = B.df2;
            for (const BF2Tile &t : f2)
                ++B.sys[size_t(t.q)].nbl;
            const std::vector<uint32_t> map = bf2_dispatch(f2, grids, a.nrhs, true, int(kNumXcd));
            OKCHK(dalloc(ctx, &B.dmap, map.size()));
            HIPCHK(ctx, hipMemcpy(B.dmap, map.data(), map.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
            a.f2map = B.dmap;
            a.f2grid = uint32_t(map.size());
            f2s = bf2_bands_kz(grids, w, a.faces, kBf2Threads, kBf2MinPlanes);
            if (f2s.size() > f2.size()) {
                OKCHK(dalloc(ctx, &B.df2_tail, f2s.size()));
                HIPCHK(ctx, hipMemcpy(B.df2_tail, f2s.data(), f2s.size() * sizeof(BF2Tile), hipMemcpyHostToDevice));
                B.nf2_tail = int(f2s.size());
                const std::vector<uint32_t> mt = bf2_dispatch(f2s, grids, a.nrhs, false, int(kNumXcd));
                OKCHK(dalloc(ctx, &B.dmap_tail, mt.size()));
                HIPCHK(ctx, hipMemcpy(B.dmap_tail, mt.data(), mt.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
                B.grid_tail = uint32_t(mt.size());
            } else {
                f2s.clear();
            }
        }
        if (a.f2) {
            a.mom = mom_fit && (o.gram == SSTEP_GRAM_MOMENTS || o.gram == SSTEP_GRAM_AUTO);
            // band entries are ordered by system: each system's range of them,
            // and its partial slots per right-hand side, one partial per band
            // (the moments kind: the 2s + 1 products and ||r||^2; the
            // recurrence kind: ||r||^2); both band tables share one buffer
            a.bres = 1;
            a.bres_slots = a.mom ? bmom_slots(s) : 1;
            a.bres_slot = a.mom ? 2 * s + 1 : 0;
            auto layout = [&](const std::vector<BF2Tile> &tab, std::vector<Batched::BandLayout> &out) {
                int64_t mofs = 0;
                size_t e = 0;
                for (int q = 0; q < a.nsys; ++q) {
                    Batched::BandLayout tb{mofs, int32_t(e), 0};
                    while (e < tab.size() && tab[e].q == q)
                        ++e;
                    tb.nf2q = int32_t(e - size_t(tb.f2first));
                    mofs += int64_t(a.nrhs) * a.bres_slots * tb.nf2q;
                    out.push_back(tb);
                }
                return mofs;
            };
            std::vector<Batched::BandLayout> whole;
            int64_t mofs = layout(f2, whole);
            for (int q = 0; q < a.nsys; ++q) {
                BSys &S = B.sys[size_t(q)];
                S.mofs = whole[size_t(q)].mofs;
                S.f2first = whole[size_t(q)].f2first;
                S.nf2q = whole[size_t(q)].nf2q;
            }
            if (!f2s.empty())
                mofs = std::max(mofs, layout(f2s, B.tail_bands));
            OKCHK(dalloc(ctx, &a.mpart, size_t(mofs)));
        }
    }
    if (o.gram == SSTEP_GRAM_MOMENTS && !a.mom)
        return fail(ctx, SSTEP_E_UNSUPPORTED, "the batched moments Gram kind needs every system to fit the two-step "
                                              "basis (rows of at most 341 points)");
    // a non-zero npairs with ndone = 0 keeps the kernels active while tuning
    BGlob g0{0, a.npairs};
    HIPCHK(ctx, hipMemcpy(a.gl, &g0, sizeof(BGlob), hipMemcpyHostToDevice));
    OKCHK(batched_tiles(ctx, kMinBatchChunk, 4, true));  // the tuner's usual pick on large batches
    if (o.autotune && B.total_n >= (int64_t(1) << 20))
        OKCHK(tune_batched(ctx));
    // graph of graph_chunk outer iterations over all pairs
    ctx->chunk = o.graph_chunk;
    HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int c = 0; c < ctx->chunk && e == hipSuccess; ++c)
        e = enqueue_batched_iteration(a, ctx->stream);
    hipGraph_t gph = nullptr;
    hipError_t e2 = hipStreamEndCapture(ctx->stream, &gph);
    if (e != hipSuccess)
        return hip_fail(ctx, "kernel launch during graph capture", e);
    if (e2 != hipSuccess)
        return hip_fail(ctx, "hipStreamEndCapture", e2);
    ctx->graph = gph;
    HIPCHK(ctx, hipGraphInstantiate(&ctx->gexec, gph, nullptr, nullptr, 0));
    if (B.nf2_tail > 0) {
        // the same iteration over the short-range band table; every other
        // field of its systems (the tile schedule just chosen) is the same
        std::vector<BSys> st = B.sys;
        if (a.bres)
            for (int q = 0; q < a.nsys; ++q) {
                st[size_t(q)].mofs = B.tail_bands[size_t(q)].mofs;
                st[size_t(q)].f2first = B.tail_bands[size_t(q)].f2first;
                st[size_t(q)].nf2q = B.tail_bands[size_t(q)].nf2q;
            }
        OKCHK(dalloc(ctx, &B.dsys_tail, st.size()));
        HIPCHK(ctx, hipMemcpy(B.dsys_tail, st.data(), st.size() * sizeof(BSys), hipMemcpyHostToDevice));
        BatchArgs at = a;
        at.sys = B.dsys_tail;
        at.f2tiles = B.df2_tail;
        at.nf2 = B.nf2_tail;
        at.f2map = B.dmap_tail;
        at.f2grid = B.grid_tail;
        HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        for (int c = 0; c < ctx->chunk && e == hipSuccess; ++c)
            e = enqueue_batched_iteration(at, ctx->stream);
        hipGraph_t gt = nullptr;
        e2 = hipStreamEndCapture(ctx->stream, &gt);
        if (e != hipSuccess)
            return hip_fail(ctx, "kernel launch during graph capture", e);
        if (e2 != hipSuccess)
            return hip_fail(ctx, "hipStreamEndCapture", e2);
        B.graph_tail = gt;
        HIPCHK(ctx, hipGraphInstantiate(&B.gexec_tail, gt, nullptr, nullptr, 0));
    }
    return SSTEP_OK;
}

sstep_status sstep_setup_batched(sstep_ctx **out, int32_t nsys, const sstep_operator *A, int32_t nrhs, int32_t s,
                                 int32_t nu, const double *lmin, const double *lmax, const sstep_options *opt)
{
    if (!out)
        return fail(nullptr, SSTEP_E_ARG, "out is NULL");
    *out = nullptr;
    sstep_ctx *ctx = new (std::nothrow) sstep_ctx();
    if (!ctx)
        return fail(nullptr, SSTEP_E_NOMEM, "out of host memory");
    const sstep_status st = setup_batched_impl(ctx, nsys, A, nrhs, s, nu, lmin, lmax, opt);
    if (st != SSTEP_OK) {
        g_setup_error = ctx->err;
        sstep_destroy(ctx);
        return st;
    }
    *out = ctx;
    return SSTEP_OK;
}

sstep_status sstep_solve_batched(sstep_ctx *ctx, const double *const *b, double *const *x, double tol,
                                 sstep_stats *st)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (!ctx->batch)
        return fail(ctx, SSTEP_E_ARG, "this context was made by sstep_setup: use sstep_solve");
    Batched &B = *ctx->batch;
    BatchArgs &a = B.ba;
    if (!b || !x)
        return fail(ctx, SSTEP_E_ARG, "b and x must not be NULL");
    if (!(tol > 0.0) || !(tol < 1.0))
        return fail(ctx, SSTEP_E_ARG, "tol must be in (0, 1)");
    for (int q = 0; q < a.nsys; ++q)
        if (!b[q] || !x[q])
            return fail(ctx, SSTEP_E_ARG, "b[q] and x[q] must not be NULL");
    for (int q = 0; q < a.nsys; ++q)
        for (int r = 0; r < a.nrhs; ++r) {
            DevState &h = B.pairs_host[q * a.nrhs + r];
            std::memset(&h, 0, sizeof(DevState));
            h.b = b[q] + int64_t(r) * B.n[size_t(q)];
            h.x = x[q] + int64_t(r) * B.n[size_t(q)];
            h.tol = tol;
            h.p0scale = 1.0;
            h.first = 1;
            h.max_outer = ctx->opt.max_outer;
        }
    *B.gl_host = BGlob{0, a.npairs};
    HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    HIPCHK(ctx, hipMemcpyAsync(a.pairs, B.pairs_host, sizeof(DevState) * size_t(a.npairs), hipMemcpyHostToDevice,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(a.gl, B.gl_host, sizeof(BGlob), hipMemcpyHostToDevice, ctx->stream));
    if (a.fp32) {
        HIPCHK(ctx, launch_bresidual(a, ctx->stream, false));
        HIPCHK(ctx, launch_bp0scale(a, ctx->stream));
    }
    const int max_replays = (ctx->opt.max_outer + 1 + ctx->chunk - 1) / ctx->chunk + 1;
    int launched = 0, checked = 0;
    // the short-range graph once the blocks the whole batch's band table
    // would still start (as of the last replay read back) fall below
    // kBf2BlocksPerCu per CU; the choice depends only on device results, so
    // a solve replays the same graphs every time
    const int64_t tail_below = int64_t(kBf2BlocksPerCu) * B.cus;
    int64_t blocks_left = int64_t(a.nf2) * a.nrhs;
    B.tail_replays = 0;
    auto enqueue = [&]() -> hipError_t {
        hipGraphExec_t gx = ctx->gexec;
        if (B.gexec_tail && blocks_left < tail_below) {
            gx = B.gexec_tail;
            ++B.tail_replays;
        }
        hipError_t e = hipGraphLaunch(gx, ctx->stream);
        if (e != hipSuccess)
            return e;
        int32_t *slot = ctx->poll_host + 4 * (launched % 2);
        e = hipMemcpyAsync(slot, a.gl, sizeof(BGlob), hipMemcpyDeviceToHost, ctx->stream);
        if (e != hipSuccess)
            return e;
        e = hipEventRecord(ctx->ev_poll[launched % 2], ctx->stream);
        ++launched;
        return e;
    };
    HIPCHK(ctx, enqueue());
    for (;;) {
        if (launched < max_replays)
            HIPCHK(ctx, enqueue());
        HIPCHK(ctx, hipEventSynchronize(ctx->ev_poll[checked % 2]));
        const int32_t ndone = ctx->poll_host[4 * (checked % 2)];
        blocks_left = int64_t(a.nf2) * a.nrhs - ctx->poll_host[4 * (checked % 2) + 2];
        ++checked;
        if (ndone >= a.npairs)
            break;
        if (checked >= launched) {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            return fail(ctx, SSTEP_E_HIP, "batched solve did not stop within the replay bound");
        }
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(B.pairs_host, a.pairs, sizeof(DevState) * size_t(a.npairs), hipMemcpyDeviceToHost));
    sstep_status first_bad = SSTEP_OK;
    for (int p = 0; p < a.npairs; ++p) {
        const DevState &h = B.pairs_host[p];
        if (st) {
            st[p].outer_iters = h.iter;
            st[p].status = h.status;
            st[p].rel_res = h.relres;
            st[p].res0 = h.rho0;
        }
        if (first_bad == SSTEP_OK && h.status != SSTEP_OK)
            first_bad = static_cast<sstep_status>(h.status);
    }
    if (first_bad != SSTEP_OK)
        return fail(ctx, first_bad, std::string("a batched pair stopped with ") + sstep_status_string(first_bad));
    return SSTEP_OK;
}


// ---------------------------------------------------------------------------
// Two-level coarse solve (Sec. 6; Sec. 8).
// ---------------------------------------------------------------------------
static sstep_status coarse_setup_impl(sstep_ctx *ctx, const sstep_operator *Af, int32_t formed,
                                      const sstep_options *opt)
{
    if (opt)
        ctx->opt = *opt;
    else
        sstep_default_options(&ctx->opt);
    OKCHK(check_operator(ctx, Af));
    if (Af->kind != SSTEP_OP_STENCIL7)
        return fail(ctx, SSTEP_E_UNSUPPORTED, "the coarse solve takes a 7-point fine-grid operator");
    if (Af->nx % 2 == 0 || Af->ny % 2 == 0 || Af->nz % 2 == 0 || Af->nx < 3 || Af->ny < 3 || Af->nz < 3)
        return fail(ctx, SSTEP_E_ARG, "fine grid sides must be odd, 2 nc + 1 with nc >= 1");
    if (formed != 0 && formed != 1)
        return fail(ctx, SSTEP_E_ARG, "formed must be 0 (streamed) or 1 (A_c formed)");
    HIPCHK(ctx, hipGetDevice(&ctx->device));
    HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    ctx->user = static_cast<hipStream_t>(ctx->opt.stream);
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    ctx->coarse = new (std::nothrow) CoarseArgs();
    if (!ctx->coarse)
        return fail(ctx, SSTEP_E_NOMEM, "out of host memory");
    CoarseArgs &c = *ctx->coarse;
    c.nfx = Af->nx, c.nfy = Af->ny, c.nfz = Af->nz;
    c.ncx = (Af->nx - 1) / 2, c.ncy = (Af->ny - 1) / 2, c.ncz = (Af->nz - 1) / 2;
    const int64_t nc = int64_t(c.ncx) * c.ncy * c.ncz;
    const int64_t nf = int64_t(c.nfx) * c.nfy * c.nfz;
    int64_t bytes = 0;
    if (Af->kx) {
        const int64_t nfx = faces_x(Af), nfy = faces_y(Af), nfz = faces_z(Af);
        double *k = nullptr;
        OKCHK(dalloc(ctx, &k, size_t(nfx + nfy + nfz)));
        OKCHK(overwrite_device(ctx, k, Af->kx, size_t(nfx), Af->ptr_space));
        OKCHK(overwrite_device(ctx, k + nfx, Af->ky, size_t(nfy), Af->ptr_space));
        OKCHK(overwrite_device(ctx, k + nfx + nfy, Af->kz, size_t(nfz), Af->ptr_space));
        c.kx = k, c.ky = k + nfx, c.kz = k + nfx + nfy;
    }
    // wavefronts t = I + 2J + 4K, unknowns ascending within each
    c.nwf = c.ncx + 2 * c.ncy + 4 * c.ncz - 6;
    std::vector<int32_t> count(static_cast<size_t>(c.nwf) + 1, 0), order(static_cast<size_t>(nc), 0),
        wf(static_cast<size_t>(c.nwf) + 1, 0);
    for (int64_t j = 0; j < nc; ++j) {
        const int I = int(j % c.ncx), J = int((j / c.ncx) % c.ncy), K = int(j / (int64_t(c.ncx) * c.ncy));
        ++count[size_t(I + 2 * J + 4 * K) + 1];
    }
    for (int t = 0; t < c.nwf; ++t)
        wf[size_t(t) + 1] = wf[size_t(t)] + count[size_t(t) + 1];
    std::vector<int32_t> fill(wf.begin(), wf.end() - 1);
    for (int64_t j = 0; j < nc; ++j) {
        const int I = int(j % c.ncx), J = int((j / c.ncx) % c.ncy), K = int(j / (int64_t(c.ncx) * c.ncy));
        order[size_t(fill[size_t(I + 2 * J + 4 * K)]++)] = int32_t(j);
    }
    int32_t *dorder = nullptr, *dwf = nullptr;
    OKCHK(to_device(ctx, &dorder, order.data(), order.size(), 0));
    OKCHK(to_device(ctx, &dwf, wf.data(), wf.size(), 0));
    c.order = dorder, c.wf = dwf;
    bytes += int64_t(order.size() + wf.size()) * int64_t(sizeof(int32_t));
    OKCHK(dalloc(ctx, &c.diag, size_t(nc)));
    bytes += nc * int64_t(sizeof(double));
    if (formed) {
        OKCHK(dalloc(ctx, &c.rows, size_t(27 * nc)));
        bytes += 27 * nc * int64_t(sizeof(double));
    } else {
        OKCHK(dalloc(ctx, &c.v, size_t(nf)));
        bytes += nf * int64_t(sizeof(double));
    }
    ctx->coarse_bytes = bytes;
    HIPCHK(ctx, launch_coarse_prepare(c, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SSTEP_OK;
}

sstep_status sstep_coarse_setup(sstep_ctx **out, const sstep_operator *Af, int32_t formed, const sstep_options *opt)
{
    if (!out)
        return fail(nullptr, SSTEP_E_ARG, "out is NULL");
    *out = nullptr;
    sstep_ctx *ctx = new (std::nothrow) sstep_ctx();
    if (!ctx)
        return fail(nullptr, SSTEP_E_NOMEM, "out of host memory");
    const sstep_status st = coarse_setup_impl(ctx, Af, formed, opt);
    if (st != SSTEP_OK) {
        g_setup_error = ctx->err;
        sstep_destroy(ctx);
        return st;
    }
    *out = ctx;
    return SSTEP_OK;
}

sstep_status sstep_coarse_fgs(sstep_ctx *ctx, const double *f, double *u, int32_t nu)
{
    if (!ctx)
        return SSTEP_E_ARG;
    if (!ctx->coarse)
        return fail(ctx, SSTEP_E_ARG, "this context was not made by sstep_coarse_setup");
    if (!f || !u || f == u)
        return fail(ctx, SSTEP_E_ARG, "f and u must be distinct non-NULL device pointers");
    if (nu < 0)
        return fail(ctx, SSTEP_E_ARG, "nu must be >= 0");
    HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    HIPCHK(ctx, launch_coarse_fgs(*ctx->coarse, f, u, nu, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SSTEP_OK;
}

sstep_status sstep_coarse_info(const sstep_ctx *ctx, int64_t *n_coarse, int64_t *workspace_bytes)
{
    if (!ctx || !ctx->coarse)
        return SSTEP_E_ARG;
    const CoarseArgs &c = *ctx->coarse;
    if (n_coarse)
        *n_coarse = int64_t(c.ncx) * c.ncy * c.ncz;
    if (workspace_bytes)
        *workspace_bytes = ctx->coarse_bytes;
    return SSTEP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace lives in a static device array of
// kNoallocBytes per GPU, located once per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoallocBytes = size_t(64) << 20;
constexpr int kNoallocMaxDevices = 64;

__device__ __align__(256) char scratch[kNoallocBytes];

std::mutex g_noalloc_mutex;
void *g_noalloc_ptr[kNoallocMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on the first call on
// the device, with the device current).
sstep_status noalloc_scratch(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(nullptr, "hipGetDevice", e);
    if (dev < 0 || dev >= kNoallocMaxDevices)
        return fail(nullptr, SSTEP_E_UNSUPPORTED, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(nullptr, "hipGetSymbolAddress(scratch)", e != hipSuccess ? e : hipErrorInvalidSymbol);
        g_noalloc_ptr[dev] = p;
    }
    *out = static_cast<char *>(g_noalloc_ptr[dev]);
    return SSTEP_OK;
}

// Byte offsets of the workspace regions in the scratch array, 256-aligned.
struct NoallocLayout {
    size_t st, rpart, gpart, gsum, dbg, hist, bad, dvec, invd, P, AP, total;
};

NoallocLayout noalloc_layout(const IterArgs &it)
{
    NoallocLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t E = size_t(gram_entries(it.s + it.gram_rec));
    const size_t ld = size_t(it.ld);
    L.st = take(sizeof(DevState));
    L.rpart = take(size_t(it.nbr) * sizeof(double));
    L.gpart = take(E * size_t(it.nbg) * sizeof(double));
    L.gsum = take((E + 1) * sizeof(double));
    L.dbg = take(size_t(dbg_size(it.s)) * sizeof(double));
    L.hist = take(3 * sizeof(double));
    L.bad = take(sizeof(int));
    const bool faces = it.op.kind == kOpFaces, csr = it.op.kind == kOpCsr;
    L.dvec = take(faces || csr ? ld * sizeof(double) : 0);
    L.invd = take(csr ? ld * sizeof(double) : 0);
    L.P = take(ld * size_t(it.s + it.gram_rec) * sizeof(double));
    L.AP = take(it.gram_op || it.gram_rec ? 0 : ld * size_t(it.s) * sizeof(double));
    L.total = o;
    return L;
}

sstep_status noalloc_impl(const sstep_operator *A, int32_t s, int32_t nu, double lmin, double lmax,
                          const sstep_options *opt, const double *b, double *x, double tol, sstep_stats *stats)
{
    sstep_options o;
    if (opt)
        o = *opt;
    else
        sstep_default_options(&o);
    if (s < 1 || s > kMaxS)
        return fail(nullptr, SSTEP_E_ARG, "s must be in [1, 32]");
    if (nu < 1)
        return fail(nullptr, SSTEP_E_ARG, "nu must be >= 1");
    if (!std::isfinite(lmin) || !std::isfinite(lmax) || lmin < 0.0 || !(lmax > lmin))
        return fail(nullptr, SSTEP_E_ARG, "bounds must be finite with 0 <= lambda_min < lambda_max");
    if (o.precision != SSTEP_FP64)
        return fail(nullptr, SSTEP_E_UNSUPPORTED, "the allocation-free solve runs in FP64 only");
    if ((o.precond != 0 && o.precond != 1) || (o.p0_mode != 0 && o.p0_mode != 1) || o.max_outer < 0 ||
        (o.basis != 0 && o.basis != 1) || (o.basis_steps != 0 && o.basis_steps != 1))
        return fail(nullptr, SSTEP_E_ARG, "invalid options");
    if (o.gram < SSTEP_GRAM_AUTO || o.gram > SSTEP_GRAM_MOMENTS)
        return fail(nullptr, SSTEP_E_ARG, "unknown gram kind");
    if (!b || !x)
        return fail(nullptr, SSTEP_E_ARG, "b and x must not be NULL");
    if (!(tol > 0.0) || !(tol < 1.0))
        return fail(nullptr, SSTEP_E_ARG, "tol must be in (0, 1)");
    OKCHK(check_operator(nullptr, A));
    const bool has_arrays = A->kind == SSTEP_OP_CSR || (A->kind == SSTEP_OP_STENCIL7 && A->kx);
    if (has_arrays && A->ptr_space != 1)
        return fail(nullptr, SSTEP_E_ARG, "the allocation-free solve takes operator arrays in device memory");
    int gram_kind = SSTEP_GRAM_STORED_AP;
    OKCHK(choose_gram_kind(nullptr, A, s, o, &gram_kind, false));

    IterArgs it;
    OpDev &op = it.op;
    op.precond = o.precond;
    if (A->kind == SSTEP_OP_CSR) {
        op.kind = kOpCsr;
        op.n = A->n;
        op.nnz = A->nnz;
        op.rp = A->row_ptr;
        op.ci = A->col_idx;
        op.val = A->val;
    } else {
        op.kind = A->kind == SSTEP_OP_STENCIL27 ? kOpPoisson27 : (A->kx ? kOpFaces : kOpPoisson);
        op.n = int64_t(A->nx) * A->ny * A->nz;
        op.g.nx = A->nx;
        op.g.ny = A->ny;
        op.g.nz = A->nz;
        op.g.nxy = int64_t(A->nx) * A->ny;
        op.g.dx = make_fastdiv(uint32_t(A->nx));
        op.g.dy = make_fastdiv(uint32_t(A->ny));
        op.kx = A->kx;
        op.ky = A->ky;
        op.kz = A->kz;
    }
    it.fp32 = 0;
    it.p0_mode = o.p0_mode;
    it.monomial = o.basis;
    it.one_step = o.basis_steps;
    it.s = s;
    it.nu = nu;
    it.theta = 2.0 / (lmax - lmin);
    it.sigma = (lmax + lmin) / 2.0;
    it.ld = round_up(op.n, kPad);
    const bool jac_p0 = o.precond == 1 && o.p0_mode == 0;
    const bool const_diag = op.kind == kOpPoisson || op.kind == kOpPoisson27;
    set_gram_kind(it, gram_kind, o.precond, const_diag);
    it.wdvec = jac_p0 && !const_diag;
    it.cscale = (jac_p0 && const_diag) ? (op.kind == kOpPoisson27 ? 26.0 : 6.0) : 1.0;
    it.inv_sqrt_n = 1.0 / std::sqrt(double(op.n));
    it.hist_cap = 0;
    set_residual_schedule(it);
    set_gram_schedule(it, default_gram_schedule(it));  // the context path's schedule without autotuning
    const NoallocLayout L = noalloc_layout(it);
    if (L.total > kNoallocBytes)
        return fail(nullptr, SSTEP_E_ARG,
                    "problem too large for the allocation-free solve: needs " + std::to_string(L.total) +
                        " bytes of workspace, the static scratch holds " + std::to_string(kNoallocBytes));

    char *base = nullptr;
    OKCHK(noalloc_scratch(&base));
    it.st = reinterpret_cast<DevState *>(base + L.st);
    it.rpart = reinterpret_cast<double *>(base + L.rpart);
    it.gpart = reinterpret_cast<double *>(base + L.gpart);
    it.gsum = reinterpret_cast<double *>(base + L.gsum);
    it.dbg = reinterpret_cast<double *>(base + L.dbg);
    it.hist = reinterpret_cast<double *>(base + L.hist);
    int *bad = reinterpret_cast<int *>(base + L.bad);
    it.P = base + L.P;
    it.AP = it.gram_op || it.gram_rec ? nullptr : base + L.AP;

    hipStream_t st = static_cast<hipStream_t>(o.stream);
    // the array keeps the previous call's contents: clear everything that is
    // read before it is written (padding rows of P, AP and the diagonal)
    HIPCHK(nullptr, launch_fill_zero(base, L.total, st));
    if (op.kind == kOpCsr) {
        HIPCHK(nullptr, launch_check_csr_rows(op.rp, op.n, op.nnz, bad, st));
        int hbad = 0;
        HIPCHK(nullptr, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(nullptr, hipStreamSynchronize(st));
        if (!hbad) {
            HIPCHK(nullptr, launch_check_csr_cols(op.rp, op.ci, op.n, bad, st));
            HIPCHK(nullptr, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(nullptr, hipStreamSynchronize(st));
        }
        if (hbad)
            return fail(nullptr, SSTEP_E_ARG, "malformed CSR pattern");
        double *dvec = reinterpret_cast<double *>(base + L.dvec), *invd = reinterpret_cast<double *>(base + L.invd);
        op.dvec = dvec;
        op.invd = invd;
        HIPCHK(nullptr, launch_diag_from_csr(op, dvec, bad, st));
        HIPCHK(nullptr, launch_invert(dvec, invd, op.n, op.precond, st));
    } else if (op.kind == kOpFaces) {
        double *dvec = reinterpret_cast<double *>(base + L.dvec);
        op.dvec = dvec;
        HIPCHK(nullptr, launch_diag_from_faces(op, dvec, bad, st));
    }
    if (op.kind == kOpCsr || op.kind == kOpFaces) {
        int hbad = 0;
        HIPCHK(nullptr, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(nullptr, hipStreamSynchronize(st));
        if (hbad)
            return fail(nullptr, SSTEP_E_ARG, "matrix has a missing, non-positive or non-finite diagonal entry");
    }
    HIPCHK(nullptr, launch_init_state(it.st, b, x, tol, o.max_outer, st));

    // outer iterations in chunks of graph_chunk launches, then a look at the
    // device's stop flag (every kernel returns at once after the stop)
    const int chunk = o.graph_chunk > 0 ? o.graph_chunk : 4;
    const int64_t max_chunks = (int64_t(o.max_outer) + 1 + chunk - 1) / chunk + 1;
    int32_t done = 0;
    for (int64_t c = 0; c < max_chunks && !done; ++c) {
        for (int q = 0; q < chunk; ++q)
            HIPCHK(nullptr, enqueue_iteration(it, st));
        HIPCHK(nullptr, hipMemcpyAsync(&done, &it.st->done, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(nullptr, hipStreamSynchronize(st));
    }
    DevState h;
    HIPCHK(nullptr, hipMemcpyAsync(&h, it.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
    HIPCHK(nullptr, hipStreamSynchronize(st));
    if (!h.done)
        return fail(nullptr, SSTEP_E_HIP, "solve did not stop within the launch bound");
    if (stats) {
        stats->outer_iters = h.iter;
        stats->status = h.status;
        stats->rel_res = h.relres;
        stats->res0 = h.rho0;
    }
    if (h.status != SSTEP_OK)
        return fail(nullptr, static_cast<sstep_status>(h.status),
                    std::string("solve stopped: ") + sstep_status_string(static_cast<sstep_status>(h.status)));
    return SSTEP_OK;
}

}  // namespace

extern "C" sstep_status sstep_solve_noalloc(const sstep_operator *A, int32_t s, int32_t nu, double lambda_min,
                                            double lambda_max, const sstep_options *opt, const double *b, double *x,
                                            double tol, sstep_stats *st)
{
    return noalloc_impl(A, s, nu, lambda_min, lambda_max, opt, b, x, tol, st);
}
