// Batched outer iteration over many stencil systems and right-hand sides:
// residual + basis start, basis step, update and the FP32 scaling pre-pass.
// Each kernel is persistent: a fixed grid walks a table of tiles, and the work
// of pairs whose solve has stopped is skipped.  The Gram and FGS kernels of
// the batched iteration live with the single-system ones (batched_impl.h).
#include "basis_f2.h"
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

// Jacobi weights of one face-coefficient system, 1 / diag (1 without Jacobi),
// formed by the expression the single-step kernel uses, in T from the faces
// in T, for the two-step kernel to read.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bdinv(BSys S, int precond, T *__restrict__ out)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= S.n)
        return;
    const T *kx, *ky, *kz;
    if constexpr (sizeof(T) == 8)
        kx = reinterpret_cast<const T *>(S.kx), ky = reinterpret_cast<const T *>(S.ky),
        kz = reinterpret_cast<const T *>(S.kz);
    else
        kx = reinterpret_cast<const T *>(S.kx32), ky = reinterpret_cast<const T *>(S.ky32),
        kz = reinterpret_cast<const T *>(S.kz32);
    PointStencil<T, true> op;
    op.init(S, c, precond, kx, ky, kz);
    out[c] = op.dinv;
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

// Two basis steps for one pair per block (Sec. 2, Definition, taken twice):
//   q       = p_{j+1} from p_j and p_{j-1} (from p_0 alone when j = 0)
//   p_{j+2} = 2 theta (M^{-1} A q - sigma q) - p_j
// with every value formed by the operations, in the order, of k_bbasis, so
// the pair equals two single steps bit for bit.  A block owns a band of whole
// grid rows [y0, y1) of one system and a range of planes [k0, k1), and forms
// q on the band and on the row below and the row above it (when the grid has
// them), so that the second step finds every in-plane neighbour in the
// block; it marches the range in z with the current plane of p_j and of q in
// LDS and the planes above and below in registers, as the single-system pair
// kernel does.  Face coefficients are read once per point and plane (the
// bottom face is the top face of the plane below), the Jacobi weight from the
// system's array of 1 / diag (formed at set-up by the same expression).
// Logical blocks take the right-hand sides of one band fastest, so the blocks
// that read the same coefficients run together on one XCD and share them
// through its L2.
//
// The loop body has no branch: a neighbour that does not exist is read from
// a zero slot past the end of each LDS plane (or, across the block's first
// and last rows, taken from the register loaded from global memory), and
// every value is formed and then selected.  Every memory access is a buffer
// access at a per-lane base plus a block-uniform plane offset; either is
// kMark when the point or the plane does not exist, and since every window
// stays below 1 GiB = kMark, such a sum lies outside it (the load returns 0,
// the store is dropped).
//
// MOM (moments Gram kind): the block also sums, over the points it stores,
// <q, M p_j>, <q, M q>, <p_{j+2}, M q>, <p_{j+2}, M p_{j+2}> (and
// <p_0, M p_0> first when FIRST), M the face diagonal with Jacobi (1 for the
// constant operator, whose diagonal the FGS kernel applies), and writes them
// to the pair's product slots from slot 2j + 1 (0 when FIRST), one partial
// per band (BSys::mofs).
constexpr uint32_t kMark = 0x40000000u;
template <typename T, bool FACES, bool FIRST, int D, int NT, bool MOM>
__global__ __launch_bounds__(NT) void k_bbasis_f2(const BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                                  const BF2Tile *__restrict__ tiles, uint32_t nbl,
                                                  const uint32_t *__restrict__ map,
                                                  const DevState *__restrict__ pairs, int nrhs, int precond, int j,
                                                  T *__restrict__ P, double *__restrict__ mpart, int s)
{
    constexpr uint32_t ES = sizeof(T);
    __shared__ T ps[2][NT + 1];  // slot NT holds 0
    __shared__ T qs[2][NT + 1];
    if (gl->ndone == gl->npairs)
        return;
    const uint32_t lb = map[blockIdx.x];
    if (lb >= nbl)
        return;  // whole block: no barrier is skipped by part of it
    const BF2Tile tl = tiles[lb / static_cast<uint32_t>(nrhs)];
    const int r = static_cast<int>(lb % static_cast<uint32_t>(nrhs));
    const BSys &S = sys[tl.q];
    if (pairs[S.pair0 + r].done)
        return;
    const int nx = S.g.nx, ny = S.g.ny, nz = S.g.nz;
    const uint32_t nxy = static_cast<uint32_t>(S.g.nxy);
    const int tid = threadIdx.x;
    if (tid < 2) {
        ps[tid][NT] = T(0);
        qs[tid][NT] = T(0);
    }
    // rows of the block: the band and the row on each side of it
    const int ye0 = tl.y0 > 0 ? tl.y0 - 1 : 0;
    const int ye1 = tl.y1 < ny ? tl.y1 + 1 : ny;
    const int er = tid / nx;
    const int i = tid - er * nx;
    const int ey = ye0 + er;
    const bool in_dom = ey < ye1;
    const bool interior = in_dom && ey >= tl.y0 && ey < tl.y1;
    const bool hs = ey > ye0, hn = ey + 1 < ye1;
    // LDS neighbours: the point's own slot index, or the zero slot
    const int iw = in_dom && i > 0 ? tid - 1 : NT;
    const int ie = in_dom && i + 1 < nx ? tid + 1 : NT;
    const int is = in_dom && hs ? tid - nx : NT;
    const int in = in_dom && hn ? tid + nx : NT;
    // A point of the first or last row of the block reads its one neighbour
    // outside the block from global memory (0 where the grid ends there).
    const bool ring_s = in_dom && !hs && ey > 0;
    const bool ring = ring_s || (in_dom && !hn && ey + 1 < ny);
    const uint32_t pl = in_dom ? static_cast<uint32_t>(ey * nx + i) : 0u;
    const uint32_t b_pt = in_dom ? pl * ES : kMark;            // the point
    const uint32_t b_in = interior ? pl * ES : kMark;          // the point, stored by this block
    const uint32_t b_rg = ring ? (ring_s ? pl - nx : pl + nx) * ES : kMark;
    const int k0 = tl.k0, k1 = tl.k1;
    const int kj_hi = k1 + 1 < nz ? k1 + 1 : nz - 1;  // last plane of p_j the range reads
    const int kv_hi = k1 < nz ? k1 : nz - 1;          // last plane of q, p_{j-1}, ring values, faces
    const uint32_t pbytes = nxy * ES;
    // block-uniform plane offsets
    auto po = [&](int k, int klo, int khi) -> uint32_t {
        return k >= klo && k <= khi ? static_cast<uint32_t>(k) * pbytes : kMark;
    };
    const int64_t step = static_cast<int64_t>(nrhs) * S.ld;
    T *const col = P + S.pofs + static_cast<int64_t>(r) * S.ld + static_cast<int64_t>(j) * step;
    const uint32_t cbytes = static_cast<uint32_t>(S.n) * ES;
    const __amdgpu_buffer_rsrc_t rj = make_window(col, cbytes);
    const __amdgpu_buffer_rsrc_t rv = make_window(FIRST ? col : col - step, cbytes);
    const __amdgpu_buffer_rsrc_t rq = make_window(col + step, cbytes);
    const __amdgpu_buffer_rsrc_t r2 = make_window(col + 2 * step, cbytes);
    const T *kxp = nullptr, *kyp = nullptr, *kzp = nullptr, *dvp = nullptr;
    if constexpr (FACES) {
        if constexpr (sizeof(T) == 8)
            kxp = reinterpret_cast<const T *>(S.kx), kyp = reinterpret_cast<const T *>(S.ky),
            kzp = reinterpret_cast<const T *>(S.kz), dvp = reinterpret_cast<const T *>(S.dinv);
        else
            kxp = reinterpret_cast<const T *>(S.kx32), kyp = reinterpret_cast<const T *>(S.ky32),
            kzp = reinterpret_cast<const T *>(S.kz32), dvp = reinterpret_cast<const T *>(S.dinv32);
    }
    // faces: x-faces (nx + 1 per grid row), y-faces (ny + 1 rows of nx per
    // plane), z-faces (nz + 1 planes)
    const uint32_t xrow = static_cast<uint32_t>(nx + 1);
    const uint32_t xplane = static_cast<uint32_t>(ny) * xrow * ES, yplane = static_cast<uint32_t>(ny + 1) * nx * ES;
    const __amdgpu_buffer_rsrc_t rfx = make_window(kxp, static_cast<uint32_t>(nz) * xplane);
    const __amdgpu_buffer_rsrc_t rfy = make_window(kyp, static_cast<uint32_t>(nz) * yplane);
    const __amdgpu_buffer_rsrc_t rfz = make_window(kzp, (static_cast<uint32_t>(nz) + 1) * pbytes);
    const __amdgpu_buffer_rsrc_t rdv = make_window(dvp, cbytes);
    const uint32_t b_fx = in_dom ? (static_cast<uint32_t>(ey) * xrow + static_cast<uint32_t>(i)) * ES : kMark;
    const uint32_t b_fy = b_pt;  // (ey * nx + i) within a plane of y-faces
    auto fxo = [&](int k) -> uint32_t { return k >= 0 && k <= kv_hi ? static_cast<uint32_t>(k) * xplane : kMark; };
    auto fyo = [&](int k) -> uint32_t { return k >= 0 && k <= kv_hi ? static_cast<uint32_t>(k) * yplane : kMark; };
    const T theta = static_cast<T>(S.theta), sigma = static_cast<T>(S.sigma);
    const T two_theta = T(2) * theta;
    const T minv_c = precond ? T(1) / T(6) : T(1);
    T pm = buf_load(T(), rj, b_pt + po(k0 - 2, 0, kj_hi));  // p_j one plane below the current one
    T p0 = buf_load(T(), rj, b_pt + po(k0 - 1, 0, kj_hi));  // p_j on the current plane
    T qb = T(0), qc = T(0);  // q two planes and one plane below the current one
    T fb = T(0);             // bottom face of the current plane
    if constexpr (FACES)
        fb = buf_load(T(), rfz, b_pt + po(k0 - 1, 0, kv_hi + 1));
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;  // products (MOM)
    // coefficients of the plane below (the second step's plane)
    T gw = T(0), ge = T(0), gs = T(0), gn = T(0), gb = T(0), gt = T(0), gd = T(0);
    // slot u holds, for plane kq = k0 - 1 + u (mod D): p_j on plane kq + 1,
    // p_{j-1}, the ring neighbour, the faces and the Jacobi weight of plane kq
    T pjs[D], pps[D], rgs[D];
    T fws[FACES ? D : 1], fes[FACES ? D : 1], fss[FACES ? D : 1], fns[FACES ? D : 1], fts[FACES ? D : 1],
        fds[FACES ? D : 1];
    auto fill = [&](int u, int kq) {
        pjs[u] = buf_load(T(), rj, b_pt + po(kq + 1, 0, kj_hi));
        if constexpr (!FIRST)
            pps[u] = buf_load(T(), rv, b_pt + po(kq, 0, kv_hi));
        rgs[u] = buf_load(T(), rj, b_rg + po(kq, 0, kv_hi));
        if constexpr (FACES) {
            const uint32_t ox = b_fx + fxo(kq), oy = b_fy + fyo(kq);
            fws[u] = buf_load(T(), rfx, ox);
            fes[u] = buf_load(T(), rfx, ox + ES);
            fss[u] = buf_load(T(), rfy, oy);
            fns[u] = buf_load(T(), rfy, oy + static_cast<uint32_t>(nx) * ES);
            fts[u] = buf_load(T(), rfz, b_pt + po(kq + 1, 0, kv_hi + 1));
            fds[u] = buf_load(T(), rdv, b_pt + po(kq, 0, kv_hi));
        }
    };
#pragma unroll
    for (int u = 0; u < D; ++u) {
        if constexpr (FIRST)
            pps[u] = T(0);
        fill(u, k0 - 1 + u);
    }
    // planes k0 - 1 .. k1, padded to a multiple of D: a padding step loads
    // nothing (its offsets lie outside the windows) and stores nothing
    const int nstep = (k1 - k0 + 2 + D - 1) / D * D;
    for (int base = k0 - 1; base < k0 - 1 + nstep; base += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int kq = base + u;
            const int buf = kq & 1;
            const T pp = pjs[u], pv = pps[u], rg = rgs[u];
            T fw = T(0), fe = T(0), fs = T(0), fn = T(0), ft = T(0), dinv = minv_c;
            if constexpr (FACES)
                fw = fws[u], fe = fes[u], fs = fss[u], fn = fns[u], ft = fts[u], dinv = fds[u];
            ps[buf][tid] = p0;
            lds_barrier();
            T q;
            {
                const T w = ps[buf][iw], e = ps[buf][ie];
                const T sl = ps[buf][is], nl = ps[buf][in];
                const T s = hs ? sl : rg;
                const T n = hn ? nl : rg;
                T y;
                if constexpr (FACES)
                    y = fw * (p0 - w) + fe * (p0 - e) + fs * (p0 - s) + fn * (p0 - n) + fb * (p0 - pm) +
                        ft * (p0 - pp);
                else
                    y = T(6) * p0 - (((((w + e) + s) + n) + pm) + pp);
                T qv;
                if constexpr (FIRST)
                    qv = theta * (dinv * y - sigma * p0);
                else
                    qv = two_theta * (dinv * y - sigma * p0) - pv;
                const bool act = kq >= 0 && kq <= k1 && kq < nz;  // block-uniform
                q = in_dom && act ? qv : T(0);
            }
            buf_store_out(q, rq, b_in + po(kq, k0, k1 - 1));
            qs[buf][tid] = q;
            // the second step on the plane below: q there is in qs[buf ^ 1]
            // (stored before this plane's barrier), q below it in qb, above in q
            {
                const T *qp = qs[buf ^ 1];
                const T w = qp[iw], e = qp[ie], s = qp[is], n = qp[in];
                T y;
                if constexpr (FACES)
                    y = gw * (qc - w) + ge * (qc - e) + gs * (qc - s) + gn * (qc - n) + gb * (qc - qb) +
                        gt * (qc - q);
                else
                    y = T(6) * qc - (((((w + e) + s) + n) + qb) + q);
                const T p2 = two_theta * ((FACES ? gd : minv_c) * y - sigma * qc) - pm;
                buf_store_out(p2, r2, b_in + po(kq - 1, k0, k1 - 1));
                if constexpr (MOM) {
                    // the plane just stored: p_j, q and p_{j+2} of plane kq - 1
                    const bool own = interior && kq - 1 >= k0 && kq - 1 < k1;
                    double w = 1.0;
                    if constexpr (FACES)
                        w = precond ? static_cast<double>(((((gw + ge) + gs) + gn) + gb) + gt) : 1.0;
                    w = own ? w : 0.0;
                    const double a = static_cast<double>(pm), b = static_cast<double>(qc);
                    const double c2 = static_cast<double>(p2);
                    if constexpr (FIRST)
                        m0 += w * a * a;
                    m1 += w * b * a;
                    m2 += w * b * b;
                    m3 += w * c2 * b;
                    m4 += w * c2 * c2;
                }
            }
            qb = qc;
            qc = q;
            pm = p0;
            p0 = pp;
            if constexpr (FACES) {
                gw = fw, ge = fe, gs = fs, gn = fn, gb = fb, gt = ft, gd = dinv;
                fb = ft;
            }
            // refill the slot for plane kq + D once its values are used
            fill(u, kq + D);
        }
    }
    if constexpr (MOM) {
        const int ns = bmom_slots(s);
        double *out = mpart + S.mofs + (static_cast<int64_t>(r) * ns + (FIRST ? 0 : 2 * j + 1)) * S.nf2q +
                      (static_cast<int32_t>(lb / static_cast<uint32_t>(nrhs)) - S.f2first);
        if constexpr (FIRST) {
            const double v[5] = {m0, m1, m2, m3, m4};
            block_partials<5, NT>(v, out, S.nf2q);
        } else {
            const double v[4] = {m1, m2, m3, m4};
            block_partials<4, NT>(v, out, S.nf2q);
        }
    }
}

// x += P alpha for every pair whose solve continues.
// Residual over the two-step basis's band table (FP64 arithmetic; p_0 stored
// in TP): on the band's rows of one right-hand side, r = b - A x, p_0 =
// p0scale M^{-1} r (p0scale r with p0_mode 1), and the band's partial of
// ||r||^2 in slot `slot` of the pair's `slots` band partials.  The block marches its range of planes:
// x of the current plane (the band's rows and the row on each side) sits in
// LDS, double-buffered with one barrier per plane, and the planes below and
// above in registers, so each range reads x once (plus one plane on each
// side).  The operator expression is PointStencil's, as in k_bresidual; the
// Jacobi weights are the stored ones, which k_bdinv forms with PointStencil's
// expression.
template <typename TP, bool FACES, int NT>
__global__ __launch_bounds__(NT) void k_bres_f2(const BGlob *__restrict__ gl, const BSys *__restrict__ sys,
                                               const BF2Tile *__restrict__ tiles, uint32_t nbl,
                                               const uint32_t *__restrict__ map, const DevState *__restrict__ pairs,
                                               int nrhs, int precond, int p0_mode, TP *__restrict__ P,
                                               double *__restrict__ mpart, int slots, int slot)
{
    __shared__ double xs[2][NT];
    if (gl->ndone == gl->npairs)
        return;
    const uint32_t lb = map[blockIdx.x];
    if (lb >= nbl)
        return;  // whole block: no barrier is skipped by part of it
    const BF2Tile tl = tiles[lb / static_cast<uint32_t>(nrhs)];
    const int r = static_cast<int>(lb % static_cast<uint32_t>(nrhs));
    const BSys &S = sys[tl.q];
    const DevState &ps = pairs[S.pair0 + r];
    if (ps.done)
        return;
    const int nx = S.g.nx, ny = S.g.ny, nz = S.g.nz;
    const int64_t nxy = S.g.nxy;
    const int tid = threadIdx.x;
    const int ye0 = tl.y0 > 0 ? tl.y0 - 1 : 0;
    const int ye1 = tl.y1 < ny ? tl.y1 + 1 : ny;
    const int er = tid / nx;
    const int i = tid - er * nx;
    const int ey = ye0 + er;
    const bool in_dom = ey < ye1;
    const bool interior = in_dom && ey >= tl.y0 && ey < tl.y1;
    const int64_t pl = in_dom ? static_cast<int64_t>(ey) * nx + i : 0;
    const double *__restrict__ x = ps.x;
    const double *__restrict__ b = ps.b;
    const double scale = ps.p0scale;
    TP *__restrict__ p0 = P + S.pofs + static_cast<int64_t>(r) * S.ld;
    const double dconst = precond ? 1.0 / 6.0 : 1.0;
    const int k0 = tl.k0, k1 = tl.k1;
    double xb = in_dom && k0 > 0 ? x[pl + (k0 - 1) * nxy] : 0.0;
    double xc = in_dom ? x[pl + k0 * nxy] : 0.0;
    double acc = 0.0;
    for (int k = k0; k < k1; ++k) {
        const int64_t c = pl + static_cast<int64_t>(k) * nxy;
        const double xt = in_dom && k + 1 < nz ? x[c + nxy] : 0.0;
        double bc = 0.0, fw = 0.0, fe = 0.0, fs = 0.0, fn = 0.0, fb = 0.0, ft = 0.0, dv = dconst;
        if (interior) {
            bc = b[c];
            if constexpr (FACES) {
                const int64_t fx = c + static_cast<int64_t>(k) * ny + ey;  // x-faces: nx + 1 per grid row
                const int64_t fy = c + static_cast<int64_t>(k) * nx;       // y-faces: ny + 1 rows per plane
                fw = S.kx[fx], fe = S.kx[fx + 1], fs = S.ky[fy], fn = S.ky[fy + nx], fb = S.kz[c],
                ft = S.kz[c + nxy];
                dv = S.dinv[c];
            }
        }
        double *buf = xs[k & 1];
        buf[tid] = xc;
        __syncthreads();
        if (interior) {
            const double w = i > 0 ? buf[tid - 1] : 0.0;
            const double e = i + 1 < nx ? buf[tid + 1] : 0.0;
            const double so = ey > 0 ? buf[tid - nx] : 0.0;
            const double no = ey + 1 < ny ? buf[tid + nx] : 0.0;
            double ax;
            if constexpr (FACES)
                ax = fw * (xc - w) + fe * (xc - e) + fs * (xc - so) + fn * (xc - no) + fb * (xc - xb) +
                     ft * (xc - xt);
            else
                ax = 6.0 * xc - (((((w + e) + so) + no) + xb) + xt);
            const double rr = bc - ax;
            acc += rr * rr;
            p0[c] = static_cast<TP>(scale * (p0_mode ? rr : dv * rr));
        }
        xb = xc;
        xc = xt;
    }
    const double v[1] = {acc};
    block_partials<1, NT>(v,
                          mpart + S.mofs + (static_cast<int64_t>(r) * slots + slot) * S.nf2q +
                              (static_cast<int32_t>(lb / static_cast<uint32_t>(nrhs)) - S.f2first),
                          S.nf2q);
}

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

namespace {
template <typename T, bool FACES, int D, int NT, bool MOM>
hipError_t bbasis_pair_v(const BatchArgs &a, int j, hipStream_t st)
{
    const dim3 grid(a.f2grid);
    const uint32_t nbl = static_cast<uint32_t>(a.nf2) * static_cast<uint32_t>(a.nrhs);
    T *P = static_cast<T *>(a.P);
    if (j == 0)
        hipLaunchKernelGGL((k_bbasis_f2<T, FACES, true, D, NT, MOM>), grid, dim3(NT), 0, st, a.gl, a.sys,
                           a.f2tiles, nbl, a.f2map, a.pairs, a.nrhs, a.precond, j, P, a.mpart, a.s);
    else
        hipLaunchKernelGGL((k_bbasis_f2<T, FACES, false, D, NT, MOM>), grid, dim3(NT), 0, st, a.gl, a.sys,
                           a.f2tiles, nbl, a.f2map, a.pairs, a.nrhs, a.precond, j, P, a.mpart, a.s);
    return hipGetLastError();
}
// Planes of loads in flight: 2 in FP64, 3 in FP32 (fastest on MI355X for the
// batched workload among 2..4 with 512- and 1024-thread blocks).
template <typename T, bool FACES>
hipError_t bbasis_pair_t(const BatchArgs &a, int j, hipStream_t st)
{
    constexpr int D = sizeof(T) == 8 ? 2 : 3;
    if (a.mom)
        return bbasis_pair_v<T, FACES, D, kBf2Threads, true>(a, j, st);
    return bbasis_pair_v<T, FACES, D, kBf2Threads, false>(a, j, st);
}
}  // namespace

namespace {
template <typename TP, bool FACES>
hipError_t bres_f2_t(const BatchArgs &a, hipStream_t st)
{
    const uint32_t nbl = static_cast<uint32_t>(a.nf2) * static_cast<uint32_t>(a.nrhs);
    hipLaunchKernelGGL((k_bres_f2<TP, FACES, kBf2Threads>), dim3(a.f2grid), dim3(kBf2Threads), 0, st, a.gl, a.sys,
                       a.f2tiles, nbl, a.f2map, a.pairs, a.nrhs, a.precond, a.p0_mode, static_cast<TP *>(a.P),
                       a.mpart, a.bres_slots, a.bres_slot);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_bres_f2(const BatchArgs &a, hipStream_t st)
{
    if (!a.f2 || !a.bres)
        return hipErrorInvalidValue;  // only over a band table with its partial slots
    if (a.fp32)
        return a.faces ? bres_f2_t<float, true>(a, st) : bres_f2_t<float, false>(a, st);
    return a.faces ? bres_f2_t<double, true>(a, st) : bres_f2_t<double, false>(a, st);
}

hipError_t launch_bdinv(const BSys &S, int precond, int fp32, double *dinv, float *dinv32, hipStream_t st)
{
    const dim3 grid(static_cast<uint32_t>((S.n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_bdinv<double>, grid, dim3(kBlock), 0, st, S, precond, dinv);
    if (fp32)
        hipLaunchKernelGGL(k_bdinv<float>, grid, dim3(kBlock), 0, st, S, precond, dinv32);
    return hipGetLastError();
}

// Steps j and j + 1 of every active pair's basis (recurrence Gram kind, the
// band table built on the host).
hipError_t launch_bbasis_pair(const BatchArgs &a, int j, hipStream_t st)
{
    if (!a.f2 || j < 0 || j + 2 > a.s)
        return hipErrorInvalidValue;
    if (a.fp32)
        return a.faces ? bbasis_pair_t<float, true>(a, j, st) : bbasis_pair_t<float, false>(a, j, st);
    return a.faces ? bbasis_pair_t<double, true>(a, j, st) : bbasis_pair_t<double, false>(a, j, st);
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
