"""Benchmark of the s-step CG hot path on one MI355X.

Headline (``value``): time-to-1e-8 relative residual of the FP64 solve of the
224^3 (11,239,424-unknown) 3D 7-point Poisson problem, matrix-free stencil,
Jacobi, Chebyshev basis s = 16 with exact bounds, nu = 25 FGS sweeps,
x0 = 0, b = A x* with x* ~ U[-1, 1] (seed 0); effective HBM bandwidth =
algorithmic bytes per outer iteration x outer iterations / time.

A step runs every leg once, one solve each, all to 1e-8:
  c2_fp64       the headline solve
  c2_fp32ir     the same system, FP32 basis/SpMV/Gram inside FP64 refinement
  c2_csr_fp64   the same system as an assembled CSR matrix
  c1_csr_fp64   2D 5-point Poisson 64^2 (n = 4096), CSR, s = 8, nu = 20
  c5_adjoint    128^3 diffusion (log-normal faces, sigma 0.5): forward solve,
                then the backward pass (adjoint solve + face-gradient scatter)
  c4_batched_*  64 diffusion systems (N ~ U{32..96}, faces sigma 1) x 8
                right-hand sides, FP64 and FP32+IR
Inputs are resident in device memory before the timed region.  Prints one
JSON line on stdout (progress on stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "time-to-1e-8 residual & HBM GB/s, 11.2M-unknown Poisson: FP64 vs FP32+IR"
HBM_PEAK_GBPS = 8000.0
ALL_LEGS = ("c2_fp64", "c2_fp32ir", "c2_csr_fp64", "c1_csr_fp64", "c5_adjoint", "c4_batched_fp64",
            "c4_batched_fp32ir")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def basis_vectors(s: int, kind: str = "stored", pairs: int = 0) -> int:
    """Vectors one basis moves per unknown, each read or write of a column
    counted once.  Single steps: the first reads p_0 and writes p_1 (2), each
    later one reads p_j, p_{j-1} and writes p_{j+1} (3); the apply kind takes
    s - 1 steps (3s - 4), the recurrence and moments kinds s (3s - 1); with AP stored every
    launch also writes A p_j and the last writes only that (4s - 3).  Two
    steps per launch (pairs > 0): the first pair reads p_0 and writes p_1, p_2
    (3), each later pair reads two columns and writes two (4), and an odd
    column count ends with one single step (3)."""
    m = s - 1 if kind == "apply" else s
    if pairs > 0:
        return 3 + 4 * (pairs - 1) + 3 * (m - 2 * pairs)
    if kind == "apply":
        return 3 * s - 4
    if kind in ("recurrence", "moments"):
        return 3 * s - 1
    return 4 * s - 3


def stencil_bytes_per_outer(n: int, s: int, w: int, kind: str = "stored", pairs: int = 0) -> float:
    """Bytes an outer iteration must move, constant-coefficient stencil:
    residual 16 + w (x, b read in FP64, p_0 written), the basis (above), the
    Gram reading its columns (stored: P and AP, 2s; apply: P, s; recurrence:
    p_0 .. p_s, s + 1; moments: none, the basis kernels form its products),
    the update sw + 16 (P read, x read and written)."""
    gram_cols = {"stored": 2 * s, "apply": s, "recurrence": s + 1, "moments": 0}[kind]
    return float(n) * (32 + w * (1 + basis_vectors(s, kind, pairs) + gram_cols + s))


def csr_bytes_per_outer(n: int, nnz: int, s: int, w: int, kind: str = "stored", pairs: int = 0) -> float:
    """The stencil figure plus the matrix (values and column indices, row
    pointers) read by s basis SpMVs in precision w and one FP64 residual SpMV,
    and the M-diagonal read by the Gram kernel (none with the moments kind)."""
    mat_w = float(nnz) * (4 + w) + 4.0 * (n + 1)
    mat_64 = float(nnz) * 12 + 4.0 * (n + 1)
    dvec = 0.0 if kind == "moments" else float(n) * w
    return stencil_bytes_per_outer(n, s, w, kind, pairs) + s * mat_w + mat_64 + dvec


def faces_bytes_per_outer(n: int, s: int, w: int, nrhs: int = 1, kind: str = "stored") -> float:
    """Stencil figure per right-hand side plus the three face arrays read by the
    FP64 residual and s more times (the s basis steps, or the s - 1 basis
    steps and the Gram when it forms A p_j itself), shared by nrhs right-hand
    sides, and the M-diagonal read by the Gram kernel (none with the moments kind)."""
    dvec = 0.0 if kind == "moments" else float(n) * w
    return nrhs * (stencil_bytes_per_outer(n, s, w, kind) + dvec) + float(n) * 3 * (8 + s * w)


def batched_system_bytes(n: int, s: int, w: int, kind: str, pairs: int) -> tuple:
    """Bytes of one outer iteration of one batched face-coefficient system of
    n unknowns: (per right-hand side, shared by its right-hand sides).  Per
    right-hand side: the stencil figure with the basis launches used, and the
    M diagonal read by the Gram kernel (not with the moments kind).  Shared:
    the three face arrays read by the FP64 residual (8-byte) and once per
    basis launch in width w, and with two steps per launch the array of
    Jacobi weights too."""
    launches = s - pairs
    per_rhs = stencil_bytes_per_outer(n, s, w, kind, pairs) + (0.0 if kind == "moments" else float(n) * w)
    shared = float(n) * (3 * 8 + launches * (3 + (1 if pairs else 0)) * w)
    return per_rhs, shared


def basis_bytes_per_launch(n: int, s: int, w: int, kind: str = "stored", pairs: int = 0,
                           launches: int = 0) -> float:
    """Average algorithmic bytes of one basis launch: basis_vectors over the
    launches of one basis (s, or s - 1 for the apply kind, with single steps)."""
    if launches <= 0:
        launches = s - 1 if kind == "apply" else s
    return float(n) * w * basis_vectors(s, kind, pairs) / launches


def measured_traffic(N: int, s: int, nu: int):
    """HBM bytes recorded from hardware counters for the 224^3, s = 16, nu = 25
    FP64 workload (per basis launch and per outer iteration), or None when the
    workload differs or the kernel sources have changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_poisson224_s16_fp64.json")
    if (N, s, nu) != (224, 16, 25) or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in rec["source_files"]:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    return rec if h.hexdigest() == rec["source_sha256"] else None


def _host_description() -> dict:
    """CPU model and core counts of the host the oracle is timed on."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return info


def cpu_baseline(N: int, s: int, nu: int, gpu_iters: int, sample_outer: int) -> dict:
    """The FP64 oracle on the headline problem, timed on this host over a
    bounded sample of outer iterations of its own solve loop (its stopping
    test set out of reach, so exactly ``sample_outer`` updates run) and scaled
    to the GPU's iteration count: once as the sequential reference build the
    tests pin (one core) and once as the OpenMP build of the same loops on
    every core the process may use (``value``)."""
    import gen
    import oracle

    pr = gen.config2(0, N=N, s=s, nu=nu)
    A = oracle.assemble_stencil7(N, N, N)
    b = oracle.spmv(A, pr.xstar)
    runs = {}
    for omp in (False, True):
        threads = oracle.select_build(omp)
        t0 = time.perf_counter()
        out = oracle.solve(A, b, None, s, nu, pr.lmin, pr.lmax, 1e-300, max_outer=sample_outer)
        dt = time.perf_counter() - t0
        assert out["iters"] == sample_outer, out["iters"]
        runs[omp] = (threads, dt, 1e3 * dt / sample_outer)
    oracle.select_build(False)
    threads, dt, ms = runs[True]
    _, dt1, ms1 = runs[False]
    return {
        "value": ms * gpu_iters,
        "unit": "ms",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{sample_outer} outer iterations of the oracle's solve of the {N}^3 FP64 problem (s={s}, "
                  f"nu={nu}), OpenMP build on {threads} threads: {dt:.1f} s, {ms:.0f} ms per outer iteration, "
                  f"scaled to the GPU's {gpu_iters} outer iterations to 1e-8",
        "single_thread": {"value": ms1 * gpu_iters, "ms_per_outer": ms1, "seconds": dt1, "cores": 1},
        "host": _host_description(),
    }


def c5_gradient_error(grads) -> dict | None:
    """Entry-wise error of the differentiable solve's gradient at tol 1e-8
    against the oracle's reference gradient (forward and adjoint at 1e-12;
    tests/golden/c5_oracle_grad.json, written from the oracle alone): the
    largest |difference| over the fixture's sampled entries relative to the
    largest |entry|."""
    path = os.path.join(ROOT, "tests", "golden", "c5_oracle_grad.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f)
    gk, gb, x = (t.detach().cpu().numpy() for t in grads)
    out = {}
    for name, got, idx, want in (("dL_dk", gk, ref["idx_k"], ref["dk"]), ("dL_db", gb, ref["idx_v"], ref["lam"]),
                                 ("x", x, ref["idx_v"], ref["x"])):
        want = np.asarray(want)
        out[name] = float(np.abs(got[np.asarray(idx)] - want).max() / np.abs(want).max())
    out["samples"] = len(ref["idx_k"])
    return out


class Leg:
    """One timed workload: setup() builds inputs and solvers, run() does one
    solve (or forward + backward) and returns the outer-iteration count."""

    def __init__(self, name):
        self.name = name
        self.times = []
        self.iters = None
        self.extra = {}

    def timed(self, sync):
        t0 = time.perf_counter()
        it = self.run()
        sync()
        self.times.append(1e3 * (time.perf_counter() - t0))
        self.iters = it


def build_legs(lib, torch, legs, N, s, nu, c4_nsys, gram="auto"):
    import gen

    dev = torch.device("cuda:0")
    out = {}

    if {"c2_fp64", "c2_fp32ir", "c2_csr_fp64"} & set(legs):
        pr = gen.config2(0, N=N, s=s, nu=nu)
        op = lib.Operator.stencil(N, N, N)
        xstar = torch.as_tensor(pr.xstar, device=dev)
        base = lib.Solver(op, s, nu, pr.lmin, pr.lmax, gram=gram)
        b = base.apply(xstar)
        for name, prec in (("c2_fp64", "fp64"), ("c2_fp32ir", "fp32ir")):
            if name not in legs:
                continue
            leg = Leg(name)
            leg.solver = base if prec == "fp64" else lib.Solver(op, s, nu, pr.lmin, pr.lmax, precision=prec,
                                                                gram="stored" if gram == "apply" else gram)
            leg.b, leg.x = b, torch.zeros_like(b)

            def run(leg=leg):
                leg.x.zero_()
                _, st = leg.solver.solve(leg.b, leg.x, 1e-8)
                return st.outer_iters

            leg.run = run
            leg.bytes_per_outer = stencil_bytes_per_outer(pr.n, s, 8 if prec == "fp64" else 4,
                                                          leg.solver.gram_kind, leg.solver.basis_pairs)
            leg.n = pr.n
            out[name] = leg
        if "c2_csr_fp64" in legs:
            rp, ci, v = gen.poisson3d_csr(N, N, N)
            leg = Leg("c2_csr_fp64")
            leg.solver = lib.Solver(lib.Operator.csr(rp, ci, v), s, nu, pr.lmin, pr.lmax,
                                    gram="stored" if gram == "apply" else gram)
            leg.b, leg.x = b, torch.zeros_like(b)

            def run(leg=leg):
                leg.x.zero_()
                _, st = leg.solver.solve(leg.b, leg.x, 1e-8)
                return st.outer_iters

            leg.run = run
            leg.bytes_per_outer = csr_bytes_per_outer(pr.n, ci.size, s, 8, leg.solver.gram_kind, leg.solver.basis_pairs)
            leg.n = pr.n
            out["c2_csr_fp64"] = leg
        log("c2 legs ready")

    if "c1_csr_fp64" in legs:
        pr = gen.config1(0)
        rp, ci, v = pr.csr()
        leg = Leg("c1_csr_fp64")
        leg.solver = lib.Solver(lib.Operator.csr(rp, ci, v), pr.s, pr.nu, pr.lmin, pr.lmax,
                                gram="stored" if gram == "apply" else gram)
        leg.b = leg.solver.apply(torch.as_tensor(pr.xstar, device=dev))
        leg.x = torch.zeros_like(leg.b)

        def run(leg=leg):
            leg.x.zero_()
            _, st = leg.solver.solve(leg.b, leg.x, 1e-8)
            return st.outer_iters

        leg.run = run
        leg.bytes_per_outer = None  # cache-resident: latency-bound, no bandwidth claim
        leg.n = pr.n
        out["c1_csr_fp64"] = leg

    if "c5_adjoint" in legs:
        pr = gen.config5(0)
        leg = Leg("c5_adjoint")
        leg.solver = lib.Solver(lib.Operator.stencil(*pr.dims, pr.kx, pr.ky, pr.kz), pr.s, pr.nu, pr.lmin, pr.lmax,
                                gram=gram)
        leg.coeffs = torch.as_tensor(np.concatenate([pr.kx, pr.ky, pr.kz]), device=dev)
        leg.b = torch.as_tensor(pr.rhs[0], device=dev)
        leg.xt = torch.as_tensor(pr.xtarget, device=dev)
        leg.fwd, leg.bwd = [], []

        def run(leg=leg):
            cf = leg.coeffs.clone().requires_grad_(True)
            bb = leg.b.clone().requires_grad_(True)
            t0 = time.perf_counter()
            x = lib.sstep_solve(cf, bb, leg.solver, 1e-8)
            loss = 0.5 * torch.sum((x - leg.xt) ** 2)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            leg.fwd.append(1e3 * (t1 - t0))
            leg.bwd.append(1e3 * (t2 - t1))
            leg.grads = (cf.grad, bb.grad, x.detach())
            return leg.solver.last_forward_stats.outer_iters

        leg.run = run
        leg.bytes_per_outer = faces_bytes_per_outer(pr.n, pr.s, 8, kind=leg.solver.gram_kind)
        leg.n = pr.n
        out["c5_adjoint"] = leg

    for prec in ("fp64", "fp32ir"):
        name = f"c4_batched_{prec}"
        if name not in legs:
            continue
        probs = gen.config4(seed=0, nsys=c4_nsys)
        ops = [lib.Operator.stencil(*p.dims, p.kx, p.ky, p.kz) for p in probs]
        leg = Leg(name)
        leg.solver = lib.BatchedSolver(ops, 8, 16, 25, [p.lmin for p in probs], [p.lmax for p in probs],
                                       precision=prec)
        leg.b = [torch.as_tensor(np.concatenate(p.rhs), device=dev) for p in probs]
        leg.x = [torch.zeros_like(bq) for bq in leg.b]

        def run(leg=leg):
            for xq in leg.x:
                xq.zero_()
            _, st = leg.solver.solve(leg.b, leg.x, 1e-8)
            leg.pair_iters = [p.outer_iters for p in st]
            leg.pair_relres = [p.rel_res for p in st]
            return max(leg.pair_iters)

        leg.run = run
        w = 8 if prec == "fp64" else 4
        sizes = [p.n for p in probs]
        # per system: (bytes per right-hand side per outer iteration, face-array bytes shared by the rhs),
        # for the Gram kind the batched solver uses
        kind = leg.solver.gram_kind
        leg.pair_bytes = [batched_system_bytes(nq, 16, w, kind, leg.solver.basis_pairs) for nq in sizes]
        leg.bytes_per_outer = None
        leg.n = sum(sizes)
        leg.nsys = len(probs)
        leg.sides = [p.dims[0] for p in probs]
        out[name] = leg
        log(f"{name} ready: {len(probs)} systems, {leg.n} unknowns x 8 rhs")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=224, help="grid edge of the headline problem (224 -> 11.2M)")
    ap.add_argument("--s", type=int, default=16)
    ap.add_argument("--nu", type=int, default=25)
    ap.add_argument("--legs", default=",".join(ALL_LEGS), help="comma-separated subset of " + ",".join(ALL_LEGS))
    ap.add_argument("--c4-nsys", type=int, default=64)
    ap.add_argument("--kernel-reps", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=10, help="oracle outer iterations for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the one-time measurements after the timed steps (C3 sweep, Lanczos bounds, the "
                         "27-point table, the coarse solve)")
    ap.add_argument("--N27", type=int, default=230, help="grid edge of the paper's 27-point workload")
    ap.add_argument("--gram", default="auto", choices=["auto", "stored", "apply", "recurrence", "moments"],
                    help="Gram kind of the single-system legs (default: the library's choice; 'apply' falls back "
                         "to 'stored' where the operator-applying kernel does not exist)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain device copy of n doubles (calibrates traffic counters)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the step: FP32+IR vs FP64 time-to-tol for s in {8,16,24,32} x nu in {20,30}")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of this "
              "solver is a design, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2512_09642_amd as lib

    lib.require_gpu()
    if args.sweep:
        return sweep(lib, torch, args)
    if args.calib_copy:
        src = torch.ones(args.N ** 3, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.N ** 3} doubles ({16 * args.N ** 3} bytes read + written)")
        del src, dst
    legs_wanted = [x for x in args.legs.split(",") if x]
    legs = build_legs(lib, torch, legs_wanted, args.N, args.s, args.nu, args.c4_nsys, args.gram)
    torch.cuda.synchronize()
    sync = torch.cuda.synchronize
    order = [name for name in ALL_LEGS if name in legs]
    for w in range(args.warmup):
        for name in order:
            legs[name].timed(sync)
        log(f"warmup {w}: " + ", ".join(f"{nm} {legs[nm].times[-1]:.1f} ms" for nm in order))
    for name in order:
        legs[name].times.clear()
        if hasattr(legs[name], "fwd"):
            legs[name].fwd.clear()
            legs[name].bwd.clear()
    sync()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        for name in order:
            legs[name].timed(sync)
    sync()
    total_ms = 1e3 * (time.perf_counter() - t_start)
    log("timed steps: " + ", ".join(f"{nm} {np.median(legs[nm].times):.1f} ms" for nm in order))

    results = {}
    for name in order:
        leg = legs[name]
        t = float(np.median(leg.times))
        r = {"time_ms": t, "outer_iters": leg.iters}
        if name.startswith("c4"):
            tot_bytes = 0.0
            for q in range(leg.nsys):
                its = leg.pair_iters[q * 8:(q + 1) * 8]
                per_rhs, faces = leg.pair_bytes[q]
                tot_bytes += per_rhs * sum(its) + faces * max(its)
            per_sys = [max(leg.pair_iters[q * 8:(q + 1) * 8]) for q in range(leg.nsys)]
            g = tot_bytes / (t * 1e-3) / 1e9
            r.update(frac_of_hbm_peak=g / HBM_PEAK_GBPS, tiles=leg.solver.tiles,
                     basis_launches=leg.solver.basis_launches, basis_pairs=leg.solver.basis_pairs)
            r.update(outer_iters_min=min(leg.pair_iters), outer_iters_max=max(leg.pair_iters),
                     pairs=len(leg.pair_iters), unknown_rhs=leg.n * 8,
                     max_rel_res=max(leg.pair_relres), gbps_effective=tot_bytes / (t * 1e-3) / 1e9,
                     # the spread of iteration counts against the grid side N of each system (cubic N^3 grids):
                     # Spearman rank correlation and the slowest system
                     iters_vs_side_spearman=float(np.corrcoef(np.argsort(np.argsort(leg.sides)),
                                                              np.argsort(np.argsort(per_sys)))[0, 1]),
                     slowest_system={"side": leg.sides[int(np.argmax(per_sys))], "outer_iters": max(per_sys)},
                     system_side_and_iters=[[int(a), int(b)] for a, b in zip(leg.sides, per_sys)])
        elif name == "c5_adjoint":
            f, bw = float(np.median(leg.fwd)), float(np.median(leg.bwd))
            fi = leg.solver.last_forward_stats.outer_iters
            ai = leg.solver.last_adjoint_stats.outer_iters
            r.update(forward_ms=f, backward_ms=bw, backward_over_forward=bw / f, n=leg.n, forward_outer_iters=fi,
                     adjoint_outer_iters=ai, forward_ms_per_outer=f / max(fi, 1), backward_ms_per_outer=bw / max(ai, 1),
                     gradient_error_vs_oracle=c5_gradient_error(leg.grads))
        else:
            r.update(ms_per_outer=t / max(leg.iters, 1))
            if leg.bytes_per_outer:
                g = leg.bytes_per_outer * leg.iters / (t * 1e-3) / 1e9
                r.update(gbps_effective=g, frac_of_hbm_peak=g / HBM_PEAK_GBPS,
                         algorithmic_bytes_per_outer=leg.bytes_per_outer)
        if getattr(leg.solver, "gram_kind", None):
            r["gram"] = leg.solver.gram_kind
        results[name] = r

    out = {
        "metric": METRIC,
        "value": results["c2_fp64"]["time_ms"] if "c2_fp64" in results else None,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"poisson3d_{args.N}^3_7pt_stencil_jacobi_chebyshev_s{args.s}_nu{args.nu}_tol1e-8",
            "n": args.N ** 3,
            "s": args.s,
            "nu": args.nu,
            "step": "one solve to 1e-8 per leg: " + ", ".join(order),
        },
        "results": results,
    }
    if "c2_fp64" in legs:
        main_leg = legs["c2_fp64"]
        kt = main_leg.solver.kernel_times(main_leg.b, torch.zeros_like(main_leg.b), reps=args.kernel_reps)
        results["c2_fp64"]["kernel_ms"] = kt
        if "c2_fp32ir" in legs:
            results["c2_fp32ir"]["kernel_ms"] = legs["c2_fp32ir"].solver.kernel_times(
                main_leg.b, torch.zeros_like(main_leg.b), reps=args.kernel_reps)
        kind = main_leg.solver.gram_kind
        sv0 = main_leg.solver
        traffic = measured_traffic(args.N, args.s, args.nu)
        # counter-measured HBM bytes of one outer iteration (all its kernels), next to the algorithmic ones
        results["c2_fp64"]["counter_bytes_per_outer"] = traffic.get("bytes_per_outer") if traffic else None
        per_launch = basis_bytes_per_launch(main_leg.n, args.s, 8, kind, sv0.basis_pairs, sv0.basis_launches)
        achieved = per_launch / (kt["basis"] * 1e-3) / 1e9
        if sv0.basis_pairs:
            kname = (f"k_basis_f2 (7-point stencil + Jacobi + two Chebyshev steps per launch, FP64), average of the "
                     f"{sv0.basis_launches} basis launches ({sv0.basis_pairs} pairs"
                     + (", one single step" if sv0.basis_launches > sv0.basis_pairs else "") + ")")
        else:
            kname = ("k_basis_p2 (7-point stencil + Jacobi + Chebyshev step, FP64), average of the "
                     + {"apply": "s - 1 launches (AP not written)", "recurrence": "s launches (the last writes p_s)",
                        "moments": "s launches (the last writes p_s)", "stored": "s launches (AP written)"}[kind])
        out["roofline"] = {
            "bound": "hbm",
            "kernel": kname,
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic["basis_avg_bytes_per_launch"] if traffic else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 read requests by size + WRITE_SIZE, copy-calibrated)",
            "bytes_per_launch": per_launch,
            "avg_launch_ms": kt["basis"],
            # the whole FP64 solve: algorithmic bytes of its outer iterations over its time
            "solve_achieved": results["c2_fp64"].get("gbps_effective"),
            "solve_frac": results["c2_fp64"].get("frac_of_hbm_peak"),
        }
        r = main_leg.b - main_leg.solver.apply(main_leg.x)
        results["c2_fp64"]["rel_res_true"] = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(main_leg.b))
        log(f"kernel times (ms): {kt}")
        if not args.no_extras:
            log("one-time measurements (not in the timed steps)")
            out["extras"] = {
                "c3_sweep": extra_c3(lib, torch, args.N),
                "lanczos_bounds": extra_lanczos(lib, torch, args.c4_nsys),
                "paper27_table": extra_paper27(lib, torch, args.N27),
                "coarse_solve": extra_coarse(lib, torch),
            }
        if not args.no_cpu_baseline:
            log("timing the oracle on the host (cpu_baseline)")
            out["cpu_baseline"] = cpu_baseline(args.N, args.s, args.nu, results["c2_fp64"]["outer_iters"],
                                               args.cpu_sample)
    for leg in legs.values():
        leg.solver.close()
    print(json.dumps(out), flush=True)


def _finite(v):
    """A float for the JSON line, or None when it is not finite."""
    v = float(v)
    return v if np.isfinite(v) else None


def _kappa(sv, b, x):
    """2-norm condition number of the scaled Gram matrix of one outer
    iteration from x = 0 (None on a breakdown or an infinite value)."""
    x.zero_()
    try:
        return _finite(np.linalg.cond(sv.step(b, x)["G"]))
    except Exception:  # a breakdown of the badly conditioned monomial basis
        return None


def _timed_solve(sv, b, x, tol, torch, reps=2, warm=True):
    """Median wall time (ms) of ``reps`` solves after one warm-up, and stats."""
    if warm:
        x.zero_()
        sv.solve(b, x, tol, raise_on_error=False)
    ts, st = [], None
    for _ in range(reps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = sv.solve(b, x, tol, raise_on_error=False)
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(ts)), st


def extra_c3(lib, torch, N):
    """The mixed-precision sweep of the 224^3 problem: for every (s, nu), the
    FP64 and FP32+IR times to 1e-8, their iteration counts, and the FP32 inner
    error of the first outer iteration against the FP64 step from the same
    x_0 = 0 (the FP64 step is the one the parity tests hold to the oracle)."""
    import gen

    dev = torch.device("cuda:0")
    rows = []
    b = None
    for s, nu in gen.config3_sweep():
        pr = gen.config2(0, N=N, s=s, nu=nu)
        row = {"s": s, "nu": nu}
        steps = {}
        for prec in ("fp64", "fp32ir"):
            with lib.Solver(lib.Operator.stencil(N, N, N), s, nu, pr.lmin, pr.lmax, precision=prec) as sv:
                if b is None:
                    b = sv.apply(torch.as_tensor(pr.xstar, device=dev))
                x = torch.zeros_like(b)
                t, st = _timed_solve(sv, b, x, 1e-8, torch)
                bpo = stencil_bytes_per_outer(pr.n, s, 8 if prec == "fp64" else 4, sv.gram_kind, sv.basis_pairs)
                row[prec] = {"time_ms": t, "outer_iters": st.outer_iters, "status": st.status, "gram": sv.gram_kind,
                             "gbps_effective": bpo * st.outer_iters / (t * 1e-3) / 1e9}
                x.zero_()
                steps[prec] = sv.step(b, x)
                steps[prec]["x"] = x.clone()
        d64 = steps["fp64"]["x"]
        row["fp32_inner_error_dx"] = float(torch.linalg.vector_norm(steps["fp32ir"]["x"] - d64)
                                           / torch.linalg.vector_norm(d64))
        row["fp32_inner_error_G"] = float(np.linalg.norm(steps["fp32ir"]["G"] - steps["fp64"]["G"])
                                          / np.linalg.norm(steps["fp64"]["G"]))
        row["fp32ir_speedup"] = row["fp64"]["time_ms"] / row["fp32ir"]["time_ms"]
        rows.append(row)
        log(f"c3 s={s} nu={nu}: fp64 {row['fp64']['time_ms']:.1f} ms ({row['fp64']['outer_iters']}), fp32ir "
            f"{row['fp32ir']['time_ms']:.1f} ms ({row['fp32ir']['outer_iters']}), inner error "
            f"{row['fp32_inner_error_dx']:.1e}")
    return rows


def extra_lanczos(lib, torch, c4_nsys):
    """Chebyshev bounds from 10 Lanczos steps with a 10% margin (Sec. 8 setup)
    against the Gershgorin bounds [0, 2] on the face-coefficient workloads:
    outer iterations and time to 1e-8 of the 128^3 differentiable-solve
    problem and of the batched workload."""
    import gen

    dev = torch.device("cuda:0")
    out = {}
    pr = gen.config5(0)
    b = torch.as_tensor(pr.rhs[0], device=dev)
    u = torch.as_tensor(gen.uniform(gen.rng(101), pr.n), device=dev)
    res = {}
    for kind in ("gershgorin", "lanczos"):
        with lib.Solver(lib.Operator.stencil(*pr.dims, pr.kx, pr.ky, pr.kz), pr.s, pr.nu, pr.lmin, pr.lmax) as sv:
            bounds = (pr.lmin, pr.lmax)
            if kind == "lanczos":
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                bounds = sv.lanczos_bounds(u, 10, 0.1)
                res["lanczos_ms"] = 1e3 * (time.perf_counter() - t0)
            x = torch.zeros_like(b)
            t, st = _timed_solve(sv, b, x, 1e-8, torch)
            res[kind] = {"bounds": list(bounds), "outer_iters": st.outer_iters, "time_ms": t, "status": st.status}
    out["c5_128"] = res
    probs = gen.config4(seed=0, nsys=c4_nsys)
    lo, hi = [], []
    for q, p in enumerate(probs):
        with lib.Solver(lib.Operator.stencil(*p.dims, p.kx, p.ky, p.kz), 16, 25, p.lmin, p.lmax,
                        autotune=False) as sv:
            uq = torch.as_tensor(gen.uniform(gen.rng(200 + q), p.n), device=dev)
            a, z = sv.lanczos_bounds(uq, 10, 0.1)
            lo.append(a)
            hi.append(z)
    ops = [lib.Operator.stencil(*p.dims, p.kx, p.ky, p.kz) for p in probs]
    bq = [torch.as_tensor(np.concatenate(p.rhs), device=dev) for p in probs]
    res = {}
    for kind, (l, h) in (("gershgorin", ([p.lmin for p in probs], [p.lmax for p in probs])), ("lanczos", (lo, hi))):
        with lib.BatchedSolver(ops, 8, 16, 25, l, h) as bs:
            x = [torch.zeros_like(v) for v in bq]
            bs.solve(bq, x, 1e-8, raise_on_error=False)
            for v in x:
                v.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = bs.solve(bq, x, 1e-8, raise_on_error=False)
            torch.cuda.synchronize()
            its = [p.outer_iters for p in st]
            res[kind] = {"time_ms": 1e3 * (time.perf_counter() - t0), "outer_iters_min": min(its),
                         "outer_iters_max": max(its), "outer_iters_median": float(np.median(its)),
                         "pairs_converged": sum(p.status == 0 for p in st)}
    out["c4_batched"] = res
    log(f"lanczos bounds: {out}")
    return out


def extra_paper27(lib, torch, N27):
    """The paper's own workload (Sec. 8): 27-point Poisson on 230^3 (12.2M
    unknowns), Chebyshev bounds from 10 Lanczos steps with a 10% margin, s in
    {10, 20}, nu in {6, 15, 30}, Jacobi instead of the paper's AMG: outer
    iterations to the paper's 1e-6 and to 1e-8, time, and the condition
    number of the first scaled Gram matrix for the Chebyshev and the monomial
    basis (Sec. 4)."""
    import gen

    dev = torch.device("cuda:0")
    pr = gen.paper27(0, N=N27)
    rows = []
    b = None
    u = torch.as_tensor(gen.uniform(gen.rng(41), pr.n), device=dev)
    for s in (10, 20):
        for nu in (6, 15, 30):
            row = {"s": s, "nu": nu}
            with lib.Solver(lib.Operator.stencil27(N27, N27, N27), s, nu, pr.lmin, pr.lmax, max_outer=1000) as sv:
                if b is None:
                    b = sv.apply(torch.as_tensor(pr.xstar, device=dev))
                row["bounds"] = list(sv.lanczos_bounds(u, 10, 0.1))
                x = torch.zeros_like(b)
                for tol in (1e-6, 1e-8):
                    t, st = _timed_solve(sv, b, x, tol, torch, reps=1, warm=(tol == 1e-6))
                    row[f"tol{tol:.0e}"] = {"outer_iters": st.outer_iters, "time_ms": t, "status": st.status,
                                            "rel_res": _finite(st.rel_res)}
                if nu == 30:
                    row["kappa_G_chebyshev"] = _kappa(sv, b, x)
            if nu == 30:
                with lib.Solver(lib.Operator.stencil27(N27, N27, N27), s, nu, *row["bounds"],
                                basis="monomial") as sv:
                    row["kappa_G_monomial"] = _kappa(sv, b, torch.zeros_like(b))
            rows.append(row)
            log(f"paper27 {row}")
    return rows


def extra_coarse(lib, torch):
    """The streaming coarse solve (Sec. 8, AMG and performance): nu_coarse = 20
    FGS sweeps on A_c = P^T A_f P of a two-level hierarchy with n_c = 17^3 =
    4913, A_c never formed against A_c formed on the device: time per coarse
    solve and the library workspace of each."""
    import gen

    dev = torch.device("cuda:0")
    tl = gen.two_level(0)
    f = torch.as_tensor(tl.f, device=dev)
    out = {"n_coarse": tl.n_coarse, "n_fine": int(np.prod(tl.nf)), "nu": tl.nu,
           "dense_A_c_bytes": 8 * tl.n_coarse ** 2}
    us = {}
    for formed in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cs = lib.CoarseSolver(lib.Operator.stencil(*tl.nf, tl.kx, tl.ky, tl.kz), formed=formed)
        setup = 1e3 * (time.perf_counter() - t0)
        u = cs.fgs(f, tl.nu)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cs.fgs(f, tl.nu, u)
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        us[formed] = u.clone()
        out["formed" if formed else "streamed"] = {"setup_ms": setup, "fgs_ms": float(np.median(ts)),
                                                   "workspace_bytes": cs.workspace_bytes}
        cs.close()
    out["streamed_vs_formed_rel_diff"] = float(torch.linalg.vector_norm(us[False] - us[True])
                                               / torch.linalg.vector_norm(us[True]))
    log(f"coarse {out}")
    return out


def sweep(lib, torch, args):
    """FP32+IR against FP64 on the headline problem for each (s, nu)."""
    import gen

    N = args.N
    dev = torch.device("cuda:0")
    rows = []
    b = None
    for s in (8, 16, 24, 32):
        for nu in (20, 30):
            pr = gen.config2(0, N=N, s=s, nu=nu)
            row = {"s": s, "nu": nu}
            for prec in ("fp64", "fp32ir"):
                with lib.Solver(lib.Operator.stencil(N, N, N), s, nu, pr.lmin, pr.lmax, precision=prec) as sv:
                    if b is None:
                        b = sv.apply(torch.as_tensor(pr.xstar, device=dev))
                    x = torch.zeros_like(b)
                    sv.solve(b, x, 1e-8)  # warm-up
                    ts = []
                    for _ in range(3):
                        x.zero_()
                        t0 = time.perf_counter()
                        _, st = sv.solve(b, x, 1e-8)
                        torch.cuda.synchronize()
                        ts.append(1e3 * (time.perf_counter() - t0))
                    w = 8 if prec == "fp64" else 4
                    t = float(np.median(ts))
                    bpo = stencil_bytes_per_outer(pr.n, s, w, sv.gram_kind, sv.basis_pairs)
                    row[prec] = {"time_ms": t, "outer_iters": st.outer_iters, "rel_res": st.rel_res,
                                 "gram": sv.gram_kind,
                                 "gbps_effective": bpo * st.outer_iters / (t * 1e-3) / 1e9}
            row["fp32ir_speedup"] = row["fp64"]["time_ms"] / row["fp32ir"]["time_ms"]
            rows.append(row)
            log(f"s={s} nu={nu}: {row}")
    print(json.dumps({"metric": METRIC + " (s, nu sweep)", "N": N, "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
