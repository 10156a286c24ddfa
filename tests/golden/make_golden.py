"""Write tests/golden/c1_oracle.json from the oracle alone (no GPU code).

The fixture freezes the oracle's trajectory on the 2D 64 x 64 Poisson problem
(s = 8, nu = 20, seed 0, tol 1e-8): outer-iteration count, the relative
residual history and the first outer iteration's scaled FGS coefficients.  It
guards the oracle against unintended changes; any deliberate change to the
oracle's arithmetic regenerates it and says why in its commit message.
Run from the repository root: ``python tests/golden/make_golden.py``.

``--c2`` writes tests/golden/c2_oracle.json instead: the oracle's full solve of
the 224^3 Poisson problem (s = 16, nu = 25, seed 0, tol 1e-8), its outer
iteration count and relative residual history, which the full-size GPU test
compares against (the oracle takes minutes there, too long for a test).

``--c5`` writes tests/golden/c5_oracle_grad.json: the oracle's reference
gradient of the 128^3 differentiable solve (forward and adjoint at tol 1e-12),
as entries at fixed random positions plus full-vector norms.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402


def main():
    pr = gen.config1(0)
    A = pr.csr()
    b = oracle.spmv(A, pr.xstar)
    out = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, pr.tol, hist_cap=1000)
    first = oracle.step(A, b, np.zeros(pr.n), pr.s, pr.nu, pr.lmin, pr.lmax)
    data = {
        "what": "oracle trajectory, 2D 5-point Poisson 64x64, CSR, s=8, nu=20, Jacobi, exact bounds, "
                "x* ~ U[-1,1] seed 0, b = A x*, x0 = 0, tol 1e-8",
        "iters": out["iters"],
        "relres": out["relres"],
        "hist_relres": [float(v) for v in out["hist_relres"]],
        "atil_first": [float(v) for v in first["atil"]],
        "lmin": pr.lmin,
        "lmax": pr.lmax,
    }
    path = os.path.join(ROOT, "tests", "golden", "c1_oracle.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print(path, data["iters"])


def main_c2():
    pr = gen.config2(0)
    N = pr.dims[0]
    A = oracle.assemble_stencil7(N, N, N)
    b = oracle.spmv(A, pr.xstar)
    out = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, 1e-8, hist_cap=1000)
    data = {
        "what": f"oracle trajectory, 3D 7-point Poisson {N}^3, s={pr.s}, nu={pr.nu}, Jacobi, exact bounds, "
                "x* ~ U[-1,1] seed 0, b = A x*, x0 = 0, tol 1e-8",
        "status": out["status"],
        "iters": out["iters"],
        "relres": out["relres"],
        "hist_relres": [float(v) for v in out["hist_relres"]],
    }
    path = os.path.join(ROOT, "tests", "golden", "c2_oracle.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print(path, data["iters"])


def main_c5(nsample: int = 4096):
    """The differentiable solve's reference gradient: the 128^3 face problem
    (sigma 0.5, s = 16, nu = 25, Gershgorin bounds, seed 0), forward and adjoint
    solved by the oracle to tol 1e-12, L = 1/2 ||x - x_target||^2, so
    dL/db = lambda with A lambda = x - x_target and dL/dk_f from the face
    scatter.  The fixture keeps entries at fixed random positions (indices
    stored with them) and the full vectors' 2-norms."""
    pr = gen.config5(0)
    nx, ny, nz = pr.dims
    A = oracle.problem_csr(pr)
    b = pr.rhs[0]
    fw = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, 1e-12)
    x = fw["x"]
    g = x - pr.xtarget
    ad = oracle.solve(A, g, None, pr.s, pr.nu, pr.lmin, pr.lmax, 1e-12)
    lam = ad["x"]
    dk = np.concatenate(oracle.grad_faces(nx, ny, nz, lam, x))
    pick = np.random.default_rng(20251209)
    ik = np.sort(pick.choice(dk.size, nsample, replace=False))
    iv = np.sort(pick.choice(pr.n, nsample, replace=False))
    data = {
        "what": f"oracle gradient, 3D face-coefficient diffusion {nx}^3, sigma 0.5, s={pr.s}, nu={pr.nu}, Jacobi, "
                "Gershgorin bounds [0, 2], b and x_target ~ U[-1,1] seed 0, forward and adjoint to tol 1e-12, "
                "L = 1/2 ||x - x_target||^2; sampled entries of x, dL/db = lambda and dL/dk",
        "status": [fw["status"], ad["status"]],
        "iters": [fw["iters"], ad["iters"]],
        "norm_x": float(np.linalg.norm(x)),
        "norm_lam": float(np.linalg.norm(lam)),
        "norm_dk": float(np.linalg.norm(dk)),
        "loss": float(0.5 * g @ g),
        "idx_k": [int(v) for v in ik],
        "dk": [float(v) for v in dk[ik]],
        "idx_v": [int(v) for v in iv],
        "x": [float(v) for v in x[iv]],
        "lam": [float(v) for v in lam[iv]],
    }
    path = os.path.join(ROOT, "tests", "golden", "c5_oracle_grad.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=0)
    print(path, data["iters"])


if __name__ == "__main__":
    if "--c2" in sys.argv[1:]:
        main_c2()
    elif "--c5" in sys.argv[1:]:
        main_c5()
    else:
        main()
