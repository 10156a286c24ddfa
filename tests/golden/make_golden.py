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


if __name__ == "__main__":
    main_c2() if "--c2" in sys.argv[1:] else main()
