"""The two-level coarse solve (Sec. 6; Sec. 8, "AMG and performance") on the
GPU, through the C ABI, against the oracle, which forms A_c = P^T A_f P and
runs the natural-order Gauss-Seidel sweeps sequentially: the streamed variant
(A_c never formed) and the formed variant agree with it to 1e-10, entry by
entry, on ragged grids, the paper's n_c of about 5000 (17^3) and a larger
hierarchy; nu = 0 and nu = 1 edge cases; argument errors."""
import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def fine_operator(hip, tl, constant=False):
    if constant:
        return hip.Operator.stencil(*tl.nf)
    return hip.Operator.stencil(*tl.nf, tl.kx, tl.ky, tl.kz)


CASES = {
    "paper_nc_17": dict(seed=0, nc=(17, 17, 17), sigma=1.0, nu=20),
    "ragged": dict(seed=1, nc=(9, 5, 7), sigma=0.5, nu=20),
    "thin": dict(seed=2, nc=(1, 6, 3), sigma=1.0, nu=7),
    "larger": dict(seed=3, nc=(31, 29, 33), sigma=1.0, nu=20),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("formed", [False, True])
def test_coarse_fgs_matches_oracle(hip, name, formed):
    c = CASES[name]
    tl = gen.two_level(c["seed"], nc=c["nc"], sigma=c["sigma"], nu=c["nu"])
    want, _ = oracle.coarse_fgs(tl.nc, tl.kx, tl.ky, tl.kz, tl.f, tl.nu)
    with hip.CoarseSolver(fine_operator(hip, tl), formed=formed) as cs:
        assert cs.n == tl.n_coarse
        got = cs.fgs(t64(tl.f), tl.nu).cpu().numpy()
    assert rel(got, want) <= 1e-10, (name, formed, rel(got, want))


def test_coarse_constant_fine_operator_and_sweep_counts(hip):
    """Constant fine coefficients (A_f the 7-point Poisson matrix); nu = 0
    returns zeros, nu = 1 is one sweep."""
    tl = gen.two_level(4, nc=(6, 7, 5))
    ones = [np.ones_like(tl.kx), np.ones_like(tl.ky), np.ones_like(tl.kz)]
    for formed in (False, True):
        with hip.CoarseSolver(fine_operator(hip, tl, constant=True), formed=formed) as cs:
            for nu in (0, 1, 3):
                want, _ = oracle.coarse_fgs(tl.nc, *ones, tl.f, nu)
                got = cs.fgs(t64(tl.f), nu).cpu().numpy()
                if nu == 0:
                    assert np.all(got == 0.0)
                else:
                    assert rel(got, want) <= 1e-10, (formed, nu)


def test_coarse_streamed_uses_less_memory_and_errors(hip):
    tl = gen.two_level(0)
    with hip.CoarseSolver(fine_operator(hip, tl), formed=False) as s, \
            hip.CoarseSolver(fine_operator(hip, tl), formed=True) as f:
        n_c = s.n
        # streamed: a_jj + tables + the fine vector; formed: 27 entries per row
        assert f.workspace_bytes >= 27 * 8 * n_c
        print(f"n_c = {n_c}: workspace streamed {s.workspace_bytes} B, formed {f.workspace_bytes} B, "
              f"dense A_c would be {8 * n_c * n_c} B")
    with pytest.raises(hip.SStepError):
        hip.CoarseSolver(hip.Operator.stencil(34, 35, 35))  # even fine side
    with pytest.raises(hip.SStepError):
        hip.CoarseSolver(hip.Operator.stencil27(35, 35, 35))
