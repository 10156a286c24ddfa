"""The moments Gram kind's arithmetic on the CPU, against the oracle's G.

The GPU path's moments kind never forms P^T A P directly.  It keeps, per basis
column, two M inner products, d_i = <p_i, M p_i> and e_i = <p_i, M p_{i-1}>.
The Chebyshev product rule T_i T_j = (T_{i+j} + T_{|i-j|}) / 2 turns those
into the moments mu_0 .. mu_2s, and then into H_ij = <p_i, M p_j> =
(mu_{i+j} + mu_{|i-j|}) / 2 for the basis p_0 .. p_s of Sec. 2 (Definition).
The recurrence then maps H onto G_raw = P^T A P, and c_i = <p_i, M p_0> =
mu_i.

These tests restate that chain in NumPy on the oracle's own basis columns.
They check it against the oracle's G_raw, formed directly, and against P^T r.
A wrong index in the moment formulas, a dropped weight or a wrong recurrence
coefficient fails them.  They cover Jacobi with p_0 = M^{-1} r and no
preconditioner (M = I), the cases the kind accepts, and widths 1 to 16."""
import numpy as np
import pytest

import gen
import oracle


def csr_matrix(A):
    import scipy.sparse as sp
    rp, ci, v = A
    n = rp.size - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def gram_from_moments(P, w, theta, sigma):
    """G_raw (s x s) and c (s) of the columns p_0 .. p_s (rows of P), from
    the 2s + 1 products alone."""
    s = P.shape[0] - 1
    d = np.array([np.dot(P[i], w * P[i]) for i in range(s + 1)])
    e = np.array([np.nan] + [np.dot(P[i], w * P[i - 1]) for i in range(1, s + 1)])
    mu = np.empty(2 * s + 1)
    for k in range(2 * s + 1):
        if k <= 1:
            mu[k] = d[0] if k == 0 else e[1]
        elif k % 2 == 0:
            mu[k] = 2.0 * d[k // 2] - mu[0]
        else:
            mu[k] = 2.0 * e[(k + 1) // 2] - mu[1]
    H = np.array([[0.5 * (mu[i + j] + mu[abs(i - j)]) for j in range(s + 1)] for i in range(s + 1)])
    G = np.empty((s, s))
    for i in range(s):
        for j in range(s):
            if j == 0:
                G[i, j] = H[i, 1] / theta + sigma * H[i, 0]
            else:
                G[i, j] = (H[i, j + 1] + H[i, j - 1]) / (2.0 * theta) + sigma * H[i, j]
    return G, mu[:s]


PROBLEMS = {
    "poisson_12x10x9": lambda: gen.small_poisson3d(12, 10, 9, seed=1),
    "faces_9x8x7": lambda: gen.small_faces3d(9, 8, 7, seed=2, sigma=1.0),
    "poisson2d_64x64_csr": lambda: gen.config1(0),
}


@pytest.mark.parametrize("name", [k for k in PROBLEMS])
@pytest.mark.parametrize("s", [1, 2, 3, 8, 16])
@pytest.mark.parametrize("precond", [1, 0])
def test_moments_give_the_oracle_gram(name, s, precond):
    pr = PROBLEMS[name]()
    A = oracle.problem_csr(pr)
    M = csr_matrix(A)
    n = pr.n
    b = np.random.default_rng(5).uniform(-1.0, 1.0, n)
    x0 = np.random.default_rng(6).uniform(-1.0, 1.0, n) * 0.1
    lmin, lmax = (pr.lmin, pr.lmax) if precond else (0.0, 2.0 * float(np.max(np.abs(M).sum(axis=1))))
    o = oracle.step(A, b, x0, s, 5, lmin, lmax, precond=precond, want_basis=True)
    assert o["status"] == 0
    theta = 2.0 / (lmax - lmin)
    sigma = (lmax + lmin) / 2.0
    diag = M.diagonal()
    dinv = 1.0 / diag if precond else np.ones(n)
    # p_s by the recurrence of Sec. 2 (Definition), from the oracle's columns
    P = o["P"]
    y = M @ P[s - 1]
    if s == 1:
        ps = theta * (dinv * y - sigma * P[0])
    else:
        ps = 2.0 * theta * (dinv * y - sigma * P[s - 1]) - P[s - 2]
    Pall = np.vstack([P, ps])
    w = diag if precond else np.ones(n)
    G, c = gram_from_moments(Pall, w, theta, sigma)
    Graw = o["Graw"]
    assert np.linalg.norm(G - Graw) <= 1e-12 * np.linalg.norm(Graw), np.linalg.norm(G - Graw) / np.linalg.norm(Graw)
    r = b - M @ x0
    c_direct = P @ r
    assert np.linalg.norm(c - c_direct) <= 1e-12 * np.linalg.norm(c_direct)


def test_a_wrong_moment_index_is_caught():
    """The same chain with mu_{2i-1} taken from mu_0 instead of mu_1 misses the
    oracle's G by far more than rounding."""
    pr = gen.small_faces3d(9, 8, 7, seed=2, sigma=1.0)
    A = oracle.problem_csr(pr)
    M = csr_matrix(A)
    n, s = pr.n, 6
    b = np.random.default_rng(5).uniform(-1.0, 1.0, n)
    o = oracle.step(A, b, np.zeros(n), s, 5, pr.lmin, pr.lmax, want_basis=True)
    theta, sigma = 2.0 / (pr.lmax - pr.lmin), (pr.lmax + pr.lmin) / 2.0
    P, diag = o["P"], M.diagonal()
    ps = 2.0 * theta * ((M @ P[s - 1]) / diag - sigma * P[s - 1]) - P[s - 2]
    Pall = np.vstack([P, ps])
    d = np.array([np.dot(Pall[i], diag * Pall[i]) for i in range(s + 1)])
    e = np.array([0.0] + [np.dot(Pall[i], diag * Pall[i - 1]) for i in range(1, s + 1)])
    mu = np.empty(2 * s + 1)
    mu[0], mu[1] = d[0], e[1]
    for k in range(2, 2 * s + 1):
        mu[k] = 2.0 * (d[k // 2] if k % 2 == 0 else e[(k + 1) // 2]) - mu[0]  # wrong for odd k
    H = np.array([[0.5 * (mu[i + j] + mu[abs(i - j)]) for j in range(s + 1)] for i in range(s + 1)])
    assert np.linalg.norm(H[:s, :s] - P @ (diag[:, None] * P.T)) > 1e-3 * np.linalg.norm(H)
