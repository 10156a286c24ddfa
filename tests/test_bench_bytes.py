"""The benchmark's algorithmic byte counts, pinned to counts made by hand
from the kernels' reads and writes (every column read or written once per
launch; FP64 w = 8, FP32 w = 4).  These figures are the numerators of every
bandwidth the benchmark reports, including the roofline's."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_basis_vectors_single_steps():
    # s = 4, stored AP: p1 <- p0 (r1 w2: p1, Ap0), p2 <- p1, p0 (r2 w2),
    # p3 <- p2, p1 (r2 w2), Ap3 <- p3 (r1 w1): 3 + 4 + 4 + 2 = 13 = 4s - 3
    assert bench.basis_vectors(4, "stored") == 13
    # apply kind, s = 4: p1 (2), p2 (3), p3 (3) = 8 = 3s - 4
    assert bench.basis_vectors(4, "apply") == 8
    # recurrence kind, s = 4: p1 (2), p2, p3, p4 (3 each) = 11 = 3s - 1
    assert bench.basis_vectors(4, "recurrence") == 11
    # the moments kind forms the same columns
    assert bench.basis_vectors(4, "moments") == 11


def test_basis_vectors_pairs():
    # recurrence, s = 16: (p1, p2) <- p0 (3), seven pairs (4 each) = 31
    assert bench.basis_vectors(16, "recurrence", pairs=8) == 31
    # apply, s = 16: 15 columns = seven pairs (3 + 6 * 4) + one single step (3)
    assert bench.basis_vectors(16, "apply", pairs=7) == 30
    # recurrence, s = 7: three pairs (3 + 4 + 4) + one single step (3)
    assert bench.basis_vectors(7, "recurrence", pairs=3) == 14
    # s = 2: the first pair only
    assert bench.basis_vectors(2, "recurrence", pairs=1) == 3


@pytest.mark.parametrize("kind,pairs,expect", [
    # 32 = x read by the residual (8), b (8), x read and written by the update (16)
    ("stored", 0, 32 + 8 * (1 + 61 + 32 + 16)),
    ("apply", 0, 32 + 8 * (1 + 44 + 16 + 16)),
    ("recurrence", 0, 32 + 8 * (1 + 47 + 17 + 16)),
    ("recurrence", 8, 32 + 8 * (1 + 31 + 17 + 16)),
    ("apply", 7, 32 + 8 * (1 + 30 + 16 + 16)),
    # moments: no Gram pass over the columns
    ("moments", 8, 32 + 8 * (1 + 31 + 0 + 16)),
])
def test_stencil_bytes_per_outer(kind, pairs, expect):
    assert bench.stencil_bytes_per_outer(1, 16, 8, kind, pairs) == expect


def test_moments_drop_the_diagonal_read():
    # the CSR and face figures count the M diagonal for the Gram kernel's
    # right-hand side; the moments kind takes the weights from the operator
    n, nnz, s = 1000, 7000, 16
    assert (bench.csr_bytes_per_outer(n, nnz, s, 8, "recurrence", 8)
            - bench.csr_bytes_per_outer(n, nnz, s, 8, "moments", 8)) == n * 8 * (17 + 1)
    assert (bench.faces_bytes_per_outer(n, s, 8, 1, "recurrence")
            - bench.faces_bytes_per_outer(n, s, 8, 1, "moments")) == n * 8 * (17 + 1)


def test_batched_system_bytes():
    n, s = 1000, 16
    # single steps, recurrence kind: 47 basis vectors, 17 Gram columns, the M
    # diagonal; faces read by the residual (3 x 8) and 16 launches (3 arrays)
    per, shared = bench.batched_system_bytes(n, s, 8, "recurrence", 0)
    assert per == n * (32 + 8 * (1 + 47 + 17 + 16)) + n * 8
    assert shared == n * (24 + 16 * 3 * 8)
    # two steps per launch, moments kind: 31 basis vectors, no Gram pass, no
    # diagonal; 8 launches reading the faces and the Jacobi weights
    per, shared = bench.batched_system_bytes(n, s, 8, "moments", 8)
    assert per == n * (32 + 8 * (1 + 31 + 0 + 16))
    assert shared == n * (24 + 8 * 4 * 8)


def test_basis_bytes_per_launch():
    n = 224 ** 3
    # the headline basis: 8 pair launches moving 31 vectors of n doubles
    assert bench.basis_bytes_per_launch(n, 16, 8, "recurrence", pairs=8, launches=8) == n * 8 * 31 / 8
    # single steps of the recurrence kind: 16 launches, 47 vectors
    assert bench.basis_bytes_per_launch(n, 16, 8, "recurrence") == n * 8 * 47 / 16
