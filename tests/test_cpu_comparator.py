"""The host-core comparator (plain restarted Arnoldi, C++/OpenMP) against closed-form exp(-tA) b.

The comparator is timed beside the GPU solver; these tests pin its result to the oracle's exact
solutions, so its timing is of a method that reaches the same accuracy.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import exact

cpu = pytest.importorskip("cpu_baseline")


@pytest.fixture(scope="module", autouse=True)
def _built():
    import os
    if not os.path.exists(cpu.LIB):
        cpu.build()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N,t,m", [(32, 1e-3, 20), (48, 1e-3, 8)])
def test_plain_cpu_laplacian_matches_sine_closed_form(N, t, m):
    """m = 20 converges in about two cycles; m = 8 needs several (the restart recursion is used)."""
    A = wl.laplacian_2d(N)
    b = wl.gaussian_vector(A.n, 0)
    x, info = cpu.expv(A.rowptr, A.colind, A.vals, b, t, m, tol=1e-12, max_cycles=200)
    ref = exact.sine_fab("exp", b, N, [1, 1], t=t)
    assert info["status"] == "converged", info
    if m == 8:
        assert info["cycles"] >= 3
    assert _rel(x, ref) <= 1e-10


def test_plain_cpu_nonsymmetric_matches_kronecker_exp():
    """Convection-diffusion (Pe = 50): the Kronecker product of 1-D exponentials."""
    N, pe, t = 12, 50.0, 1e-3
    A = wl.convdiff_3d(N, pe)
    b = wl.gaussian_vector(A.n, 1)
    x, info = cpu.expv(A.rowptr, A.colind, A.vals, b, t, 20, tol=1e-12, max_cycles=100)
    ref = exact.kron_exp_fab(b, [exact.convdiff_factor(N, pe)] * 3, t)
    assert info["status"] == "converged", info
    assert _rel(x, ref) <= 1e-10


def test_plain_cpu_breakdown_is_exact():
    """b an eigenvector: the first step breaks down and the result is exp(-t lambda) b."""
    N, t = 16, 1e-3
    Phi, lam = exact.sine_basis(N)
    b = np.kron(Phi[:, 2], Phi[:, 4])
    A = wl.laplacian_2d(N)
    x, info = cpu.expv(A.rowptr, A.colind, A.vals, b, t, 10, tol=1e-12)
    assert info["status"] == "breakdown" and info["matvecs"] == 1, info
    assert _rel(x, np.exp(-t * (lam[2] + lam[4])) * b) <= 1e-12


def test_plain_cpu_rejects_bad_arguments():
    A = wl.laplacian_2d(8)
    b = wl.gaussian_vector(A.n, 0)
    with pytest.raises(ValueError):
        cpu.expv(A.rowptr, A.colind, A.vals, b, -1.0, 10, tol=1e-8)
    with pytest.raises(ValueError):
        cpu.expv(A.rowptr[:-1], A.colind, A.vals, b, 1e-3, 10, tol=1e-8)
