"""Pins of the oracle's Givens rotations and FGMRES (CPU only)."""
import numpy as np

from oracle.krylov import fgmres, givens


def test_givens_zeroes_and_is_unitary():
    rng = np.random.default_rng(2)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s, r = givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([a, b])
        assert abs(out[1]) < 1e-14 * abs(a)
        assert abs(out[0] - r) < 1e-14 * abs(r)
        assert np.allclose(G.conj().T @ G, np.eye(2), atol=1e-14)
    c, s, r = givens(0.0, 2.0 - 1.0j)
    assert c == 0.0 and s == 1.0 and r == 2.0 - 1.0j


def _system(n=80, seed=4):
    rng = np.random.default_rng(seed)
    A = np.diag(np.linspace(1, 4, n) * np.exp(1j * np.linspace(0, 2.5, n)))
    A = A + 0.5 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_fgmres_solves_dense_system_with_restarts():
    A, b = _system()
    x, it, est, tru = fgmres(lambda v: A @ v, lambda v: v, b, 1e-10, 15, 500)
    xd = np.linalg.solve(A, b)
    assert tru <= 1e-10
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert it > 15   # at least one restart happened


def test_fgmres_residual_history_is_minimal_residual():
    # with a fixed preconditioner and no restart, |g_{j+1}| equals
    # min_y ||b - A P K_j y|| over the j-dimensional Krylov space of A P
    A, b = _system(n=50, seed=8)
    P = np.diag(1.0 / np.diag(A))
    hist = []
    fgmres(lambda v: A @ v, lambda v: P @ v, b, 1e-30, 12, 12, history=hist)
    AP = A @ P
    nb = np.linalg.norm(b)
    K = np.zeros((50, 12), complex)
    v = b / nb
    for j in range(12):
        K[:, j] = v
        v = AP @ v
        v /= np.linalg.norm(v)
    for j in range(1, 13):
        Q, _ = np.linalg.qr(K[:, :j])
        y, *_ = np.linalg.lstsq(AP @ Q, b, rcond=None)
        ref = np.linalg.norm(b - AP @ Q @ y) / nb
        assert abs(hist[j - 1] - ref) <= 1e-8 * max(ref, 1e-12) + 1e-13


def test_fgmres_zero_rhs_and_initial_guess():
    A, b = _system(n=20)
    x, it, est, tru = fgmres(lambda v: A @ v, lambda v: v, np.zeros(20, complex), 1e-8, 5, 10)
    assert it == 0 and np.all(x == 0)
    xd = np.linalg.solve(A, b)
    x, it, est, tru = fgmres(lambda v: A @ v, lambda v: v, b, 1e-8, 5, 10, x0=xd)
    assert it == 0 and tru <= 1e-8


def test_fgmres_maxit_reports_not_converged():
    A, b = _system()
    x, it, est, tru = fgmres(lambda v: A @ v, lambda v: v, b, 1e-14, 5, 3)
    assert it == 3 and tru > 1e-14 and abs(est - tru) <= 1e-10
