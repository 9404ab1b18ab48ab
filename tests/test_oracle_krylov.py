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


# ---- block FGMRES (one Krylov space shared by the right-hand sides) ----------

def _dense_system(n=40, s=5, seed=11):
    rng = np.random.default_rng(seed)
    A = np.diag(np.linspace(1, 4, n)) + 0.4 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    B = rng.standard_normal((n, s)) + 1j * rng.standard_normal((n, s))
    P = np.diag(1.0 / (1.0 + 0.05 * np.arange(n)))
    return A, B, P


def test_block_fgmres_solves_dense_systems_with_restarts():
    from oracle.krylov import block_fgmres
    A, B, P = _dense_system()
    X, it, est, tru = block_fgmres(lambda v: A @ v, lambda v: P @ v, B, 1e-10, 3, 500)
    ref = np.linalg.solve(A, B)
    assert np.all(tru <= 1e-10) and np.all(it == it[0])
    assert np.linalg.norm(X - ref) <= 1e-8 * np.linalg.norm(ref)


def test_block_fgmres_is_minimal_residual_over_the_block_krylov_space():
    # after k block steps without restart, X minimises ||B - A X||_F over the
    # block Krylov space P [R, (AP) R, ..., (AP)^(k-1) R] (explicit basis, QR, lstsq)
    from oracle.krylov import block_fgmres
    A, B, P = _dense_system(n=60, s=3, seed=2)
    AP = A @ P
    for k in (1, 2, 4):
        X, it, est, tru = block_fgmres(lambda v: A @ v, lambda v: P @ v, B, 0.0, 10, k)
        assert it[0] == k
        K = [B]
        for _ in range(k - 1):
            K.append(AP @ K[-1])
        Q, _ = np.linalg.qr(np.concatenate(K, axis=1))
        Y = np.linalg.lstsq(AP @ Q, B, rcond=None)[0]
        Xref = P @ (Q @ Y)
        assert np.linalg.norm(X - Xref) <= 1e-8 * np.linalg.norm(Xref)
        assert np.allclose(np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0), tru, rtol=1e-8)


def test_block_fgmres_with_one_column_is_fgmres():
    from oracle.krylov import block_fgmres
    A, B, P = _dense_system(s=1, seed=7)
    hb, hs = [], []
    X, it, est, tru = block_fgmres(lambda v: A @ v, lambda v: P @ v, B, 1e-9, 5, 200, history=hb)
    x, its, ests, trus = fgmres(lambda v: A @ v, lambda v: P @ v, B[:, 0], 1e-9, 5, 200, history=hs)
    assert it[0] == its
    assert np.linalg.norm(X[:, 0] - x) <= 1e-10 * np.linalg.norm(x)
    assert np.allclose([h[0] for h in hb], hs, rtol=1e-7)


def test_block_fgmres_zero_columns_and_maxit():
    from oracle.krylov import block_fgmres
    A, B, P = _dense_system(s=3, seed=3)
    B[:, 1] = 0.0
    X, it, est, tru = block_fgmres(lambda v: A @ v, lambda v: P @ v, B, 1e-12, 4, 3)
    assert it[1] == 0 and not np.any(X[:, 1]) and tru[1] == 0
    assert it[0] == it[2] == 3 and tru[0] > 1e-12
