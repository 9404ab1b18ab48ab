"""Krylov solvers of the oracle (test infrastructure).

Paper, domain-decomposition section: the system is solved by GMRES
preconditioned with the two-level ORAS preconditioner; the coarse problem is
itself solved by 10 GMRES iterations preconditioned with one-level ORAS.  Since
10 fixed inner iterations make the preconditioner a nonlinear map, the outer
solver is taken in its flexible, right-preconditioned form (FGMRES, Saad
2003).  Readings where the paper is silent: classical Gram-Schmidt applied
twice (CGS2) with the two coefficient sets accumulated; complex Givens
rotations; stop when the least-squares residual estimate |g_{j+1}| falls to
tol*||b||, then confirm with the true residual ||b - A x||/||b|| and restart
from x if it is still above tol; a happy breakdown when h_{j+1,j} <= 1e-14 times
the norm of A z_j before orthogonalisation; maxit counts outer iterations.
"""
from __future__ import annotations

import numpy as np

BREAKDOWN = 1e-14


def givens(a, b):
    """Complex Givens rotation G = [[c, s], [-conj(s), c]] with G [a, b]^T = [rho, 0]^T.

    rho = sqrt(|a|^2+|b|^2), c = |a|/rho, s = (a/|a|) conj(b)/rho; if a = 0: c = 0, s = 1.
    Returns (c, s, r) with r the new top entry.
    """
    if a == 0:
        return 0.0, 1.0 + 0j, b
    aa = abs(a)
    rho = np.sqrt(aa * aa + abs(b) ** 2)
    c = aa / rho
    s = (a / aa) * np.conj(b) / rho
    return c, s, (a / aa) * rho


def _cgs2(V, w):
    """Two classical Gram-Schmidt passes of w against the columns in V; returns (h, w)."""
    h = np.zeros(len(V), dtype=np.complex128)
    for _ in range(2):
        hp = np.array([np.vdot(v, w) for v in V])
        for i, v in enumerate(V):
            w = w - hp[i] * v
        h += hp
    return h, w


def _arnoldi_step(V, rot, g, j, z, w):
    """Orthogonalise w, apply the previous rotations and a new one; returns (hnext, wnorm0, w, col)."""
    wnorm0 = np.linalg.norm(w)
    h, w = _cgs2(V, w)
    hnext = np.linalg.norm(w)
    col = np.concatenate([h, [hnext]]).astype(np.complex128)
    for i, (c, s) in enumerate(rot):
        a, b = col[i], col[i + 1]
        col[i] = c * a + s * b
        col[i + 1] = -np.conj(s) * a + c * b
    c, s, r = givens(col[j], col[j + 1])
    col[j] = r
    col[j + 1] = 0.0
    rot.append((c, s))
    g[j + 1] = -np.conj(s) * g[j]
    g[j] = c * g[j]
    return hnext, wnorm0, w, col


def _back_solve(Hcols, g, k):
    """Solve the k x k upper-triangular system R y = g[:k] (R from the rotated columns)."""
    R = np.zeros((k, k), dtype=np.complex128)
    for j in range(k):
        R[: j + 1, j] = Hcols[j][: j + 1]
    y = np.zeros(k, dtype=np.complex128)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:] @ y[i + 1:]) / R[i, i]
    return y


def gmres_fixed(matvec, precond, c, nit=10):
    """Right-preconditioned GMRES from x0 = 0 with exactly nit iterations, no restart.

    Stops earlier only on a happy breakdown.  Returns x = sum_j y_j M^{-1} v_j.
    """
    beta = np.linalg.norm(c)
    if beta == 0.0:
        return np.zeros_like(c)
    V = [c / beta]
    Z = []
    rot = []
    g = np.zeros(nit + 1, dtype=np.complex128)
    g[0] = beta
    Hcols = []
    k = 0
    for j in range(nit):
        z = precond(V[j])
        w = matvec(z)
        Z.append(z)
        hnext, wnorm0, w, col = _arnoldi_step(V, rot, g, j, z, w)
        Hcols.append(col)
        k = j + 1
        if hnext <= BREAKDOWN * wnorm0:
            break
        V.append(w / hnext)
    y = _back_solve(Hcols, g, k)
    x = np.zeros_like(c)
    for i in range(k):
        x = x + y[i] * Z[i]
    return x


def fgmres(matvec, precond, b, tol, m, maxit, x0=None, history=None):
    """Right-preconditioned flexible GMRES(m) for one right-hand side.

    Returns (x, iters, relres_est, relres_true).  relres_est is |g_{j+1}|/||b||
    at exit, relres_true = ||b - A x||/||b|| in FP64.  ``history`` (a list)
    receives the estimate after every iteration.
    """
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0, 0.0
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    it = 0
    r = b - matvec(x) if x0 is not None else b.copy()
    est = np.linalg.norm(r) / nb
    while True:
        beta = np.linalg.norm(r)
        if beta <= tol * nb or it >= maxit:
            return x, it, est, beta / nb
        V = [r / beta]
        Z = []
        rot = []
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        Hcols = []
        k = 0
        for j in range(m):
            z = precond(V[j])
            w = matvec(z)
            Z.append(z)
            hnext, wnorm0, w, col = _arnoldi_step(V, rot, g, j, z, w)
            Hcols.append(col)
            it += 1
            k = j + 1
            est = abs(g[j + 1]) / nb
            if history is not None:
                history.append(est)
            if est <= tol or hnext <= BREAKDOWN * wnorm0 or it >= maxit:
                break
            V.append(w / hnext)
        y = _back_solve(Hcols, g, k)
        for i in range(k):
            x = x + y[i] * Z[i]
        r = b - matvec(x)


def block_fgmres(matvec, precond, B, tol, m, maxit, X0=None, history=None):
    """Right-preconditioned flexible block GMRES(m): one Krylov space shared by
    all right-hand sides (the columns of B, [n][s]).

    The many-sources setting of the paper (Summary, Introduction) read as a
    block method: the residual block is factored R0 = V_0 beta (QR); block j
    gives Z_j = M^{-1} V_j (column by column), W = A Z_j, two classical block
    Gram-Schmidt passes H_ij = V_i^H W, W -= V_i H_ij (coefficients
    accumulated), and W = V_{j+1} H_{j+1,j} (QR); the iterate minimises the
    Frobenius norm of E_1 beta - Hbar_j Y over Y (the block least-squares
    problem, numpy lstsq), each column's residual norm being that column of the
    least-squares residual.  Stop when every column is at tol ||b_r|| (or a
    breakdown: the smallest |diagonal| of H_{j+1,j} at most 1e-14 ||W|| before
    orthogonalisation; or maxit), form X += [Z_0 ..] Y, confirm with the true
    residual and restart from X while some column is above tol.  Zero columns
    of B are answered with zero and left out of the block.

    Returns (X, iters, relres_est, relres_true): iters counts block iterations
    (the same for every column of the block).
    """
    B = np.asarray(B, dtype=np.complex128)
    n, s = B.shape
    nb = np.linalg.norm(B, axis=0)
    act = nb > 0
    X = np.zeros_like(B) if X0 is None else X0.astype(np.complex128).copy()
    X[:, ~act] = 0.0
    it = np.zeros(s, dtype=np.int64)
    est = np.zeros(s)
    tru = np.zeros(s)
    if not act.any():
        return X, it, est, tru
    Ba, nba = B[:, act], nb[act]
    Xa = X[:, act]
    sa = Ba.shape[1]

    def block_apply(f, Y):
        return np.stack([f(Y[:, c]) for c in range(Y.shape[1])], axis=1)

    R = Ba - block_apply(matvec, Xa) if X0 is not None else Ba.copy()
    k = 0
    esta = np.linalg.norm(R, axis=0) / nba
    while True:
        rn = np.linalg.norm(R, axis=0)
        if np.all(rn <= tol * nba) or k >= maxit:
            X[:, act] = Xa
            it[act] = k
            est[act] = esta
            tru[act] = rn / nba
            return X, it, est, tru
        V0, beta = np.linalg.qr(R)
        Vs, Zs = [V0], []
        H = np.zeros(((m + 1) * sa, m * sa), dtype=np.complex128)
        for j in range(m):
            Z = block_apply(precond, Vs[j])
            W = block_apply(matvec, Z)
            Zs.append(Z)
            w0 = np.linalg.norm(W)
            for _ in range(2):
                for i, Vi in enumerate(Vs):
                    C = Vi.conj().T @ W
                    W = W - Vi @ C
                    H[i * sa:(i + 1) * sa, j * sa:(j + 1) * sa] += C
            Q, Rn = np.linalg.qr(W)
            H[(j + 1) * sa:(j + 2) * sa, j * sa:(j + 1) * sa] = Rn
            k += 1
            E = np.zeros(((j + 2) * sa, sa), dtype=np.complex128)
            E[:sa] = beta
            Hj = H[:(j + 2) * sa, :(j + 1) * sa]
            Y = np.linalg.lstsq(Hj, E, rcond=None)[0]
            esta = np.linalg.norm(E - Hj @ Y, axis=0) / nba
            if history is not None:
                history.append(esta.copy())
            breakdown = np.min(np.abs(np.diag(Rn))) <= BREAKDOWN * w0
            if np.all(esta <= tol) or breakdown or k >= maxit:
                break
            Vs.append(Q)
        for i, Z in enumerate(Zs):
            Xa = Xa + Z @ Y[i * sa:(i + 1) * sa]
        R = Ba - block_apply(matvec, Xa)
