"""Whole oracle solve for many right-hand sides (test infrastructure).

Setup = assembly of A + local operators + banded LU factorisations (the
paper's "setup" column of Table 2); solve = FGMRES per right-hand side, each
with its own Krylov space (the paper's T_GM column).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from .coarse import TwoLevel
from .dd import Oras, decompose
from .krylov import fgmres
from .operator import Problem, assemble


@dataclass
class Setup:
    prob: Problem
    A: object
    M: object
    boxes: list
    t_setup: float


def setup(prob: Problem, parts, delta=2, levels=1, robin=True, coarse_iters=10, workers=1):
    t0 = time.perf_counter()
    A = assemble(prob)
    k = prob.k().ravel()
    boxes = decompose(prob.shape, parts, delta)
    if levels == 1:
        M = Oras(A, prob.shape, boxes, k, prob.h, robin, workers)
    elif levels == 2:
        M = TwoLevel(A, prob.shape, boxes, k, prob.h, delta, robin, coarse_iters, workers)
    else:
        raise ValueError("levels must be 1 or 2")
    return Setup(prob, A, M, boxes, time.perf_counter() - t0)


def solve(st: Setup, B, tol, m, maxit, X0=None):
    """Solve A X[r] = B[r] for every right-hand side r (B: [nrhs][nz][ny][nx] or [nrhs][n]).

    Returns dict(X, iters, relres_est, relres_true, t_solve, history).
    """
    nrhs = B.shape[0]
    Bf = B.reshape(nrhs, -1)
    X = np.zeros_like(Bf)
    iters = np.zeros(nrhs, dtype=np.int64)
    est = np.zeros(nrhs)
    tru = np.zeros(nrhs)
    hist = []
    t0 = time.perf_counter()
    for r in range(nrhs):
        h = []
        x0 = None if X0 is None else X0.reshape(nrhs, -1)[r]
        X[r], iters[r], est[r], tru[r] = fgmres(lambda v: st.A @ v, st.M.apply, Bf[r], tol, m, maxit,
                                                 x0=x0, history=h)
        hist.append(h)
    t = time.perf_counter() - t0
    return dict(X=X.reshape(B.shape), iters=iters, relres_est=est, relres_true=tru, t_solve=t,
                history=hist)
