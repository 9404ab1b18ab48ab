"""Block FGMRES on the GPU (HELM_BLOCK: one Krylov space shared by the
right-hand sides of a batch) against the oracle's block_fgmres, through the C
ABI: same block iteration count, each solution within 10 x tol of the
oracle's and at the FP64 true residual recomputed with the oracle's A."""
import numpy as np
import pytest

import inputs
from oracle.krylov import block_fgmres
from oracle.operator import Pml, Problem, fit_weights
from oracle.solve import setup as oracle_setup
from oracle.solve import solve as oracle_solve

pytestmark = pytest.mark.gpu

WO = fit_weights()
W = {k: getattr(WO, k) for k in ("w1", "w2", "w3", "wm1", "wm2", "wm3", "wm4")}


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _case(shape=(28, 26, 24)):
    h, f = 25.0, 10.0
    c = inputs.velocity_thrust_belt(*shape, h=h)
    return shape, h, c, f


@pytest.mark.parametrize("levels,restart", [(2, 20), (1, 6)])
def test_block_fgmres_matches_oracle(levels, restart):
    from paper_2103_14921_amd import helm
    shape, h, c, f = _case()
    tol = 1e-8
    src = inputs.source_grid(shape[0], shape[1], 5, 5, 3, 2, iz=4)
    b = inputs.point_source_rhs(*shape, src).reshape(len(src), -1)
    prob = Problem(shape, h, c, f, Pml(5, 5, 5, 0), WO)
    st = oracle_setup(prob, (2, 2, 2), 2, levels)
    Xo, ito, esto, truo = block_fgmres(lambda v: st.A @ v, st.M.apply, b.T.copy(), tol, restart, 400)
    say("block", levels, restart, "oracle block iterations", ito)
    S = helm.Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=levels,
                    restart=restart)
    X, info = S.solve(b, tol=tol, maxit=400, block=True)
    say("gpu block iterations", info["iters"])
    assert list(info["iters"]) == list(ito)
    for r in range(len(src)):
        assert rel(X[r], Xo[:, r]) <= 10 * tol
        assert info["relres_true"][r] <= tol
        res = b[r] - st.A @ X[r]
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= tol
    S.close()


def test_block_fgmres_zero_rhs_and_single_column():
    from paper_2103_14921_amd import helm
    shape, h, c, f = _case()
    tol = 1e-8
    b = inputs.point_source_rhs(*shape, [(6, 6, 4), (14, 13, 4), (21, 19, 4)]).reshape(3, -1)
    B = np.concatenate([b[:1], np.zeros_like(b[:1]), b[1:]], 0)
    S = helm.Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=20)
    say("block with a zero right-hand side")
    X, info = S.solve(B, tol=tol, maxit=400, block=True)
    assert info["iters"][1] == 0 and not np.any(X[1]) and info["relres_true"][1] == 0
    assert len(set(int(i) for i in np.delete(info["iters"], 1))) == 1
    assert np.all(info["relres_true"] <= tol)
    # one column: block FGMRES is FGMRES
    say("block of one")
    X1, i1 = S.solve(b[:1], tol=tol, maxit=400, block=True)
    X2, i2 = S.solve(b[:1], tol=tol, maxit=400)
    assert int(i1["iters"][0]) == int(i2["iters"][0])
    assert rel(X1[0], X2[0]) <= 1e-9
    S.close()


def test_block_fgmres_fewer_iterations_than_separate_spaces():
    from paper_2103_14921_amd import helm
    shape, h, c, f = _case((40, 40, 32))
    tol = 1e-6
    src = inputs.source_grid(shape[0], shape[1], 6, 6, 4, 4, iz=4)
    b = inputs.point_source_rhs(*shape, src).reshape(len(src), -1)
    S = helm.Solver(shape, h, c, f, (6, 6, 6, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=20)
    Xs, iseparate = S.solve(b, tol=tol, maxit=400)
    Xb, iblock = S.solve(b, tol=tol, maxit=400, block=True)
    say("separate", iseparate["iters"], "block", iblock["iters"])
    assert np.all(iblock["relres_true"] <= tol)
    assert iblock["iters"].max() < iseparate["iters"].mean()
    for r in range(len(src)):
        assert rel(Xb[r], Xs[r]) <= 1e-4
    S.close()
