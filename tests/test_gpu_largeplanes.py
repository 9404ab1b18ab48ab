"""FP64 two-level end-to-end parity against the oracle with the plane size of
the 128^3 FP64 workload: boxes of 34^2 core nodes per plane extended to 36 x 36
= 1296-node planes (the domain-decomposition section's local problems; FGMRES
with the two-level ORAS preconditioner of eq. 2lvl)."""
import numpy as np
import pytest

import inputs
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


@pytest.mark.timeout(600)
def test_fp64_two_level_parity_with_1296_node_planes():
    from paper_2103_14921_amd import helm
    shape, h, f, tol, pml = (68, 68, 8), 25.0, 10.0, 1e-8, (8, 8, 3, 0)
    c = inputs.velocity_thrust_belt(*shape, h=h)
    src = inputs.source_grid(shape[0], shape[1], 8, 8, 2, 1, iz=3)
    b = inputs.point_source_rhs(*shape, src)
    say("oracle set-up", shape, "parts (2, 2, 1)")
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    st = oracle_setup(prob, (2, 2, 1), 2, 2)
    say("oracle solve")
    ref = oracle_solve(st, b, tol, 30, 300)
    say("gpu solve")
    S = helm.Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 1), overlap=2, levels=2, restart=30,
                    precision="fp64")
    box = S.subdomain_box(0, 0)
    ex, ey = box["ehi"][0] - box["elo"][0], box["ehi"][1] - box["elo"][1]
    assert ex * ey == 1296
    X, info = S.solve(b, tol=tol, maxit=300)
    say("iters gpu", info["iters"], "oracle", ref["iters"])
    assert list(info["iters"]) == list(ref["iters"])
    for r in range(len(src)):
        assert rel(X[r], ref["X"][r]) <= 10 * tol
        assert info["relres_true"][r] <= tol
        res = b[r].ravel() - st.A @ X[r].ravel()
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= tol
    S.close()


@pytest.mark.timeout(600)
def test_sweep_with_operand_in_global_memory_matches_oracle():
    # 36 x 36 = 1296-node planes: the operand of a plane product no longer fits
    # in LDS (complex FP64 or FP32), so the sweep keeps it in global memory; 12
    # right-hand sides make one full and one partial group of 8
    from oracle.dd import Oras, decompose
    from oracle.operator import assemble
    from paper_2103_14921_amd import helm
    shape, h, f, pml = (68, 68, 8), 25.0, 10.0, (8, 8, 3, 0)
    c = inputs.velocity_thrust_belt(*shape, h=h, q=100.0)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    say("oracle one-level ORAS", shape)
    M = Oras(assemble(prob), shape, decompose(shape, (2, 2, 1), 2), prob.k().ravel(), h)
    R = inputs.random_field((12, prob.n), seed=61)
    ref = np.stack([M.apply(R[r]) for r in range(12)])
    for prec, tol in (("fp64", 1e-10), ("mixed", 5e-4)):
        say("gpu sweep", prec)
        S = helm.Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 1), overlap=2, levels=1, precision=prec)
        Z = S.apply_oras(R)
        for r in range(12):
            assert rel(Z[r], ref[r]) <= tol, (prec, r)
        S.close()
