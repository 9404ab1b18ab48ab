"""The implementations of the batched local solves against the oracle.

The one-workgroup-per-box sweep, the pipelined persistent sweep (two boxes
per compute unit), the one-workgroup-per-box sweep built for two
workgroups per compute unit (FP64, groups of 32) and the paired sweep (two
right-hand-side groups of a box per workgroup; 20 and 40 right-hand sides
pair; at 64 two pairs per box), and the sweeps with the plane solutions
kept in LDS (complex FP64 paired at 20 and 64 right-hand sides, one group
otherwise and in complex FP32) are forced in turn through the process-wide
sweep policy, on right-hand-side batches that use full and partial groups of 16 and 32
columns, on the fine level (FP64 and complex FP32 factors) and on the coarse
level; each result is compared with the oracle's one-level ORAS applied per
right-hand side.
"""
import numpy as np
import pytest

import inputs
from oracle.coarse import TwoLevel
from oracle.dd import Oras, decompose
from oracle.operator import Pml, Problem, assemble, fit_weights

pytestmark = pytest.mark.gpu

WO = fit_weights()
W = {k: getattr(WO, k) for k in ("w1", "w2", "w3", "wm1", "wm2", "wm3", "wm4")}


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(autouse=True)
def _restore_policy():
    from paper_2103_14921_amd import helm
    yield
    helm.set_sweep_policy("auto")


@pytest.mark.parametrize("policy", ["item", "pipelined", "two_per_cu", "pipelined16", "paired", "lds_solutions"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 5e-4)])
@pytest.mark.parametrize("nrhs", [12, 20, 40])
def test_fine_sweep_variants_match_oracle(policy, prec, tol, nrhs):
    from paper_2103_14921_amd import helm
    helm.set_sweep_policy(policy)
    shape, h, f, pml = (21, 18, 16), 25.0, 10.0, (3, 3, 3, 0)
    c = inputs.velocity_thrust_belt(*shape, h=h)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    M = Oras(A, shape, decompose(shape, (2, 2, 2), 2), prob.k().ravel(), h)
    say("fine sweep", policy, prec, nrhs)
    S = helm.Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 2), overlap=2, levels=1, precision=prec)
    R = inputs.random_field((nrhs, prob.n), seed=50 + nrhs)
    Z = S.apply_oras(R)
    for r in range(nrhs):
        assert rel(Z[r], M.apply(R[r])) <= tol, r
    S.close()


@pytest.mark.parametrize("policy", ["item", "pipelined", "two_per_cu", "pipelined16", "paired", "paired_lds"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("single_local", 5e-4)])
@pytest.mark.parametrize("nrhs", [20, 12, 64])
def test_coarse_sweep_variants_match_oracle(policy, prec, tol, nrhs):
    from paper_2103_14921_amd import helm
    helm.set_sweep_policy(policy)
    shape, h, f, pml = (28, 26, 24), 25.0, 10.0, (5, 5, 5, 0)
    c = inputs.velocity_thrust_belt(*shape, h=h)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    tl = TwoLevel(A, shape, decompose(shape, (2, 2, 2), 2), prob.k().ravel(), h, 2)
    say("coarse sweep", policy, prec, nrhs)
    S = helm.Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 2), overlap=2, levels=2, precision=prec)
    Cc = inputs.random_field((nrhs, S.nc), seed=77)
    Zc = S.apply_oras(Cc, level=1)
    for r in range(nrhs):
        assert rel(Zc[r], tl.coarse.apply(Cc[r])) <= tol, r
    S.close()


def test_policies_agree_in_a_two_level_solve():
    from paper_2103_14921_amd import helm
    shape, h, f, tol = (28, 26, 24), 25.0, 10.0, 1e-8
    c = inputs.velocity_thrust_belt(*shape, h=h)
    src = inputs.source_grid(shape[0], shape[1], 5, 5, 4, 5, iz=4)
    b = inputs.point_source_rhs(*shape, src)
    out = {}
    for policy in ("item", "pipelined", "two_per_cu", "pipelined16", "paired", "paired_lds"):
        helm.set_sweep_policy(policy)
        say("two-level solve", policy, len(src))
        S = helm.Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=20)
        out[policy] = S.solve(b, tol=tol, maxit=300)
        S.close()
    Xa, ia = out["item"]
    for other in ("pipelined", "two_per_cu", "pipelined16", "paired", "paired_lds"):
        Xb, ib = out[other]
        assert np.all(ia["relres_true"] <= tol) and np.all(ib["relres_true"] <= tol)
        assert np.max(np.abs(ia["iters"] - ib["iters"])) <= 1
        for r in range(len(src)):
            assert rel(Xb[r], Xa[r]) <= 10 * tol
