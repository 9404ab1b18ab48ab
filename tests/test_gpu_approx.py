"""Approximate local solves (HELM_APPROX_LOCAL; the paper's incomplete-Cholesky
rows of Table 2 made approximate here by complex-FP16 plane inverses on FP16
matrix cores) against the FP64 oracle, through the C ABI.

The local solves are approximate by design: the operator-level check bounds
their distance from the oracle's exact local solves; the end-to-end checks are
the method's own bar -- the FP64 true residual, recomputed with the oracle's
assembled A, at the tolerance, and the solution within 10 x tol of the
oracle's FP64 solution.
"""
import numpy as np
import pytest

import inputs
from oracle.dd import Oras, decompose
from oracle.operator import Pml, Problem, assemble, fit_weights
from oracle.solve import setup as oracle_setup
from oracle.solve import solve as oracle_solve

pytestmark = pytest.mark.gpu

WO = fit_weights()
W = {k: getattr(WO, k) for k in ("w1", "w2", "w3", "wm1", "wm2", "wm3", "wm4")}


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("nrhs", [5, 20, 40])
def test_approximate_local_solves_stay_close_to_the_exact_ones(nrhs):
    # FP16 factors and operand (unit roundoff 2^-11) with FP32 accumulation:
    # each plane product is within a few 1e-3 of the exact one relative to the
    # plane's size; through the forward and backward sweeps the local solution
    # stays within 2e-2 of the exact local solve (measured: a few 1e-3)
    from paper_2103_14921_amd import helm
    shape, h, f, pml = (21, 18, 16), 25.0, 10.0, (3, 3, 3, 0)
    c = inputs.velocity_thrust_belt(*shape, h=h, q=100.0)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    M = Oras(assemble(prob), shape, decompose(shape, (2, 2, 2), 2), prob.k().ravel(), h)
    say("approx one-level ORAS", nrhs)
    S = helm.Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 2), overlap=2, levels=1, precision="approx_local")
    R = inputs.random_field((nrhs, prob.n), seed=90 + nrhs)
    Z = S.apply_oras(R)
    errs = [rel(Z[r], M.apply(R[r])) for r in range(nrhs)]
    say("max rel err", max(errs))
    assert max(errs) <= 2e-2
    assert max(errs) > 0  # approximate, not exact: the FP16 path really ran
    S.close()


@pytest.mark.parametrize("nrhs", [12, 20])
def test_fp16_sweep_with_plane_solutions_in_lds(nrhs):
    # the FP16 sweep forced to keep its plane solutions in LDS (groups of 16,
    # sweep policy 6) against the same sweep tuned without that form (policy 1)
    # and against the oracle's exact local solves
    from paper_2103_14921_amd import helm
    shape, h, f, pml = (21, 18, 16), 25.0, 10.0, (3, 3, 3, 0)
    c = inputs.velocity_thrust_belt(*shape, h=h, q=100.0)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    M = Oras(assemble(prob), shape, decompose(shape, (2, 2, 2), 2), prob.k().ravel(), h)
    R = inputs.random_field((nrhs, prob.n), seed=70 + nrhs)
    out = {}
    try:
        for policy in ("item", "lds_solutions"):
            helm.set_sweep_policy(policy)
            say("approx one-level ORAS", policy, nrhs)
            S = helm.Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 2), overlap=2, levels=1,
                            precision="approx_local")
            out[policy] = S.apply_oras(R)
            S.close()
    finally:
        helm.set_sweep_policy("auto")
    for r in range(nrhs):
        assert rel(out["lds_solutions"][r], out["item"][r]) <= 1e-6, r
        assert rel(out["lds_solutions"][r], M.apply(R[r])) <= 2e-2, r


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_approximate_two_level_solve_reaches_the_fp64_residual(tol):
    from paper_2103_14921_amd import helm
    shape, h, f = (28, 26, 24), 25.0, 10.0
    c = inputs.velocity_thrust_belt(*shape, h=h)
    src = inputs.source_grid(shape[0], shape[1], 5, 5, 2, 2, iz=4)
    b = inputs.point_source_rhs(*shape, src)
    prob = Problem(shape, h, c, f, Pml(5, 5, 5, 0), WO)
    st = oracle_setup(prob, (2, 2, 2), 2, 2)
    ref = oracle_solve(st, b, tol, 20, 300)
    say("approx two-level e2e", shape, tol)
    S = helm.Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=20,
                    precision="approx_local")
    X, info = S.solve(b, tol=tol, maxit=300)
    say("iters approx", info["iters"], "oracle fp64", ref["iters"])
    for r in range(len(src)):
        res = b[r].ravel() - st.A @ X[r].ravel()
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= tol
        assert info["relres_true"][r] <= tol
        assert rel(X[r], ref["X"][r]) <= 10 * tol
    assert np.all(info["iters"] <= ref["iters"] + 3)
    S.close()


def test_approximate_factors_take_half_the_memory_of_complex_fp32():
    from paper_2103_14921_amd import helm
    shape, h, f = (40, 36, 32), 25.0, 10.0
    c = inputs.velocity_thrust_belt(*shape, h=h)
    held = {}
    for prec in ("mixed", "approx_local"):
        S = helm.Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=1,
                        precision=prec)
        held[prec] = S.resident_bytes()
        S.close()
    say("resident bytes", held)
    assert held["approx_local"] < 0.75 * held["mixed"]
