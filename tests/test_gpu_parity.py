"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Same seeded inputs on both sides (module ``inputs``), same stencil weights.
Tolerances: operator-level FP64 pieces agree to rounding (relative 1e-12 for
the stencil, 1e-10 for local solves, whose explicit block inverses carry a
condition-number factor); complex-FP32 local solves to 5e-4; end-to-end FP64
solves agree in iteration count and to a relative L2 of 10 x tol.
"""
import numpy as np
import pytest

import inputs
from oracle.coarse import TwoLevel
from oracle.dd import Oras, decompose
from oracle.operator import Pml, Problem, assemble, fit_weights
from oracle.solve import setup as oracle_setup
from oracle.solve import solve as oracle_solve

pytestmark = pytest.mark.gpu

WO = fit_weights()
W = {k: getattr(WO, k) for k in ("w1", "w2", "w3", "wm1", "wm2", "wm3", "wm4")}


def helm():
    from paper_2103_14921_amd import helm as h
    return h


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _thrust_case(shape=(23, 19, 17), pml=(4, 3, 5, 2), q=100.0):
    h, f = 25.0, 10.0
    c = inputs.velocity_thrust_belt(*shape, h=h, q=q)
    return shape, h, c, f, pml


@pytest.mark.parametrize("nrhs", [1, 3, 8, 12, 20])
def test_stencil_matches_csr(nrhs):
    shape, h, c, f, pml = _thrust_case()
    say("stencil", shape, nrhs)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    S = helm().Solver(shape, h, c, f, pml, weights=W, parts=(1, 1, 1), levels=1)
    X = inputs.random_field((nrhs, prob.n), seed=100 + nrhs)
    Y = S.apply_A(X)
    ref = (A @ X.T).T
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))
    S.close()


@pytest.mark.parametrize("parts,delta,prec,tol", [((2, 2, 2), 2, "fp64", 1e-10), ((3, 2, 2), 2, "fp64", 1e-10),
                                                  ((2, 2, 2), 2, "mixed", 5e-4)])
def test_one_level_oras_matches_oracle(parts, delta, prec, tol):
    shape, h, c, f, pml = _thrust_case(shape=(21, 18, 16), pml=(3, 3, 3, 0))
    say("oras", shape, parts, prec)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    boxes = decompose(shape, parts, delta)
    M = Oras(A, shape, boxes, prob.k().ravel(), h)
    S = helm().Solver(shape, h, c, f, pml, weights=W, parts=parts, overlap=delta, levels=1, precision=prec)
    R = inputs.random_field((2, prob.n), seed=7)
    Z = S.apply_oras(R)
    for r in range(2):
        assert rel(Z[r], M.apply(R[r])) <= tol
    S.close()


@pytest.mark.parametrize("shape,parts,widths", [((21, 18, 16), (2, 2, 2), (16, 8)),
                                                 ((44, 44, 8), (2, 2, 1), (8, 4))])
def test_lu_panel_widths_match_oracle(shape, parts, widths):
    # every admissible panel width of the plane inversions, forced, and the
    # autotuned one: one-level ORAS matches the oracle; planes of 576 rows use
    # the wide-plane widths
    h, f, pml = 25.0, 10.0, (3, 3, 3, 0)
    c = inputs.velocity_thrust_belt(*shape, h=h, q=100.0)
    say("lu panels", shape, parts, widths)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    M = Oras(A, shape, decompose(shape, parts, 2), prob.k().ravel(), h)
    R = inputs.random_field((2, prob.n), seed=17)
    ref = [M.apply(R[r]) for r in range(2)]
    hm = helm()
    try:
        for nb in widths + (0,):
            hm.set_lu_panel(nb)
            S = hm.Solver(shape, h, c, f, pml, weights=W, parts=parts, overlap=2, levels=1)
            Z = S.apply_oras(R)
            S.close()
            for r in range(2):
                assert rel(Z[r], ref[r]) <= 1e-10, (nb, r)
    finally:
        hm.set_lu_panel(0)


def test_coarse_pieces_match_oracle():
    shape, h, c, f, pml = _thrust_case(shape=(20, 18, 17), pml=(3, 3, 3, 0))
    say("coarse pieces", shape)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    boxes = decompose(shape, (2, 2, 2), 2)
    tl = TwoLevel(A, shape, boxes, prob.k().ravel(), h, 2)
    S = helm().Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 2), overlap=2, levels=2)
    R = inputs.random_field((2, prob.n), seed=8)
    Cc = S.restrict(R)
    assert rel(Cc, (tl.ZT @ R.T).T) <= 1e-14
    P = S.prolong(Cc)
    assert rel(P, (tl.Z @ Cc.T).T) <= 1e-14
    Ec = S.apply_E(Cc)
    assert rel(Ec, (tl.E @ Cc.T).T) <= 1e-12
    Zc = S.apply_oras(Cc, level=1)
    for r in range(2):
        assert rel(Zc[r], tl.coarse.apply(Cc[r])) <= 1e-10
    Q = S.apply_Q(R)
    for r in range(2):
        assert rel(Q[r], tl.q(R[r])) <= 1e-9
    Mz = S.apply_M(R)
    for r in range(2):
        assert rel(Mz[r], tl.apply(R[r])) <= 1e-9
    S.close()


def test_single_local_coarse_oras_matches_oracle():
    # complex-FP32 factors and sweeps on the coarse level too: the coarse
    # one-level ORAS within single-precision rounding of the FP64 oracle, the
    # operators around it (E, transfers) still FP64-exact
    shape, h, c, f, pml = _thrust_case(shape=(20, 18, 17), pml=(3, 3, 3, 0))
    say("coarse pieces single_local", shape)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    tl = TwoLevel(A, shape, decompose(shape, (2, 2, 2), 2), prob.k().ravel(), h, 2)
    S = helm().Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 2), overlap=2, levels=2, precision="single_local")
    R = inputs.random_field((2, prob.n), seed=8)
    Cc = S.restrict(R)
    assert rel(S.apply_E(Cc), (tl.E @ Cc.T).T) <= 1e-12
    Zc = S.apply_oras(Cc, level=1)
    Zf = S.apply_oras(R, level=0)
    for r in range(2):
        assert rel(Zc[r], tl.coarse.apply(Cc[r])) <= 5e-4
        assert rel(Zf[r], tl.fine.apply(R[r])) <= 5e-4
    S.close()


@pytest.mark.parametrize("nrhs", [2, 12])
def test_coarse_operator_batches_match_oracle(nrhs):
    # coarse product E x on batches below and above the row-tiled threshold,
    # on a grid whose rows do not divide into the tile width
    shape, h, c, f, pml = _thrust_case(shape=(30, 22, 19), pml=(3, 3, 3, 0))
    say("coarse E", shape, nrhs)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    tl = TwoLevel(A, shape, decompose(shape, (2, 2, 2), 2), prob.k().ravel(), h, 2)
    S = helm().Solver(shape, h, c, f, pml, weights=W, parts=(2, 2, 2), overlap=2, levels=2)
    Cc = inputs.random_field((nrhs, S.nc), seed=90 + nrhs)
    assert rel(S.apply_E(Cc), (tl.E @ Cc.T).T) <= 1e-12
    S.close()


def test_row_tilings_agree_bitwise():
    # the fine and coarse 27-point products under each forced schedule (row
    # tiles of 2, 4, 8 nodes per thread; plane-marching with 2 or 3) and the
    # autotuned one: every schedule matches the oracle and all are bitwise
    # equal; 70 nodes per row leave ragged segments, 37 planes a ragged plane
    # chunk; 12 and 9 right-hand sides take row tiles under every schedule,
    # 16 and 32 the plane-marching blocks of 16 and 32
    shape, h, c, f, pml = _thrust_case(shape=(70, 13, 37), pml=(3, 3, 3, 0))
    say("row tilings", shape)
    prob = Problem(shape, h, c, f, Pml(*pml), WO)
    A = assemble(prob)
    tl = TwoLevel(A, shape, decompose(shape, (2, 1, 2), 2), prob.k().ravel(), h, 2)
    hm = helm()
    S = hm.Solver(shape, h, c, f, pml, weights=W, parts=(2, 1, 2), overlap=2, levels=2)
    for nf, nc in ((12, 9), (32, 16), (16, 32)):
        X = inputs.random_field((nf, prob.n), seed=55 + nf)
        Cc = inputs.random_field((nc, S.nc), seed=56 + nc)
        ref, refE = (A @ X.T).T, (tl.E @ Cc.T).T
        B = inputs.random_field((nf, prob.n), seed=57 + nf)
        res = np.linalg.norm(B - ref, axis=1) / np.linalg.norm(B, axis=1)
        outs = []
        try:
            for sched in (2, 4, 8, hm.HELM_TILE_MARCH | 2, hm.HELM_TILE_MARCH | 3, 0):
                say("  batch", nf, nc, "schedule", sched)
                hm.set_row_tiling(sched)
                Y, E = S.apply_A(X), S.apply_E(Cc)
                assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref)), sched
                assert rel(E, refE) <= 1e-12, sched
                # the residual form b - A x: a solve with the initial guess X and no iteration
                # reports ||b - A x|| / ||b|| from it
                _, info = S.solve(B, tol=1e-30, maxit=0, X0=X.copy())
                assert np.all(np.abs(info["relres_true"] - res) <= 1e-10 * res), sched
                outs.append((Y, E, info["relres_true"]))
        finally:
            hm.set_row_tiling(0)
        for Y, E, rr in outs[1:]:
            assert np.array_equal(Y, outs[0][0]) and np.array_equal(E, outs[0][1])
            assert np.array_equal(rr, outs[0][2])
    S.close()


def test_config1_end_to_end_parity():
    # 24^3, h = 50 m, c = 1500 + 0.7 z, 3.75 Hz, 6-node PML on sides and bottom,
    # one-level ORAS 2x2x2, overlap 2, FGMRES(30), tol 1e-8, one source at (12, 12, 4)
    shape, h, f, tol = (24, 24, 24), 50.0, 3.75, 1e-8
    say("config1 e2e")
    c = inputs.velocity_linear(*shape, h)
    b = inputs.point_source_rhs(*shape, [(12, 12, 4)])
    prob = Problem(shape, h, c, f, Pml(6, 6, 6, 0), WO)
    st = oracle_setup(prob, (2, 2, 2), 2, 1)
    ref = oracle_solve(st, b, tol, 30, 300)
    S = helm().Solver(shape, h, c, f, (6, 6, 6, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=1, restart=30)
    X, info = S.solve(b, tol=tol, maxit=300)
    say("iters gpu", info["iters"], "oracle", ref["iters"])
    assert list(info["iters"]) == list(ref["iters"])
    assert rel(X, ref["X"]) <= 10 * tol
    assert info["relres_true"][0] <= tol
    r = b.reshape(1, -1)[0] - st.A @ X.reshape(-1)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= tol
    S.close()


def test_two_level_end_to_end_parity_many_rhs():
    shape, h, f, tol = (28, 26, 24), 25.0, 10.0, 1e-8
    say("two-level e2e", shape)
    c = inputs.velocity_thrust_belt(*shape, h=h)
    src = inputs.source_grid(shape[0], shape[1], 5, 5, 2, 2, iz=4)
    b = inputs.point_source_rhs(*shape, src)
    prob = Problem(shape, h, c, f, Pml(5, 5, 5, 0), WO)
    st = oracle_setup(prob, (2, 2, 2), 2, 2)
    ref = oracle_solve(st, b, tol, 20, 300)
    S = helm().Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=20)
    X, info = S.solve(b, tol=tol, maxit=300)
    say("iters gpu", info["iters"], "oracle", ref["iters"])
    assert list(info["iters"]) == list(ref["iters"])
    for r in range(len(src)):
        assert rel(X[r], ref["X"][r]) <= 10 * tol
        assert info["relres_true"][r] <= tol
    S.close()


def test_batch_narrows_at_restarts():
    # right-hand sides of different difficulty in one batch (a zero one done at
    # once, point sources, a random field) with short restart cycles, so they
    # leave the batch at different restarts: each matches its solve alone in
    # iteration count and solution (rounding of the batch-width dependent
    # reductions aside), and the zero one returns zero after no iteration
    shape, h, f, tol = (28, 26, 24), 25.0, 10.0, 1e-8
    say("narrowing batch", shape)
    c = inputs.velocity_thrust_belt(*shape, h=h)
    b = inputs.point_source_rhs(*shape, [(6, 6, 4), (14, 13, 4), (21, 19, 4)]).reshape(3, -1)
    rnd = inputs.random_field((1, b.shape[1]), seed=31)
    B = np.concatenate([b[:1], np.zeros_like(b[:1]), rnd, b[1:]], 0)
    S = helm().Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=5)
    X, info = S.solve(B, tol=tol, maxit=300)
    say("iters batch", info["iters"])
    assert len(set(int(i) for i in info["iters"])) >= 3
    for r in range(B.shape[0]):
        Xr, ir = S.solve(B[r:r + 1], tol=tol, maxit=300)
        assert int(ir["iters"][0]) == int(info["iters"][r]), r
        if r == 1:
            assert int(info["iters"][r]) == 0 and not np.any(X[r]) and info["relres_true"][r] == 0
            continue
        assert rel(X[r], Xr[0]) <= 1e-10, r
        assert info["relres_true"][r] <= tol
    S.close()


def test_batch_narrowing_with_iteration_limit_and_initial_guess():
    # right-hand sides that stop at maxit leave the batch like converged ones
    # (status NOT_CONVERGED, their residuals reported); with an initial guess
    # (one exact, one zero, one rough) each column matches its solve alone
    shape, h, f, tol = (28, 26, 24), 25.0, 10.0, 1e-10
    say("narrowing batch, maxit and x0", shape)
    c = inputs.velocity_thrust_belt(*shape, h=h)
    b = inputs.point_source_rhs(*shape, [(6, 6, 4), (14, 13, 4), (21, 19, 4)]).reshape(3, -1)
    S = helm().Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=4)
    ref, _ = S.solve(b, tol=tol, maxit=400)
    X0 = np.stack([ref[0], np.zeros_like(ref[1]), ref[2] + 1e-3 * inputs.random_field((1, b.shape[1]), seed=3)[0]])
    X, info = S.solve(b, tol=tol, maxit=9, X0=X0.copy())
    say("iters", info["iters"], "status", info["status"])
    assert info["status"] == helm().HELM_NOT_CONVERGED
    assert int(info["iters"][0]) == 0 and info["relres_true"][0] <= tol
    assert int(info["iters"][1]) == 9 and info["relres_true"][1] > tol
    for r in range(3):
        Xr, ir = S.solve(b[r:r + 1], tol=tol, maxit=9, X0=X0[r:r + 1].copy())
        assert int(ir["iters"][0]) == int(info["iters"][r]), r
        assert rel(X[r], Xr[0]) <= 1e-10, r
        assert abs(ir["relres_true"][0] - info["relres_true"][r]) <= 1e-6 * ir["relres_true"][0] + 1e-300, r
    S.close()


@pytest.mark.parametrize("prec", ["mixed", "single_local"])
def test_mixed_precision_reaches_fp64_residual(prec):
    shape, h, f = (28, 26, 24), 25.0, 10.0
    say("mixed e2e", shape, prec)
    c = inputs.velocity_thrust_belt(*shape, h=h)
    src = inputs.source_grid(shape[0], shape[1], 5, 5, 2, 2, iz=4)
    b = inputs.point_source_rhs(*shape, src)
    prob = Problem(shape, h, c, f, Pml(5, 5, 5, 0), WO)
    A = assemble(prob)
    S64 = helm().Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=20)
    X64, i64 = S64.solve(b, tol=1e-10, maxit=300)
    S = helm().Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=20,
                      precision=prec)
    X, info = S.solve(b, tol=1e-6, maxit=300)
    say(prec, "iters", info["iters"], "fp64(1e-10) iters", i64["iters"])
    for r in range(len(src)):
        tr = np.linalg.norm(b[r].ravel() - A @ X[r].ravel()) / np.linalg.norm(b[r])
        assert tr <= 1e-6 and info["relres_true"][r] <= 1e-6
        assert rel(X[r], X64[r]) <= 1e-3
    S.close()
    S64.close()


def test_batch_equals_alone():
    shape, h, f, tol = (24, 24, 24), 50.0, 3.75, 1e-8
    say("batch invariance")
    c = inputs.velocity_linear(*shape, h)
    src = inputs.source_grid(24, 24, 6, 6, 3, 2, iz=4)
    b = inputs.point_source_rhs(*shape, src)
    S = helm().Solver(shape, h, c, f, (6, 6, 6, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2, restart=30)
    Xb, ib = S.solve(b, tol=tol, maxit=200)
    for r in range(len(src)):
        Xa, ia = S.solve(np.ascontiguousarray(b[r:r + 1]), tol=tol, maxit=200)
        assert ia["iters"][0] == ib["iters"][r]
        assert rel(Xa[0], Xb[r]) <= 1e-12
    S.close()


def test_error_paths():
    hm = helm()
    shape = (16, 16, 16)
    c = inputs.velocity_linear(*shape, 50.0)
    bad = c.copy()
    bad[3, 3, 3] = np.nan
    say("errors")
    with pytest.raises(hm.HelmError) as e:
        hm.Solver(shape, 50.0, bad, 3.75, (4, 4, 4, 0), weights=W, parts=(2, 2, 2))
    assert e.value.code == hm.HELM_EINVAL
    neg = c.copy()
    neg[0, 0, 0] = -1500.0
    with pytest.raises(hm.HelmError) as e:
        hm.Solver(shape, 50.0, neg, 3.75, (4, 4, 4, 0), weights=W, parts=(2, 2, 2))
    assert e.value.code == hm.HELM_EINVAL
    import os
    os.environ["HELM_MEM_BUDGET"] = "1000"
    try:
        with pytest.raises(hm.HelmError) as e:
            hm.Solver(shape, 50.0, c, 3.75, (4, 4, 4, 0), weights=W, parts=(2, 2, 2))
        assert e.value.code == hm.HELM_ENOMEM
    finally:
        del os.environ["HELM_MEM_BUDGET"]
    S = hm.Solver(shape, 50.0, c, 3.75, (4, 4, 4, 0), weights=W, parts=(2, 2, 2))
    b = inputs.point_source_rhs(*shape, [(8, 8, 4), (4, 4, 4)])
    b[1] = 0.0
    X, info = S.solve(b, tol=1e-12, maxit=1)
    assert info["status"] == hm.HELM_NOT_CONVERGED
    assert info["iters"][0] == 1 and info["relres_true"][0] > 1e-12
    assert info["iters"][1] == 0 and np.all(X[1] == 0)
    S.close()
