"""Captured outer iterations (HIP graphs) against direct launches.

Each outer FGMRES iteration (two-level preconditioner with its ten coarse GMRES
iterations, operator product, Arnoldi step) is captured once and replayed; the
replays run between direct launches and host synchronisations of the same
solve.  The same kernels with the same arguments run either way, so every
iterate -- and hence the solution, the iteration counts and the residuals --
must be bitwise those of direct launches, over several replays of every graph,
across solves on one handle and across batch widths.
"""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

H, F, NPML = 25.0, 10.0, 6


def say(*a):
    print("[case]", *a, flush=True)


def _pair(shape, parts, levels, precision, restart):
    import torch
    from paper_2103_14921_amd import helm
    dev = torch.device("cuda:0")
    c = torch.from_numpy(inputs.velocity_thrust_belt(*shape, H)).to(dev)
    mk = lambda: helm.Solver(shape, H, c, F, (NPML, NPML, NPML, 0), parts=parts, overlap=2, levels=levels,
                             precision=precision, restart=restart)
    g, d = mk(), mk()
    d.set_graphs(False)
    return g, d, dev


def _rhs(shape, grid, dev, shift=0):
    import torch
    nx, ny, nz = shape
    src = inputs.source_grid(nx, ny, NPML + shift, NPML, grid[0], grid[1], iz=4 + shift)
    B = inputs.point_source_rhs(nx, ny, nz, src).reshape(len(src), -1)
    return torch.from_numpy(np.ascontiguousarray(B)).to(dev)


def _same(a, b, tag):
    import torch
    Xa, ia = a
    Xb, ib = b
    assert np.array_equal(ia["iters"], ib["iters"]), (tag, ia["iters"], ib["iters"])
    assert np.array_equal(ia["relres_true"], ib["relres_true"]), tag
    assert torch.equal(Xa, Xb), (tag, float((Xa - Xb).abs().max()))


@pytest.mark.parametrize("prec", ["mixed", "single_local"])
def test_two_level_mixed_graphs_bitwise_equal_direct(prec):
    shape = (48, 48, 48)
    say("graphs", prec)
    g, d, dev = _pair(shape, (3, 3, 3), 2, prec, 6)
    # 12 RHS: the sweep tuner runs in the first iteration, the rest is captured;
    # restart 6 makes every captured iteration replay in later cycles
    for tag, grid, shift in (("solve 12 rhs", (4, 3), 0), ("again, new rhs", (3, 4), 2), ("5 rhs", (5, 1), 1)):
        B = _rhs(shape, grid, dev, shift)
        say(tag, tuple(B.shape))
        a = g.solve(B, tol=1e-6, maxit=200)
        b = d.solve(B, tol=1e-6, maxit=200)
        assert np.all(a[1]["relres_true"] <= 1e-6)
        _same(a, b, tag)
        # the solve's lower bound counts a replayed iteration like a direct one
        bg, bd = g.solve_bound(), d.solve_bound()
        assert bg["seconds"] > 0 and bg["bytes"] > 0 and bg["flops"] > 0
        for k in bg:
            assert abs(bg[k] - bd[k]) <= 1e-9 * bd[k], (tag, k, bg[k], bd[k])
        st = g.graph_stats()
        say(tag, "iters", a[1]["iters"].max(), st)
        assert st["replays"] > st["captures"] > 0
    assert d.graph_stats() == {"captures": 0, "replays": 0}
    g.close()
    d.close()


def test_one_level_fp64_graphs_bitwise_equal_direct():
    shape = (40, 36, 32)
    g, d, dev = _pair(shape, (2, 2, 2), 1, "fp64", 5)
    B = _rhs(shape, (3, 1), dev)
    say("one-level fp64", tuple(B.shape))
    a = g.solve(B, tol=1e-8, maxit=300)
    b = d.solve(B, tol=1e-8, maxit=300)
    _same(a, b, "one-level")
    st = g.graph_stats()
    assert st["replays"] > st["captures"] > 0
    g.close()
    d.close()


def test_sweep_timing_inside_graphs():
    shape = (48, 48, 48)
    g, d, dev = _pair(shape, (3, 3, 3), 2, "mixed", 6)
    B = _rhs(shape, (4, 3), dev)
    say("timing warm-up")
    g.solve(B, tol=1e-6, maxit=200)  # captures untimed graphs, tunes the sweeps
    d.solve(B, tol=1e-6, maxit=200)
    for s in (g, d):
        s.set_sweep_timing(True)
    before = g.graph_stats()["replays"]
    a = g.solve(B, tol=1e-6, maxit=200)
    b = d.solve(B, tol=1e-6, maxit=200)
    _same(a, b, "timed")
    for lv in (0, 1):
        sg, sd = g.sweep_stats(lv), d.sweep_stats(lv)
        say("level", lv, "graph", sg, "direct", sd)
        assert sg["launches"] == sd["launches"] > 0
        assert sg["flops"] == sd["flops"]
        assert 0.25 * sd["ms"] < sg["ms"] < 4.0 * sd["ms"]
    for kind in (0, 1):  # the fine 27-point products, timed the same way
        sg, sd = g.stencil_stats(kind), d.stencil_stats(kind)
        say("stencil", kind, "graph", sg, "direct", sd)
        assert sg["launches"] == sd["launches"] > 0
        assert sg["bytes"] == sd["bytes"] and sg["flops"] == sd["flops"]
        assert 0.25 * sd["ms"] < sg["ms"] < 4.0 * sd["ms"]
    # the timed iterations themselves ran from graphs (event-record nodes)
    assert g.graph_stats()["replays"] > before
    g.close()
    d.close()


def test_capture_concurrent_with_setup_and_trim():
    # one thread solves (capturing its outer iterations) while another sets up
    # and destroys handles and trims the device cache: captures never see a
    # device-wide operation and set-ups never touch the legacy stream
    import threading

    import torch
    from paper_2103_14921_amd import helm
    shape = (40, 40, 40)
    g, d, dev = _pair(shape, (2, 2, 2), 2, "mixed", 5)
    d.close()
    B = _rhs(shape, (3, 3), dev)
    c2 = torch.from_numpy(inputs.velocity_thrust_belt(32, 32, 32, H)).to(dev)
    errors = []

    def churn():
        try:
            for i in range(6):
                S = helm.Solver((32, 32, 32), H, c2, F, (NPML, NPML, NPML, 0), parts=(2, 2, 2), overlap=2, levels=2,
                                precision="mixed", restart=5)
                S.close()
                helm.trim_cache()
        except Exception as exc:  # reported below
            errors.append(exc)

    say("concurrent capture and set-up")
    t = threading.Thread(target=churn)
    t.start()
    results = [g.solve(B, tol=1e-6, maxit=200) for _ in range(3)]
    t.join()
    assert not errors, errors
    for X, info in results:
        assert np.all(info["relres_true"] <= 1e-6)
    assert g.graph_stats()["replays"] > 0
    g.close()
