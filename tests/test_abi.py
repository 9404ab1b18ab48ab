"""Host-side checks of the C ABI (CPU only): the library loads, exports every
symbol include/helm.h declares, and its host-only weight fit agrees with the
oracle's independent fit."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "helm.h")).read()
    return sorted(set(re.findall(r"\b(helm_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declares_binding_exports():
    from paper_2103_14921_amd import helm
    assert sorted(helm.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2103_14921_amd import helm
    for name in _declared():
        assert hasattr(helm.lib, name), name


def test_native_weight_fit_matches_oracle():
    from paper_2103_14921_amd import helm
    from oracle.operator import fit_weights
    a = helm.fit_weights()
    b = fit_weights()
    for k in a:
        assert abs(a[k] - getattr(b, k)) <= 1e-10, k


def test_fit_rejects_bad_arguments():
    from paper_2103_14921_amd import helm
    with pytest.raises(helm.HelmError) as e:
        helm.fit_weights(ng=0)
    assert e.value.code == helm.HELM_EINVAL


def test_footprint_grows_with_rhs_and_rejects_bad_decomposition():
    from paper_2103_14921_amd import helm
    a = helm.footprint((64, 64, 64), (4, 4, 4), levels=2, nrhs_chunk=1)
    b = helm.footprint((64, 64, 64), (4, 4, 4), levels=2, nrhs_chunk=8)
    assert 0 < a < b
    # boxes thinner than 2*overlap+1 are rejected (footprint 0)
    assert helm.footprint((16, 16, 16), (8, 1, 1)) == 0


def test_workspace_bytes_is_the_rhs_dependent_part_of_the_footprint():
    # a solve on a set-up handle allocates the Krylov workspace alone: it is the
    # part of the footprint that grows with the batch, and less than the whole
    from paper_2103_14921_amd import helm
    for levels, prec in ((1, "fp64"), (2, "mixed")):
        f = [helm.footprint((48, 40, 32), (3, 2, 2), levels=levels, precision=prec, nrhs_chunk=k) for k in (1, 8)]
        w = [helm.workspace_bytes((48, 40, 32), (3, 2, 2), levels=levels, precision=prec, nrhs_chunk=k)
             for k in (1, 8)]
        assert 0 < w[0] < f[0] and w[0] < w[1]
        assert f[1] - f[0] == w[1] - w[0]
    assert helm.workspace_bytes((48, 40, 32), (3, 2, 2), nrhs_chunk=0) == 0
    assert helm.workspace_bytes((16, 16, 16), (8, 1, 1)) == 0


def test_process_wide_settings_reject_bad_values():
    from paper_2103_14921_amd import helm
    for bad in (1, 3, 16, -2, helm.HELM_TILE_MARCH | 4, helm.HELM_TILE_MARCH):
        with pytest.raises(helm.HelmError) as e:
            helm.set_row_tiling(bad)
        assert e.value.code == helm.HELM_EINVAL
    helm.set_row_tiling(helm.HELM_TILE_MARCH | 3)
    assert helm.lib.helm_set_sweep_policy(7) == helm.HELM_EINVAL
    for bad in (1, 2, 12, 32):
        with pytest.raises(helm.HelmError):
            helm.set_lu_panel(bad)
    helm.set_lu_panel(0)
    helm.set_row_tiling(0)


def test_statistics_entry_points_reject_null_handles_and_bad_kinds():
    import ctypes as C

    from paper_2103_14921_amd import helm
    out = (C.c_double * 4)()
    for kind in (0, 1):
        assert helm.lib.helm_stencil_stats(None, kind, out) == helm.HELM_EINVAL
        assert helm.lib.helm_sweep_stats(None, kind, out) == helm.HELM_EINVAL
    assert helm.lib.helm_resident_bytes(None) == 0
    # an unknown precision code is refused before any device work
    d = helm.DecompT(2, 2, 2, 2, 2, 10, 7, 20, 1, 0)
    assert helm.footprint((32, 32, 32), (2, 2, 2), precision="approx_local") > 0
    # approximate local solves need fine planes of at most 960 nodes
    assert helm.footprint((68, 68, 16), (2, 2, 1), precision="approx_local") == 0
    assert helm.lib.helm_footprint(C.byref(helm.Grid(32, 32, 32, 25.0)), C.byref(d), 1) == 0
    with pytest.raises(ValueError):
        helm.footprint((32, 32, 32), (2, 2, 2), precision="half")


def test_no_kernel_uses_scratch(tmp_path):
    # every kernel of the built library keeps its state in registers and LDS:
    # per-wave scratch would be allocated by the runtime at dispatch, where a
    # failure under memory pressure aborts the queue instead of returning an error
    import shutil
    import subprocess
    objdump, readelf = "/opt/rocm/llvm/bin/llvm-objdump", "/opt/rocm/llvm/bin/llvm-readelf"
    if not (os.path.exists(objdump) and os.path.exists(readelf)):
        pytest.skip("ROCm LLVM tools not installed")
    lib = os.path.join(ROOT, "paper_2103_14921_amd", "libhelm.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    shutil.copy(lib, tmp_path / "libhelm.so")
    subprocess.run([objdump, "--offloading", str(tmp_path / "libhelm.so")], check=True, capture_output=True,
                   cwd=tmp_path)
    objs = sorted(p for p in tmp_path.iterdir() if "amdgcn" in p.name and "gfx950" in p.name)
    assert objs, "no gfx950 code objects in the library"
    kernels = {}
    for o in objs:
        notes = subprocess.run([readelf, "--notes", str(o)], check=True, capture_output=True, text=True).stdout
        name = None
        for line in notes.splitlines():
            s = line.strip()
            if s.startswith(".name:"):
                name = s.split(":", 1)[1].strip()
            elif s.startswith(".private_segment_fixed_size:") and name:
                kernels[name] = int(s.split(":", 1)[1])
                name = None
    assert len(kernels) > 40
    spilled = {k: v for k, v in kernels.items() if v != 0}
    assert not spilled, spilled


def test_serving_admission_reserves_whole_workspace_and_staging():
    # a batch on a resident problem allocates the full Krylov workspace (it is
    # released after every batch) and stages B and X on the device; a problem
    # not yet set up needs its whole footprint on top of the staging
    from paper_2103_14921_amd import helm
    from paper_2103_14921_amd.serving import ProblemSpec, Server
    srv = Server.__new__(Server)  # host-side accounting only: no device, no threads
    spec = ProblemSpec("p", (48, 40, 32), 25.0, 4.0, parts=(3, 2, 2))
    for nr in (1, 5, 16):
        ws = helm.workspace_bytes(spec.shape, spec.parts, spec.overlap, spec.levels, spec.coarse_iters,
                                  spec.precision, spec.restart, nr)
        fp = helm.footprint(spec.shape, spec.parts, spec.overlap, spec.levels, spec.coarse_iters, spec.precision,
                            spec.restart, nr)
        staging = 2 * 16 * nr * spec.n
        assert srv._need(spec, nr, resident=True) >= ws + staging
        assert srv._need(spec, nr, resident=False) >= fp + staging
        assert srv._need(spec, nr, resident=True) < srv._need(spec, nr, resident=False)


def test_serving_splits_a_request_that_does_not_fit_into_chunks():
    from paper_2103_14921_amd.serving import ProblemSpec, Server
    srv = Server.__new__(Server)
    spec = ProblemSpec("p", (48, 40, 32), 25.0, 4.0, parts=(3, 2, 2))
    for resident in (True, False):
        srv.budget = srv._need(spec, 9, resident, chunk=3)
        assert srv._largest_chunk(spec, 9, resident) == 3
        srv.budget -= 1
        assert srv._largest_chunk(spec, 9, resident) == 2
    srv.budget = srv._staging(spec, 9)  # not even one right-hand side fits
    assert srv._largest_chunk(spec, 9, True) == 0


def test_poisson_stream_reports_each_completion_once():
    # progress comes from completions as they happen (also while later requests
    # are still arriving), once per request, and the results keep submission order
    import threading
    from concurrent.futures import Future

    import numpy as np
    from paper_2103_14921_amd.serving import run_poisson

    class Fake:
        def __init__(self):
            self.stats = type("S", (), {"latencies": [0.1, 0.2, 0.3]})()

        def submit(self, spec, B, tol):
            f = Future()
            threading.Timer(0.01 * (3 - spec), lambda: f.set_result({"X": B, "iters": np.array([spec])})).start()
            return f

        def latency_percentiles(self):
            return {"p50_s": 0.2, "p99_s": 0.3, "mean_s": 0.2, "max_s": 0.3}

    seen = []
    out = run_poisson(Fake(), [(k, np.zeros((k + 1, 4)), 1e-6) for k in range(3)], rate_hz=1000.0,
                      progress=lambda i, n: seen.append((i, n)))
    import time
    t0 = time.time()
    while len(seen) < 3 and time.time() - t0 < 5:  # a callback may still be running as result() returns
        time.sleep(0.01)
    assert sorted(seen) == [(1, 3), (2, 3), (3, 3)]
    assert [r["nrhs"] for r in out["results"]] == [1, 2, 3]


def test_bench_module_imports_and_summarises_timings():
    # bench.py imports without a GPU (its work is under main()) and turns live
    # timings into roofline entries
    import importlib
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    bench = importlib.import_module("bench")
    assert "thrust192_mixed" in bench.WORKLOADS and "thrust192_single_local" in bench.WORKLOADS
    e = bench.stencil_entry([{"launches": 2, "ms": 4.0, "flops": 1.0, "bytes": 16e9},
                             {"launches": 1, "ms": 2.0, "flops": 1.0, "bytes": 12e9}])
    assert e["bound"] == "hbm" and abs(e["A_x"]["achieved"] - 4000.0) < 1e-9
    assert abs(e["achieved"] - 28e9 / 6.0 * 1e-6) < 1e-6 and abs(e["frac"] - e["achieved"] / 8000.0) < 1e-12
    r = bench.roofline_entry({"launches": 2, "ms": 2.0, "flops": 2e12, "bytes": 1e9}, "c128")
    assert abs(r["achieved"] - 1000.0) < 1e-9 and abs(r["frac"] - 1000.0 / 78.6) < 1e-12
    class Boxes:  # two boxes: 4 x 3 planes x 5 and 2 x 2 planes x 3
        def num_subdomains(self, level):
            return 2

        def subdomain_box(self, s, level):
            return [{"elo": (0, 0, 0), "ehi": (4, 3, 5)}, {"elo": (1, 1, 1), "ehi": (3, 3, 4)}][s]
    assert bench.factor_flops(Boxes()) == 5 * 8.0 * 12 ** 3 + 3 * 8.0 * 4 ** 3
    import torch
    from paper_2103_14921_amd import helm
    X = torch.randn(20, 7, dtype=torch.complex128)
    e = bench.rel_err(helm, torch, X, X * (1 + 1e-3))  # in chunks of 8 rows, the last one ragged
    assert e.shape == (20,) and torch.allclose(e, torch.full((20,), 1e-3 / (1 + 1e-3), dtype=torch.float64))


def test_bench_attaches_profile_traffic_only_to_matching_launches():
    # bench.py copies a committed counter profile's HBM traffic into its line
    # only for the same sweep source (hash), the same average algorithmic
    # bytes per launch and the same tuned launches; anything else gives null
    import hashlib
    import importlib
    import json
    import os
    import re
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    bench = importlib.import_module("bench")
    for md in ("oras_sweep_coarse_thrust192_mixed_pmc.md", "oras_sweep_coarse_thrust192_single_local_pmc.md"):
        text = open(os.path.join(root, "profiles", md)).read()
        data = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        src = open(os.path.join(root, "paper_2103_14921_amd", "csrc", "ops_sweep.hip"), "rb").read()
        same_source = hashlib.sha256(src).hexdigest()[:16] == data["source_sha256_16"]
        alg, cfg = data["algorithmic_bytes_per_launch"], data["sweep_config"]
        got, where = bench.measured_traffic("ops_sweep.hip", md, alg, cfg)
        if same_source:
            assert got == data["traffic_bytes_per_launch"] and md in where
        else:
            assert got is None
        other = json.loads(json.dumps(cfg))
        other["32"]["waves"] += 1
        assert bench.measured_traffic("ops_sweep.hip", md, alg, other) == (None, None)
        assert bench.measured_traffic("ops_sweep.hip", md, alg * 1.01, cfg) == (None, None)
        assert bench.measured_traffic("ops_sweep.hip", md, alg, None) == (None, None)


def test_serving_requeue_hold_is_lifted_when_the_other_batch_ends_first():
    # A batch that finds the device short while another is in flight goes back
    # to the queue and holds new launches until that other batch ends.  Force
    # the interleaving where the other batch ends between the failing batch's
    # re-queue and the end of its worker: the hold must not outlive it (the
    # scheduler would wait for an end that already happened).
    import collections
    import threading
    from concurrent.futures import Future

    import numpy as np
    import torch
    from paper_2103_14921_amd import helm
    from paper_2103_14921_amd.serving import ProblemSpec, Server, ServerStats, _Entry, _Request

    class Stub:
        def __init__(self, fail):
            self.fail = fail

        def solve(self, B, tol, maxit):
            if self.fail:
                raise helm.HelmError(helm.HELM_ENOMEM, "short")
            n = B.shape[0]
            return B.clone(), {"iters": np.ones(n, np.int32), "relres_true": np.zeros(n), "status": 0}

        def release_workspace(self):
            pass

        def resident_bytes(self):
            return 0

    srv = Server.__new__(Server)  # host-side state only: no device, no scheduler thread
    srv.torch, srv.device = torch, torch.device("cpu")
    srv._queue, srv._entries = collections.deque(), collections.OrderedDict()
    srv._inflight, srv._hold, srv._closed, srv.stats = 0, False, False, ServerStats()
    cv = threading.Condition()
    calls = {"n": 0}
    specs = [ProblemSpec(nm, (4, 4, 4), 25.0, 4.0) for nm in ("x", "y")]
    ex, ey = _Entry(specs[0], Stub(True), busy=True), _Entry(specs[1], Stub(False), busy=True)
    srv._entries[specs[0]], srv._entries[specs[1]] = ex, ey

    def req(spec):
        return _Request(spec, np.zeros((1, 64), np.complex128), 1e-6, 10, 0.0, Future(), 1)

    rx, ry = req(specs[0]), req(specs[1])

    class Hooked:  # runs the other batch to its end right before the failing worker's last critical section
        def __enter__(self):
            if threading.current_thread().name == "x":
                calls["n"] += 1
                if calls["n"] == 2:
                    srv._work(ey, [ry], 1, 0, 1)
            return cv.__enter__()

        def __exit__(self, *a):
            return cv.__exit__(*a)

        def notify_all(self):
            cv.notify_all()

    srv._cv = Hooked()
    t = threading.Thread(target=srv._work, args=(ex, [rx], 1, 0, 1), name="x")
    t.start()
    t.join(10)
    assert not t.is_alive()
    assert ry.future.done() and not rx.future.done()
    assert list(srv._queue) == [rx] and srv.stats.retries == 1
    assert not ex.busy and not ey.busy
    assert not srv._hold and not srv._held()


def test_native_weight_table_matches_oracle():
    # the adaptive coefficients' table: the library's fit (Householder QR) and
    # the oracle's (numpy least squares) agree entry by entry
    from paper_2103_14921_amd import helm
    from oracle.operator import ADAPT_DG, ADAPT_G0, ADAPT_N, adaptive_table
    a = helm.fit_weight_table(ADAPT_G0, ADAPT_DG, ADAPT_N, 15)
    b = adaptive_table()
    assert len(a) == len(b) == ADAPT_N
    for wa, wb in zip(a, b):
        for k in wa:
            assert abs(wa[k] - getattr(wb, k)) <= 1e-10 * max(1.0, abs(getattr(wb, k))), k
    with pytest.raises(helm.HelmError):
        helm.fit_weight_table(n=0)
