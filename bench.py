"""Benchmark: right-hand sides solved per second to a 1e-6 FP64 true residual.

One step = the whole hot path on one batch: set-up (medium and PML, local
operators with absorbing interfaces, block-tridiagonal factorisations, coarse
operator and its factorisations) and the batched two-level ORAS-FGMRES solve
of every right-hand side to a true relative residual of 1e-6.  Inputs
(velocity and right-hand sides) are resident in HBM before the timed region.

Default workload: seeded thrust-belt model on a 192^3 grid (h = 25 m, 10 Hz =
8 points per minimum wavelength, 10-node PML on sides and bottom, Dirichlet
top), 12 x 12 x 12 subdomains of 16^3 with overlap 2, two-level ORAS with the
coarse grid at 2h, 64 point sources on an 8 x 8 grid at depth index 4; the
fine level's local factors and solves in complex FP32, everything else
(FGMRES, orthogonalisation, Givens, residuals and the whole coarse level) FP64
("mixed").  Beside the headline, one step of each comparison form on the same
inputs: plain FP64 (and the error of the mixed solution against it), the
oracle's CPU baseline, approximate fine local solves (complex-FP16 plane
inverses), block FGMRES (one Krylov space per batch), optionally the coarse
local solves in complex FP32 too ("single_local"), and a Poisson serving
stream.  These legs run in that order while their estimated cost fits
--time-budget (default 540 s of wall clock); a skipped leg is listed.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

T_START = time.perf_counter()

WORKLOADS = {
    # name: (shape, parts, n_src grid, restart)
    "thrust192_mixed": dict(shape=(192, 192, 192), parts=(12, 12, 12), src=(8, 8), restart=20, levels=2,
                            precision="mixed", tol=1e-6, q=None),
    "thrust192_single_local": dict(shape=(192, 192, 192), parts=(12, 12, 12), src=(8, 8), restart=20, levels=2,
                                  precision="single_local", tol=1e-6, q=None),
    "thrust128_fp64": dict(shape=(128, 128, 128), parts=(4, 4, 4), src=(4, 2), restart=30, levels=2,
                           precision="fp64", tol=1e-6, q=None),
    "thrust256x128_q100": dict(shape=(256, 256, 128), parts=(16, 16, 8), src=(16, 8), restart=20, levels=2,
                               precision="mixed", tol=1e-6, q=100.0),
    "thrust96_small": dict(shape=(96, 96, 96), parts=(6, 6, 6), src=(4, 4), restart=20, levels=2,
                           precision="mixed", tol=1e-6, q=None),
}
H, FREQ, NPML = 25.0, 10.0, 10


def describe(name, w):
    nx, ny, nz = w["shape"]
    px, py, pz = w["parts"]
    return (f"thrust-belt {nx}x{ny}x{nz}, h={H:g} m, {FREQ:g} Hz, PML {NPML}, {px}x{py}x{pz} boxes, overlap 2, "
            f"two-level ORAS-FGMRES({w['restart']}), {w['src'][0] * w['src'][1]} RHS, tol {w['tol']:g}"
            + (f", Q={w['q']:g}" if w["q"] else ""))


def make_inputs(w):
    import inputs
    nx, ny, nz = w["shape"]
    c = inputs.velocity_thrust_belt(nx, ny, nz, H, q=w["q"])
    src = inputs.source_grid(nx, ny, NPML, NPML, w["src"][0], w["src"][1], iz=4)
    b = inputs.point_source_rhs(nx, ny, nz, src)
    return c, b


def gpu_solve(helm, w, c_dev, b_dev, precision, weights, timing=False, graphs=True, block=False):
    S = helm.Solver(w["shape"], H, c_dev, FREQ, (NPML, NPML, NPML, 0), weights=weights, parts=w["parts"],
                    overlap=2, levels=w["levels"], coarse_iters=10, precision=precision, restart=w["restart"])
    if timing:
        S.set_sweep_timing(True)
    if not graphs:
        S.set_graphs(False)
    X, info = S.solve(b_dev, tol=w["tol"], maxit=400, block=block)
    if timing:
        info["sweeps"] = [S.sweep_stats(0), S.sweep_stats(w["levels"] - 1)]
        # the launches the tuner chose for the dominant sweep, at the batch widths of this solve
        lv = w["levels"] - 1
        info["sweep_config"] = {str(nr): S.sweep_config(lv, nr) for nr in (32, 16)
                                if S.sweep_config(lv, nr)["group"] > 0}
        info["stencil"] = [S.stencil_stats(0), S.stencil_stats(1)]
        info["factor_flops"] = factor_flops(S)
    info["graphs"] = S.graph_stats()
    info["bound"] = S.solve_bound()
    S.close()
    return X, info


PEAK = {"c64": 157.3, "c128": 78.6, "c32": 2500.0}  # dense MFMA TFLOP/s of one MI355X (fp32, fp64, fp16)


def measured_traffic(kernel_file, profile_md, algorithmic_bytes, sweep_config=None):
    """HBM bytes per launch from a committed PMC summary (FETCH_SIZE + WRITE_SIZE of a separate rocprofv3
    run, calibrated on a plain copy), if the kernel source is unchanged since, the step's launches have
    the same algorithmic bytes and the tuner chose the same launches (sweep_config, per batch width) as
    in the counter runs; else None.  Returns (bytes, source description): the figure is not measured in
    this run, and the line says where it comes from."""
    import hashlib
    import re as _re
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(root, "profiles", profile_md)).read()
        data = json.loads(_re.search(r"```json\n(.*?)\n```", text, _re.S).group(1))
        src = open(os.path.join(root, "paper_2103_14921_amd", "csrc", kernel_file), "rb").read()
        if hashlib.sha256(src).hexdigest()[:16] != data["source_sha256_16"]:
            return None, None
        if abs(algorithmic_bytes - data["algorithmic_bytes_per_launch"]) > 1e-6 * algorithmic_bytes:
            return None, None
        if data.get("sweep_config") is None or sweep_config != data["sweep_config"]:
            return None, None
        return data["traffic_bytes_per_launch"], (f"profiles/{profile_md}: PMC counters of an earlier run of the "
                                                  f"same kernel source ({data['source_sha256_16']}) and launch "
                                                  f"shape, not measured in this run")
    except Exception:
        return None, None


def set_traffic(entry, kernel_file, profile_md, sweep_config=None):
    """Attach the measured HBM traffic (or null) and its source to a roofline entry, with the arithmetic
    intensity on that traffic beside the algorithmic one."""
    traffic, source = measured_traffic(kernel_file, profile_md, entry["bytes_per_launch"], sweep_config)
    entry["sweep_config"] = sweep_config
    entry["traffic"], entry["traffic_source"] = traffic, source
    label_bound(entry)
    return entry


def label_bound(entry):
    """The kernel's roofline from its algorithmic intensity (flops over the algorithmic bytes: every
    factor once per application, the plane vectors): above the ridge of its arithmetic it is bound by
    the matrix cores (achieved TFLOP/s against that peak), below by HBM (algorithmic GB/s against 8 TB/s).
    With measured traffic, its intensity is reported beside: below the ridge, the implementation's own
    re-reads make it bandwidth-limited in practice although its algorithm is not."""
    peak_flops = entry["mfma_peak"] * 1e12
    ridge = peak_flops / 8.0e12
    ai = entry["flops_per_launch"] / entry["bytes_per_launch"]
    entry["arithmetic_intensity"] = ai
    entry["ridge"] = ridge
    if entry.get("traffic"):
        entry["measured_arithmetic_intensity"] = entry["flops_per_launch"] / entry["traffic"]
        entry["bandwidth_limited_in_practice"] = entry["measured_arithmetic_intensity"] < ridge
        # the measured HBM traffic against the HBM roof (how busy the memory system is)
        gbs = entry["traffic"] / (entry["avg_ms"] * 1e-3) * 1e-9
        entry["measured_traffic_gbs"] = gbs
        entry["measured_traffic_frac_of_hbm_peak"] = gbs / 8000.0
    if ai >= ridge:
        entry.update(bound="mfma", achieved=entry["tflops"], peak=entry["mfma_peak"], unit="TFLOP/s",
                     frac=entry["tflops"] / entry["mfma_peak"])
    else:
        gbs = entry["bytes_per_launch"] / (entry["avg_ms"] * 1e-3) * 1e-9
        entry.update(bound="hbm", achieved=gbs, peak=8000.0, unit="GB/s", frac=gbs / 8000.0)
    return entry


def factor_flops(S):
    """Algorithmic real flops of the fine level's block factorisation: per box
    and plane, the explicit inverse of a b x b complex Schur block by
    Gauss-Jordan (b^3 complex multiply-adds = 8 b^3 real flops; the sparse
    plane couplings add O(b^2))."""
    f = 0.0
    for s in range(S.num_subdomains(0)):
        bx = S.subdomain_box(s, 0)
        ex, ey, ez = (bx["ehi"][a] - bx["elo"][a] for a in range(3))
        f += ez * 8.0 * float(ex * ey) ** 3
    return f


def rel_err(helm, torch, X, Y, rows=8):
    """Relative L2 difference of each right-hand side, a few rows at a time (no full-size temporary)."""
    out = []
    for i in range(0, X.shape[0], rows):
        d = helm.torch_alloc(lambda: X[i:i + rows] - Y[i:i + rows])
        out.append(torch.linalg.vector_norm(d, dim=1) / torch.linalg.vector_norm(Y[i:i + rows], dim=1))
        del d
    return torch.cat(out)


def stencil_entry(kinds):
    """HBM roofline of the fine 27-point products of the timed solve, from live HIP events."""
    out = {"bound": "hbm", "peak": 8000.0, "unit": "GB/s"}
    tot_b = tot_ms = 0.0
    for name, st in zip(("A_x", "b_minus_A_x"), kinds):
        n = max(st["launches"], 1)
        out[name] = {"launches": st["launches"], "avg_ms": st["ms"] / n, "bytes_per_launch": st["bytes"] / n,
                     "achieved": st["bytes"] / max(st["ms"], 1e-9) * 1e-6,
                     "frac": st["bytes"] / max(st["ms"], 1e-9) * 1e-6 / 8000.0}
        tot_b += st["bytes"]
        tot_ms += st["ms"]
    out["achieved"] = tot_b / max(tot_ms, 1e-9) * 1e-6
    out["frac"] = out["achieved"] / 8000.0
    return out


def roofline_entry(st, dtype):
    ms = st["ms"] / max(st["launches"], 1)
    flops = st["flops"] / max(st["launches"], 1)
    achieved = flops / (ms * 1e-3) / 1e12
    e = {"bound": "mfma", "achieved": achieved, "peak": PEAK[dtype], "unit": "TFLOP/s",
         "frac": achieved / PEAK[dtype], "traffic": None, "traffic_source": None, "launches": st["launches"],
         "avg_ms": ms, "flops_per_launch": flops, "bytes_per_launch": st["bytes"] / max(st["launches"], 1),
         "tflops": achieved, "mfma_peak": PEAK[dtype]}
    return label_bound(e)


def cpu_baseline(w, its_per_rhs, nrhs, budget_s=25.0):
    """Oracle on a bounded sample of the workload, extrapolated to the full job.

    Sample: the same physics, spacing, box size (cores of 16^3 + overlap 2) and
    two-level method on a 3x3x3-box grid, one right-hand side.  Set-up cost
    scales with the number of boxes; solve cost per iteration with the number
    of boxes; the full job takes the GPU's iteration counts.
    """
    import inputs
    from oracle.operator import Pml, Problem, fit_weights
    from oracle.solve import setup, solve

    core = w["shape"][0] // w["parts"][0]
    ns = 3 * core
    nboxes_full = int(np.prod(w["parts"]))
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = 1
    ncpu = os.cpu_count() or 1
    # the local factorisations run in a process pool, one worker per box up to one per host core
    workers = max(1, min(27, ncpu, 16))
    c = inputs.velocity_thrust_belt(ns, ns, ns, H, q=w["q"])
    src = inputs.source_grid(ns, ns, NPML, NPML, 1, 1, iz=4)
    b = inputs.point_source_rhs(ns, ns, ns, src)
    prob = Problem((ns, ns, ns), H, c, FREQ, Pml(NPML, NPML, NPML, 0), fit_weights())
    from threadpoolctl import threadpool_limits
    t0 = time.perf_counter()
    with threadpool_limits(1):  # one LAPACK thread per worker process
        st = setup(prob, (3, 3, 3), 2, 2, workers=workers)
    t_setup = time.perf_counter() - t0
    res = solve(st, b, w["tol"], w["restart"], 60)
    it_s = max(1, int(res["iters"][0]))
    t_iter = res["t_solve"] / it_s
    scale = nboxes_full / 27.0
    t_full = t_setup * scale + t_iter * scale * float(np.sum(its_per_rhs))
    return {"value": nrhs / t_full, "unit": "RHS/s", "cores": max(workers, threads), "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": ncpu,
            "sample": (f"oracle set-up + one FGMRES solve of one source on a {ns}^3 grid with 3x3x3 boxes of the "
                       f"same size ({t_setup:.1f} s set-up with the banded factorisations in a pool of {workers} "
                       f"processes of one LAPACK thread each, {res['t_solve']:.1f} s for {it_s} iterations in one "
                       f"process with LAPACK on "
                       f"{threads} threads), scaled by {scale:.0f}x boxes and the GPU's iteration counts summed "
                       f"over all right-hand sides"),
            "extrapolated": True, "t_setup_full_s": t_setup * scale,
            "t_solve_full_s": t_iter * scale * float(np.sum(its_per_rhs))}


def cpu_model():
    """Host CPU model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def serving_phase(n_requests, max_rhs=64, seed=4, deadline=None):
    """Poisson stream over the seeded serving catalogue (grids 64^3..160^3, 2-8 Hz, 1-64 sources,
    two-level ORAS with 16^3 boxes, complex-FP32 local solves, tol 1e-6) at 0.8 x the capacity measured on a
    burst of the first requests; returns p50/p99 latency and RHS/s.  No request of the stream is submitted
    after ``deadline`` (time.perf_counter())."""
    import inputs
    from paper_2103_14921_amd.serving import ProblemSpec, Server, run_poisson
    cat = inputs.serving_catalogue(seed=seed)
    specs = [ProblemSpec(e["name"], (e["n"],) * 3, e["h"], e["freq"], (e["npml"],) * 3 + (0,), e["parts"])
             for e in cat]
    vel_cache = {}

    def vel(spec):
        if spec.name not in vel_cache:
            vel_cache[spec.name] = inputs.serving_velocity(cat[[s.name for s in specs].index(spec.name)])
        return vel_cache[spec.name]

    reqs = []
    for e, src in inputs.serving_requests(cat, n_requests, seed=seed, max_rhs=max_rhs):
        n = cat[e]["n"]
        B = inputs.point_source_rhs(n, n, n, src).reshape(len(src), -1)
        reqs.append((specs[e], B, 1e-6))
    ncal = max(4, n_requests // 4)
    srv = Server(vel, workers=4)
    t0 = time.perf_counter()
    for i, f in enumerate([srv.submit(*r) for r in reqs[:ncal]]):
        f.result()
        print(f"[bench] serving calibration {i + 1}/{ncal} done", file=sys.stderr, flush=True)
    capacity = ncal / (time.perf_counter() - t0)  # requests/s with set-ups included
    srv.stats.latencies.clear()
    out = run_poisson(srv, reqs[ncal:], rate_hz=0.8 * capacity, seed=seed, deadline=deadline,
                      progress=lambda i, n: print(f"[bench] serving request {i}/{n} done", file=sys.stderr,
                                                  flush=True))
    st = srv.stats
    srv.close()
    worst = max(float(r["relres_true"].max()) for r in out["results"])
    return {"requests": out["requests"], "requests_planned": len(reqs) - ncal, "calibration_requests": ncal,
            "rate_hz": 0.8 * capacity,
            "p50_s": out["p50_s"], "p99_s": out["p99_s"], "mean_s": out["mean_s"], "rhs_per_s": out["rhs_per_s"],
            "rhs": out["rhs"], "elapsed_s": out["elapsed_s"], "setups": st.setups, "evictions": st.evictions,
            "batches": st.batches, "retries": st.retries, "max_true_relres": worst}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="thrust192_mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--single-local", action="store_true",
                    help="also run with the coarse level's local solves in complex FP32")
    ap.add_argument("--no-block", action="store_true",
                    help="skip the block FGMRES run (one Krylov space per batch of right-hand sides)")
    ap.add_argument("--no-approx", action="store_true",
                    help="skip the run with approximate fine local solves (complex-FP16 plane inverses)")
    ap.add_argument("--serving-requests", type=int, default=12,
                    help="requests in the serving stream reported beside the main line (0: skip); a quarter "
                         "of them calibrate the capacity, the rest arrive as a Poisson stream")
    ap.add_argument("--serving-max-rhs", type=int, default=64, help="largest request of the serving stream")
    ap.add_argument("--no-graphs", action="store_true", help="launch every kernel directly (no captured iterations)")
    ap.add_argument("--retune", action="store_true",
                    help="tune the local-solve sweeps live instead of starting from the sweep decisions shipped in "
                         "paper_2103_14921_amd/tuned/mi355x_sweeps.txt (decisions within the timing noise of each "
                         "other can differ between processes; the shipped ones are those the committed counter "
                         "profiles were taken with)")
    ap.add_argument("--sweep-policy", default="auto",
                    help="force a local-solve sweep implementation (helm.SWEEP_POLICIES; e.g. for counter runs "
                         "that must see the same launches)")
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="wall-clock seconds (from start) the whole run aims to stay within: after the timed "
                         "steps, each comparison leg runs only if its estimated cost still fits (skipped legs "
                         "are listed), and the serving stream submits no request past the budget")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver is a single-device library (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if not args.retune and "HELM_TUNE_FILE" not in os.environ:
        # a private copy: decisions for shapes the file does not hold are appended to it, not to the shipped file
        import shutil
        import tempfile
        shipped = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2103_14921_amd", "tuned",
                               "mi355x_sweeps.txt")
        fd, tune_copy = tempfile.mkstemp(prefix="helm_tune_", suffix=".txt")
        os.close(fd)
        shutil.copyfile(shipped, tune_copy)
        os.environ["HELM_TUNE_FILE"] = tune_copy
        import atexit
        atexit.register(lambda: os.path.exists(tune_copy) and os.remove(tune_copy))

    import torch

    from paper_2103_14921_amd import helm

    w = WORKLOADS[args.workload]
    helm.set_sweep_policy(args.sweep_policy)
    c, b = make_inputs(w)
    nrhs = b.shape[0]
    dev = torch.device("cuda:0")
    c_dev = torch.from_numpy(c).to(dev)
    b_dev = torch.from_numpy(np.ascontiguousarray(b.reshape(nrhs, -1))).to(dev)
    weights = helm.fit_weights()
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)  # reads and writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()
    print(f"[bench] {describe(args.workload, w)}", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        _, info = gpu_solve(helm, w, c_dev, b_dev, w["precision"], weights, graphs=not args.no_graphs)
        print(f"[bench] warmup {i}: setup {info['timings']['setup']:.3f} s solve {info['timings']['solve']:.3f} s "
              f"iters {info['iters'].tolist()}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    setups, solves, infos = [], [], []
    for i in range(args.steps):
        X, info = gpu_solve(helm, w, c_dev, b_dev, w["precision"], weights, timing=True, graphs=not args.no_graphs)
        setups.append(info["timings"]["setup"])
        solves.append(info["timings"]["solve"])
        infos.append(info)
        print(f"[bench] step {i}: setup {setups[-1]:.3f} s solve {solves[-1]:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    info = infos[-1]
    value = nrhs * args.steps / T
    out = {
        "metric": "RHS solved/s to 1e-6 residual (mixed ORAS-FGMRES; FP64 form alongside; serving p50/p99)",
        "value": value, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"mixed": "c64 fine local factors/solves, c128 elsewhere",
                  "single_local": "c64 local factors/solves (both levels), c128 elsewhere"}.get(w["precision"], "c128"),
        "data": "synthetic (seeded thrust-belt velocity, unit point sources)",
        "config": {"workload": describe(args.workload, w), "grid": list(w["shape"]), "boxes": list(w["parts"]),
                   "nrhs": nrhs, "tol": w["tol"], "precision": w["precision"]},
        "solve_only_rhs_per_s": nrhs / float(np.mean(solves)),
        "setup_s": float(np.mean(setups)), "solve_s": float(np.mean(solves)),
        "iters": {"min": int(info["iters"].min()), "max": int(info["iters"].max()),
                  "mean": float(info["iters"].mean())},
        "max_true_relres": float(info["relres_true"].max()),
        "graphs": info["graphs"],
        # the whole solve against its roofline: every launch at max(bytes / 8 TB/s, flops / peak)
        "solve_roofline": {"bound_s": info["bound"]["seconds"], "solve_s": float(solves[-1]),
                           "frac": info["bound"]["seconds"] / float(solves[-1]),
                           "algorithmic_bytes": info["bound"]["bytes"], "algorithmic_flops": info["bound"]["flops"]},
    }
    # dominant kernel: the batched local solves of the coarse level (on MFMA in
    # the precision of its factors); the fine-level sweep alongside
    fine_dtype = "c128" if w["precision"] == "fp64" else "c64"
    coarse_dtype = "c64" if w["precision"] == "single_local" else "c128"
    if w["levels"] == 2:
        out["roofline"] = roofline_entry(info["sweeps"][1], coarse_dtype)
        out["roofline"]["kernel"] = ("k_oras_fused (coarse level, FP64 complex, MFMA 16x16x4 f64)" if coarse_dtype == "c128"
                                     else "k_oras_fused (coarse level, FP32 complex, MFMA f32)")
        set_traffic(out["roofline"], "ops_sweep.hip", f"oras_sweep_coarse_{args.workload}_pmc.md",
                    info.get("sweep_config"))
        out["roofline_fine_sweep"] = roofline_entry(info["sweeps"][0], fine_dtype)
    else:
        out["roofline"] = roofline_entry(info["sweeps"][0], fine_dtype)
        out["roofline"]["kernel"] = "k_oras_fused (fine level)"
    out["roofline_stencil"] = stencil_entry(info["stencil"])
    # the fine level's block factorisation (set-up), on MFMA in its factor precision
    t_fact = info["timings"]["factor"]
    ach = info["factor_flops"] / max(t_fact, 1e-9) / 1e12
    out["roofline_factorisation"] = {"bound": "mfma", "achieved": ach, "peak": PEAK[fine_dtype], "unit": "TFLOP/s",
                                     "frac": ach / PEAK[fine_dtype], "flops": info["factor_flops"], "seconds": t_fact}
    # comparison legs, most important first, each only while its estimated cost fits the time budget
    t_step = T / args.steps
    skipped = {}

    def fits(name, est_s):
        left = args.time_budget - (time.perf_counter() - T_START)
        if est_s <= left:
            return True
        skipped[name] = f"time budget: needs about {est_s:.0f} s, {max(left, 0.0):.0f} s left"
        print(f"[bench] skipping {name} ({skipped[name]})", file=sys.stderr, flush=True)
        return False

    if not args.no_fp64 and w["precision"] != "fp64" and fits("fp64_form", 1.9 * t_step):
        X64, i64 = gpu_solve(helm, w, c_dev, b_dev, "fp64", weights, graphs=not args.no_graphs)
        t64 = i64["timings"]["setup"] + i64["timings"]["solve"]
        err = rel_err(helm, torch, X, X64)
        out["fp64_form"] = {"rhs_per_s": nrhs / t64, "solve_only_rhs_per_s": nrhs / i64["timings"]["solve"],
                            "setup_s": i64["timings"]["setup"], "solve_s": i64["timings"]["solve"],
                            "iters_mean": float(i64["iters"].mean()),
                            "max_true_relres": float(i64["relres_true"].max())}
        out["mixed_vs_fp64_rel_l2_max"] = float(err.max().item())
        out["speedup_mixed_vs_fp64"] = value / out["fp64_form"]["rhs_per_s"]
        print("[bench] fp64 form done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        # the oracle on the host cores (a bounded sample, about 10-30 s); always run when asked for
        out["cpu_baseline"] = cpu_baseline(w, info["iters"], nrhs)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    if not args.no_approx and w["precision"] == "mixed" and fits("approx_local_form", 1.2 * t_step):
        # approximate fine local solves (complex-FP16 plane inverses on FP16 matrix cores; one step)
        Xa, iap = gpu_solve(helm, w, c_dev, b_dev, "approx_local", weights, timing=True, graphs=not args.no_graphs)
        tap = iap["timings"]["setup"] + iap["timings"]["solve"]
        out["approx_local_form"] = {
            "rhs_per_s": nrhs / tap, "solve_only_rhs_per_s": nrhs / iap["timings"]["solve"],
            "setup_s": iap["timings"]["setup"], "solve_s": iap["timings"]["solve"],
            "iters_mean": float(iap["iters"].mean()), "iters_max": int(iap["iters"].max()),
            "max_true_relres": float(iap["relres_true"].max()),
            "fine_sweep": roofline_entry(iap["sweeps"][0], "c32"),
            "solve_roofline_frac": iap["bound"]["seconds"] / iap["timings"]["solve"]}
        if "fp64_form" in out:
            out["approx_local_form"]["vs_fp64_rel_l2_max"] = float(rel_err(helm, torch, Xa, X64).max().item())
        del Xa
        print("[bench] approx_local form done", file=sys.stderr, flush=True)
    if not args.no_block and fits("block_form", 1.5 * t_step):
        # block FGMRES: the right-hand sides of each batch share one Krylov space (one step, same inputs)
        Xb, ibl = gpu_solve(helm, w, c_dev, b_dev, w["precision"], weights, graphs=not args.no_graphs, block=True)
        tbl = ibl["timings"]["setup"] + ibl["timings"]["solve"]
        out["block_form"] = {
            "rhs_per_s": nrhs / tbl, "solve_only_rhs_per_s": nrhs / ibl["timings"]["solve"],
            "setup_s": ibl["timings"]["setup"], "solve_s": ibl["timings"]["solve"],
            "block_iters_mean": float(ibl["iters"].mean()), "block_iters_max": int(ibl["iters"].max()),
            "max_true_relres": float(ibl["relres_true"].max()),
            "solve_roofline_frac": ibl["bound"]["seconds"] / ibl["timings"]["solve"]}
        if "fp64_form" in out:
            out["block_form"]["vs_fp64_rel_l2_max"] = float(rel_err(helm, torch, Xb, X64).max().item())
        del Xb
        print("[bench] block form done", file=sys.stderr, flush=True)
    if args.single_local and w["precision"] == "mixed" and fits("single_local_form", 1.2 * t_step):
        # the coarse level's local solves in complex FP32 too (one step, same inputs)
        Xs, isl = gpu_solve(helm, w, c_dev, b_dev, "single_local", weights, timing=True, graphs=not args.no_graphs)
        tsl = isl["timings"]["setup"] + isl["timings"]["solve"]
        out["single_local_form"] = {
            "rhs_per_s": nrhs / tsl, "solve_only_rhs_per_s": nrhs / isl["timings"]["solve"],
            "setup_s": isl["timings"]["setup"], "solve_s": isl["timings"]["solve"],
            "iters_mean": float(isl["iters"].mean()), "max_true_relres": float(isl["relres_true"].max()),
            "coarse_sweep": roofline_entry(isl["sweeps"][1], "c64"), "fine_sweep": roofline_entry(isl["sweeps"][0], "c64"),
            "solve_roofline_frac": isl["bound"]["seconds"] / isl["timings"]["solve"]}
        if args.workload == "thrust192_mixed":
            set_traffic(out["single_local_form"]["coarse_sweep"], "ops_sweep.hip",
                        "oras_sweep_coarse_thrust192_single_local_pmc.md", isl.get("sweep_config"))
        if "fp64_form" in out:
            err = rel_err(helm, torch, Xs, X64)
            out["single_local_form"]["vs_fp64_rel_l2_max"] = float(err.max().item())
        del Xs
    if "fp64_form" in out:
        del X64
    # the serving stream needs its calibration burst (about 30 s) and room for a few requests
    if args.serving_requests > 0 and fits("serving", 60.0):
        del X
        torch.cuda.empty_cache()
        helm.trim_cache()
        out["serving"] = serving_phase(args.serving_requests, args.serving_max_rhs,
                                       deadline=T_START + args.time_budget - 15.0)
    if skipped:
        out["skipped_legs"] = skipped
    out["bench_wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out))


if __name__ == "__main__":
    main()
