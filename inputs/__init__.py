"""Seeded synthetic inputs shared by the CPU oracle and the HIP library.

This module holds no arithmetic of the solver: it only draws velocity models,
source positions and right-hand sides, so that both sides of a parity test see
byte-identical inputs.

Velocity models follow the two media the paper uses:
  * a velocity increasing linearly with depth, c = c0 + alpha*z (the analytic
    test medium of the FD-vs-FE section, Table 1);
  * a layered "thrust belt" that stands in for the SEG/EAGE Overthrust model
    of the numerical-results section (that dataset is not available here).
    It is a seeded, Gaussian-smoothed layered model with dipping, gently
    folded interfaces and one thrust fault, velocities 2000-6000 m/s.

Array convention: node (ix, iy, iz) sits at (ix*h, iy*h, iz*h) with z the depth
axis pointing down; fields are C-ordered [nz][ny][nx] (x fastest).
"""
from __future__ import annotations

import numpy as np

THRUST_SEED = 210314921


def velocity_linear(nx, ny, nz, h, c0=1500.0, alpha=0.7, q=None):
    """c(z) = c0 + alpha*z evaluated at z = iz*h; complex128 [nz][ny][nx].

    With q given, the velocity is made complex, c*(1 - i/(2q)) (viscous medium).
    """
    z = np.arange(nz, dtype=np.float64) * h
    c = np.broadcast_to((c0 + alpha * z)[:, None, None], (nz, ny, nx)).astype(np.complex128)
    if q is not None:
        c = c * (1.0 - 0.5j / q)
    return np.ascontiguousarray(c)


def velocity_homogeneous(nx, ny, nz, c0=2000.0, q=None):
    c = np.full((nz, ny, nx), c0, dtype=np.complex128)
    if q is not None:
        c = c * (1.0 - 0.5j / q)
    return c


def velocity_thrust_belt(nx, ny, nz, h, seed=THRUST_SEED, q=None, vtop=2000.0, vbot=6000.0):
    """Seeded thrust-belt model on the box [0, nx*h) x [0, ny*h) x [0, nz*h).

    Eight interfaces at depths (l+1)*Lz/9 with a random jitter, a common dip
    across x (strike along y), gentle folding; nine layers whose velocities
    run from vtop to vbot with sorted random intermediates; one thrust fault
    whose hanging wall is the layered model shifted up-dip by a random slip;
    clipped to [vtop, vbot] and Gaussian-smoothed with sigma = 2 cells.
    Returns complex128 [nz][ny][nx]; with q given, c*(1 - i/(2q)).
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    lx, ly, lz = nx * h, ny * h, nz * h
    nl = 8
    base = (np.arange(nl) + 1.0) * lz / 9.0 + rng.uniform(-0.3, 0.3, nl) * lz / 9.0
    dip = np.deg2rad(rng.uniform(5.0, 20.0))
    amp = rng.uniform(0.0, 0.03 * lz, nl)
    lam = rng.uniform(0.5, 1.5, nl) * lx
    phase = rng.uniform(0.0, 2.0 * np.pi, nl)
    vmid = np.sort(rng.uniform(vtop, vbot, nl - 1))
    vel_layers = np.concatenate([[vtop], vmid, [vbot]])
    fdip = np.deg2rad(rng.uniform(25.0, 40.0))
    xf = rng.uniform(0.35, 0.65) * lx
    slip = rng.uniform(0.08, 0.15) * lz
    # a gentle along-strike undulation of the fault trace makes the model 3-D
    yamp = rng.uniform(0.02, 0.06) * lx
    yphase = rng.uniform(0.0, 2.0 * np.pi)

    x = np.arange(nx, dtype=np.float64) * h
    y = np.arange(ny, dtype=np.float64) * h
    z = np.arange(nz, dtype=np.float64) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")

    def layered(xx, zz):
        idx = np.zeros(zz.shape, dtype=np.int64)
        for l in range(nl):
            depth = base[l] + np.tan(dip) * (xx - 0.5 * lx) + amp[l] * np.sin(2.0 * np.pi * xx / lam[l] + phase[l])
            idx += (zz > depth).astype(np.int64)
        return vel_layers[idx]

    # fault plane: x_fault(z, y) = xf + yamp*sin(2 pi y/ly + yphase) - z/tan(fdip)
    xfault = xf + yamp * np.sin(2.0 * np.pi * Y / ly + yphase) - Z / np.tan(fdip)
    hanging = X < xfault
    v = layered(X, Z)
    # the hanging wall came from further down-dip: sample the layering there
    xs = X - slip * np.cos(fdip)
    zs = Z + slip * np.sin(fdip)
    v_hw = layered(xs, zs)
    v = np.where(hanging, v_hw, v)
    v = np.clip(v, vtop, vbot)
    v = gaussian_filter(v, sigma=2.0, mode="nearest")
    c = v.astype(np.complex128)
    if q is not None:
        c = c * (1.0 - 0.5j / q)
    return np.ascontiguousarray(c)


def source_grid(nx, ny, npml_x, npml_y, n_sx, n_sy, iz=4):
    """Regular grid of point sources over the non-PML interior at depth index iz.

    Source r = j*n_sx + i sits at x index npml_x + floor((i+1/2)*(nx-2*npml_x)/n_sx)
    and likewise in y.  Returns an int array [n_sx*n_sy][3] of (ix, iy, iz).
    """
    out = []
    for j in range(n_sy):
        for i in range(n_sx):
            ix = npml_x + int(np.floor((i + 0.5) * (nx - 2 * npml_x) / n_sx))
            iy = npml_y + int(np.floor((j + 0.5) * (ny - 2 * npml_y) / n_sy))
            out.append((ix, iy, iz))
    return np.array(out, dtype=np.int64)


def point_source_rhs(nx, ny, nz, sources, value=1.0 + 0.0j):
    """Unit point sources: B[r] = value at sources[r], zero elsewhere.

    Returns complex128 [nrhs][nz][ny][nx] (each right-hand side a contiguous field).
    """
    sources = np.asarray(sources, dtype=np.int64).reshape(-1, 3)
    b = np.zeros((len(sources), nz, ny, nx), dtype=np.complex128)
    for r, (ix, iy, iz) in enumerate(sources):
        b[r, iz, iy, ix] = value
    return b


def random_field(shape, seed, dtype=np.complex128):
    """Seeded standard-normal complex field (real and imaginary parts independent)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return np.ascontiguousarray(a.astype(dtype))


# ---------------------------------------------------------------------------
# Workload catalogue.  Sizes, media, decompositions and tolerances of the five
# workloads the solver is measured on.  "parts" is the number of subdomains per
# axis; delta the overlap in added layers; levels 1 or 2.
# ---------------------------------------------------------------------------

WORKLOADS = {
    "c1_gradient24": dict(
        shape=(24, 24, 24), h=50.0, freq=3.75, model="linear", npml=(6, 6, 6, 0),
        parts=(2, 2, 2), delta=2, levels=1, restart=30, tol=1e-8, sources="single",
        precision="fp64"),
    "c2_thrust128": dict(
        shape=(128, 128, 128), h=25.0, freq=10.0, model="thrust", npml=(10, 10, 10, 0),
        parts=(4, 4, 4), delta=2, levels=2, restart=30, tol=1e-8, sources=(4, 2),
        precision="fp64"),
    "c3_thrust192_mixed": dict(
        shape=(192, 192, 192), h=25.0, freq=10.0, model="thrust", npml=(10, 10, 10, 0),
        parts=(12, 12, 12), delta=2, levels=2, restart=20, tol=1e-6, sources=(8, 8),
        precision="mixed"),
    "c5_thrust256_q100": dict(
        shape=(256, 256, 128), h=25.0, freq=10.0, model="thrust_q100", npml=(10, 10, 10, 0),
        parts=(16, 16, 8), delta=2, levels=2, restart=20, tol=1e-6, sources=(16, 8),
        precision="mixed"),
}


def workload_inputs(name, shape=None, n_src=None):
    """Velocity (complex128 [nz][ny][nx]) and RHS ([nrhs][nz][ny][nx]) of a workload.

    ``shape`` / ``n_src`` optionally override the grid and the source grid
    (scaled-down copies for tests).
    """
    w = dict(WORKLOADS[name])
    nx, ny, nz = shape if shape is not None else w["shape"]
    h = w["h"]
    if w["model"] == "linear":
        c = velocity_linear(nx, ny, nz, h)
    elif w["model"] == "thrust":
        c = velocity_thrust_belt(nx, ny, nz, h)
    elif w["model"] == "thrust_q100":
        c = velocity_thrust_belt(nx, ny, nz, h, q=100.0)
    else:
        raise ValueError(w["model"])
    npx, npy = w["npml"][0], w["npml"][1]
    if w["sources"] == "single":
        src = np.array([[nx // 2, ny // 2, 4]], dtype=np.int64)
    else:
        sx, sy = n_src if n_src is not None else w["sources"]
        src = source_grid(nx, ny, npx, npy, sx, sy, iz=4)
    b = point_source_rhs(nx, ny, nz, src)
    return c, b, src


# ---------------------------------------------------------------------------
# Serving workload: a seeded catalogue of (model, grid, frequency) problems and
# a stream of requests drawn from it (grids 64^3..160^3, 2-8 Hz, 1-64 sources).
# ---------------------------------------------------------------------------

def serving_catalogue(n_entries=16, seed=4, grids=(64, 96, 128, 160), core=16, npml=10, pml_wavelengths=0.3):
    """List of dicts(name, model, n, h, freq, parts, npml): n^3 grids, h = min(25, vmin/(8 f)),
    boxes of core^3 nodes per axis, PML at least pml_wavelengths of the longest wavelength
    (and at least npml nodes) thick: a layer much thinner than the wavelength leaves the
    low-frequency problems of the catalogue nearly undamped cavities."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_entries):
        model = "thrust" if rng.uniform() < 0.5 else "linear"
        n = int(grids[rng.integers(0, len(grids))])
        f = float(rng.uniform(2.0, 8.0))
        vmin = 2000.0 if model == "thrust" else 1500.0
        h = min(25.0, vmin / (8.0 * f))
        vmax = 6000.0 if model == "thrust" else 1500.0 + 0.7 * (n - 1) * h
        layer = max(npml, int(np.ceil(pml_wavelengths * vmax / (f * h))))
        out.append(dict(name=f"{model}{n}_{i}", model=model, n=n, h=h, freq=f, parts=(n // core,) * 3, npml=layer))
    return out


def serving_velocity(entry):
    n, h = entry["n"], entry["h"]
    if entry["model"] == "thrust":
        return velocity_thrust_belt(n, n, n, h)
    return velocity_linear(n, n, n, h)


def serving_requests(catalogue, n_requests, seed=4, max_rhs=64):
    """(entry index, sources [nrhs][3]) per request: entry uniform over the catalogue,
    1..max_rhs sources at distinct random positions of the non-PML interior, depth index 4."""
    rng = np.random.default_rng(seed + 1)
    reqs = []
    for _ in range(n_requests):
        e = int(rng.integers(0, len(catalogue)))
        ent = catalogue[e]
        n, p = ent["n"], ent["npml"]
        k = int(rng.integers(1, max_rhs + 1))
        cells = rng.choice((n - 2 * p) * (n - 2 * p), size=k, replace=False)
        src = np.stack([p + cells % (n - 2 * p), p + cells // (n - 2 * p), np.full(k, 4)], axis=1)
        reqs.append((e, src.astype(np.int64)))
    return reqs
