"""The FD-vs-FE experiment of the paper (FD-vs-FE section, Table 1) on the GPU.

A 2 km x 4 km x 12 km medium (12 km deep) with c = c0 + alpha z, c0 = 1 km/s,
alpha = 0.8 and 2 /s, a point source at 1 km depth, 8 Hz, h = 31.25 m (4
points per wavelength at c0).  The HIP path solves it (two-level
ORAS-FGMRES, complex-FP32 local solves, FP64 true residual 1e-7) and the
solution is compared with the closed-form Green's function of the linear
gradient on the nodes outside the PML and more than 3 h from the source.

Readings where the paper gives no detail: PML of 40 nodes (1.25 km) on all six
faces (the analytic solution is the free-space one; with these layers the
grid has 14.1 M nodes, the paper's FD row has 13 M dof), velocity c0 in the
top layer, and the source spread over its 27 nodes with the consistent-mass
weights (b = M e_s / h^3): with a bare point source the discrete solution is
about 8 % too large at 4 points per wavelength, the consistent-mass symbol
at that sampling.

The paper prints relative l2 errors of 0.0079 (alpha = 0.8) and 0.044
(alpha = 2) for its FD scheme with adaptive stencil coefficients; those are
context (parity unpinned), and the test bounds the error loosely.  It runs
with the one fixed weight set and with the adaptive coefficients (weights
matched to each node's points per wavelength).
"""
import numpy as np
import pytest

from oracle.analytic import green_linear_gradient

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("adaptive", [False, True], ids=["fixed", "adaptive"])
@pytest.mark.parametrize("alpha,paper", [(0.8, 0.0079), (2.0, 0.044)])
def test_table1_linear_gradient_against_analytic(alpha, paper, adaptive):
    from paper_2103_14921_amd import helm
    h, f, c0, npml = 31.25, 8.0, 1000.0, 40
    ni = (65, 129, 385)  # 2 x 4 x 12 km, nodes on both ends
    nx, ny, nz = (n + 2 * npml for n in ni)
    z = (np.arange(nz) - npml) * h
    cz = c0 + alpha * np.maximum(z, 0.0)
    c = np.ascontiguousarray(np.broadcast_to(cz[:, None, None], (nz, ny, nx)).astype(np.complex128))
    sx, sy, sz = npml + 32, npml + 64, npml + 32  # centre of x and y, 1 km deep
    say("table1", alpha, "adaptive" if adaptive else "fixed", (nx, ny, nz))
    w = helm.fit_weights()
    if adaptive:  # the source spread with its own node's weights
        from oracle.operator import adaptive_table, interpolate_weights
        ws = interpolate_weights(adaptive_table(), c[sz, sy, sx].real / (f * h))
        wm = (ws.wm1, ws.wm2, ws.wm3, ws.wm4)
    else:
        wm = (w["wm1"], w["wm2"], w["wm3"], w["wm4"])
    b = np.zeros((1, nz, ny, nx), np.complex128)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                b[0, sz + dz, sy + dy, sx + dx] = wm[abs(dx) + abs(dy) + abs(dz)] / h ** 3
    S = helm.Solver((nx, ny, nz), h, c, f, (npml, npml, npml, npml), weights=w, parts=(8, 12, 27), overlap=2,
                    levels=2, precision="mixed", restart=30, adaptive=adaptive)
    X, info = S.solve(b, tol=1e-7, maxit=1000)
    S.close()
    assert info["relres_true"][0] <= 1e-7
    u = X.reshape(nz, ny, nx)[npml:nz - npml, npml:ny - npml, npml:nx - npml]
    zz, yy, xx = np.meshgrid(np.arange(ni[2]) * h, np.arange(ni[1]) * h, np.arange(ni[0]) * h, indexing="ij")
    xs, ys, zs = 32 * h, 64 * h, 32 * h
    r = np.sqrt((xx - xs) ** 2 + (yy - ys) ** 2 + (zz - zs) ** 2)
    m = r > 3 * h
    G = green_linear_gradient(xx[m], yy[m], zz[m], xs, ys, zs, 2 * np.pi * f, c0, alpha)
    um = u[m]
    err = float(np.linalg.norm(um - G) / np.linalg.norm(G))
    near = r[m] < 500.0
    err_near = float(np.linalg.norm(um[near] - G[near]) / np.linalg.norm(G[near]))
    say("alpha", alpha, "adaptive" if adaptive else "fixed", "dof", nx * ny * nz, "iterations",
        int(info["iters"][0]), "l2 error", round(err, 4), "within 500 m", round(err_near, 4), "paper FD", paper)
    assert err <= 0.06 and err_near <= 0.02
