"""27-point mixed-grid FD Helmholtz operator with PML (oracle; test infrastructure).

Paper: Helmholtz equation (Delta + k^2) u = b with k = omega/c, c complex in
viscous media (eq. eqh); its discretisation A u = b (eq. eq1); absorbing
boundaries on the vertical and bottom faces and a homogeneous Dirichlet top;
the 27-point stencil that mixes consistent mass and stiffness on rotated
coordinate systems, weighted by coefficients fitted by least squares on the
numerical dispersion (FD-vs-FE section).  The paper gives no formulas for the
stencil, the PML or the weights; the readings taken here are:

  * time dependence e^{-i omega t}; PML stretch xi_d = 1 + i gamma_d/omega with
    gamma_d = gamma_max (dist/L)^2, gamma_max = 3 vmax/(2L) ln(1/R), R = 1e-3,
    L = npml*h, vmax = max Re c over the grid;
  * symmetric stretched form: row i multiplied by s_i = xi_x xi_y xi_z;
  * stiffness of lattice direction e (13 directions, both signs) has coefficient
    (alpha_e/h^2) a_e(m), a_e(m) = s(m) sum_d (e_d^2/|e|^2)/xi_d(m_d)^2 at the
    edge midpoint m; alpha_face = w1 + w2/3, alpha_edge = w2/6,
    alpha_corner = w3/4 (Cartesian system + mean of three 45-degree rotated
    systems + body-diagonal system);
  * consistent mass: off-diagonal wm_class * (sigma_i + sigma_j)/2 with
    sigma = s k^2 (the arithmetic mean keeps A = A^T); diagonal wm1 sigma_i;
  * ghost neighbours outside the grid are zero (Dirichlet): their stiffness
    still enters the diagonal, their off-diagonal entries are dropped; the top
    Dirichlet plane is the ghost plane iz = -1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

FACE = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
EDGE = ((1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1))
CORNER = ((1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1))
DIRECTIONS = FACE + EDGE + CORNER  # 13 lattice directions; each is used with both signs

PML_R = 1e-3


@dataclass
class Weights:
    """Mixed-grid stencil weights: stiffness w1+w2+w3 = 1, mass wm1+6wm2+12wm3+8wm4 = 1."""
    w1: float = 1.0
    w2: float = 0.0
    w3: float = 0.0
    wm1: float = 1.0
    wm2: float = 0.0
    wm3: float = 0.0
    wm4: float = 0.0

    def alphas(self):
        return (self.w1 + self.w2 / 3.0, self.w2 / 6.0, self.w3 / 4.0)

    def masses(self):
        return (self.wm2, self.wm3, self.wm4)

    def as_array(self):
        return np.array([self.w1, self.w2, self.w3, self.wm1, self.wm2, self.wm3, self.wm4])


SEVEN_POINT = Weights()  # textbook 7-point Laplacian with lumped mass


def _classes():
    return [(FACE, 0), (EDGE, 1), (CORNER, 2)]


def fit_weights(g_values=tuple(range(4, 11)), n_angles=15):
    """Least-squares fit of the mixed-grid weights on the dispersion relation.

    For a plane wave exp(i kappa n.x) the stencil gives
        sum_e alpha_e 2(1 - cos(kappa h n.e)) / h^2 = k^2 M(kappa),
        M = wm1 + 2 sum_e wm_class(e) cos(kappa h n.e),
    exact dispersion being k = kappa.  With kappa h = 2 pi/G (G points per
    wavelength), the residual  stiffness/(kappa h)^2 - M  is linear in the
    weights; it is minimised in the least-squares sense over G in g_values and
    n_angles x n_angles propagation directions in the first octant, with the two
    consistency constraints eliminated (w1 and wm1 are the dependent weights).
    Returns Weights.
    """
    rows, rhs = [], []
    for G in g_values:
        kh = 2.0 * np.pi / G
        for th in np.linspace(0.0, 0.5 * np.pi, n_angles):
            for ph in np.linspace(0.0, 0.5 * np.pi, n_angles):
                n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
                stiff = [sum(2.0 * (1.0 - np.cos(kh * np.dot(n, e))) for e in cls) / kh ** 2
                         for cls in (FACE, EDGE, CORNER)]
                cosm = [sum(2.0 * np.cos(kh * np.dot(n, e)) for e in cls) for cls in (FACE, EDGE, CORNER)]
                # unknowns p = (w2, w3, wm2, wm3, wm4); w1 = 1-w2-w3, wm1 = 1-6wm2-12wm3-8wm4
                # stiffness = (w1 + w2/3) S_f + (w2/6) S_e + (w3/4) S_c
                # mass      = wm1 + wm2 C_f + wm3 C_e + wm4 C_c
                row = [(-1.0 + 1.0 / 3.0) * stiff[0] + stiff[1] / 6.0,
                       -stiff[0] + stiff[2] / 4.0,
                       -(cosm[0] - 6.0), -(cosm[1] - 12.0), -(cosm[2] - 8.0)]
                rows.append(row)
                rhs.append(-(stiff[0] - 1.0))
    p, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
    w2, w3, wm2, wm3, wm4 = (float(v) for v in p)
    return Weights(1.0 - w2 - w3, w2, w3, 1.0 - 6.0 * wm2 - 12.0 * wm3 - 8.0 * wm4, wm2, wm3, wm4)


# Adaptive coefficients (FD-vs-FE section: the stencil's coefficients are
# matched to the local wavespeed).  Reading: a table of weight sets, entry j
# fitted on the band [G_j / 1.05, G_j * 1.05] (three G values) around
# G_j = ADAPT_G0 + j * ADAPT_DG points per wavelength, j < ADAPT_N (G from 3 to
# 10; above 10 every consistent stencil is accurate and the fit loses its
# conditioning, so larger G take the last entry); a node with G = Re(c)/(f h)
# takes the weights interpolated linearly in G between the two entries around
# it (clamped at the ends).
ADAPT_G0, ADAPT_DG, ADAPT_N = 3.0, 0.25, 29


def adaptive_table(g0=ADAPT_G0, dg=ADAPT_DG, n=ADAPT_N, n_angles=15):
    """Weight sets fitted per points-per-wavelength band (list of Weights, entry j at G = g0 + j dg)."""
    out = []
    for j in range(n):
        G = g0 + j * dg
        out.append(fit_weights(g_values=np.linspace(G / 1.05, G * 1.05, 3), n_angles=n_angles))
    return out


def interpolate_weights(table, G, g0=ADAPT_G0, dg=ADAPT_DG):
    """Weights at points per wavelength G (scalar): linear in G between table entries, clamped."""
    n = len(table)
    x = min(max((G - g0) / dg, 0.0), n - 1.0)
    j = min(int(np.floor(x)), n - 2)
    t = x - j
    a, b = table[j].as_array(), table[j + 1].as_array()
    return Weights(*((1.0 - t) * a + t * b))


def phase_velocity_ratio(w: Weights, G, theta, phi):
    """v_phase / c of the discrete stencil for a plane wave of G points per wavelength."""
    kh = 2.0 * np.pi / G
    n = np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    al = w.alphas()
    ms = w.masses()
    stiff = 0.0
    mass = w.wm1
    for (cls, ci) in _classes():
        for e in cls:
            ce = np.cos(kh * np.dot(n, e))
            stiff += al[ci] * 2.0 * (1.0 - ce)
            mass += ms[ci] * 2.0 * ce
    return np.sqrt(stiff / mass) / kh


@dataclass
class Pml:
    """PML thickness in nodes per side; zero means no PML on that side.

    ztop = 0 gives the homogeneous Dirichlet top of the paper.
    """
    x: int = 0
    y: int = 0
    zbot: int = 0
    ztop: int = 0
    R: float = PML_R


def pml_xi(n, npml_lo, npml_hi, h, omega, vmax, R=PML_R):
    """Stretch factors xi(t) = 1 + i gamma(t)/omega along one axis.

    Returns (xi_int[n], xi_half[n+1]): xi at the nodes t = 0..n-1 and at the
    half-integer positions t = j - 1/2, j = 0..n (xi_half[j] is the midpoint
    between nodes j-1 and j).  dist(t) = (npml_lo - t) h for t < npml_lo,
    (t - (n-1-npml_hi)) h for t > n-1-npml_hi, else 0.
    """
    def gamma(t):
        g = np.zeros_like(t)
        if npml_lo > 0:
            L = npml_lo * h
            gmax = 1.5 * vmax / L * np.log(1.0 / R)
            m = t < npml_lo
            g[m] = gmax * (((npml_lo - t[m]) * h) / L) ** 2
        if npml_hi > 0:
            L = npml_hi * h
            gmax = 1.5 * vmax / L * np.log(1.0 / R)
            m = t > (n - 1 - npml_hi)
            g[m] = gmax * (((t[m] - (n - 1 - npml_hi)) * h) / L) ** 2
        return g

    t_int = np.arange(n, dtype=np.float64)
    t_half = np.arange(n + 1, dtype=np.float64) - 0.5
    return 1.0 + 1j * gamma(t_int) / omega, 1.0 + 1j * gamma(t_half) / omega


@dataclass
class Problem:
    """Discrete Helmholtz problem: grid (nx, ny, nz), spacing h, complex velocity c[nz][ny][nx].

    adaptive=True replaces the one weight set by per-node weights from
    ``adaptive_table`` (``node_weights``): each edge (i, j) takes the mean of its
    two end nodes' stiffness weights, the mass coupling the mean of
    wm_class sigma at its two ends, the diagonal the node's own wm1 sigma_i (and
    its own stiffness weights toward ghost neighbours), so that A = A^T.
    """
    shape: tuple
    h: float
    c: np.ndarray
    freq: float
    pml: Pml
    weights: Weights = field(default_factory=lambda: SEVEN_POINT)
    adaptive: bool = False

    @property
    def n(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    @property
    def omega(self):
        return 2.0 * np.pi * self.freq

    def k(self):
        """Wavenumber k = omega/c per node, complex, [nz][ny][nx]."""
        return self.omega / self.c

    def profiles(self):
        nx, ny, nz = self.shape
        vmax = float(np.max(self.c.real))
        p = self.pml
        px = pml_xi(nx, p.x, p.x, self.h, self.omega, vmax, p.R)
        py = pml_xi(ny, p.y, p.y, self.h, self.omega, vmax, p.R)
        pz = pml_xi(nz, p.ztop, p.zbot, self.h, self.omega, vmax, p.R)
        return px, py, pz

    def sigma(self):
        """sigma = s k^2 with s = xi_x xi_y xi_z at the node, [nz][ny][nx]."""
        (xx, _), (xy, _), (xz, _) = self.profiles()
        s = xz[:, None, None] * xy[None, :, None] * xx[None, None, :]
        return s * self.k() ** 2

    def node_weights(self):
        """Per-node (alphas [3][nz][ny][nx], wm [4][nz][ny][nx]): the fixed weights everywhere, or with
        adaptive=True the table's weights at each node's G = Re(c)/(f h)."""
        nz_ny_nx = self.c.shape
        if not self.adaptive:
            al = np.array(self.weights.alphas())[:, None, None, None] * np.ones((1,) + nz_ny_nx)
            wm = np.array([self.weights.wm1, *self.weights.masses()])[:, None, None, None] * np.ones((1,) + nz_ny_nx)
            return al, wm
        if "_table" not in self.__dict__:
            self.__dict__["_table"] = np.array([w.as_array() for w in adaptive_table()])  # [n][7]
        T = self.__dict__["_table"]
        n = T.shape[0]
        G = self.c.real / (self.freq * self.h)
        x = np.clip((G - ADAPT_G0) / ADAPT_DG, 0.0, n - 1.0)
        j = np.minimum(np.floor(x).astype(np.int64), n - 2)
        t = x - j
        W = (1.0 - t)[..., None] * T[j] + t[..., None] * T[j + 1]  # [nz][ny][nx][7]: w1 w2 w3 wm1 wm2 wm3 wm4
        w1, w2, w3 = W[..., 0], W[..., 1], W[..., 2]
        al = np.stack([w1 + w2 / 3.0, w2 / 6.0, w3 / 4.0])
        wm = np.moveaxis(W[..., 3:7], -1, 0)
        return al, wm


def _midpoint_factor(profiles, e, sign):
    """a_e at the midpoint between each node i and i + sign*e, as a [nz][ny][nx] array."""
    sel = []
    for d in range(3):
        xi_int, xi_half = profiles[d]
        ed = sign * e[d]
        if ed == 0:
            sel.append(xi_int)
        elif ed > 0:
            sel.append(xi_half[1:])   # between i and i+1
        else:
            sel.append(xi_half[:-1])  # between i-1 and i
    xx, xy, xz = sel
    s = xz[:, None, None] * xy[None, :, None] * xx[None, None, :]
    e2 = float(e[0] ** 2 + e[1] ** 2 + e[2] ** 2)
    inv = (e[0] ** 2 / e2) / xx[None, None, :] ** 2 + (e[1] ** 2 / e2) / xy[None, :, None] ** 2 \
        + (e[2] ** 2 / e2) / xz[:, None, None] ** 2
    return s * inv


def assemble(prob: Problem):
    """Assemble A (scipy CSR, complex128, n x n) of the 27-point PML operator.

    Index of node (ix, iy, iz) is ix + nx (iy + ny iz).  Entries:
      A[i, i+-e] = (alpha_e/h^2) a_e(i +- e/2) + wm_class (sigma_i + sigma_{i+-e})/2
      A[i, i]    = -sum_{e,+-} (alpha_e/h^2) a_e(i +- e/2) + wm1 sigma_i
    (the diagonal sum runs over ghost neighbours too).
    """
    if prob.adaptive:
        return _assemble_adaptive(prob)
    nx, ny, nz = prob.shape
    h2 = prob.h ** 2
    prof = prob.profiles()
    sig = prob.sigma()
    al = prob.weights.alphas()
    ms = prob.weights.masses()
    idx = np.arange(prob.n, dtype=np.int64).reshape(nz, ny, nx)
    diag = prob.weights.wm1 * sig
    rows, cols, vals = [], [], []
    for cls, ci in _classes():
        for e in cls:
            ap = _midpoint_factor(prof, e, +1)
            am = _midpoint_factor(prof, e, -1)
            diag = diag - (al[ci] / h2) * (ap + am)
            # pairs (i, j = i + e) with both nodes in the grid
            ex, ey, ez = e
            sx = slice(max(0, -ex), nx - max(0, ex))
            sy = slice(max(0, -ey), ny - max(0, ey))
            sz = slice(max(0, -ez), nz - max(0, ez))
            tx = slice(max(0, ex), nx - max(0, -ex))
            ty = slice(max(0, ey), ny - max(0, -ey))
            tz = slice(max(0, ez), nz - max(0, -ez))
            i_idx = idx[sz, sy, sx].ravel()
            j_idx = idx[tz, ty, tx].ravel()
            v = (al[ci] / h2) * ap[sz, sy, sx].ravel() \
                + ms[ci] * 0.5 * (sig[sz, sy, sx].ravel() + sig[tz, ty, tx].ravel())
            rows += [i_idx, j_idx]
            cols += [j_idx, i_idx]
            vals += [v, v]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(prob.n, prob.n)).tocsr()
    A.sum_duplicates()
    return A


def _shifted(a, e, sign):
    """b[i] = a[i + sign e] where that node is in the grid, else a[i] (a: [..., nz, ny, nx])."""
    b = a.copy()
    nz, ny, nx = a.shape[-3:]
    ex, ey, ez = (sign * v for v in e)
    dst = (Ellipsis, slice(max(0, -ez), nz - max(0, ez)), slice(max(0, -ey), ny - max(0, ey)),
           slice(max(0, -ex), nx - max(0, ex)))
    src = (Ellipsis, slice(max(0, ez), nz - max(0, -ez)), slice(max(0, ey), ny - max(0, -ey)),
           slice(max(0, ex), nx - max(0, -ex)))
    b[dst] = a[src]
    return b


def _assemble_adaptive(prob: Problem):
    """``assemble`` with per-node weights (Problem.adaptive):
      A[i, j] = (alpha_e(i, j)/h^2) a_e(m) + (wm_class,i sigma_i + wm_class,j sigma_j)/2,
      alpha_e(i, j) = (alpha_e,i + alpha_e,j)/2,
      A[i, i] = -sum_{e,+-} (alpha_e(i, i+-e)/h^2) a_e(i +- e/2) + wm1,i sigma_i,
    a ghost neighbour j taking alpha_e(i, j) = alpha_e,i."""
    nx, ny, nz = prob.shape
    h2 = prob.h ** 2
    prof = prob.profiles()
    sig = prob.sigma()
    al, wm = prob.node_weights()
    idx = np.arange(prob.n, dtype=np.int64).reshape(nz, ny, nx)
    diag = wm[0] * sig
    rows, cols, vals = [], [], []
    for cls, ci in _classes():
        for e in cls:
            ap = _midpoint_factor(prof, e, +1)
            am = _midpoint_factor(prof, e, -1)
            a_p = 0.5 * (al[ci] + _shifted(al[ci], e, +1))
            a_m = 0.5 * (al[ci] + _shifted(al[ci], e, -1))
            diag = diag - (a_p / h2) * ap - (a_m / h2) * am
            ex, ey, ez = e
            sx = slice(max(0, -ex), nx - max(0, ex))
            sy = slice(max(0, -ey), ny - max(0, ey))
            sz = slice(max(0, -ez), nz - max(0, ez))
            tx = slice(max(0, ex), nx - max(0, -ex))
            ty = slice(max(0, ey), ny - max(0, -ey))
            tz = slice(max(0, ez), nz - max(0, -ez))
            i_idx = idx[sz, sy, sx].ravel()
            j_idx = idx[tz, ty, tx].ravel()
            ws = wm[ci + 1] * sig
            v = (a_p[sz, sy, sx].ravel() / h2) * ap[sz, sy, sx].ravel() \
                + 0.5 * (ws[sz, sy, sx].ravel() + ws[tz, ty, tx].ravel())
            rows += [i_idx, j_idx]
            cols += [j_idx, i_idx]
            vals += [v, v]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(prob.n, prob.n)).tocsr()
    A.sum_duplicates()
    return A


def row(prob: Problem, ix, iy, iz):
    """Row (ix, iy, iz) of A computed on its own: (global column indices, values).

    The same entries as ``assemble`` (FD-vs-FE section, readings in the module
    docstring), evaluated one neighbour at a time so that single rows of very
    large grids can be checked without assembling the matrix.
    """
    if prob.adaptive:
        return _row_adaptive(prob, ix, iy, iz)
    if "_row_cache" not in prob.__dict__:
        prob.__dict__["_row_cache"] = (prob.profiles(), prob.sigma())
    prof, sig = prob.__dict__["_row_cache"]
    nx, ny, nz = prob.shape
    h2 = prob.h ** 2
    al = prob.weights.alphas()
    ms = prob.weights.masses()
    pos = (ix, iy, iz)
    si = sig[iz, iy, ix]
    diag = prob.weights.wm1 * si
    cols, vals = [], []
    for cls, ci in _classes():
        for e in cls:
            for sign in (+1, -1):
                s = 1.0 + 0j
                inv = 0j
                e2 = float(e[0] ** 2 + e[1] ** 2 + e[2] ** 2)
                for d in range(3):
                    xi_int, xi_half = prof[d]
                    ed = sign * e[d]
                    xv = xi_int[pos[d]] if ed == 0 else (xi_half[pos[d] + 1] if ed > 0 else xi_half[pos[d]])
                    s = s * xv
                    inv = inv + (e[d] ** 2 / e2) / xv ** 2
                st = (al[ci] / h2) * (s * inv)
                diag = diag - st
                jx, jy, jz = ix + sign * e[0], iy + sign * e[1], iz + sign * e[2]
                if 0 <= jx < nx and 0 <= jy < ny and 0 <= jz < nz:
                    cols.append(jx + nx * (jy + ny * jz))
                    vals.append(st + ms[ci] * 0.5 * (si + sig[jz, jy, jx]))
    cols.append(ix + nx * (iy + ny * iz))
    vals.append(diag)
    return np.array(cols, dtype=np.int64), np.array(vals, dtype=np.complex128)


def _row_adaptive(prob: Problem, ix, iy, iz):
    """``row`` with per-node weights (the entries of ``_assemble_adaptive``), one neighbour at a time."""
    if "_row_cache_adaptive" not in prob.__dict__:
        prob.__dict__["_row_cache_adaptive"] = (prob.profiles(), prob.sigma(), prob.node_weights())
    prof, sig, (al, wm) = prob.__dict__["_row_cache_adaptive"]
    nx, ny, nz = prob.shape
    h2 = prob.h ** 2
    pos = (ix, iy, iz)
    si = sig[iz, iy, ix]
    diag = wm[0][iz, iy, ix] * si
    cols, vals = [], []
    for cls, ci in _classes():
        for e in cls:
            for sign in (+1, -1):
                s = 1.0 + 0j
                inv = 0j
                e2 = float(e[0] ** 2 + e[1] ** 2 + e[2] ** 2)
                for d in range(3):
                    xi_int, xi_half = prof[d]
                    ed = sign * e[d]
                    xv = xi_int[pos[d]] if ed == 0 else (xi_half[pos[d] + 1] if ed > 0 else xi_half[pos[d]])
                    s = s * xv
                    inv = inv + (e[d] ** 2 / e2) / xv ** 2
                jx, jy, jz = ix + sign * e[0], iy + sign * e[1], iz + sign * e[2]
                inside = 0 <= jx < nx and 0 <= jy < ny and 0 <= jz < nz
                a_i = al[ci][iz, iy, ix]
                a_e = 0.5 * (a_i + al[ci][jz, jy, jx]) if inside else a_i
                st = (a_e / h2) * (s * inv)
                diag = diag - st
                if inside:
                    cols.append(jx + nx * (jy + ny * jz))
                    vals.append(st + 0.5 * (wm[ci + 1][iz, iy, ix] * si + wm[ci + 1][jz, jy, jx] * sig[jz, jy, jx]))
    cols.append(ix + nx * (iy + ny * iz))
    vals.append(diag)
    return np.array(cols, dtype=np.int64), np.array(vals, dtype=np.complex128)
