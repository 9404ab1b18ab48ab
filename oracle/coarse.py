"""Coarse space and two-level preconditioner (oracle; test infrastructure).

Paper, domain-decomposition section (eq. 2lvl):
    M^{-1} = M1^{-1} (I - A Q) + Q,   Q = Z E^{-1} Z^T,   E = Z^T A Z,
with M1^{-1} the one-level ORAS; the coarse problem E is solved by 10 GMRES
iterations preconditioned by a one-level ORAS on the same spatial partition.

Readings for the FD grid (the paper describes the coarse space for FE meshes):
  * the coarse grid has spacing 2h: coarse node (I, J, K) sits at fine node
    (2I, 2J, 2K), I < ceil(nx/2) and likewise in y and z;
  * Z (fine x coarse) is trilinear interpolation, weight
    prod_d max(0, 1 - |x_d - 2 I_d|/2); Z^T its transpose (restriction);
  * E is the Galerkin product Z^T A Z (a 27-point coarse stencil);
  * coarse core i = coarse nodes whose fine position lies in fine core i,
    extended by delta coarse layers; the absorbing fold uses the k of the
    co-located fine node and h_c = 2h; Boolean partition of unity;
  * coarse solve: GMRES from x0 = 0, exactly 10 iterations, no restart.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .dd import Box, Oras, extend
from .krylov import gmres_fixed


def coarse_shape(shape):
    return tuple((n + 1) // 2 for n in shape)


def _interp_1d(n):
    """1-D linear interpolation from the coarse points 2I (I < ceil(n/2)) to the fine points 0..n-1."""
    nc = (n + 1) // 2
    rows, cols, vals = [], [], []
    for i in range(n):
        for I in range(nc):
            w = max(0.0, 1.0 - abs(i - 2 * I) / 2.0)
            if w > 0.0:
                rows.append(i)
                cols.append(I)
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def prolongation(shape):
    """Z: trilinear interpolation, CSR (n_fine x n_coarse), index x fastest on both grids."""
    nx, ny, nz = shape
    Zx, Zy, Zz = _interp_1d(nx), _interp_1d(ny), _interp_1d(nz)
    # index = ix + nx (iy + ny iz): kron(Zz, kron(Zy, Zx))
    return sp.kron(Zz, sp.kron(Zy, Zx, format="csr"), format="csr")


def coarse_boxes(fine_boxes, fine_shape, delta):
    """Coarse core = coarse nodes I with 2I in the fine core; extended by delta coarse layers."""
    cs = coarse_shape(fine_shape)
    out = []
    for b in fine_boxes:
        lo = tuple((b.lo[d] + 1) // 2 for d in range(3))
        hi = tuple((b.hi[d] + 1) // 2 for d in range(3))
        out.append(extend(lo, hi, cs, delta))
    return out


def coarse_k(k_fine, fine_shape):
    """k of the fine node co-located with each coarse node (flat, coarse order)."""
    nx, ny, nz = fine_shape
    k3 = k_fine.reshape(nz, ny, nx)
    return np.ascontiguousarray(k3[::2, ::2, ::2]).ravel()


class TwoLevel:
    """M^{-1} r = M1^{-1} (r - A Q r) + Q r with Q r = Z GMRES10(E, Z^T r) (eq. 2lvl)."""

    def __init__(self, A, shape, boxes, k_nodes, h, delta, robin=True, coarse_iters=10, workers=1,
                 fine=None):
        self.A = A
        self.Z = prolongation(shape)
        self.ZT = self.Z.T.tocsr()
        self.E = (self.ZT @ A @ self.Z).tocsr()
        self.cshape = coarse_shape(shape)
        self.cboxes = coarse_boxes(boxes, shape, delta)
        kc = coarse_k(k_nodes, shape)
        self.fine = fine if fine is not None else Oras(A, shape, boxes, k_nodes, h, robin, workers)
        self.coarse = Oras(self.E, self.cshape, self.cboxes, kc, 2.0 * h, robin, workers)
        self.coarse_iters = coarse_iters

    def coarse_solve(self, c):
        return gmres_fixed(lambda v: self.E @ v, self.coarse.apply, c, self.coarse_iters)

    def q(self, r):
        return self.Z @ self.coarse_solve(self.ZT @ r)

    def apply(self, r):
        qr = self.q(r)
        return self.fine.apply(r - self.A @ qr) + qr

    @property
    def nbytes(self):
        return self.fine.nbytes + self.coarse.nbytes
