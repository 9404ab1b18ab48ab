"""Overlapping decomposition and one-level ORAS (oracle; test infrastructure).

Paper, domain-decomposition section: an overlapping decomposition {Gamma_i} of
the grid, Boolean restrictions R_i, diagonal partition of unity D_i, local
operators A_i carrying absorbing (transmission) conditions on the subdomain
interfaces instead of the Dirichlet conditions of plain RAS, and the one-level
preconditioner M1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i (eq. oras).  Local
problems are solved by a direct method.

Readings where the paper is silent:
  * core boxes split each axis into p contiguous ranges of floor(n/p) nodes,
    the first (n mod p) one longer; the extended box adds delta layers on every
    side that is not a global boundary ("overlap 2" = 2 added layers per side);
  * D_i is Boolean: 1 on the core, 0 on the added layers, so sum R^T D R = I;
  * absorbing interface: for a box node l with a grid neighbour j outside the
    box, A_i[l, l] += A[l, j] (1 + i k_l h) -- the ghost value is replaced by
    the first-order outgoing condition u_j ~ (1 + i k h) u_l (a diagonal change,
    A_i stays complex symmetric); robin=False gives plain RAS;
  * local direct solver: LAPACK banded LU with partial pivoting in the natural
    ordering of the box (x fastest).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg.lapack as lapack
import scipy.sparse as sp


def split_axis(n, p):
    """Split range(n) into p contiguous ranges; sizes floor(n/p), the first n mod p one longer."""
    q, r = divmod(n, p)
    out, lo = [], 0
    for i in range(p):
        sz = q + (1 if i < r else 0)
        out.append((lo, lo + sz))
        lo += sz
    return out


@dataclass
class Box:
    """A subdomain: core [lo, hi) and extended [elo, ehi) ranges per axis (x, y, z)."""
    lo: tuple
    hi: tuple
    elo: tuple
    ehi: tuple

    @property
    def ext_shape(self):
        return tuple(self.ehi[d] - self.elo[d] for d in range(3))


def decompose(shape, parts, delta):
    """Boxes of a px x py x pz decomposition of grid ``shape`` = (nx, ny, nz), overlap delta.

    Subdomain order: x fastest, then y, then z.
    """
    ranges = [split_axis(shape[d], parts[d]) for d in range(3)]
    boxes = []
    for kz in range(parts[2]):
        for ky in range(parts[1]):
            for kx in range(parts[0]):
                lo = (ranges[0][kx][0], ranges[1][ky][0], ranges[2][kz][0])
                hi = (ranges[0][kx][1], ranges[1][ky][1], ranges[2][kz][1])
                boxes.append(extend(lo, hi, shape, delta))
    return boxes


def extend(lo, hi, shape, delta):
    elo = tuple(max(0, lo[d] - delta) for d in range(3))
    ehi = tuple(min(shape[d], hi[d] + delta) for d in range(3))
    return Box(tuple(lo), tuple(hi), elo, ehi)


def box_indices(shape, elo, ehi):
    """Global indices of the nodes of box [elo, ehi), in the box's natural order (x fastest)."""
    nx, ny, _ = shape
    z = np.arange(elo[2], ehi[2])
    y = np.arange(elo[1], ehi[1])
    x = np.arange(elo[0], ehi[0])
    return (x[None, None, :] + nx * (y[None, :, None] + ny * z[:, None, None])).ravel()


def core_mask(box):
    """Boolean D_i on the extended box (natural order): True on core nodes."""
    ex, ey, ez = box.ext_shape
    mx = np.zeros(ex, bool)
    my = np.zeros(ey, bool)
    mz = np.zeros(ez, bool)
    mx[box.lo[0] - box.elo[0]: box.hi[0] - box.elo[0]] = True
    my[box.lo[1] - box.elo[1]: box.hi[1] - box.elo[1]] = True
    mz[box.lo[2] - box.elo[2]: box.hi[2] - box.elo[2]] = True
    return (mz[:, None, None] & my[None, :, None] & mx[None, None, :]).ravel()


def local_matrix(A, shape, box, k_nodes, h, robin=True):
    """A_i = R_i A R_i^T plus the absorbing-interface fold on the diagonal.

    A: global CSR operator; k_nodes: complex wavenumber per global node (flat);
    h: grid spacing of this level.  For every box node l and every column j of
    row l that lies outside the box, A_i[l, l] += A[l, j] (1 + i k_l h).
    """
    idx = box_indices(shape, box.elo, box.ehi)
    rows = A[idx]                       # rows of the box nodes, all columns
    Ai = rows[:, idx].tocsr()
    if robin:
        inside = np.zeros(A.shape[1], bool)
        inside[idx] = True
        rc = rows.tocoo()
        outside = ~inside[rc.col]
        fold = np.zeros(len(idx), dtype=np.complex128)
        np.add.at(fold, rc.row[outside], rc.data[outside])
        kl = k_nodes[idx]
        Ai = Ai + sp.diags(fold * (1.0 + 1j * kl * h))
    return Ai.tocsr(), idx


class BandedLU:
    """Banded LU (LAPACK zgbtrf/zgbtrs, partial pivoting) of a local operator."""

    def __init__(self, Ai, ext_shape):
        ex, ey, _ = ext_shape
        n = Ai.shape[0]
        kl = ku = min(n - 1, ex * ey + ex + 1)
        coo = Ai.tocoo()
        ab = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128)
        ab[kl + ku + coo.row - coo.col, coo.col] = coo.data
        lu, piv, info = lapack.zgbtrf(ab, kl, ku, overwrite_ab=1)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrf info={info}")
        self.lu, self.piv, self.kl, self.ku = lu, piv, kl, ku

    def solve(self, b):
        b2 = b.reshape(b.shape[0], -1)
        x, info = lapack.zgbtrs(self.lu, self.kl, self.ku, b2, self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrs info={info}")
        return x.reshape(b.shape)

    @property
    def nbytes(self):
        return self.lu.nbytes


def _factor_one(args):
    Ai, ext_shape = args
    return BandedLU(Ai, ext_shape)


class Oras:
    """One-level ORAS  M1^{-1} r = sum_i R_i^T D_i A_i^{-1} R_i r  (eq. oras), Boolean D_i."""

    def __init__(self, A, shape, boxes, k_nodes, h, robin=True, workers=1):
        self.shape = shape
        self.boxes = boxes
        self.idx, self.core = [], []
        mats = []
        for b in boxes:
            Ai, idx = local_matrix(A, shape, b, k_nodes, h, robin)
            mats.append((Ai, b.ext_shape))
            self.idx.append(idx)
            self.core.append(core_mask(b))
        if workers > 1 and len(mats) > 1:
            from concurrent.futures import ProcessPoolExecutor
            with ProcessPoolExecutor(workers) as ex:
                self.lu = list(ex.map(_factor_one, mats))
        else:
            self.lu = [_factor_one(m) for m in mats]
        self.n = A.shape[0]

    def apply(self, r):
        out = np.zeros_like(r)
        for idx, core, lu in zip(self.idx, self.core, self.lu):
            xi = lu.solve(r[idx])
            out[idx[core]] = xi[core]
        return out

    @property
    def nbytes(self):
        return sum(lu.nbytes for lu in self.lu)


def local_matrix_from_rows(prob, box, robin=True):
    """A_i built row by row from ``operator.row`` (no global assembly): the same
    matrix as ``local_matrix`` (restriction + absorbing fold), usable on grids
    too large to assemble.  Returns CSR in the box's natural order."""
    from .operator import row
    nx, ny, _ = prob.shape
    idx = box_indices(prob.shape, box.elo, box.ehi)
    pos = -np.ones(prob.n, dtype=np.int64) if prob.n <= 50_000_000 else None
    lookup = {}
    if pos is not None:
        pos[idx] = np.arange(len(idx))
    else:
        lookup = {g: l for l, g in enumerate(idx)}
    k = prob.k()
    rows, cols, vals = [], [], []
    for l, g in enumerate(idx):
        ix, iy, iz = g % nx, (g // nx) % ny, g // (nx * ny)
        c, v = row(prob, ix, iy, iz)
        loc = pos[c] if pos is not None else np.array([lookup.get(int(cc), -1) for cc in c])
        inside = loc >= 0
        d = 0j
        if robin:
            d = v[~inside].sum() * (1.0 + 1j * k[iz, iy, ix] * prob.h)
        rows.append(np.full(inside.sum(), l))
        cols.append(loc[inside])
        vv = v[inside].copy()
        vv[loc[inside] == l] += d
        vals.append(vv)
    n = len(idx)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
