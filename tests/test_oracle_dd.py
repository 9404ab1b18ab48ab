"""Pins of the oracle's decomposition, local operators, ORAS and two-level preconditioner (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import inputs
from oracle.coarse import TwoLevel, coarse_boxes, coarse_shape, prolongation
from oracle.dd import BandedLU, Oras, box_indices, core_mask, decompose, local_matrix, split_axis
from oracle.krylov import fgmres, gmres_fixed
from oracle.operator import Pml, Problem, assemble, fit_weights

W = fit_weights()


def _prob(shape=(12, 10, 9), h=50.0, f=3.75, pml=(3, 3, 3, 0), q=None):
    c = inputs.velocity_linear(*shape, h=h, q=q)
    return Problem(shape, h, c, f, Pml(*pml), W)


def test_split_axis():
    assert split_axis(10, 3) == [(0, 4), (4, 7), (7, 10)]
    assert split_axis(192, 12) == [(16 * i, 16 * i + 16) for i in range(12)]
    assert split_axis(5, 5) == [(i, i + 1) for i in range(5)]


def test_partition_of_unity_is_identity():
    shape = (13, 9, 11)
    boxes = decompose(shape, (3, 2, 2), 2)
    n = 13 * 9 * 11
    acc = np.zeros(n)
    for b in boxes:
        idx = box_indices(shape, b.elo, b.ehi)
        acc[idx[core_mask(b)]] += 1.0
        # the extension is delta on interior sides only
        for d in range(3):
            assert b.elo[d] == max(0, b.lo[d] - 2) and b.ehi[d] == min(shape[d], b.hi[d] + 2)
    assert np.all(acc == 1.0)


def test_robin_fold_is_diagonal_outside_row_sum():
    prob = _prob()
    A = assemble(prob)
    k = prob.k().ravel()
    boxes = decompose(prob.shape, (2, 2, 2), 2)
    for b in boxes:
        Ai, idx = local_matrix(A, prob.shape, b, k, prob.h, robin=True)
        Ad, _ = local_matrix(A, prob.shape, b, k, prob.h, robin=False)
        D = (Ai - Ad).tocoo()
        assert np.all(D.row == D.col)
        # outside row sums via a global matvec with the indicator of the outside
        out = np.ones(prob.n)
        out[idx] = 0.0
        rs = (A @ out)[idx]
        ref = rs * (1.0 + 1j * k[idx] * prob.h)
        diag = np.asarray((Ai - Ad).diagonal())
        assert np.allclose(diag, ref, rtol=1e-13, atol=1e-13 * np.abs(A.diagonal()).max())
        assert (Ai - Ai.T).count_nonzero() == 0


def test_banded_lu_matches_dense():
    prob = _prob(q=30.0)
    A = assemble(prob)
    b = decompose(prob.shape, (2, 2, 2), 2)[5]
    Ai, _ = local_matrix(A, prob.shape, b, prob.k().ravel(), prob.h)
    lu = BandedLU(Ai, b.ext_shape)
    rhs = inputs.random_field((Ai.shape[0], 3), seed=7)
    x = lu.solve(rhs)
    xd = np.linalg.solve(Ai.toarray(), rhs)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_oras_matches_dense_sum():
    prob = _prob(shape=(8, 7, 6), pml=(2, 2, 2, 0))
    A = assemble(prob)
    k = prob.k().ravel()
    boxes = decompose(prob.shape, (2, 2, 1), 1)
    M = Oras(A, prob.shape, boxes, k, prob.h)
    r = inputs.random_field(prob.n, seed=11)
    ref = np.zeros(prob.n, complex)
    for b in boxes:
        Ai, idx = local_matrix(A, prob.shape, b, k, prob.h)
        D = core_mask(b).astype(float)
        ref[idx] += D * np.linalg.solve(Ai.toarray(), r[idx])
    assert np.linalg.norm(M.apply(r) - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("levels", [1, 2])
def test_single_subdomain_converges_in_one_iteration(levels):
    prob = _prob(shape=(10, 9, 8), pml=(3, 3, 3, 0))
    A = assemble(prob)
    k = prob.k().ravel()
    boxes = decompose(prob.shape, (1, 1, 1), 2)
    if levels == 1:
        M = Oras(A, prob.shape, boxes, k, prob.h)
    else:
        M = TwoLevel(A, prob.shape, boxes, k, prob.h, 2)
    b = np.zeros(prob.n, complex)
    b[4 + 10 * (4 + 9 * 3)] = 1.0
    x, it, est, tru = fgmres(lambda v: A @ v, M.apply, b, 1e-10, 20, 20)
    assert it == 1 and tru <= 1e-10


def test_two_level_with_exact_coarse_solve_reproduces_Z():
    # M^{-1} A Z = Z when E^{-1} is applied exactly (eq. 2lvl)
    prob = _prob(shape=(9, 8, 7), pml=(2, 2, 2, 0))
    A = assemble(prob)
    boxes = decompose(prob.shape, (2, 2, 1), 2)
    tl = TwoLevel(A, prob.shape, boxes, prob.k().ravel(), prob.h, 2)
    Elu = spla.splu(tl.E.tocsc())
    tl.coarse_solve = Elu.solve
    Z = tl.Z.toarray()
    for j in (0, 7, Z.shape[1] - 1):
        got = tl.apply(A @ Z[:, j])
        assert np.linalg.norm(got - Z[:, j]) <= 1e-10 * np.linalg.norm(Z[:, j])


def test_prolongation_interpolates_linear_functions():
    shape = (9, 7, 5)       # odd sizes: every fine node lies in the coarse hull
    Z = prolongation(shape)
    cs = coarse_shape(shape)
    assert cs == (5, 4, 3)
    I = np.arange(cs[0]) * 2.0
    J = np.arange(cs[1]) * 2.0
    K = np.arange(cs[2]) * 2.0
    fc = (1.0 + 0.5 * I[None, None, :] - 0.25 * J[None, :, None] + 2.0 * K[:, None, None]).ravel()
    x = np.arange(shape[0])
    y = np.arange(shape[1])
    z = np.arange(shape[2])
    ff = (1.0 + 0.5 * x[None, None, :] - 0.25 * y[None, :, None] + 2.0 * z[:, None, None]).ravel()
    assert np.allclose(Z @ fc, ff, atol=1e-13)
    assert np.allclose(np.asarray(Z.sum(axis=1)).ravel(), 1.0)


def test_galerkin_coarse_operator_symmetric_27_point():
    prob = _prob(shape=(12, 10, 9))
    A = assemble(prob)
    Z = prolongation(prob.shape)
    E = (Z.T @ A @ Z).tocsr()
    assert abs(E - E.T).max() <= 1e-12 * abs(E).max()
    assert max(np.diff(E.indptr)) == 27


def test_coarse_boxes_cover_coarse_grid():
    shape = (20, 18, 14)
    boxes = decompose(shape, (3, 2, 2), 2)
    cb = coarse_boxes(boxes, shape, 2)
    cs = coarse_shape(shape)
    acc = np.zeros(np.prod(cs))
    for b in cb:
        acc[box_indices(cs, b.elo, b.ehi)[core_mask(b)]] += 1
    assert np.all(acc == 1)


def test_gmres_fixed_exact_when_dimension_at_most_iterations():
    rng = np.random.default_rng(5)
    n = 8
    E = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    P = np.diag(1.0 / np.diag(E))
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = gmres_fixed(lambda v: E @ v, lambda v: P @ v, c, 10)
    assert np.linalg.norm(E @ x - c) <= 1e-10 * np.linalg.norm(c)


def test_gmres_fixed_is_minimal_residual():
    # the 10-step iterate minimises ||c - E M^{-1} K y|| over the Krylov space,
    # computed here from an explicit power basis, QR and least squares
    rng = np.random.default_rng(9)
    n = 60
    E = np.diag(np.linspace(1, 3, n)) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    P = np.diag(1.0 / (1.0 + 0.1 * np.arange(n)))
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = gmres_fixed(lambda v: E @ v, lambda v: P @ v, c, 10)
    EP = E @ P
    K = np.zeros((n, 10), complex)
    v = c / np.linalg.norm(c)
    for j in range(10):
        K[:, j] = v
        v = EP @ v
        v /= np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(EP @ Q, c, rcond=None)
    x_ref = P @ (Q @ y)
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def test_absorbing_interfaces_beat_dirichlet_and_wrong_sign():
    # the paper's point about ORAS: absorbing interface conditions make the
    # preconditioner far better than the Dirichlet conditions of plain RAS; the
    # outgoing sign (1 + i k h) for e^{-i omega t} must also beat (1 - i k h)
    prob = _prob(shape=(20, 20, 20), pml=(5, 5, 5, 0))
    A = assemble(prob)
    k = prob.k().ravel()
    boxes = decompose(prob.shape, (2, 2, 2), 2)
    b = np.zeros(prob.n, complex)
    b[10 + 20 * (10 + 20 * 4)] = 1.0
    its = {}
    for name, kk, robin in (("oras", k, True), ("ras", k, False), ("wrong", -k, True)):
        M = Oras(A, prob.shape, boxes, kk, prob.h, robin)
        its[name] = fgmres(lambda v: A @ v, M.apply, b, 1e-8, 30, 300)[1]
    assert its["oras"] < its["ras"] / 2
    assert its["oras"] < its["wrong"]


def test_local_matrix_from_rows_matches_restriction():
    from oracle.dd import local_matrix_from_rows
    prob = _prob(shape=(13, 11, 10), pml=(3, 3, 3, 0), q=40.0)
    A = assemble(prob)
    for b in decompose(prob.shape, (2, 2, 2), 2)[::3]:
        Ai, _ = local_matrix(A, prob.shape, b, prob.k().ravel(), prob.h)
        Bi = local_matrix_from_rows(prob, b)
        assert abs(Ai - Bi).max() <= 1e-13 * abs(Ai).max()


def _co_located_rows(Z):
    # fine node co-located with each coarse node: the one fine row where the
    # trilinear weight of that coarse node is exactly 1 (Z is pinned above by
    # reproducing linear functions)
    Zc = Z.tocsc()
    rows = []
    for c in range(Z.shape[1]):
        col = Zc[:, c].tocoo()
        one = col.row[col.data == 1.0]
        assert len(one) == 1
        rows.append(int(one[0]))
    return np.array(rows)


def test_coarse_k_takes_k_of_the_co_located_fine_node():
    from oracle.coarse import coarse_k
    shape = (9, 8, 7)  # odd and even sizes, not a cube
    rng = np.random.default_rng(3)
    n = int(np.prod(shape))
    k = rng.standard_normal(n) + 1j * rng.standard_normal(n)  # distinct per node
    rows = _co_located_rows(prolongation(shape))
    assert np.array_equal(coarse_k(k, shape), k[rows])


def test_coarse_fold_uses_co_located_k_and_the_coarse_spacing():
    # the coarse local problems of eq. 2lvl carry the absorbing fold with the k
    # of each coarse node's co-located fine node and the coarse grid's own node
    # spacing (the distance between co-located fine nodes of neighbouring
    # coarse nodes), both read here off Z, not off the oracle's coarse code
    import scipy.sparse.linalg as spla
    prob = _prob(shape=(14, 12, 11), pml=(3, 3, 3, 0), q=30.0)
    A = assemble(prob)
    k = prob.k().ravel()
    boxes = decompose(prob.shape, (2, 2, 1), 2)
    tl = TwoLevel(A, prob.shape, boxes, k, prob.h, 2)
    rows = _co_located_rows(tl.Z)
    nx, ny, _ = prob.shape
    pos = np.stack([rows % nx, (rows // nx) % ny, rows // (nx * ny)], 1) * prob.h
    spacing = np.linalg.norm(pos[1] - pos[0])  # coarse nodes 0 and 1 are neighbours along x
    assert spacing > prob.h
    kc = k[rows]
    rng = np.random.default_rng(8)
    for i, cb in enumerate(tl.cboxes):
        Ai, idx = local_matrix(tl.E, tl.cshape, cb, kc, spacing)
        r = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
        want = spla.spsolve(Ai.tocsc(), r)
        got = tl.coarse.lu[i].solve(r)
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


def test_coarse_outgoing_fold_beats_the_wrong_sign():
    # on the coarse grid too, the fold (1 + i k h_c) for e^{-i omega t} is the
    # outgoing condition: the opposite sign makes the coarse one-level ORAS a
    # far worse preconditioner of E
    from oracle.coarse import coarse_k
    prob = _prob(shape=(24, 22, 20), pml=(4, 4, 4, 0))
    A = assemble(prob)
    k = prob.k().ravel()
    boxes = decompose(prob.shape, (2, 2, 2), 2)
    Z = prolongation(prob.shape)
    E = (Z.T @ A @ Z).tocsr()
    cs, cb = coarse_shape(prob.shape), coarse_boxes(boxes, prob.shape, 2)
    kc = coarse_k(k, prob.shape)
    b = np.zeros(prob.n, complex)
    b[12 + 24 * (11 + 22 * 4)] = 1.0
    c = Z.T @ b
    its = {}
    for name, kk in (("outgoing", kc), ("wrong", -kc)):
        M = Oras(E, cs, cb, kk, 2 * prob.h)
        its[name] = fgmres(lambda v: E @ v, M.apply, c, 1e-8, 30, 400)[1]
    assert 2 * its["outgoing"] < its["wrong"]
