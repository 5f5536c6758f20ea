"""Pins of the CPU oracle against closed forms, textbook solvers and invariants.

Every oracle function is checked here against something other than itself
(see ``pins.py``).  Chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one test.
"""
import functools
import json
import os

import numpy as np
import pytest

import pins
from paper_1410_8568_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --------------------------------------------------------------------------- operator

@pytest.mark.parametrize("n", [(5, 6, 7), (8, 8, 8), (3, 4, 2)])
def test_operator_matches_assembled_matrix_and_is_symmetric(oracle_lib, n):
    rng = np.random.default_rng(1)
    bx, by, bz = pins.random_faces(n, rng)
    nx, ny, nz = n
    u = rng.standard_normal((nz, ny, nx))
    v = rng.standard_normal((nz, ny, nx))
    Lu = oracle_lib.apply(bx, by, bz, u)
    Lv = oracle_lib.apply(bx, by, bz, v)
    A = pins.assemble(bx, by, bz)
    assert rel(Lu.ravel(), A @ u.ravel()) < 1e-14
    # symmetry (u, Lv) = (Lu, v)
    assert abs(np.vdot(u, Lv) - np.vdot(Lu, v)) <= 1e-13 * np.linalg.norm(Lu) * np.linalg.norm(v)
    # L 1 = 0 and sum(L u) = 0 (Neumann walls, conservative form)
    assert np.max(np.abs(oracle_lib.apply(bx, by, bz, np.ones_like(u)))) < 1e-14
    assert abs(Lu.sum()) < 1e-12 * np.abs(Lu).sum()


def test_operator_ignores_wall_entries(oracle_lib):
    rng = np.random.default_rng(2)
    n = (6, 5, 4)
    bx, by, bz = pins.random_faces(n, rng)
    u = rng.standard_normal((4, 5, 6))
    ref = oracle_lib.apply(bx, by, bz, u)
    bx2, by2, bz2 = bx.copy(), by.copy(), bz.copy()
    bx2[:, :, 0] = 7.0; bx2[:, :, -1] = 3.0; by2[:, 0, :] = 5.0; bz2[-1] = 11.0
    # apply never reads wall faces as links
    assert np.array_equal(oracle_lib.apply(bx2, by2, bz2, u), ref)


def test_residual_is_b_minus_Lp(oracle_lib):
    rng = np.random.default_rng(3)
    n = (7, 5, 6)
    bx, by, bz = pins.random_faces(n, rng)
    p = rng.standard_normal((6, 5, 7)); b = rng.standard_normal((6, 5, 7))
    r = oracle_lib.residual(bx, by, bz, p, b)
    A = pins.assemble(bx, by, bz)
    assert rel(r.ravel(), b.ravel() - A @ p.ravel()) < 1e-14


@pytest.mark.parametrize("n", [8, 16, 32])
def test_manufactured_solution_second_order(oracle_lib, n):
    """The discrete operator is a second-order approximation of div(alpha grad p)."""
    errs = []
    for m in (n, 2 * n):
        bx, by, bz, b, P = pins.manufactured(m)
        r = oracle_lib.solve(bx, by, bz, b, tol=1e-12, n_coarsest=4)
        assert r["status"] == "converged"
        errs.append(np.sqrt(np.mean((r["p"] - (P - P.mean())) ** 2)))
    assert errs[0] / errs[1] > 3.8, errs


# --------------------------------------------------------------------------- smoother

@pytest.mark.parametrize("colour", [0, 1])
def test_half_sweep_zeroes_residual_on_its_colour(oracle_lib, colour):
    rng = np.random.default_rng(4)
    n = (9, 6, 7)
    bx, by, bz = pins.random_faces(n, rng, contrast=1000.0)
    p = rng.standard_normal((7, 6, 9)); b = rng.standard_normal((7, 6, 9))
    q = oracle_lib.rb_half(bx, by, bz, p, b, colour)
    k, j, i = np.meshgrid(range(7), range(6), range(9), indexing="ij")
    mine = ((i + j + k) & 1) == colour
    A = pins.assemble(bx, by, bz)
    r = b.ravel() - A @ q.ravel()
    assert np.max(np.abs(r[mine.ravel()])) < 1e-12 * np.max(np.abs(b))
    # the other colour is untouched
    assert np.array_equal(q[~mine], p[~mine])


# --------------------------------------------------------------------------- transfers

def test_restriction_of_constant_is_four_c(oracle_lib):
    r = np.full((8, 6, 4), 2.5)
    assert np.allclose(oracle_lib.restrict(r), 10.0, rtol=0, atol=1e-15)


def test_restriction_is_half_block_sum(oracle_lib):
    rng = np.random.default_rng(5)
    r = rng.standard_normal((6, 4, 8))
    blocks = r.reshape(3, 2, 2, 2, 4, 2).sum(axis=(1, 3, 5))
    assert np.allclose(oracle_lib.restrict(r), 0.5 * blocks, rtol=1e-15, atol=1e-15)


def test_prolongation_uniform_weights_is_trilinear(oracle_lib):
    rng = np.random.default_rng(6)
    ec = rng.standard_normal((3, 4, 5))
    a = np.full_like(ec, 0.37)
    base = rng.standard_normal((6, 8, 10))
    out = oracle_lib.prolong_add(a, ec, base)
    assert np.allclose(out - base, pins.trilinear_prolong(ec), rtol=0, atol=1e-14)


def test_prolongation_preserves_constants(oracle_lib):
    rng = np.random.default_rng(7)
    a = rng.uniform(1e-3, 1.0, (4, 4, 4))
    out = oracle_lib.prolong_add(a, np.full((4, 4, 4), -1.75), np.zeros((8, 8, 8)))
    assert np.allclose(out, -1.75, rtol=0, atol=1e-14)


def test_prolongation_flux_continuity_1d(oracle_lib):
    """Coarse error and weights varying along x only: every fine value is the
    midpoint of the coarse centre value and the face value that makes the flux
    continuous, a_C (e_f - e_C) = a_N (e_N - e_f) (eqs. 13-14)."""
    rng = np.random.default_rng(8)
    cx = 6
    e1 = rng.standard_normal(cx)
    a1 = rng.uniform(1e-3, 1.0, cx)
    ec = np.broadcast_to(e1, (2, 3, cx)).copy()
    a = np.broadcast_to(a1, (2, 3, cx)).copy()
    out = oracle_lib.prolong_add(a, ec, np.zeros((4, 6, 2 * cx)))
    expect = np.empty(2 * cx)
    for I in range(cx):
        for child, nb in ((2 * I, max(I - 1, 0)), (2 * I + 1, min(I + 1, cx - 1))):
            ef = (a1[I] * e1[I] + a1[nb] * e1[nb]) / (a1[I] + a1[nb])
            # flux continuity holds for the face value
            assert abs(a1[I] * (ef - e1[I]) - a1[nb] * (e1[nb] - ef)) < 1e-14
            expect[child] = 0.5 * (e1[I] + ef)
    assert np.allclose(out, np.broadcast_to(expect, out.shape), rtol=0, atol=1e-14)


def _flux_face_values_1d(e1, a1):
    """Per fine child along one axis: the coarse centre value and the face value of
    eqs. 13-14 read as flux continuity, a_C (e_f - e_C) = a_N (e_N - e_f), with the
    neighbour beyond a wall replaced by the cell itself (zero normal derivative)."""
    cn = len(e1)
    centre = np.empty(2 * cn)
    face = np.empty(2 * cn)
    for I in range(cn):
        for child, nb in ((2 * I, max(I - 1, 0)), (2 * I + 1, min(I + 1, cn - 1))):
            centre[child] = e1[I]
            face[child] = (a1[I] * e1[I] + a1[nb] * e1[nb]) / (a1[I] + a1[nb])
    return centre, face


@pytest.mark.parametrize("axis", [0, 1])
def test_prolongation_flux_continuity_1d_along_y_and_z(oracle_lib, axis):
    """The same closed form with coarse error and weights varying along y (axis 1
    of the [k][j][i] arrays) or along z (axis 0) only, so that the y- and z-corner
    weights of the prolongation are pinned as well as the x ones."""
    rng = np.random.default_rng(18 + axis)
    cn = 5
    e1 = rng.standard_normal(cn)
    a1 = rng.uniform(1e-3, 1.0, cn)
    cshape = [3, 4, 2]
    cshape[axis] = cn
    view = [1, 1, 1]
    view[axis] = cn
    ec = np.broadcast_to(e1.reshape(view), cshape).copy()
    a = np.broadcast_to(a1.reshape(view), cshape).copy()
    out = oracle_lib.prolong_add(a, ec, np.zeros(tuple(2 * s for s in cshape)))
    centre, face = _flux_face_values_1d(e1, a1)
    expect = 0.5 * (centre + face)
    fview = [1, 1, 1]
    fview[axis] = 2 * cn
    assert np.allclose(out, np.broadcast_to(expect.reshape(fview), out.shape), rtol=0, atol=1e-14)


@pytest.mark.parametrize("plane", [(1, 2), (0, 2), (0, 1)])
def test_prolongation_edge_corner_is_weighted_mean_of_four(oracle_lib, plane):
    """Data varying in two directions only (the third is constant): a fine value is
    the mean of four octant corners, the coarse cell, its two face values (the 1-D
    flux-continuity closed forms along each direction, pinned above) and the edge
    value, which the 3-D extension of eqs. 13-14 defines as the coefficient-weighted
    mean of the four coarse cells sharing the edge.  Checked cell by cell with
    non-uniform weights, in each of the three coordinate planes (axes of the
    [k][j][i] arrays)."""
    rng = np.random.default_rng(30 + plane[0] + 2 * plane[1])
    pa, pb = plane                      # the two varying axes
    flat = 3 - pa - pb                  # the constant axis
    na, nb = 4, 3
    e2 = rng.standard_normal((na, nb))
    a2 = rng.uniform(1e-3, 1.0, (na, nb))
    cshape = [0, 0, 0]
    cshape[pa], cshape[pb], cshape[flat] = na, nb, 2
    ec = np.moveaxis(np.broadcast_to(e2[:, :, None], (na, nb, 2)), (0, 1, 2), (pa, pb, flat)).copy()
    a = np.moveaxis(np.broadcast_to(a2[:, :, None], (na, nb, 2)), (0, 1, 2), (pa, pb, flat)).copy()
    assert ec.shape == tuple(cshape)
    out = oracle_lib.prolong_add(a, ec, np.zeros(tuple(2 * s for s in cshape)))
    out2 = np.moveaxis(out, (pa, pb, flat), (0, 1, 2))   # [fine a][fine b][flat]
    # the constant direction leaves every fine value unchanged along it
    assert np.array_equal(out2[:, :, 0], out2[:, :, 1])
    for fa in range(2 * na):
        for fb in range(2 * nb):
            I, J = fa // 2, fb // 2
            sa, sb = (1 if fa & 1 else -1), (1 if fb & 1 else -1)
            In, Jn = min(max(I + sa, 0), na - 1), min(max(J + sb, 0), nb - 1)
            # face values from the 1-D closed form along each direction
            va = (a2[I, J] * e2[I, J] + a2[In, J] * e2[In, J]) / (a2[I, J] + a2[In, J])
            vb = (a2[I, J] * e2[I, J] + a2[I, Jn] * e2[I, Jn]) / (a2[I, J] + a2[I, Jn])
            cells = [(I, J), (In, J), (I, Jn), (In, Jn)]
            edge = sum(a2[c] * e2[c] for c in cells) / sum(a2[c] for c in cells)
            want = 0.25 * (e2[I, J] + va + vb + edge)
            assert abs(out2[fa, fb, 0] - want) < 1e-14, (fa, fb, out2[fa, fb, 0], want)
            # and the edge value read back from the output is that weighted mean
            assert abs(4.0 * out2[fa, fb, 0] - e2[I, J] - va - vb - edge) < 1e-13


@pytest.mark.parametrize("perm", [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)])
def test_prolongation_commutes_with_axis_permutations(oracle_lib, perm):
    """The prolongation treats the three directions alike: permuting the axes of
    random 3-D coarse data and weights (non-cubic grid) permutes the result.  An
    index that reads one direction's offset in another breaks this."""
    rng = np.random.default_rng(40)
    ec = rng.standard_normal((3, 4, 5))
    a = rng.uniform(1e-3, 1.0, ec.shape)
    base = np.zeros(tuple(2 * s for s in ec.shape))
    out = oracle_lib.prolong_add(a, ec, base)
    outp = oracle_lib.prolong_add(np.transpose(a, perm), np.transpose(ec, perm), np.transpose(base, perm))
    assert np.allclose(outp, np.transpose(out, perm), rtol=0, atol=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_prolongation_commutes_with_reflections(oracle_lib, axis):
    """Mirroring the grid along one axis mirrors the result: the octant on the low
    side of a coarse cell takes its corners below it, the high octant above, and
    walls clamp alike at both ends."""
    rng = np.random.default_rng(41 + axis)
    ec = rng.standard_normal((4, 3, 5))
    a = rng.uniform(1e-3, 1.0, ec.shape)
    base = np.zeros(tuple(2 * s for s in ec.shape))
    out = oracle_lib.prolong_add(a, ec, base)
    outf = oracle_lib.prolong_add(np.flip(a, axis), np.flip(ec, axis), base)
    assert np.allclose(outf, np.flip(out, axis), rtol=0, atol=1e-14)


def test_prolongation_node_corner_by_linearity(oracle_lib):
    """Full 3-D data: with the weights fixed the prolongation is linear in the
    coarse error, and the coarse unit vector of one interior cell C spreads to the
    fine cells with exactly the weight shares of the corners that contain C.  Its
    fine child in octant s gets (1/8)(1 + sum over the 7 non-empty T of
    a_C / sum_{m in T-set} a_m), the 2^|T| cells of each T-set being C and its
    neighbours towards s; checked for all 8 children of an interior cell, which
    involves the node (|T| = 3) corner and all edges."""
    rng = np.random.default_rng(43)
    shape = (4, 5, 6)
    a = rng.uniform(1e-3, 1.0, shape)
    K, J, I = 2, 2, 3
    ec = np.zeros(shape)
    ec[K, J, I] = 1.0
    out = oracle_lib.prolong_add(a, ec, np.zeros(tuple(2 * s for s in shape)))
    for ck in (0, 1):
        for cj in (0, 1):
            for ci in (0, 1):
                sz, sy, sx = (1 if ck else -1), (1 if cj else -1), (1 if ci else -1)
                total = 1.0
                for T in range(1, 8):
                    den = 0.0
                    for d in range(8):
                        if d & ~T:
                            continue
                        den += a[K + (sz if d & 4 else 0), J + (sy if d & 2 else 0), I + (sx if d & 1 else 0)]
                    total += a[K, J, I] / den
                got = out[2 * K + ck, 2 * J + cj, 2 * I + ci]
                assert abs(got - total / 8.0) < 1e-14, (ck, cj, ci, got, total / 8.0)


# --------------------------------------------------------------------------- hierarchy

def test_plan_levels(oracle_lib):
    assert oracle_lib.plan((32, 32, 32), 4) == [(32,) * 3, (16,) * 3, (8,) * 3, (4,) * 3]
    assert oracle_lib.plan((96, 96, 96), 8)[-1] == (6, 6, 6)
    assert oracle_lib.plan((96, 96, 96), 4)[-1] == (3, 3, 3)
    assert oracle_lib.plan((5, 5, 5), 4) == [(5, 5, 5)]
    assert oracle_lib.plan((64, 64, 16), 8)[-1] == (8, 8, 2)


def test_coarsening_preserves_uniform_and_layered(oracle_lib):
    n = (8, 6, 4)
    bx = np.full((4, 6, 9), 0.3); by = np.full((4, 7, 8), 0.3); bz = np.full((5, 6, 8), 0.3)
    cbx, cby, cbz = oracle_lib.coarsen_faces(bx, by, bz)
    assert np.allclose(cbx[:, :, 1:-1], 0.3) and np.allclose(cby[:, 1:-1, :], 0.3)
    assert np.allclose(cbz[1:-1], 0.3)
    assert np.all(cbx[:, :, [0, -1]] == 0) and np.all(cby[:, [0, -1], :] == 0)
    assert np.all(cbz[[0, -1]] == 0)
    # z-layered coefficients: coarse z-face K equals fine z-face 2K, coarse x-face is the
    # mean of the two fine layers it spans
    rng = np.random.default_rng(9)
    lay = rng.uniform(0.1, 1.0, 5)
    cell = rng.uniform(0.1, 1.0, 4)
    bz = np.broadcast_to(lay[:, None, None], (5, 6, 8)).copy()
    bx = np.broadcast_to(cell[:, None, None], (4, 6, 9)).copy()
    cbx, cby, cbz = oracle_lib.coarsen_faces(bx, by, bz)
    assert np.allclose(cbz[1, :, :], lay[2])
    assert np.allclose(cbx[1, :, 1], 0.5 * (cell[2] + cell[3]))


@pytest.mark.parametrize("n", [(8, 6, 4), (4, 10, 6)])
def test_coarsening_conserves_plane_conductance(oracle_lib, n):
    """On random faces, the coarse faces of each coarse plane carry one quarter of
    the total conductance of the fine plane they sit on (2x2 fine faces per coarse
    face, parallel), and the coarse wall planes carry none."""
    rng = np.random.default_rng(13)
    bx, by, bz = pins.random_faces(n, rng, lo=0.01, hi=1.0)
    cbx, cby, cbz = oracle_lib.coarsen_faces(bx, by, bz)
    nx, ny, nz = n
    for m in range(1, nx // 2):
        assert np.isclose(cbx[:, :, m].sum(), 0.25 * bx[:, :, 2 * m].sum(), rtol=1e-14)
    for m in range(1, ny // 2):
        assert np.isclose(cby[:, m, :].sum(), 0.25 * by[:, 2 * m, :].sum(), rtol=1e-14)
    for m in range(1, nz // 2):
        assert np.isclose(cbz[m].sum(), 0.25 * bz[2 * m].sum(), rtol=1e-14)
    # each coarse face depends on its own 2x2 bundle only: perturbing one fine
    # face changes exactly one coarse face, by a quarter of the perturbation
    bz2 = bz.copy()
    bz2[2, 1, 3] += 1.0
    d = oracle_lib.coarsen_faces(bx, by, bz2)[2] - cbz
    assert np.count_nonzero(d) == 1 and np.isclose(d[1, 0, 1], 0.25)


def test_cell_weights_uniform_and_corner(oracle_lib):
    n = (4, 4, 4)
    rng = np.random.default_rng(10)
    bx, by, bz = pins.random_faces(n, rng)
    a = oracle_lib.cell_weights(bx, by, bz)
    # corner cell (0,0,0): interior faces x+ (bx[0,0,1]), y+ (by[0,1,0]), z+ (bz[1,0,0])
    assert np.isclose(a[0, 0, 0], (bx[0, 0, 1] + by[0, 1, 0] + bz[1, 0, 0]) / 3)
    u = np.full((5, 4, 4), 0.8)
    assert np.allclose(oracle_lib.cell_weights(np.full((4, 4, 5), 0.8), np.full((4, 5, 4), 0.8), u), 0.8)


# --------------------------------------------------------------------------- exact solves

def test_dense_coarse_solve_matches_bordered_lu(oracle_lib):
    rng = np.random.default_rng(11)
    n = (3, 4, 5)
    bx, by, bz = pins.random_faces(n, rng, contrast=1000.0)
    rhs = rng.standard_normal((5, 4, 3))
    e = oracle_lib.dense_solve(bx, by, bz, rhs)
    ref = pins.bordered_direct_solve(bx, by, bz, rhs)
    assert rel(e, ref) < 1e-12
    assert abs(e.mean()) < 1e-14 * np.abs(e).max()


@pytest.mark.parametrize("contrast", [None, 1000.0])
def test_multigrid_equals_direct_solve_8cubed(oracle_lib, contrast):
    rng = np.random.default_rng(12)
    bx, by, bz = pins.random_faces((8, 8, 8), rng, contrast=contrast)
    b = rng.standard_normal((8, 8, 8))
    r = oracle_lib.solve(bx, by, bz, b, tol=1e-13, n_coarsest=2)
    assert r["status"] == "converged"
    assert rel(r["p"], pins.bordered_direct_solve(bx, by, bz, b)) < 1e-11


@functools.lru_cache(maxsize=None)
def config0_direct():
    P = inputs.config0()
    return P, pins.bordered_direct_solve(P.bx, P.by, P.bz, P.b)


def test_config0_equals_direct_solve(oracle_lib):
    """The 32^3 sphere workload: oracle multigrid vs sparse direct LU."""
    P, ref = config0_direct()
    r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, n_coarsest=4)
    assert r["status"] == "converged" and r["history"][-1] <= 1e-10
    assert rel(r["p"], ref) < 1e-8
    r2 = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-13, n_coarsest=4)
    assert rel(r2["p"], ref) < 1e-10


def test_fp32_refined_reaches_fp64_solution(oracle_lib):
    P, ref = config0_direct()
    for m in (1, 2, 3):
        r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, precision="fp32_refined", inner_m=m)
        assert r["status"] == "converged"
        assert rel(r["p"], ref) < 1e-8


@pytest.mark.parametrize("n", [16, 48])
def test_layered_closed_form(oracle_lib, n):
    P = inputs.layered_problem(n)
    r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-11, n_coarsest=4, max_cycles=200)
    assert r["status"] == "converged"
    p1 = pins.layered_solve(P.bz[:, 0, 0], P.b[:, 0, 0])
    assert rel(r["p"], np.broadcast_to(p1[:, None, None], r["p"].shape)) < 1e-9


@pytest.mark.parametrize("n", [16, 24])
def test_constant_coefficient_dct(oracle_lib, n):
    P = inputs.constant_problem(n, beta=0.7)
    r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-13, n_coarsest=4)
    assert r["status"] == "converged"
    assert rel(r["p"], pins.dct_solve(P.b, beta=0.7)) < 1e-11
    # V(2,2) with constant coefficients converges at a textbook rate
    assert r["gamma"] < 0.2


def test_warm_start_and_zero_rhs(oracle_lib):
    P = inputs.config0()
    r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-10)
    r2 = oracle_lib.solve(P.bx, P.by, P.bz, P.b, p0=r["p"], tol=1e-10)
    assert r2["cycles"] == 0 and r2["status"] == "converged"
    z = oracle_lib.solve(P.bx, P.by, P.bz, np.full_like(P.b, 3.0), tol=1e-10)
    assert z["status"] == "converged" and np.all(z["p"] == 0)


def test_gamma_is_eq15_and_within_paper_bound(oracle_lib):
    figs = json.load(open(GOLDEN))
    P = inputs.config1(64)
    r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-10)
    h = r["history"]
    nc = r["cycles"]
    assert np.isclose(r["gamma"], (h[nc] / h[0]) ** (1.0 / nc), rtol=1e-14)
    lo, hi = figs["gamma_interval"]["value"]
    assert lo <= r["gamma"] <= figs["gamma_worst_observed"]["value"] <= hi
    assert h[-1] <= figs["mg_residual_tolerance"]["value"]


def test_generator_divergence_rhs_is_compatible():
    P = inputs.config1(32)
    assert abs(P.b.sum()) < 1e-10
    assert np.all(P.bx[:, :, 1:-1] > 0) and np.all(P.bx[:, :, [0, -1]] == 0)
    ratio = P.bx[:, :, 1:-1].max() / P.bx[:, :, 1:-1].min()
    assert 900 < ratio < 1001


@pytest.mark.parametrize("n", [16, 48])
def test_layered_profile_reproduces_layered_problem(n):
    """The 1-D profiles used to build the 1024^3 layered case on the device are
    the layered problem's own values, so its closed form applies there too."""
    P = inputs.layered_problem(n)
    a, bz, b = inputs.layered_profile(n)
    assert np.array_equal(P.bz, np.broadcast_to(bz[:, None, None], P.bz.shape))
    assert np.array_equal(P.bx[:, :, 1:-1], np.broadcast_to(a[:, None, None], (n, n, n - 1)))
    assert np.array_equal(P.by[:, 1:-1, :], np.broadcast_to(a[:, None, None], (n, n - 1, n)))
    assert np.array_equal(P.b, np.broadcast_to(b[:, None, None], P.b.shape))
