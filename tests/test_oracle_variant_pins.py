"""Pins of the oracle's paper-faithful cycle variants: successive over-relaxation
in the red-black smoother (feature 5 names SOR), the 64-point restriction (the
transpose of trilinear interpolation, a common alternative to feature 3's
8-child mean) and restarted GMRES on the coarsest grid (feature 6).
"""
import numpy as np
import pytest

import pins
from paper_1410_8568_amd import inputs


def colour_mask(shape, colour):
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + j + k) & 1) == colour


def test_sor_with_omega_one_is_gauss_seidel(oracle_lib):
    rng = np.random.default_rng(21)
    n = (7, 6, 5)
    bx, by, bz = pins.random_faces(n, rng)
    p = rng.standard_normal((5, 6, 7)); b = rng.standard_normal((5, 6, 7))
    for colour in (0, 1):
        assert np.array_equal(oracle_lib.rb_half_sor(bx, by, bz, p, b, colour, 1.0),
                              oracle_lib.rb_half(bx, by, bz, p, b, colour))


@pytest.mark.parametrize("omega", [0.7, 1.3, 1.8])
@pytest.mark.parametrize("colour", [0, 1])
def test_sor_scales_the_swept_colours_residual_by_one_minus_omega(oracle_lib, omega, colour):
    """Cells of one colour couple only to the other colour, so an SOR update of a
    colour multiplies that colour's residual by exactly (1 - omega)."""
    rng = np.random.default_rng(22)
    n = (8, 7, 6)
    bx, by, bz = pins.random_faces(n, rng, contrast=100.0)
    p = rng.standard_normal((6, 7, 8)); b = rng.standard_normal((6, 7, 8))
    before = oracle_lib.residual(bx, by, bz, p, b)
    after = oracle_lib.residual(bx, by, bz, oracle_lib.rb_half_sor(bx, by, bz, p, b, colour, omega), b)
    m = colour_mask(p.shape, colour)
    assert np.max(np.abs(after[m] - (1 - omega) * before[m])) <= 1e-12 * np.abs(before[m]).max()


def test_restrict64_is_half_the_transpose_of_trilinear_interpolation(oracle_lib):
    rng = np.random.default_rng(23)
    cz, cy, cx = 3, 2, 4
    # the textbook trilinear matrix, column by column
    P = np.stack([pins.trilinear_prolong(np.eye(cz * cy * cx)[q].reshape(cz, cy, cx)).ravel()
                  for q in range(cz * cy * cx)], axis=1)
    r = rng.standard_normal((2 * cz, 2 * cy, 2 * cx))
    rc = oracle_lib.restrict64(r)
    assert np.max(np.abs(rc.ravel() - 0.5 * P.T @ r.ravel())) <= 1e-13 * np.abs(rc).max()
    # constants: R c = 4 c; totals: sum(R r) = sum(r) / 2 (as for the 8-child mean)
    assert np.allclose(oracle_lib.restrict64(np.full((6, 4, 8), 2.5)), 10.0, rtol=0, atol=1e-14)
    assert abs(rc.sum() - 0.5 * r.sum()) <= 1e-13 * np.abs(r).sum()


def test_gmres_finite_termination_and_exact_limit(oracle_lib):
    rng = np.random.default_rng(24)
    bx, by, bz = pins.random_faces((3, 3, 3), rng, contrast=1000.0)
    rhs = rng.standard_normal((3, 3, 3))
    e, it, rr = oracle_lib.gmres(bx, by, bz, rhs, m=30, tol=1e-12, maxit=100)
    assert it <= 26 and rr <= 1e-12
    ref = oracle_lib.dense_solve(bx, by, bz, rhs)
    assert np.linalg.norm(e - ref) <= 1e-9 * np.linalg.norm(ref)
    assert abs(e.mean()) <= 1e-14


@pytest.mark.parametrize("m", [4, 16])
def test_restarted_gmres_converges_to_the_dense_solve(oracle_lib, m):
    rng = np.random.default_rng(25)
    bx, by, bz = pins.random_faces((8, 8, 8), rng, contrast=1000.0)
    rhs = rng.standard_normal((8, 8, 8))
    ref = oracle_lib.dense_solve(bx, by, bz, rhs)
    its = []
    for tol in (1e-3, 1e-6, 1e-11):
        e, it, rr = oracle_lib.gmres(bx, by, bz, rhs, m=m, tol=tol, maxit=20000)
        assert rr <= tol
        its.append(it)
    assert its == sorted(its)
    assert np.linalg.norm(e - ref) <= 1e-7 * np.linalg.norm(ref)


@pytest.mark.parametrize("kw", [dict(omega=1.3), dict(omega=0.8), dict(restrict64=True),
                                dict(gmres_m=8, gmres_tol=1e-2), dict(omega=1.2, restrict64=True, gmres_m=16,
                                                                     gmres_tol=1e-4)])
def test_variant_cycles_reach_the_direct_solve(oracle_lib, kw):
    rng = np.random.default_rng(26)
    n = (8, 8, 8)
    bx, by, bz = pins.random_faces(n, rng, contrast=1000.0)
    b = rng.standard_normal((8, 8, 8))
    ref = pins.bordered_direct_solve(bx, by, bz, b)
    for precision in ("fp64", "fp32_refined"):
        r = oracle_lib.solve(bx, by, bz, b, tol=1e-11, n_coarsest=2, precision=precision, max_cycles=200, **kw)
        assert r["status"] == "converged"
        assert np.linalg.norm(r["p"] - ref) <= 1e-9 * np.linalg.norm(ref)


def test_variants_on_the_drop_splash_field(oracle_lib):
    """32^3 drop splash, ratio 1000: every variant converges within the paper's
    gamma <= 0.5 and reaches the default cycle's p."""
    P = inputs.drop_splash_problem(32, 0.1, (0.5, 0.5, 0.2, 0.08), 1000.0, 1.0, seed=2, perturb=True)
    base = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-11)
    for kw in (dict(omega=1.2), dict(restrict64=True), dict(gmres_m=16, gmres_tol=1e-3)):
        r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-11, **kw)
        assert r["status"] == "converged" and r["gamma"] <= 0.5, kw
        assert np.linalg.norm(r["p"] - base["p"]) <= 1e-8 * np.linalg.norm(base["p"]), kw


def test_invalid_variant_options(oracle_lib):
    P = inputs.config0()
    for kw in (dict(omega=0.0), dict(omega=2.0), dict(gmres_m=-1), dict(gmres_m=4, gmres_tol=0.0)):
        assert oracle_lib.solve(P.bx, P.by, P.bz, P.b, **kw)["status"] == "invalid"


def test_variant_cycle_is_the_composition_of_its_pinned_steps(oracle_lib):
    """One two-level cycle with SOR and the 64-point restriction, built by hand
    from the pinned primitives, equals the oracle solve's first cycle."""
    rng = np.random.default_rng(27)
    n = (8, 6, 4)
    bx, by, bz = pins.random_faces(n, rng, contrast=100.0)
    b = rng.standard_normal((4, 6, 8))
    b -= b.mean()
    omega = 1.25
    p = np.zeros_like(b)
    for _ in range(2):
        p = oracle_lib.rb_half_sor(bx, by, bz, p, b, 0, omega)
        p = oracle_lib.rb_half_sor(bx, by, bz, p, b, 1, omega)
    rc = oracle_lib.restrict64(oracle_lib.residual(bx, by, bz, p, b))
    cbx, cby, cbz = oracle_lib.coarsen_faces(bx, by, bz)
    ec = oracle_lib.dense_solve(cbx, cby, cbz, rc)
    p = oracle_lib.prolong_add(oracle_lib.cell_weights(cbx, cby, cbz), ec, p)
    for _ in range(2):
        p = oracle_lib.rb_half_sor(bx, by, bz, p, b, 1, omega)
        p = oracle_lib.rb_half_sor(bx, by, bz, p, b, 0, omega)
    r = oracle_lib.solve(bx, by, bz, b, tol=1e-14, n_coarsest=4, max_cycles=1, omega=omega, restrict64=True)
    assert len(oracle_lib.plan(n, 4)) == 2
    assert np.max(np.abs(r["p"] - (p - p.mean()))) <= 1e-13 * np.abs(p).max()


def test_one_level_cycle_is_the_coarse_gmres(oracle_lib):
    """On a grid that is its own coarsest level the cycle is the coarse solve: with
    the GMRES variant the first cycle leaves exactly GMRES's residual.  (Without
    restarts: restarted GMRES on this contrast amplifies the rounding difference
    between the solve's projected right-hand side and the standalone call's.)"""
    rng = np.random.default_rng(28)
    bx, by, bz = pins.random_faces((5, 7, 3), rng, contrast=1000.0)
    b = rng.standard_normal((3, 7, 5))
    e, it, rr = oracle_lib.gmres(bx, by, bz, b, m=64, tol=1e-2, maxit=1000)
    r = oracle_lib.solve(bx, by, bz, b, tol=1e-14, max_cycles=1, gmres_m=64, gmres_tol=1e-2, gmres_maxit=1000)
    assert 1e-4 < rr <= 1e-2 and it <= 64
    assert abs(r["history"][1] - rr) <= 1e-12
    assert np.max(np.abs(r["p"] - e)) <= 1e-13 * np.abs(e).max()
