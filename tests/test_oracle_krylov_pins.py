"""Pins of the oracle's Krylov-accelerated solve (flexible CG preconditioned by one
V-cycle per iteration) and of its unpreconditioned form.

With the identity preconditioner the flexible recurrences reduce to textbook
conjugate gradients, so they are pinned against scipy's CG on the assembled
matrix (iteration by iteration) and against finite termination in exact
dimension; the preconditioned solve is pinned against the bordered direct solve
at density ratios up to 1e5, the paper's robustness range.
"""
import numpy as np
import pytest

import pins
from paper_1410_8568_amd import inputs


def scipy_cg_history(bx, by, bz, b, maxiter):
    import scipy.sparse.linalg as sla
    A = pins.assemble(bx, by, bz)
    nb = np.linalg.norm(b)
    hist = []
    sla.cg(-A, -b.ravel(), x0=np.zeros(b.size), rtol=1e-12, maxiter=maxiter,
           callback=lambda xk: hist.append(np.linalg.norm(b.ravel() - A @ xk) / nb))
    return np.array(hist)


@pytest.mark.parametrize("n,seed", [((5, 4, 3), 3), ((6, 6, 2), 5)])
def test_unpreconditioned_cg_matches_scipy(oracle_lib, n, seed):
    rng = np.random.default_rng(seed)
    bx, by, bz = pins.random_faces(n, rng)
    nx, ny, nz = n
    b = rng.standard_normal((nz, ny, nx))
    b -= b.mean()
    r = oracle_lib.solve(bx, by, bz, b, tol=1e-12, krylov="cg", max_cycles=100)
    ref = scipy_cg_history(bx, by, bz, b, 100)
    assert r["status"] == "converged" and r["cycles"] == len(ref)
    h = r["history"][1:16]
    assert np.max(np.abs(h - ref[:15]) / ref[:15]) <= 1e-9
    assert np.linalg.norm(r["p"] - pins.bordered_direct_solve(bx, by, bz, b)) <= 1e-10 * np.linalg.norm(r["p"])


def test_cg_terminates_within_the_mean_free_dimension(oracle_lib):
    """27 cells: the mean-free subspace has dimension 26, so CG needs at most 26
    iterations (exactly, up to rounding)."""
    rng = np.random.default_rng(4)
    bx, by, bz = pins.random_faces((3, 3, 3), rng)
    b = rng.standard_normal((3, 3, 3))
    r = oracle_lib.solve(bx, by, bz, b, tol=1e-12, krylov="cg", max_cycles=60)
    assert r["status"] == "converged" and r["cycles"] <= 26


@pytest.mark.parametrize("contrast", [1000.0, 1e5])
def test_fcg_equals_direct_solve(oracle_lib, contrast):
    rng = np.random.default_rng(6)
    n = (8, 8, 8)
    bx, by, bz = pins.random_faces(n, rng, contrast=contrast)
    b = rng.standard_normal((8, 8, 8))
    ref = pins.bordered_direct_solve(bx, by, bz, b)
    for tol, bar in ((1e-10, 1e-8), (1e-13, 1e-10)):
        r = oracle_lib.solve(bx, by, bz, b, tol=tol, krylov="fcg")
        assert r["status"] == "converged" and r["history"][-1] <= tol
        assert np.linalg.norm(r["p"] - ref) <= bar * np.linalg.norm(ref)
        assert abs(r["p"].mean()) <= 1e-13 * np.abs(r["p"]).max()


@pytest.mark.parametrize("faces,ratio", [("arith", 1e3), ("harmonic", 1e3), ("harmonic", 1e5)])
def test_fcg_beats_the_vcycle_iteration(oracle_lib, faces, ratio):
    """On the drop-splash field the Krylov-accelerated solve needs fewer
    iterations (each one V-cycle) than the plain cycle, reaches the same p, and
    the plain cycle itself stays within the paper's gamma <= 0.5 up to 1e5."""
    P = inputs.drop_splash_problem(32, 0.1, (0.5, 0.5, 0.2, 0.08), ratio, 1.0, seed=2, perturb=True, faces=faces)
    mg = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-10)
    kr = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, krylov="fcg")
    assert mg["status"] == kr["status"] == "converged"
    assert kr["cycles"] < mg["cycles"] and kr["gamma"] < mg["gamma"] <= 0.5
    assert np.linalg.norm(kr["p"] - mg["p"]) <= 1e-8 * np.linalg.norm(mg["p"])


def test_fcg_zero_rhs_and_warm_start(oracle_lib):
    P = inputs.config0()
    z = oracle_lib.solve(P.bx, P.by, P.bz, np.full_like(P.b, 3.0), krylov="fcg")
    assert z["status"] == "converged" and z["cycles"] == 0 and not z["p"].any()
    r = oracle_lib.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, krylov="fcg")
    again = oracle_lib.solve(P.bx, P.by, P.bz, P.b, p0=r["p"], tol=1e-10, krylov="fcg")
    assert again["cycles"] == 0
