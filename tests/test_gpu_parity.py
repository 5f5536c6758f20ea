"""GPU parity: the HIP library (called through its C ABI) against the CPU oracle.

Bars: setup arrays (coarsened faces, cell weights) bit-exact; per-cycle relative
residual histories equal to rounding; the final p within 1e-8 relative L2 of the
oracle's p with a final relative residual <= 1e-10.
"""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import check_history, gpu_solve, rel
from paper_1410_8568_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_8568_amd import mg
    mg.lib()


def ragged_problem(n, seed=21, ratio=1000.0):
    """Non-cubic grid with a sphere and random N(0,1) rhs (cells are cubic in index space)."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid((np.arange(nz) + .5) / nz, (np.arange(ny) + .5) / ny, (np.arange(nx) + .5) / nx,
                          indexing="ij")
    phi = 0.3 - np.sqrt((x - .4) ** 2 + (y - .6) ** 2 + (z - .5) ** 2)
    ind = inputs.smoothed_heaviside(phi, 1.5 / max(n))
    alpha = 1.0 / (1.0 + (ratio - 1.0) * ind)
    bx, by, bz = inputs.faces_from_alpha(alpha)
    return inputs.Problem(n, bx, by, bz, rng.standard_normal((nz, ny, nx)), dict(kind="ragged"))


@pytest.mark.parametrize("n,nc", [((32, 32, 32), 4), ((40, 24, 12), 4), ((96, 96, 96), 8)])
def test_setup_hierarchy_bit_exact(n, nc):
    import torch
    from paper_1410_8568_amd import mg
    P = ragged_problem(n) if n[0] != 96 else inputs.batch_problems(1, sizes=(96,), build=True)[0]
    bx, by, bz, _ = mg.to_device(P)
    S = mg.Solver(bx, by, bz, n_coarsest=nc)
    levels = S.levels()
    assert levels == oracle.plan(n, nc)
    for l in range(len(levels)):
        g = [t.cpu().numpy() for t in S.level_arrays(l)]
        o = oracle.hierarchy_level(P.bx, P.by, P.bz, nc, l)
        for name, a, b in zip("xyza", g, o):
            assert np.array_equal(a, b), (l, name, np.abs(a - b).max())
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_config0_matches_oracle(precision):
    P = inputs.config0()
    ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, n_coarsest=4, precision=precision)
    p, st = gpu_solve(P, precision=precision, tol=1e-10, n_coarsest=4)
    assert st["rc"] == 0, st
    assert st["history"][-1] <= 1e-10
    check_history(st["history"], ref["history"], precision)
    assert rel(p, ref["p"]) <= 1e-8
    assert abs(p.mean()) <= 1e-12 * np.abs(p).max()
    # against the independent direct solve as well
    assert rel(p, pins.bordered_direct_solve(P.bx, P.by, P.bz, P.b)) <= 1e-8
    assert np.isclose(st["gamma"], ref["gamma"], rtol=1e-6)


@pytest.mark.parametrize("n,nc", [((40, 24, 12), 4), ((48, 48, 48), 4), ((96, 96, 96), 8), ((6, 10, 4), 4),
                                  ((2, 2, 2), 4), ((5, 7, 3), 4)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_ragged_and_small_grids(n, nc, precision):
    P = ragged_problem(n)
    ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, n_coarsest=nc, precision=precision)
    p, st = gpu_solve(P, precision=precision, tol=1e-10, n_coarsest=nc)
    assert st["rc"] == 0, st
    check_history(st["history"], ref["history"], precision)
    assert rel(p, ref["p"]) <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_batch_scene_problems(precision):
    for P in inputs.batch_problems(3, sizes=(32, 64)):
        ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, precision=precision)
        p, st = gpu_solve(P, precision=precision, tol=1e-10)
        assert st["rc"] == 0
        check_history(st["history"], ref["history"], precision)
        assert rel(p, ref["p"]) <= 1e-8


def test_layered_closed_form_256():
    """Full-size property check: z-only coefficients and rhs, exact 1-D solution."""
    P = inputs.layered_problem(256)
    p, st = gpu_solve(P, tol=1e-10, max_cycles=100)
    assert st["rc"] == 0, st["history"]
    p1 = pins.layered_solve(P.bz[:, 0, 0], P.b[:, 0, 0])
    assert rel(p, np.broadcast_to(p1[:, None, None], p.shape)) <= 1e-8


def test_constant_coefficient_dct_128():
    P = inputs.constant_problem(128, beta=0.7)
    for precision in ("fp64", "fp32_refined"):
        p, st = gpu_solve(P, precision=precision, tol=1e-12)
        assert st["rc"] == 0, st
        assert rel(p, pins.dct_solve(P.b, beta=0.7)) <= 1e-9


def test_config1_full_size_matches_oracle():
    """256^3 drop splash, the FP64 workload: per-cycle history and final p vs the oracle."""
    P = inputs.config1(256)
    ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10)
    for precision in ("fp64", "fp32_refined"):
        p, st = gpu_solve(P, precision=precision, tol=1e-10)
        assert st["rc"] == 0, st
        assert st["history"][-1] <= 1e-10
        if precision == "fp64":
            check_history(st["history"], ref["history"])
        assert rel(p, ref["p"]) <= 1e-8


def test_zero_rhs_and_warm_start():
    import torch
    from paper_1410_8568_amd import mg
    P = inputs.config0()
    bx, by, bz, b = mg.to_device(P)
    S = mg.Solver(bx, by, bz)
    p = torch.full_like(b, 5.0)
    st = S.solve(torch.full_like(b, 2.0), p)
    assert st["rc"] == 0 and torch.count_nonzero(p).item() == 0
    p.zero_()
    st = S.solve(b, p, tol=1e-10)
    st2 = S.solve(b, p, tol=1e-10)
    assert st2["rc"] == 0 and st2["cycles"] == 0
    S.close()


def test_error_paths():
    import torch
    from paper_1410_8568_amd import mg
    P = inputs.config0()
    bx, by, bz, b = mg.to_device(P)
    bad = bx.clone()
    bad[3, 4, 5] = -1.0
    with pytest.raises(mg.MGError) as ei:
        mg.Solver(bad, by, bz)
    assert ei.value.status == mg.MG_E_INVALID
    bad[3, 4, 5] = float("nan")
    with pytest.raises(mg.MGError):
        mg.Solver(bad, by, bz)
    # coarsest grid too large: odd 9^3 = 729 cells
    P9 = ragged_problem((9, 9, 9))
    with pytest.raises(mg.MGError):
        mg.Solver(*mg.to_device(P9)[:3])
    # not converged within max_cycles: p is the last iterate, status reported
    S = mg.Solver(bx, by, bz, max_cycles=2)
    p = torch.zeros_like(b)
    st = S.solve(b, p, tol=1e-10, check=False)
    assert st["rc"] == mg.MG_E_NOT_CONVERGED and st["cycles"] == 2
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("n", [(64, 48, 40), (144, 80, 48), (16, 16, 36), (16, 16, 52)])
def test_fused_sweep_tiles_bit_identical(precision, n):
    """The fused red-black sweep (halo recomputed per tile, chunked in z) gives
    exactly the same iterates as the one-colour-per-pass reference kernels, for
    every tile shape, including ragged tiles and chunks.  nz = 36 and 52 give
    chunks of 9 planes (and a last one of 7), so a chunk has an odd number of
    plane steps (the FP32 two-sweep pass runs two steps per iteration).  This also covers the
    zero-input first pass of each coarse correction (the reference fills instead)
    and, in FP32 for the tiles that have it, the pre-smoothing pass that forms and
    restricts the residual itself (the reference restricts in a separate pass), the
    pre-smoothing pass that leaves out its red stage from the second inner cycle on,
    and the two-sweep post-smoothing pass that applies the FP64 refinement update
    (the reference updates in a separate pass)."""
    from paper_1410_8568_amd import mg
    P = ragged_problem(n, seed=5)
    ref_p, ref_st = gpu_solve(P, precision=precision, tol=1e-10, tile=-1)
    for tile in range(1, mg.MG_NUM_TILES + 1):
        p, st = gpu_solve(P, precision=precision, tol=1e-10, tile=tile)
        assert st["history"] == ref_st["history"], tile
        assert np.array_equal(p, ref_p), tile


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("n", [(64, 64, 64), (96, 48, 32)])
def test_graph_replay_bit_identical(precision, n):
    """One captured iteration replayed for every iteration (with the host's
    convergence test and copies in between) gives exactly the eager results."""
    P = ragged_problem(n, seed=9)
    ref_p, ref_st = gpu_solve(P, precision=precision, tol=1e-10, graph=False)
    p, st = gpu_solve(P, precision=precision, tol=1e-10, graph=True)
    assert st["cycles"] == ref_st["cycles"] and st["cycles"] > 3
    assert st["history"] == ref_st["history"]
    assert np.array_equal(p, ref_p)


@pytest.fixture(scope="module")
def config2_reference():
    """The 512^3 benchmark input and three oracle solves of it: FP64 to relative
    residual 1e-10 (the benchmark's tolerance), continued to 1e-13 to give p*, so
    that the oracle is not the parity bottleneck, and the oracle's own FP32-refined
    solve to 1e-10."""
    P = inputs.config2(512)
    ref64 = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, n_coarsest=8)
    assert ref64["status"] == "converged"
    star = oracle.solve(P.bx, P.by, P.bz, P.b, p0=ref64["p"], tol=1e-13, n_coarsest=8, max_cycles=40)
    print(f"512^3 oracle: FP64 {ref64['cycles']} cycles to {ref64['history'][-1]:.3e}; p* after "
          f"{star['cycles']} more cycles, relative residual {star['history'][-1]:.3e}", flush=True)
    assert star["history"][-1] <= 1e-12
    ref32 = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, n_coarsest=8, precision="fp32_refined")
    assert ref32["status"] == "converged"
    return P, ref64["p"], star["p"], ref32["p"]


def test_config2_full_size_matches_oracle(config2_reference):
    """512^3 Fourier-perturbed drop splash in the benchmark's configuration
    (coarsest 8^3, default options).  At the benchmark's tolerance 1e-10 each GPU
    solver matches the oracle's solve of the same kind and tolerance to <= 1e-8
    (FP64 against the FP64 oracle, FP32-refined against the oracle's FP32-refined
    solve), and its residual recomputed with the oracle's operator is <= 1e-10.
    Against p* (oracle residual <= 1e-12) a residual of 1e-10 leaves an error of
    about 1e-8 on this 1000:1 field (the error is bounded by the condition number
    times the residual); the solve is continued from its result to 1e-11 and
    1e-12, every error is printed, and the 1e-8 bar on p* must hold by 1e-11."""
    import torch
    from paper_1410_8568_amd import mg
    P, p64, pstar, p32 = config2_reference
    bbar = P.b - P.b.mean()
    nb = np.linalg.norm(bbar)
    bx, by, bz, b = mg.to_device(P)
    for precision, pref in (("fp64", p64), ("fp32_refined", p32)):
        S = mg.Solver(bx, by, bz, precision=precision, n_coarsest=8)
        pt = torch.zeros_like(b)
        st = S.solve(b, pt, tol=1e-10)
        assert st["rc"] == 0, st
        p = pt.cpu().numpy()
        rr = np.linalg.norm(oracle.residual(P.bx, P.by, P.bz, p, bbar)) / nb
        err_same, err_star = rel(p, pref), rel(p, pstar)
        print(f"512^3 {precision}: cycles {st['cycles']} rel residual {st['rel_residual']:.3e} "
              f"(oracle operator {rr:.3e}); vs the oracle's {precision} solve {err_same:.3e} "
              f"(margin {1e-8 / err_same:.1f}x); vs p* {err_star:.3e}", flush=True)
        errs = {}
        for tol in (1e-11, 1e-12):
            st2 = S.solve(b, pt, tol=tol)
            errs[tol] = rel(pt.cpu().numpy(), pstar)
            print(f"  continued to {tol:g}: rel residual {st2['rel_residual']:.3e} vs p* {errs[tol]:.3e}",
                  flush=True)
        S.close()
        assert rr <= 1e-10
        assert abs(p.mean()) <= 1e-12 * np.abs(p).max()
        assert err_same <= 1e-8
        assert errs[1e-11] <= 1e-8
        del p, pt


def _layered_on_device(n, ratio, dev="cuda"):
    """The layered problem of n^3 cells built on the device from its z profiles."""
    import torch
    a, bz1, b1 = inputs.layered_profile(n, ratio=ratio)
    ta = torch.from_numpy(a).to(dev)[:, None, None]
    bx = torch.zeros((n, n, n + 1), dtype=torch.float64, device=dev)
    bx[:, :, 1:n] = ta
    by = torch.zeros((n, n + 1, n), dtype=torch.float64, device=dev)
    by[:, 1:n, :] = ta
    bz = torch.from_numpy(bz1).to(dev)[:, None, None].expand(n + 1, n, n).contiguous()
    b = torch.from_numpy(b1).to(dev)[:, None, None].expand(n, n, n).contiguous()
    return (bx, by, bz, b), bz1, b1


@pytest.mark.parametrize("ratio", [10.0, 1000.0])
def test_layered_closed_form_1024(ratio):
    """The largest benchmark size: 1024^3 with coefficients and rhs varying in z
    only (a flat film), checked against the exact 1-D flux-form solution (a closed
    form, no oracle) in both precisions.  Density ratio 10: both solvers reach
    relative residual 1e-10.  Density ratio 1000: the solution grows to |p| ~ 3e6
    while b ~ 1, so rounding in the FP64 residual b - L p leaves a floor near 4e-10
    and 1e-10 cannot be reached by any FP64 evaluation; the solve runs into that
    floor and the error against the closed form is checked there.  The 1e-8 bar is
    on the error in both cases, with its margin printed."""
    import torch
    from paper_1410_8568_amd import mg
    n = 1024
    (bx, by, bz, b), bz1, b1 = _layered_on_device(n, ratio)
    p1 = torch.from_numpy(pins.layered_solve(bz1, b1)).cuda()[:, None, None]
    norm_star = float(torch.linalg.vector_norm(p1.expand(n, n, n)))
    for precision in ("fp32_refined", "fp64"):
        cap = 30 if precision == "fp32_refined" else 80
        S = mg.Solver(bx, by, bz, precision=precision, n_coarsest=8, max_cycles=cap, graph=True)
        p = torch.zeros_like(b)
        st = S.solve(b, p, tol=1e-10, check=False)
        err = float(torch.linalg.vector_norm(p - p1)) / norm_star
        h = st["history"]
        print(f"1024^3 layered ratio {ratio:g} {precision}: rc {st['rc']} cycles {st['cycles']} "
              f"rel residual {st['rel_residual']:.3e} error {err:.3e} (margin {1e-8 / err:.0f}x); "
              f"residual every 5 iterations {['%.1e' % x for x in h[::5]]}", flush=True)
        S.close()
        del p
        if ratio == 10.0:
            assert st["rc"] == 0
        else:
            assert st["rc"] in (0, mg.MG_E_NOT_CONVERGED) and st["rel_residual"] <= 1e-9
        assert err <= 1e-8


def cylinder_problem(n, seed=17, ratio=1000.0):
    """A liquid cylinder along z (radius 0.3 in index-normalised x, y), N(0,1) rhs."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid((np.arange(ny) + .5) / ny, (np.arange(nx) + .5) / nx, indexing="ij")
    ind = inputs.smoothed_heaviside(0.3 - np.sqrt((x - .4) ** 2 + (y - .6) ** 2), 1.5 / nx)
    alpha = np.broadcast_to(1.0 / (1.0 + (ratio - 1.0) * ind), (nz, ny, nx)).copy()
    bx, by, bz = inputs.faces_from_alpha(alpha)
    return inputs.Problem(n, bx, by, bz, rng.standard_normal((nz, ny, nx)), dict(kind="cylinder"))


@pytest.mark.parametrize("precision,krylov", [("fp64", "none"), ("fp32_refined", "none"), ("fp64", "fcg")])
def test_level0_column_residual_kernels(precision, krylov):
    """A level-0 plane of 1024 x 512 cells (more than 512 x 512) sends the finest
    residual of every mode (convergence norm, refinement residual with its FP32
    copy, Krylov residual) through the cell-pair column kernels instead of the flat
    one; the grid coarsens 1024x512x32 -> ... -> 32x16x1 (512 cells, solved
    exactly).  The field is a 1000:1 cylinder along z (a sphere on this flat grid
    is resolved by too few planes on the coarse levels and converges slowly, in
    the oracle alike).  p against the oracle at 1e-8 in every mode.  The FP64
    residual arithmetic of the kernel is checked by the FP64 and Krylov
    histories at 1e-9; in FP32-refined mode the history after each outer
    iteration also carries the FP32 rounding of three inner cycles, which on this
    field differs from the oracle's FP32 emulation by up to 5.4e-4 relative after
    the first outer iteration (FMA contraction, reciprocal-based quotient and
    summation order, amplified by the cycle), so there it is compared at the FP32
    late-regime bound 1e-3 together with an equal number of outer iterations."""
    n = (1024, 512, 32)
    P = cylinder_problem(n)
    ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, precision=precision, krylov=krylov)
    assert ref["status"] == "converged"
    p, st = gpu_solve(P, precision=precision, tol=1e-10, krylov=krylov)
    assert st["rc"] == 0, st
    assert st["levels"] == 6
    err = rel(p, ref["p"])
    dev = max(abs(g - o) / o for g, o in zip(st["history"], ref["history"]))
    print(f"{n} {precision} {krylov}: cycles {st['cycles']} oracle rel err {err:.3e}, "
          f"largest relative history deviation {dev:.2e}", flush=True)
    assert err <= 1e-8
    if precision == "fp64":
        check_history(st["history"], ref["history"], precision)
    else:
        assert len(st["history"]) == len(ref["history"])
        assert dev <= 1e-3


def test_unaligned_solve_arrays_rejected():
    """p or rhs 8 bytes past a 16-byte boundary: refused before any launch."""
    import torch
    from paper_1410_8568_amd import mg
    P = inputs.config0()
    bx, by, bz, b = mg.to_device(P)
    S = mg.Solver(bx, by, bz)
    buf = torch.zeros(b.numel() + 1, dtype=torch.float64, device="cuda")
    pu = buf[1:].view(b.shape)
    assert pu.data_ptr() % 16 == 8
    st = S.solve(b, pu, check=False)
    assert st["rc"] == mg.MG_E_INVALID
    bu = torch.empty_like(buf)[1:].view(b.shape)
    bu.copy_(b)
    st = S.solve(bu, torch.zeros_like(b), check=False)
    assert st["rc"] == mg.MG_E_INVALID
    assert torch.count_nonzero(buf).item() == 0
    S.close()
