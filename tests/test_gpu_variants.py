"""GPU parity of the paper-faithful cycle variants (SOR factor, 64-point
restriction, GMRES on the coarsest grid) against the CPU oracle, through the
C ABI.  Bars as for the standard cycle: per-cycle residual histories equal to
rounding (the precision's tolerance), p within 1e-8 of the oracle's p."""
import numpy as np
import pytest

import oracle
from gpu_util import check_history, gpu_solve, rel
from paper_1410_8568_amd import inputs
from test_gpu_parity import ragged_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_8568_amd import mg
    mg.lib()


VARIANTS = {
    "sor1.3": (dict(omega=1.3), dict(omega=1.3)),
    "sor0.8": (dict(omega=0.8), dict(omega=0.8)),
    "restrict64": (dict(restrict64=True), dict(restrict64=True)),
    "gmres16": (dict(coarse_gmres=16, coarse_gmres_tol=1e-3, coarse_gmres_maxit=300),
                dict(gmres_m=16, gmres_tol=1e-3, gmres_maxit=300)),
    "all": (dict(omega=1.2, restrict64=True, coarse_gmres=8, coarse_gmres_tol=1e-4, coarse_gmres_maxit=500),
            dict(omega=1.2, restrict64=True, gmres_m=8, gmres_tol=1e-4, gmres_maxit=500)),
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("n,nc", [((40, 24, 12), 4), ((64, 48, 40), 8), ((6, 10, 4), 4)])
def test_variant_matches_oracle(variant, precision, n, nc):
    gkw, okw = VARIANTS[variant]
    P = ragged_problem(n)
    ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, n_coarsest=nc, precision=precision, **okw)
    p, st = gpu_solve(P, precision=precision, tol=1e-10, n_coarsest=nc, **gkw)
    assert st["rc"] == 0, st
    check_history(st["history"], ref["history"], precision)
    assert rel(p, ref["p"]) <= 1e-8


@pytest.mark.parametrize("variant", ["sor1.3", "all"])
def test_variant_under_krylov_matches_oracle(variant):
    gkw, okw = VARIANTS[variant]
    P = ragged_problem((48, 40, 24))
    ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, krylov="fcg", **okw)
    p, st = gpu_solve(P, tol=1e-10, krylov="fcg", **gkw)
    assert st["rc"] == 0, st
    check_history(st["history"], ref["history"])
    assert rel(p, ref["p"]) <= 1e-8


def test_variants_graph_replay_bit_identical():
    P = ragged_problem((64, 64, 64), seed=9)
    gkw = VARIANTS["all"][0]
    for precision in ("fp64", "fp32_refined"):
        ref_p, ref_st = gpu_solve(P, precision=precision, tol=1e-10, graph=False, **gkw)
        p, st = gpu_solve(P, precision=precision, tol=1e-10, graph=True, **gkw)
        assert st["history"] == ref_st["history"] and np.array_equal(p, ref_p)


def test_variant_options_are_validated():
    from paper_1410_8568_amd import mg
    P = inputs.config0()
    bx, by, bz, _ = mg.to_device(P)
    for kw in (dict(omega=0.0), dict(omega=2.0), dict(coarse_gmres=17), dict(coarse_gmres=-1),
               dict(coarse_gmres=4, coarse_gmres_tol=0.0), dict(coarse_gmres=4, coarse_gmres_maxit=0)):
        with pytest.raises(mg.MGError) as ei:
            mg.Solver(bx, by, bz, **kw)
        assert ei.value.status == mg.MG_E_INVALID, kw
    S = mg.Solver(bx, by, bz, restrict64=True)
    assert all(t == -1 or 1 <= t <= mg.MG_NUM_TILES for t in S.tiles()[:-1])
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_restrict64_fused_tiles_bit_identical_to_reference(precision):
    """With the 64-point restriction the smoother runs the fused passes too (the
    residual goes to whichever iterate buffer the passes left free, one or two
    sweeps per pass, ragged tiles and chunks): every tile gives exactly the
    reference one-colour kernels' iterates."""
    from paper_1410_8568_amd import mg
    P = ragged_problem((64, 48, 40), seed=6)
    ref_p, ref_st = gpu_solve(P, precision=precision, tol=1e-10, tile=-1, restrict64=True)
    for tile in range(1, mg.MG_NUM_TILES + 1):
        p, st = gpu_solve(P, precision=precision, tol=1e-10, tile=tile, restrict64=True)
        assert st["history"] == ref_st["history"], tile
        assert np.array_equal(p, ref_p), tile


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_fused_sor_tiles_bit_identical_to_reference(precision):
    """The fused red-black passes with over-relaxation (every tile shape, one or
    two sweeps per pass, the pre-smoothing pass that restricts, zero-input first
    passes) give exactly the reference one-colour SOR kernels' iterates."""
    from paper_1410_8568_amd import mg
    P = ragged_problem((64, 48, 40), seed=5)
    ref_p, ref_st = gpu_solve(P, precision=precision, tol=1e-10, tile=-1, omega=1.3)
    for tile in range(1, mg.MG_NUM_TILES + 1):
        p, st = gpu_solve(P, precision=precision, tol=1e-10, tile=tile, omega=1.3)
        assert st["history"] == ref_st["history"], tile
        assert np.array_equal(p, ref_p), tile


def test_variants_config1_full_size_matches_oracle():
    """256^3 drop splash (FP64): SOR 1.2 with the 64-point restriction and coarse
    GMRES against the oracle with the same variants."""
    P = inputs.config1(256)
    gkw, okw = VARIANTS["all"]
    ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, **okw)
    assert ref["status"] == "converged"
    p, st = gpu_solve(P, tol=1e-10, **gkw)
    assert st["rc"] == 0, st
    check_history(st["history"], ref["history"])
    err = rel(p, ref["p"])
    print(f"256^3 variants: cycles {st['cycles']} (oracle {ref['cycles']}) gamma {st['gamma']:.3f} "
          f"oracle rel err {err:.3e}", flush=True)
    assert err <= 1e-8
