"""Helpers shared by the GPU tests (device transfer, oracle comparison)."""
import numpy as np


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gpu_solve(P, precision="fp64", tol=1e-10, p0=None, **kw):
    import torch
    from paper_1410_8568_amd import mg
    bx, by, bz, b = mg.to_device(P)
    S = mg.Solver(bx, by, bz, precision=precision, **kw)
    p = torch.zeros_like(b) if p0 is None else torch.from_numpy(p0).cuda()
    st = S.solve(b, p, tol=tol, check=False)
    out = p.cpu().numpy()
    S.close()
    return out, st


def check_history(h_gpu, h_or, precision="fp64"):
    """Per-cycle relative residuals agree; tight while far above rounding, looser near
    the attainable-accuracy floor (different FMA contraction and summation order).

    FP64: 1e-9 relative above 1e-7, 1e-5 below.  FP32-refined: the inner cycles
    round at FP32 epsilon (6e-8) differently from the oracle's FP32 emulation (FMA
    contraction, the reciprocal-based FP32 quotient, the summation order of the
    prolongation corners), and the residual after a cycle is a small difference of
    large terms that amplifies those roundings a few hundred times, so 1e-4 / 1e-3.
    The formulas themselves are the same templates that the FP64 runs check at 1e-9."""
    early_rtol, late_rtol = (1e-9, 1e-5) if precision == "fp64" else (1e-4, 1e-3)
    assert len(h_gpu) == len(h_or), (len(h_gpu), len(h_or))
    for c, (g, o) in enumerate(zip(h_gpu, h_or)):
        tol = early_rtol if o > 1e-7 else late_rtol
        # below ~1e-13 both sides sit at the rounding floor of an FP64 residual
        assert abs(g - o) <= tol * o + 1e-13, (c, g, o)
