"""GPU parity of the projection step (MAC divergence, pressure solve, velocity
correction) against the CPU oracle, through the C ABI.

Bars: the divergence and the correction evaluate the same expressions in the
same order without fused multiply-adds, so they must equal the oracle bit for
bit; the composed step inherits the solve's bar (p within 1e-8 relative L2 of
the oracle's p) and its velocity must agree with the oracle's to 1e-8 of the
size of the correction, with a discrete divergence at the solve's tolerance.
"""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import rel
from paper_1410_8568_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_8568_amd import mg
    mg.lib()


def dev(*arrays):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays)


def host(*tensors):
    import torch
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in tensors)


def velocity(n, seed, walls):
    return inputs.velocity_field(n, np.random.default_rng(seed), walls=walls)


# one thread per two cells of a row (odd nx: per cell), 512 per workgroup: grids
# below span several workgroups with ragged ends, odd and even nx, and the
# degenerate one-cell and one-plane cases
GRIDS = [(1, 1, 1), (5, 7, 3), (70, 9, 13), (128, 8, 64), (130, 6, 2), (64, 4, 1), (3, 200, 5)]


@pytest.mark.parametrize("n", GRIDS)
def test_divergence_bit_exact(n):
    from paper_1410_8568_amd import mg
    u, v, w = velocity(n, 31, walls=True)
    scale = 0.37
    b, = host(mg.divergence(*dev(u, v, w), scale))
    assert np.array_equal(b, oracle.divergence(u, v, w, scale))


def test_divergence_empty_grid_is_a_no_op():
    import ctypes
    import torch
    from paper_1410_8568_amd import mg
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    for n in [(0, 3, 3), (3, 0, 3), (3, 3, 0)]:
        rc = mg.lib().mg_divergence(ctypes.byref(mg.Grid(*n)), mg._ptr(t), mg._ptr(t), mg._ptr(t),
                                    ctypes.c_double(1.0), mg._ptr(t), mg._stream(None))
        assert rc == mg.MG_OK
    assert torch.count_nonzero(t).item() == 0
    rc = mg.lib().mg_divergence(ctypes.byref(mg.Grid(-1, 3, 3)), mg._ptr(t), mg._ptr(t), mg._ptr(t),
                                ctypes.c_double(1.0), mg._ptr(t), mg._stream(None))
    assert rc == mg.MG_E_INVALID
    rc = mg.lib().mg_divergence(ctypes.byref(mg.Grid(3, 3, 3)), mg._ptr(t), mg._ptr(t), mg._ptr(t),
                                ctypes.c_double(float("nan")), mg._ptr(t), mg._stream(None))
    assert rc == mg.MG_E_INVALID


# grids the solver accepts (coarsest level <= 512 cells), across tiles and chunks
@pytest.mark.parametrize("n", [(2, 2, 2), (5, 7, 3), (72, 12, 16), (128, 8, 64), (4, 200, 8), (130, 6, 2)])
def test_correction_bit_exact(n):
    """Random faces, pressure and velocity (walls included: they must come back
    unchanged), against the oracle's correction."""
    from paper_1410_8568_amd import mg
    rng = np.random.default_rng(32)
    bx, by, bz = pins.random_faces(n, rng, contrast=1000.0)
    nx, ny, nz = n
    p = rng.standard_normal((nz, ny, nx))
    u, v, w = velocity(n, 33, walls=True)
    S = mg.Solver(*dev(bx, by, bz))
    gu, gv, gw, gp = dev(u, v, w, p)
    S.correct_velocity(gp, gu, gv, gw, 0.61)
    ou, ov, ow = oracle.correct_velocity(bx, by, bz, p, u, v, w, 0.61)
    hu, hv, hw = host(gu, gv, gw)
    assert np.array_equal(hu, ou) and np.array_equal(hv, ov) and np.array_equal(hw, ow)
    S.close()


def unaligned(a):
    """Device copy of `a` that starts 8 bytes past a 16-byte boundary (the kernels
    then take their one-cell-per-thread path)."""
    import torch
    buf = torch.empty(a.size + 1, dtype=torch.float64, device="cuda")
    t = buf[1:].view(a.shape)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    assert t.data_ptr() % 16 == 8 and t.is_contiguous()
    return t


def test_unaligned_arrays_take_the_scalar_path_bit_exactly():
    from paper_1410_8568_amd import mg
    n = (72, 12, 16)
    rng = np.random.default_rng(38)
    bx, by, bz = pins.random_faces(n, rng, contrast=1000.0)
    p = rng.standard_normal((16, 12, 72))
    u, v, w = velocity(n, 39, walls=True)
    b, = host(mg.divergence(unaligned(u), unaligned(v), unaligned(w), 1.7, unaligned(np.zeros((16, 12, 72)))))
    assert np.array_equal(b, oracle.divergence(u, v, w, 1.7))
    S = mg.Solver(*dev(bx, by, bz))
    gu, gv, gw, gp = unaligned(u), unaligned(v), unaligned(w), unaligned(p)
    S.correct_velocity(gp, gu, gv, gw, 0.3)
    ou, ov, ow = oracle.correct_velocity(bx, by, bz, p, u, v, w, 0.3)
    hu, hv, hw = host(gu, gv, gw)
    assert np.array_equal(hu, ou) and np.array_equal(hv, ov) and np.array_equal(hw, ow)
    S.close()


def ragged_drop(n, seed=2):
    """Drop-splash geometry on a non-cubic grid (cells cubic in index space)."""
    nx, ny, nz = n
    z, y, x = np.meshgrid((np.arange(nz) + .5) / nz, (np.arange(ny) + .5) / ny, (np.arange(nx) + .5) / nx,
                          indexing="ij")
    phi = np.maximum(0.1 - z, 0.08 - np.sqrt((x - .5) ** 2 + (y - .5) ** 2 + (z - .2) ** 2))
    ind = inputs.smoothed_heaviside(phi, 1.5 / max(n))
    return inputs.faces_from_alpha(1.0 / (1.0 + 999.0 * ind))


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("n", [(48, 40, 24), (64, 64, 64), (96, 48, 32)])
def test_project_matches_oracle(precision, n):
    from paper_1410_8568_amd import mg
    bx, by, bz = ragged_drop(n)
    u, v, w = velocity(n, 34, walls=False)
    h, dt = 1.0 / max(n), 1e-3
    ref = oracle.project(bx, by, bz, u, v, w, dt, h, tol=1e-10, precision=precision)
    S = mg.Solver(*dev(bx, by, bz), precision=precision)
    gu, gv, gw = dev(u, v, w)
    st = S.project(gu, gv, gw, dt, h, tol=1e-10)
    assert st["rc"] == 0 and st["rel_residual"] <= 1e-10
    hu, hv, hw, hb, hp = host(gu, gv, gw, st["b"], st["p"])
    assert np.array_equal(hb, ref["b"])
    assert rel(hp, ref["p"]) <= 1e-8
    corr = np.sqrt(sum(np.sum((r - a) ** 2) for r, a in zip((ref["u"], ref["v"], ref["w"]), (u, v, w))))
    diff = np.sqrt(sum(np.sum((g - r) ** 2) for g, r in zip((hu, hv, hw), (ref["u"], ref["v"], ref["w"]))))
    assert diff <= 1e-8 * corr
    # the projected field is discretely divergence-free to the solve's tolerance
    d = oracle.divergence(hu, hv, hw, h / dt)
    assert np.linalg.norm(d) <= 2e-10 * np.linalg.norm(hb)
    S.close()


def test_project_divergence_free_input_is_unchanged():
    """A discrete curl (edge potentials zero on the walls) has b = 0 to rounding:
    p comes back 0 and the velocity unchanged."""
    from paper_1410_8568_amd import mg
    rng = np.random.default_rng(35)
    n = (40, 24, 16)
    nx, ny, nz = n
    pz = np.zeros((nz, ny + 1, nx + 1)); pz[:, 1:ny, 1:nx] = rng.standard_normal((nz, ny - 1, nx - 1))
    u = pz[:, 1:, :] - pz[:, :-1, :]
    v = -(pz[:, :, 1:] - pz[:, :, :-1])
    w = np.zeros((nz + 1, ny, nx))
    bx, by, bz = ragged_drop(n)
    S = mg.Solver(*dev(bx, by, bz))
    gu, gv, gw = dev(u, v, w)
    st = S.project(gu, gv, gw, 0.01, 1.0 / 40, tol=1e-10)
    assert st["rc"] == 0
    hu, hv, hw, hb = host(gu, gv, gw, st["b"])
    assert np.abs(hb).max() <= 1e-12
    # the solve of a right-hand side of rounding noise moves the velocity by noise only
    umax = max(np.abs(a).max() for a in (u, v, w))
    for g, a in ((hu, u), (hv, v), (hw, w)):
        assert np.abs(g - a).max() <= 1e-9 * umax
    S.close()


def test_project_error_paths():
    import torch
    from paper_1410_8568_amd import mg
    n = (8, 8, 8)
    bx, by, bz = ragged_drop(n)
    u, v, w = velocity(n, 36, walls=False)
    S = mg.Solver(*dev(bx, by, bz), max_cycles=1)
    gu, gv, gw = dev(u, v, w)
    for dt, h in ((0.0, 0.1), (0.1, -1.0), (float("inf"), 0.1)):
        with pytest.raises(mg.MGError) as ei:
            S.project(gu, gv, gw, dt, h)
        assert ei.value.status == mg.MG_E_INVALID
    # a solve that does not converge leaves the velocity untouched
    u0 = gu.clone()
    st = S.project(gu, gv, gw, 0.01, 0.125, tol=1e-14, check=False)
    assert st["rc"] == mg.MG_E_NOT_CONVERGED
    assert torch.equal(gu, u0)
    S.close()


def test_project_full_size_512():
    """The 512^3 drop splash of the benchmark with a random velocity (FP32-refined,
    coarsest 8^3): the divergence and the correction equal the oracle's at full size
    (the correction fed the GPU pressure), and the projected field is divergence-free
    to the solve's tolerance."""
    import torch
    from paper_1410_8568_amd import mg
    P = inputs.config2(512)
    n = P.n
    h, dt = 1.0 / 512, 1e-3
    u, v, w = velocity(n, 37, walls=False)
    S = mg.Solver(*dev(P.bx, P.by, P.bz), precision="fp32_refined", n_coarsest=8)
    gu, gv, gw = dev(u, v, w)
    st = S.project(gu, gv, gw, dt, h, tol=1e-10)
    assert st["rc"] == 0 and st["rel_residual"] <= 1e-10
    cycles = st["cycles"]
    hb, hp = host(st["b"], st["p"])
    assert np.array_equal(hb, oracle.divergence(u, v, w, h / dt))
    del st, hb
    hu, = host(gu)
    del gu
    hv, = host(gv)
    del gv
    hw, = host(gw)
    del gw
    torch.cuda.empty_cache()
    ou, ov, ow = oracle.correct_velocity(P.bx, P.by, P.bz, hp, u, v, w, dt / h)
    assert np.array_equal(hu, ou) and np.array_equal(hv, ov) and np.array_equal(hw, ow)
    del ou, ov, ow
    d = oracle.divergence(hu, hv, hw, h / dt)
    b = oracle.divergence(u, v, w, h / dt)
    print(f"512^3 projection: cycles {cycles} div rel {np.linalg.norm(d) / np.linalg.norm(b):.3e}", flush=True)
    assert np.linalg.norm(d) <= 2e-10 * np.linalg.norm(b)
    S.close()
