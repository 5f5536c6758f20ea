"""GPU parity of the level-set property kernel (indicator, eq. 8, alpha = 1/rho,
face means) against the CPU oracle, through the C ABI.

Bar: the kernel evaluates the oracle's expressions in the oracle's order
without fused multiply-adds, so every face both of whose cells lie outside the
interface band is bit-identical; inside the band the device sine may differ
from the host's in the last bit, which after eq. (8) and the face mean stays
below 1e-13 relative."""
import numpy as np
import pytest

import oracle
from gpu_util import gpu_solve, rel
from paper_1410_8568_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_8568_amd import mg
    mg.lib()


def sphere_levelset(n, r=0.3, c=(0.45, 0.55, 0.5)):
    nx, ny, nz = n
    z, y, x = np.meshgrid((np.arange(nz) + .5) / nz, (np.arange(ny) + .5) / ny, (np.arange(nx) + .5) / nx,
                          indexing="ij")
    return r - np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)


def band_faces(phi, eps):
    """Masks of the faces with a cell inside the band |phi| < eps, per direction."""
    inb = np.abs(phi) < eps
    nz, ny, nx = phi.shape
    mx = np.zeros((nz, ny, nx + 1), bool); mx[:, :, 1:nx] = inb[:, :, 1:] | inb[:, :, :-1]
    my = np.zeros((nz, ny + 1, nx), bool); my[:, 1:ny, :] = inb[:, 1:, :] | inb[:, :-1, :]
    mz = np.zeros((nz + 1, ny, nx), bool); mz[1:nz] = inb[1:] | inb[:-1]
    return mx, my, mz


def check_faces(got, ref, phi, eps):
    for g, r, m in zip(got, ref, band_faces(phi, eps)):
        assert g.shape == r.shape
        assert np.array_equal(g[~m], r[~m])
        if m.any():
            assert np.max(np.abs(g[m] - r[m]) / np.abs(r[m])) <= 1e-13


@pytest.mark.parametrize("faces", ["arith", "harmonic"])
@pytest.mark.parametrize("n", [(1, 1, 1), (2, 3, 4), (5, 7, 3), (70, 9, 13), (128, 8, 64), (40, 200, 6)])
def test_faces_match_oracle(n, faces):
    import torch
    from paper_1410_8568_amd import mg
    phi = sphere_levelset(n)
    eps = 1.5 / max(n)
    got = mg.faces_from_levelset(torch.from_numpy(phi).cuda(), 1000.0, 1.0, eps, faces)
    torch.cuda.synchronize()
    check_faces([t.cpu().numpy() for t in got], oracle.faces_from_levelset(phi, 1000.0, 1.0, eps, faces), phi, eps)


def test_unaligned_arrays_take_the_scalar_path_bit_exactly():
    import torch
    from paper_1410_8568_amd import mg
    n = (64, 12, 10)
    phi = sphere_levelset(n)
    eps = 1.5 / 64
    ref = [t.cpu().numpy() for t in mg.faces_from_levelset(torch.from_numpy(phi).cuda(), 50.0, 2.0, eps, "harmonic")]
    buf = torch.empty(phi.size + 1, dtype=torch.float64, device="cuda")
    uphi = buf[1:].view(phi.shape)
    uphi.copy_(torch.from_numpy(phi))
    assert uphi.data_ptr() % 16 == 8
    got = [t.cpu().numpy() for t in mg.faces_from_levelset(uphi, 50.0, 2.0, eps, "harmonic")]
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_invalid_arguments():
    import torch
    from paper_1410_8568_amd import mg
    phi = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    for args in ((0.0, 1.0, 0.1), (1.0, -1.0, 0.1), (1.0, 1.0, 0.0), (float("nan"), 1.0, 0.1)):
        with pytest.raises(mg.MGError) as ei:
            mg.faces_from_levelset(phi, *args)
        assert ei.value.status == mg.MG_E_INVALID


def test_full_size_512_faces_and_solve():
    """The 512^3 benchmark field built on the device from its level set: faces as
    the oracle's, and the FP32-refined solve with them equal to the solve with the
    host-built faces."""
    import torch
    from paper_1410_8568_amd import mg
    phi = inputs.drop_splash_levelset(512, seed=2, perturb=True)
    eps = 1.5 / 512
    gphi = torch.from_numpy(phi).cuda()
    got = mg.faces_from_levelset(gphi, 1000.0, 1.0, eps)
    del gphi
    hgot = [t.cpu().numpy() for t in got]
    check_faces(hgot, oracle.faces_from_levelset(phi, 1000.0, 1.0, eps), phi, eps)
    del phi
    P = inputs.config2(512)
    for g, r in zip(hgot, (P.bx, P.by, P.bz)):   # the host generator, to its clip rounding
        assert np.max(np.abs(g - r)) <= 1e-13 * np.abs(r).max()
    del hgot
    b = torch.from_numpy(P.b).cuda()
    S = mg.Solver(*got, precision="fp32_refined", n_coarsest=8)
    p = torch.zeros_like(b)
    st = S.solve(b, p, tol=1e-10)
    S.close()
    del got
    p_host, st_host = gpu_solve(P, precision="fp32_refined", tol=1e-10, n_coarsest=8)
    err = rel(p.cpu().numpy(), p_host)
    print(f"512^3 device-built faces: cycles {st['cycles']} / {st_host['cycles']}, p rel diff {err:.2e}", flush=True)
    assert st["rc"] == 0 and err <= 1e-8
