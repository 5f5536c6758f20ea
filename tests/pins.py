"""Independent references that pin the oracle (CPU only, no GPU).

None of these call the oracle.  Each reduces the problem to a textbook routine
or a closed form:

* ``bordered_direct_solve`` - the unique mean-zero solution of L p = b - mean(b),
  from a sparse LU of the bordered system [[L, 1], [1^T, 0]];
* ``layered_solve`` - coefficients and rhs that vary with z only: the 3-D
  solution is a 1-D Neumann problem solved by two cumulative sums (flux form);
* ``dct_solve`` - constant coefficients: the operator is diagonalised by the
  DCT-II with eigenvalues -beta * sum_d 4 sin^2(pi m_d / (2 n_d));
* ``manufactured`` - a smooth alpha and p with zero normal derivative, whose
  analytic divergence gives a right-hand side with an O(h^2) discrete error;
* ``trilinear_prolong`` - cell-centred trilinear interpolation (weights 3/4, 1/4
  per axis), built as a Kronecker product of 1-D matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def assemble(bx, by, bz):
    """Sparse matrix of the 7-point operator of eq. (10) in 3-D (h^2 form)."""
    nz, ny, nxp = bx.shape
    nx = nxp - 1
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []

    def link(a, b, w):
        rows.extend([a, b, a, b]); cols.extend([b, a, a, b]); vals.extend([w, w, -w, -w])

    w = bx[:, :, 1:nx].ravel()
    a, b = idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()
    link(a, b, w)
    w = by[:, 1:ny, :].ravel()
    a, b = idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()
    link(a, b, w)
    w = bz[1:nz, :, :].ravel()
    a, b = idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()
    link(a, b, w)
    rows = np.concatenate([np.asarray(r) for r in rows])
    cols = np.concatenate([np.asarray(c) for c in cols])
    vals = np.concatenate([np.asarray(v) for v in vals])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def bordered_direct_solve(bx, by, bz, b):
    """Unique mean-zero p with L p = b - mean(b), by sparse LU.

    The null space (constants) is removed by grounding cell 0 (deleting its row
    and column); the compatible right-hand side makes the deleted equation hold
    automatically.  The result is then shifted to zero mean."""
    L = assemble(bx, by, bz).tocsc()
    bb = b.ravel() - b.mean()
    x = spla.spsolve(L[1:, 1:], bb[1:])
    p = np.concatenate([[0.0], x])
    return (p - p.mean()).reshape(b.shape)


def layered_solve(bz_line, b_line):
    """1-D flux form: F_{k+1/2} = sum_{m<=k} b_bar_m, p_{k+1} = p_k + F_{k+1/2} / beta_{k+1}."""
    bbar = b_line - b_line.mean()
    F = np.cumsum(bbar)[:-1]                 # fluxes through interior faces 1..n-1
    p = np.concatenate([[0.0], np.cumsum(F / bz_line[1:-1])])
    return p - p.mean()


def dct_solve(b, beta=1.0):
    """Constant-coefficient exact solve by DCT-II diagonalisation (mean-zero)."""
    nz, ny, nx = b.shape
    bb = b - b.mean()
    bh = scipy.fft.dctn(bb, type=2, norm="ortho")
    lam = np.zeros_like(bh)
    for axis, n in zip((2, 1, 0), (nx, ny, nz)):
        m = np.arange(n)
        shape = [1, 1, 1]
        shape[axis] = n
        lam = lam + (4.0 * np.sin(np.pi * m / (2.0 * n)) ** 2).reshape(shape)
    lam = -beta * lam
    ph = np.zeros_like(bh)
    nz0 = lam != 0
    ph[nz0] = bh[nz0] / lam[nz0]
    return scipy.fft.idctn(ph, type=2, norm="ortho")


def manufactured(n):
    """alpha = 1 + cos(pi x) cos(pi y) cos(pi z) / 2, p = cos(pi x) cos(pi y) cos(pi z).

    grad p . n = 0 on the walls of the unit cube and p has zero mean over the
    cell-centre grid.  f = div(alpha grad p); b = h^2 f at cell centres; face
    coefficients are alpha at face centres."""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    f = np.arange(n + 1) * h
    pi = np.pi

    def alpha(x, y, z):
        return 1.0 + 0.5 * np.cos(pi * x) * np.cos(pi * y) * np.cos(pi * z)

    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    P = np.cos(pi * X) * np.cos(pi * Y) * np.cos(pi * Z)
    A = alpha(X, Y, Z)
    gx = -pi * np.sin(pi * X) * np.cos(pi * Y) * np.cos(pi * Z)
    gy = -pi * np.cos(pi * X) * np.sin(pi * Y) * np.cos(pi * Z)
    gz = -pi * np.cos(pi * X) * np.cos(pi * Y) * np.sin(pi * Z)
    # div(alpha grad p) = alpha lap p + grad alpha . grad p, grad alpha = grad p / 2
    fval = A * (-3.0 * pi * pi * P) + 0.5 * (gx * gx + gy * gy + gz * gz)
    b = h * h * fval
    Zx, Yx, Xx = np.meshgrid(c, c, f, indexing="ij")
    bx = alpha(Xx, Yx, Zx)
    Zy, Yy, Xy = np.meshgrid(c, f, c, indexing="ij")
    by = alpha(Xy, Yy, Zy)
    Zz, Yz, Xz = np.meshgrid(f, c, c, indexing="ij")
    bz = alpha(Xz, Yz, Zz)
    bx[:, :, 0] = bx[:, :, -1] = 0
    by[:, 0, :] = by[:, -1, :] = 0
    bz[0, :, :] = bz[-1, :, :] = 0
    return bx, by, bz, b, P


def _interp_1d(nc):
    """Cell-centred linear interpolation coarse (nc) -> fine (2 nc), mirror at walls."""
    M = np.zeros((2 * nc, nc))
    for I in range(nc):
        lo, hi = 2 * I, 2 * I + 1
        M[lo, I] += 0.75
        M[lo, max(I - 1, 0)] += 0.25
        M[hi, I] += 0.75
        M[hi, min(I + 1, nc - 1)] += 0.25
    return M


def trilinear_prolong(ec):
    """Textbook trilinear cell-centred prolongation of ec (uniform weights)."""
    cz, cy, cx = ec.shape
    Mx, My, Mz = _interp_1d(cx), _interp_1d(cy), _interp_1d(cz)
    out = np.einsum("kK,KJI->kJI", Mz, ec)
    out = np.einsum("jJ,kJI->kjI", My, out)
    return np.einsum("iI,kjI->kji", Mx, out)


def random_faces(n, rng, lo=0.5, hi=2.0, contrast=None):
    """Random positive interior faces; with ``contrast`` a random half of the cells
    is 'liquid' with alpha / contrast (faces arithmetic)."""
    nx, ny, nz = n
    if contrast is None:
        bx = rng.uniform(lo, hi, (nz, ny, nx + 1))
        by = rng.uniform(lo, hi, (nz, ny + 1, nx))
        bz = rng.uniform(lo, hi, (nz + 1, ny, nx))
    else:
        alpha = np.where(rng.random((nz, ny, nx)) < 0.5, 1.0, 1.0 / contrast)
        bx = np.zeros((nz, ny, nx + 1)); by = np.zeros((nz, ny + 1, nx)); bz = np.zeros((nz + 1, ny, nx))
        bx[:, :, 1:nx] = 0.5 * (alpha[:, :, 1:] + alpha[:, :, :-1])
        by[:, 1:ny, :] = 0.5 * (alpha[:, 1:, :] + alpha[:, :-1, :])
        bz[1:nz, :, :] = 0.5 * (alpha[1:, :, :] + alpha[:-1, :, :])
    bx[:, :, 0] = bx[:, :, -1] = 0
    by[:, 0, :] = by[:, -1, :] = 0
    bz[0, :, :] = bz[-1, :, :] = 0
    return bx, by, bz
