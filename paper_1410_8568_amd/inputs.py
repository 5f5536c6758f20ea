"""Seeded synthetic inputs for the pressure solve: drop-splash density fields,
face coefficients and right-hand sides.

This module builds the *inputs* of the solve and nothing else.  It is shared by
the CPU oracle tests and by the GPU path; it contains none of the solver's
arithmetic (no operator, smoothing, transfer or coarse solve).

Geometry and properties follow the paper's description of its workloads:

* the indicator function is a numerical Heaviside that goes from 0 to 1 over
  three to four cells (Sec. 2.2, text after eq. 3); we use the standard smoothed
  Heaviside of a signed distance with half-width 1.5 h;
* material properties are mixed linearly by the indicator, eq. (8):
  rho = rho_g + (rho_l - rho_g) * I;
* the pressure equation (9) has coefficient alpha = 1 / rho; the face
  coefficients are the arithmetic mean of the two adjacent cells' alpha
  (default) or the harmonic mean of eqs. (11)-(12) (``faces='harmonic'``).

Conventions: an n_x x n_y x n_z grid of cubic cells on the unit cube (h = 1/n),
arrays in C order [k][j][i] with i fastest, x-faces [n_z][n_y][n_x+1] (face i
lies between cells i-1 and i), y-faces [n_z][n_y+1][n_x], z-faces
[n_z+1][n_y][n_x].  Wall faces are returned as 0 (homogeneous Neumann).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "smoothed_heaviside", "cell_centres", "faces_from_alpha",
    "divergence_rhs", "velocity_field", "normal_rhs", "drop_splash_levelset", "sphere_problem", "drop_splash_problem",
    "config0", "config1", "config2", "batch_problems", "request_stream",
    "layered_problem", "layered_profile", "constant_problem", "scene_levelset",
]


@dataclasses.dataclass
class Problem:
    """One pressure solve: faces (walls 0), right-hand side and a description."""
    n: tuple            # (nx, ny, nz)
    bx: np.ndarray      # [nz][ny][nx+1] float64
    by: np.ndarray      # [nz][ny+1][nx] float64
    bz: np.ndarray      # [nz+1][ny][nx] float64
    b: np.ndarray       # [nz][ny][nx] float64 (not projected)
    info: dict

    @property
    def cells(self) -> int:
        nx, ny, nz = self.n
        return nx * ny * nz


def smoothed_heaviside(phi: np.ndarray, eps: float) -> np.ndarray:
    """0 for phi < -eps, 1 for phi > eps, 1/2 (1 + phi/eps + sin(pi phi/eps)/pi) between."""
    x = np.clip(phi / eps, -1.0, 1.0)
    return 0.5 * (1.0 + x + np.sin(np.pi * x) / np.pi)


def cell_centres(n: int) -> np.ndarray:
    h = 1.0 / n
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def faces_from_alpha(alpha: np.ndarray, faces: str = "arith"):
    """Face coefficients from cell values alpha (walls 0).

    ``arith``: (alpha_L + alpha_R)/2.  ``harmonic``: 2 alpha_L alpha_R/(alpha_L+alpha_R),
    the harmonic estimate of eqs. (11)-(12)."""
    nz, ny, nx = alpha.shape

    def mean(l, r):
        if faces == "arith":
            return 0.5 * (l + r)
        if faces == "harmonic":
            return 2.0 * l * r / (l + r)
        raise ValueError(f"unknown face averaging {faces!r}")

    bx = np.zeros((nz, ny, nx + 1))
    by = np.zeros((nz, ny + 1, nx))
    bz = np.zeros((nz + 1, ny, nx))
    bx[:, :, 1:nx] = mean(alpha[:, :, :-1], alpha[:, :, 1:])
    by[:, 1:ny, :] = mean(alpha[:, :-1, :], alpha[:, 1:, :])
    bz[1:nz, :, :] = mean(alpha[:-1, :, :], alpha[1:, :, :])
    return bx, by, bz


def normal_rhs(n, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) per cell (not projected; the solver removes the mean)."""
    nx, ny, nz = n
    return np.random.default_rng(seed).standard_normal((nz, ny, nx))


def divergence_rhs(n, rng: np.random.Generator) -> np.ndarray:
    """Discrete divergence of a random face velocity field.

    Interior face velocities are i.i.d. N(0,1), drawn x-faces first, then y, then
    z, each in C order over the interior faces only; wall velocities are 0 (no
    penetration), so the result sums to zero exactly up to rounding.
    b_c = (u_x[i+1]-u_x[i]) + (u_y[j+1]-u_y[j]) + (u_z[k+1]-u_z[k])."""
    nx, ny, nz = n
    b = np.zeros((nz, ny, nx))
    ux = np.zeros((nz, ny, nx + 1))
    ux[:, :, 1:nx] = rng.standard_normal((nz, ny, nx - 1))
    b += ux[:, :, 1:] - ux[:, :, :-1]
    del ux
    uy = np.zeros((nz, ny + 1, nx))
    uy[:, 1:ny, :] = rng.standard_normal((nz, ny - 1, nx))
    b += uy[:, 1:, :] - uy[:, :-1, :]
    del uy
    uz = np.zeros((nz + 1, ny, nx))
    uz[1:nz, :, :] = rng.standard_normal((nz - 1, ny, nx))
    b += uz[1:, :, :] - uz[:-1, :, :]
    return b


def velocity_field(n, rng: np.random.Generator, walls: bool = False):
    """Random face velocity (u on x-faces, v on y-faces, w on z-faces) for the
    projection step.

    Interior faces are i.i.d. N(0,1), drawn x-faces first, then y, then z, each in
    C order over the interior faces only (the same draws as ``divergence_rhs``).
    Wall faces are 0 (no penetration) or, with ``walls``, N(0,1) drawn after the
    interior faces in the order x-lower, x-upper, y-lower, y-upper, z-lower,
    z-upper."""
    nx, ny, nz = n
    u = np.zeros((nz, ny, nx + 1))
    v = np.zeros((nz, ny + 1, nx))
    w = np.zeros((nz + 1, ny, nx))
    u[:, :, 1:nx] = rng.standard_normal((nz, ny, nx - 1))
    v[:, 1:ny, :] = rng.standard_normal((nz, ny - 1, nx))
    w[1:nz, :, :] = rng.standard_normal((nz - 1, ny, nx))
    if walls:
        u[:, :, 0] = rng.standard_normal((nz, ny))
        u[:, :, nx] = rng.standard_normal((nz, ny))
        v[:, 0, :] = rng.standard_normal((nz, nx))
        v[:, ny, :] = rng.standard_normal((nz, nx))
        w[0] = rng.standard_normal((ny, nx))
        w[nz] = rng.standard_normal((ny, nx))
    return u, v, w


def _alpha_from_phi_planes(n, phi_plane, rho_l, rho_g, chunk=16):
    """alpha = 1/rho on the grid, rho from eq. (8) with the smoothed indicator.

    ``phi_plane(z_centres)`` returns the signed distance (positive in liquid) for a
    chunk of z planes, shape [len(z)][ny][nx]."""
    nx, ny, nz = n
    h = 1.0 / nx
    eps = 1.5 * h
    zc = cell_centres(nz)
    alpha = np.empty((nz, ny, nx))
    for k0 in range(0, nz, chunk):
        phi = phi_plane(zc[k0:k0 + chunk])
        ind = smoothed_heaviside(phi, eps)
        rho = rho_g + (rho_l - rho_g) * ind
        alpha[k0:k0 + chunk] = 1.0 / rho
    return alpha


def _geometry_phi(n, drops, film):
    """Signed distance of a union of spheres and a bottom film (max of the parts).

    drops: list of (cx, cy, cz, r); film: None, a float depth, or an array
    eta[ny][nx] of local film heights."""
    nx, ny, nz = n
    xc = cell_centres(nx)[None, None, :]
    yc = cell_centres(ny)[None, :, None]

    def phi_plane(z):
        z = z[:, None, None]
        phi = np.full((z.shape[0], ny, nx), -np.inf)
        if film is not None:
            eta = film if np.ndim(film) == 0 else film[None, :, :]
            phi = np.maximum(phi, eta - z)
        for (cx, cy, cz, r) in drops:
            d = np.sqrt((xc - cx) ** 2 + (yc - cy) ** 2 + (z - cz) ** 2)
            phi = np.maximum(phi, r - d)
        return phi

    return phi_plane


def sphere_problem(n=32, radius=0.2, centre=(0.5, 0.5, 0.5), rho_l=1000.0,
                   rho_g=1.0, seed=0, faces="arith") -> Problem:
    """A liquid sphere in gas, N(0,1) right-hand side (the small-grid workload)."""
    dims = (n, n, n)
    phi = _geometry_phi(dims, [(*centre, radius)], None)
    alpha = _alpha_from_phi_planes(dims, phi, rho_l, rho_g)
    bx, by, bz = faces_from_alpha(alpha, faces)
    b = normal_rhs(dims, seed)
    return Problem(dims, bx, by, bz, b,
                   dict(kind="sphere", n=n, radius=radius, ratio=rho_l / rho_g, seed=seed))


def drop_splash_problem(n=256, film_depth=0.1, drop=(0.5, 0.5, 0.2, 0.08),
                        rho_l=1000.0, rho_g=1.0, seed=1, perturb=False,
                        faces="arith") -> Problem:
    """Film of depth ``film_depth`` plus a drop above it; divergence right-hand side.

    With ``perturb`` the film height is 0.1 + 0.01 P/max|P|, P a sum of
    cos(m pi x) cos(n pi y) modes, m,n = 1..8, with N(0,1) amplitudes drawn first
    from the same generator as the velocities."""
    dims = (n, n, n)
    rng = np.random.default_rng(seed)
    film = film_depth
    if perturb:
        c = rng.standard_normal((8, 8))
        xc = cell_centres(n)
        m = np.arange(1, 9)
        cx = np.cos(np.pi * m[:, None] * xc[None, :])      # [m][x]
        # P[y][x] = sum_{m,n} c[m,n] cos(m pi x) cos(n pi y)
        P = np.einsum("mn,mx,ny->yx", c, cx, cx)
        film = film_depth + 0.01 * P / np.max(np.abs(P))
    phi = _geometry_phi(dims, [drop], film)
    alpha = _alpha_from_phi_planes(dims, phi, rho_l, rho_g)
    bx, by, bz = faces_from_alpha(alpha, faces)
    del alpha
    b = divergence_rhs(dims, rng)
    return Problem(dims, bx, by, bz, b,
                   dict(kind="drop_splash", n=n, film=film_depth, drop=drop,
                        ratio=rho_l / rho_g, seed=seed, perturbed=perturb))


def drop_splash_levelset(n=256, film_depth=0.1, drop=(0.5, 0.5, 0.2, 0.08), seed=1, perturb=False):
    """The level set phi (signed distance, positive in the liquid) of the drop-splash
    scene of ``drop_splash_problem`` with the same arguments (the same Fourier draws
    when ``perturb``), as one [nz][ny][nx] array, for building the properties on
    the device."""
    dims = (n, n, n) if np.ndim(n) == 0 else tuple(n)
    rng = np.random.default_rng(seed)
    film = film_depth
    if perturb:
        c = rng.standard_normal((8, 8))
        xc = cell_centres(dims[0])
        yc = cell_centres(dims[1])
        m = np.arange(1, 9)
        P = np.einsum("mn,mx,ny->yx", c, np.cos(np.pi * m[:, None] * xc[None, :]),
                      np.cos(np.pi * m[:, None] * yc[None, :]))
        film = film_depth + 0.01 * P / np.max(np.abs(P))
    return _geometry_phi(dims, [drop], film)(cell_centres(dims[2]))


def config0() -> Problem:
    """32^3 sphere r=0.2, ratio 1000, N(0,1) rhs, seed 0."""
    return sphere_problem(32, 0.2, (0.5, 0.5, 0.5), 1000.0, 1.0, seed=0)


def config1(n=256) -> Problem:
    """256^3 film d=0.1 plus drop r=0.08 at (0.5,0.5,0.2), ratio 1000, divergence rhs, seed 1."""
    return drop_splash_problem(n, 0.1, (0.5, 0.5, 0.2, 0.08), 1000.0, 1.0, seed=1)


def config2(n=512) -> Problem:
    """512^3 drop splash with a Fourier-perturbed film, seed 2."""
    return drop_splash_problem(n, 0.1, (0.5, 0.5, 0.2, 0.08), 1000.0, 1.0, seed=2,
                               perturb=True)


def _random_scene(rng, n):
    ndrops = int(rng.integers(1, 9))
    depth = float(rng.uniform(0.05, 0.2))
    ratio = float(rng.choice([10.0, 100.0, 1000.0]))
    drops = []
    for _ in range(ndrops):
        r = float(rng.uniform(0.05, 0.2))
        x = float(rng.uniform(r, 1.0 - r))
        y = float(rng.uniform(r, 1.0 - r))
        z = float(rng.uniform(depth + r, 1.0 - r))
        drops.append((x, y, z, r))
    return depth, ratio, drops


def scene_problem(n, depth, ratio, drops, rhs_seed, faces="arith") -> Problem:
    dims = (n, n, n)
    phi = _geometry_phi(dims, drops, depth)
    alpha = _alpha_from_phi_planes(dims, phi, ratio, 1.0)
    bx, by, bz = faces_from_alpha(alpha, faces)
    b = normal_rhs(dims, rhs_seed)
    return Problem(dims, bx, by, bz, b,
                   dict(kind="scene", n=n, film=depth, drops=drops, ratio=ratio,
                        seed=rhs_seed))


def scene_levelset(desc):
    """The level set phi [n][n][n] (signed distance of the union of the film and the
    drops, positive in the liquid) of a scene description from ``batch_problems``
    or ``request_stream``, for building its properties on the device; with the
    half-width 1.5/n and the description's density ratio it gives the faces of
    ``problem_from_desc(desc)``."""
    n = desc["n"]
    return _geometry_phi((n, n, n), desc["drops"], desc["film"])(cell_centres(n))


def batch_problems(count=64, sizes=(32, 64, 96, 128), seed=3, rhs_seed0=3000,
                   build=True):
    """Uneven batch: sizes, drop count, radii, centres, film depth and density
    ratio drawn from ``seed``; problem i's N(0,1) rhs from ``rhs_seed0 + i``.
    With ``build=False`` only the scene descriptions are returned."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        depth, ratio, drops = _random_scene(rng, n)
        desc = dict(n=n, film=depth, ratio=ratio, drops=drops, seed=rhs_seed0 + i)
        out.append(scene_problem(n, depth, ratio, drops, rhs_seed0 + i) if build else desc)
    return out


def request_stream(count, rate, sizes=(64, 128, 192, 256), seed=4, rhs_seed0=4000):
    """Open-loop Poisson arrivals: (arrival time, scene description) per request."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        depth, ratio, drops = _random_scene(rng, n)
        out.append((float(t[i]), dict(n=n, film=depth, ratio=ratio, drops=drops,
                                      seed=rhs_seed0 + i)))
    return out


def layered_problem(n, seed=7, ratio=1000.0, depth=0.3) -> Problem:
    """Coefficients and rhs that depend on z only (a flat film, no drop).

    The exact solution then depends on z only and solves a 1-D tridiagonal
    Neumann problem with the z-face weights."""
    nx = ny = nz = n
    dims = (n, n, n)
    phi = _geometry_phi(dims, [], depth)
    alpha = _alpha_from_phi_planes(dims, phi, ratio, 1.0)
    bx, by, bz = faces_from_alpha(alpha, "arith")
    bz1 = np.random.default_rng(seed).standard_normal(nz)
    b = np.broadcast_to(bz1[:, None, None], (nz, ny, nx)).copy()
    return Problem(dims, bx, by, bz, b, dict(kind="layered", n=n, ratio=ratio, seed=seed))


def layered_profile(n, seed=7, ratio=1000.0, depth=0.3):
    """The z profiles of ``layered_problem(n, ...)`` without the 3-D arrays, for
    grids too large to build on the host: (alpha per layer [n], z-faces [n+1] with
    walls 0, rhs per layer [n]).  Broadcasting them (x- and y-faces equal to the
    layer's alpha, the arithmetic mean of two equal values) reproduces
    ``layered_problem`` value for value."""
    zc = cell_centres(n)
    ind = smoothed_heaviside(depth - zc, 1.5 / n)
    alpha = 1.0 / (1.0 + (ratio - 1.0) * ind)
    bz = np.zeros(n + 1)
    bz[1:n] = 0.5 * (alpha[:-1] + alpha[1:])
    b = np.random.default_rng(seed).standard_normal(n)
    return alpha, bz, b


def constant_problem(n, seed=8, beta=1.0) -> Problem:
    """Constant interior coefficient beta, N(0,1) rhs (DCT-diagonalisable)."""
    dims = (n, n, n)
    alpha = np.full((n, n, n), beta)
    bx, by, bz = faces_from_alpha(alpha, "arith")
    return Problem(dims, bx, by, bz, normal_rhs(dims, seed),
                   dict(kind="constant", n=n, beta=beta, seed=seed))


def problem_from_desc(desc) -> Problem:
    return scene_problem(desc["n"], desc["film"], desc["ratio"], desc["drops"], desc["seed"])


def footprint_cells(n) -> int:
    return int(n) ** 3 if np.ndim(n) == 0 else int(math.prod(n))
