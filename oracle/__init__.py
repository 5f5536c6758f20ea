"""FP64 CPU oracle for the multigrid pressure solve (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never calls it.  The C source
(``mg_oracle.c`` + ``mg_ops.inc``) is a plain, unoptimised transcription of the
method of Sec. 2.3 of the paper (features 1-6, eqs. 10-15); this module only
marshals numpy arrays into it.

Parity pins for every function live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_mg.so")
SOURCES = [os.path.join(HERE, "mg_oracle.c"), os.path.join(HERE, "mg_ops.inc")]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP, no FMA contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-D_POSIX_C_SOURCE=200809L", "-o", tmp, SOURCES[0], "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


class OgOpts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("n_coarsest", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_m", ctypes.c_int), ("tol", ctypes.c_double), ("krylov", ctypes.c_int),
                ("omega", ctypes.c_double), ("restrict64", ctypes.c_int), ("gmres_m", ctypes.c_int),
                ("gmres_tol", ctypes.c_double), ("gmres_maxit", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        i = ctypes.c_int
        L.og_plan.argtypes = [i, i, i, i, _I]
        L.og_plan.restype = i
        L.og_apply.argtypes = [i, i, i, _D, _D, _D, _D, _D]
        L.og_residual.argtypes = [i, i, i, _D, _D, _D, _D, _D, _D]
        L.og_rb_half.argtypes = [i, i, i, _D, _D, _D, _D, _D, i]
        L.og_restrict.argtypes = [i, i, i, _D, _D]
        L.og_restrict64.argtypes = [i, i, i, _D, _D]
        L.og_rb_half_sor.argtypes = [i, i, i, _D, _D, _D, _D, _D, i, ctypes.c_double]
        L.og_gmres.argtypes = [i, i, i, _D, _D, _D, _D, _D, i, ctypes.c_double, i, _D]
        L.og_gmres.restype = i
        L.og_prolong_add.argtypes = [i, i, i, _D, _D, _D]
        L.og_coarsen_faces.argtypes = [i, i, i, _D, _D, _D, _D, _D, _D]
        L.og_cell_weights.argtypes = [i, i, i, _D, _D, _D, _D]
        L.og_dense_solve.argtypes = [i, i, i, _D, _D, _D, _D, _D]
        L.og_dense_solve.restype = i
        L.og_hierarchy_level.argtypes = [i, i, i, _D, _D, _D, i, i, _D, _D, _D, _D]
        L.og_hierarchy_level.restype = i
        L.og_solve.argtypes = [i, i, i, _D, _D, _D, _D, _D, ctypes.POINTER(OgOpts), _D, _I, _D, _D]
        L.og_solve.restype = i
        L.og_divergence.argtypes = [i, i, i, _D, _D, _D, ctypes.c_double, _D]
        L.og_correct_velocity.argtypes = [i, i, i, _D, _D, _D, _D, ctypes.c_double, _D, _D, _D]
        L.og_faces_from_levelset.argtypes = [i, i, i, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, i,
                                             _D, _D, _D]
        L.og_num_threads.restype = i
        L.og_last_timing.argtypes = [_D, _D]
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def dims_of(b):
    nz, ny, nx = b.shape
    return nx, ny, nz


def plan(n, n_coarsest):
    nx, ny, nz = n
    out = (ctypes.c_int * 72)()
    L = lib().og_plan(nx, ny, nz, n_coarsest, out)
    return [tuple(out[3 * l:3 * l + 3]) for l in range(L)]


def apply(bx, by, bz, p):
    p = _c(p)
    nx, ny, nz = dims_of(p)
    out = np.empty_like(p)
    bx, by, bz = _c(bx), _c(by), _c(bz)
    lib().og_apply(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(p), _p(out))
    return out


def residual(bx, by, bz, p, b):
    p, b = _c(p), _c(b)
    nx, ny, nz = dims_of(p)
    r = np.empty_like(p)
    bx, by, bz = _c(bx), _c(by), _c(bz)
    lib().og_residual(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(p), _p(b), _p(r))
    return r


def rb_half(bx, by, bz, p, b, colour):
    p = _c(p).copy()
    b = _c(b)
    nx, ny, nz = dims_of(p)
    bx, by, bz = _c(bx), _c(by), _c(bz)
    lib().og_rb_half(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(p), _p(b), int(colour))
    return p


def rb_half_sor(bx, by, bz, p, b, colour, omega):
    """One SOR half-sweep with factor omega over one colour (feature 5)."""
    p = _c(p).copy()
    b = _c(b)
    nx, ny, nz = dims_of(p)
    bx, by, bz = _c(bx), _c(by), _c(bz)
    lib().og_rb_half_sor(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(p), _p(b), int(colour), float(omega))
    return p


def restrict64(r):
    """64-point restriction: the transpose of trilinear interpolation, times 4."""
    r = _c(r)
    nx, ny, nz = dims_of(r)
    rc = np.empty((nz // 2, ny // 2, nx // 2))
    lib().og_restrict64(nx, ny, nz, _p(r), _p(rc))
    return rc


def gmres(bx, by, bz, rhs, m=16, tol=1e-10, maxit=1000):
    """Restarted GMRES(m) for L e = rhs - mean(rhs) from 0 (feature 6's coarse
    solver).  Returns (mean-zero e, iterations, final relative residual)."""
    rhs = _c(rhs)
    nx, ny, nz = dims_of(rhs)
    e = np.empty_like(rhs)
    rr = ctypes.c_double(0)
    bx, by, bz = _c(bx), _c(by), _c(bz)
    it = lib().og_gmres(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(rhs), _p(e), int(m), float(tol), int(maxit),
                        ctypes.byref(rr))
    return e, it, rr.value


def restrict(r):
    r = _c(r)
    nx, ny, nz = dims_of(r)
    rc = np.empty((nz // 2, ny // 2, nx // 2))
    lib().og_restrict(nx, ny, nz, _p(r), _p(rc))
    return rc


def prolong_add(a, ec, ef):
    a, ec = _c(a), _c(ec)
    ef = _c(ef).copy()
    cnx, cny, cnz = dims_of(ec)
    assert ef.shape == (2 * cnz, 2 * cny, 2 * cnx)
    lib().og_prolong_add(cnx, cny, cnz, _p(a), _p(ec), _p(ef))
    return ef


def coarsen_faces(bx, by, bz):
    bx, by, bz = _c(bx), _c(by), _c(bz)
    nz, ny, nxp = bx.shape
    nx = nxp - 1
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    cbx = np.empty((cz, cy, cx + 1))
    cby = np.empty((cz, cy + 1, cx))
    cbz = np.empty((cz + 1, cy, cx))
    lib().og_coarsen_faces(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(cbx), _p(cby), _p(cbz))
    return cbx, cby, cbz


def cell_weights(bx, by, bz):
    bx, by, bz = _c(bx), _c(by), _c(bz)
    nz, ny, nxp = bx.shape
    a = np.empty((nz, ny, nxp - 1))
    lib().og_cell_weights(nxp - 1, ny, nz, _p(bx), _p(by), _p(bz), _p(a))
    return a


def dense_solve(bx, by, bz, rhs):
    rhs = _c(rhs)
    nx, ny, nz = dims_of(rhs)
    e = np.empty_like(rhs)
    bx, by, bz = _c(bx), _c(by), _c(bz)
    rc = lib().og_dense_solve(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(rhs), _p(e))
    if rc != 0:
        raise ValueError("coarse operator is not positive definite")
    return e


def hierarchy_level(bx, by, bz, n_coarsest, level):
    """Faces and cell weights of hierarchy level ``level``."""
    bx, by, bz = _c(bx), _c(by), _c(bz)
    nz, ny, nxp = bx.shape
    n = (nxp - 1, ny, nz)
    dims = plan(n, n_coarsest)
    cx, cy, cz = dims[level]
    obx = np.empty((cz, cy, cx + 1))
    oby = np.empty((cz, cy + 1, cx))
    obz = np.empty((cz + 1, cy, cx))
    oa = np.empty((cz, cy, cx))
    rc = lib().og_hierarchy_level(n[0], n[1], n[2], _p(bx), _p(by), _p(bz), n_coarsest, level,
                                  _p(obx), _p(oby), _p(obz), _p(oa))
    if rc != 0:
        raise ValueError("bad level")
    return obx, oby, obz, oa


STATUS = {0: "converged", 1: "not_converged", 2: "diverged", -1: "invalid"}


KRYLOV = {"none": 0, "fcg": 1, "cg": 2}


def solve(bx, by, bz, b, p0=None, nu1=2, nu2=2, n_coarsest=4, max_cycles=100, tol=1e-10,
          precision="fp64", inner_m=3, krylov="none", omega=1.0, restrict64=False, gmres_m=0,
          gmres_tol=1e-3, gmres_maxit=200):
    """Run the oracle solve.  Returns dict(p, history, cycles, status, gamma, mean_b).

    krylov: "none" (V-cycle iteration), "fcg" (flexible CG preconditioned by one
    V-cycle per iteration, FP64) or "cg" (unpreconditioned CG, for the tests).
    Cycle variants: omega (SOR factor of the smoother), restrict64 (64-point
    restriction), gmres_m > 0 (coarsest grid by GMRES(gmres_m) to gmres_tol
    relative, at most gmres_maxit iterations, instead of exactly)."""
    b = _c(b)
    nx, ny, nz = dims_of(b)
    p = np.zeros_like(b) if p0 is None else _c(p0).copy()
    o = OgOpts(nu1, nu2, n_coarsest, max_cycles, {"fp64": 0, "fp32_refined": 1}[precision],
               inner_m, tol, KRYLOV[krylov], float(omega), int(bool(restrict64)), int(gmres_m),
               float(gmres_tol), int(gmres_maxit))
    hist = np.zeros(max_cycles + 1)
    ncyc = ctypes.c_int(0)
    mean_b = ctypes.c_double(0)
    gamma = ctypes.c_double(0)
    bx, by, bz = _c(bx), _c(by), _c(bz)
    rc = lib().og_solve(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(b), _p(p), ctypes.byref(o),
                        _p(hist), ctypes.byref(ncyc), ctypes.byref(mean_b), ctypes.byref(gamma))
    return dict(p=p, history=hist[:ncyc.value + 1].copy(), cycles=ncyc.value,
                status=STATUS[rc], gamma=gamma.value, mean_b=mean_b.value)


def _faces_dims(u, v, w):
    nz, ny, nxp = u.shape
    nx = nxp - 1
    assert v.shape == (nz, ny + 1, nx) and w.shape == (nz + 1, ny, nx), (u.shape, v.shape, w.shape)
    return nx, ny, nz


def divergence(u, v, w, scale):
    """Right-hand side of the projection step: b = scale * sum_d (u_d upper - u_d lower),
    scale = h / dt (Sec. 2.2 with eqs. 9-10; see og_divergence)."""
    u, v, w = _c(u), _c(v), _c(w)
    nx, ny, nz = _faces_dims(u, v, w)
    b = np.empty((nz, ny, nx))
    lib().og_divergence(nx, ny, nz, _p(u), _p(v), _p(w), float(scale), _p(b))
    return b


def correct_velocity(bx, by, bz, p, u, v, w, scale):
    """Projected velocity (new arrays): every interior face f between c- and c+ gets
    u_f - scale * beta_f * (p(c+) - p(c-)), scale = dt / h; wall faces are copied."""
    u, v, w = _c(u).copy(), _c(v).copy(), _c(w).copy()
    nx, ny, nz = _faces_dims(u, v, w)
    bx, by, bz, p = _c(bx), _c(by), _c(bz), _c(p)
    assert p.shape == (nz, ny, nx) and bx.shape == u.shape and by.shape == v.shape and bz.shape == w.shape
    lib().og_correct_velocity(nx, ny, nz, _p(bx), _p(by), _p(bz), _p(p), float(scale), _p(u), _p(v), _p(w))
    return u, v, w


def project(bx, by, bz, u, v, w, dt, h, tol=1e-10, **solve_kw):
    """The projection step in the paper's order: b = divergence(u*) with scale h/dt,
    the pressure solve of L p = b - mean(b), then the velocity correction with scale
    dt/h.  Returns dict(b, p, u, v, w, solve=<solve() result>)."""
    b = divergence(u, v, w, h / dt)
    res = solve(bx, by, bz, b, tol=tol, **solve_kw)
    un, vn, wn = correct_velocity(bx, by, bz, res["p"], u, v, w, dt / h)
    return dict(b=b, p=res["p"], u=un, v=vn, w=wn, solve=res)


def faces_from_levelset(phi, rho_l, rho_g, eps, faces="arith"):
    """Face coefficients (walls 0) from a level set: smoothed Heaviside of
    half-width eps -> rho (eq. 8) -> alpha = 1/rho -> arithmetic or harmonic
    (eqs. 11-12) face mean.  Returns (bx, by, bz)."""
    phi = _c(phi)
    nx, ny, nz = dims_of(phi)
    bx = np.empty((nz, ny, nx + 1)); by = np.empty((nz, ny + 1, nx)); bz = np.empty((nz + 1, ny, nx))
    lib().og_faces_from_levelset(nx, ny, nz, _p(phi), float(rho_l), float(rho_g), float(eps),
                                 {"arith": 0, "harmonic": 1}[faces], _p(bx), _p(by), _p(bz))
    return bx, by, bz


def last_timing():
    """(setup seconds, seconds after setup) of the last solve()."""
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().og_last_timing(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def num_threads() -> int:
    return lib().og_num_threads()
