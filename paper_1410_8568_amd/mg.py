"""Thin Python binding of the C ABI in ``include/mg.h`` (argument marshalling only).

torch supplies device memory (tensors -> raw pointers) and streams
(``torch.cuda.Stream`` -> hipStream_t); every step of the solve runs in the HIP
library ``libmg355x.so``.  There is no fallback: if the library is missing the
import of this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg355x.so")

MG_OK, MG_PENDING = 0, 1
MG_E_INVALID, MG_E_WORKSPACE, MG_E_HIP = -1, -2, -3
MG_E_NOT_CONVERGED, MG_E_DIVERGED, MG_E_BUDGET, MG_E_NOT_FOUND = -4, -5, -6, -7
MG_FP64, MG_FP32_REFINED = 0, 1
MG_BC_NEUMANN = 0
MG_MAX_LEVELS = 24
MG_MAX_COARSE_CELLS = 512
MG_MAX_HISTORY = 256
MG_NUM_TILES = 24
KERNEL_CLASSES = ["smooth", "restrict", "prolong", "coarse", "norm", "refine", "other", "smooth_fine", "krylov"]
MG_KRYLOV_NONE, MG_KRYLOV_FCG = 0, 1
MG_K_COUNT = len(KERNEL_CLASSES)

# every function declared in include/mg.h
EXPORTS = [
    "mg_default_options", "mg_workspace_bytes", "mg_setup", "mg_solve", "mg_destroy",
    "mg_level_dims", "mg_level_tile", "mg_copy_level", "mg_server_create", "mg_batch_submit", "mg_poll",
    "mg_server_destroy", "mg_status_string", "mg_last_error", "mg_divergence", "mg_correct_velocity",
    "mg_project", "mg_faces_from_levelset", "mg_solve_static", "mg_server_request_bytes", "mg_server_stats",
]
MG_STATIC_WORKSPACE_BYTES = 160 * 1024 * 1024


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("n_coarsest", ctypes.c_int), ("inner_m", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("profile", ctypes.c_int), ("tile", ctypes.c_int),
                ("graph", ctypes.c_int), ("krylov", ctypes.c_int), ("omega", ctypes.c_double),
                ("restrict64", ctypes.c_int), ("coarse_gmres", ctypes.c_int), ("coarse_gmres_maxit", ctypes.c_int),
                ("coarse_gmres_tol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("levels", ctypes.c_int), ("cycles", ctypes.c_int),
                ("outer", ctypes.c_int), ("nhist", ctypes.c_int),
                ("history", ctypes.c_double * MG_MAX_HISTORY),
                ("rel_residual", ctypes.c_double), ("gamma", ctypes.c_double),
                ("mean_b", ctypes.c_double), ("norm_b", ctypes.c_double),
                ("solve_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double * MG_K_COUNT),
                ("kernel_launches", ctypes.c_longlong * MG_K_COUNT),
                ("kernel_bytes", ctypes.c_double * MG_K_COUNT)]

    def to_dict(self):
        return dict(
            status=self.status, levels=self.levels, cycles=self.cycles, outer=self.outer,
            history=list(self.history[:self.nhist]), rel_residual=self.rel_residual,
            gamma=self.gamma, mean_b=self.mean_b, norm_b=self.norm_b, solve_ms=self.solve_ms,
            kernel_ms={k: self.kernel_ms[i] for i, k in enumerate(KERNEL_CLASSES)},
            kernel_launches={k: self.kernel_launches[i] for i, k in enumerate(KERNEL_CLASSES)},
            kernel_bytes={k: self.kernel_bytes[i] for i, k in enumerate(KERNEL_CLASSES)},
        )


class ServerOptions(ctypes.Structure):
    _fields_ = [("solver", Options), ("max_slots", ctypes.c_int), ("nstreams", ctypes.c_int),
                ("streams", ctypes.POINTER(ctypes.c_void_p))]


class Request(ctypes.Structure):
    _fields_ = [("grid", Grid), ("bx", ctypes.c_void_p), ("by", ctypes.c_void_p),
                ("bz", ctypes.c_void_p), ("rhs", ctypes.c_void_p), ("p", ctypes.c_void_p),
                ("tol", ctypes.c_double), ("stream", ctypes.c_void_p)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("classes", ctypes.c_int), ("graphs", ctypes.c_int), ("replays", ctypes.c_longlong),
                ("problem_iterations", ctypes.c_longlong), ("max_batch", ctypes.c_int), ("resident", ctypes.c_int),
                ("completed", ctypes.c_longlong)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("stats", Stats), ("submit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("finish_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libmg355x.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_1410_8568_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    L.mg_default_options.argtypes = [ctypes.POINTER(Options)]
    L.mg_workspace_bytes.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Options), ctypes.POINTER(sz)]
    L.mg_setup.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Options), vp, vp, vp, i, vp, sz, vp,
                           ctypes.POINTER(vp)]
    L.mg_solve.argtypes = [vp, vp, vp, d, ctypes.POINTER(Stats), vp]
    L.mg_destroy.argtypes = [vp]
    L.mg_destroy.restype = None
    L.mg_level_dims.argtypes = [vp, i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    L.mg_copy_level.argtypes = [vp, i, vp, vp, vp, vp, vp]
    L.mg_level_tile.argtypes = [vp, i, ctypes.POINTER(i)]
    L.mg_server_create.argtypes = [vp, sz, ctypes.POINTER(ServerOptions), ctypes.POINTER(vp)]
    L.mg_batch_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.mg_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.mg_server_request_bytes.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Options), ctypes.POINTER(sz)]
    L.mg_server_stats.argtypes = [vp, ctypes.POINTER(ServerInfo)]
    L.mg_server_destroy.argtypes = [vp]
    L.mg_server_destroy.restype = None
    L.mg_divergence.argtypes = [ctypes.POINTER(Grid), vp, vp, vp, d, vp, vp]
    L.mg_correct_velocity.argtypes = [vp, vp, d, vp, vp, vp, vp]
    L.mg_project.argtypes = [vp, vp, vp, vp, d, d, vp, vp, d, ctypes.POINTER(Stats), vp]
    L.mg_faces_from_levelset.argtypes = [ctypes.POINTER(Grid), vp, d, d, d, i, vp, vp, vp, vp]
    L.mg_solve_static.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Options), vp, vp, vp, i, vp, vp, d,
                                  ctypes.POINTER(Stats), vp]
    L.mg_status_string.argtypes = [i]
    L.mg_status_string.restype = ctypes.c_char_p
    L.mg_last_error.argtypes = []
    L.mg_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("mg_destroy", "mg_server_destroy", "mg_status_string", "mg_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class MGError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.mg_status_string(status).decode()
        detail = L.mg_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")
        self.status = status


def options(precision="fp64", nu1=2, nu2=2, n_coarsest=4, inner_m=3, max_cycles=100, profile=False,
            tile=0, graph=False, krylov="none", omega=1.0, restrict64=False, coarse_gmres=0,
            coarse_gmres_tol=1e-3, coarse_gmres_maxit=200):
    o = Options()
    lib().mg_default_options(ctypes.byref(o))
    o.precision = {"fp64": MG_FP64, "fp32_refined": MG_FP32_REFINED}[precision]
    o.nu1, o.nu2, o.n_coarsest, o.inner_m, o.max_cycles = nu1, nu2, n_coarsest, inner_m, max_cycles
    o.profile = 1 if profile else 0
    o.tile = tile
    o.graph = 1 if graph else 0
    o.krylov = {"none": MG_KRYLOV_NONE, "fcg": MG_KRYLOV_FCG}[krylov]
    o.omega = omega
    o.restrict64 = 1 if restrict64 else 0
    o.coarse_gmres = coarse_gmres
    o.coarse_gmres_tol = coarse_gmres_tol
    o.coarse_gmres_maxit = coarse_gmres_maxit
    return o


def workspace_bytes(n, opts: Options) -> int:
    g = Grid(*n)
    out = ctypes.c_size_t(0)
    st = lib().mg_workspace_bytes(ctypes.byref(g), ctypes.byref(opts), ctypes.byref(out))
    if st != MG_OK:
        raise MGError(st, "mg_workspace_bytes")
    return out.value


def server_request_bytes(n, opts: Options) -> int:
    """Arena bytes one request of grid n takes in a server with solver options opts."""
    out = ctypes.c_size_t(0)
    st = lib().mg_server_request_bytes(ctypes.byref(Grid(*n)), ctypes.byref(opts), ctypes.byref(out))
    if st != MG_OK:
        raise MGError(st, "mg_server_request_bytes")
    return out.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_field(t, shape, name):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
        raise ValueError(f"{name}: expected contiguous float64 CUDA tensor of shape {shape}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def _check_velocity(u, v, w, n):
    nx, ny, nz = n
    _check_field(u, (nz, ny, nx + 1), "u")
    _check_field(v, (nz, ny + 1, nx), "v")
    _check_field(w, (nz + 1, ny, nx), "w")


def divergence(u, v, w, scale, b=None, stream=None):
    """b = scale * (net face-velocity outflow of each cell) (scale = h/dt: the
    right-hand side of the projection step).  Asynchronous on the stream."""
    import torch
    nz, ny, nxp = u.shape
    n = (nxp - 1, ny, nz)
    _check_velocity(u, v, w, n)
    if b is None:
        b = torch.empty((nz, ny, n[0]), dtype=torch.float64, device=u.device)
    _check_field(b, (nz, ny, n[0]), "b")
    g = Grid(*n)
    rc = lib().mg_divergence(ctypes.byref(g), _ptr(u), _ptr(v), _ptr(w), ctypes.c_double(scale), _ptr(b),
                             _stream(stream))
    if rc != MG_OK:
        raise MGError(rc, "mg_divergence")
    return b


def faces_from_levelset(phi, rho_l, rho_g, eps, faces="arith", out=None, stream=None):
    """Face coefficients (bx, by, bz) from a device level set phi [nz][ny][nx]
    (positive in the liquid): smoothed Heaviside of half-width eps, density by
    eq. (8), alpha = 1/rho, arithmetic or harmonic (eqs. 11-12) face mean, walls 0.
    Asynchronous on the stream; ``out`` may supply the three face tensors."""
    import torch
    nz, ny, nx = phi.shape
    _check_field(phi, (nz, ny, nx), "phi")
    if out is None:
        out = (torch.empty((nz, ny, nx + 1), dtype=torch.float64, device=phi.device),
               torch.empty((nz, ny + 1, nx), dtype=torch.float64, device=phi.device),
               torch.empty((nz + 1, ny, nx), dtype=torch.float64, device=phi.device))
    _check_velocity(*out, (nx, ny, nz))
    g = Grid(nx, ny, nz)
    rc = lib().mg_faces_from_levelset(ctypes.byref(g), _ptr(phi), ctypes.c_double(rho_l), ctypes.c_double(rho_g),
                                      ctypes.c_double(eps), {"arith": 0, "harmonic": 1}[faces], _ptr(out[0]),
                                      _ptr(out[1]), _ptr(out[2]), _stream(stream))
    if rc != MG_OK:
        raise MGError(rc, "mg_faces_from_levelset")
    return out


def solve_static(bx, by, bz, b, p, tol=1e-10, precision="fp64", stream=None, check=True, **kw):
    """Setup and solve of one field in the library's static device workspace
    (``mg_solve_static``: no allocation by the library; grids up to 128^3).
    p is in/out as in ``Solver.solve``.  Returns the stats dict with "rc"."""
    nz, ny, nxp = bx.shape
    n = (nxp - 1, ny, nz)
    nx = n[0]
    _check_field(bx, (nz, ny, nx + 1), "bx")
    _check_field(by, (nz, ny + 1, nx), "by")
    _check_field(bz, (nz + 1, ny, nx), "bz")
    _check_field(b, (nz, ny, nx), "b")
    _check_field(p, (nz, ny, nx), "p")
    o = options(precision=precision, **kw)
    st = Stats()
    rc = lib().mg_solve_static(ctypes.byref(Grid(*n)), ctypes.byref(o), _ptr(bx), _ptr(by), _ptr(bz), MG_BC_NEUMANN,
                               _ptr(b), _ptr(p), ctypes.c_double(tol), ctypes.byref(st), _stream(stream))
    if check and rc != MG_OK:
        raise MGError(rc, "mg_solve_static")
    out = st.to_dict()
    out["rc"] = rc
    return out


class Solver:
    """One coefficient field: ``Solver(bx, by, bz)`` then ``solve(b, p)``.

    bx, by, bz: float64 device tensors [nz][ny][nx+1], [nz][ny+1][nx], [nz+1][ny][nx].
    The workspace is a torch uint8 device tensor owned by this object."""

    def __init__(self, bx, by, bz, precision="fp64", stream=None, **kw):
        import torch
        nz, ny, nxp = bx.shape
        self.n = (nxp - 1, ny, nz)
        nx = self.n[0]
        _check_field(bx, (nz, ny, nx + 1), "bx")
        _check_field(by, (nz, ny + 1, nx), "by")
        _check_field(bz, (nz + 1, ny, nx), "bz")
        self.opts = options(precision=precision, **kw)
        self.ws_bytes = workspace_bytes(self.n, self.opts)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=bx.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = stream
        h = ctypes.c_void_p()
        g = Grid(*self.n)
        st = lib().mg_setup(ctypes.byref(g), ctypes.byref(self.opts), _ptr(bx), _ptr(by), _ptr(bz),
                            MG_BC_NEUMANN, ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(self.ws_bytes),
                            _stream(stream), ctypes.byref(h))
        if st != MG_OK:
            raise MGError(st, "mg_setup")
        self.h = h

    def solve(self, b, p, tol=1e-10, check=True):
        """Solve in place into p (initial guess on entry).  Returns the stats dict."""
        nx, ny, nz = self.n
        _check_field(b, (nz, ny, nx), "b")
        _check_field(p, (nz, ny, nx), "p")
        st = Stats()
        rc = lib().mg_solve(self.h, _ptr(b), _ptr(p), ctypes.c_double(tol), ctypes.byref(st),
                            _stream(self.stream))
        if check and rc not in (MG_OK,):
            raise MGError(rc, "mg_solve")
        out = st.to_dict()
        out["rc"] = rc
        return out

    def correct_velocity(self, p, u, v, w, scale):
        """In place: u -= scale * beta * (pressure difference) on every interior face
        (scale = dt/h for the projection step).  Asynchronous on the solver's stream."""
        nx, ny, nz = self.n
        _check_field(p, (nz, ny, nx), "p")
        _check_velocity(u, v, w, self.n)
        rc = lib().mg_correct_velocity(self.h, _ptr(p), ctypes.c_double(scale), _ptr(u), _ptr(v), _ptr(w),
                                       _stream(self.stream))
        if rc != MG_OK:
            raise MGError(rc, "mg_correct_velocity")

    def project(self, u, v, w, dt, h, p=None, b=None, tol=1e-10, check=True):
        """The projection step in place on (u, v, w): right-hand side into b, pressure
        into p (both allocated if None), velocity corrected on success.  Returns the
        stats dict with the tensors under "p" and "b"."""
        import torch
        nx, ny, nz = self.n
        _check_velocity(u, v, w, self.n)
        if p is None:
            p = torch.zeros((nz, ny, nx), dtype=torch.float64, device=u.device)
        if b is None:
            b = torch.empty((nz, ny, nx), dtype=torch.float64, device=u.device)
        _check_field(p, (nz, ny, nx), "p")
        _check_field(b, (nz, ny, nx), "b")
        st = Stats()
        rc = lib().mg_project(self.h, _ptr(u), _ptr(v), _ptr(w), ctypes.c_double(dt), ctypes.c_double(h),
                              _ptr(b), _ptr(p), ctypes.c_double(tol), ctypes.byref(st), _stream(self.stream))
        if check and rc != MG_OK:
            raise MGError(rc, "mg_project")
        out = st.to_dict()
        out.update(rc=rc, p=p, b=b)
        return out

    def levels(self):
        out = []
        for l in range(MG_MAX_LEVELS):
            a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            if lib().mg_level_dims(self.h, l, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) != MG_OK:
                break
            out.append((a.value, b.value, c.value))
        return out

    def tiles(self):
        out = []
        for l in range(len(self.levels())):
            t = ctypes.c_int()
            lib().mg_level_tile(self.h, l, ctypes.byref(t))
            out.append(t.value)
        return out

    def level_arrays(self, l):
        """FP64 faces and cell weights of level l as device tensors."""
        import torch
        nx, ny, nz = self.levels()[l]
        dev = self.ws.device
        bx = torch.empty((nz, ny, nx + 1), dtype=torch.float64, device=dev)
        by = torch.empty((nz, ny + 1, nx), dtype=torch.float64, device=dev)
        bz = torch.empty((nz + 1, ny, nx), dtype=torch.float64, device=dev)
        a = torch.empty((nz, ny, nx), dtype=torch.float64, device=dev)
        st = lib().mg_copy_level(self.h, l, _ptr(bx), _ptr(by), _ptr(bz), _ptr(a), _stream(self.stream))
        if st != MG_OK:
            raise MGError(st, "mg_copy_level")
        return bx, by, bz, a

    def close(self):
        if getattr(self, "h", None):
            lib().mg_destroy(self.h)
            self.h = None
        self.ws = None   # release the workspace (the hierarchy lived in it)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server over a torch uint8 arena (the HBM budget).

    The server's device work runs on torch streams (``nstreams`` of them, default
    priority) created here and passed to the library.  ``submit`` queues a solve and
    returns a ticket; the server starts on it after the work already enqueued on the
    submitting stream (the current torch stream by default).  The caller keeps the
    request's tensors alive until ``poll`` returns a result (the binding holds
    references)."""

    def __init__(self, arena_bytes, precision="fp64", max_slots=16, device="cuda", nstreams=None, **kw):
        import torch
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=device)
        self._arena_ptr = (self.arena.data_ptr() + 255) & ~255
        n = max_slots if nstreams is None else nstreams
        self.streams = [torch.cuda.Stream(device=self.arena.device) for _ in range(n)]
        self._stream_arr = (ctypes.c_void_p * max(n, 1))(*[s.cuda_stream for s in self.streams])
        self.opts = ServerOptions(options(precision=precision, **kw), max_slots, n,
                                  ctypes.cast(self._stream_arr, ctypes.POINTER(ctypes.c_void_p)))
        h = ctypes.c_void_p()
        st = lib().mg_server_create(ctypes.c_void_p(self._arena_ptr), ctypes.c_size_t(arena_bytes),
                                    ctypes.byref(self.opts), ctypes.byref(h))
        if st != MG_OK:
            raise MGError(st, "mg_server_create")
        self.h = h
        self._keep = {}

    def submit(self, bx, by, bz, b, p, tol=1e-10, stream=None):
        nz, ny, nxp = bx.shape
        n = (nxp - 1, ny, nz)
        nx = n[0]
        _check_field(bx, (nz, ny, nx + 1), "bx")
        _check_field(by, (nz, ny + 1, nx), "by")
        _check_field(bz, (nz + 1, ny, nx), "bz")
        _check_field(b, (nz, ny, nx), "b")
        _check_field(p, (nz, ny, nx), "p")
        r = Request(Grid(*n), bx.data_ptr(), by.data_ptr(), bz.data_ptr(), b.data_ptr(), p.data_ptr(), tol,
                    _stream(stream))
        t = ctypes.c_uint64()
        st = lib().mg_batch_submit(self.h, ctypes.byref(r), ctypes.byref(t))
        if st != MG_OK:
            raise MGError(st, "mg_batch_submit")
        self._keep[t.value] = (bx, by, bz, b, p)
        return t.value

    def poll(self, ticket):
        """None while pending, else dict(rc, stats, submit_ms, start_ms, finish_ms)."""
        res = Result()
        st = lib().mg_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(res))
        if st == MG_PENDING:
            return None
        if st == MG_E_NOT_FOUND:
            raise MGError(st, "mg_poll")
        self._keep.pop(ticket, None)
        return dict(rc=st, stats=res.stats.to_dict(), submit_ms=res.submit_ms, start_ms=res.start_ms,
                    finish_ms=res.finish_ms)

    def stats(self):
        """Counters of the batched execution: classes, graphs, replays, problem_iterations,
        max_batch, resident, completed."""
        info = ServerInfo()
        st = lib().mg_server_stats(self.h, ctypes.byref(info))
        if st != MG_OK:
            raise MGError(st, "mg_server_stats")
        return {k: getattr(info, k) for k, _ in ServerInfo._fields_}

    def wait(self, ticket, timeout_s=120.0):
        import time
        t0 = time.time()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.time() - t0 > timeout_s:
                raise TimeoutError(f"ticket {ticket} not finished after {timeout_s} s")
            time.sleep(0.0002)

    def close(self):
        if getattr(self, "h", None):
            lib().mg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device(problem, device="cuda"):
    import torch
    return tuple(torch.from_numpy(a).to(device) for a in (problem.bx, problem.by, problem.bz, problem.b))
