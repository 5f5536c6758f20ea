"""CPU checks of the C ABI: the library loads and exports every declared function,
and the pure host entry points validate their arguments (no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(mg_[A-Za-z0-9_]+)\s*\(", src,
                            flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1410_8568_amd import mg
    L = mg.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/*.h but not exported"
    assert sorted(mg.EXPORTS) == sorted(names)


def test_workspace_bytes_and_validation():
    from paper_1410_8568_amd import mg
    o = mg.options()
    w32 = mg.workspace_bytes((32, 32, 32), o)
    w64 = mg.workspace_bytes((64, 64, 64), o)
    assert 40 * 32 ** 3 < w32 < 90 * 32 ** 3
    assert 7.0 < w64 / w32 < 9.0
    r = mg.options(precision="fp32_refined")
    assert mg.workspace_bytes((64, 64, 64), r) > w64 * 0.8
    for bad in [(1, 8, 8), (9, 9, 9), (0, 0, 0)]:
        with pytest.raises(mg.MGError) as ei:
            mg.workspace_bytes(bad, o)
        assert ei.value.status == mg.MG_E_INVALID
    o2 = mg.options(max_cycles=0)
    with pytest.raises(mg.MGError):
        mg.workspace_bytes((8, 8, 8), o2)


def test_status_strings_and_null_handles():
    from paper_1410_8568_amd import mg
    L = mg.lib()
    assert L.mg_status_string(mg.MG_OK) == b"MG_OK"
    assert b"BUDGET" in L.mg_status_string(mg.MG_E_BUDGET)
    assert L.mg_solve(None, None, None, ctypes.c_double(1e-10), None, None) == mg.MG_E_INVALID
    assert L.mg_level_dims(None, 0, None, None, None) == mg.MG_E_INVALID
    L.mg_destroy(None)
    L.mg_server_destroy(None)
    assert L.mg_default_options(None) == mg.MG_E_INVALID


def test_new_option_validation_on_the_host():
    """Krylov and cycle-variant options are checked by the workspace planner
    (no device call)."""
    from paper_1410_8568_amd import mg
    n = (32, 32, 32)
    base = mg.workspace_bytes(n, mg.options())
    # the Krylov solve keeps four more FP64 vectors on the finest level
    assert mg.workspace_bytes(n, mg.options(krylov="fcg")) - base >= 32 * 32 ** 3
    for kw in (dict(precision="fp32_refined", krylov="fcg"), dict(omega=0.0), dict(omega=2.0),
               dict(coarse_gmres=mg_max_m() + 1), dict(coarse_gmres=-1), dict(coarse_gmres=4, coarse_gmres_tol=0.0),
               dict(coarse_gmres=4, coarse_gmres_maxit=0)):
        with pytest.raises(mg.MGError) as ei:
            mg.workspace_bytes(n, mg.options(**kw))
        assert ei.value.status == mg.MG_E_INVALID, kw
    o = mg.options()
    o.krylov = 2
    with pytest.raises(mg.MGError):
        mg.workspace_bytes(n, o)
    for kw in (dict(omega=1.3), dict(restrict64=True), dict(coarse_gmres=16), dict(krylov="fcg", omega=1.2)):
        assert mg.workspace_bytes(n, mg.options(**kw)) > 0


def mg_max_m():
    import re
    src = open(os.path.join(ROOT, "include", "mg.h")).read()
    return int(re.search(r"#define MG_GMRES_MAX_M (\d+)", src).group(1))


def test_new_entry_points_reject_bad_arguments_without_a_device():
    from paper_1410_8568_amd import mg
    L = mg.lib()
    d = ctypes.c_double
    g = mg.Grid(4, 4, 4)
    assert L.mg_divergence(None, None, None, None, d(1.0), None, None) == mg.MG_E_INVALID
    assert L.mg_divergence(ctypes.byref(mg.Grid(-1, 4, 4)), None, None, None, d(1.0), None, None) == mg.MG_E_INVALID
    # an empty grid is a no-op (nothing is launched, no array is touched)
    assert L.mg_divergence(ctypes.byref(mg.Grid(0, 4, 4)), None, None, None, d(1.0), None, None) == mg.MG_OK
    assert L.mg_correct_velocity(None, None, d(1.0), None, None, None, None) == mg.MG_E_INVALID
    assert L.mg_project(None, None, None, None, d(0.1), d(0.1), None, None, d(1e-10), None, None) == mg.MG_E_INVALID
    assert L.mg_faces_from_levelset(None, None, d(1.0), d(1.0), d(0.1), 0, None, None, None, None) == mg.MG_E_INVALID
    fake = ctypes.c_void_p(256)   # never dereferenced: the arguments are rejected first
    for rho_l, rho_g, eps, harm in ((0.0, 1.0, 0.1, 0), (1.0, -1.0, 0.1, 0), (1.0, 1.0, 0.0, 0), (1.0, 1.0, 0.1, 2)):
        assert L.mg_faces_from_levelset(ctypes.byref(g), fake, d(rho_l), d(rho_g), d(eps), harm, fake, fake, fake,
                                        None) == mg.MG_E_INVALID


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_traffic_figure_is_tied_to_workload_and_kernel_code(tmp_path, monkeypatch):
    """The committed HBM-traffic figure is reported only for the grid size and
    kernel code it was measured on; comments do not count as code."""
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.h"
    src.write_text("// a kernel\nint f() { return 1; }   // trailing note\n/* block\n comment */\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.h"])
    sha = bench.kernel_source_sha()
    tf = tmp_path / "traffic.json"
    tf.write_text(json.dumps({"class": "smooth_fine", "n": 512, "bytes_per_launch": 3.0e9, "source_sha": sha}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tf))
    assert bench.traffic_for("smooth_fine", 512) == 3.0e9
    assert bench.traffic_for("smooth_fine", 1024) is None
    assert bench.traffic_for("other_kernel", 512) is None
    src.write_text("// reworded\nint f() { return 1; }\n")
    assert bench.traffic_for("smooth_fine", 512) == 3.0e9
    src.write_text("int f() { return 2; }\n")
    assert bench.traffic_for("smooth_fine", 512) is None
    # one entry per grid size
    sha = bench.kernel_source_sha()
    tf.write_text(json.dumps({"entries": [
        {"class": "smooth_fine", "n": 512, "bytes_per_launch": 3.0e9, "source_sha": sha},
        {"class": "smooth_fine", "n": 1024, "bytes_per_launch": 2.4e10, "source_sha": sha}]}))
    assert bench.traffic_for("smooth_fine", 512) == 3.0e9
    assert bench.traffic_for("smooth_fine", 1024) == 2.4e10
    assert bench.traffic_for("smooth_fine", 256) is None


def test_static_solve_refuses_before_any_device_call():
    """mg_solve_static validates on the host first: null arrays, a bad bc, an
    unaligned p, and a grid whose workspace exceeds the static array (160^3 in
    FP32-refined mode) are refused without touching the device (the pointers
    below are never dereferenced)."""
    from paper_1410_8568_amd import mg
    L = mg.lib()
    fake = ctypes.c_void_p(1 << 20)
    st = mg.Stats()

    def call(n, opts, bc=mg.MG_BC_NEUMANN, p=fake):
        return L.mg_solve_static(ctypes.byref(mg.Grid(*n)), ctypes.byref(opts), fake, fake, fake, bc, fake, p,
                                 ctypes.c_double(1e-10), ctypes.byref(st), None)

    o = mg.options(precision="fp32_refined")
    assert L.mg_solve_static(None, None, None, None, None, 0, None, None, ctypes.c_double(1e-10), None,
                             None) == mg.MG_E_INVALID
    assert call((32, 32, 32), o, bc=7) == mg.MG_E_INVALID
    assert call((32, 32, 32), o, p=ctypes.c_void_p((1 << 20) + 8)) == mg.MG_E_INVALID
    assert mg.workspace_bytes((160, 160, 160), o) > mg.MG_STATIC_WORKSPACE_BYTES
    assert call((160, 160, 160), o) == mg.MG_E_WORKSPACE
    assert b"static workspace" in L.mg_last_error()
    for n in ((128, 128, 128),):
        for prec in ("fp64", "fp32_refined"):
            assert mg.workspace_bytes(n, mg.options(precision=prec, n_coarsest=8)) <= mg.MG_STATIC_WORKSPACE_BYTES


def test_server_request_bytes_is_workspace_plus_a_copy_of_p():
    from paper_1410_8568_amd import mg
    for n in ((32, 32, 32), (40, 24, 12), (64, 64, 64)):
        for prec in ("fp64", "fp32_refined"):
            o = mg.options(precision=prec)
            w = mg.workspace_bytes(n, o)
            r = mg.server_request_bytes(n, o)
            cells = n[0] * n[1] * n[2]
            assert w + 8 * cells <= r <= w + 8 * cells + 512 and r % 256 == 0
    with pytest.raises(mg.MGError):
        mg.server_request_bytes((9, 9, 9), mg.options())
    assert mg.lib().mg_server_stats(None, None) == mg.MG_E_INVALID
