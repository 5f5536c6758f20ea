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


def _counter_csv(d, rows):
    import csv
    d.mkdir(parents=True, exist_ok=True)
    with open(d / "bench_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_bench_traffic_pairs_the_finest_level_of_each_run(tmp_path, monkeypatch):
    """bench.py --traffic: the finest-level smoother dispatches are picked in each
    counter run by its own counter before FETCH and WRITE are paired, so a run
    whose coarser levels were tuned to another kernel (the two runs tune
    separately) pairs the same finest-level launches; tuning dispatches before
    the first residual pass are left out; the copy calibration scales KiB to
    bytes (FETCH x2, WRITE x1 here)."""
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.h"
    src.write_text("int f() { return 1; }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.h"])
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    A = "void mgk::k_rb_sweep<float, 64, 16, 2, false, false, false, false>(args)"
    B = "void mgk::k_rb_sweep<float, 64, 8, 2, false, false, false, false>(args)"
    U = "void mgk::k_rb_sweep<float, 64, 16, 2, false, false, false, true>(args)"
    R = "void mgk::k_resid_flat<1>(args)"
    # FETCH run: a tuning dispatch, then per cycle level 0 on A (and U), level 1 on A
    fetch = [(1, A, 100, 9.0e6), (2, R, 5, 1.0)]
    write = [(1, B, 100, 9.0e6), (2, R, 5, 1.0)]
    d = 3
    for cyc in range(3):
        lvl0 = U if cyc == 2 else A
        fetch += [(d, lvl0, 100, 3.0e6 + cyc), (d + 1, A, 100, 4.0e5)]
        write += [(d, lvl0, 100, 5.0e5 + cyc), (d + 1, B, 50, 6.0e4)]   # level 1 tuned to B here
        d += 2
    _counter_csv(tmp_path / "F", fetch)
    _counter_csv(tmp_path / "W", write)
    _counter_csv(tmp_path / "CF", [(1, "__amd_rocclr_copyBuffer(x)", 1, 524288.0)])
    _counter_csv(tmp_path / "CW", [(1, "__amd_rocclr_copyBuffer(x)", 1, 1048576.0)])
    bench.write_traffic(str(tmp_path / "F"), str(tmp_path / "W"), str(tmp_path / "CF"), str(tmp_path / "CW"), 512)
    e = json.load(open(tmp_path / "traffic.json"))["entries"][0]
    assert e["n"] == 512 and e["dispatches"] == 3
    kib = 1024.0
    fetch0 = [(3.0e6 + c) * kib * 2.0 for c in range(3)]
    write0 = [(5.0e5 + c) * kib for c in range(3)]
    assert abs(e["fetch_bytes"] - sum(fetch0) / 3) < 1.0
    assert abs(e["write_bytes"] - sum(write0) / 3) < 1.0
    assert abs(e["bytes_per_launch"] - (sum(fetch0) + sum(write0)) / 3) < 1.0
    assert sorted(e["kernels"]) == sorted([A.split("(")[0].replace("void mgk::", ""),
                                           U.split("(")[0].replace("void mgk::", "")])


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
