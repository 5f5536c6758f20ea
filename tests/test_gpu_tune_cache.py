"""The smoother tuner's cache file (MG_TUNE_CACHE): choices are written with the
variant count, read back by a later process, and entries written for another
variant list are ignored.  Each process runs in a child of the test (the cache is
loaded once per process)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_1410_8568_amd import mg, inputs
P = inputs.config0()
dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
S = mg.Solver(dev(P.bx), dev(P.by), dev(P.bz))
print(json.dumps(S.tiles()), flush=True)
S.close()
"""


def run_child(cache):
    env = dict(os.environ, MG_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_tune_cache_round_trip(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_8568_amd import mg
    cache = tmp_path / "tune.jsonl"
    first = run_child(cache)
    lines = [json.loads(ln) for ln in cache.read_text().splitlines() if ln.strip()]
    assert len(lines) >= 1 and all(e["variants"] == mg.MG_NUM_TILES for e in lines)
    assert all(-1 <= e["variant"] <= mg.MG_NUM_TILES and e["variant"] != 0 for e in lines)
    assert first[:len(lines)] == [e["variant"] for e in lines]
    # force a valid two-sweep variant, then add entries of an older list for the
    # same grids (later lines win, so they would override if they were read)
    forced = 13
    out = [json.dumps(dict(e, variant=forced, restrict=0)) for e in lines]
    out += [json.dumps({k: e[k] for k in ("bytes", "nx", "ny", "nz")} | {"variant": 1, "restrict": 0})
            for e in lines]
    cache.write_text("\n".join(out) + "\n")
    second = run_child(cache)
    assert second[:len(lines)] == [forced] * len(lines)
