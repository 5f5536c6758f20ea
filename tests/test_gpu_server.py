"""GPU tests of the continuous-batching solve server (through the C ABI):
each request gives the same result alone (mg_solve) and in a mix with others,
requests wait for HBM budget and still all complete, and errors are reported
per request."""
import numpy as np
import pytest

import oracle
from paper_1410_8568_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problems():
    out = inputs.batch_problems(6, sizes=(32, 64, 96))
    out.append(inputs.config0())
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_mix_equals_alone(precision):
    import torch
    from paper_1410_8568_amd import mg
    probs = _problems()
    dev = [mg.to_device(P) for P in probs]
    alone = []
    for (bx, by, bz, b) in dev:
        S = mg.Solver(bx, by, bz, precision=precision)
        p = torch.zeros_like(b)
        st = S.solve(b, p, tol=1e-10)
        assert st["rc"] == 0
        alone.append((p.clone(), st))
        S.close()
    # budget for about three of the largest at once, so the mix queues for memory
    o = mg.options(precision=precision)
    need = [mg.server_request_bytes(P.n, o) for P in probs]
    srv = mg.Server(3 * max(need) + 4096, precision=precision, max_slots=4)
    outs, tickets = [], []
    for rep in range(2):
        for (bx, by, bz, b) in dev:
            p = torch.zeros_like(b)
            outs.append(p)
            tickets.append(srv.submit(bx, by, bz, b, p, tol=1e-10))
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for q, (res, p) in enumerate(zip(results, outs)):
        ref_p, ref_st = alone[q % len(dev)]
        assert res["rc"] == 0, res
        assert res["stats"]["history"] == ref_st["history"]
        assert torch.equal(p, ref_p), q
        assert res["submit_ms"] <= res["start_ms"] <= res["finish_ms"]
    # and the results are the oracle's
    for P, (p, _) in zip(probs, alone):
        ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, precision=precision)
        pn = p.cpu().numpy()
        assert np.linalg.norm(pn - ref["p"]) / np.linalg.norm(ref["p"]) <= 1e-8


def test_budget_and_errors():
    import torch
    from paper_1410_8568_amd import mg
    P = inputs.config0()
    bx, by, bz, b = mg.to_device(P)
    need = mg.server_request_bytes(P.n, mg.options())
    srv = mg.Server(need + 1024, max_slots=8)   # room for one request at a time
    with pytest.raises(mg.MGError) as ei:
        big = inputs.sphere_problem(64)
        srv.submit(*mg.to_device(big), torch.zeros(64, 64, 64, dtype=torch.float64, device="cuda"))
    assert ei.value.status == mg.MG_E_BUDGET
    bad = bx.clone()
    bad[1, 2, 3] = -1.0
    ps = [torch.zeros_like(b) for _ in range(4)]
    tk = [srv.submit(bx, by, bz, b, ps[0]), srv.submit(bad, by, bz, b, ps[1]),
          srv.submit(bx, by, bz, b, ps[2]), srv.submit(bx, by, bz, b, ps[3], tol=0.0)]
    res = [srv.wait(t) for t in tk]
    assert res[0]["rc"] == 0 and res[2]["rc"] == 0
    assert res[1]["rc"] == mg.MG_E_INVALID
    assert res[3]["rc"] == mg.MG_E_NOT_CONVERGED
    assert torch.equal(ps[0], ps[2])
    # one at a time: each started after the previous finished
    assert res[1]["start_ms"] >= res[0]["finish_ms"] - 1e-6
    with pytest.raises(mg.MGError) as ei:
        srv.poll(tk[0])
    assert ei.value.status == mg.MG_E_NOT_FOUND
    srv.close()


@pytest.mark.parametrize("nstreams", [1, 3])
def test_submit_waits_for_producer_stream(nstreams):
    """The request's rhs and initial guess are written on a busy torch stream just
    before the submit; the server (running on torch streams passed in its options,
    fewer streams than slots) must read them only after that work, so the result
    equals the alone solve bit for bit.  Reading early would see the stale guess of
    1e3 (or an unwritten rhs) and give another iterate."""
    import torch
    from paper_1410_8568_amd import mg
    probs = inputs.batch_problems(3, sizes=(32, 64))
    dev = [mg.to_device(P) for P in probs]
    alone = []
    for (bx, by, bz, b) in dev:
        S = mg.Solver(bx, by, bz, precision="fp32_refined")
        p = torch.zeros_like(b)
        st = S.solve(b, p, tol=1e-10)
        assert st["rc"] == 0
        alone.append((p.clone(), st))
        S.close()
    srv = mg.Server(1 << 30, precision="fp32_refined", max_slots=4, nstreams=nstreams)
    assert len(srv.streams) == nstreams
    prod = torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    outs, tickets = [], []
    for rep in range(2):
        for (bx, by, bz, b) in dev:
            p = torch.full_like(b, 1e3)
            bb = torch.empty_like(b)
            torch.cuda.synchronize()
            with torch.cuda.stream(prod):
                for _ in range(8):          # keep the producer stream busy for a while
                    big = (big @ big).clamp_(-1.0, 1.0)
                p.zero_()
                bb.copy_(b)
                tickets.append(srv.submit(bx, by, bz, bb, p, tol=1e-10, stream=prod))
            outs.append((p, bb))
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for q, (res, (p, _)) in enumerate(zip(results, outs)):
        ref_p, ref_st = alone[q % len(dev)]
        assert res["rc"] == 0, res
        assert res["stats"]["history"] == ref_st["history"], q
        assert torch.equal(p, ref_p), q


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_size_classes_run_batched(precision):
    """Problems of one grid size advance together: each replay of a size class's
    graph is one outer iteration of all of its resident problems, every launch
    covering all of them.  Five 32^3, six 64^3 and three 128^3 problems (uneven
    scenes, ratios 10-1000) submitted at once: every result equals its alone solve
    (mg_solve) bit for bit, matches the oracle to 1e-8, and the counters show
    replays that advanced several problems at once."""
    import torch
    from paper_1410_8568_amd import mg
    probs = (inputs.batch_problems(5, sizes=(32,), seed=51, rhs_seed0=5100)
             + inputs.batch_problems(6, sizes=(64,), seed=52, rhs_seed0=5200)
             + inputs.batch_problems(3, sizes=(128,), seed=53, rhs_seed0=5300))
    dev = [mg.to_device(P) for P in probs]
    alone = []
    for (bx, by, bz, b) in dev:
        S = mg.Solver(bx, by, bz, precision=precision)
        p = torch.zeros_like(b)
        st = S.solve(b, p, tol=1e-10)
        assert st["rc"] == 0
        alone.append((p.clone(), st))
        S.close()
    o = mg.options(precision=precision)
    arena = sum(mg.server_request_bytes(P.n, o) for P in probs) + (1 << 20)
    srv = mg.Server(arena, precision=precision, max_slots=16)
    outs = [torch.zeros_like(b) for (_, _, _, b) in dev]
    tickets = [srv.submit(bx, by, bz, b, p, tol=1e-10) for (bx, by, bz, b), p in zip(dev, outs)]
    results = [srv.wait(t) for t in tickets]
    info = srv.stats()
    srv.close()
    print(f"{precision}: {info}", flush=True)
    for q, (res, p) in enumerate(zip(results, outs)):
        ref_p, ref_st = alone[q]
        assert res["rc"] == 0, (q, res)
        assert res["stats"]["history"] == ref_st["history"], q
        assert torch.equal(p, ref_p), q
    assert info["classes"] == 3 and info["completed"] == len(probs) and info["resident"] == 0
    assert info["max_batch"] >= 5
    assert info["problem_iterations"] >= 2 * info["replays"]
    for P, (p, _) in zip(probs, alone):
        ref = oracle.solve(P.bx, P.by, P.bz, P.b, tol=1e-10, precision=precision)
        pn = p.cpu().numpy()
        assert np.linalg.norm(pn - ref["p"]) / np.linalg.norm(ref["p"]) <= 1e-8
