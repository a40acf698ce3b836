"""Serving loop through the C ABI (dg_server_*): requests that overlap on the
device give exactly the results they give alone; admission keeps the held
device memory within the budget and serves requests first-in first-out; a
request that can never fit is refused; the footprint formula bounds what a
context really allocates; a short Poisson stream completes."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1812_04789_amd import binding, inputs, serve     # noqa: E402

L = 2 * math.pi
GAS = serve.GAS
MIXED_REQS = [((3, 3, 3), 2, False, 0.2, 21), ((2, 2, 2), 3, True, 0.3, 22), ((4, 4, 4), 2, True, 0.1, 23),
              ((2, 2, 2), 4, False, 0.4, 24), ((3, 3, 3), 3, True, 0.25, 25), ((2, 2, 2), 2, False, 0.15, 26)]


def _reqs(spec):
    return [dict(t=0.0, n=n, lo=(0.0, 0.0, 0.0), hi=(L, L, L), p=p, mixed=mx, mach=m, seed=s)
            for n, p, mx, m, s in spec]


def _submit_all(server, reqs, bufs):
    for i, r in enumerate(reqs):
        po, fo = serve.solver_opts(r["p"], r["mixed"])
        server.submit(i, r["n"], r["lo"], r["hi"], r["p"], bufs[i][0], bufs[i][1], 0.05, po, fo, **GAS)


def test_result_is_the_same_alone_and_in_the_mix():
    reqs = _reqs(MIXED_REQS)
    bufs = serve.prepare(reqs)
    # alone: one slot, one request at a time
    alone = []
    for i, r in enumerate(reqs):
        sv = binding.Server(slots=1)
        _submit_all(sv, [r], [bufs[i]])
        sv.drain()
        (resp,) = sv.poll()
        assert resp.status == binding.DG_OK, sv.last_error()
        assert resp.stats.max_rel_res_true <= 1e-8
        alone.append(bufs[i][1].clone())
        sv.close()
    # the same requests together on four slots
    for b in bufs:
        b[1].zero_()
    torch.cuda.synchronize()
    sv = binding.Server(slots=4)
    _submit_all(sv, reqs, bufs)
    sv.drain()
    resps = sv.poll(max_n=len(reqs))
    assert max(r.concurrent for r in resps) >= 2          # they did overlap
    for r in resps:
        assert r.status == binding.DG_OK
        print("request", r.tag, "concurrent", r.concurrent, "latency", r.t_done - r.t_submit, flush=True)
        assert torch.equal(bufs[r.tag][1], alone[r.tag]), r.tag
    sv.close()
    # and the same as a plain context's step
    r = reqs[1]
    ctx = binding.Context(r["n"], r["lo"], r["hi"], r["p"], **GAS)
    po, fo = serve.solver_opts(r["p"], r["mixed"])
    W1, _ = ctx.bdf2_step(bufs[1][0], None, 0.05, po, fo)
    assert torch.equal(W1, alone[1])
    ctx.close()


def test_admission_budget_and_fifo():
    reqs = _reqs(MIXED_REQS) * 2
    bufs = serve.prepare(reqs)
    fps = [binding.footprint_bytes(r["n"], r["lo"], r["hi"], r["p"], *serve.solver_opts(r["p"], r["mixed"]))
           for r in reqs]
    budget = 1.2 * max(fps) + 0.5 * sorted(fps)[-2]
    sv = binding.Server(slots=4, hbm_budget=budget)
    _submit_all(sv, reqs, bufs)
    sv.drain()
    info = sv.info()
    resps = sorted(sv.poll(max_n=len(reqs)), key=lambda r: r.tag)
    assert all(r.status == binding.DG_OK for r in resps), sv.last_error()
    assert info["peak_held_bytes"] <= budget
    admits = [r.t_admit for r in resps]
    assert admits == sorted(admits)                       # first in, first out
    sv.close()


def test_oversized_request_is_refused():
    reqs = _reqs(MIXED_REQS[:2])
    bufs = serve.prepare(reqs)
    fp = binding.footprint_bytes(reqs[0]["n"], reqs[0]["lo"], reqs[0]["hi"], reqs[0]["p"],
                                 *serve.solver_opts(reqs[0]["p"], reqs[0]["mixed"]))
    sv = binding.Server(slots=2, hbm_budget=0.5 * fp)
    _submit_all(sv, reqs[:1], bufs[:1])
    sv.drain()
    (r,) = sv.poll()
    assert r.status == binding.DG_ENOMEM
    sv.close()


@pytest.mark.parametrize("n,p,mixed", [((3, 3, 3), 2, False), ((2, 2, 2), 3, True), ((2, 2, 2), 4, False),
                                       ((4, 4, 4), 1, False)])
def test_footprint_bounds_allocation(n, p, mixed):
    r = _reqs([(n, p, mixed, 0.2, 31)])[0]
    (buf,) = serve.prepare([r])
    ctx = binding.Context(n, r["lo"], r["hi"], p, **GAS)
    po, fo = serve.solver_opts(p, mixed)
    ctx.bdf2_step(buf[0], None, 0.05, po, fo, Wnp1=buf[1])
    used = ctx.device_bytes()
    fp = binding.footprint_bytes(n, r["lo"], r["hi"], p, po, fo)
    print("footprint", n, p, mixed, fp, used, flush=True)
    assert used <= fp <= 1.25 * used
    ctx.close()


def test_short_poisson_stream():
    out = serve.run(count=40, rate=200.0, seed=5, slots=4)
    print(out, flush=True)
    assert out["ok"] == 40
    assert out["max_rel_res_true"] <= 1e-8
    assert out["latency_s"]["p99"] >= out["latency_s"]["p50"] > 0
    assert out["aggregate_gdof_s"] > 0
