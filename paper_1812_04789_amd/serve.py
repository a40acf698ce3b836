"""Serving run: a seeded Poisson stream of implicit time-step requests through
the library's serving loop (dg_server_*).

Each request is one BDF2 step (Sec. 4) of a Navier-Stokes case on a periodic
cube mesh, solved by FGMRES with a p-multigrid V-cycle (Sec. 6), in FP64 or
mixed precision (FP32 fine block factors, BF16 assembled coarsest operator).
The client prepares every request's initial state on the device before the
clock starts (random-phase Fourier velocity field, projected with a staging
context of the same mesh), then submits each request at its arrival time and
collects responses.  Reported: latency percentiles (submit to done), queueing
and service time, aggregate GDOF/s and the device memory the server held.
"""
import math
import time

import numpy as np

from . import binding, inputs

GAS = dict(gamma=1.4, mu=1.0 / 1600, Pr=0.71, eta=7.0)


def levels_for(p):
    return {1: [1], 2: [2, 1], 3: [3, 2, 1], 4: [4, 2, 1]}[p]


def solver_opts(p, mixed, restart=40, rtol=1e-8):
    if mixed:
        po = binding.pmg_opts(levels_for(p), prec_fine=binding.DG_FP32, prec_coarse=binding.DG_BF16,
                              coarse_matrix_free=2)
    else:
        po = binding.pmg_opts(levels_for(p), prec_fine=binding.DG_FP64, prec_coarse=binding.DG_FP64,
                              coarse_matrix_free=2)
    return po, binding.fgmres_opts(restart=restart, rtol=rtol)


def prepare(requests):
    """Initial states (device) of every request, projected by a staging context
    per distinct (mesh, degree); the staging contexts are closed afterwards."""
    import torch
    staging = {}
    out = []
    for r in requests:
        key = (r["n"], r["p"])
        if key not in staging:
            staging[key] = binding.Context(r["n"], r["lo"], r["hi"], r["p"], **GAS)
        ctx = staging[key]
        ks, ph = inputs.fourier_phases(r["seed"])
        vals = inputs.fourier_state_torch(ctx.quad_points(), ks, ph, gamma=GAS["gamma"], mach=r["mach"])
        Wn = ctx.project(vals.reshape(-1).contiguous())
        out.append((Wn, torch.empty_like(Wn)))
    torch.cuda.synchronize()
    for c in staging.values():
        c.close()
    return out


def run(count=400, rate=200.0, seed=1812, slots=8, hbm_budget=0.0, dt=0.05, requests=None, log=None):
    """Serve `count` requests of the seeded stream; returns a summary dict."""
    import torch
    reqs = requests if requests is not None else inputs.serving_requests(count, rate, seed)
    t_prep = time.perf_counter()
    bufs = prepare(reqs)
    t_prep = time.perf_counter() - t_prep
    server = binding.Server(slots=slots, hbm_budget=hbm_budget, cache=True)
    responses = []
    wall0 = time.perf_counter()
    for i, r in enumerate(reqs):
        target = wall0 + r["t"]
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            responses += server.poll(wait_ms=max(1, min(5, int((target - now) * 1000))))
        po, fo = solver_opts(r["p"], r["mixed"])
        server.submit(i, r["n"], r["lo"], r["hi"], r["p"], bufs[i][0], bufs[i][1], dt, po, fo, **GAS)
        if log and i % 100 == 99:
            log("submitted %d/%d, done %d" % (i + 1, len(reqs), len(responses)))
    server.drain()
    responses += server.poll(max_n=max(1, len(reqs)))
    wall = time.perf_counter() - wall0
    info = server.info()
    err = server.last_error()
    server.close()
    torch.cuda.synchronize()
    by_tag = {int(x.tag): x for x in responses}
    assert len(by_tag) == len(reqs), (len(by_tag), len(reqs))
    lat = np.array([by_tag[i].t_done - by_tag[i].t_submit for i in range(len(reqs))])
    queue = np.array([by_tag[i].t_admit - by_tag[i].t_submit for i in range(len(reqs))])
    serv = np.array([by_tag[i].t_done - by_tag[i].t_admit for i in range(len(reqs))])
    status = [by_tag[i].status for i in range(len(reqs))]
    ndof = sum(int(by_tag[i].ndof) for i in range(len(reqs)))
    t_first = min(x.t_submit for x in responses)
    t_last = max(x.t_done for x in responses)
    ok = [s in (binding.DG_OK,) for s in status]
    worst = max(by_tag[i].stats.max_rel_res_true for i in range(len(reqs)) if ok[i]) if any(ok) else None
    return {
        "requests": len(reqs), "rate_req_s": rate, "slots": slots, "ok": int(sum(ok)),
        "statuses": sorted(set(status)), "last_error": err or None,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                      "p99": float(np.percentile(lat, 99)), "max": float(lat.max())},
        "queue_s": {"p50": float(np.percentile(queue, 50)), "p99": float(np.percentile(queue, 99)),
                    # queueing of the first and last third of the arrivals: a growing queue
                    # (offered rate above what the device serves) shows as last >> first
                    "first_third_p50": float(np.percentile(queue[:max(1, len(queue) // 3)], 50)),
                    "last_third_p50": float(np.percentile(queue[-max(1, len(queue) // 3):], 50))},
        "service_s": {"p50": float(np.percentile(serv, 50)), "p99": float(np.percentile(serv, 99))},
        "aggregate_gdof_s": ndof / (t_last - t_first) / 1e9,
        "throughput_req_s": len(reqs) / (t_last - t_first),
        "makespan_s": t_last - t_first, "wall_s": wall, "prepare_s": t_prep,
        "total_dof": ndof, "max_rel_res_true": worst,
        "peak_held_gb": info["peak_held_bytes"] / 1e9, "budget_gb": info["budget_bytes"] / 1e9,
        "contexts_at_end": info["contexts"],
        "max_concurrent": int(max(x.concurrent for x in responses)),
        "mixed_fraction": float(np.mean([r["mixed"] for r in reqs])),
    }
