"""Serving loop: admission against an HBM budget, continuous batching, and
independence of each request's result from the mix it is served in."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _requests(n=6, steps=4):
    trace = W.serving_trace(n=n, lam=50.0, seed=11, steps=steps, nmin=64, nmax=192)
    return trace


@pytest.mark.parametrize("rounds", [False, True])
def test_served_alone_equals_served_in_mix(rounds):
    """Each request's fields are the same, bit for bit, served alone (one
    simulation stepping on its own) as served in the mix: with a step worker
    per simulation, and with the time steps of all running simulations
    batched in fused rounds."""
    from paper_2211_10698_amd import serve
    reqs = _requests()
    srv = serve.Server(hbm_budget=8 << 30, precision=1, threads=4, prep_workers=3, keep_fields=True, rounds=rounds)
    mix = srv.run(reqs)
    assert all(r.status == 0 for r in mix)
    assert all(r.div_rel_max <= 1e-8 for r in mix)
    for k in (0, 3, 5):
        print(f"[serve] alone {k}", flush=True)
        alone = serve.Server(hbm_budget=8 << 30, precision=1, threads=1, prep_workers=1,
                             keep_fields=True).run([W.Request(reqs[k].case, 0.0)])[0]
        for name in ("ux", "uy", "p"):
            assert np.array_equal(alone.fields[name], mix[k].fields[name]), (k, name)


@pytest.mark.parametrize("rounds", [False, True])
def test_admission_respects_budget_and_queues(rounds):
    from paper_2211_10698_amd import serve
    reqs = _requests(n=8, steps=3)
    srv = serve.Server(precision=0, threads=4, prep_workers=2, rounds=rounds)
    sizes = [serve.footprint(r.case, srv._params(r.case)) for r in reqs]
    srv.budget = 2 * max(sizes)          # at most a couple of simulations at a time
    recs = srv.run(reqs)
    assert srv.max_used <= srv.budget
    assert all(np.isfinite(r.completion) and r.completion >= r.admit >= r.arrival for r in recs)
    assert max(r.queue for r in recs) > 0.0     # the budget made someone wait
    s = serve.summarize(recs, max(r.completion for r in recs))
    assert s["latency_p99_s"] >= s["latency_p50_s"] > 0.0
    assert s["div_rel_max"] <= 1e-8 and s["statuses"] == [0]
    # a request larger than the budget is refused up front
    with pytest.raises(ValueError):
        serve.Server(hbm_budget=1 << 20, precision=0).run(reqs[:1])
