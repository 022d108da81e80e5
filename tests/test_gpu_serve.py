"""The continuous-batching server (brt_server_*) on the GPU.

* a served request's coefficients equal the oracle's over the same trees (the trees of point i of a
  request with stream id s are trees 0..n-1 with Philox point id s*1024 + i);
* a request's results are bit-identical served alone and inside a mix of other requests (requests that
  differ only in their initial data, and requests with other coefficients);
* admission by device slots and the bounded queue.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2402_06491_amd import inputs

from . import _parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "no GPU"
    import paper_2402_06491_amd as brt

    c = brt.Context(0)
    yield c
    c.close()


def _mc(**kw):
    return inputs.mc_params(seed=21, max_order=12, prune=1, precision=32, **kw)


def _request(seed, n, rng):
    prob = inputs.problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], inputs.cubic_2d_u0(seed))
    x = rng.uniform(-8, 8, size=(n, 2))
    t = np.exp(rng.uniform(np.log(0.25), np.log(1.0), size=n))
    return prob, x, t


def _wait(srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for tk, n in tickets.items():
            if tk in out:
                continue
            r = srv.poll(tk, n)
            if r is not None:
                out[tk] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return out


@pytest.mark.parametrize("round_trees", [8192, 32768])
def test_served_request_matches_oracle(ctx, round_trees):
    """Two rounds of a served request against the oracle's walk of the same trees.  Rounds of 8192
    trees are reduced in one 8192-tree segment each, rounds of 32768 in one 32768-tree segment."""
    import paper_2402_06491_amd as brt

    n = 2 * round_trees
    print(f"\n[case] serve_vs_oracle: 1 request x 6 points, 2 rounds of {round_trees} trees", flush=True)
    mc = _mc()
    srv = brt.Server(ctx, 2, "gauss_sum", mc, max_points=64, round_trees=round_trees, max_trees=n, target_se=0.0)
    rng = np.random.default_rng(3)
    prob, x, t = _request(5, 6, rng)
    tk = srv.submit(prob, x, t, stream_id=7)
    res = _wait(srv, {tk: 6})[tk]
    srv.close()
    assert np.all(res["trees"] == n)
    B = mc["max_order"] + 2
    for i in range(6):
        rec = oracle.walk(prob, mc, np.repeat(x[i:i + 1], n, axis=0), t[i], 7 * 1024 + i, np.arange(n))
        mom = oracle.moments(rec, mc)
        nz = oracle.normalize(prob, mc)
        a, _ = oracle.coefficients(mom, nz.mu, float(t[i]))
        scale = np.abs(a).max()
        np.testing.assert_allclose(res["coef"][i][:B], a, rtol=0, atol=(P.FP32_TOL + 1e-6) * scale + 1e-300)


def _other(k, n, rng, mix):
    """Another request of the mix.  "family": the probe's coefficients with Gaussian sums of 2, 4 or 6
    terms (a launch group keeps only their initial data per problem); "table": other coefficients too
    (the group keeps every problem's full record)."""
    r = np.random.default_rng(500 + k)
    nterms = (2, 4, 6)[k % 3]
    u0 = inputs.gauss_sum([(r.uniform(0.2, 1.0), r.uniform(-6, 6), r.uniform(-6, 6), r.uniform(0.5, 2.0))
                           for _ in range(nterms)])
    coef = [0.0, 1.0, 0.0, -1.0] if mix == "family" else [0.0, 1.0, -0.25 * (k % 3), -1.0 + 0.1 * (k % 2)]
    prob = inputs.problem(2, 1.0, coef, u0)
    x = rng.uniform(-8, 8, size=(n, 2))
    t = np.exp(rng.uniform(np.log(0.25), np.log(1.0), size=n))
    return prob, x, t


@pytest.mark.parametrize("mix", ["family", "table"])
def test_alone_equals_mixed(ctx, mix):
    import paper_2402_06491_amd as brt

    print(f"\n[case] serve_alone_vs_mixed ({mix}): 1 request alone, then among 12 others", flush=True)
    mc = _mc()
    kw = dict(max_points=2048, round_trees=8192, max_trees=32768, target_se=2e-2)
    rng = np.random.default_rng(11)
    probe = _request(1, 40, rng)
    others = [_other(k, int(rng.integers(1, 200)), rng, mix) for k in range(12)]

    srv = brt.Server(ctx, 2, "gauss_sum", mc, **kw)
    tk = srv.submit(*probe, stream_id=9)
    alone = _wait(srv, {tk: 40})[tk]
    srv.close()

    srv = brt.Server(ctx, 2, "gauss_sum", mc, **kw)
    tickets = {}
    for k, (p, x, t) in enumerate(others[:6]):
        tickets[srv.submit(p, x, t, stream_id=1000 + k)] = len(t)
    tk = srv.submit(*probe, stream_id=9)
    tickets[tk] = 40
    for k, (p, x, t) in enumerate(others[6:]):
        tickets[srv.submit(p, x, t, stream_id=2000 + k)] = len(t)
    mixed = _wait(srv, tickets)[tk]
    st = srv.stats()
    srv.close()
    for key in ("u", "se", "coef", "trees", "flags"):
        np.testing.assert_array_equal(alone[key], mixed[key], err_msg=key)
    assert st["completed"] == 13 and st["trees"] > 0 and st["p99_latency_s"] >= st["p50_latency_s"] > 0


def test_admission_and_queue_bound(ctx):
    import paper_2402_06491_amd as brt

    print("\n[case] serve_admission: 8 slots, queue of 2", flush=True)
    mc = _mc()
    srv = brt.Server(ctx, 2, "gauss_sum", mc, max_points=8, round_trees=8192, max_trees=8192 * 4, target_se=0.0,
                     queue_cap=2)
    rng = np.random.default_rng(5)
    accepted, busy = {}, 0
    for k in range(8):
        p, x, t = _request(k, 6, rng)
        try:
            accepted[srv.submit(p, x, t, stream_id=k)] = 6
        except brt.BrtError as e:
            assert e.code == -4
            busy += 1
    assert busy > 0 and len(accepted) >= 2
    res = _wait(srv, accepted)
    assert all(np.all(r["trees"] == 8192 * 4) for r in res.values())
    with pytest.raises(brt.BrtError):
        srv.submit(*_request(0, 9, rng), stream_id=99)  # more points than the server has slots
    st = srv.stats()
    assert st["rejected"] == busy and st["completed"] == len(accepted)
    srv.close()
