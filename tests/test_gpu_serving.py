"""GPU tests of the request server (continuous batching of solves).

The bar: a request's result in the mix is bitwise the result of the same
solve run alone through the context API (a one-member batched context for
mixed precision, a plain context for FP64); requests of one size that wait
together share one batched context; admission never lets the contexts of
running requests exceed the HBM budget; requests overlap on the device when
the budget allows it; errors are reported per request.
"""

import sys
import time

import numpy as np
import pytest

from synth import grf, spheres

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_05266_amd as P
    P.load()
    return P


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def requests_mix():
    """(mask, force, precond, precision) of a small heterogeneous request set."""
    out = []
    for i, (N, kind, prec, pc) in enumerate([(32, "s", 1, 1), (24, "g", 0, 1), (40, "s", 1, 0), (48, "g", 1, 1),
                                             (32, "g", 0, 0), (36, "s", 1, 1)]):
        m = spheres(N, 3.0, 0.45, 100 + i) if kind == "s" else grf(N, 4.0, 0.35, 100 + i)
        out.append((m, (1.0, 0.0, 0.0), pc, prec))
    return out


def test_estimate_bounds_what_a_context_holds(P):
    for N in (16, 32, 48, 64):
        m = spheres(N, 3.0, 0.5, 7)
        with P.Stokes(m) as s:
            held64 = s.info()["device_bytes"]
            s.set_option("precision", 1)
            held32 = s.info()["device_bytes"]
        e64, e32 = P.stokes_estimate_bytes(N, 0), P.stokes_estimate_bytes(N, 1)
        say(f"    N={N}: fp64 held {held64} est {e64}; mixed held {held32} est {e32}")
        # slack: component arrays at their limit (2048), the label array, the
        # alignment allowance of a batched member's part, whole pages
        slack = 256 * 2048 * 8 + 2 * 2048 * 8 + 2 * N ** 3 + 256 * 256 + 4096
        assert held64 <= e64 <= held64 + slack
        assert held32 <= e32 <= held32 + slack


def test_result_alone_equals_result_in_the_mix(P):
    reqs = requests_mix()
    alone = []
    for m, f, pc, prec in reqs:
        if prec == 1:
            with P.StokesBatch([m], f) as b:
                alone.append(b.solve(pc, 1e-8)[0])
        else:
            with P.Stokes(m, f, precision=prec) as s:
                alone.append(s.solve(pc, 1e-8))
    budget = 4 * max(P.stokes_estimate_bytes(m.shape[0], prec) for m, _, _, prec in reqs)
    with P.Server(4, budget) as srv:
        # filler requests before and after, so every request shares the device
        fill = [srv.submit(spheres(32, 2.5, 0.4, 900 + q), precision=1) for q in range(2)]
        ids = [srv.submit(m, f, pc, 1e-8, prec) for m, f, pc, prec in reqs]
        fill += [srv.submit(grf(32, 5.0, 0.4, 950 + q), precision=0) for q in range(2)]
        res = [srv.wait(i) for i in ids]
        for i in fill:
            assert srv.wait(i)["status"] == 0
        st = srv.stats()
    say(f"    server stats {st}")
    assert st["completed"] == len(ids) + len(fill) and st["peak_running"] >= 2
    for a, r in zip(alone, res):
        say(f"    N={r['N']}: k alone {a['k_hat']:.16e} in mix {r['k_hat']:.16e} outer {a['outer_iters']}/"
            f"{r['outer_iters']}")
        assert r["status"] == 0
        assert r["k_hat"] == a["k_hat"]
        assert (r["outer_iters"], r["inner_A_iters"], r["inner_S_iters"]) == \
            (a["outer_iters"], a["inner_A_iters"], a["inner_S_iters"])
        assert r["div_norm"] == a["div_norm"]


def test_waiting_requests_of_one_size_share_a_batched_context(P):
    """One slot, held by a larger FP64 request while ten 32^3 mixed requests queue
    up: they then run as one batched context, each bitwise as alone."""
    small = [spheres(32, 3.0, 0.45, 500 + q) if q % 2 else grf(32, 4.0, 0.35, 500 + q) for q in range(10)]
    alone = []
    for m in small:
        with P.StokesBatch([m]) as b:
            alone.append(b.solve(P.STOKES_SIMPLE, 1e-8)[0])
    budget = P.stokes_estimate_bytes(64, 0) + 10 * P.stokes_estimate_bytes(32, 1)
    with P.Server(1, budget) as srv:
        first = srv.submit(spheres(64, 3.0, 0.5, 499), precision=0)
        ids = [srv.submit(m, precision=1) for m in small]
        r0 = srv.wait(first)
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    say(f"    {st}; members per context: {[r['batch_members'] for r in res]}")
    assert r0["status"] == 0 and r0["batch_members"] == 1
    assert st["contexts"] == 2 and st["requests_on_contexts"] == 11
    for a, r in zip(alone, res):
        assert r["status"] == 0 and r["batch_members"] == 10
        assert r["k_hat"] == a["k_hat"] and r["div_norm"] == a["div_norm"]
        assert (r["outer_iters"], r["inner_A_iters"], r["inner_S_iters"]) == \
            (a["outer_iters"], a["inner_A_iters"], a["inner_S_iters"])
        assert r["device_bytes"] == P.stokes_estimate_bytes(32, 1)
    # without batching each request gets a context of its own, with the same results
    with P.Server(1, budget, max_members=1) as srv:
        ids = [srv.submit(m, precision=1) for m in small[:3]]
        res1 = [srv.wait(i) for i in ids]
    for a, r in zip(alone, res1):
        assert r["batch_members"] == 1 and r["k_hat"] == a["k_hat"]


def test_admission_respects_the_budget_and_overlaps(P):
    N = 48
    budget = int(2.5 * P.stokes_estimate_bytes(N, 1))
    with P.Server(4, budget) as srv:
        ids = [srv.submit(spheres(N, 3.0, 0.5, 300 + q), precision=1) for q in range(6)]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    say(f"    {st}")
    assert all(r["status"] == 0 for r in res)
    assert st["peak_bytes"] <= budget
    assert st["peak_running"] == 2          # the budget holds two contexts of this size, the slots four
    assert st["bytes_in_use"] == 0 and st["running"] == 0 and st["queued"] == 0
    # FIFO admission, and the work of admitted requests overlaps in time
    starts = [r["t_start"] for r in res]
    assert starts == sorted(starts)
    spans = sorted((r["t_start"], r["t_end"]) for r in res)
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    for r in res:
        assert r["device_bytes"] <= P.stokes_estimate_bytes(N, 1)
        assert r["t_submit"] <= r["t_start"] <= r["t_end"]


def test_request_errors_are_reported_per_request(P):
    with P.Server(2, P.stokes_estimate_bytes(32, 1)) as srv:
        with pytest.raises(P.StokesError) as e:
            srv.submit(spheres(64, 3.0, 0.5, 1))          # alone larger than the budget
        assert e.value.status == -6
        bad = np.ones((16, 16, 16), np.uint8)
        bad[0, 0, 0] = 2                                   # not a 0/1 mask
        ib = srv.submit(bad)
        ig = srv.submit(spheres(16, 2.0, 0.5, 2))
        rb, rg = srv.wait(ib), srv.wait(ig)
        with pytest.raises(P.StokesError):
            srv.wait(12345)
    assert rb["status"] == -1
    assert rg["status"] == 0 and rg["k_hat"] > 0


def test_destroy_cancels_queued_requests(P):
    t0 = time.time()
    srv = P.Server(1, P.stokes_estimate_bytes(32, 1))
    for q in range(4):
        srv.submit(spheres(32, 3.0, 0.5, 40 + q), precision=1)
    srv.close()                                            # the running request finishes, the rest are dropped
    assert time.time() - t0 < 60
