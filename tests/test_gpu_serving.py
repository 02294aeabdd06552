"""Serving: continuous batching under an HBM budget.  Each request's result
is bitwise the same alone and in the mix; timestamps are ordered; a request
that cannot fit the budget is refused; latency percentiles are reported."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import ctx, log, torch_dev

pytestmark = pytest.mark.gpu


def pool():
    probs = [inputs.hpcg27(n) for n in (8, 12, 16, 22, 30, 36, 44)]
    probs += [inputs.banded_spd(N, h, seed=s) for N, h, s in [(1200, 4, 1), (9000, 30, 2), (60000, 12, 3)]]
    mats = []
    for p in probs:
        A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val)
        A.select()
        mats.append(A)
    return probs, mats


def run(server, reqs, probs, mats, torch, dev, one_by_one):
    out = {}
    pending = []
    for r, k in enumerate(reqs):
        b = torch.from_numpy(probs[k].b).to(dev)
        x = torch.zeros(probs[k].nrows, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = server.submit(mats[k], b, x, tol=1e-8)
        pending.append((r, k, t, b, x))
        if one_by_one:
            res, ts = server.wait(t)
            out[r] = (x.cpu().numpy(), res, ts)
    for r, k, t, b, x in pending:
        if r not in out:
            res, ts = server.wait(t)
            out[r] = (x.cpu().numpy(), res, ts)
    return out


@pytest.mark.parametrize("small_rows", [None, 40000])
def test_serving_alone_equals_mix_and_budget(small_rows):
    """small_rows: the default (only the tiny systems batched) and the
    one-workgroup solver's limit (every system up to 40,000 rows batched)."""
    torch, dev = torch_dev()
    probs, mats = pool()
    rng = inputs.uniform(77, 1, np.arange(60, dtype=np.uint64))
    reqs = [int(u * len(probs)) for u in rng]
    biggest = max(m.info()["bytes"] for m in mats)
    kw = {} if small_rows is None else {"small_rows": small_rows}
    srv = dsm.Server(ctx(), slots=8, hbm_budget=int(biggest * 2.5), streams=3, **kw)
    log("[serving] mix")
    mix = run(srv, reqs, probs, mats, torch, dev, one_by_one=False)
    log("[serving] alone")
    alone = run(srv, reqs, probs, mats, torch, dev, one_by_one=True)
    lat = []
    for r, k in enumerate(reqs):
        xm, rm, tm = mix[r]
        xa, ra, ta = alone[r]
        assert np.array_equal(xm.view(np.uint64), xa.view(np.uint64)), (r, k)
        assert rm["iters"] == ra["iters"] and rm["status"] == "converged"
        assert tm["arrival"] <= tm["start"] <= tm["finish"]
        p = probs[k]
        assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xm) <= 1.5e-8
        lat.append(tm["finish"] - tm["arrival"])
    log(f"[serving] p50 {np.percentile(lat, 50) * 1e3:.2f} ms p99 {np.percentile(lat, 99) * 1e3:.2f} ms")
    srv.close()
    tiny = dsm.Server(ctx(), hbm_budget=1024)
    with pytest.raises(dsm.DsmError) as e:
        tiny.submit(mats[0], torch.ones(probs[0].nrows, dtype=torch.float64, device=dev),
                    torch.zeros(probs[0].nrows, dtype=torch.float64, device=dev))
    assert e.value.status == dsm.L.E_NOMEM
    tiny.close()
    for A in mats:
        A.close()


def max_concurrency(intervals):
    """Largest number of [start, finish] intervals that overlap at one time."""
    ev = sorted([(s, 1) for s, f in intervals] + [(f, -1) for s, f in intervals], key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_serving_requests_overlap_on_the_device():
    """Requests admitted together run at the same time on different worker
    streams: their start-finish intervals overlap, and the mix finishes in
    clearly less time than the same solves one after another."""
    torch, dev = torch_dev()
    probs = [inputs.hpcg27(40), inputs.banded_spd(60000, 12, seed=3), inputs.hpcg27(36)]
    mats = [dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val).convert("csr") for p in probs]
    reqs = [i % len(probs) for i in range(12)]
    srv = dsm.Server(ctx(), slots=16, streams=4, small_rows=0)
    run(srv, reqs[:3], probs, mats, torch, dev, one_by_one=True)  # warm the workers
    alone = run(srv, reqs, probs, mats, torch, dev, one_by_one=True)
    t0 = srv.now()
    mix = run(srv, reqs, probs, mats, torch, dev, one_by_one=False)
    wall_mix = max(ts["finish"] for _, _, ts in mix.values()) - t0
    seq = sum(ts["finish"] - ts["start"] for _, _, ts in alone.values())
    conc = max_concurrency([(ts["start"], ts["finish"]) for _, _, ts in mix.values()])
    st = srv.stats()
    log(f"[serving-overlap] sequential {seq * 1e3:.1f} ms, mix wall {wall_mix * 1e3:.1f} ms, "
        f"max concurrent {conc}, busy {st['busy_s']:.3f} s of {st['elapsed_s']:.3f} s")
    for r in range(len(reqs)):
        assert np.array_equal(mix[r][0].view(np.uint64), alone[r][0].view(np.uint64)), r
        assert mix[r][1]["status"] == "converged"
    assert conc >= 2
    assert wall_mix < 0.8 * seq
    srv.close()
    for A in mats:
        A.close()


def test_serving_budget_forces_waits():
    """A server budget that holds the largest request (its matrix and the
    workspaces of two workers) but not two of the larger matrices at once:
    requests wait at the head of the queue for budget, the charged bytes
    never exceed it, and every result equals the same request run alone."""
    torch, dev = torch_dev()
    probs, mats = pool()
    rng = inputs.uniform(78, 1, np.arange(48, dtype=np.uint64))
    reqs = [int(u * len(probs)) for u in rng]
    biggest = max(m.info()["bytes"] for m in mats)
    nmax = max(p.nrows for p in probs)
    ws_bound = 1 << int(np.ceil(np.log2(48 * nmax + (1 << 16))))  # >= a CG workspace, rounded as the server does
    budget = biggest + 2 * ws_bound + (1 << 20)
    srv = dsm.Server(ctx(), slots=16, hbm_budget=budget, streams=3)
    mix = run(srv, reqs, probs, mats, torch, dev, one_by_one=False)
    st = srv.stats()
    alone = run(srv, reqs, probs, mats, torch, dev, one_by_one=True)
    log(f"[serving-budget] budget {budget / 1e6:.1f} MB: {st['budget_waits']} waits, peak charged "
        f"{st['peak_charged_bytes'] / 1e6:.1f} MB, workers hold {st['workspace_bytes'] / 1e6:.1f} MB")
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["budget_waits"] > 0
    assert st["peak_charged_bytes"] <= budget
    for r, k in enumerate(reqs):
        assert np.array_equal(mix[r][0].view(np.uint64), alone[r][0].view(np.uint64)), (r, k)
        assert mix[r][1]["status"] == "converged"
    srv.close()
    for A in mats:
        A.close()


def test_serving_context_budget():
    """No server budget: the server takes the context's and counts what the
    context really holds.  With room for about one worker's workspaces beyond
    the resident matrices, requests wait for it instead of failing, and
    every result converges and equals the same request alone."""
    torch, dev = torch_dev()
    probs = [inputs.hpcg27(n) for n in (8, 16, 30, 44)] + [inputs.banded_spd(60000, 12, seed=3)]
    probe = dsm.Context(0)
    tmp = [dsm.Matrix.from_csr(probe, p.nrows, p.ncols, p.row_ptr, p.col, p.val) for p in probs]
    resident = probe.bytes_in_use()
    for A in tmp:
        A.close()
    probe.close()
    c = dsm.Context(0, hbm_budget=resident + 6 * (1 << 20))
    mats = [dsm.Matrix.from_csr(c, p.nrows, p.ncols, p.row_ptr, p.col, p.val) for p in probs]
    assert c.bytes_in_use() == resident
    rng = inputs.uniform(79, 1, np.arange(40, dtype=np.uint64))
    reqs = [int(u * len(probs)) for u in rng]
    srv = dsm.Server(c, slots=16, streams=3)
    mix = run(srv, reqs, probs, mats, torch, dev, one_by_one=False)
    st = srv.stats()
    alone = run(srv, reqs, probs, mats, torch, dev, one_by_one=True)
    log(f"[serving-ctx-budget] {st['budget_waits']} waits, {st['requeued']} requeued, peak "
        f"{st['peak_charged_bytes'] / 1e6:.2f} MB of {(resident + 6 * (1 << 20)) / 1e6:.2f} MB")
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["budget_waits"] > 0
    for r, k in enumerate(reqs):
        assert mix[r][1]["status"] == "converged", (r, k, mix[r][1])
        assert np.array_equal(mix[r][0].view(np.uint64), alone[r][0].view(np.uint64)), (r, k)
    srv.close()
    for A in mats:
        A.close()
    assert c.bytes_in_use() == 0
    c.close()
