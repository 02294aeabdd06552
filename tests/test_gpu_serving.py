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
