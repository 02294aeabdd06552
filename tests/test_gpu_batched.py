"""Batched persistent CG: each system's iterate and iteration count are
bitwise the same alone and in a mixed batch; every result passes the CG
parity checks against the oracle."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import ctx, log, torch_dev

pytestmark = pytest.mark.gpu


def systems():
    out = []
    for n, f in [(8, "dia"), (12, "csr"), (16, "ell"), (20, "dia"), (10, "csr"), (24, "csr"), (41, "dia")]:
        out.append((inputs.hpcg27(n), f))
    for N, hbw, seed in [(1000, 3, 1), (5000, 17, 2), (30000, 64, 3), (2500, 1, 4)]:
        out.append((inputs.banded_spd(N, hbw, seed=seed), "csr"))
    out.append((inputs.hpcg27(9), "coo"))  # not eligible for the one-workgroup path
    return out


def solve(mats, probs, torch, dev, tol=1e-8):
    bs = [torch.from_numpy(p.b).to(dev) for p in probs]
    xs = [torch.zeros(p.nrows, dtype=torch.float64, device=dev) for p in probs]
    res = dsm.cg_batched(mats, bs, xs, tol=tol)
    return [x.cpu().numpy() for x in xs], res


def test_batched_alone_equals_mixed_bitwise():
    torch, dev = torch_dev()
    sysl = systems()
    probs = [p for p, _ in sysl]
    mats = []
    for p, f in sysl:
        A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val)
        A.convert(f)
        mats.append(A)
    log(f"[batched] mixed batch of {len(mats)}")
    xs_mix, res_mix = solve(mats, probs, torch, dev)
    for k, (A, p) in enumerate(zip(mats, probs)):
        xa, ra = solve([A], [p], torch, dev)
        assert np.array_equal(xa[0].view(np.uint64), xs_mix[k].view(np.uint64)), k
        assert ra[0]["iters"] == res_mix[k]["iters"], k
        _, it, _, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-8)
        assert res_mix[k]["status"] == "converged"
        assert abs(res_mix[k]["iters"] - it) <= 1, (k, res_mix[k], it)
        assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xs_mix[k]) <= 1.5e-8
    # repeat the mix: same bits
    xs2, _ = solve(mats, probs, torch, dev)
    for a, b in zip(xs_mix, xs2):
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    for A in mats:
        A.close()


def test_batched_large_batch_of_small_systems():
    torch, dev = torch_dev()
    probs = [inputs.hpcg27(8 + (k % 9)) for k in range(600)]
    mats = []
    for p in probs[:9]:
        A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val)
        A.convert("dia")
        mats.append(A)
    mm = [mats[k % 9] for k in range(600)]
    xs, res = solve(mm, probs, torch, dev, tol=1e-10)
    for k in range(9):
        _, it, _, _ = oracle.cg(probs[k].row_ptr, probs[k].col, probs[k].val, probs[k].b, tol=1e-10)
        for j in range(k, 600, 9):
            assert res[j]["status"] == "converged" and abs(res[j]["iters"] - it) <= 1
            assert np.array_equal(xs[j].view(np.uint64), xs[k].view(np.uint64))
    for A in mats:
        A.close()
