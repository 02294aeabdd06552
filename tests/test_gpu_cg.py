"""CG parity: iteration count within +-1 of the FP64 oracle, true residual
<= 1.5 tol (recomputed by the oracle), ||x - x_oracle|| <= 10 kappa tol ||x||,
special cases and failure statuses."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import anchors, FORMATS, log, make_matrix, problem, torch_dev

pytestmark = pytest.mark.gpu

KAPPA = {5: 10.0, 16: 39.05, 104: 1489.4}


def solve(p, fmt, tol=1e-10, **kw):
    torch, dev = torch_dev()
    A = make_matrix(p)
    A.convert(fmt)
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=tol, **kw)
    xh = x.cpu().numpy()
    A.close()
    return xh, res


@pytest.mark.parametrize("fmt", FORMATS)
def test_cg_hpcg16_every_format(fmt):
    p = problem("hpcg16")
    xo, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    log(f"[cg] hpcg16 {fmt}")
    x, res = solve(p, fmt)
    assert res["status"] == "converged"
    assert abs(res["iters"] - it) <= 1, (res, it)
    assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x) <= 1.5e-10
    assert np.linalg.norm(x - xo) <= 10 * KAPPA[16] * 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("fmt,variant", [("dia", v) for v in (0, 2, 8, 13, 16, 19, 21, 31)] + [("hdc", 18), ("ell", 10)]
                         + [("csr", v) for v in (0, 7, 2, 6, 8, 15)])
def test_cg_sweep_variants(fmt, variant):
    """The three-kernel loop with the SpMV's p.q epilogue in every kind of
    sweep (gathered x, paired rows, LDS-staged x with 1, 2 and 4 row groups,
    both tile orders) and every kind of CSR launch (adaptive row blocks in
    both orders, 4- and 64-lane rows, nontemporal loads) reaches the
    oracle's iterate."""
    torch, dev = torch_dev()
    p = problem("hpcg16")
    xo, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    log(f"[cg] hpcg16 {fmt} v{variant}")
    A = make_matrix(p)
    A.convert(fmt)
    A.variant = variant
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=1e-10)
    x = x.cpu().numpy()
    A.close()
    assert res["status"] == "converged"
    assert abs(res["iters"] - it) <= 1, (res, it)
    assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x) <= 1.5e-10
    assert np.linalg.norm(x - xo) <= 10 * KAPPA[16] * 1e-10 * np.linalg.norm(xo)


def test_cg_hpcg104_dia_and_csr():
    p = problem("hpcg104")
    for fmt in ["dia", "csr"]:
        log(f"[cg] hpcg104 {fmt}")
        x, res = solve(p, fmt)
        assert res["status"] == "converged"
        assert abs(res["iters"] - anchors()["cg_hpcg27_104_tol1e-10"]["iters"]) <= 1, res
        assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x) <= 1.5e-10
        assert np.linalg.norm(x - 1.0) <= 10 * KAPPA[104] * 1e-10 * np.sqrt(p.nrows)


def test_cg_special_cases():
    torch, dev = torch_dev()
    for n in (1, 2):
        x, res = solve(inputs.hpcg27(n), "csr")
        assert res["status"] == "converged" and res["iters"] == 1
        assert np.max(np.abs(x - 1)) <= 1e-15
    p = problem("hpcg5")
    A = make_matrix(p)
    x, res = A.cg(torch.zeros(p.nrows, dtype=torch.float64, device=dev))
    assert res["status"] == "converged" and res["iters"] == 0 and not x.any()
    x, res = A.cg(torch.from_numpy(p.b).to(dev), maxit=3)
    assert res["status"] == "not_converged" and res["iters"] == 3
    bb = p.b.copy()
    bb[7] = np.nan
    x, res = A.cg(torch.from_numpy(bb).to(dev))
    assert res["status"] == "breakdown"
    A.close()


def test_cg_breakdown_on_negative_definite():
    torch, dev = torch_dev()
    n = 50
    rp = np.arange(n + 1, dtype=np.int32)
    A = dsm.Matrix.from_csr(dsm.Context(0), n, n, rp, np.arange(n, dtype=np.int32), -np.ones(n))
    x, res = A.cg(torch.ones(n, dtype=torch.float64, device=dev))
    assert res["status"] == "breakdown" and res["iters"] == 1
    A.close()


def test_cg_nonzero_initial_guess():
    torch, dev = torch_dev()
    p = problem("hpcg16")
    x0 = inputs.uniform_vector(p.nrows, seed=3)
    xo, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, x0=x0, tol=1e-10)
    A = make_matrix(p)
    x, res = A.cg(torch.from_numpy(p.b).to(dev), x=torch.from_numpy(x0.copy()).to(dev), tol=1e-10)
    assert abs(res["iters"] - it) <= 1
    assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x.cpu().numpy()) <= 1.5e-10
    A.close()


@pytest.mark.parametrize("graph", ["1", "0"])
@pytest.mark.parametrize("offset", [0, 1])
def test_cg_ragged_sizes_and_unaligned_x(offset, graph, monkeypatch):
    """The FP64 vector updates load two elements per lane where every vector
    is 16-byte aligned: odd sizes end them with a ragged tail, and an x that
    starts 8 bytes past a 16-byte boundary (offset 1) takes one element per
    load (eager launches; the replayed loop works on an aligned copy of x).
    IR on the same systems covers its FP32 inner loop at odd sizes."""
    torch, dev = torch_dev()
    monkeypatch.setenv("DSM_CG_GRAPH", graph)
    for p in [inputs.hpcg27(7), inputs.banded_spd(1203, 5, seed=4), inputs.hpcg27(1)]:
        n = p.nrows
        xo, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
        b = torch.from_numpy(p.b).to(dev)
        log(f"[cg] {p.name} n={n} x offset {offset}")
        for fmt, vdt, mode in [("csr", "f64", "f64"), ("dia", "f64", "f64"), ("csr", "f32", "ir")]:
            A = make_matrix(p)
            A.convert(fmt, value_dtype=vdt)
            buf = torch.full((n + 1,), 7.0, dtype=torch.float64, device=dev)
            buf[offset:offset + n] = 0
            x, res = A.cg(b, x=buf[offset:offset + n], tol=1e-10, mode=mode)
            assert (x.data_ptr() % 16 != 0) == (offset == 1)
            xh = x.cpu().numpy()
            A.close()
            assert res["status"] == "converged", (fmt, mode, res)
            if mode == "f64":
                assert abs(res["iters"] - it) <= 1, (fmt, res, it)
                assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh) <= 1.5e-10
            else:
                # IR converges for the stored (rounded) values
                lowvals = oracle.cast_f32(p.val).astype(np.float64)
                assert oracle.true_relres(p.row_ptr, p.col, lowvals, p.b, xh) <= 1e-10
            # the element outside the view is untouched
            assert buf[0 if offset == 1 else n].item() == 7.0


def test_cg_rejects_rectangular():
    torch, dev = torch_dev()
    p = problem("rect_empty")
    A = make_matrix(p)
    with pytest.raises(dsm.DsmError):
        A.cg(torch.ones(p.nrows, dtype=torch.float64, device=dev))
    A.close()


def test_cg_graph_replay_matches_eager():
    """The loop replayed from a captured HIP graph gives the same bits as
    eager launches, on every replay, with eager work in between."""
    import os
    torch, dev = torch_dev()
    p = problem("hpcg16")
    A = make_matrix(p)
    A.convert("dia")
    b = torch.from_numpy(p.b).to(dev)
    os.environ["DSM_CG_GRAPH"] = "0"
    xe, re = A.cg(b)
    xe = xe.cpu().numpy()
    try:
        for rep in range(3):
            os.environ["DSM_CG_GRAPH"] = "1"
            xg, rg = A.cg(b)
            assert rg["iters"] == re["iters"], rep
            assert np.array_equal(xg.cpu().numpy().view(np.uint64), xe.view(np.uint64)), rep
            os.environ["DSM_CG_GRAPH"] = "0"
            xe2, _ = A.cg(b)
            assert np.array_equal(xe2.cpu().numpy().view(np.uint64), xe.view(np.uint64)), rep
    finally:
        os.environ.pop("DSM_CG_GRAPH", None)
    A.close()


@pytest.mark.parametrize("fmt", ["dia", "ell"])
@pytest.mark.parametrize("variant", [0, 4, 9, 10])
def test_cg_fused_iteration_matches_oracle(fmt, variant):
    """DIA/ELL solves run the three-kernel loop whose SpMV also writes the
    p.q partials, or (DSM_CG_FUSED=1) the two-kernel loop that forms p on
    the fly; both pass the oracle checks and agree within +-1 iteration."""
    import os
    torch, dev = torch_dev()
    p = problem("hpcg16")
    xo, it, _, _ = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    A = make_matrix(p)
    A.convert(fmt)
    A.variant = variant
    b = torch.from_numpy(p.b).to(dev)
    xu, ru = A.cg(b)
    os.environ["DSM_CG_FUSED"] = "1"
    try:
        xf, rf = A.cg(b)
    finally:
        os.environ.pop("DSM_CG_FUSED", None)
    for x, r in ((xf, rf), (xu, ru)):
        xh = x.cpu().numpy()
        assert r["status"] == "converged" and abs(r["iters"] - it) <= 1, (r, it)
        assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh) <= 1.5e-10
        assert np.linalg.norm(xh - xo) <= 10 * KAPPA[16] * 1e-10 * np.linalg.norm(xo)
    A.close()


@pytest.mark.parametrize("fused", ["0", "1"])
def test_cg_fused_maxit_and_breakdown(fused):
    import os
    torch, dev = torch_dev()
    p = problem("hpcg16")
    A = make_matrix(p)
    A.convert("dia")
    os.environ["DSM_CG_FUSED"] = fused
    try:
        x, res = A.cg(torch.from_numpy(p.b).to(dev), maxit=5)
        assert res["status"] == "not_converged" and res["iters"] == 5
        x, res = A.cg(torch.from_numpy(p.b).to(dev), maxit=5, check_every=3)
        assert res["status"] == "not_converged" and res["iters"] == 5
        bb = p.b.copy()
        bb[100] = np.inf
        x, res = A.cg(torch.from_numpy(bb).to(dev))
        assert res["status"] == "breakdown"
    finally:
        os.environ.pop("DSM_CG_FUSED", None)
    A.close()


def test_values_exact_and_lossless_narrow_storage():
    """dsm_values_exact: the HPCG values (26, -1) survive a cast to FP32 and
    BF16, N(0,1) values do not; from FP32 storage BF16 is checked on the FP32
    words; widening is always exact.  FP64 CG over DIA values stored in BF16
    (exact) gives the iterates of FP64 storage bit for bit when the same
    sweep runs, and the oracle's iteration count."""
    torch, dev = torch_dev()
    p = problem("hpcg16")
    A = make_matrix(p)
    assert A.values_exact("f32") and A.values_exact("bf16") and A.values_exact("f64")
    q = inputs.banded_spd(2000, 8, seed=21)
    Q = make_matrix(q)
    assert not Q.values_exact("f32") and not Q.values_exact("bf16") and Q.values_exact("f64")
    for fmt in ("csr", "dia", "ell", "hyb", "hdc", "coo"):
        Q.convert(fmt)
        assert not Q.values_exact("bf16"), fmt
    Q.convert("csr", value_dtype="f32")
    assert Q.values_exact("f32") and Q.values_exact("f64") and not Q.values_exact("bf16")
    Q.close()
    b = torch.from_numpy(p.b).to(dev)
    _, it, _, _ = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    sols = []
    for vdt in ("f64", "bf16"):
        A.convert("dia", value_dtype=vdt)
        A.variant = 0
        x, res = A.cg(b, tol=1e-10)
        assert res["status"] == "converged" and abs(res["iters"] - it) <= 1, (vdt, res, it)
        sols.append((x.cpu().numpy(), res["iters"]))
    assert sols[0][1] == sols[1][1]
    assert np.array_equal(sols[0][0], sols[1][0])
    A.close()
