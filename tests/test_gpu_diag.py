"""Diagonal extraction/update in every format and Jacobi-preconditioned CG
against the oracle."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import FORMATS, ctx, log, make_matrix, problem, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["hpcg5", "rect_empty", "rand_dense", "long_row", "banded20k"])
def test_extract_and_update_every_format(name):
    torch, dev = torch_dev()
    p = problem(name)
    want = oracle.extract_diagonal(p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    present = np.zeros(want.size, bool)
    for i in range(want.size):
        seg = p.col[p.row_ptr[i]:p.row_ptr[i + 1]]
        present[i] = np.any(seg == i)
    newd = np.where(present, 3.0 + inputs.uniform_vector(want.size, seed=9), 0.0)
    v2, bad = oracle.update_diagonal(p.nrows, p.ncols, p.row_ptr, p.col, p.val, newd)
    assert bad == 0
    for f in FORMATS:
        A = make_matrix(p)
        try:
            A.convert(f, max_pad_ratio=1e4 if name in ("rect_empty",) else 16.0)
        except dsm.DsmError as e:
            assert e.status == dsm.L.E_INFEASIBLE
            A.close()
            continue
        log(f"[diag] {name} {f}")
        got = A.diagonal().cpu().numpy()
        assert np.array_equal(got, want), (name, f)
        A.set_diagonal(torch.from_numpy(newd).to(dev))
        A.convert("csr")
        ex = A.export()
        if f in ("dia", "hdc"):
            # a diagonal slot set to 0 disappears on the way back (padding rule)
            keep = v2 != 0
            assert np.array_equal(ex["val"], v2[keep]) or np.array_equal(ex["val"], v2)
        else:
            assert np.array_equal(ex["col"], p.col) and np.array_equal(ex["val"], v2), (name, f)
        if (~present).any():
            bad_d = newd.copy()
            bad_d[np.flatnonzero(~present)[0]] = 1.0
            with pytest.raises(dsm.DsmError) as e:
                A.set_diagonal(torch.from_numpy(bad_d).to(dev))
            assert e.value.status == dsm.L.E_INVALID
            assert np.array_equal(A.export()["val"], ex["val"])
        A.close()


def scaled_spd(N=20000, hbw=12, seed=31):
    p = inputs.banded_spd(N, hbw, seed=seed)
    rows = np.repeat(np.arange(N), np.diff(p.row_ptr))
    scale = 1.0 + 50.0 * inputs.uniform_vector(N, seed=seed)
    val = p.val.copy()
    val[rows == p.col] *= scale
    b = np.bincount(rows, weights=val, minlength=N)
    return p, val, b


@pytest.mark.parametrize("fmt", ["csr", "dia", "hyb"])
def test_jacobi_pcg_matches_oracle(fmt):
    torch, dev = torch_dev()
    p, val, b = scaled_spd()
    xo, it, _, st = oracle.pcg_jacobi(p.row_ptr, p.col, val, b, tol=1e-10)
    xp, itp, _, _ = oracle.cg(p.row_ptr, p.col, val, b, tol=1e-10)
    A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, val)
    A.convert(fmt)
    x, res = A.cg(torch.from_numpy(b).to(dev), tol=1e-10, mode="jacobi")
    log(f"[pcg] {fmt}: jacobi {res['iters']} (oracle {it}), plain oracle {itp}")
    assert res["status"] == "converged" and abs(res["iters"] - it) <= 1
    assert oracle.true_relres(p.row_ptr, p.col, val, b, x.cpu().numpy()) <= 1.5e-10
    assert it < itp  # the preconditioner pays off on this matrix
    A.close()


@pytest.mark.parametrize("fmt", ["csr", "dia"])
def test_jacobi_pcg_graph_matches_eager(fmt, monkeypatch):
    """The Jacobi loop replayed from a captured graph (on a workspace copy of
    x, reused by a second solve into a new x) gives the eager launches'
    bits and iteration count."""
    torch, dev = torch_dev()
    p, val, b = scaled_spd()
    A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, val)
    A.convert(fmt)
    bd = torch.from_numpy(b).to(dev)
    monkeypatch.setenv("DSM_CG_GRAPH", "0")
    xe, re = A.cg(bd, tol=1e-10, mode="jacobi")
    xe = xe.cpu().numpy()
    monkeypatch.setenv("DSM_CG_GRAPH", "1")
    for rep in range(2):
        xg, rg = A.cg(bd, x=torch.zeros(p.nrows, dtype=torch.float64, device=dev), tol=1e-10, mode="jacobi")
        assert rg["iters"] == re["iters"] and rg["status"] == "converged", (rep, rg, re)
        assert np.array_equal(xg.cpu().numpy().view(np.uint64), xe.view(np.uint64)), rep
    A.close()


def test_jacobi_pcg_hpcg_equals_plain():
    torch, dev = torch_dev()
    p = problem("hpcg16")
    A = make_matrix(p)
    b = torch.from_numpy(p.b).to(dev)
    _, r1 = A.cg(b, mode="jacobi")
    _, r2 = A.cg(b)
    assert abs(r1["iters"] - r2["iters"]) <= 1
    z = dsm.Matrix.from_csr(ctx(), 3, 3, [0, 1, 1, 2], [0, 2], [1.0, 1.0])
    with pytest.raises(dsm.DsmError):
        z.cg(torch.ones(3, dtype=torch.float64, device=dev), mode="jacobi", raise_on_status=True)
    z.close()
    A.close()
