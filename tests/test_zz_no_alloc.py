"""The allocation-free SpMV entry point (dsm_spmv_noalloc) against dsm_spmv:
same result bit for bit, and within the oracle's row-scaled 1e-14 for FP64
vectors, on two calls in a row where the second has the smaller input; no
bytes allocated through the context; a COO part beyond the static buffer is
refused before any launch."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import log, row_scaled_err, torch_dev, x_for

pytestmark = pytest.mark.gpu


def _case(c, p, fmt, vec, torch, dev):
    """One allocation-free call, then the allocating entry point on the same
    input; returns (x, noalloc y, spmv y)."""
    A = dsm.Matrix.from_csr(c, p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    A.convert(fmt)
    x = x_for(p)
    tdt = torch.float64 if vec == "f64" else torch.float32
    xt = torch.from_numpy(x).to(dev).to(tdt)
    y1 = torch.full((p.nrows,), float("nan"), dtype=tdt, device=dev)
    y2 = torch.full((p.nrows,), float("nan"), dtype=tdt, device=dev)
    torch.cuda.synchronize()
    before = c.bytes_in_use()
    log(f"[noalloc] {p.name} {fmt} {vec} rows={p.nrows} nnz={p.col.size}")
    A.spmv_noalloc(xt, y1)
    torch.cuda.synchronize()
    assert c.bytes_in_use() == before, "the allocation-free call allocated through the context"
    A.spmv(xt, out=y2)
    torch.cuda.synchronize()
    A.close()
    return x, y1.cpu().numpy(), y2.cpu().numpy()


@pytest.mark.parametrize("vec", ["f64", "f32"])
@pytest.mark.parametrize("fmt", ["coo", "hyb", "csr", "dia"])
def test_noalloc_matches_spmv_twice(fmt, vec):
    """A larger matrix, then a smaller one: the second call reuses the
    static buffer that still holds the first call's partials."""
    torch, dev = torch_dev()
    c = dsm.Context(0)
    big = inputs.zipf(nrows=50000, seed=5) if fmt in ("coo", "hyb") else inputs.hpcg27(24)
    small = inputs.hpcg27(5)
    for p in (big, small):
        x, y1, y2 = _case(c, p, fmt, vec, torch, dev)
        assert np.array_equal(y1.view(np.uint8), y2.view(np.uint8)), (p.name, fmt, vec)
        if vec == "f64":
            yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x)
            assert row_scaled_err(y1, yref, scale) <= 1e-14, (p.name, fmt)
        else:
            # FP32 accumulation of exact products of the rounded x
            x32 = x.astype(np.float32).astype(np.float64)
            yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x32)
            bound = (np.diff(p.row_ptr) + 2) * 2.0 ** -24 * scale + 2.0 ** -24 * np.abs(yref)
            assert np.all(np.abs(y1.astype(np.float64) - yref) <= bound + 1e-30), (p.name, fmt)
    assert c.bytes_in_use() == 0
    c.close()


def test_noalloc_refuses_coo_beyond_the_buffer():
    """A COO matrix of 34,000,000 entries needs 132,813 tiles x 16 bytes of
    FP64 partials (2,125,008 > 2 MiB): refused with DSM_E_NOMEM and y left
    as it was; the same matrix with FP32 vectors (8 bytes a tile) fits and
    matches dsm_spmv."""
    torch, dev = torch_dev()
    c = dsm.Context(0)
    n = 34_000_000
    idx = torch.arange(n, dtype=torch.int32, device=dev)
    val = (idx % 7 + 1).to(torch.float64)
    A = dsm.Matrix.from_coo(c, n, n, idx, idx, val)
    A.convert("coo")
    x = torch.ones(n, dtype=torch.float64, device=dev)
    y = torch.full((n,), -3.0, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    with pytest.raises(dsm.DsmError) as e:
        A.spmv_noalloc(x, y)
    assert e.value.status == dsm.L.E_NOMEM
    torch.cuda.synchronize()
    assert bool((y == -3.0).all())
    x32 = x.float()
    y1 = torch.empty(n, dtype=torch.float32, device=dev)
    y2 = torch.empty(n, dtype=torch.float32, device=dev)
    A.spmv_noalloc(x32, y1)
    A.spmv(x32, out=y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    assert torch.equal(y1, val.float())
    A.close()
    del idx, val, x, y, x32, y1, y2
    assert c.bytes_in_use() == 0
    c.close()
