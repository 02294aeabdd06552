"""Error paths at the boundary: malformed inputs, budget exhaustion with a
transactional convert, infeasible padding."""
import numpy as np
import pytest

import oracle
import paper_2209_06478_amd as dsm
from gpu_common import log, make_matrix, problem, row_scaled_err, torch_dev, x_for

pytestmark = pytest.mark.gpu


def test_invalid_csr_rejected():
    ctx = dsm.Context(0)
    bad = [
        ([1, 2, 3], [0, 1, 1]),      # row_ptr[0] != 0
        ([0, 2, 3], [0, 1]),         # row_ptr[n] != nnz
        ([0, 2, 3], [1, 0, 1]),      # unsorted row
        ([0, 2, 3], [1, 1, 1]),      # duplicate
        ([0, 2, 3], [0, 5, 1]),      # column out of range
        ([0, 3, 2], [0, 1, 1]),      # decreasing pointers
    ]
    for rp, col in bad:
        log(f"[errors] invalid csr {rp} {col}")
        with pytest.raises(dsm.DsmError) as e:
            dsm.Matrix.from_csr(ctx, 2, 2, rp, col, np.ones(len(col)))
        assert e.value.status == dsm.L.E_INVALID, (rp, col)
    with pytest.raises(dsm.DsmError) as e:
        dsm.Matrix.from_coo(ctx, 2, 2, [0, 0], [1, 1], [1.0, 2.0], sorted=False)
    assert e.value.status == dsm.L.E_INVALID
    assert ctx.bytes_in_use() == 0


def test_budget_exhaustion_keeps_old_format():
    torch, dev = torch_dev()
    p = problem("hpcg16")
    x = x_for(p)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x)
    ctx0 = dsm.Context(0)
    A0 = dsm.Matrix.from_csr(ctx0, p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    csr_bytes = A0.info()["bytes"]
    A0.close()
    ctx0.close()
    ctx = dsm.Context(0, hbm_budget=int(csr_bytes * 1.5))
    A = dsm.Matrix.from_csr(ctx, p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    before = ctx.bytes_in_use()
    assert before >= A.info()["bytes"]
    with pytest.raises(dsm.DsmError) as e:
        A.convert("coo")  # COO + CSR together exceed the budget
    assert e.value.status == dsm.L.E_NOMEM
    assert A.format == "csr"
    assert ctx.bytes_in_use() == before  # the failed build released what it had taken
    y = A.spmv(torch.from_numpy(x).to(dev)).cpu().numpy()
    assert row_scaled_err(y, yref, scale) <= 1e-14
    A.close()
    ctx.close()


def test_infeasible_padding():
    p = problem("zipf50k")
    A = make_matrix(p)
    with pytest.raises(dsm.DsmError) as e:
        A.convert("dia")
    assert e.value.status == dsm.L.E_INFEASIBLE
    assert A.format == "csr"
    A.convert("ell", max_pad_ratio=1000.0)
    assert A.info()["ell_width"] == oracle.ell_width(p.row_ptr)
    A.close()


def test_spmv_argument_checks():
    torch, dev = torch_dev()
    p = problem("hpcg5")
    A = make_matrix(p)
    x = torch.ones(p.ncols, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        A.spmv(torch.ones(p.ncols + 1, dtype=torch.float64, device=dev))
    with pytest.raises(dsm.DsmError):
        A.spmv(x, out=x) if p.nrows == p.ncols else None
    A.close()
