"""One rank's local/remote split (Section V-A, Fig. 2; Section V-E): the
merged rank matrix is irregular (DIA refuses it), while a regular local
block plus an irregular ghost block, each in its own format and added into
one y, reproduces the merged SpMV of the oracle."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import FORMATS, ctx, log, row_scaled_err, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("procs,coords", [((3, 3, 3), (1, 1, 1)), ((2, 2, 2), (0, 0, 0)), ((4, 1, 2), (2, 0, 1))])
def test_split_spmv_matches_merged(procs, coords):
    torch, dev = torch_dev()
    n = 12
    merged, local, ghost = inputs.hpcg27_rank(n, procs, coords)
    x = inputs.uniform_vector(merged.ncols, seed=5) - 0.5
    yref, scale = oracle.spmv_csr_ref(merged.row_ptr, merged.col, merged.val, x)
    M = dsm.Matrix.from_csr(ctx(), merged.nrows, merged.ncols, merged.row_ptr, merged.col, merged.val)
    with pytest.raises(dsm.DsmError) as e:
        M.convert("dia")  # the ghost columns scatter the diagonals
    assert e.value.status == dsm.L.E_INFEASIBLE
    xt = torch.from_numpy(x).to(dev)
    assert row_scaled_err(M.spmv(xt).cpu().numpy(), yref, scale) <= 1e-14
    L = dsm.Matrix.from_csr(ctx(), local.nrows, local.ncols, local.row_ptr, local.col, local.val)
    G = dsm.Matrix.from_csr(ctx(), ghost.nrows, ghost.ncols, ghost.row_ptr, ghost.col, ghost.val)
    xl, xg = xt[: local.ncols].contiguous(), xt[local.ncols:].contiguous()
    for fl in ("dia", "csr", "ell"):
        L.convert(fl)
        for fg in FORMATS:
            try:
                G.convert(fg)
            except dsm.DsmError as err:
                assert err.status == dsm.L.E_INFEASIBLE
                continue
            log(f"[split] {procs} {coords} local {fl} ghost {fg}")
            y = L.spmv(xl)
            G.spmv_accumulate(xg, y)
            assert row_scaled_err(y.cpu().numpy(), yref, scale) <= 1e-14, (fl, fg)
    # per-part selection
    rl, rg = L.select(use_cache=False), G.select(use_cache=False)
    log(f"[split] chosen local {rl['chosen']} ghost {rg['chosen']}")
    y = L.spmv(xl)
    G.spmv_accumulate(xg, y)
    assert row_scaled_err(y.cpu().numpy(), yref, scale) <= 1e-14
    for A in (M, L, G):
        A.close()


def test_spmv_accumulate_every_format():
    torch, dev = torch_dev()
    p = inputs.random_sparse(300, 200, 0.05, 21, empty_rows=0.2)
    x = inputs.uniform_vector(p.ncols, seed=2)
    y0 = inputs.uniform_vector(p.nrows, seed=3)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x)
    A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    for f in FORMATS:
        A.convert(f, max_pad_ratio=1e4)
        y = torch.from_numpy(y0.copy()).to(dev)
        A.spmv_accumulate(torch.from_numpy(x).to(dev), y)
        assert row_scaled_err(y.cpu().numpy() - y0, yref, scale + np.abs(y0)) <= 2e-14, f
    A.close()
