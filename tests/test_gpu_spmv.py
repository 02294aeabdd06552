"""SpMV parity: every format and kernel variant against the FP64 oracle,
entry by entry, row-scaled |y - y*| <= 1e-14 * sum_j |a_ij x_j| for FP64
(the oracle's compensated y* and row scale)."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import FORMATS, ctx, log, make_matrix, problem, row_scaled_err, torch_dev, x_for

pytestmark = pytest.mark.gpu

SMALL = ["hpcg2", "hpcg5", "hpcg16", "rect_empty", "rand_dense", "one_by_one", "no_entries", "long_row",
         "zipf50k", "banded20k"]


def run_formats(name, formats=FORMATS, tol=1e-14):
    torch, dev = torch_dev()
    p = problem(name)
    x = x_for(p)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x)
    A = make_matrix(p)
    xt = torch.from_numpy(x).to(dev)
    out = {}
    for f in formats:
        log(f"[spmv] {name} {f}")
        try:
            A.convert(f)
        except dsm.DsmError as e:  # infeasible padding is a legal outcome, asserted per case
            if e.status == dsm.L.E_INFEASIBLE:
                out[f] = "infeasible"
                continue
            raise
        variants = range(16) if f == "csr" else (range(64) if f in ("dia", "hdc") else (range(16) if f in ("ell", "hyb") else [0]))
        for v in variants:
            A.variant = v
            y = A.spmv(xt)
            torch.cuda.synchronize()
            err = row_scaled_err(y.cpu().numpy(), yref, scale)
            assert err <= tol, (name, f, v, err)
        out[f] = err
    A.close()
    return out


@pytest.mark.parametrize("name", SMALL)
def test_spmv_all_formats_small(name):
    out = run_formats(name)
    if name in ("hpcg16", "hpcg5", "rand_dense"):
        assert all(v != "infeasible" for v in out.values()), out


def test_spmv_hpcg104_all_formats():
    """The 104^3 HPCG problem (1,124,864 rows, 29,791,000 nnz), all six formats."""
    p = problem("hpcg104")
    assert p.nnz == 29_791_000
    out = run_formats("hpcg104")
    assert all(v != "infeasible" for v in out.values())


def test_spmv_zipf_1m():
    out = run_formats("zipf1m", formats=["csr", "coo", "hyb", "ell"])
    assert out["ell"] == "infeasible"  # K = longest row ~ 4096 pads far beyond 16x nnz


def test_spmv_banded_1m():
    run_formats("banded1m", formats=["csr", "coo", "hyb", "ell", "dia", "hdc"])


def test_spmv_repeatable_bitwise():
    """No atomics: two runs give identical bits, in every format."""
    torch, dev = torch_dev()
    p = problem("zipf50k")
    A = make_matrix(p)
    xt = torch.from_numpy(x_for(p)).to(dev)
    for f in ["coo", "csr", "hyb"]:
        A.convert(f)
        a = A.spmv(xt).cpu().numpy()
        b = A.spmv(xt).cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), f
    A.close()


@pytest.mark.parametrize("vdt", ["f32", "bf16"])
def test_spmv_reduced_precision_values(vdt):
    """Values stored in FP32/BF16: with FP64 vectors the result equals the
    FP64 product of the rounded values (row-scaled 1e-14); with FP32 vectors
    the FP32 accumulation error stays within (len_i + 2) * 2^-24 * S_i."""
    torch, dev = torch_dev()
    for name in ["hpcg16", "hpcg24", "rand_dense", "zipf50k", "long_row"]:
        p = problem(name)
        vals = oracle.cast_f32(p.val).astype(np.float64) if vdt == "f32" else oracle.bf16_to_f64(oracle.cast_bf16(p.val))
        x = x_for(p)
        x32 = x.astype(np.float32).astype(np.float64)
        yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, vals, x)
        yref32, scale32 = oracle.spmv_csr_ref(p.row_ptr, p.col, vals, x32)
        lens = np.diff(p.row_ptr)
        A = make_matrix(p)
        for f in FORMATS:
            try:
                A.convert(f, value_dtype=vdt)
            except dsm.DsmError as e:
                if e.status == dsm.L.E_INFEASIBLE:
                    continue
                raise
            log(f"[spmv-{vdt}] {name} {f}")
            # every sweep variant: the FP32/BF16 sweeps have interior paths of
            # their own (plain loads where a tile lies inside the matrix)
            variants = range(64) if f in ("dia", "hdc") else (range(16) if f in ("ell", "hyb") else [0])
            for v in variants:
                A.variant = v
                y = A.spmv(torch.from_numpy(x).to(dev)).cpu().numpy()
                assert row_scaled_err(y, yref, scale) <= 1e-14, (name, f, v)
                y32 = A.spmv(torch.from_numpy(x).to(dev).float()).cpu().numpy().astype(np.float64)
                bound = (lens + 2) * 2.0 ** -24 * scale32 + 2.0 ** -24 * np.abs(yref32)
                assert np.all(np.abs(y32 - yref32) <= bound + 1e-30), (name, f, v)
        A.close()


def test_spmv_eigenvector_pin():
    """A v = lambda v for the HPCG eigenvector, in every format."""
    import math
    torch, dev = torch_dev()
    n = 24
    p = problem(f"hpcg{n}")
    i = np.arange(1, n + 1)
    k = (3, 1, 2)
    vx, vy, vz = (np.sin(kd * math.pi * i / (n + 1)) for kd in k)
    v = np.einsum("k,j,i->kji", vz, vy, vx).ravel()
    lam = 27.0 - np.prod([1 + 2 * math.cos(kd * math.pi / (n + 1)) for kd in k])
    _, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, v)
    A = make_matrix(p)
    for f in FORMATS:
        A.convert(f)
        y = A.spmv(torch.from_numpy(v).to(dev)).cpu().numpy()
        assert np.max(np.abs(y - lam * v) / scale) <= 1e-14, f
    A.close()


@pytest.mark.parametrize("name", ["hpcg5", "rect_empty", "banded20k"])
def test_spmv_nonfinite_x_stays_in_its_rows(name):
    """Non-finite x entries reach exactly the rows that store an entry in
    their column: padding slots, slots past the last diagonal or ELL slot and
    entries past a row's end must not turn into 0 * Inf = NaN elsewhere.
    Rows that touch no non-finite column match the oracle (row-scaled 1e-14);
    rows that do are non-finite, with the sign of an infinite result fixed by
    the definition when the row sees only one infinity and no NaN."""
    torch, dev = torch_dev()
    p = problem(name)
    x = x_for(p).copy()
    bad = {0: np.inf, p.ncols - 1: np.nan, p.ncols // 2: -np.inf}
    for j, v in bad.items():
        x[j] = v
    clean = x.copy()
    for j in bad:
        clean[j] = 0.0
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, clean)
    touches = np.zeros(p.nrows, dtype=bool)
    expect_inf = np.zeros(p.nrows)
    for i in range(p.nrows):
        cols = p.col[p.row_ptr[i]:p.row_ptr[i + 1]]
        vals = p.val[p.row_ptr[i]:p.row_ptr[i + 1]]
        hit = [(c, v) for c, v in zip(cols, vals) if c in bad]
        touches[i] = bool(hit)
        if len(hit) == 1 and np.isinf(bad[hit[0][0]]):
            expect_inf[i] = np.sign(hit[0][1]) * np.sign(bad[hit[0][0]])
    assert touches.any() and (~touches).any()
    A = make_matrix(p)
    xt = torch.from_numpy(x).to(dev)
    for f in FORMATS:
        log(f"[spmv nonfinite] {name} {f}")
        try:
            A.convert(f)
        except dsm.DsmError as e:
            if e.status == dsm.L.E_INFEASIBLE:
                continue
            raise
        variants = range(16) if f == "csr" else (range(64) if f in ("dia", "hdc") else (range(16) if f in ("ell", "hyb") else [0]))
        for v in variants:
            A.variant = v
            y = A.spmv(xt).cpu().numpy()
            ok = ~touches
            assert np.all(np.isfinite(y[ok])), (name, f, v)
            assert row_scaled_err(y[ok], yref[ok], scale[ok]) <= 1e-14, (name, f, v)
            assert not np.any(np.isfinite(y[touches])), (name, f, v)
            sel = expect_inf != 0
            assert np.array_equal(np.sign(y[sel]), expect_inf[sel]), (name, f, v)
    A.close()


@pytest.mark.parametrize("name", ["hpcg16", "banded20k", "rect_empty"])
def test_spmv_nontemporal_variants_bitwise(name):
    """Bit 5 of a DIA/HDC variant changes only the cache hint of the value
    loads: y is bitwise the same as with the variant without it."""
    torch, dev = torch_dev()
    p = problem(name)
    A = make_matrix(p)
    xt = torch.from_numpy(x_for(p)).to(dev)
    for f in ("dia", "hdc"):
        try:
            A.convert(f)
        except dsm.DsmError as e:
            if e.status == dsm.L.E_INFEASIBLE:
                continue
            raise
        for v in range(32):
            A.variant = v
            a = A.spmv(xt).cpu().numpy()
            A.variant = v | 32
            b = A.spmv(xt).cpu().numpy()
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (name, f, v)
    A.close()


def test_spmv_kernel_time():
    """dsm_spmv_kernel_time computes the same y as dsm_spmv and times only
    the kernels: positive, and at most the event pair around the call on the
    same stream; 0 for a matrix with no rows."""
    torch, dev = torch_dev()
    p = problem("hpcg16")
    A = make_matrix(p)
    xt = torch.from_numpy(x_for(p)).to(dev)
    for f in FORMATS:
        A.convert(f)
        y1 = A.spmv(xt)
        y2 = torch.empty_like(y1)
        ks, es = [], []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            ks.append(A.kernel_time(xt, y2))
            b.record()
            torch.cuda.synchronize()
            es.append(a.elapsed_time(b) * 1e3)
        log(f"[kernel_time] {f}: kernel {np.median(ks):.2f} us, event pair {np.median(es):.2f} us")
        assert torch.equal(y1, y2), f
        assert all(k > 0 for k in ks) and np.median(ks) <= np.median(es), (f, ks, es)
    A.close()
    e = dsm.Matrix.from_csr(ctx(), 0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert e.kernel_time(torch.zeros(5, dtype=torch.float64, device=dev),
                         torch.zeros(0, dtype=torch.float64, device=dev)) == 0.0
    e.close()
