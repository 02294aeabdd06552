"""Conversion parity: every on-device conversion, exported, is bit-identical
to the oracle's canonical encoding, and converting back to CSR gives the
original arrays bit for bit."""
import numpy as np
import pytest

import oracle
import paper_2209_06478_amd as dsm
from gpu_common import FORMATS, log, make_matrix, problem

pytestmark = pytest.mark.gpu

CASES = ["hpcg2", "hpcg5", "hpcg16", "rect_empty", "rand_dense", "one_by_one", "no_entries", "long_row",
         "zipf50k", "banded20k"]


def eq(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and a.dtype.itemsize == b.dtype.itemsize and np.array_equal(
        a.view(f"u{a.dtype.itemsize}"), b.view(f"u{b.dtype.itemsize}"))


def expected(p, f):
    n, m = p.nrows, p.ncols
    if f == "csr":
        return dict(row_ptr=p.row_ptr, col=p.col, val=p.val)
    if f == "coo":
        return dict(row=oracle.csr_to_coo(p.row_ptr), col=p.col, val=p.val)
    if f == "dia":
        offs, dv = oracle.csr_to_dia(n, m, p.row_ptr, p.col, p.val)
        return dict(offsets=offs, dia_val=dv)
    if f == "ell":
        K, ec, ev = oracle.csr_to_ell(p.row_ptr, p.col, p.val)
        return dict(ell_col=ec, ell_val=ev)
    if f == "hyb":
        h = oracle.csr_to_hyb(p.row_ptr, p.col, p.val)
        return dict(ell_col=h["ell_col"], ell_val=h["ell_val"], coo_row=h["coo_row"], coo_col=h["coo_col"],
                    coo_val=h["coo_val"])
    if f == "hdc":
        h = oracle.csr_to_hdc(n, m, p.row_ptr, p.col, p.val, 0.5)
        return dict(offsets=h["offsets"], dia_val=h["dia_val"], row_ptr=h["csr_row_ptr"], col=h["csr_col"],
                    val=h["csr_val"])


# formats whose padding exceeds the default guard (16 x nnz) on a case
INFEASIBLE = {"rect_empty": {"dia"}, "long_row": {"dia", "ell"}, "zipf50k": {"dia", "ell"},
              "zipf1m": {"dia", "ell"}}


def check_case(name, formats=FORMATS):
    p = problem(name)
    A = make_matrix(p)
    for f in formats:
        log(f"[convert] {name} csr->{f}->csr")
        if f in INFEASIBLE.get(name, ()):
            with pytest.raises(dsm.DsmError) as e:
                A.convert(f)
            assert e.value.status == dsm.L.E_INFEASIBLE and A.format == "csr"
            if name != "rect_empty":
                continue
            A.convert(f, max_pad_ratio=1e4)  # small enough to build anyway
        else:
            A.convert(f)
        exp = expected(p, f)
        got = A.export()
        for k, v in exp.items():
            assert eq(got[k], v), (name, f, k)
        info = A.info()
        if f in ("ell", "hyb"):
            assert info["ell_width"] == exp["ell_col"].shape[0]
        if f in ("dia", "hdc"):
            assert info["ndiag"] == exp["offsets"].size
        A.convert("csr")
        back = A.export()
        for k, v in dict(row_ptr=p.row_ptr, col=p.col, val=p.val).items():
            assert eq(back[k], v), (name, f, "roundtrip", k)
    A.close()


@pytest.mark.parametrize("name", CASES)
def test_convert_exact(name):
    check_case(name)


def test_convert_exact_hpcg104():
    check_case("hpcg104")


def test_convert_exact_banded_1m():
    check_case("banded1m", formats=["coo", "dia", "hyb", "hdc"])


def test_convert_exact_zipf_1m():
    check_case("zipf1m", formats=["coo", "hyb", "hdc"])


def test_convert_between_non_csr_formats():
    """X -> Y directly (through the CSR hub) equals the canonical Y."""
    p = problem("rand_dense")
    A = make_matrix(p)
    for a, b in [("coo", "hyb"), ("hyb", "dia"), ("dia", "ell"), ("ell", "hdc"), ("hdc", "coo")]:
        A.convert(a)
        A.convert(b)
        got = A.export()
        for k, v in expected(p, b).items():
            assert eq(got[k], v), (a, b, k)
    A.close()


@pytest.mark.parametrize("vdt", ["f32", "bf16"])
def test_value_casts_exact(vdt):
    p = problem("zipf50k")
    A = make_matrix(p)
    A.convert("csr", value_dtype=vdt)
    got = A.export()
    want = oracle.cast_f32(p.val) if vdt == "f32" else oracle.cast_bf16(p.val)
    assert eq(got["val"], want)
    A.convert("hyb")
    h = oracle.csr_to_hyb(p.row_ptr, p.col, p.val)
    cast = oracle.cast_f32 if vdt == "f32" else oracle.cast_bf16
    assert eq(A.export()["coo_val"], cast(h["coo_val"]))
    assert eq(A.export()["ell_val"], cast(h["ell_val"].ravel()).reshape(h["ell_val"].shape))
    A.close()


def test_hdc_theta_and_hyb_width_options():
    p = problem("banded20k")
    A = make_matrix(p)
    for theta in (0.25, 0.5, 1.0):
        A.convert("hdc", hdc_theta=theta)
        h = oracle.csr_to_hdc(p.nrows, p.ncols, p.row_ptr, p.col, p.val, theta)
        got = A.export()
        assert eq(got["offsets"], h["offsets"]) and eq(got["col"], h["csr_col"]), theta
        assert A.info()["hdc_theta"] == theta
    A.convert("hyb", hyb_width=5)
    h = oracle.csr_to_hyb(p.row_ptr, p.col, p.val, Kh=5)
    got = A.export()
    assert eq(got["ell_col"], h["ell_col"]) and eq(got["coo_val"], h["coo_val"])
    A.close()


def test_create_from_coo_sorted_and_unsorted():
    import inputs
    p = problem("long_row")
    row = oracle.csr_to_coo(p.row_ptr)
    ctx = dsm.Context(0)
    A = dsm.Matrix.from_coo(ctx, p.nrows, p.ncols, row, p.col, p.val, sorted=True)
    got = A.export()
    assert eq(got["row_ptr"], p.row_ptr) and eq(got["col"], p.col) and eq(got["val"], p.val)
    A.close()
    perm = np.argsort(inputs.uniform(3, 3, np.arange(row.size, dtype=np.uint64)))
    B = dsm.Matrix.from_coo(ctx, p.nrows, p.ncols, row[perm], p.col[perm], p.val[perm], sorted=False)
    got = B.export()
    assert eq(got["row_ptr"], p.row_ptr) and eq(got["col"], p.col) and eq(got["val"], p.val)
    B.close()
    ctx.close()


def test_row_stats_match_oracle():
    for name in ["zipf50k", "rect_empty", "hpcg16"]:
        p = problem(name)
        A = make_matrix(p)
        for f in ["csr", "hyb"]:
            A.convert(f)
            got = A.row_stats()
            exp = oracle.row_stats(p.row_ptr)
            for k in ("max", "min", "sum", "sumsq", "empty"):
                assert got[k] == exp[k], (name, f, k)
            assert np.array_equal(got["hist"], exp["hist"])
        A.close()
