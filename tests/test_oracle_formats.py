"""Pins of the oracle's canonical encodings: a hand-worked example, closed
forms of the HPCG matrix, brute-force definitions on dense copies, and
round-trip identities on random patterns (hypothesis)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st

import inputs
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_gold():
    return json.load(open(os.path.join(GOLD, "worked_4x5.json")))


def dense_of(nrows, ncols, rp, col, val):
    return sp.csr_matrix((np.asarray(val, float), np.asarray(col), np.asarray(rp)), shape=(nrows, ncols)).toarray()


# ----------------------------------------------------------------- worked example
def test_worked_example_all_formats():
    g = load_gold()
    n, m = g["nrows"], g["ncols"]
    c = g["csr"]
    rp, col, val = (np.array(c[k]) for k in ("row_ptr", "col", "val"))
    assert oracle.csr_to_coo(rp).tolist() == g["coo"]["row"]
    offs, dv = oracle.csr_to_dia(n, m, rp, col, val)
    assert offs.tolist() == g["dia"]["offsets"] and dv.tolist() == g["dia"]["vals"]
    K, ec, ev = oracle.csr_to_ell(rp, col, val)
    assert K == g["ell"]["K"] and ec.tolist() == g["ell"]["col"] and ev.tolist() == g["ell"]["val"]
    h = oracle.csr_to_hyb(rp, col, val)
    gh = g["hyb"]
    assert h["Kh"] == gh["Kh"]
    for k in ("ell_col", "ell_val", "coo_row", "coo_col", "coo_val"):
        assert h[k].tolist() == gh[k], k
    d = oracle.csr_to_hdc(n, m, rp, col, val, theta=0.5)
    gd = g["hdc"]
    for k in ("offsets", "dia_val", "csr_row_ptr", "csr_col", "csr_val"):
        assert d[k].tolist() == gd[k], k
    x = np.array(g["x"], float)
    for y in (oracle.spmv_dia(n, m, offs, dv, x), oracle.spmv_ell(n, ec, ev, x),
              oracle.spmv_coo(n, g["coo"]["row"], g["coo"]["col"], g["coo"]["val"], x)):
        assert y.tolist() == g["y"]


# ----------------------------------------------------------------- HPCG closed forms
@pytest.mark.parametrize("n", [1, 2, 3, 5, 16])
def test_hpcg_dia_closed_forms(n):
    p = inputs.hpcg27(n)
    offs, dv = oracle.csr_to_dia(p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    expect = sorted({dx + n * dy + n * n * dz for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                     if n > 1 or (dx, dy, dz) == (0, 0, 0)})
    if n == 1:
        expect = [0]
    assert offs.tolist() == expect
    assert len(expect) == {1: 1, 2: 15}.get(n, 27)
    if n >= 3:
        assert math.isclose(np.count_nonzero(dv) / dv.size, (1 - 2 / (3 * n)) ** 3, rel_tol=1e-12)
    assert np.count_nonzero(dv) == p.nnz
    assert oracle.ell_width(p.row_ptr) == {1: 1, 2: 8}.get(n, 27)
    d = oracle.csr_to_hdc(p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    if n >= 5:  # every diagonal is at least half full from n = 5 on
        assert d["offsets"].tolist() == offs.tolist()
        assert d["csr_col"].size == 0
        assert np.array_equal(d["dia_val"], dv)
    else:
        D = dense_of(p.nrows, p.ncols, p.row_ptr, p.col, p.val)
        assert d["offsets"].tolist() == true_diags_bruteforce(D, 0.5)


def test_hpcg_hyb_width():
    """HPCG: rows of length 27 are (n-2)^3 >= N/3 for n >= 7 -> K_h = 27."""
    for n in (7, 16):
        p = inputs.hpcg27(n)
        h = oracle.csr_to_hyb(p.row_ptr, p.col, p.val)
        assert h["Kh"] == 27 and h["coo_row"].size == 0
    p = inputs.hpcg27(6)  # (4/6)^3 = 0.296 < 1/3 of rows reach 27
    assert oracle.hyb_width(p.row_ptr) < 27


def kh_bruteforce(lens):
    n = len(lens)
    need = math.ceil(n / 3)
    best = 0
    for k in range(0, max(lens, default=0) + 1):
        if sum(1 for l in lens if l >= k) >= need:
            best = k
    return best


def true_diags_bruteforce(D, theta):
    n, m = D.shape
    out = []
    for d in range(-(n - 1), m):
        pos = [(i, i + d) for i in range(n) if 0 <= i + d < m]
        cnt = sum(1 for i, j in pos if D[i, j] != 0)
        if cnt > 0 and cnt >= theta * len(pos):
            out.append(d)
    return out


# ----------------------------------------------------------------- property tests
shapes = st.tuples(st.integers(1, 40), st.integers(1, 40))


@settings(max_examples=60, deadline=None)
@given(shape=shapes, dens=st.floats(0.0, 1.0), seed=st.integers(0, 2 ** 32), er=st.sampled_from([0.0, 0.3]))
def test_roundtrips_and_definitions(shape, dens, seed, er):
    nr, nc = shape
    p = inputs.random_sparse(nr, nc, dens, seed, empty_rows=er)
    rp, col, val = p.row_ptr, p.col, p.val
    D = dense_of(nr, nc, rp, col, val)
    lens = np.diff(rp).tolist()
    x = inputs.uniform_vector(nc, seed=seed % 1000) - 0.5
    y = oracle.spmv_csr(rp, col, val, x)

    # COO: expansion and sort back (from a shuffled order)
    row = oracle.csr_to_coo(rp)
    assert np.array_equal(row, np.repeat(np.arange(nr), np.diff(rp)))
    perm = np.argsort(inputs.uniform(seed, 9, np.arange(row.size, dtype=np.uint64)))
    r2 = oracle.coo_to_csr(nr, nc, row[perm], col[perm], val[perm])
    assert all(np.array_equal(a, b) for a, b in zip(r2, (rp, col, val)))
    assert np.array_equal(oracle.spmv_coo(nr, row, col, val, x), y)

    # DIA: vals[k, i] = A(i, i + off_k) by definition
    offs, dv = oracle.csr_to_dia(nr, nc, rp, col, val)
    assert offs.tolist() == sorted({int(c) - i for i in range(nr) for c in col[rp[i]:rp[i + 1]]})
    for k, o in enumerate(offs):
        for i in range(nr):
            assert dv[k, i] == (D[i, i + o] if 0 <= i + o < nc else 0.0)
    back = oracle.dia_to_csr(nr, nc, offs, dv)
    assert all(np.array_equal(a, b) for a, b in zip(back, (rp, col, val)))
    assert np.array_equal(oracle.spmv_dia(nr, nc, offs, dv, x), y)

    # ELL
    K, ec, ev = oracle.csr_to_ell(rp, col, val)
    assert K == max(lens, default=0)
    for i in range(nr):
        js = np.flatnonzero(D[i])
        assert ec[: len(js), i].tolist() == js.tolist()
        assert (ec[len(js):, i] == -1).all() and (ev[len(js):, i] == 0).all()
    back = oracle.ell_to_csr(nr, ec, ev)
    assert all(np.array_equal(a, b) for a, b in zip(back, (rp, col, val)))
    assert np.array_equal(oracle.spmv_ell(nr, ec, ev, x), y)

    # HYB
    h = oracle.csr_to_hyb(rp, col, val)
    assert h["Kh"] == kh_bruteforce(lens)
    assert h["coo_row"].size == sum(max(0, l - h["Kh"]) for l in lens)
    back = oracle.hyb_to_csr(nr, h)
    assert all(np.array_equal(a, b) for a, b in zip(back, (rp, col, val)))

    # HDC
    for theta in (0.5, 0.0, 1.0):
        d = oracle.csr_to_hdc(nr, nc, rp, col, val, theta=theta)
        assert d["offsets"].tolist() == true_diags_bruteforce(D, theta)
        assert np.count_nonzero(d["dia_val"]) + d["csr_col"].size == rp[-1]
        back = oracle.hdc_to_csr(nr, nc, d)
        assert all(np.array_equal(a, b) for a, b in zip(back, (rp, col, val)))


def test_dia_drops_stored_zero_by_definition():
    """A stored zero is indistinguishable from DIA padding: CSR->DIA->CSR drops it."""
    rp, col, val = np.array([0, 2, 3]), np.array([0, 1, 1]), np.array([1.0, 0.0, 2.0])
    offs, dv = oracle.csr_to_dia(2, 2, rp, col, val)
    r2, c2, v2 = oracle.dia_to_csr(2, 2, offs, dv)
    assert r2.tolist() == [0, 1, 2] and c2.tolist() == [0, 1] and v2.tolist() == [1.0, 2.0]


def test_coo_duplicates_rejected():
    with pytest.raises(ValueError):
        oracle.coo_to_csr(2, 2, [0, 0], [1, 1], [1.0, 2.0])


def test_banded_hdc_keeps_only_main_diagonal():
    p = inputs.banded(nrows=20000, hbw=8, p=0.3, seed=4)
    offs = oracle.hdc_true_diags(p.nrows, p.ncols, p.row_ptr, p.col, 0.5)
    assert offs.tolist() == [0]
    assert oracle.dia_offsets(p.nrows, p.ncols, p.row_ptr, p.col).tolist() == list(range(-8, 9))


def test_dia_spmv_nonfinite_x_reaches_only_stored_entries():
    """A DIA zero slot (padding, or an entry the matrix does not store) is no
    entry: infinite and NaN x values reach exactly the rows that store a
    nonzero in their column, as the CSR definition gives, and the other rows
    keep their finite sums.  A dense product would spread 0 * Inf = NaN."""
    p = inputs.random_sparse(60, 70, 0.08, 31)
    x = inputs.uniform_vector(p.ncols, seed=4) - 0.5
    x[[3, 40]] = [np.inf, np.nan]
    x[p.ncols - 1] = -np.inf
    offs, dv = oracle.csr_to_dia(p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    y_dia = oracle.spmv_dia(p.nrows, p.ncols, offs, dv, x)
    y_csr = oracle.spmv_csr(p.row_ptr, p.col, p.val, x)
    np.testing.assert_array_equal(y_dia, y_csr)  # NaN where NaN, same infinities
    touch = np.array([bool(set(p.col[p.row_ptr[i]:p.row_ptr[i + 1]]) & {3, 40, p.ncols - 1})
                      for i in range(p.nrows)])
    assert touch.any() and (~touch).any()
    assert np.all(np.isfinite(y_dia[~touch])) and not np.any(np.isfinite(y_dia[touch]))
    dense = np.zeros((p.nrows, p.ncols))
    for i in range(p.nrows):
        dense[i, p.col[p.row_ptr[i]:p.row_ptr[i + 1]]] = p.val[p.row_ptr[i]:p.row_ptr[i + 1]]
    with np.errstate(invalid="ignore"):
        assert np.all(np.isnan(dense @ x))  # every row meets 0 * Inf in the dense product
