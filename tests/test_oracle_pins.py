"""Pins of the FP64 oracle against things other than itself: closed forms of
the HPCG problem, dense brute force, exact rational arithmetic, library
routines (numpy, scipy, torch CPU) and a hand-worked example."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import inputs
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense(p):
    return sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(p.nrows, p.ncols)).toarray()


# ----------------------------------------------------------------- generator
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 16])
def test_hpcg_closed_forms(n):
    """nnz = (3n-2)^3; b_i = 27 - nnz_i by row class (interior/face/edge/corner)."""
    p = inputs.hpcg27(n)
    assert p.nrows == n ** 3
    assert p.nnz == (3 * n - 2) ** 3
    assert oracle.csr_validate(p.nrows, p.ncols, p.row_ptr, p.col) == 0
    vals, cnts = np.unique(p.b, return_counts=True)
    expect = {}
    if n >= 3:
        expect[0.0] = (n - 2) ** 3
        expect[9.0] = 6 * (n - 2) ** 2
        expect[15.0] = 12 * (n - 2)
        expect[19.0] = 8
    elif n == 2:
        expect[19.0] = 8
    else:
        expect[26.0] = 1
    assert dict(zip(vals.tolist(), cnts.tolist())) == expect


def test_aniso7_closed_forms():
    n = 6
    p = inputs.aniso7(n)
    assert p.nnz == n ** 3 * 7 - 6 * n * n
    assert set(np.unique(p.val).tolist()) == {204.0, -1.0, -100.0}
    D = dense(p)
    assert np.array_equal(D, D.T)
    assert np.linalg.eigvalsh(D).min() > 0


# ----------------------------------------------------------------- SpMV
def row_scaled_err(y, yref, scale):
    return np.max(np.abs(y - yref) / np.maximum(scale, 1e-300))


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_spmv_vs_dense_hpcg(n):
    p = inputs.hpcg27(n)
    x = inputs.uniform_vector(p.nrows, seed=n)
    y = oracle.spmv_csr(p.row_ptr, p.col, p.val, x)
    yd = dense(p) @ x
    _, s = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x)
    assert row_scaled_err(y, yd, s) <= 1e-14


@pytest.mark.parametrize("shape,dens,seed", [((64, 64), 0.1, 1), ((37, 53), 0.3, 2), ((50, 20), 0.05, 3),
                                             ((1, 1), 1.0, 4), ((64, 64), 0.9, 5)])
def test_spmv_vs_dense_random(shape, dens, seed):
    """Non-symmetric random matrices: a transposed operand would fail here."""
    p = inputs.random_sparse(shape[0], shape[1], dens, seed, empty_rows=0.1)
    x = inputs.uniform_vector(p.ncols, seed=seed) - 0.5
    y = oracle.spmv_csr(p.row_ptr, p.col, p.val, x)
    D = dense(p)
    _, s = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x)
    assert row_scaled_err(y, D @ x, s) <= 1e-14
    if shape[0] == shape[1] and shape[0] > 1:
        assert not np.allclose(D, D.T)  # a transposed operand would change y


@pytest.mark.parametrize("n", [5, 9])
def test_spmv_eigenpairs(n):
    """A = 27 I - T(x)T(x)T with T = tridiag(1,1,1): A v = lambda v for
    v = sin(k pi i/(n+1)) per axis, lambda = 27 - prod(1 + 2 cos(k pi/(n+1)))."""
    p = inputs.hpcg27(n)
    i = np.arange(1, n + 1)
    for k in [(1, 1, 1), (2, 3, 1), (n, n - 1, 2)]:
        vx, vy, vz = (np.sin(kd * math.pi * i / (n + 1)) for kd in k)
        v = np.einsum("k,j,i->kji", vz, vy, vx).ravel()  # x fastest
        lam = 27.0 - np.prod([1 + 2 * math.cos(kd * math.pi / (n + 1)) for kd in k])
        y = oracle.spmv_csr(p.row_ptr, p.col, p.val, v)
        _, s = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, v)
        assert np.max(np.abs(y - lam * v) / (s + 1e-300)) <= 1e-14


def test_aniso7_eigenpair():
    n = 7
    p = inputs.aniso7(n)
    i = np.arange(1, n + 1)
    k = (2, 1, 3)
    vx, vy, vz = (np.sin(kd * math.pi * i / (n + 1)) for kd in k)
    v = np.einsum("k,j,i->kji", vz, vy, vx).ravel()
    lam = sum(w * 4 * math.sin(kd * math.pi / (2 * (n + 1))) ** 2 for w, kd in zip((1, 1, 100), k))
    y = oracle.spmv_csr(p.row_ptr, p.col, p.val, v)
    _, s = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, v)
    assert np.max(np.abs(y - lam * v) / (s + 1e-300)) <= 1e-13


def test_compensated_reference_vs_exact_rationals():
    """Dot2 must agree with the exactly rounded sum up to ~2u|y| + O(u^2) S."""
    p = inputs.random_sparse(40, 300, 0.5, 11)
    x = (inputs.uniform_vector(300, seed=5) - 0.5) * 1e3
    yref, s = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x)
    u = 2.0 ** -53
    for r in range(p.nrows):
        lo, hi = p.row_ptr[r], p.row_ptr[r + 1]
        ex = sum((Fraction(float(a)) * Fraction(float(x[c])) for a, c in zip(p.val[lo:hi], p.col[lo:hi])),
                 Fraction(0))
        exf = float(ex)
        assert abs(yref[r] - exf) <= 2 * u * abs(exf) + 1e-28 * s[r]
        sab = float(sum(abs(Fraction(float(a)) * Fraction(float(x[c]))) for a, c in zip(p.val[lo:hi], p.col[lo:hi])))
        assert abs(s[r] - sab) <= 1e-13 * sab + 1e-300


def test_worked_example_spmv_and_stats():
    g = json.load(open(os.path.join(GOLD, "worked_4x5.json")))
    c = g["csr"]
    y = oracle.spmv_csr(c["row_ptr"], c["col"], c["val"], g["x"])
    assert y.tolist() == g["y"]
    st = oracle.row_stats(c["row_ptr"])
    for k in ("max", "min", "sum", "sumsq", "empty"):
        assert st[k] == g["row_stats"][k]
    assert st["hist"][:3].tolist() == g["row_stats"]["hist_first3"]
    assert st["hist"][3:].sum() == 0


def test_row_stats_vs_numpy():
    z = inputs.zipf(nrows=20000, seed=3)
    st = oracle.row_stats(z.row_ptr)
    lens = np.diff(z.row_ptr).astype(np.int64)
    assert st["max"] == lens.max() and st["min"] == lens.min() and st["sum"] == lens.sum()
    assert st["sumsq"] == (lens * lens).sum() and st["empty"] == (lens == 0).sum()
    bins = np.where(lens == 0, 0, np.floor(np.log2(np.maximum(lens, 1))).astype(np.int64) + 1)
    assert np.array_equal(st["hist"], np.bincount(bins, minlength=33))


# ----------------------------------------------------------------- validation
def test_csr_validation_codes():
    rp, col = [0, 2, 3], [0, 1, 1]
    assert oracle.csr_validate(2, 2, rp, col) == 0
    assert oracle.csr_validate(2, 2, [1, 2, 3], col) == 2
    assert oracle.csr_validate(2, 2, [0, 2, 2], col) == 3
    assert oracle.csr_validate(2, 2, [0, 3, 3], [0, 1, 1]) == 6       # duplicate / unsorted
    assert oracle.csr_validate(2, 2, [0, 2, 3], [0, 2, 1]) == 5       # column out of range
    assert oracle.csr_validate(2, 2, [0, 2, 1], [0, 1, 1]) in (3, 4)  # decreasing pointers


# ----------------------------------------------------------------- casts
def test_cast_f32_matches_numpy():
    v = np.concatenate([inputs.normal(7, 1, np.arange(10000, dtype=np.uint64)) * 10.0 ** np.arange(-5, 5).repeat(1000),
                        [0.0, -0.0, np.inf, -np.inf, 1e300, -1e-300, 3.4028235677973366e38]])
    with np.errstate(over="ignore"):
        ref = v.astype(np.float32)
    assert np.array_equal(oracle.cast_f32(v).view(np.uint32), ref.view(np.uint32))


def test_cast_bf16_matches_torch_rne():
    torch = pytest.importorskip("torch")
    base = inputs.normal(9, 1, np.arange(20000, dtype=np.uint64))
    f = base.astype(np.float32)
    bits = f.view(np.uint32)
    # exact ties between two bf16 neighbours, with even and odd kept parts
    ties = ((bits[:2000] & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)
    v = np.concatenate([base, ties.astype(np.float64), [0.0, -0.0, np.inf, -np.inf, 1.0, -3.0]])
    ours = oracle.cast_bf16(v)
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    back = oracle.bf16_to_f64(ours)
    assert np.array_equal(back, torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).float().double().numpy())


def test_cast_bf16_nan_stays_nan():
    out = oracle.bf16_to_f64(oracle.cast_bf16(np.array([np.nan, -np.nan])))
    assert np.isnan(out).all()


# ----------------------------------------------------------------- CG
def test_cg_n1_and_n2_one_iteration():
    for n in (1, 2):
        p = inputs.hpcg27(n)
        x, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, p.b)
        assert st == "converged" and it == 1
        assert np.max(np.abs(x - 1.0)) <= 1e-15


def test_cg_b_zero():
    p = inputs.hpcg27(3)
    x, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, np.zeros(p.nrows))
    assert st == "converged" and it == 0 and not x.any()


@pytest.mark.parametrize("n", [3, 4])
def test_cg_vs_dense_solve(n):
    p = inputs.hpcg27(n)
    b = inputs.uniform_vector(p.nrows, seed=n) - 0.3
    x, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, b, tol=1e-13)
    xs = np.linalg.solve(dense(p), b)
    assert st == "converged"
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


@pytest.mark.parametrize("n,anchor", [(3, 4), (8, 13), (16, 27), (32, 54), (64, 105)])
def test_cg_iteration_anchors(n, anchor):
    """Iterations to 1e-10 within +-1 of an independent plain CG (scipy), and
    of the anchors 4/13/27/54/105; x close to ones within 10*kappa*tol."""
    p = inputs.hpcg27(n)
    x, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    assert st == "converged"
    assert abs(it - anchor) <= 1
    A = sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(p.nrows, p.nrows))
    count = [0]
    spla.cg(A, p.b, x0=np.zeros(p.nrows), rtol=1e-10, atol=0.0, maxiter=10000,
            callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert abs(it - count[0]) <= 1
    tr = oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x)
    assert tr <= 1.5e-10
    kappa = {3: 2.28, 8: 10.96, 16: 39.05, 32: 147.1, 64: 570.8}[n]
    assert np.linalg.norm(x - 1) <= 10 * kappa * 1e-10 * np.linalg.norm(np.ones(p.nrows))


def test_cg_breakdown_and_maxit():
    n = 10
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    x, it, rr, st = oracle.cg(rp, col, -np.ones(n), np.ones(n))
    assert st == "breakdown" and it == 1
    p = inputs.hpcg27(8)
    x, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, maxit=3)
    assert st == "not_converged" and it == 3 and rr > 1e-10
    bb = p.b.copy()
    bb[5] = np.nan
    x, it, rr, st = oracle.cg(p.row_ptr, p.col, p.val, bb)
    assert st == "breakdown"


def test_true_relres():
    p = inputs.hpcg27(4)
    assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, np.ones(p.nrows)) == 0.0
    x = np.ones(p.nrows)
    x[3] += 1e-3
    r = p.b - dense(p) @ x
    ref = np.linalg.norm(r) / np.linalg.norm(p.b)
    assert abs(oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x) - ref) <= 1e-12 * ref


def test_cg_independent_of_thread_count():
    """The oracle's CG runs its SpMV rows and element-wise updates on OpenMP
    threads and its dot products sequentially: the iterate is bitwise the
    same on one thread and on several."""
    p = inputs.banded_spd(3000, 12, seed=4)
    saved = oracle.set_threads(0)
    try:
        oracle.set_threads(1)
        x1, it1, rr1, st1 = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-12)
        oracle.set_threads(max(2, os.cpu_count() or 2))
        x8, it8, rr8, st8 = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-12)
    finally:
        oracle.set_threads(saved)
    assert st1 == st8 == "converged" and it1 == it8 and rr1 == rr8
    assert np.array_equal(x1.view(np.uint64), x8.view(np.uint64))
