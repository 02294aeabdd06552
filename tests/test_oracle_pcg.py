"""Pins of the oracle's diagonal extraction/update and Jacobi-preconditioned
CG: dense brute force, scipy's preconditioned CG, and special cases."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import inputs
import oracle


def dense(p):
    return sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(p.nrows, p.ncols)).toarray()


@pytest.mark.parametrize("shape,dens,seed", [((40, 40), 0.2, 1), ((30, 50), 0.3, 2), ((50, 30), 0.1, 3), ((1, 1), 1.0, 4)])
def test_extract_and_update_diagonal_vs_dense(shape, dens, seed):
    p = inputs.random_sparse(shape[0], shape[1], dens, seed, empty_rows=0.2)
    D = dense(p)
    d = oracle.extract_diagonal(p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    assert np.array_equal(d, np.diag(D))
    present = np.array([D[i, i] != 0 for i in range(min(shape))])
    newd = inputs.uniform_vector(min(shape), seed=seed) + 1.0
    v2, bad = oracle.update_diagonal(p.nrows, p.ncols, p.row_ptr, p.col, p.val, newd)
    assert bad == int((~present).sum())
    if bad:
        assert np.array_equal(v2, p.val)  # nothing written
    v3, bad3 = oracle.update_diagonal(p.nrows, p.ncols, p.row_ptr, p.col, p.val, np.where(present, newd, 0.0))
    assert bad3 == 0
    D3 = sp.csr_matrix((v3, p.col, p.row_ptr), shape=shape).toarray()
    for i in range(min(shape)):
        assert D3[i, i] == (newd[i] if present[i] else 0.0)
    off = ~np.eye(*shape, dtype=bool)
    assert np.array_equal(D3[off], D[off])


@pytest.mark.parametrize("n", [8, 16])
def test_pcg_on_hpcg_equals_plain_cg(n):
    """HPCG's diagonal is 26 I: Jacobi only rescales, the Krylov iterates are
    those of plain CG."""
    p = inputs.hpcg27(n)
    x1, it1, _, s1 = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    x2, it2, _, s2 = oracle.pcg_jacobi(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    assert s1 == s2 == "converged" and abs(it1 - it2) <= 1
    assert np.linalg.norm(x2 - x1) <= 1e-8 * np.linalg.norm(x1)


@pytest.mark.parametrize("N,hbw,seed", [(300, 5, 1), (1000, 20, 2)])
def test_pcg_vs_scipy_and_dense_solve(N, hbw, seed):
    p = inputs.banded_spd(N, hbw, seed=seed)
    # make the diagonal strongly non-uniform so the preconditioner matters
    p.val = p.val.copy()
    rows = np.repeat(np.arange(N), np.diff(p.row_ptr))
    scale = 1.0 + 10.0 * inputs.uniform_vector(N, seed=seed)
    diag_mask = rows == p.col
    p.val[diag_mask] *= scale
    A = sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(N, N))
    b = A @ np.ones(N)
    x, it, rr, st = oracle.pcg_jacobi(p.row_ptr, p.col, p.val, b, tol=1e-12)
    assert st == "converged"
    assert np.linalg.norm(x - np.linalg.solve(A.toarray(), b)) <= 1e-9 * np.sqrt(N)
    x, it, rr, st = oracle.pcg_jacobi(p.row_ptr, p.col, p.val, b, tol=1e-10)
    count = [0]
    Minv = sp.diags(1.0 / A.diagonal())
    spla.cg(A, b, x0=np.zeros(N), rtol=1e-10, atol=0.0, M=Minv, maxiter=5000,
            callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert abs(it - count[0]) <= 1, (it, count[0])


def test_pcg_special_cases():
    n = 10
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    d = 1.0 + np.arange(n, dtype=float)
    x, it, rr, st = oracle.pcg_jacobi(rp, col, d, d * 3.0)
    assert st == "converged" and it == 1 and np.allclose(x, 3.0, rtol=0, atol=1e-15)
    p = inputs.random_sparse(10, 10, 0.3, 5)
    dd = oracle.extract_diagonal(10, 10, p.row_ptr, p.col, p.val)
    if (dd == 0).any():
        x, it, rr, st = oracle.pcg_jacobi(p.row_ptr, p.col, p.val, np.ones(10))
        assert st == "zero_diagonal" and it == 0
