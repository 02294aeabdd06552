"""Pins of the oracle's HPCG preconditioner (symmetric Gauss-Seidel and the
multigrid V-cycle) and of the CG it preconditions: dense triangular solves
(scipy), the two-level cycle composed from dense matrices, permutation and
multicolour invariances, symmetry and positivity of the preconditioner,
and convergence on the HPCG problem."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import inputs
import oracle


def dense(p):
    return sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(p.nrows, p.ncols)).toarray()


def symgs_dense(A, r, x0):
    """Forward sweep x1 = (D + L)^-1 (r - U x0), backward x2 = (D + U)^-1 (r - L x1)."""
    L = np.tril(A, -1)
    U = np.triu(A, 1)
    D = np.diag(np.diag(A))
    x1 = sla.solve_triangular(D + L, r - U @ x0, lower=True)
    return sla.solve_triangular(D + U, r - L @ x1, lower=False)


def levels_of(n, nlev):
    L = inputs.hpcg27_levels(n, nlev)
    out = []
    for lv in L:
        p = lv["problem"]
        d = {"row_ptr": p.row_ptr, "col": p.col, "val": p.val,
             "order": np.argsort(lv["colour"], kind="stable").astype(np.int32)}
        if "f2c" in lv:
            d["f2c"] = lv["f2c"]
        out.append(d)
    return L, out


@pytest.mark.parametrize("case", ["hpcg4", "banded"])
def test_symgs_natural_order_is_two_triangular_solves(case):
    p = inputs.hpcg27(4) if case == "hpcg4" else inputs.banded_spd(300, 7, seed=11)
    A = dense(p)
    r = inputs.uniform_vector(p.nrows, seed=3) - 0.5
    x0 = inputs.uniform_vector(p.nrows, seed=4)
    x, bad = oracle.symgs(p.row_ptr, p.col, p.val, r, x0)
    assert bad == 0
    ref = symgs_dense(A, r, x0)
    assert np.max(np.abs(x - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_symgs_order_is_a_symmetric_permutation():
    """Sweeping in order o equals the natural sweep on P A P^T (row t of the
    permuted matrix is row o[t])."""
    p = inputs.banded_spd(200, 5, seed=12)
    A = dense(p)
    o = np.random.default_rng(5).permutation(p.nrows).astype(np.int32)
    r = inputs.uniform_vector(p.nrows, seed=6)
    x0 = inputs.uniform_vector(p.nrows, seed=7)
    x, _ = oracle.symgs(p.row_ptr, p.col, p.val, r, x0, order=o)
    Ap = A[np.ix_(o, o)]
    ref = np.empty_like(x)
    ref[o] = symgs_dense(Ap, r[o], x0[o])
    assert np.max(np.abs(x - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_multicolour_rows_are_independent():
    """Rows of one parity colour share no stencil entry, so the order inside
    a colour does not change a single bit."""
    L, lv = levels_of(8, 1)
    p, colour = L[0]["problem"], L[0]["colour"]
    A = sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(p.nrows, p.ncols))
    rows, cols = A.nonzero()
    off = rows != cols
    assert not np.any(colour[rows[off]] == colour[cols[off]])
    r = inputs.uniform_vector(p.nrows, seed=8)
    x0 = np.zeros(p.nrows)
    base = np.argsort(colour, kind="stable").astype(np.int32)
    xa, _ = oracle.symgs(p.row_ptr, p.col, p.val, r, x0, order=base)
    rng = np.random.default_rng(9)
    shuffled = np.concatenate([rng.permutation(np.flatnonzero(colour == c)) for c in range(8)]).astype(np.int32)
    xb, _ = oracle.symgs(p.row_ptr, p.col, p.val, r, x0, order=shuffled)
    assert np.array_equal(xa, xb)
    xn, _ = oracle.symgs(p.row_ptr, p.col, p.val, r, x0)
    assert not np.array_equal(xa, xn)  # a different order is a different smoother


def test_symgs_reports_missing_diagonal():
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    x, bad = oracle.symgs(rp, col, np.array([1.0, 1.0]), np.ones(2), np.zeros(2))
    assert bad == 2 and np.array_equal(x, np.zeros(2))


def test_one_level_cycle_is_one_sweep_from_zero():
    L, lv = levels_of(8, 1)
    p = L[0]["problem"]
    r = inputs.uniform_vector(p.nrows, seed=10)
    z = oracle.mg(lv, r)
    x, _ = oracle.symgs(p.row_ptr, p.col, p.val, r, np.zeros(p.nrows), order=lv[0]["order"])
    assert np.array_equal(z, x)


def test_two_level_cycle_matches_dense_composition():
    """Pre-smooth, restrict the residual by injection, coarse sweep,
    prolongate by adding at the coarse points, post-smooth."""
    L, lv = levels_of(8, 2)
    A0, A1 = dense(L[0]["problem"]), dense(L[1]["problem"])
    o0, o1 = lv[0]["order"], lv[1]["order"]
    f2c = L[0]["f2c"]
    r = inputs.uniform_vector(A0.shape[0], seed=11) - 0.3

    def S(A, o, rhs, x0):
        out = np.empty_like(x0)
        out[o] = symgs_dense(A[np.ix_(o, o)], rhs[o], x0[o])
        return out

    x1 = S(A0, o0, r, np.zeros_like(r))
    rc = (r - A0 @ x1)[f2c]
    xc = S(A1, o1, rc, np.zeros(A1.shape[0]))
    x2 = x1.copy()
    x2[f2c] += xc
    ref = S(A0, o0, r, x2)
    z = oracle.mg(lv, r)
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_injected_residual_is_not_rounding_noise():
    """The coarse points (all coordinates even) are the colour the forward
    sweep visits last, so after the pre-smoothing sweep their neighbours have
    moved and the injected residual is a real fraction of r.  Were they the
    colour that sweep updates last, each would have been solved exactly
    against its final neighbours and the injected residual would be rounding
    noise (checked on the reversed colour order)."""
    L, lv = levels_of(16, 2)
    p, f2c, colour = L[0]["problem"], L[0]["f2c"], L[0]["colour"]
    ix = np.arange(p.nrows) % 16
    iy = (np.arange(p.nrows) // 16) % 16
    iz = np.arange(p.nrows) // 256
    even = (ix % 2 == 0) & (iy % 2 == 0) & (iz % 2 == 0)
    assert np.array_equal(np.flatnonzero(even), np.sort(f2c))
    assert np.all(colour[even] == colour.max())
    r = inputs.uniform_vector(p.nrows, seed=14) - 0.3
    for order, lo, hi in ((lv[0]["order"], 0.05, 1.0),
                          (np.argsort(colour.max() - colour, kind="stable").astype(np.int32), 0.0, 1e-14)):
        x, _ = oracle.symgs(p.row_ptr, p.col, p.val, r, np.zeros(p.nrows), order=order)
        rc = (r - oracle.spmv_csr(p.row_ptr, p.col, p.val, x))[f2c]
        rel = np.linalg.norm(rc) / np.linalg.norm(r[f2c])
        assert lo <= rel <= hi, rel


@pytest.mark.parametrize("nlev", [1, 2, 3])
def test_preconditioner_is_symmetric_positive(nlev):
    """Symmetric smoother, prolongation = transpose of injection: M is
    symmetric and positive definite, as CG needs."""
    L, lv = levels_of(8, nlev)
    n = L[0]["problem"].nrows
    u = inputs.uniform_vector(n, seed=12) - 0.5
    v = inputs.uniform_vector(n, seed=13) - 0.5
    Mu, Mv = oracle.mg(lv, u), oracle.mg(lv, v)
    assert abs(u @ Mv - v @ Mu) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Mv)
    assert u @ Mu > 0 and v @ Mv > 0


def test_pcg_mg_converges_fast_on_hpcg():
    L, lv = levels_of(16, 4)
    p = L[0]["problem"]
    x, it, rel, st = oracle.pcg_mg(lv, p.b, tol=1e-10)
    assert st == "converged" and rel <= 1e-10
    assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x) <= 1.5e-10
    assert np.max(np.abs(x - 1.0)) <= 1e-8
    _, it_cg, _, _ = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    # one level (Gauss-Seidel only) already beats plain CG, the coarse
    # correction cuts the count further (16^3: 27 -> 23 -> 15)
    _, it1, _, st1 = oracle.pcg_mg(lv[:1], p.b, tol=1e-10)
    assert st1 == "converged" and it < it1 < it_cg, (it, it1, it_cg)


def test_pcg_mg_special_cases():
    L, lv = levels_of(8, 2)
    p = L[0]["problem"]
    x, it, rel, st = oracle.pcg_mg(lv, np.zeros(p.nrows))
    assert st == "converged" and it == 0 and not x.any()
    x, it, rel, st = oracle.pcg_mg(lv, p.b, maxit=2)
    assert st == "not_converged" and it == 2
    bad = [dict(d) for d in lv]
    v = bad[1]["val"].copy()
    rp, col = bad[1]["row_ptr"], bad[1]["col"]
    v[[k for k in range(rp[3], rp[4]) if col[k] == 3]] = 0.0
    bad[1]["val"] = v
    x, it, rel, st = oracle.pcg_mg(bad, p.b)
    assert st == "zero_diagonal" and it == 0


def test_pcg_mg_loop_matches_scipy_pcg():
    """The preconditioned loop against scipy's PCG driven by the same V-cycle:
    same iteration count within one, same solution to the tolerance."""
    import scipy.sparse.linalg as spla
    L, lv = levels_of(16, 3)
    p = L[0]["problem"]
    A = sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(p.nrows, p.ncols))
    M = spla.LinearOperator(A.shape, matvec=lambda v: oracle.mg(lv, np.ravel(v)), dtype=np.float64)
    count = [0]
    xs, info = spla.cg(A, p.b, x0=np.zeros(p.nrows), rtol=1e-10, atol=0.0, M=M, maxiter=500,
                       callback=lambda xk: count.__setitem__(0, count[0] + 1))
    x, it, rel, st = oracle.pcg_mg(lv, p.b, tol=1e-10)
    assert info == 0 and st == "converged"
    assert abs(it - count[0]) <= 1, (it, count[0])
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
