"""HPCG's preconditioner on the GPU against the oracle: the multicolour
symmetric Gauss-Seidel sweep, the multigrid V-cycle and the PCG it
preconditions, on CSR and DIA level matrices, plus the boundary's checks."""
import functools

import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import anchors, ctx, log, torch_dev

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def hierarchy(n, nlev):
    return inputs.hpcg27_levels(n, nlev)


def oracle_levels(L):
    out = []
    for lv in L:
        p = lv["problem"]
        d = {"row_ptr": p.row_ptr, "col": p.col, "val": p.val,
             "order": np.argsort(lv["colour"], kind="stable").astype(np.int32)}
        if "f2c" in lv:
            d["f2c"] = lv["f2c"]
        out.append(d)
    return out


def build(L, fmt):
    mats = []
    for lv in L:
        p = lv["problem"]
        A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val)
        if fmt != "csr":
            A.convert(fmt)
        mats.append(A)
    mg = dsm.Multigrid(ctx(), mats, [lv["f2c"] for lv in L[:-1]], [lv["colour"] for lv in L])
    return mg, mats


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@functools.lru_cache(maxsize=None)
def seven_point_hierarchy(n, nlev):
    """The HPCG grids, colourings and coarse maps with the anisotropic
    7-point operator on every level (7 diagonals: the 7-diagonal forms of
    the DIA smoother)."""
    out = []
    for lv in inputs.hpcg27_levels(n, nlev):
        m = round(lv["problem"].nrows ** (1 / 3))
        d = dict(lv)
        d["problem"] = inputs.aniso7(m)
        out.append(d)
    return out


@pytest.mark.parametrize("fmt", ["csr", "dia"])
@pytest.mark.parametrize("n", [2, 5, 16, 24])
def test_symgs_matches_oracle(fmt, n):
    torch, dev = torch_dev()
    L = hierarchy(n, 1)
    mg, mats = build(L, fmt)
    p = L[0]["problem"]
    r = inputs.uniform_vector(p.nrows, seed=21) - 0.5
    x0 = inputs.uniform_vector(p.nrows, seed=22)
    xr, bad = oracle.symgs(p.row_ptr, p.col, p.val, r, x0, order=oracle_levels(L)[0]["order"])
    assert bad == 0
    x = torch.from_numpy(x0).to(dev)
    mg.symgs(0, torch.from_numpy(r).to(dev), x)
    torch.cuda.synchronize()
    err = rel_err(x.cpu().numpy(), xr)
    log(f"[mg] symgs {fmt} {n}^3 err {err:.2e}")
    assert err <= 1e-12
    if fmt == "dia":
        # same products, same order, no fused multiply-add: the same bits
        assert np.array_equal(x.cpu().numpy(), xr)
    mg.close()


@pytest.mark.parametrize("n", [5, 24])
def test_symgs_non_lattice_colouring(n):
    """A valid 12-colouring other than the grid's parity colouring (x
    coordinate mod 3, y and z parities): the DIA sweep follows any colour
    order, bit for bit the oracle's sweep in that order."""
    torch, dev = torch_dev()
    p = inputs.hpcg27(n)
    i = np.arange(p.nrows)
    ix, iy, iz = i % n, (i // n) % n, i // (n * n)
    colour = ((ix % 3) + 3 * ((iy & 1) + 2 * (iz & 1))).astype(np.int32)
    A = dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    A.convert("dia")
    mg = dsm.Multigrid(ctx(), [A], [], [colour])
    r = inputs.uniform_vector(p.nrows, seed=31) - 0.5
    x0 = inputs.uniform_vector(p.nrows, seed=32)
    xr, bad = oracle.symgs(p.row_ptr, p.col, p.val, r, x0, order=np.argsort(colour, kind="stable").astype(np.int32))
    assert bad == 0
    x = torch.from_numpy(x0).to(dev)
    mg.symgs(0, torch.from_numpy(r).to(dev), x)
    log(f"[mg] symgs 12 colours {n}^3")
    assert np.array_equal(x.cpu().numpy(), xr)
    mg.close()


@pytest.mark.parametrize("n,nlev", [(8, 1), (24, 1), (24, 2)])
def test_seven_point_levels_match_oracle(n, nlev):
    """7-diagonal DIA levels: the LDS sweep (8^3, 12^3) and the per-colour
    launches (24^3), one sweep and one V-cycle, bit for bit."""
    torch, dev = torch_dev()
    L = seven_point_hierarchy(n, nlev)
    mg, mats = build(L, "dia")
    p = L[0]["problem"]
    r = inputs.uniform_vector(p.nrows, seed=24) - 0.4
    x0 = inputs.uniform_vector(p.nrows, seed=25)
    xr, bad = oracle.symgs(p.row_ptr, p.col, p.val, r, x0, order=oracle_levels(L)[0]["order"])
    assert bad == 0
    x = torch.from_numpy(x0).to(dev)
    mg.symgs(0, torch.from_numpy(r).to(dev), x)
    assert np.array_equal(x.cpu().numpy(), xr)
    zr = oracle.mg(oracle_levels(L), r)
    z = mg.apply(torch.from_numpy(r).to(dev))
    err = rel_err(z.cpu().numpy(), zr)
    log(f"[mg] seven-point {n}^3 x{nlev} vcycle err {err:.2e}")
    assert np.array_equal(z.cpu().numpy(), zr)
    mg.close()


@pytest.mark.parametrize("fmt", ["csr", "dia"])
@pytest.mark.parametrize("n,nlev", [(8, 2), (16, 4), (24, 3)])
def test_vcycle_matches_oracle(fmt, n, nlev):
    torch, dev = torch_dev()
    L = hierarchy(n, nlev)
    mg, mats = build(L, fmt)
    r = inputs.uniform_vector(L[0]["problem"].nrows, seed=23) - 0.3
    zr = oracle.mg(oracle_levels(L), r)
    z = mg.apply(torch.from_numpy(r).to(dev))
    torch.cuda.synchronize()
    err = rel_err(z.cpu().numpy(), zr)
    log(f"[mg] vcycle {fmt} {n}^3 x{nlev} err {err:.2e}")
    assert err <= 1e-12
    if fmt == "dia":
        assert np.array_equal(z.cpu().numpy(), zr)
    # a second application reuses the coarse vectors: same bits
    z2 = mg.apply(torch.from_numpy(r).to(dev))
    torch.cuda.synchronize()
    assert torch.equal(z, z2)
    mg.close()


@pytest.mark.parametrize("fmt", ["csr", "dia"])
@pytest.mark.parametrize("n,nlev", [(16, 4), (32, 4)])
def test_pcg_mg_matches_oracle(fmt, n, nlev):
    torch, dev = torch_dev()
    L = hierarchy(n, nlev)
    p = L[0]["problem"]
    mg, mats = build(L, fmt)
    xo, it, rel, st = oracle.pcg_mg(oracle_levels(L), p.b, tol=1e-10)
    assert st == "converged"
    x, res = mg.pcg(torch.from_numpy(p.b).to(dev), tol=1e-10)
    xh = x.cpu().numpy()
    log(f"[mg] pcg {fmt} {n}^3 x{nlev}: {res['iters']} iters (oracle {it}), true {res['relres_true']:.2e}")
    assert res["status"] == "converged" and abs(res["iters"] - it) <= 1
    assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh) <= 1.5e-10
    assert abs(res["relres_true"] - oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh)) <= 1e-11
    assert np.linalg.norm(xh - xo) <= 1e-8 * np.linalg.norm(xo)
    mg.close()


def test_pcg_mg_limits():
    torch, dev = torch_dev()
    L = hierarchy(16, 3)
    p = L[0]["problem"]
    mg, mats = build(L, "dia")
    x, res = mg.pcg(torch.from_numpy(p.b).to(dev), maxit=3)
    assert res["status"] == "not_converged" and res["iters"] == 3
    x, res = mg.pcg(torch.zeros(p.nrows, dtype=torch.float64, device=dev))
    assert res["status"] == "converged" and res["iters"] == 0 and not bool(x.any())
    bb = p.b.copy()
    bb[7] = np.nan
    x, res = mg.pcg(torch.from_numpy(bb).to(dev))
    assert res["status"] == "breakdown"
    mg.close()


def test_mg_boundary_checks():
    torch, dev = torch_dev()
    L = hierarchy(8, 2)
    mats = []
    for lv in L:
        p = lv["problem"]
        mats.append(dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val))
    f2c = [L[0]["f2c"]]
    cols = [lv["colour"] for lv in L]
    # one colour for coupled rows
    with pytest.raises(dsm.DsmError) as e:
        dsm.Multigrid(ctx(), mats, f2c, [np.zeros_like(cols[0]), cols[1]])
    assert e.value.status == dsm.L.E_INVALID
    # f2c out of range, then not injective
    bad = f2c[0].copy()
    bad[0] = L[0]["problem"].nrows
    with pytest.raises(dsm.DsmError) as e:
        dsm.Multigrid(ctx(), mats, [bad], cols)
    assert e.value.status == dsm.L.E_INVALID
    bad = f2c[0].copy()
    bad[1] = bad[0]
    with pytest.raises(dsm.DsmError) as e:
        dsm.Multigrid(ctx(), mats, [bad], cols)
    assert e.value.status == dsm.L.E_INVALID
    # colour out of range
    with pytest.raises(dsm.DsmError) as e:
        dsm.Multigrid(ctx(), mats, f2c, [cols[0] + 300, cols[1]])
    assert e.value.status == dsm.L.E_INVALID
    # unsupported level format
    mats[1].convert("ell")
    with pytest.raises(dsm.DsmError) as e:
        dsm.Multigrid(ctx(), mats, f2c, cols)
    assert e.value.status == dsm.L.E_UNSUPPORTED
    # a level converted after creation is refused at apply
    mats[1].convert("csr")
    mg = dsm.Multigrid(ctx(), mats, f2c, cols)
    mats[1].convert("dia")
    r = torch.ones(L[0]["problem"].nrows, dtype=torch.float64, device=dev)
    with pytest.raises(dsm.DsmError) as e:
        mg.apply(r)
    assert e.value.status == dsm.L.E_INVALID
    mg.close()
    # zero diagonal on a coarse level
    p1 = L[1]["problem"]
    v = p1.val.copy()
    v[(p1.col == 3) & (np.repeat(np.arange(p1.nrows), np.diff(p1.row_ptr)) == 3)] = 0.0
    z1 = dsm.Matrix.from_csr(ctx(), p1.nrows, p1.ncols, p1.row_ptr, p1.col, v)
    with pytest.raises(dsm.DsmError) as e:
        dsm.Multigrid(ctx(), [mats[0], z1], f2c, cols)
    assert e.value.status == dsm.L.E_INVALID


def test_pcg_mg_full_size_dia():
    """HPCG 104^3 with four levels (104, 52, 26, 13), DIA at every level, in
    the launch configuration the benchmark times: converges to 1e-10 with
    the oracle's true residual check on the result."""
    torch, dev = torch_dev()
    L = hierarchy(104, 4)
    p = L[0]["problem"]
    mg, mats = build(L, "dia")
    x, res = mg.pcg(torch.from_numpy(p.b).to(dev), tol=1e-10)
    xh = x.cpu().numpy()
    log(f"[mg] pcg dia 104^3 x4: {res}")
    assert res["status"] == "converged"
    assert abs(res["iters"] - anchors()["pcg_mg_hpcg27_104_4levels_tol1e-10"]["iters"]) <= 1, res
    assert oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh) <= 1.5e-10
    assert np.max(np.abs(xh - 1.0)) <= 1e-7
    mg.close()
