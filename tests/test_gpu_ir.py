"""Mixed-precision iterative-refinement CG: values stored in FP32/BF16, inner
CG in FP32, outer residual/dots/update in FP64.  Pin: the true FP64 residual
(recomputed by the oracle with the FP64 values) reaches 1e-10 when the values
are exact in the storage type; otherwise IR solves A_low x = b and the
forward error is reported and bounded by the perturbation."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import log, make_matrix, problem, torch_dev

pytestmark = pytest.mark.gpu


def kappa(name, n):
    """Condition number from the closed-form spectra: 27-point HPCG,
    27 - prod_d (1 + 2 cos(k_d pi / (n + 1))); 7-point with z-coupling 100,
    sum_d w_d 4 sin^2(k_d pi / (2 (n + 1)))."""
    k = np.arange(1, n + 1)
    if name.startswith("hpcg"):
        f = 1 + 2 * np.cos(k * np.pi / (n + 1))
        lam = 27 - f[:, None, None] * f[None, :, None] * f[None, None, :]
    else:
        s = 4 * np.sin(k * np.pi / (2 * (n + 1))) ** 2
        lam = s[:, None, None] + s[None, :, None] + 100 * s[None, None, :]
    return float(lam.max() / lam.min())


@pytest.mark.parametrize("mode", ["ir", "ir_cont"])
@pytest.mark.parametrize("name", ["hpcg32", "aniso32"])
@pytest.mark.parametrize("vdt", ["f32", "bf16"])
@pytest.mark.parametrize("fmt", ["dia", "csr"])
def test_ir_reaches_fp64_residual(name, vdt, fmt, mode):
    """The values are exact in both storage types, so IR solves A x = b: the
    true FP64 residual reaches 1e-10, and the distance to the oracle's FP64
    CG solution obeys ||x_IR - x_64|| <= kappa (rr_IR + rr_64) ||x*||
    (x* = ones, b = A 1)."""
    torch, dev = torch_dev()
    p = problem(name)
    x64, it64, _, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    A = make_matrix(p)
    A.convert(fmt, value_dtype=vdt)
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=1e-10, mode=mode)
    xh = x.cpu().numpy()
    tr = oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh)
    tr64 = oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x64)
    fwd = np.linalg.norm(xh - x64) / np.linalg.norm(x64)
    bound = kappa(name, 32) * (tr + tr64) * np.sqrt(p.nrows) / np.linalg.norm(x64)
    log(f"[ir] {name} {fmt} {vdt} {mode}: outer {res['outer_iters']} inner {res['iters']} (fp64 CG {it64}) "
        f"true relres {tr:.2e} fwd err vs fp64 {fwd:.2e} (bound {bound:.2e})")
    assert res["status"] == "converged"
    assert tr <= 1e-10
    assert res["relres_true"] <= 1e-10
    assert fwd <= bound
    A.close()


@pytest.mark.parametrize("name", ["hpcg32", "aniso32"])
def test_ir_cont_continues_the_krylov_space(name):
    """At the same inner tolerance (1e-2: several refinement steps),
    continuing the search direction across steps needs fewer inner
    iterations than restarting it at every step."""
    torch, dev = torch_dev()
    p = problem(name)
    A = make_matrix(p)
    A.convert("dia", value_dtype="bf16")
    b = torch.from_numpy(p.b).to(dev)
    _, r1 = A.cg(b, tol=1e-10, mode="ir", inner_tol=1e-2)
    _, r2 = A.cg(b, tol=1e-10, mode="ir_cont", inner_tol=1e-2)
    log(f"[ir-cont] {name} bf16: restarted {r1['iters']} inner in {r1['outer_iters']} steps, "
        f"continued {r2['iters']} in {r2['outer_iters']}")
    assert r1["status"] == r2["status"] == "converged"
    assert r2["outer_iters"] >= 2 and r2["iters"] < r1["iters"]
    A.close()


@pytest.mark.parametrize("mode", ["ir", "ir_cont"])
@pytest.mark.parametrize("vdt,bound", [("f32", 1e-5), ("bf16", 5e-2)])
def test_ir_inexact_values_forward_error(vdt, bound, mode):
    """Values not representable in the storage type: IR converges for the
    rounded matrix; the forward error vs the FP64 solution is of the order of
    kappa * unit roundoff of the storage type."""
    torch, dev = torch_dev()
    p = inputs.banded_spd(2000, 8, seed=21)
    xs = np.linalg.solve(
        __import__("scipy.sparse", fromlist=["csr_matrix"]).csr_matrix((p.val, p.col, p.row_ptr)).toarray(), p.b)
    A = make_matrix(p)
    A.convert("csr", value_dtype=vdt)
    x, res = A.cg(torch.from_numpy(p.b).to(dev), tol=1e-10, mode=mode)
    xh = x.cpu().numpy()
    fwd = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    lowvals = oracle.cast_f32(p.val).astype(np.float64) if vdt == "f32" else oracle.bf16_to_f64(oracle.cast_bf16(p.val))
    tr_low = oracle.true_relres(p.row_ptr, p.col, lowvals, p.b, xh)
    log(f"[ir-inexact] {vdt} {mode}: forward error {fwd:.2e}, residual w.r.t. rounded matrix {tr_low:.2e}")
    assert res["status"] == "converged" and tr_low <= 1e-10
    assert fwd <= bound
    A.close()


def test_ir_needs_low_precision_values():
    torch, dev = torch_dev()
    p = problem("hpcg5")
    A = make_matrix(p)
    with pytest.raises(dsm.DsmError) as e:
        A.cg(torch.from_numpy(p.b).to(dev), mode="ir", raise_on_status=True)
    assert e.value.status == dsm.L.E_UNSUPPORTED
    A.close()


@pytest.mark.parametrize("mode", ["ir", "ir_cont"])
def test_ir_special_cases(mode):
    """b = 0 gives x = 0 with no inner iteration; an inner-iteration limit
    ends the solve as not converged within that many SpMVs; a NaN in b is a
    breakdown, not a result."""
    torch, dev = torch_dev()
    p = problem("hpcg16")
    A = make_matrix(p)
    A.convert("dia", value_dtype="bf16")
    x, res = A.cg(torch.zeros(p.nrows, dtype=torch.float64, device=dev), tol=1e-10, mode=mode)
    assert res["status"] == "converged" and res["iters"] == 0 and not x.any()
    x, res = A.cg(torch.from_numpy(p.b).to(dev), tol=1e-10, mode=mode, maxit=5)
    assert res["status"] == "not_converged" and res["iters"] <= 5, res
    bb = p.b.copy()
    bb[11] = np.nan
    x, res = A.cg(torch.from_numpy(bb).to(dev), tol=1e-10, mode=mode)
    assert res["status"] == "breakdown", res
    A.close()
