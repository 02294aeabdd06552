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


@pytest.mark.parametrize("name", ["hpcg32", "aniso32"])
@pytest.mark.parametrize("vdt", ["f32", "bf16"])
@pytest.mark.parametrize("fmt", ["dia", "csr"])
def test_ir_reaches_fp64_residual(name, vdt, fmt):
    torch, dev = torch_dev()
    p = problem(name)
    x64, it64, _, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
    A = make_matrix(p)
    A.convert(fmt, value_dtype=vdt)
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=1e-10, mode="ir")
    xh = x.cpu().numpy()
    tr = oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh)
    fwd = np.linalg.norm(xh - x64) / np.linalg.norm(x64)
    log(f"[ir] {name} {fmt} {vdt}: outer {res['outer_iters']} inner {res['iters']} (fp64 CG {it64}) "
        f"true relres {tr:.2e} fwd err vs fp64 {fwd:.2e}")
    assert res["status"] == "converged"
    assert tr <= 1e-10
    assert res["relres_true"] <= 1e-10
    A.close()


@pytest.mark.parametrize("vdt,bound", [("f32", 1e-5), ("bf16", 5e-2)])
def test_ir_inexact_values_forward_error(vdt, bound):
    """Values not representable in the storage type: IR converges for the
    rounded matrix; the forward error vs the FP64 solution is of the order of
    kappa * unit roundoff of the storage type."""
    torch, dev = torch_dev()
    p = inputs.banded_spd(2000, 8, seed=21)
    xs = np.linalg.solve(
        __import__("scipy.sparse", fromlist=["csr_matrix"]).csr_matrix((p.val, p.col, p.row_ptr)).toarray(), p.b)
    A = make_matrix(p)
    A.convert("csr", value_dtype=vdt)
    x, res = A.cg(torch.from_numpy(p.b).to(dev), tol=1e-10, mode="ir")
    xh = x.cpu().numpy()
    fwd = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    lowvals = oracle.cast_f32(p.val).astype(np.float64) if vdt == "f32" else oracle.bf16_to_f64(oracle.cast_bf16(p.val))
    tr_low = oracle.true_relres(p.row_ptr, p.col, lowvals, p.b, xh)
    log(f"[ir-inexact] {vdt}: forward error {fwd:.2e}, residual w.r.t. rounded matrix {tr_low:.2e}")
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
