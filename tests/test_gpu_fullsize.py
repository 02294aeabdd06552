"""Parity at the full workload sizes, in the configurations the benchmark
times: plain FP64 CG on HPCG 128^3 and the anisotropic 7-point Laplacian at
128^3 (CSR and DIA with the kernel variant the selector picks), iterative
refinement with FP32/BF16 values at 128^3, CG on HPCG 104^3 with the DIA
sweeps the benchmark runs, FP32-valued SpMV on the irregular 1M-row
matrices, and the re-timing check of the selection on those matrices.

Expected values come from the oracle, run here on the same seeded inputs
(its iteration counts are also stored as anchors in tests/golden)."""
import numpy as np
import pytest

import oracle
import paper_2209_06478_amd as dsm
from gpu_common import (anchors, FORMATS, log, make_matrix, oracle_cg, problem, row_scaled_err, selection_acceptable,
                        selection_retime,
                        torch_dev, x_for)

pytestmark = pytest.mark.gpu

# condition numbers from the closed-form spectra (27-point: 27 - prod(1 + 2 cos);
# 7-point with z-coupling 100: sum of w_d 4 sin^2)
KAPPA = {"hpcg104": 1489.4, "hpcg128": 2248.1, "aniso128": 6743.7}
ANCHOR = {"hpcg104": "cg_hpcg27_104_tol1e-10", "hpcg128": "cg_hpcg27_128_tol1e-10",
          "aniso128": "cg_aniso7_128_tol1e-10"}


def check_fp64_cg(name, x, res, tol=1e-10):
    """Iterations within +-1 of the oracle and of the stored anchor, true
    residual (recomputed by the oracle) <= 1.5 tol, and the distance to the
    oracle's iterate within 10 kappa tol ||x_oracle||."""
    p = problem(name)
    xo, it, _, st = oracle_cg(name)
    assert st == "converged" and res["status"] == "converged", res
    assert abs(res["iters"] - it) <= 1, (res, it)
    assert abs(res["iters"] - anchors()[ANCHOR[name]]["iters"]) <= 1, res
    tr = oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x)
    assert tr <= 1.5 * tol, tr
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    log(f"[fullsize] {name}: {res['iters']} iterations (oracle {it}), true relres {tr:.2e}, "
        f"||x - x_oracle||/||x_oracle|| {err:.2e}")
    assert err <= 10 * KAPPA[name] * tol
    return tr


@pytest.mark.parametrize("name", ["hpcg128", "aniso128"])
@pytest.mark.parametrize("fmt", ["csr", "dia"])
def test_fp64_cg_128_selected_variant(name, fmt):
    """FP64 CG at 128^3 with the format fixed and its kernel variant chosen
    by the timed selection (what the mixed-precision comparison runs)."""
    torch, dev = torch_dev()
    p = problem(name)
    A = make_matrix(p)
    rep = A.select(mask=[fmt], use_cache=False)
    log(f"[fullsize] {name} {fmt}: selector variant {rep['chosen_variant']}")
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=1e-10)
    check_fp64_cg(name, x.cpu().numpy(), res)
    A.close()


@pytest.mark.parametrize("variant", [16, "selected"])
def test_fp64_cg_hpcg104_bench_sweeps(variant):
    """CG on HPCG 104^3 in DIA with the LDS-staged sweep and its p.q
    epilogue (variant 16), and with whatever variant the selection picks."""
    torch, dev = torch_dev()
    p = problem("hpcg104")
    A = make_matrix(p)
    if variant == "selected":
        rep = A.select(use_cache=False)
        log(f"[fullsize] hpcg104 selection: {rep['chosen']} v{rep['chosen_variant']}")
    else:
        A.convert("dia")
        A.variant = variant
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=1e-10)
    check_fp64_cg("hpcg104", x.cpu().numpy(), res)
    A.close()


@pytest.mark.parametrize("variant", [16, "selected"])
def test_jacobi_pcg_hpcg104(variant):
    """Jacobi PCG on HPCG 104^3, as the benchmark runs it: the diagonal is
    26 in every row, and with M = c I the preconditioned iterates are CG's
    (z = r / c scales p by 1/c and alpha by c), so CG's oracle checks
    apply."""
    torch, dev = torch_dev()
    p = problem("hpcg104")
    A = make_matrix(p)
    if variant == "selected":
        A.select(use_cache=False)
    else:
        A.convert("dia")
        A.variant = variant
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=1e-10, mode="jacobi")
    log(f"[fullsize] hpcg104 jacobi {A.format} v{A.variant}")
    check_fp64_cg("hpcg104", x.cpu().numpy(), res)
    A.close()


@pytest.mark.parametrize("mode", ["ir", "ir_cont"])
@pytest.mark.parametrize("name", ["hpcg128", "aniso128"])
@pytest.mark.parametrize("vdt", ["f32", "bf16"])
@pytest.mark.parametrize("fmt", ["dia", "csr"])
def test_ir_128(name, vdt, fmt, mode):
    """Iterative refinement with FP32/BF16 values at 128^3, the variant tuned
    for FP32 vectors as the benchmark does.  The values (26/-1, 204/-1/-100)
    are exact in both storage types, so IR solves A x = b itself: the true
    FP64 residual recomputed by the oracle reaches 1e-10, and the distance to
    the oracle's FP64 CG solution obeys the perturbation bound
    ||x_IR - x_64|| <= kappa (rr_IR + rr_64) ||x*|| with x* = ones (b = A 1),
    from ||x - x*|| <= kappa ||b - A x|| / ||b|| ||x*||."""
    torch, dev = torch_dev()
    p = problem(name)
    x64, it64, _, _ = oracle_cg(name)
    A = make_matrix(p)
    rep = A.select(mask=[fmt], value_dtype=vdt, vec_dtype="f32", use_cache=False)
    b = torch.from_numpy(p.b).to(dev)
    x, res = A.cg(b, tol=1e-10, mode=mode)
    xh = x.cpu().numpy()
    tr = oracle.true_relres(p.row_ptr, p.col, p.val, p.b, xh)
    tr64 = oracle.true_relres(p.row_ptr, p.col, p.val, p.b, x64)
    fwd = np.linalg.norm(xh - x64) / np.linalg.norm(x64)
    xnorm = np.sqrt(p.nrows)
    bound = KAPPA[name] * (tr + tr64) * xnorm / np.linalg.norm(x64)
    log(f"[fullsize-ir] {name} {fmt} {vdt} {mode} v{rep['chosen_variant']}: outer {res['outer_iters']} inner "
        f"{res['iters']} (fp64 CG {it64}), true relres {tr:.2e}, ||x_IR - x_64||/||x_64|| {fwd:.2e} "
        f"(bound {bound:.2e}), ||x_IR - 1||/||1|| {np.linalg.norm(xh - 1) / xnorm:.2e}")
    assert res["status"] == "converged", res
    assert tr <= 1e-10 and res["relres_true"] <= 1e-10
    assert fwd <= bound
    assert np.linalg.norm(xh - 1) <= KAPPA[name] * tr * xnorm
    A.close()


@pytest.mark.parametrize("name", ["zipf1m", "banded1m"])
@pytest.mark.parametrize("vdt", ["f32", "bf16"])
def test_spmv_1m_reduced_precision_values(name, vdt):
    """FP32/BF16-valued SpMV on the irregular 1M-row matrices, every feasible
    format and kernel variant.  With FP64 vectors the result is the FP64
    product of the rounded values (row-scaled 1e-14); with FP32 vectors the
    FP32 accumulation stays within (len_i + 2) 2^-24 S_i (+ the final
    rounding)."""
    torch, dev = torch_dev()
    p = problem(name)
    vals = oracle.cast_f32(p.val).astype(np.float64) if vdt == "f32" else oracle.bf16_to_f64(oracle.cast_bf16(p.val))
    x = x_for(p)
    x32 = x.astype(np.float32).astype(np.float64)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, vals, x)
    yref32, scale32 = oracle.spmv_csr_ref(p.row_ptr, p.col, vals, x32)
    bound = (np.diff(p.row_ptr) + 2) * 2.0 ** -24 * scale32 + 2.0 ** -24 * np.abs(yref32)
    A = make_matrix(p)
    xt = torch.from_numpy(x).to(dev)
    xt32 = xt.float()
    done = []
    for f in FORMATS:
        try:
            A.convert(f, value_dtype=vdt)
        except dsm.DsmError as e:
            if e.status == dsm.L.E_INFEASIBLE:
                continue
            raise
        log(f"[spmv-1m-{vdt}] {name} {f}")
        variants = range(16) if f == "csr" else (range(64) if f in ("dia", "hdc") else (range(16) if f in ("ell", "hyb") else [0]))
        for v in variants:
            A.variant = v
            y = A.spmv(xt).cpu().numpy()
            assert row_scaled_err(y, yref, scale) <= 1e-14, (name, f, v)
            y32 = A.spmv(xt32).cpu().numpy().astype(np.float64)
            assert np.all(np.abs(y32 - yref32) <= bound + 1e-30), (name, f, v)
        done.append(f)
    A.close()
    assert {"csr", "coo", "hyb", "hdc"} <= set(done), done
    if name == "banded1m":
        assert {"dia", "ell"} <= set(done), done


@pytest.mark.parametrize("name", ["zipf1m", "banded1m"])
@pytest.mark.parametrize("vdt", ["f64", "f32"])
def test_select_1m_is_near_best(name, vdt):
    """Selection on the 1M-row irregular matrices: the chosen format is
    feasible, computes the oracle's product, and re-timed beside fresh
    conversions of every other candidate it is within 5% of the fastest."""
    torch, dev = torch_dev()
    p = problem(name)
    A = make_matrix(p)
    rep = A.select(use_cache=False, value_dtype=vdt)
    log(f"[select-1m] {name} {vdt}: chose {rep['chosen']} v{rep['chosen_variant']} medians {rep['median_us']}")
    assert rep["status"][rep["chosen"]] == 0
    vals = p.val if vdt == "f64" else oracle.cast_f32(p.val).astype(np.float64)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, vals, x_for(p))
    xt = torch.from_numpy(x_for(p)).to(dev)
    assert row_scaled_err(A.spmv(xt).cpu().numpy(), yref, scale) <= 1e-14
    chosen_t, best_t, best_f = selection_retime(p, A, rep, value_dtype=vdt)
    log(f"[select-1m] {name} {vdt}: chosen {chosen_t:.2f} us, best re-timed {best_f} {best_t:.2f} us")
    assert selection_acceptable(rep, chosen_t, best_t, best_f), (rep["bytes"], chosen_t, best_t, best_f)
    A.close()
