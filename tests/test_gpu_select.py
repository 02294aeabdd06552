"""Format selection: the chosen format is feasible and, re-timed against
fresh conversions of every candidate, within 5% of the fastest median;
repeated structures hit the cache; the one-workgroup target picks among
CSR/DIA/ELL and tunes CSR lanes."""
import numpy as np
import pytest

import inputs
import oracle
import paper_2209_06478_amd as dsm
from gpu_common import selection_acceptable, selection_retime_cold, log, make_matrix, median_launch_us, problem, row_scaled_err, selection_retime, torch_dev, x_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["hpcg16", "hpcg104", "zipf50k", "banded20k"])
def test_select_is_near_best(name):
    """The chosen (format, variant), re-timed beside fresh conversions of
    every candidate and every variant the selector tries, each timed the same
    way and the same number of times, is within 5% of the fastest."""
    torch, dev = torch_dev()
    p = problem(name)
    A = make_matrix(p)
    rep = A.select(use_cache=False)
    log(f"[select] {name}: chose {rep['chosen']} v{rep['chosen_variant']} medians {rep['median_us']}")
    assert rep["status"][rep["chosen"]] == 0
    x = torch.from_numpy(x_for(p)).to(dev)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x_for(p))
    assert row_scaled_err(A.spmv(x).cpu().numpy(), yref, scale) <= 1e-14
    chosen_t, best_t, best_f = selection_retime(p, A, rep)
    log(f"[select] {name}: chosen {chosen_t:.2f} us, best re-timed {best_f} {best_t:.2f} us")
    assert selection_acceptable(rep, chosen_t, best_t, best_f), (rep["bytes"], chosen_t, best_t, best_f)
    A.close()


@pytest.mark.parametrize("name", ["hpcg104", "banded20k"])
def test_cold_select_is_near_best(name):
    """Cold selection (a 1 GiB read before every timed SpMV, kernel-only
    times): the chosen (format, variant), re-timed the same way beside every
    candidate, is within 5% of the fastest, and the result still matches the
    oracle."""
    torch, dev = torch_dev()
    p = problem(name)
    A = make_matrix(p)
    rep = A.select(use_cache=False, flush_bytes=1 << 30)
    log(f"[select cold] {name}: chose {rep['chosen']} v{rep['chosen_variant']} medians {rep['median_us']}")
    assert rep["status"][rep["chosen"]] == 0
    x = torch.from_numpy(x_for(p)).to(dev)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x_for(p))
    assert row_scaled_err(A.spmv(x).cpu().numpy(), yref, scale) <= 1e-14
    chosen_t, best_t, best_f = selection_retime_cold(p, A, rep)
    log(f"[select cold] {name}: chosen {chosen_t:.2f} us, best re-timed {best_f} {best_t:.2f} us")
    assert selection_acceptable(rep, chosen_t, best_t, best_f), (rep["bytes"], chosen_t, best_t, best_f)
    A.close()


def test_select_cache_hit_on_same_structure():
    p = problem("hpcg16")
    A = make_matrix(p)
    r1 = A.select(use_cache=True)
    B = dsm.Matrix.from_csr(A.ctx, p.nrows, p.ncols, p.row_ptr, p.col, p.val * 2.0)
    r2 = B.select(use_cache=True)
    assert r2["cache_hit"] and r2["chosen"] == r1["chosen"] and B.format == r1["chosen"]
    A.close()
    B.close()


def test_select_prunes_infeasible():
    p = problem("zipf50k")
    A = make_matrix(p)
    rep = A.select(use_cache=False)
    assert rep["status"]["dia"] == dsm.L.E_INFEASIBLE and rep["status"]["ell"] == dsm.L.E_INFEASIBLE
    assert rep["chosen"] in ("csr", "hyb", "coo", "hdc")
    A.close()


def test_select_batched_target():
    torch, dev = torch_dev()
    p = problem("hpcg16")
    A = make_matrix(p)
    rep = A.select(target=1, use_cache=False)
    log(f"[select-batched] chose {rep['chosen']} lanes {rep['chosen_variant']} times {rep['median_us']}")
    assert rep["chosen"] in ("csr", "dia", "ell")
    assert all(rep["status"][f] == dsm.L.E_UNSUPPORTED for f in ("coo", "hyb", "hdc"))
    res = dsm.cg_batched([A], [torch.from_numpy(p.b).to(dev)], [torch.zeros(p.nrows, dtype=torch.float64,
                                                                          device=dev)])[0]
    assert res["status"] == "converged" and abs(res["iters"] - 27) <= 1
    A.close()


@pytest.mark.parametrize("name", ["hpcg104", "zipf50k", "banded20k", "rect_empty"])
def test_online_model_choice(name):
    """reps = 0 picks by the context's cost model (no profiling runs): the
    predicted bytes equal the bytes of the built format, and the model's
    choice, re-timed, is within 25% of the empirically fastest format."""
    torch, dev = torch_dev()
    p = problem(name)
    c = dsm.Context(0)
    A = dsm.Matrix.from_csr(c, p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    emp = A.select(use_cache=False)  # also teaches the context's model
    B = dsm.Matrix.from_csr(c, p.nrows, p.ncols, p.row_ptr, p.col, p.val)
    mod = B.select(use_cache=False, reps=0)
    log(f"[online] {name}: model {mod['chosen']} (pred {mod['median_us']}), timed {emp['chosen']} ({emp['median_us']})")
    for f, st in emp["status"].items():
        if st == 0:
            assert abs(mod["bytes"][f] - emp["bytes"][f]) <= 1e-6 * emp["bytes"][f], f
    x = torch.from_numpy(x_for(p)).to(dev)
    y = torch.empty(p.nrows, dtype=torch.float64, device=dev)
    tm, te = [], []
    for _ in range(3):  # interleaved rounds, the same protocol for both
        tm.append(median_launch_us(B, x, y, 3, 20))
        te.append(median_launch_us(A, x, y, 3, 20))
    t_model, t_emp = float(np.median(tm)), float(np.median(te))
    log(f"[online] {name}: model's pick {t_model:.2f} us, timed pick {t_emp:.2f} us")
    assert t_model <= 1.25 * t_emp, (mod["chosen"], t_model, emp["chosen"], t_emp)
    yref, scale = oracle.spmv_csr_ref(p.row_ptr, p.col, p.val, x_for(p))
    assert row_scaled_err(B.spmv(x).cpu().numpy(), yref, scale) <= 1e-14
    A.close()
    B.close()
    c.close()
