"""The streaming probes that give the bandwidth ceiling: exact results on
sizes that leave a ragged tail, and argument checks before any launch."""
import pytest

import paper_2209_06478_amd as dsm
from gpu_common import log, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [2, 1000, 4096 * 256 * 4 * 2 + 6])
def test_probe_results(n):
    torch, dev = torch_dev()
    log(f"[probe] n={n}")
    g = torch.Generator().manual_seed(n)
    src = torch.rand(n, dtype=torch.float64, generator=g).to(dev)
    part = torch.full((dsm.PROBE_PARTIALS,), float("nan"), dtype=torch.float64, device=dev)
    dsm.stream_probe("read", part, src)
    torch.cuda.synchronize()
    assert torch.isfinite(part).all()
    assert abs(float(part.sum()) - float(src.sum())) <= 1e-12 * n
    dst = torch.full((n,), -1.0, dtype=torch.float64, device=dev)
    dsm.stream_probe("copy", dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    dsm.stream_probe("write", dst)
    torch.cuda.synchronize()
    assert int((dst != 0).sum()) == 0


def test_probe_rejects_bad_arguments():
    torch, dev = torch_dev()
    a = torch.zeros(64, dtype=torch.float64, device=dev)
    L = dsm.lib()
    import ctypes as C
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = C.c_void_p(a.data_ptr())
    assert L.dsm_stream_probe(7, p, p, 64, s) == dsm.L.E_INVALID                     # mode
    assert L.dsm_stream_probe(dsm.L.PROBE_COPY, p, p, 24, s) == dsm.L.E_INVALID      # not a multiple of 16
    assert L.dsm_stream_probe(dsm.L.PROBE_COPY, None, p, 64, s) == dsm.L.E_INVALID   # null src
    odd = C.c_void_p(a.data_ptr() + 8)
    assert L.dsm_stream_probe(dsm.L.PROBE_WRITE, None, odd, 32, s) == dsm.L.E_INVALID  # misaligned
    torch.cuda.synchronize()
    assert int((a != 0).sum()) == 0


@pytest.mark.parametrize("n,xlen", [(0, 10), (5, 3), (1000, 777), (4096 * 256 * 16 + 11, 100003)])
def test_gather_probe_sums(n, xlen):
    """The gather probe adds x[idx[k]] over every index in range and nothing
    for the ones outside [0, xlen) (negative and too large alike)."""
    torch, dev = torch_dev()
    import numpy as np
    import inputs
    x = inputs.uniform_vector(xlen, seed=n + 1)
    idx = (inputs.uniform(5, n, np.arange(n, dtype=np.uint64)) * (xlen + 20)).astype(np.int64) - 10
    ok = (idx >= 0) & (idx < xlen)
    expect = float(np.sum(x[idx[ok]])) if n else 0.0
    part = torch.full((dsm.PROBE_PARTIALS,), float("nan"), dtype=torch.float64, device=dev)
    dsm.gather_probe(torch.from_numpy(x).to(dev), torch.from_numpy(idx.astype(np.int32)).to(dev), part)
    torch.cuda.synchronize()
    assert abs(float(part.sum()) - expect) <= 1e-12 * max(n, 1)
