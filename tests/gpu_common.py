"""Shared helpers of the GPU parity tests (inputs from `inputs`, expected
values from `oracle`, results from the HIP library through its binding)."""
import functools
import sys

import numpy as np

import inputs
import oracle

FORMATS = ["coo", "csr", "dia", "ell", "hyb", "hdc"]


@functools.lru_cache(maxsize=None)
def anchors():
    """Oracle iteration counts at full sizes (tests/golden/cg_anchors.json,
    written by tests/golden/make_cg_anchors.py from the oracle)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cg_anchors.json")) as f:
        return json.load(f)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


@functools.lru_cache(maxsize=None)
def ctx():
    import paper_2209_06478_amd as dsm
    return dsm.Context(0)


@functools.lru_cache(maxsize=None)
def problem(name):
    """Named seeded workloads (cached for the session)."""
    if name.startswith("hpcg"):
        return inputs.hpcg27(int(name[4:]))
    if name.startswith("aniso"):
        return inputs.aniso7(int(name[5:]))
    if name == "zipf1m":
        return inputs.zipf()
    if name == "banded1m":
        return inputs.banded()
    if name == "zipf50k":
        return inputs.zipf(nrows=50000, seed=5)
    if name == "banded20k":
        return inputs.banded(nrows=20000, seed=6)
    if name == "rect_empty":
        return inputs.random_sparse(300, 217, 0.04, 11, empty_rows=0.3)
    if name == "rand_dense":
        return inputs.random_sparse(257, 257, 0.35, 12)
    if name == "one_by_one":
        return inputs.random_sparse(1, 1, 1.0, 13)
    if name == "no_entries":
        return inputs.random_sparse(70, 90, 0.0, 14)
    if name == "long_row":
        return long_row_problem()
    raise KeyError(name)


def long_row_problem():
    """A few rows with thousands of entries among short rows: exercises the
    long-row path of the CSR kernel and COO rows spanning many tiles."""
    nr, nc = 3000, 9000
    lens = np.full(nr, 3, np.int64)
    lens[[0, 5, 1500, 2999]] = [5000, 1025, 8999, 2048]
    lens[100:140] = 0
    rows = np.repeat(np.arange(nr), lens)
    cols = np.concatenate([np.sort(np.argsort(inputs.uniform(7, 100 + r, np.arange(nc, dtype=np.uint64)))[:l])
                           for r, l in enumerate(lens) if l > 0])
    vals = inputs.normal(7, 3, np.arange(rows.size, dtype=np.uint64))
    vals[vals == 0] = 1.0
    from inputs.generators import _finish
    return _finish("long_row", nr, nc, rows, cols, vals, {})


def make_matrix(p):
    import paper_2209_06478_amd as dsm
    return dsm.Matrix.from_csr(ctx(), p.nrows, p.ncols, p.row_ptr, p.col, p.val)


def x_for(p, seed=0x16C0FFEE):
    return inputs.uniform_vector(p.ncols, seed=seed)


def row_scaled_err(y, yref, scale):
    if y.size == 0:
        return 0.0
    d = np.abs(y - yref)
    return float(np.max(np.where(d == 0, 0.0, d / np.maximum(scale, 1e-300))))
