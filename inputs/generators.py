"""Synthetic matrices in canonical CSR (rows ascending, columns strictly
ascending within a row, no stored zeros) and the dense vectors that go with
them.

Matrix families:

* ``hpcg27(n)``: the HPCG problem the paper ports (Section II-B): a
  27-point stencil on an n x n x n grid, diagonal 26, -1 for every neighbour
  that exists, b = A * ones so the exact solution is all ones.  Grid point
  (ix, iy, iz) is row ix + n*iy + n*n*iz; neighbours are generated in
  (dz, dy, dx) nested order, which is ascending column order.
* ``aniso7(n, wz)``: a Dirichlet 7-point Laplacian with z-coupling wz:
  diagonal 2 + 2 + 2*wz, x/y neighbours -1, z neighbours -wz; missing
  neighbours are dropped and the diagonal kept, so A is SPD.
* ``zipf``: row lengths with P(len = k) proportional to k**-s on
  [1, kmax], s fixed so that the mean is 16; distinct uniform columns;
  N(0,1) values.
* ``banded``: diagonal always present, every (i, j) with
  1 <= |i - j| <= hbw present independently with probability p; N(0,1)
  values.
* ``banded_spd``: symmetric banded pattern, off-diagonals N(0,1) mirrored,
  a_ii = sum_j |a_ij| + 1 (strictly diagonally dominant, hence SPD).
* ``random_sparse``: small random patterns for property tests.

Nothing here computes a product, a conversion or a solve; the right-hand
side b = A * ones is part of the problem definition and is formed as a row
sum while the matrix is built.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .rng import uniform, normal

# Exponent s of P(len = k) ~ k**-s on [1, 4096] whose mean is 16 (bisection).
ZIPF_EXPONENT = None  # filled lazily by _zipf_exponent


@dataclass
class Problem:
    name: str
    nrows: int
    ncols: int
    row_ptr: np.ndarray  # int32[nrows + 1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]
    b: np.ndarray = None  # float64[nrows], b = A * ones (square problems)
    params: dict = field(default_factory=dict)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


def _finish(name, nrows, ncols, rows, cols, vals, params, with_b=True):
    """rows/cols/vals in canonical order -> Problem (row_ptr by counting)."""
    counts = np.bincount(rows, minlength=nrows) if rows.size else np.zeros(nrows, np.int64)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("nnz exceeds the int32 index range")
    b = None
    if with_b and nrows == ncols:
        b = np.bincount(rows, weights=vals, minlength=nrows).astype(np.float64)
    return Problem(name, nrows, ncols, row_ptr.astype(np.int32),
                   np.ascontiguousarray(cols, dtype=np.int32),
                   np.ascontiguousarray(vals, dtype=np.float64), b, params)


def _stencil(n, offsets, weights, diag, name, params):
    """Generic structured-grid stencil: offsets (dx, dy, dz) in ascending
    column order, weights per offset (the diagonal uses ``diag``)."""
    N = n ** 3
    idx = np.arange(N, dtype=np.int64)
    ix = idx % n
    iy = (idx // n) % n
    iz = idx // (n * n)
    K = len(offsets)
    cols = np.empty((N, K), dtype=np.int64)
    mask = np.empty((N, K), dtype=bool)
    vals = np.empty((N, K), dtype=np.float64)
    for k, ((dx, dy, dz), w) in enumerate(zip(offsets, weights)):
        m = np.ones(N, dtype=bool)
        if dx:
            m &= (ix + dx >= 0) & (ix + dx < n)
        if dy:
            m &= (iy + dy >= 0) & (iy + dy < n)
        if dz:
            m &= (iz + dz >= 0) & (iz + dz < n)
        mask[:, k] = m
        cols[:, k] = idx + dx + n * dy + n * n * dz
        vals[:, k] = diag if (dx, dy, dz) == (0, 0, 0) else w
    lens = mask.sum(axis=1)
    rows = np.repeat(np.arange(N, dtype=np.int64), lens)
    c = cols[mask]
    v = vals[mask]
    del cols, mask, vals
    return _finish(name, N, N, rows, c, v, params)


def hpcg27(n):
    """HPCG 27-point stencil on n^3 (diagonal 26, neighbours -1)."""
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return _stencil(n, offs, [-1.0] * 27, 26.0, f"hpcg27_{n}", {"n": n})


def hpcg27_levels(n, nlev=4):
    """HPCG's multigrid hierarchy: the 27-point problem on n^3, (n/2)^3, ...
    (n divisible by 2^(nlev-1)).  Per level: the Problem, an 8-colour
    parity colouring (rows of one colour share no stencil entry), and, for
    every level but the coarsest, f2c: the fine row under each row of the
    next level (coarse point (ix, iy, iz) sits on fine point (2 ix, 2 iy,
    2 iz)).

    colour = 7 - ((ix & 1) + 2 (iy & 1) + 4 (iz & 1)): the all-even points,
    where the residual is injected, form colour 7, the colour a forward
    sweep visits last and a backward sweep first.  Had they been the colour
    the pre-smoothing sweep updates last, each of them would be solved
    exactly against neighbours that no longer change, the injected residual
    would be rounding noise and the coarse levels would add nothing."""
    if n % (1 << (nlev - 1)):
        raise ValueError(f"n={n} is not divisible by 2^{nlev - 1}")
    levels = []
    for l in range(nlev):
        m = n >> l
        idx = np.arange(m ** 3, dtype=np.int64)
        ix, iy, iz = idx % m, (idx // m) % m, idx // (m * m)
        colour = (7 - ((ix & 1) + 2 * (iy & 1) + 4 * (iz & 1))).astype(np.int32)
        lv = {"problem": hpcg27(m), "colour": colour}
        if l < nlev - 1:
            c = m // 2
            cidx = np.arange(c ** 3, dtype=np.int64)
            cx, cy, cz = cidx % c, (cidx // c) % c, cidx // (c * c)
            lv["f2c"] = (2 * cx + m * 2 * cy + m * m * 2 * cz).astype(np.int32)
        levels.append(lv)
    return levels


def aniso7(n, wz=100.0):
    """Dirichlet 7-point Laplacian on n^3 with z-coupling wz."""
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    w = [-wz, -1.0, -1.0, 0.0, -1.0, -1.0, -wz]
    return _stencil(n, offs, w, 4.0 + 2.0 * wz, f"aniso7_{n}", {"n": n, "wz": wz})


def _nonzero_normals(seed, stream, count):
    """N(0,1) draws with exact zeros redrawn from follow-on streams."""
    v = normal(seed, stream, np.arange(count, dtype=np.uint64))
    extra = 1
    while True:
        z = np.flatnonzero(v == 0.0)
        if z.size == 0:
            return v
        v[z] = normal(seed, stream + 1000 * extra, z.astype(np.uint64))
        extra += 1


def _zipf_exponent(mean=16.0, kmax=4096):
    k = np.arange(1, kmax + 1, dtype=np.float64)
    lo, hi = 1.0, 4.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        p = k ** -mid
        if (k * p).sum() / p.sum() > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def zipf(nrows=1_000_000, mean=16.0, kmax=4096, seed=0x21FF, ncols=None):
    """Zipf row lengths (pmf ~ k^-s, mean ``mean``, max ``kmax``), distinct
    uniform columns per row, N(0,1) values."""
    global ZIPF_EXPONENT
    ncols = nrows if ncols is None else ncols
    s = _zipf_exponent(mean, kmax)
    ZIPF_EXPONENT = s
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** -s
    cdf = np.cumsum(p) / p.sum()
    u = uniform(seed, 1, np.arange(nrows, dtype=np.uint64))
    lens = np.minimum(np.searchsorted(cdf, u, side="right") + 1, min(kmax, ncols))
    nnz = int(lens.sum())
    rows = np.repeat(np.arange(nrows, dtype=np.int64), lens)
    cols = np.floor(uniform(seed, 2, np.arange(nnz, dtype=np.uint64)) * ncols).astype(np.int64)
    rnd = 0
    while True:
        key = rows * ncols + cols
        order = np.argsort(key, kind="stable")
        key = key[order]
        rows, cols = rows[order], cols[order]
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            break
        rnd += 1
        cols[dup] = np.floor(uniform(seed, 100 + rnd, dup.astype(np.uint64)) * ncols).astype(np.int64)
    vals = _nonzero_normals(seed, 3, nnz)
    return _finish(f"zipf_{nrows}", nrows, ncols, rows, cols, vals,
                   {"mean": mean, "kmax": kmax, "seed": seed, "s": s})


def banded(nrows=1_000_000, hbw=64, p=0.3, seed=0xBA4D, chunk=1 << 17):
    """Banded: diagonal always, off-diagonals within hbw present w.p. p."""
    W = 2 * hbw + 1
    rows_l, cols_l = [], []
    for r0 in range(0, nrows, chunk):
        r1 = min(nrows, r0 + chunk)
        i = np.arange(r0, r1, dtype=np.int64)[:, None]
        d = np.arange(-hbw, hbw + 1, dtype=np.int64)[None, :]
        j = i + d
        cnt = (i * W + (d + hbw)).astype(np.uint64)
        keep = uniform(seed, 1, cnt.ravel()).reshape(j.shape) < p
        keep |= d == 0
        keep &= (j >= 0) & (j < nrows)
        rows_l.append(np.broadcast_to(i, j.shape)[keep])
        cols_l.append(j[keep])
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = _nonzero_normals(seed, 3, rows.size)
    return _finish(f"banded_{nrows}", nrows, nrows, rows, cols, vals,
                   {"hbw": hbw, "p": p, "seed": seed})


def banded_spd(nrows, hbw, fill=0.3, seed=0x5E4E):
    """Symmetric banded SPD: mirrored N(0,1) off-diagonals, a_ii = sum|a_ij| + 1."""
    i = np.arange(nrows, dtype=np.int64)[:, None]
    d = np.arange(1, hbw + 1, dtype=np.int64)[None, :]
    j = i + d
    cnt = (i * hbw + (d - 1)).astype(np.uint64)
    keep = (uniform(seed, 1, cnt.ravel()).reshape(j.shape) < fill) & (j < nrows)
    ui = np.broadcast_to(i, j.shape)[keep]
    uj = j[keep]
    uv = _nonzero_normals(seed, 3, ui.size)
    absum = np.bincount(ui, weights=np.abs(uv), minlength=nrows) + \
        np.bincount(uj, weights=np.abs(uv), minlength=nrows)
    dg = absum + 1.0
    rows = np.concatenate([ui, uj, np.arange(nrows, dtype=np.int64)])
    cols = np.concatenate([uj, ui, np.arange(nrows, dtype=np.int64)])
    vals = np.concatenate([uv, uv, dg])
    order = np.argsort(rows * nrows + cols, kind="stable")
    return _finish(f"banded_spd_{nrows}_{hbw}", nrows, nrows, rows[order], cols[order],
                   vals[order], {"hbw": hbw, "fill": fill, "seed": seed})


def random_sparse(nrows, ncols, density, seed, max_row=None, empty_rows=0.0):
    """Small random pattern for property tests (canonical CSR, no zeros).

    ``empty_rows`` is the fraction of rows forced empty; ``max_row`` caps the
    row length by dropping the highest columns of a longer row.
    """
    cnt = np.arange(nrows * ncols, dtype=np.uint64)
    keep = (uniform(seed, 1, cnt) < density).reshape(nrows, ncols)
    if empty_rows > 0:
        er = uniform(seed, 2, np.arange(nrows, dtype=np.uint64)) < empty_rows
        keep[er, :] = False
    if max_row is not None:
        csum = np.cumsum(keep, axis=1)
        keep &= csum <= max_row
    rows, cols = np.nonzero(keep)
    vals = _nonzero_normals(seed, 3, rows.size)
    return _finish(f"rand_{nrows}x{ncols}", nrows, ncols, rows.astype(np.int64),
                   cols.astype(np.int64), vals, {"density": density, "seed": seed})


def hpcg27_rank(n, procs=(2, 2, 2), coords=(0, 0, 0)):
    """One rank's share of an HPCG 27-point problem decomposed over a
    px x py x pz process grid: the rank owns an n^3 sub-grid at `coords`.

    Returns (merged, local, ghost):
      merged  rows = the rank's n^3 points; columns = its own points
              (0 .. n^3-1, same order as hpcg27(n)) followed by the ghost
              points it couples to (sorted by global index) - the
              "local system matrix" a distributed HPCG rank holds;
      local   the square n^3 x n^3 block of couplings inside the sub-grid;
      ghost   the rectangular n^3 x n_ghost block of couplings to
              neighbouring sub-grids.
    merged.b = merged * ones (the global right-hand side of these rows)."""
    px, py, pz = procs
    cx, cy, cz = coords
    gx, gy, gz = n * px, n * py, n * pz
    N = n ** 3
    idx = np.arange(N, dtype=np.int64)
    ix = idx % n + cx * n
    iy = (idx // n) % n + cy * n
    iz = idx // (n * n) + cz * n
    rows_l, gcols_l, vals_l = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                jx, jy, jz = ix + dx, iy + dy, iz + dz
                ok = (jx >= 0) & (jx < gx) & (jy >= 0) & (jy < gy) & (jz >= 0) & (jz < gz)
                rows_l.append(idx[ok])
                gcols_l.append((jx + gx * (jy + gy * jz))[ok])
                vals_l.append(np.full(int(ok.sum()), 26.0 if (dx, dy, dz) == (0, 0, 0) else -1.0))
    rows = np.concatenate(rows_l)
    gcol = np.concatenate(gcols_l)
    vals = np.concatenate(vals_l)
    # local column index of an owned point, or -1
    lx = gcol % gx - cx * n
    ly = (gcol // gx) % gy - cy * n
    lz = gcol // (gx * gy) - cz * n
    own = (lx >= 0) & (lx < n) & (ly >= 0) & (ly < n) & (lz >= 0) & (lz < n)
    lcol = np.where(own, lx + n * ly + n * n * lz, -1)
    ghosts = np.unique(gcol[~own])
    gidx = np.searchsorted(ghosts, gcol[~own])
    mcol = lcol.copy()
    mcol[~own] = N + gidx
    order = np.lexsort((mcol, rows))
    merged = _finish(f"hpcg27_rank_{n}", N, N + ghosts.size, rows[order], mcol[order], vals[order],
                     {"n": n, "procs": procs, "coords": coords}, with_b=False)
    merged.b = np.bincount(rows, weights=vals, minlength=N).astype(np.float64)
    o = np.lexsort((lcol[own], rows[own]))
    local = _finish(f"hpcg27_rank_local_{n}", N, N, rows[own][o], lcol[own][o], vals[own][o], {}, with_b=False)
    g = ~own
    og = np.lexsort((gidx, rows[g]))
    ghost = _finish(f"hpcg27_rank_ghost_{n}", N, ghosts.size, rows[g][og], gidx[og], vals[g][og], {}, with_b=False)
    merged.params["ghost_global"] = ghosts
    return merged, local, ghost


def uniform_vector(n, seed=0x16C0FFEE, stream=7):
    """Seeded uniform[0,1) vector (the SpMV operand of the workloads)."""
    return uniform(seed, stream, np.arange(n, dtype=np.uint64))


def serving_stream(nreq=10_000, seed=0x5E4E, rate=1.0, nmin=8, nmax=96,
                   spd_min=1_000, spd_max=200_000, hbw_max=64):
    """Request descriptors for the serving workload: half 27-point stencils
    with n ~ U{nmin..nmax}, half banded SPD with N log-uniform in
    [spd_min, spd_max] and half-bandwidth ~ U{1..hbw_max}; Poisson arrivals
    at ``rate`` requests per second.  Matrices are built on demand."""
    idx = np.arange(nreq, dtype=np.uint64)
    kind = uniform(seed, 11, idx) < 0.5
    n = nmin + np.floor(uniform(seed, 12, idx) * (nmax - nmin + 1)).astype(np.int64)
    lo, hi = math.log(spd_min), math.log(spd_max)
    N = np.exp(lo + uniform(seed, 13, idx) * (hi - lo)).astype(np.int64)
    hbw = 1 + np.floor(uniform(seed, 14, idx) * hbw_max).astype(np.int64)
    gaps = -np.log(1.0 - uniform(seed, 15, idx)) / rate
    t = np.cumsum(gaps)
    out = []
    for r in range(nreq):
        if kind[r]:
            out.append({"id": r, "kind": "hpcg27", "n": int(n[r]), "arrival": float(t[r])})
        else:
            out.append({"id": r, "kind": "banded_spd", "nrows": int(N[r]), "hbw": int(hbw[r]),
                        "seed": int(seed + r), "arrival": float(t[r])})
    return out
