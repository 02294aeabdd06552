"""ctypes view of the FP64 reference oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The library never imports this package.
Every function takes and returns numpy arrays; the arithmetic is in C.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

_i64 = C.c_int64
_i32 = C.c_int32
_dbl = C.c_double
_p = C.c_void_p


def build(force=True):
    """Compile oracle.c with gcc (no FMA contraction, OpenMP row loops)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def build_timing(out_dir):
    """Timing build of the same source for the CPU baseline: -O3
    -march=native -fopenmp (the compiler may contract multiply-adds), built on
    the machine that runs it, since -march=native describes that host.  Its
    results are timed, never used as expected values."""
    path = os.path.join(out_dir, "liboracle_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-o", path, SRC_PATH, "-lm"]
    subprocess.check_call(cmd)
    return path


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _load(LIB_PATH)
    return _lib


def use_build(path):
    """Routes this module's functions to another build of oracle.c (the
    timing build); use_build(None) returns to the check build."""
    global _lib
    _lib = _load(path) if path else None


def _load(path):
    L = C.CDLL(path)
    sig = {
        "orc_set_threads": (_i32, [_i32]),
        "orc_csr_validate": (_i32, [_i64, _i64, _i64, _p, _p]),
        "orc_spmv_csr": (None, [_i64, _p, _p, _p, _p, _p]),
        "orc_spmv_csr_ref": (None, [_i64, _p, _p, _p, _p, _p, _p]),
        "orc_csr_to_coo": (None, [_i64, _p, _p]),
        "orc_coo_to_csr": (_i32, [_i64, _i64, _i64, _p, _p, _p, _p, _p, _p]),
        "orc_spmv_coo": (None, [_i64, _i64, _p, _p, _p, _p, _p]),
        "orc_dia_count": (_i64, [_i64, _i64, _p, _p, _p]),
        "orc_csr_to_dia": (None, [_i64, _i64, _p, _p, _p, _i64, _p, _p]),
        "orc_dia_to_csr": (_i64, [_i64, _i64, _i64, _p, _p, _p, _p, _p]),
        "orc_spmv_dia": (None, [_i64, _i64, _i64, _p, _p, _p, _p]),
        "orc_ell_width": (_i32, [_i64, _p]),
        "orc_csr_to_ell_part": (None, [_i64, _p, _p, _p, _i32, _p, _p]),
        "orc_ell_to_csr": (_i64, [_i64, _i32, _p, _p, _p, _p, _p]),
        "orc_spmv_ell": (None, [_i64, _i32, _p, _p, _p, _p]),
        "orc_hyb_width": (_i32, [_i64, _p]),
        "orc_hyb_coo_count": (_i64, [_i64, _p, _i32]),
        "orc_csr_to_hyb": (None, [_i64, _p, _p, _p, _i32, _p, _p, _p, _p, _p]),
        "orc_hyb_to_csr": (_i64, [_i64, _i32, _p, _p, _i64, _p, _p, _p, _p, _p, _p]),
        "orc_hdc_true_diags": (_i64, [_i64, _i64, _p, _p, _dbl, _p]),
        "orc_csr_to_hdc": (_i64, [_i64, _i64, _p, _p, _p, _i64, _p, _p, _p, _p, _p]),
        "orc_hdc_to_csr": (_i64, [_i64, _i64, _i64, _p, _p, _p, _p, _p, _p, _p, _p]),
        "orc_cast_f32": (None, [_i64, _p, _p]),
        "orc_cast_bf16": (None, [_i64, _p, _p]),
        "orc_bf16_to_f64": (None, [_i64, _p, _p]),
        "orc_row_stats": (None, [_i64, _p, _p]),
        "orc_cg": (_i32, [_i64, _p, _p, _p, _p, _p, _dbl, _i64, _p, _p]),
        "orc_true_relres": (_dbl, [_i64, _p, _p, _p, _p, _p]),
        "orc_extract_diagonal": (None, [_i64, _i64, _p, _p, _p, _p]),
        "orc_update_diagonal": (_i64, [_i64, _i64, _p, _p, _p, _p]),
        "orc_pcg_jacobi": (_i32, [_i64, _p, _p, _p, _p, _p, _dbl, _i64, _p, _p]),
        "orc_symgs": (_i64, [_i64, _p, _p, _p, _p, _p, _p]),
        "orc_mg": (None, [_i32, _p, _p, _p, _p, _p, _p, _p, _p]),
        "orc_pcg_mg": (_i32, [_i32, _p, _p, _p, _p, _p, _p, _p, _p, _dbl, _i64, _p, _p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def set_threads(n):
    return lib().orc_set_threads(int(n))


def csr_validate(nrows, ncols, row_ptr, col):
    rp, c = _c(row_ptr, np.int32), _c(col, np.int32)
    nnz = int(rp[-1]) if rp.size else 0
    return lib().orc_csr_validate(nrows, ncols, len(c), _ptr(rp), _ptr(c)) if rp.size == nrows + 1 else 1


def spmv_csr(row_ptr, col, val, x):
    rp, c, v, xx = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64), _c(x, np.float64)
    n = rp.size - 1
    y = np.empty(n, np.float64)
    lib().orc_spmv_csr(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(y))
    return y


def spmv_csr_ref(row_ptr, col, val, x):
    """(y*, S): Dot2-compensated products and row scales sum_j |a_ij x_j|."""
    rp, c, v, xx = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64), _c(x, np.float64)
    n = rp.size - 1
    y = np.empty(n, np.float64)
    s = np.empty(n, np.float64)
    lib().orc_spmv_csr_ref(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(y), _ptr(s))
    return y, s


def csr_to_coo(row_ptr):
    rp = _c(row_ptr, np.int32)
    n = rp.size - 1
    row = np.empty(int(rp[-1]), np.int32)
    lib().orc_csr_to_coo(n, _ptr(rp), _ptr(row))
    return row


def coo_to_csr(nrows, ncols, row, col, val):
    r, c, v = _c(row, np.int32), _c(col, np.int32), _c(val, np.float64)
    nnz = r.size
    rp = np.empty(nrows + 1, np.int32)
    co = np.empty(nnz, np.int32)
    vo = np.empty(nnz, np.float64)
    st = lib().orc_coo_to_csr(nrows, ncols, nnz, _ptr(r), _ptr(c), _ptr(v), _ptr(rp), _ptr(co), _ptr(vo))
    if st != 0:
        raise ValueError(f"coo_to_csr: status {st}")
    return rp, co, vo


def spmv_coo(nrows, row, col, val, x):
    r, c, v, xx = _c(row, np.int32), _c(col, np.int32), _c(val, np.float64), _c(x, np.float64)
    y = np.empty(nrows, np.float64)
    lib().orc_spmv_coo(nrows, r.size, _ptr(r), _ptr(c), _ptr(v), _ptr(xx), _ptr(y))
    return y


def dia_offsets(nrows, ncols, row_ptr, col):
    rp, c = _c(row_ptr, np.int32), _c(col, np.int32)
    nd = lib().orc_dia_count(nrows, ncols, _ptr(rp), _ptr(c), None)
    offs = np.empty(nd, np.int32)
    lib().orc_dia_count(nrows, ncols, _ptr(rp), _ptr(c), _ptr(offs))
    return offs


def csr_to_dia(nrows, ncols, row_ptr, col, val):
    """Canonical DIA: (offsets int32[ndiag], vals float64[ndiag, nrows])."""
    offs = dia_offsets(nrows, ncols, row_ptr, col)
    rp, c, v = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64)
    vals = np.empty((offs.size, nrows), np.float64)
    lib().orc_csr_to_dia(nrows, ncols, _ptr(rp), _ptr(c), _ptr(v), offs.size, _ptr(offs), _ptr(vals))
    return offs, vals


def dia_to_csr(nrows, ncols, offsets, vals):
    o, dv = _c(offsets, np.int32), _c(vals, np.float64)
    rp = np.empty(nrows + 1, np.int32)
    nnz = lib().orc_dia_to_csr(nrows, ncols, o.size, _ptr(o), _ptr(dv), _ptr(rp), None, None)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    lib().orc_dia_to_csr(nrows, ncols, o.size, _ptr(o), _ptr(dv), _ptr(rp), _ptr(col), _ptr(val))
    return rp, col, val


def spmv_dia(nrows, ncols, offsets, vals, x):
    o, dv, xx = _c(offsets, np.int32), _c(vals, np.float64), _c(x, np.float64)
    y = np.empty(nrows, np.float64)
    lib().orc_spmv_dia(nrows, ncols, o.size, _ptr(o), _ptr(dv), _ptr(xx), _ptr(y))
    return y


def ell_width(row_ptr):
    rp = _c(row_ptr, np.int32)
    return lib().orc_ell_width(rp.size - 1, _ptr(rp))


def csr_to_ell(row_ptr, col, val, K=None):
    """Canonical ELL: (K, col int32[K, nrows], val float64[K, nrows])."""
    rp, c, v = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64)
    n = rp.size - 1
    if K is None:
        K = ell_width(rp)
    ec = np.empty((K, n), np.int32)
    ev = np.empty((K, n), np.float64)
    lib().orc_csr_to_ell_part(n, _ptr(rp), _ptr(c), _ptr(v), K, _ptr(ec), _ptr(ev))
    return K, ec, ev


def ell_to_csr(nrows, ecol, evals):
    ec, ev = _c(ecol, np.int32), _c(evals, np.float64)
    K = ec.shape[0] if ec.ndim == 2 else 0
    rp = np.empty(nrows + 1, np.int32)
    nnz = lib().orc_ell_to_csr(nrows, K, _ptr(ec), _ptr(ev), _ptr(rp), None, None)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    lib().orc_ell_to_csr(nrows, K, _ptr(ec), _ptr(ev), _ptr(rp), _ptr(col), _ptr(val))
    return rp, col, val


def spmv_ell(nrows, ecol, evals, x):
    ec, ev, xx = _c(ecol, np.int32), _c(evals, np.float64), _c(x, np.float64)
    K = ec.shape[0] if ec.ndim == 2 else 0
    y = np.empty(nrows, np.float64)
    lib().orc_spmv_ell(nrows, K, _ptr(ec), _ptr(ev), _ptr(xx), _ptr(y))
    return y


def hyb_width(row_ptr):
    rp = _c(row_ptr, np.int32)
    return lib().orc_hyb_width(rp.size - 1, _ptr(rp))


def csr_to_hyb(row_ptr, col, val, Kh=None):
    """Canonical HYB: dict(Kh, ell_col[Kh, n], ell_val[Kh, n], coo_row, coo_col, coo_val)."""
    rp, c, v = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64)
    n = rp.size - 1
    if Kh is None:
        Kh = hyb_width(rp)
    nc = lib().orc_hyb_coo_count(n, _ptr(rp), Kh)
    ec = np.empty((Kh, n), np.int32)
    ev = np.empty((Kh, n), np.float64)
    cr = np.empty(nc, np.int32)
    cc = np.empty(nc, np.int32)
    cv = np.empty(nc, np.float64)
    lib().orc_csr_to_hyb(n, _ptr(rp), _ptr(c), _ptr(v), Kh, _ptr(ec), _ptr(ev), _ptr(cr), _ptr(cc), _ptr(cv))
    return dict(Kh=Kh, ell_col=ec, ell_val=ev, coo_row=cr, coo_col=cc, coo_val=cv)


def hyb_to_csr(nrows, h):
    ec, ev = _c(h["ell_col"], np.int32), _c(h["ell_val"], np.float64)
    cr, cc, cv = _c(h["coo_row"], np.int32), _c(h["coo_col"], np.int32), _c(h["coo_val"], np.float64)
    nnz = int((ec >= 0).sum()) + cr.size
    rp = np.empty(nrows + 1, np.int32)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    lib().orc_hyb_to_csr(nrows, int(h["Kh"]), _ptr(ec), _ptr(ev), cr.size, _ptr(cr), _ptr(cc), _ptr(cv),
                         _ptr(rp), _ptr(col), _ptr(val))
    return rp, col, val


def hdc_true_diags(nrows, ncols, row_ptr, col, theta=0.5):
    rp, c = _c(row_ptr, np.int32), _c(col, np.int32)
    nt = lib().orc_hdc_true_diags(nrows, ncols, _ptr(rp), _ptr(c), float(theta), None)
    out = np.empty(nt, np.int32)
    lib().orc_hdc_true_diags(nrows, ncols, _ptr(rp), _ptr(c), float(theta), _ptr(out))
    return out


def csr_to_hdc(nrows, ncols, row_ptr, col, val, theta=0.5):
    """Canonical HDC: dict(offsets, dia_val[nt, n], csr_row_ptr, csr_col, csr_val)."""
    offs = hdc_true_diags(nrows, ncols, row_ptr, col, theta)
    rp, c, v = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64)
    dv = np.empty((offs.size, nrows), np.float64)
    crp = np.empty(nrows + 1, np.int32)
    nz = lib().orc_csr_to_hdc(nrows, ncols, _ptr(rp), _ptr(c), _ptr(v), offs.size, _ptr(offs), _ptr(dv),
                              _ptr(crp), None, None)
    ccol = np.empty(nz, np.int32)
    cval = np.empty(nz, np.float64)
    lib().orc_csr_to_hdc(nrows, ncols, _ptr(rp), _ptr(c), _ptr(v), offs.size, _ptr(offs), _ptr(dv),
                         _ptr(crp), _ptr(ccol), _ptr(cval))
    return dict(offsets=offs, dia_val=dv, csr_row_ptr=crp, csr_col=ccol, csr_val=cval, theta=theta)


def hdc_to_csr(nrows, ncols, h):
    o, dv = _c(h["offsets"], np.int32), _c(h["dia_val"], np.float64)
    crp, cc, cv = _c(h["csr_row_ptr"], np.int32), _c(h["csr_col"], np.int32), _c(h["csr_val"], np.float64)
    cap = int(np.count_nonzero(dv)) + cc.size
    rp = np.empty(nrows + 1, np.int32)
    col = np.empty(cap, np.int32)
    val = np.empty(cap, np.float64)
    nnz = lib().orc_hdc_to_csr(nrows, ncols, o.size, _ptr(o), _ptr(dv), _ptr(crp), _ptr(cc), _ptr(cv),
                               _ptr(rp), _ptr(col), _ptr(val))
    return rp, col[:nnz].copy(), val[:nnz].copy()


def cast_f32(v):
    a = _c(v, np.float64)
    out = np.empty(a.size, np.float32)
    lib().orc_cast_f32(a.size, _ptr(a), _ptr(out))
    return out


def cast_bf16(v):
    """BF16 bit patterns (uint16) of RNE(RNE_f32(v))."""
    a = _c(v, np.float64)
    out = np.empty(a.size, np.uint16)
    lib().orc_cast_bf16(a.size, _ptr(a), _ptr(out))
    return out


def bf16_to_f64(bits):
    a = _c(bits, np.uint16)
    out = np.empty(a.size, np.float64)
    lib().orc_bf16_to_f64(a.size, _ptr(a), _ptr(out))
    return out


def row_stats(row_ptr):
    """dict(max, min, sum, sumsq, empty, hist[33])."""
    rp = _c(row_ptr, np.int32)
    out = np.empty(38, np.int64)
    lib().orc_row_stats(rp.size - 1, _ptr(rp), _ptr(out))
    return dict(max=int(out[0]), min=int(out[1]), sum=int(out[2]), sumsq=int(out[3]),
                empty=int(out[4]), hist=out[5:].copy())


STATUS = {0: "converged", 1: "not_converged", 2: "breakdown"}


def cg(row_ptr, col, val, b, x0=None, tol=1e-10, maxit=None):
    """Plain FP64 CG; returns (x, iters, relres_recursive, status)."""
    rp, c, v, bb = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64), _c(b, np.float64)
    n = rp.size - 1
    x = np.zeros(n, np.float64) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if maxit is None:
        maxit = min(10 * n, 20000)
    it = C.c_int64(0)
    rr = C.c_double(0.0)
    st = lib().orc_cg(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(bb), _ptr(x), float(tol), int(maxit),
                      C.addressof(it), C.addressof(rr))
    return x, int(it.value), float(rr.value), STATUS[st]


def true_relres(row_ptr, col, val, b, x):
    rp, c, v, bb, xx = (_c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64),
                        _c(b, np.float64), _c(x, np.float64))
    return lib().orc_true_relres(rp.size - 1, _ptr(rp), _ptr(c), _ptr(v), _ptr(bb), _ptr(xx))


def extract_diagonal(nrows, ncols, row_ptr, col, val):
    rp, c, v = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64)
    d = np.empty(min(nrows, ncols), np.float64)
    lib().orc_extract_diagonal(nrows, ncols, _ptr(rp), _ptr(c), _ptr(v), _ptr(d))
    return d


def update_diagonal(nrows, ncols, row_ptr, col, val, d):
    """Returns (new values, number of missing entries with d != 0)."""
    rp, c, dd = _c(row_ptr, np.int32), _c(col, np.int32), _c(d, np.float64)
    v = np.array(val, dtype=np.float64, copy=True)
    bad = lib().orc_update_diagonal(nrows, ncols, _ptr(rp), _ptr(c), _ptr(v), _ptr(dd))
    return v, int(bad)


PCG_STATUS = {0: "converged", 1: "not_converged", 2: "breakdown", 3: "zero_diagonal"}


def pcg_jacobi(row_ptr, col, val, b, x0=None, tol=1e-10, maxit=None):
    """Jacobi-preconditioned FP64 CG; returns (x, iters, relres, status)."""
    rp, c, v, bb = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64), _c(b, np.float64)
    n = rp.size - 1
    x = np.zeros(n, np.float64) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if maxit is None:
        maxit = min(10 * n, 20000)
    it = C.c_int64(0)
    rr = C.c_double(0.0)
    st = lib().orc_pcg_jacobi(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(bb), _ptr(x), float(tol), int(maxit),
                              C.addressof(it), C.addressof(rr))
    return x, int(it.value), float(rr.value), PCG_STATUS[st]


def symgs(row_ptr, col, val, r, x0, order=None):
    """One symmetric Gauss-Seidel sweep (forward then backward over `order`,
    natural order when None) on A x = r from x0; returns (x, bad) where bad
    counts rows with a zero or missing diagonal (x unchanged then)."""
    rp, c, v, rr = _c(row_ptr, np.int32), _c(col, np.int32), _c(val, np.float64), _c(r, np.float64)
    n = rp.size - 1
    x = np.array(x0, dtype=np.float64, copy=True)
    o = None if order is None else _c(order, np.int32)
    bad = lib().orc_symgs(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(rr), _ptr(x), _ptr(o) if o is not None else None)
    return x, int(bad)


class _Levels:
    """Keeps the per-level arrays alive and exposes them as C pointer arrays.
    levels: list of dicts with row_ptr, col, val, order (None = natural) and,
    for every level but the coarsest, f2c (level l+1 row -> level l row)."""

    def __init__(self, levels):
        self.keep = []
        L = len(levels)
        self.nlev = L
        self.n = np.array([len(lv["row_ptr"]) - 1 for lv in levels], dtype=np.int64)
        P = C.c_void_p * L
        arrs = {k: [] for k in ("rp", "col", "val", "ord", "f2c")}
        for i, lv in enumerate(levels):
            rp, c, v = _c(lv["row_ptr"], np.int32), _c(lv["col"], np.int32), _c(lv["val"], np.float64)
            o = lv.get("order")
            o = np.arange(self.n[i], dtype=np.int32) if o is None else _c(o, np.int32)
            f = lv.get("f2c") if i < L - 1 else None
            f = _c(f, np.int32) if f is not None else np.zeros(1, np.int32)
            self.keep += [rp, c, v, o, f]
            arrs["rp"].append(rp.ctypes.data)
            arrs["col"].append(c.ctypes.data if c.size else None)
            arrs["val"].append(v.ctypes.data if v.size else None)
            arrs["ord"].append(o.ctypes.data if o.size else None)
            arrs["f2c"].append(f.ctypes.data)
        self.ptrs = {k: P(*vs) for k, vs in arrs.items()}

    def args(self):
        p = self.ptrs
        return (self.nlev, self.n.ctypes.data, C.addressof(p["rp"]), C.addressof(p["col"]), C.addressof(p["val"]),
                C.addressof(p["ord"]), C.addressof(p["f2c"]))


def mg(levels, r):
    """One multigrid V-cycle z = M r (from z = 0) over `levels`."""
    Lv = _Levels(levels)
    rr = _c(r, np.float64)
    z = np.empty(Lv.n[0], np.float64)
    lib().orc_mg(*Lv.args(), _ptr(rr), _ptr(z))
    return z


def pcg_mg(levels, b, x0=None, tol=1e-10, maxit=None):
    """CG preconditioned by one V-cycle per iteration; returns (x, iters,
    relres, status)."""
    Lv = _Levels(levels)
    bb = _c(b, np.float64)
    n = int(Lv.n[0])
    x = np.zeros(n, np.float64) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if maxit is None:
        maxit = min(10 * n, 20000)
    it = C.c_int64(0)
    rr = C.c_double(0.0)
    st = lib().orc_pcg_mg(*Lv.args(), _ptr(bb), _ptr(x), float(tol), int(maxit), C.addressof(it), C.addressof(rr))
    return x, int(it.value), float(rr.value), PCG_STATUS[st]
