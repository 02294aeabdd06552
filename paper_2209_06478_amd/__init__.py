"""Dynamic sparse matrices on MI355X: Python binding of libdsm (include/dsm.h).

This module only marshals arguments: torch CUDA tensors (or numpy arrays for
host-side inputs/outputs) go in, the C ABI does the work on the GPU.  If the
HIP library has not been built, every entry point raises: there is no CPU
fallback.

    ctx = Context()
    A = Matrix.from_csr(ctx, n, n, row_ptr, col, val)   # active format CSR
    A.convert("dia")                                     # on-device, in place
    y = A.spmv(x)                                        # torch tensors on cuda
    rep = A.select()                                     # timed format choice
    x, res = A.cg(b, tol=1e-10)
"""
import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import (COO, CSR, DIA, ELL, HYB, HDC, F64, F32, BF16, FORMATS, FORMAT_NAMES, DTYPES, DTYPE_NAMES,
                   CG_F64, CG_IR, CG_JACOBI, CG_IR_CONT, PROBE_PARTIALS)

__all__ = ["Context", "Matrix", "Server", "DsmError", "lib", "COO", "CSR", "DIA", "ELL", "HYB", "HDC",
           "F64", "F32", "BF16", "FORMATS", "DTYPES", "cg_batched", "stream_probe", "gather_probe", "Multigrid"]

ALL_FORMATS = (1 << 6) - 1


class DsmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status
        self.msg = msg


def lib():
    return L.load()


def _check(st, what=""):
    if st != L.OK:
        msg = lib().dsm_last_error().decode() or lib().dsm_status_string(st).decode()
        raise DsmError(st, f"{what}: {msg}" if what else msg)


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        torch = _torch()
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _fmt(f):
    return FORMATS[f.lower()] if isinstance(f, str) else int(f)


def _dt(d):
    return DTYPES[d.lower()] if isinstance(d, str) else int(d)


def _vec_dtype(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("vectors must be float64 or float32 torch tensors")


def _dev_ptr(t, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA torch tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return C.c_void_p(t.data_ptr())


class Context:
    """A device binding with an optional HBM budget (bytes, 0 = none)."""

    def __init__(self, device=0, hbm_budget=0):
        h = C.c_void_p()
        _check(lib().dsm_ctx_create(int(device), int(hbm_budget), C.byref(h)), "dsm_ctx_create")
        self.h = h
        self.device = device

    def bytes_in_use(self):
        v = C.c_size_t()
        _check(lib().dsm_ctx_bytes_in_use(self.h, C.byref(v)))
        return v.value

    def clear_select_cache(self):
        _check(lib().dsm_select_cache_clear(self.h))

    def close(self):
        if self.h:
            _check(lib().dsm_ctx_destroy(self.h), "dsm_ctx_destroy")
            self.h = None


def _as_host_or_dev(a, dtype_np, name):
    """Returns (pointer, on_device, keepalive)."""
    torch = None
    try:
        torch = _torch()
    except ImportError:
        pass
    if torch is not None and isinstance(a, torch.Tensor):
        if a.is_cuda:
            want = {np.int32: torch.int32, np.float64: torch.float64}[dtype_np]
            if a.dtype != want or not a.is_contiguous():
                raise TypeError(f"{name} must be a contiguous {want} tensor")
            return C.c_void_p(a.data_ptr()), 1, a
        a = a.numpy()
    arr = np.ascontiguousarray(a, dtype=dtype_np)
    return C.c_void_p(arr.ctypes.data if arr.size else 0), 0, arr


class Matrix:
    """A dynamic sparse matrix: one active storage format at a time."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.h = handle

    # ------------------------------------------------------------ creation
    @classmethod
    def from_csr(cls, ctx, nrows, ncols, row_ptr, col, val, stream=None):
        rp, d1, k1 = _as_host_or_dev(row_ptr, np.int32, "row_ptr")
        cc, d2, k2 = _as_host_or_dev(col, np.int32, "col")
        vv, d3, k3 = _as_host_or_dev(val, np.float64, "val")
        if not (d1 == d2 == d3):
            raise ValueError("row_ptr, col and val must all be on the host or all on the device")
        nnz = len(k2) if not hasattr(k2, "numel") else k2.numel()
        h = C.c_void_p()
        _check(lib().dsm_create_csr(ctx.h, int(nrows), int(ncols), int(nnz), rp, cc, vv, d1, _stream(stream),
                                    C.byref(h)), "dsm_create_csr")
        return cls(ctx, h)

    @classmethod
    def from_coo(cls, ctx, nrows, ncols, row, col, val, sorted=True, stream=None):
        rr, d1, k1 = _as_host_or_dev(row, np.int32, "row")
        cc, d2, k2 = _as_host_or_dev(col, np.int32, "col")
        vv, d3, k3 = _as_host_or_dev(val, np.float64, "val")
        if not (d1 == d2 == d3):
            raise ValueError("row, col and val must all be on the host or all on the device")
        nnz = len(k2) if not hasattr(k2, "numel") else k2.numel()
        h = C.c_void_p()
        _check(lib().dsm_create_coo(ctx.h, int(nrows), int(ncols), int(nnz), rr, cc, vv, int(bool(sorted)), d1,
                                    _stream(stream), C.byref(h)), "dsm_create_coo")
        return cls(ctx, h)

    def close(self):
        if self.h:
            _check(lib().dsm_matrix_destroy(self.h), "dsm_matrix_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ formats
    def convert(self, fmt, value_dtype=None, hdc_theta=0.5, max_pad_ratio=16.0, hyb_width=-1, stream=None):
        o = L.ConvertOpts()
        lib().dsm_convert_opts_default(C.byref(o))
        o.value_dtype = self.info()["value_dtype"] if value_dtype is None else _dt(value_dtype)
        o.hdc_theta = hdc_theta
        o.max_pad_ratio = max_pad_ratio
        o.hyb_width = hyb_width
        _check(lib().dsm_convert(self.h, _fmt(fmt), C.byref(o), _stream(stream)), "dsm_convert")
        return self

    def info(self):
        i = L.Info()
        _check(lib().dsm_get_info(self.h, C.byref(i)), "dsm_get_info")
        d = {k: getattr(i, k) for k, _ in L.Info._fields_}
        d["format_name"] = FORMAT_NAMES[d["format"]]
        return d

    @property
    def format(self):
        return FORMAT_NAMES[self.info()["format"]]

    @property
    def variant(self):
        v = C.c_int32()
        _check(lib().dsm_get_variant(self.h, C.byref(v)))
        return v.value

    @variant.setter
    def variant(self, v):
        _check(lib().dsm_set_variant(self.h, int(v)), "dsm_set_variant")

    def export(self, stream=None):
        """Canonical arrays of the active format as numpy arrays (host copies)."""
        i = self.info()
        n = i["nrows"]
        vnp = {F64: np.float64, F32: np.float32, BF16: np.uint16}[i["value_dtype"]]
        f = i["format"]
        out = {"format": FORMAT_NAMES[f], "value_dtype": DTYPE_NAMES[i["value_dtype"]]}
        b = L.ExportBufs()

        def buf(name, size, dt):
            a = np.empty(size, dt)
            out[name] = a
            return C.c_void_p(a.ctypes.data) if a.size else None

        if f in (CSR, HDC):
            b.row_ptr = buf("row_ptr", n + 1, np.int32)
            b.col = buf("col", i["csr_nnz"], np.int32)
            b.val = buf("val", i["csr_nnz"], vnp)
        if f in (COO, HYB):
            b.row = buf("row", i["coo_nnz"], np.int32)
            b.col = buf("col" if f == COO else "coo_col", i["coo_nnz"], np.int32)
            b.val = buf("val" if f == COO else "coo_val", i["coo_nnz"], vnp)
            if f == HYB:
                out["coo_row"] = out.pop("row")
        if f in (DIA, HDC):
            b.offsets = buf("offsets", i["ndiag"], np.int32)
            b.dia_val = buf("dia_val", i["ndiag"] * n, vnp)
        if f in (ELL, HYB):
            b.ell_col = buf("ell_col", i["ell_width"] * n, np.int32)
            b.ell_val = buf("ell_val", i["ell_width"] * n, vnp)
        _check(lib().dsm_export(self.h, C.byref(b), _stream(stream)), "dsm_export")
        if "dia_val" in out:
            out["dia_val"] = out["dia_val"].reshape(i["ndiag"], n)
        if "ell_col" in out:
            out["ell_col"] = out["ell_col"].reshape(i["ell_width"], n)
            out["ell_val"] = out["ell_val"].reshape(i["ell_width"], n)
        return out

    def row_stats(self, stream=None):
        a = (C.c_int64 * 38)()
        _check(lib().dsm_row_stats(self.h, a, _stream(stream)), "dsm_row_stats")
        v = list(a)
        return dict(max=v[0], min=v[1], sum=v[2], sumsq=v[3], empty=v[4], hist=np.array(v[5:], np.int64))

    def values_exact(self, value_dtype, stream=None):
        """True when converting the stored values to `value_dtype` ("f64",
        "f32", "bf16") loses nothing (every value survives the cast bit for
        bit)."""
        e = C.c_int32(0)
        _check(lib().dsm_values_exact(self.h, _dt(value_dtype), C.byref(e), _stream(stream)), "dsm_values_exact")
        return bool(e.value)

    def diagonal(self, out=None, stream=None):
        """A's diagonal as an FP64 CUDA tensor of length min(nrows, ncols)."""
        torch = _torch()
        i = self.info()
        n = min(i["nrows"], i["ncols"])
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib().dsm_extract_diagonal(self.h, _dev_ptr(out, n, "out"), _stream(stream)), "dsm_extract_diagonal")
        return out

    def set_diagonal(self, d, stream=None):
        """A(i, i) <- d[i] for the diagonal entries the structure holds."""
        i = self.info()
        n = min(i["nrows"], i["ncols"])
        _check(lib().dsm_update_diagonal(self.h, _dev_ptr(d, n, "d"), _stream(stream)), "dsm_update_diagonal")

    # ------------------------------------------------------------ compute
    def spmv(self, x, out=None, stream=None):
        torch = _torch()
        i = self.info()
        vdt = _vec_dtype(x)
        xp = _dev_ptr(x, i["ncols"], "x")
        if out is None:
            out = torch.empty(i["nrows"], dtype=x.dtype, device=x.device)
        if out.dtype != x.dtype:
            raise TypeError("x and out must have the same dtype")
        yp = _dev_ptr(out, i["nrows"], "out")
        _check(lib().dsm_spmv(self.h, xp, yp, vdt, _stream(stream)), "dsm_spmv")
        return out

    def spmv_noalloc(self, x, out, stream=None):
        """out = A x through the allocation-free entry point (the caller
        passes out; the library allocates nothing)."""
        i = self.info()
        vdt = _vec_dtype(x)
        if out.dtype != x.dtype:
            raise TypeError("x and out must have the same dtype")
        _check(lib().dsm_spmv_noalloc(self.h, _dev_ptr(x, i["ncols"], "x"), _dev_ptr(out, i["nrows"], "out"), vdt,
                                      _stream(stream)), "dsm_spmv_noalloc")
        return out

    def spmv_accumulate(self, x, out, stream=None):
        """out += A x (device vectors of the same dtype)."""
        i = self.info()
        vdt = _vec_dtype(x)
        if out.dtype != x.dtype:
            raise TypeError("x and out must have the same dtype")
        _check(lib().dsm_spmv_accumulate(self.h, _dev_ptr(x, i["ncols"], "x"), _dev_ptr(out, i["nrows"], "out"), vdt,
                                         _stream(stream)), "dsm_spmv_accumulate")
        return out

    def kernel_time(self, x, out, stream=None):
        """out = A x; returns the kernel-only duration of that SpMV in
        microseconds (events recorded by its own launches)."""
        i = self.info()
        vdt = _vec_dtype(x)
        if out.dtype != x.dtype:
            raise TypeError("x and out must have the same dtype")
        us = C.c_double(0)
        _check(lib().dsm_spmv_kernel_time(self.h, _dev_ptr(x, i["ncols"], "x"), _dev_ptr(out, i["nrows"], "out"), vdt,
                                          C.byref(us), _stream(stream)), "dsm_spmv_kernel_time")
        return us.value

    def time_spmv(self, x, out=None, warmup=3, reps=20, stream=None):
        """Median SpMV time in microseconds over `reps` event-bracketed
        launches after `warmup` untimed ones (the selection's protocol)."""
        torch = _torch()
        i = self.info()
        vdt = _vec_dtype(x)
        xp = _dev_ptr(x, i["ncols"], "x")
        if out is None:
            out = torch.empty(i["nrows"], dtype=x.dtype, device=x.device)
        yp = _dev_ptr(out, i["nrows"], "out")
        med = C.c_double()
        _check(lib().dsm_time_spmv(self.h, xp, yp, vdt, int(warmup), int(reps), C.byref(med), _stream(stream)),
               "dsm_time_spmv")
        return med.value

    def select(self, mask=ALL_FORMATS, warmup=3, reps=20, use_cache=True, tune_variant=True, vec_dtype="f64",
               value_dtype="f64", max_pad_ratio=16.0, bytes_prefilter=2.0, target=0, flush_bytes=0, stream=None):
        """target 0: time device-wide SpMV; 1: time one-workgroup CG solves.
        flush_bytes > 0: cold timing (a read of that many bytes before each
        timed SpMV, kernel-only times)."""
        o = L.SelectOpts()
        lib().dsm_select_opts_default(C.byref(o))
        o.warmup, o.reps, o.use_cache, o.tune_variant = warmup, reps, int(use_cache), int(tune_variant)
        o.target = int(target)
        o.flush_bytes = int(flush_bytes)
        o.vec_dtype, o.value_dtype = _dt(vec_dtype), _dt(value_dtype)
        o.max_pad_ratio, o.bytes_prefilter = max_pad_ratio, bytes_prefilter
        r = L.SelectReport()
        if isinstance(mask, (list, tuple, set)):
            mask = sum(1 << _fmt(f) for f in mask)
        _check(lib().dsm_select(self.h, int(mask), C.byref(o), C.byref(r), _stream(stream)), "dsm_select")
        return dict(chosen=FORMAT_NAMES[r.chosen], chosen_variant=r.chosen_variant, cache_hit=bool(r.cache_hit),
                    status={FORMAT_NAMES[f]: r.status[f] for f in range(6)},
                    median_us={FORMAT_NAMES[f]: r.median_us[f] for f in range(6)},
                    convert_us={FORMAT_NAMES[f]: r.convert_us[f] for f in range(6)},
                    bytes={FORMAT_NAMES[f]: r.bytes[f] for f in range(6)})

    def cg(self, b, x=None, tol=1e-10, maxit=0, mode="f64", inner_tol=0, check_every=0, max_outer=50,
           stream=None, raise_on_status=False):
        """Solves A x = b (FP64 device vectors).  Returns (x, result dict)."""
        torch = _torch()
        n = self.info()["nrows"]
        if x is None:
            x = torch.zeros(n, dtype=torch.float64, device=b.device)
        if b.dtype != torch.float64 or x.dtype != torch.float64:
            raise TypeError("b and x must be float64")
        o = _cg_opts(tol, maxit, mode, inner_tol, check_every, max_outer)
        r = L.CgResult()
        st = lib().dsm_cg_solve(self.h, _dev_ptr(b, n, "b"), _dev_ptr(x, n, "x"), C.byref(o), C.byref(r),
                                _stream(stream))
        res = _result(r)
        if st not in (L.OK, L.E_NOT_CONVERGED, L.E_BREAKDOWN) or (raise_on_status and st != L.OK):
            _check(st, "dsm_cg_solve")
        return x, res


def _cg_opts(tol, maxit, mode, inner_tol, check_every, max_outer):
    o = L.CgOpts()
    lib().dsm_cg_opts_default(C.byref(o))
    o.tol, o.maxit = tol, int(maxit)
    o.mode = {"f64": CG_F64, "ir": CG_IR, "jacobi": CG_JACOBI, "ir_cont": CG_IR_CONT}[mode] if isinstance(mode, str) else int(mode)
    o.inner_tol, o.check_every, o.max_outer = inner_tol, int(check_every), int(max_outer)
    return o


_STATUS = {L.OK: "converged", L.E_NOT_CONVERGED: "not_converged", L.E_BREAKDOWN: "breakdown"}


def _result(r):
    return dict(iters=r.iters, outer_iters=r.outer_iters, relres=r.relres, relres_true=r.relres_true,
                status=_STATUS.get(r.status, str(r.status)))


def cg_batched(mats, bs, xs, tol=1e-10, maxit=0, stream=None):
    """Solves every (A_k, b_k) pair in one batched call; x_k hold x0 on entry."""
    n = len(mats)
    H = (C.c_void_p * n)(*[m.h for m in mats])
    B = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    X = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    tols = tol if isinstance(tol, (list, tuple)) else [tol] * n
    O = (L.CgOpts * n)(*[_cg_opts(t, maxit, "f64", 1e-4, 0, 50) for t in tols])
    R = (L.CgResult * n)()
    _check(lib().dsm_cg_solve_batched(n, H, B, X, O, R, _stream(stream)), "dsm_cg_solve_batched")
    return [_result(r) for r in R]


def stream_probe(mode, dst, src=None, stream=None):
    """One streaming kernel ('read', 'copy' or 'write') over torch device
    buffers; `read` reduces src into dst (PROBE_PARTIALS float64 partials),
    `copy` and `write` move dst.numel() * itemsize bytes."""
    torch = _torch()
    m = {"read": L.PROBE_READ, "copy": L.PROBE_COPY, "write": L.PROBE_WRITE}[mode]
    if m == L.PROBE_READ:
        if dst.dtype != torch.float64 or dst.numel() < L.PROBE_PARTIALS or not dst.is_cuda:
            raise ValueError(f"read mode needs a float64 CUDA dst of at least {L.PROBE_PARTIALS} elements")
        nbytes = src.numel() * src.element_size()
    else:
        nbytes = dst.numel() * dst.element_size()
        if m == L.PROBE_COPY and (src is None or src.numel() * src.element_size() < nbytes):
            raise ValueError("copy needs a src at least as large as dst")
    sp = C.c_void_p(src.data_ptr()) if src is not None else C.c_void_p(None)
    _check(lib().dsm_stream_probe(m, sp, C.c_void_p(dst.data_ptr()), nbytes, _stream(stream)), "dsm_stream_probe")


def gather_probe(x, idx, part, stream=None):
    """Sums x[idx[k]] (FP64 x, int32 idx, CUDA tensors) into
    PROBE_PARTIALS FP64 partials: the gather traffic of an irregular SpMV."""
    torch = _torch()
    if x.dtype != torch.float64 or idx.dtype != torch.int32 or part.dtype != torch.float64:
        raise TypeError("x and part must be float64, idx int32")
    if part.numel() < L.PROBE_PARTIALS or not (x.is_cuda and idx.is_cuda and part.is_cuda):
        raise ValueError(f"CUDA tensors needed, part of at least {L.PROBE_PARTIALS} elements")
    _check(lib().dsm_gather_probe(C.c_void_p(x.data_ptr()), x.numel(), C.c_void_p(idx.data_ptr()), idx.numel(),
                                  C.c_void_p(part.data_ptr()), _stream(stream)), "dsm_gather_probe")


class Server:
    """Continuous-batching CG server over one context."""

    def __init__(self, ctx, slots=64, hbm_budget=0, streams=4, small_rows=4096, batch_max=256):
        o = L.ServerOpts()
        lib().dsm_server_opts_default(C.byref(o))
        o.slots, o.hbm_budget, o.streams, o.small_rows, o.batch_max = slots, hbm_budget, streams, small_rows, batch_max
        h = C.c_void_p()
        _check(lib().dsm_server_create(ctx.h, C.byref(o), C.byref(h)), "dsm_server_create")
        self.h = h
        self.ctx = ctx

    def submit(self, A, b, x, tol=1e-8, maxit=0):
        n = A.info()["nrows"]
        o = _cg_opts(tol, maxit, "f64", 1e-4, 0, 50)
        t = C.c_uint64()
        _check(lib().dsm_server_submit(self.h, A.h, _dev_ptr(b, n, "b"), _dev_ptr(x, n, "x"), C.byref(o),
                                       C.byref(t)), "dsm_server_submit")
        return t.value

    def poll(self, ticket):
        r, ts = L.CgResult(), L.Timestamps()
        st = lib().dsm_server_poll(self.h, ticket, C.byref(r), C.byref(ts))
        if st == L.E_PENDING:
            return None
        _check(st, "dsm_server_poll")
        return _result(r), dict(arrival=ts.arrival_s, start=ts.start_s, finish=ts.finish_s)

    def wait(self, ticket):
        r, ts = L.CgResult(), L.Timestamps()
        _check(lib().dsm_server_wait(self.h, ticket, C.byref(r), C.byref(ts)), "dsm_server_wait")
        return _result(r), dict(arrival=ts.arrival_s, start=ts.start_s, finish=ts.finish_s)

    def now(self):
        return lib().dsm_server_now(self.h)

    def stats(self):
        st = L.ServerStats()
        _check(lib().dsm_server_get_stats(self.h, C.byref(st)), "dsm_server_get_stats")
        return {k: getattr(st, k) for k, _ in L.ServerStats._fields_}

    def close(self):
        if self.h:
            _check(lib().dsm_server_destroy(self.h), "dsm_server_destroy")
            self.h = None


class Multigrid:
    """HPCG's preconditioner over a hierarchy of resident matrices: a
    symmetric Gauss-Seidel smoother (multicolour) in a multigrid V-cycle,
    and CG preconditioned by it.  `levels` are Matrix objects (CSR or DIA,
    FP64), finest first; `f2c[l]` maps level l+1 rows to level l rows;
    `colours[l]` colours level l's rows (no coupling inside a colour)."""

    def __init__(self, ctx, levels, f2c, colours, stream=None):
        import numpy as np
        n = len(levels)
        self._levels = list(levels)  # the hierarchy holds them
        self._keep = [np.ascontiguousarray(c, dtype=np.int32) for c in colours]
        self._keep += [np.ascontiguousarray(f, dtype=np.int32) for f in f2c]
        cols = (C.c_void_p * n)(*[a.ctypes.data for a in self._keep[:n]])
        f2 = (C.c_void_p * max(n - 1, 1))(*([a.ctypes.data for a in self._keep[n:]] or [None]))
        H = (C.c_void_p * n)(*[m.h for m in levels])
        out = C.c_void_p()
        _check(lib().dsm_mg_create(ctx.h, n, H, f2, cols, _stream(stream), C.byref(out)), "dsm_mg_create")
        self.h = out
        self.n = levels[0].info()["nrows"]
        self.sizes = [m.info()["nrows"] for m in levels]

    def close(self):
        if self.h:
            _check(lib().dsm_mg_destroy(self.h), "dsm_mg_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def symgs(self, level, r, x, stream=None):
        """One symmetric Gauss-Seidel sweep on `level`, x updated in place."""
        n = self.sizes[level]
        _check(lib().dsm_mg_symgs(self.h, int(level), _dev_ptr(r, n, "r"), _dev_ptr(x, n, "x"), _stream(stream)),
               "dsm_mg_symgs")
        return x

    def apply(self, r, out=None, stream=None):
        """z = M r (one V-cycle from zero)."""
        torch = _torch()
        z = torch.empty_like(r) if out is None else out
        _check(lib().dsm_mg_apply(self.h, _dev_ptr(r, self.n, "r"), _dev_ptr(z, self.n, "z"), _stream(stream)),
               "dsm_mg_apply")
        return z

    def pcg(self, b, x=None, tol=1e-10, maxit=0, check_every=0, stream=None):
        """CG preconditioned by one V-cycle per iteration; returns (x, result)."""
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        o = _cg_opts(tol, maxit, "f64", 1e-4, check_every, 50)
        R = L.CgResult()
        st = lib().dsm_pcg_mg_solve(self.h, _dev_ptr(b, self.n, "b"), _dev_ptr(x, self.n, "x"), C.byref(o),
                                    C.byref(R), _stream(stream))
        if st not in (L.OK, L.E_NOT_CONVERGED, L.E_BREAKDOWN):
            _check(st, "dsm_pcg_mg_solve")
        return x, _result(R)
