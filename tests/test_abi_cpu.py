"""CPU checks of the boundary: the built library loads, exports every symbol
the header declares, and the ctypes mirrors of the header's structs have the
C layout (checked against gcc's sizeof/offsetof).  No GPU work is issued."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsm.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dsm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2209_06478_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2209_06478_amd import build
        build.build(verbose=False)
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 30
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib._name], text=True)
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_binding_declares_every_function(lib):
    from paper_2209_06478_amd import _lib
    assert sorted(_lib.SIGNATURES) == header_functions()


def test_struct_layouts_match_c():
    from paper_2209_06478_amd import _lib
    prog = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    for cname, cls in _lib.STRUCTS.items():
        prog.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            prog.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    prog.append("return 0;}")
    d = os.path.join(ROOT, "paper_2209_06478_amd", "_build")
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, "layout.c")
    exe = os.path.join(d, "layout")
    open(c, "w").write("\n".join(prog))
    subprocess.check_call(["gcc", "-std=c99", "-o", exe, c])
    got = dict(l.split() for l in subprocess.check_output([exe], text=True).splitlines())
    for cname, cls in _lib.STRUCTS.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_pure_entry_points(lib):
    from paper_2209_06478_amd import _lib
    assert lib.dsm_version() >= 10000
    assert lib.dsm_status_string(_lib.E_NOMEM).decode().startswith("out of device memory")
    o = _lib.CgOpts()
    lib.dsm_cg_opts_default(C.byref(o))
    assert o.tol == 1e-10 and o.mode == _lib.CG_F64
    s = _lib.SelectOpts()
    lib.dsm_select_opts_default(C.byref(s))
    assert s.reps == 20 and s.warmup == 3 and s.bytes_prefilter == 2.0
    co = _lib.ConvertOpts()
    lib.dsm_convert_opts_default(C.byref(co))
    assert co.hdc_theta == 0.5 and co.hyb_width == -1


def test_missing_library_fails_loudly(tmp_path):
    from paper_2209_06478_amd import _lib
    saved = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            _lib.load(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved
