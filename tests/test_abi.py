"""The C ABI library loads and exports every entry point the header
declares (CPU only; no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsc.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("gsc_create", "gsc_pair_create", "gsc_solve", "gsc_mulliken_band",
                 "gsc_band_energy_vjp", "gsc_ased_build", "gsc_ased_vjp", "gsc_spmm",
                 "gsc_solve_batched"):
        assert must in names


def test_library_exports_every_symbol():
    from paper_1002_1202_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgsc.so not built")
    lib = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    # every binding signature names an exported symbol of the header
    assert set(_lib.SIGNATURES) <= set(declared())


def test_opts_default_and_version():
    from paper_1002_1202_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgsc.so not built")
    lib = _lib.load()
    o = _lib.Opts()
    lib.gsc_opts_default(C.byref(o))
    assert o.tol == 1e-10 and o.max_iter == 5000 and o.seed_index == -1
    assert o.carry == _lib.CARRY_FULL and o.precision == _lib.FP64
    assert lib.gsc_version().decode().startswith("gsc")


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the C structs have the header's sizes and offsets."""
    import shutil
    import subprocess
    from paper_1002_1202_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    structs = {"gsc_opts": _lib.Opts, "gsc_stats": _lib.Stats, "gsc_ased_geom": _lib.AsedGeom,
               "gsc_problem": _lib.Problem}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gsc.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_option_defaults_and_binding():
    """gsc_opts_default (a host function) gives the defaults the header
    documents, and make_opts writes every option into its own field."""
    from paper_1002_1202_amd import _lib, api
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgsc.so not built")
    o = _lib.Opts()
    _lib.load().gsc_opts_default(C.byref(o))
    assert (o.tol, o.max_iter, o.inner_tol, o.inner_max_iter) == (1e-10, 5000, 0.0, 200)
    assert (o.precision, o.carry, o.seed_index) == (_lib.FP64, _lib.CARRY_FULL, -1)
    for f in ("fuse_steps", "rhs_tile", "recheck", "spmm_kernel", "inner_method", "graph_iters",
              "stream_hint", "cheb_block", "inner_relax"):
        assert getattr(o, f) == 0, f
    assert o.batch_streams == 0 and o.batch_mem_mb == 0 and o.row_groups == 0 and list(o.reserved) == [0]
    m = api.make_opts(tol=1e-6, fuse_steps=12, cheb_block=128, inner_relax=True, graph_iters=8,
                      precision="mixed", carry="projected")
    assert (m.tol, m.fuse_steps, m.cheb_block, m.inner_relax, m.graph_iters) == (1e-6, 12, 128, 1, 8)
    assert (m.precision, m.carry) == (_lib.MIXED, _lib.CARRY_PROJECTED)
    assert api.make_opts(precision="c64").precision == _lib.C64
    assert list(m.reserved) == [0]
    assert api.make_opts(batch_streams=3).batch_streams == 3
    b = api.make_opts(batch_mem_mb=512, row_groups=64)
    assert (b.batch_mem_mb, b.row_groups) == (512, 64)
