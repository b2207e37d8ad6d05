"""CPU checks of the HIP library boundary: the shared library loads without a GPU, exports
every function the public header declares, and its host-only entry points behave."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rok4e.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rok4e_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1712_00953_amd import rok4e as R
    if not os.path.exists(R.LIB_PATH):
        from paper_1712_00953_amd import build
        build.build()
    return R.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("rok4e_mech_create", "rok4e_integrate", "rok4e_integrate_forced", "rok4e_rhs",
              "rok4e_arnoldi", "rok4e_reserve", "rok4e_get_stats", "rok4e_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1712_00953_amd import rok4e as R
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(R.EXPORTS) == names


def test_host_only_entry_points(lib):
    from paper_1712_00953_amd import rok4e as R
    assert R.strerror(0) == "ok"
    assert "invalid" in R.strerror(-1)
    assert R.strerror(12345) == "unknown error"
    o = R.Options()
    lib.rok4e_options_default(C.byref(o))
    assert o.M == 4 and o.precision == R.FP64 and o.scheduling == R.PERSISTENT


def test_argument_errors_before_any_device_work(lib):
    from paper_1712_00953_amd import rok4e as R
    # null handles and descriptions are rejected on the host
    assert lib.rok4e_mech_create(None, None, None) == R.EINVAL
    assert lib.rok4e_integrate(4, None, None, None, None, 1e-6, 1e-6, 1e-12, None) == R.EINVAL
    assert lib.rok4e_reserve(None, 10) == R.EINVAL
    assert lib.rok4e_mech_destroy(None) == R.OK
    s = R.Stats()
    assert lib.rok4e_get_stats(None, C.byref(s), None) == R.EINVAL


def test_mechanism_with_an_unbalanced_reaction_is_refused(lib):
    """A <=> B where A holds one atom of the element and B two: refused on the host, before
    any device work; so is an element count without its table."""
    import numpy as np
    from paper_1712_00953_amd import rok4e as R
    W, cp, hf = np.array([0.001, 0.002]), np.array([1000.0, 1000.0]), np.zeros(2)
    reac, prod = np.array([0, -1], np.int32), np.array([1, -1], np.int32)
    par = [np.zeros(1) for _ in range(6)]
    elem = np.array([[1], [2]], np.int8)
    arrays = [W, cp, hf, reac, prod, *par]
    for n_el, table in ((1, elem), (1, None)):
        d = R.MechDesc(2, 1, *[a.ctypes.data for a in arrays], n_el,
                       None if table is None else table.ctypes.data)
        h = C.c_void_p()
        assert lib.rok4e_mech_create(C.byref(d), None, C.byref(h)) == R.EINVAL
        assert not h.value


def test_binding_has_no_fallback(monkeypatch, tmp_path):
    from paper_1712_00953_amd import rok4e as R
    monkeypatch.setattr(R, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(R, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        R.load()


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets the C compiler
    gives the header's structs."""
    import subprocess
    from paper_1712_00953_amd import rok4e as R
    structs = {"rok4e_mech_desc": R.MechDesc, "rok4e_options": R.Options, "rok4e_tune_result": R.TuneResult,
               "rok4e_grid": R.Grid, "rok4e_stats": R.Stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rok4e.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, field, value = line.split()
        got[cname, field] = int(value)
    for cname, py in structs.items():
        assert got[cname, "size"] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[cname, fname] == getattr(py, fname).offset, (cname, fname)
