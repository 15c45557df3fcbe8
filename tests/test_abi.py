"""The C ABI library loads on the CPU and exports every function that
include/*.h declares; host-side argument validation works without a GPU."""
import ctypes
import glob
import os
import re

import pytest

from paper_2011_01740_amd import ens

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b((?:ens|sur)_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_headers_declare_the_boundary():
    names = declared_functions()
    for f in ("ens_create", "ens_set_params", "ens_set_state", "ens_solve", "ens_read",
              "ens_destroy", "sur_create", "sur_train_step", "sur_screen"):
        assert f in names, f


def test_library_exports_every_declared_symbol():
    lib = ens.load()
    missing = [f for f in sorted(declared_functions()) if not hasattr(lib, f)]
    assert not missing, missing


def test_default_opts_are_the_documented_readings():
    o = ens.default_opts()
    assert (o.dt, o.n_steps, o.t_phase, o.dt0) == (0.01, 1000, 1.0, 1e-2)
    assert (o.dt_min, o.dt_max, o.rtol, o.atol) == (1e-14, 0.1, 1e-10, 1e-10)
    assert (o.event_tol, o.t_cap, o.v_stick, o.max_event_iter) == (1e-6, 50.0, 1e-9, 20)
    with pytest.raises(TypeError):
        ens.default_opts(no_such_option=1)


def _c_layout(struct, fields, tmp_path):
    """sizeof and field offsets of a struct of include/ens.h as the C compiler
    lays it out."""
    import subprocess
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ens.h"',
             "int main(void) {", f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("name", ["ens_desc", "ens_solve_opts"])
def test_struct_layouts_match_the_header(name, tmp_path):
    cls = getattr(ens, name)
    fields = [f[0] for f in cls._fields_]
    size, offs = _c_layout(name, fields, tmp_path)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offs


def test_create_validates_before_touching_the_device():
    lib = ens.load()
    d = ens.ens_desc()
    d.model, d.solver, d.n, d.n_ensembles = 9, 0, 10, 1
    h = ctypes.c_void_p()
    assert lib.ens_create(ctypes.byref(d), ctypes.byref(h)) == ens.ENS_E_INVAL
    assert b"unknown model" in lib.ens_last_error(None)
    d.model = ens.ENS_KM
    d.solver = ens.ENS_RK4
    assert lib.ens_create(ctypes.byref(d), ctypes.byref(h)) == ens.ENS_E_UNSUPPORTED
    d.solver = ens.ENS_RKCK45
    d.n_ensembles = 2
    assert lib.ens_create(ctypes.byref(d), ctypes.byref(h)) == ens.ENS_E_INVAL
    assert lib.ens_create(None, ctypes.byref(h)) == ens.ENS_E_INVAL
    assert not h.value


def test_surrogate_create_validates_batch():
    from paper_2011_01740_amd import sur
    L = sur._lib()
    h = ctypes.c_void_p()
    assert L.sur_create(0, None, 100, ctypes.byref(h)) == ens.ENS_E_INVAL
    assert L.sur_create(0, None, 0, ctypes.byref(h)) == ens.ENS_E_INVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus N > 1 exits with status 2 and says so,
    before touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
