"""Host-side checks of the C ABI that need no GPU."""
import ctypes
import os
import re

import pytest

import paper_2105_14782_amd as exo
from paper_2105_14782_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_symbols():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(exo_\w+)\s*\(", txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.load_library()
    names = declared_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_string():
    lib = L.load_library()
    assert b"gfx950" in lib.exo_version()
    assert lib.exo_last_error() is not None


def test_argument_validation_without_device_work():
    lib = L.load_library()
    # negative sizes and NULL pointers are rejected before any launch
    assert lib.exo_hjert_f32(-1, None, None, None, None, None) == L.EXO_EINVAL
    assert lib.exo_hjert_f32(10, None, None, None, None, None) == L.EXO_EINVAL
    assert lib.exo_hjert_f64(10, None, None, None, None) == L.EXO_EINVAL
    assert lib.exo_trans2e3(5, None, None, None, None) == L.EXO_EINVAL
    assert lib.exo_hjert_f32(0, None, None, None, None, None) == L.EXO_OK
    assert lib.exo_create(0, None) == L.EXO_EINVAL
    assert lib.exo_set_grid(None, 5, None) == L.EXO_EINVAL
    assert lib.exo_emission_flux(None, None, None, 0, None, None) == L.EXO_EINVAL
    assert lib.exo_flux_vjp(None, None, None, 0, None, None, None, None, None) == L.EXO_EINVAL
    assert b"NULL" in lib.exo_last_error()


def test_create_reports_missing_device_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("device present")
    except Exception:
        pass
    lib = L.load_library()
    h = ctypes.c_void_p()
    rc = lib.exo_create(0, ctypes.byref(h))
    assert rc in (L.EXO_EINVAL, L.EXO_EDEVICE)
    assert not h.value
    assert len(lib.exo_last_error()) > 0


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2105_14782_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("oracle is the oracle", ""), f


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a struct of include/exohip.h, from gcc."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    src = tmp_path / "layout.c"
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "exohip_serve.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


def _server_counters():
    from paper_2105_14782_amd import serve
    return serve.ExoServerCounters


@pytest.mark.parametrize("struct,ctype", [("exo_atmos", L.ExoAtmos), ("exo_response", L.ExoResponse),
                                          ("exo_server_counters", None)])
def test_ctypes_structs_match_the_header(tmp_path, struct, ctype):
    """The binding's ctypes mirrors have the C layout field by field."""
    ctype = ctype or _server_counters()
    names = [f[0] for f in ctype._fields_]
    size, offsets = _c_layout(tmp_path, struct, names)
    assert ctypes.sizeof(ctype) == size
    for name, off in zip(names, offsets):
        assert getattr(ctype, name).offset == off, name


def test_bench_refuses_more_than_one_gpu():
    """One GPU only: --gpus 2 exits with status 2 and a JSON message, before
    touching a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
