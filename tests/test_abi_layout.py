"""The ctypes structures of the Python binding have the layout of the C structs that
include/*.h declares: same size, same field names in the same order, same offsets
(compiled on the host with gcc; no device calls)."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# binding class -> C typedef
PAIRS = {
    "Grid": "kfbi_grid", "Info": "kfbi_info", "Out": "kfbi_out", "Bie": "kfbi_bie",
    "GmresOpts": "kfbi_gmres_opts", "GmresStats": "kfbi_gmres_stats",
    "ThetaLParams": "thetaL_params", "ThetaLStats": "thetaL_stats",
    "ThetaLState": "thetaL_state", "StefanAniso": "stefan_aniso",
    "StefanParams": "stefan_params", "StefanStats": "stefan_stats", "WsCfg": "kfbi_ws_cfg",
    "StokesParams": "stokes_params", "StokesInfo": "stokes_info",
}


def cname(field):
    """C field name of a binding field (a trailing underscore avoids a Python keyword)."""
    return field[:-1] if field.endswith("_") else field


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    import paper_2309_01068_amd.kfbi as kf
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "kfbi.h"',
             '#include "thetal.h"', '#include "stefan.h"', '#include "warmstart.h"',
             '#include "stokes.h"',
             'int main(void) {']
    for py, c in PAIRS.items():
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for name, _ in getattr(kf, py)._fields_:
            lines.append(f'  printf("{py} {name} %zu\\n", offsetof({c}, {cname(name)}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for ln in out.splitlines():
        cls, key, val = ln.split()
        table[(cls, key)] = int(val)
    return table


@pytest.mark.parametrize("py", sorted(PAIRS))
def test_binding_struct_matches_header(py, c_layout):
    import paper_2309_01068_amd.kfbi as kf
    cls = getattr(kf, py)
    assert ctypes.sizeof(cls) == c_layout[(py, "size")], py
    for name, _ in cls._fields_:
        assert getattr(cls, name).offset == c_layout[(py, name)], (py, name)
