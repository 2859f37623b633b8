"""The C-ABI library loads, exports every entry point its header declares, and
the binary layouts of the header structs match the Python ctypes mirrors
(CPU only: no compute calls)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1811_11992_amd import inputs as I
from paper_1811_11992_amd import isc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "isc.h")


def declared():
    src = open(HDR).read()
    return sorted(set(re.findall(r"\b(isc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    if not os.path.exists(isc.LIB_PATH):
        pytest.skip("libisc.so not built")
    L = ctypes.CDLL(isc.LIB_PATH)
    names = declared()
    assert "isc_assemble" in names and "isc_newton_step" in names and "isc_adjoint" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "isc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(isc_fluid), sizeof(isc_grid), sizeof(isc_well),
         sizeof(isc_solve_opts), sizeof(isc_solve_info), sizeof(isc_newton_opts), sizeof(isc_newton_info));
  printf("%zu %zu %zu %zu\n", offsetof(isc_fluid, stoich), offsetof(isc_fluid, eps),
         offsetof(isc_fluid, krw), offsetof(isc_well, z_inj));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.dirname(HDR), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(x) for x in out]
    py = [ctypes.sizeof(I.Fluid), ctypes.sizeof(I.Grid), ctypes.sizeof(I.Well), ctypes.sizeof(isc.SolveOpts),
          ctypes.sizeof(isc.SolveInfo), ctypes.sizeof(isc.NewtonOpts), ctypes.sizeof(isc.NewtonInfo),
          I.Fluid.stoich.offset, I.Fluid.eps.offset, I.Fluid.krw.offset, I.Well.z_inj.offset]
    assert sizes == py
