"""CPU-side checks of the C ABI: the built library loads, exports every
function ``include/bop.h`` declares, and the binding's struct layouts match
the header (compiled with the host compiler).  No kernel is launched."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

import paper_1803_07491_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bop.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|size_t)\s+(bop_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    lib = P.load()
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("no host compiler / HIP headers")
    prog = tmp_path / "lay.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "bop.h"
int main(void){
 printf("%zu %zu %zu %zu %zu %zu\n", sizeof(bop_model), offsetof(bop_model,onsite),
        offsetof(bop_model,form), offsetof(bop_model,beta0), offsetof(bop_model,r0), offsetof(bop_model,q));
 printf("%zu %zu %zu\n", sizeof(bop_plan), offsetof(bop_plan,rows_k), offsetof(bop_plan,ws_bytes));
 printf("%zu %zu %zu %zu %zu\n", sizeof(bop_system), offsetof(bop_system,n_pairs), offsetof(bop_system,plan),
        offsetof(bop_system,n_elec), offsetof(bop_system,U_total));
 printf("%zu\n", sizeof(bop_tuning));
 return 0;}
''')
    exe = tmp_path / "lay"
    subprocess.check_call([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(prog), "-o", str(exe)])
    got = [list(map(int, l.split())) for l in subprocess.check_output([str(exe)]).decode().splitlines()]
    M, S = P.Model, P.System
    assert got[0] == [C.sizeof(M), M.onsite.offset, M.form.offset, M.beta0.offset, M.r0.offset, M.q.offset]
    assert got[1] == [C.sizeof(P.Plan), P.Plan.rows_k.offset, P.Plan.ws_bytes.offset]
    assert got[2] == [C.sizeof(S), S.n_pairs.offset, S.plan.offset, S.n_elec.offset, S.U_total.offset]
    assert got[3] == [C.sizeof(P.Tuning)]
