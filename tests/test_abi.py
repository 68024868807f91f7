"""CPU checks of the C boundary: the library loads, exports exactly the
symbols include/nbody.h declares, the ctypes structures match the C layout,
and argument validation that needs no device runs without a GPU."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")
LIB = os.path.join(ROOT, "paper_1803_01190_amd", "libnbody.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"NBODY_API\s+[\w\s\*]+?\b(nbody_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        sys.path.insert(0, ROOT)
        from paper_1803_01190_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for want in ("nbody_accel", "nbody_step_kdk", "nbody_step_o4", "nbody_diag", "nbody_accel_batched",
                 "nbody_step_kdk_batched", "nbody_step_o4_batched", "nbody_diag_batched",
                 "nbody_ctx_create", "nbody_autotune"):
        assert want in names


def test_exports_match_header(lib):
    names = declared()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == names


def test_struct_layout_matches_ctypes(tmp_path):
    # the binding loads the library at import; that works without a GPU
    from paper_1803_01190_amd import nbody as nbm
    src = tmp_path / "l.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "nbody.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(nbody_sys), sizeof(nbody_params), sizeof(nbody_diag_t),
         sizeof(nbody_plan), sizeof(nbody_profile_t));
  printf("%zu %zu %zu %zu\n", offsetof(nbody_sys, phi), offsetof(nbody_params, prec),
         offsetof(nbody_params, halo_rc), offsetof(nbody_profile_t, update_ms));
  return 0; }
''')
    exe = tmp_path / "l"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    a, b = subprocess.check_output([str(exe)], text=True).split("\n")[:2]
    sizes = [int(v) for v in a.split()]
    offs = [int(v) for v in b.split()]
    assert sizes == [ctypes.sizeof(nbm.c_sys), ctypes.sizeof(nbm.c_params), 14 * 8,
                     ctypes.sizeof(nbm.c_plan), ctypes.sizeof(nbm.c_profile)]
    assert offs == [nbm.c_sys.phi.offset, nbm.c_params.prec.offset, nbm.c_params.halo_rc.offset,
                    nbm.c_profile.update_ms.offset]


def test_null_context_is_rejected_without_a_device(lib):
    # every entry point validates before touching HIP; a NULL context is EINVAL
    NB_EINVAL = -1
    for name in ("nbody_accel", "nbody_step_kdk", "nbody_step_o4", "nbody_diag", "nbody_accel_batched",
                 "nbody_profile_enable"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
    lib.nbody_accel.argtypes = [ctypes.c_void_p] * 4
    assert lib.nbody_accel(None, None, None, None) == NB_EINVAL
    lib.nbody_step_kdk.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_double, ctypes.c_int64, ctypes.c_void_p]
    assert lib.nbody_step_kdk(None, None, None, 1e-3, 1, None) == NB_EINVAL
    lib.nbody_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.nbody_profile_enable(None, 1) == NB_EINVAL
    lib.nbody_last_error.restype = ctypes.c_char_p
    lib.nbody_last_error.argtypes = [ctypes.c_void_p]
    assert lib.nbody_last_error(None) == b"no context"
    lib.nbody_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.nbody_version()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_plan_class_constants_match_header():
    import re
    from paper_1803_01190_amd import nbody as nb
    text = open(HEADER).read()
    consts = {m.group(1): int(m.group(2), 16) for m in re.finditer(r"#define (NB_PLAN_\w+) (0x[0-9a-fA-F]+)", text)}
    assert consts == {"NB_PLAN_ACCEL": nb.NB_PLAN_ACCEL, "NB_PLAN_POTENTIAL": nb.NB_PLAN_POTENTIAL,
                      "NB_PLAN_JERK": nb.NB_PLAN_JERK, "NB_PLAN_BATCH": nb.NB_PLAN_BATCH}
    assert nb.plan_code("fp64/potential") == nb.NB_FP64 | nb.NB_PLAN_POTENTIAL
    assert nb.plan_code("mixed") == nb.NB_MIXED
