"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

host.cpp (mesh setup, face numbering and orientation, size classes, sampling
points, workspace layouts, variant validation, error paths) is compiled with
both sanitizers for the host compiler only, linked with the library's device
objects, and driven through the host-only calls of the C ABI in a child
process with the ASan runtime preloaded.  An out-of-bounds access, a
use-after-free or undefined behaviour (signed overflow, misaligned or null
access, bad shift) aborts the child.  No GPU is used.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2302_10917_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

# host-only instrumentation: every sanitizer flag is scoped to the host pass
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]

CHILD = r"""
import ctypes
import sys
import numpy as np
from paper_2302_10917_amd import inputs, mhdg
lib = mhdg.load_library(sys.argv[1])
proc = ctypes.CDLL(None)
assert hasattr(proc, "__asan_init") and hasattr(proc, "__ubsan_handle_add_overflow_abort")
for n, r, p, jit in ((2, 1, 2, 0.0), (3, "mixed", 3, 0.12), (4, 0, 1, 0.05), (5, 3, 3, 0.1),
                     (2, 4, 3, 0.0)):
    xy, tri = inputs.structured_mesh(n, jitter=jit, seed=5)
    lv = inputs.random_levels(len(tri), (0, 1, 2, 3), seed=1) if r == "mixed" else r
    m = mhdg.MacroMesh(xy, tri, lv, p)
    for prec in (mhdg.MHDG_FP64, mhdg.MHDG_FP32, mhdg.MHDG_BF16, mhdg.MHDG_QELIM):
        s = m.query(prec)
        assert s.factor_ws_bytes > 0 and s.n_macro == len(tri)
    node, bnd = m.sample_points()
    assert np.all(np.isfinite(node)) and np.all(np.isfinite(bnd))
    m.set_instances(3)
    m.sample_points()
    assert lib.mhdg_boundary_ws_bytes(m.h) > 0 and lib.mhdg_trace_matrix_ws_bytes(m.h) > 0
    assert lib.mhdg_condense_boundary(m.h, None, 0, None) == 7   # before factor_local
    m.set_instances(1)
    N = m.sizes.max_local
    for lu, sv in ((0, 0), (5, 1), (9, 1), (1, 9)):
        try:
            m.set_kernel_variant(N, lu, sv)
        except mhdg.MhdgError:
            pass
    del m
xy, tri = inputs.structured_mesh(2)
bad = tri.copy()
bad[0, 1] = bad[0, 0]
for t in (tri[:, ::-1], bad):
    try:
        mhdg.MacroMesh(xy, t, 1, 2)
        raise SystemExit("bad mesh accepted")
    except mhdg.MhdgError:
        pass
print("host API ok")
"""


def _objects():
    from paper_2302_10917_amd import build as B
    objs = [os.path.join(B.OBJ, os.path.splitext(s)[0] + ".o") for s in B.SOURCES
            if s != "host.cpp"]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    return B, objs


def test_host_code_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not available")
    B, objs = _objects()
    host_obj = str(tmp_path / "host_san.o")
    lib = str(tmp_path / "libmhdg_san.so")
    cc = [HIPCC, *B.HIPCC_FLAGS, *SAN, "-x", "hip", "-c", os.path.join(B.CSRC, "host.cpp"),
          "-o", host_obj]
    res = subprocess.run(cc, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    ln = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, "-shared-libsan", host_obj,
          *objs, "-o", lib]
    res = subprocess.run(ln, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    asan_rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                             capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=asan_rt, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-c", CHILD, lib], capture_output=True, text=True,
                         env=env, cwd=ROOT, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "host API ok" in res.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
