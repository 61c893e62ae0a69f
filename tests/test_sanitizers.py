"""Host-side AddressSanitizer + UndefinedBehaviorSanitizer runs (CPU only).

The oracle and the host part of the library (node classes, link and fill lists, work
items, workspace layout, parameter and grid checks) are rebuilt with the sanitizers in
a temporary directory and exercised in a child process with the sanitizer runtime
preloaded; any report aborts the child and fails the test.  Device code is built as
usual: only host code is instrumented.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SAN_ENV = dict(ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="1")


def _runtime(cmd):
    out = subprocess.run(cmd, capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def _child(code, env_extra, tmp):
    env = dict(os.environ, **SAN_ENV, **env_extra, PYTHONPATH=ROOT)
    script = os.path.join(tmp, "child.py")
    with open(script, "w") as f:
        f.write(code)
    r = subprocess.run([sys.executable, script], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "SANITIZER_CHILD_OK" in r.stdout, \
        (r.returncode, r.stdout[-2000:], r.stderr[-4000:])


ORACLE_CHILD = r'''
assert any("asan" in line for line in open("/proc/self/maps")), "sanitizer runtime not loaded"
import numpy as np
import oracle, synth
oracle.set_threads(1)
mask = np.zeros((20, 36), np.uint8); mask[6:9, 5:8] = 1
cases = [
    synth.random_periodic(36, 20, seed=1, ymode="wall", solid=mask, circles=[(24.0, 10.0, 4.3)]),
    synth.random_periodic(40, 17, seed=2, xmode="open", ymode="wall", circles=[(15.0, 8.0, 3.6)]),
    synth.random_periodic(24, 24, seed=3).with_(model="fene_p", model_param=30.0),
    synth.random_periodic(30, 18, seed=4, xmode="wall", ymode="wall").with_(model="giesekus", model_param=0.3),
]
for pr in cases:
    o = oracle.OracleSim(pr)
    o.step(12)
    r = o.read()
    assert all(np.isfinite(v).all() for v in r.values()), pr.name
    o.history()
    o.drag(-1)
    if pr.circles:
        o.drag(0)
    del o
d = oracle.OracleSim(synth.random_periodic(16, 16, seed=5), dual=True)
d.step(3)
print("SANITIZER_CHILD_OK")
'''

LIB_CHILD = r'''
assert any("asan" in line for line in open("/proc/self/maps")), "sanitizer runtime not loaded"
import ctypes as C
import numpy as np
from paper_2508_16997_amd import _lib as L
lib = L.load()
def grid(nx, ny, xmode, ymode, prec, mask=None, circles=()):
    g = L.VlbGrid()
    g.nx, g.ny, g.xmode, g.ymode, g.precision = nx, ny, xmode, ymode, prec
    keep = []
    if mask is not None:
        m = np.ascontiguousarray(mask, np.uint8); keep.append(m); g.solid_mask = m.ctypes.data
    if circles:
        c = np.ascontiguousarray(np.array(circles, np.float64).reshape(-1)); keep.append(c)
        g.circles = c.ctypes.data_as(C.POINTER(C.c_double)); g.ncircles = len(circles)
    return g, keep
mask = np.zeros((40, 70), np.uint8); mask[10:15, 20:24] = 1; mask[0, :] = 1
specs = [
    (70, 40, L.VLB_PERIODIC, L.VLB_WALL, 0, mask, [(45.0, 20.0, 7.3)]),
    (130, 33, L.VLB_OPEN, L.VLB_WALL, 0, None, [(50.0, 16.0, 7.2), (90.0, 10.0, 3.1)]),
    (64, 64, L.VLB_PERIODIC, L.VLB_PERIODIC, 1, None, [(0.5, 0.5, 6.0)]),
    (33, 17, L.VLB_WALL, L.VLB_WALL, 1, None, []),
    (1, 1, L.VLB_WALL, L.VLB_WALL, 0, None, []),
    (2, 2, L.VLB_PERIODIC, L.VLB_PERIODIC, 0, None, []),
]
for nx, ny, xm, ym, prec, m, circ in specs:
    g, keep = grid(nx, ny, xm, ym, prec, m, circ)
    h = C.c_void_p()
    assert lib.vlb_create(C.byref(g), C.byref(h)) == L.VLB_OK, (nx, ny)
    cls = np.zeros((ny, nx), np.uint8); n = C.c_int()
    assert lib.vlb_geometry(h, cls.ctypes.data, None, None, None, 0, C.byref(n)) == 0
    cnt = n.value
    node = np.zeros(max(cnt, 1), np.int32); d = np.zeros(max(cnt, 1), np.int8); q = np.zeros(max(cnt, 1))
    assert lib.vlb_geometry(h, cls.ctypes.data, node.ctypes.data, d.ctypes.data, q.ctypes.data, cnt, C.byref(n)) == 0
    ws = C.c_size_t()
    assert lib.vlb_workspace_bytes(h, C.byref(ws)) == 0 and ws.value > 0
    for ty in (1, 2, 4, 8):
        assert lib.vlb_set_tile(h, ty) == 0
    p = L.VlbParams(0.1, 0.1, 10.0, 0.01, 0.25, 1e-6, 0.0, 0.0, 0, 4, 50.0)
    assert lib.vlb_set_params(h, C.byref(p)) == 0
    p = L.VlbParams(0.1, 0.1, -1.0, 0.01, 0.25, 1e-6, 0.0, 0.0, 0, 0, 0.0)
    assert lib.vlb_set_params(h, C.byref(p)) == L.VLB_E_INVALID_ARG
    lib.vlb_destroy(h)
bad, keep = grid(0, 5, 0, 0, 0)
h = C.c_void_p()
assert lib.vlb_create(C.byref(bad), C.byref(h)) == L.VLB_E_INVALID_ARG
out = L.VlbParams(); uc = C.c_double()
assert lib.vlb_params_from_groups(1.0, 5.0, 0.5, 1e5, 0.01, 81.5, 0.25, 1e-6, C.byref(out), C.byref(uc)) == 0
print("SANITIZER_CHILD_OK")
'''


@pytest.fixture(scope="module")
def tmpdir_mod(tmp_path_factory):
    return str(tmp_path_factory.mktemp("san"))


def test_oracle_under_asan_ubsan(tmpdir_mod):
    asan = _runtime(["g++", "-print-file-name=libasan.so"])
    ubsan = _runtime(["g++", "-print-file-name=libubsan.so"])
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    so = os.path.join(tmpdir_mod, "liboracle_san.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", so,
                    os.path.join(ROOT, "oracle", "vlb_oracle.cpp")], check=True)
    _child(ORACLE_CHILD, dict(ORACLE_LIBRARY=so, LD_PRELOAD=f"{asan}:{ubsan}"), tmpdir_mod)


def test_library_host_code_under_asan_ubsan(tmpdir_mod):
    from paper_2508_16997_amd import build as B

    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    clang_dir = os.path.join(os.path.dirname(os.path.dirname(B.HIPCC)), "llvm", "bin", "clang")
    asan = _runtime([clang_dir, "-print-file-name=libclang_rt.asan-x86_64.so"])
    if not asan:
        pytest.skip("clang ASan runtime not installed")
    objs, cmds = [], []
    for src in B.SOURCES:
        obj = os.path.join(tmpdir_mod, src.replace(".", "_") + ".o")
        extra = []
        if src == "vlb_api.cpp":  # the host-only translation unit
            extra = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                     "-Xarch_host", "-fno-sanitize-recover=undefined",
                     "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
        cmds.append([B.HIPCC, *B.COMMON, *B.PER_FILE.get(src, []), *extra, "-c",
                     os.path.join(B.CSRC, src), "-o", obj, "-w"])
        objs.append(obj)
    B.compile_all(cmds)
    so = os.path.join(tmpdir_mod, "libvlb_san.so")
    subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-o", so, *objs,
                    f"-L{B.ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{B.ROCM_LIB}"],
                   check=True)
    _child(LIB_CHILD, dict(VLB_LIBRARY=so, LD_PRELOAD=asan), tmpdir_mod)
