"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
and its worker threads under ThreadSanitizer (no GPU): a host-instrumented build (device code unchanged) is loaded in a
child process with the ASan runtime preloaded, and the host-only entry points
run through their valid and invalid inputs -- ADAGRAD steps, tuning-cache
files with malformed and oversized lines, error strings, object lifetimes
with NULL handles, context creation without a device, the threaded host
eigensolver.  Any sanitizer report
aborts the child (UBSan does not recover)."""
import os
import subprocess
import sys
import textwrap

import pytest

from paper_1602_06693_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r'''
    import ctypes as C, os, sys, tempfile
    import numpy as np
    sys.path.insert(0, os.environ["PKM_ROOT"])
    from paper_1602_06693_amd import binding as pk
    from paper_1602_06693_amd import build
    lib = pk.load(build.HOSTSAN_LIB)
    assert lib.pkm_version().startswith(b"pkm")
    th, G = np.zeros(3), np.zeros(3)
    pk.pkm_adagrad_step(th, np.array([1.0, -2.0, 0.5]), G)
    assert np.allclose(G, [1.0, 4.0, 0.25]) and np.all(np.abs(th) > 0.99)
    P = C.POINTER(C.c_double)
    bad = np.array([np.nan, 0.0, 0.0])
    args = (th.ctypes.data_as(P), bad.ctypes.data_as(P), G.ctypes.data_as(P))
    assert lib.pkm_adagrad_step(3, *args, 1.0, 1e-8) == pk.PKM_ERR_INVALID
    assert lib.pkm_adagrad_step(0, *args, 1.0, 1e-8) == pk.PKM_ERR_INVALID
    assert lib.pkm_adagrad_step(3, None, None, None, 1.0, 1e-8) == pk.PKM_ERR_INVALID
    assert lib.pkm_adagrad_step(3, *args, -1.0, 1e-8) == pk.PKM_ERR_INVALID
    d = tempfile.mkdtemp()
    f = os.path.join(d, "tune.jsonl")
    with open(f, "w") as fh:
        fh.write('{"s4": 102, "kt": 1, "kr": 0, "work": 64, "u": 4, "fill": 1024}\n')
        fh.write('garbage\n{"s4": 999}\n{"s4": 3, "kt": 1, "kr": 1, "work": 64, "u": 1}\n')
        fh.write("x" * 200000 + "\n\n" + '{"s4": 3, "kt"' + "\n")
    a, r = C.c_int32(), C.c_int32()
    assert lib.pkm_tune_cache_load(f.encode(), C.byref(a), C.byref(r)) == pk.PKM_OK
    assert (a.value, r.value) == (2, 4), (a.value, r.value)
    assert lib.pkm_tune_cache_load(b"/nonexistent/tune.jsonl", C.byref(a), C.byref(r)) == pk.PKM_OK
    assert (a.value, r.value) == (0, 0)
    assert lib.pkm_tune_cache_load(None, C.byref(a), C.byref(r)) == pk.PKM_ERR_INVALID
    assert lib.pkm_last_error(None)
    out = C.c_void_p()
    assert lib.pkm_create(C.byref(out), 0, None) != pk.PKM_OK   # no device here
    assert lib.pkm_create(None, 0, None) != pk.PKM_OK
    n = C.c_int64()
    assert lib.pkm_mlp_nparams(None, C.byref(n)) == pk.PKM_ERR_INVALID
    assert lib.pkm_destroy(None) == pk.PKM_OK
    assert lib.pkm_precond_destroy(None) == pk.PKM_OK
    assert lib.pkm_mlp_destroy(None) == pk.PKM_OK
    # NULL context: rejected before anything touches the device
    assert lib.pkm_kernel_mvm(None, None, 1, pk.PKM_FP64, None, None) == pk.PKM_ERR_INVALID
    assert lib.pkm_solve(None, None, None, 1, None, None, None, None) == pk.PKM_ERR_INVALID
    assert lib.pkm_precond_apply(None, None, 1, None, None) == pk.PKM_ERR_INVALID
    assert lib.pkm_lml_grad(None, None, None, None, 1, None, None, None, None, None) \
        == pk.PKM_ERR_INVALID
    assert lib.pkm_kernel_mvm_noalloc(None, None, 1, pk.PKM_I8X, None, None) == pk.PKM_ERR_INVALID
    # host eigensolver: sizes around the 64-column blocks of its threaded
    # rotation pass, a degenerate spectrum, rejected inputs
    rng = np.random.default_rng(0)
    for m in (1, 2, 3, 63, 65, 130):
        A = rng.standard_normal((m, m)); A = A + A.T
        w, Z = pk.pkm_sym_eig(A)
        assert np.abs(Z @ np.diag(w) @ Z.T - A).max() < 1e-10 * max(1.0, np.abs(A).max())
    w, Z = pk.pkm_sym_eig(np.eye(70))
    assert np.allclose(w, 1.0) and np.allclose(Z.T @ Z, np.eye(70))
    os.environ["PKM_EIG_THREADS"] = "3"
    A = rng.standard_normal((200, 200)); A = A + A.T
    w, Z = pk.pkm_sym_eig(A)
    assert np.abs(Z @ np.diag(w) @ Z.T - A).max() < 1e-10 * np.abs(A).max()
    w0, Z0 = np.zeros(4), np.zeros(16)
    bad = np.full(16, np.nan)
    assert lib.pkm_sym_eig(4, bad.ctypes.data_as(P), w0.ctypes.data_as(P),
                           Z0.ctypes.data_as(P)) == pk.PKM_ERR_INVALID
    assert lib.pkm_sym_eig(0, None, None, None) == pk.PKM_ERR_INVALID
    print("host sanitizer run clean")
''')


def _stale():
    lib = build.HOSTSAN_LIB
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(s) > t for s in build.sources()) or \
        os.path.getmtime(os.path.join(ROOT, "include", "pkm.h")) > t


def test_host_entry_points_under_asan_and_ubsan():
    rt = build.hostsan_runtime()
    if rt is None or not os.path.exists(build.HIPCC):
        pytest.skip("hipcc or the clang ASan runtime is not installed")
    if _stale():
        build.build(host_sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, PKM_ROOT=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True,
                       timeout=300)
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-6000:]
    assert "host sanitizer run clean" in p.stdout
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr


def _tsan_stale():
    lib = build.HOSTTSAN_LIB
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(s) > t for s in build.sources()) or \
        os.path.getmtime(os.path.join(ROOT, "include", "pkm.h")) > t


def test_host_eigensolver_threads_under_tsan():
    """The eigensolver's worker threads (the only threads the library starts)
    under ThreadSanitizer: a host-instrumented libpkm driven by a small C++
    program built with -fsanitize=thread (tests/tsan_eig_main.cpp), four
    threads; any data-race report halts it."""
    clang = os.path.join(os.path.dirname(os.path.realpath(build.HIPCC)), "..", "llvm", "bin",
                         "clang++")
    if not os.path.exists(build.HIPCC) or not os.path.exists(clang):
        pytest.skip("hipcc or clang++ is not installed")
    if _tsan_stale():
        build.build(host_tsan=True)
    exe = os.path.join(build.HOSTTSAN_DIR, "tsan_eig")
    cc = subprocess.run([clang, "-fsanitize=thread", "-g", "-O1", "-std=c++17",
                         "-I", os.path.join(ROOT, "include"),
                         os.path.join(ROOT, "tests", "tsan_eig_main.cpp"), "-o", exe,
                         "-L", build.HOSTTSAN_DIR, "-lpkm_hosttsan",
                         "-Wl,-rpath," + build.HOSTTSAN_DIR], capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr[-3000:]
    env = dict(os.environ, PKM_EIG_THREADS="4", TSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-6000:]
    assert "tsan run clean" in p.stdout
    assert "ThreadSanitizer" not in p.stderr, p.stderr[-6000:]
