"""The host-side argument checks of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/test_abi_host.py (and the library's constant
and material queries) run in a child process against libhkp_asan.so -- the
host sources built with both sanitizers -- with the sanitizer runtime
preloaded; any report fails the run.  No GPU work is involved."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_LIB = os.path.join(ROOT, "paper_2607_08447_amd", "libhkp_asan.so")


def _runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _build_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_hkp_build", os.path.join(ROOT, "paper_2607_08447_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _stale(mod):
    """The sanitized library is older than a host source, a header or the normal
    library whose kernel objects it links."""
    t = os.path.getmtime(ASAN_LIB)
    deps = [os.path.join(mod.SRC, f) for f in mod.ASAN_SOURCES]
    deps += glob.glob(os.path.join(mod.SRC, "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    deps.append(mod.LIB)
    return any(os.path.exists(d) and os.path.getmtime(d) > t for d in deps)


def test_host_abi_checks_under_sanitizers():
    rt = _runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime in this image")
    if not os.path.exists(ASAN_LIB):
        pytest.skip("libhkp_asan.so not built (build() of __graft_entry__ builds it)")
    mod = _build_module()
    if _stale(mod):   # rebuilt from the current sources rather than testing an old one
        mod.build_asan()
    env = dict(os.environ, LD_PRELOAD=rt, HKP_LIB=ASAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
           "tests/test_abi_host.py",
           "tests/test_oracle_constants.py::test_library_unit_constants",
           "tests/test_oracle_constants.py::test_library_default_material_is_table_one"]
    probe = subprocess.run(
        [sys.executable, "-c", "import ctypes as C; from paper_2607_08447_amd import _lib; "
         "print(_lib.LIB_PATH); print(len([n for n in ('__asan_init', '__ubsan_handle_add_overflow')"
         " if hasattr(C.CDLL(_lib.LIB_PATH), n)]))"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-3000:]
    path, nsym = probe.stdout.split()[-2:]
    assert path == ASAN_LIB and int(nsym) >= 1, probe.stdout   # the sanitized build is in use
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, out
    assert " passed" in r.stdout, out
