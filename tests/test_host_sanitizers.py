"""The host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer: api.hip is
compiled again with both sanitizers on its host pass only (its device code and the other
kernel objects are the regular build's), linked into a second copy of the library, and the CPU
tests of the ABI (tests/test_abi.py: argument checks of every entry point, rejected problems,
error messages, the allocation-free operator's host checks) run against it in a subprocess with
the sanitizer runtime preloaded.  Any sanitizer report fails the test.  Needs the regular build
(``__graft_entry__.build()``) for the kernel objects."""

import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


def _runtime():
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return rts[0] if rts else None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    objs = [os.path.join(ROOT, "_build", n + ".o")
            for n in ("k_cg", "k_em", "k_fourier", "k_mixed", "k_operator", "k_slq")]
    if not os.path.exists(HIPCC) or _runtime() is None:
        pytest.skip("hipcc or the sanitizer runtime is not available")
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("the regular build's objects are missing (run __graft_entry__.build())")
    d = tmp_path_factory.mktemp("san")
    obj, lib = str(d / "api_san.o"), str(d / "libcmtcs_san.so")
    cflags = ["--offload-arch=gfx950", "-O1", "-fPIC", "-std=c++17", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")]
    src = os.path.join(ROOT, "paper_2310_00420_amd", "csrc", "api.hip")
    for cmd in ([HIPCC] + cflags + SAN + ["-c", src, "-o", obj],
                [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan"] + SAN[:4]
                + ["-o", lib, obj] + objs):
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert p.returncode == 0, p.stdout
    return lib


def test_abi_host_paths_under_sanitizers(sanitized_lib):
    env = dict(os.environ, CMTCS_LIB=sanitized_lib, LD_PRELOAD=_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi.py")], cwd=ROOT, env=env,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    print(p.stdout[-3000:])
    assert p.returncode == 0
    assert "AddressSanitizer" not in p.stdout and "runtime error" not in p.stdout
    assert " passed" in p.stdout
