"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the C ABI's argument checks, size queries and status text (the library built
with sanitizers on its host side, driven by tests/sanitize/abi_host.cpp), and
the oracle's direct sums and derivatives (oracle/direct.c driven by
tests/sanitize/oracle_host.c)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2301_10570_amd", "csrc")
SOURCES = ["api", "tree", "fgt", "p2p", "partner", "backward", "batch", "descent", "noalloc"]
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.slow


def _clean(out: str) -> bool:
    return "ERROR: AddressSanitizer" not in out and "runtime error" not in out


def test_oracle_under_sanitizers():
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_host")
        subprocess.run([gcc, "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        os.path.join(HERE, "oracle_host.c"), os.path.join(ROOT, "oracle", "direct.c"), "-lm",
                        "-o", exe], check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=120)
        out = r.stdout + r.stderr
        assert r.returncode == 0 and _clean(out), out[-3000:]
        assert "0 failures" in out


def test_abi_host_code_under_sanitizers():
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    inc = os.path.join(ROOT, "include")
    # sanitizers on the host side only; the device code is compiled but never run
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined", "-fno-omit-frame-pointer",
             "-Wno-unused-command-line-argument", "-I", inc]
    with tempfile.TemporaryDirectory() as tmp:
        procs = []
        for f in SOURCES:
            procs.append(subprocess.Popen([hipcc] + flags + ["-c", os.path.join(CSRC, f + ".hip"), "-o",
                                                              os.path.join(tmp, f + ".o")],
                                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        for p in procs:
            out, err = p.communicate()
            assert p.returncode == 0, err[-3000:]
        lib = os.path.join(tmp, "libmspfmm_san.so")
        subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined", "-o", lib] +
                       [os.path.join(tmp, f + ".o") for f in SOURCES], check=True, capture_output=True, text=True)
        exe = os.path.join(tmp, "abi_host")
        subprocess.run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-I", inc, os.path.join(HERE, "abi_host.cpp"), "-L", tmp, "-lmspfmm_san",
                        "-Wl,-rpath," + tmp, "-o", exe], check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
        out = r.stdout + r.stderr
        assert r.returncode == 0 and _clean(out), out[-3000:]
        assert "0 failures" in out
