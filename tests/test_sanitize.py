"""AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer runs of the
host code, on the CPU.

* The oracle, with every allocation of its allocating entry points failing
  in turn (oracle/sanitize_check.c, oracle/alloc_hook.h).
* The host side of libdof (argument checks, layouts, error paths of the
  C ABI): the library rebuilt with host-only instrumentation and the ABI
  tests run against it in a child process.  Leak checking is off there:
  the Python interpreter itself keeps allocations alive at exit."""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_2210_06158_amd", "csrc")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_leak_and_ub_sanitizers(tmp_path):
    san = ["-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    obj = str(tmp_path / "oracle.o")
    rc, out = _run(["gcc", *san, "-include", os.path.join(ORACLE, "alloc_hook.h"), "-c",
                    os.path.join(ORACLE, "dof_oracle.c"), "-o", obj])
    assert rc == 0, out
    exe = str(tmp_path / "check")
    rc, out = _run(["gcc", *san, "-I", ORACLE, os.path.join(ORACLE, "sanitize_check.c"), obj, "-lm", "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    rc, out = _run([exe], env=env, timeout=600)
    assert rc == 0, out
    assert "sanitize check ok" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out


def _asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


@pytest.mark.skipif(shutil.which("hipcc") is None or _asan_runtime() is None, reason="hipcc / clang ASan runtime missing")
def test_host_library_under_address_and_ub_sanitizers(tmp_path):
    # device code is built as usual; each sanitizer flag applies to the host pass only
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
             "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    objs = []
    procs = []
    from paper_2210_06158_amd import build as pkg_build
    for src in pkg_build.SOURCES:
        o = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(o)
        procs.append(subprocess.Popen(["hipcc", *flags, *host_san, "-c", os.path.join(CSRC, src), "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, out
    lib = str(tmp_path / "libdof_san.so")
    rc, out = _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan", *host_san, *objs,
                    *pkg_build.LINK_FLAGS, "-o", lib])
    assert rc == 0, out
    code = (
        "import sys\n"
        "from paper_2210_06158_amd import dof\n"
        f"dof.LIB_PATH = {lib!r}\n"
        f"assert dof.lib()._name == {lib!r}\n"
        "import pytest\n"
        "sys.exit(pytest.main(['tests/test_abi.py', '-q', '-p', 'no:cacheprovider', '-m', 'not gpu']))\n")
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    rc, out = _run([sys.executable, "-c", code], cwd=ROOT, env=env, timeout=600)
    assert rc == 0, out
    assert "passed" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
