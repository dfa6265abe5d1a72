"""CPU sanitizer pass: the oracle's C code and the host side of the HIP
library run under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

  * the oracle is rebuilt with gcc -fsanitize=address,undefined and the
    oracle pin tests run against it in a child process with the gcc runtimes
    preloaded;
  * the library is rebuilt with the sanitizers on its host code only (each
    flag behind -Xarch_host; the device code is unchanged) and the ABI tests
    (descriptor checks, workspace layout, piece tables of batches with empty
    volumes, every validation path) run against it with clang's runtime
    preloaded.
Any report aborts the child (no recovery), which fails the test."""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _gcc_runtime(name):
    path = subprocess.run(["gcc", "-print-file-name=%s" % name], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run_child(args, env, timeout=900):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + args,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
    return r


def test_oracle_under_asan_ubsan():
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    env = dict(os.environ, VG_ORACLE_SANITIZE="1", LD_PRELOAD=asan + ":" + ubsan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    r = _run_child(tests, env)
    assert " passed" in r.stdout


def test_library_host_code_under_asan_ubsan():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang sanitizer runtime not installed")
    sys.path.insert(0, ROOT)
    from paper_2406_04177_amd.build import build
    with tempfile.TemporaryDirectory() as d:
        lib = build(out=os.path.join(d, "libvgsim.so"), extra_flags=HOST_SAN)
        env = dict(os.environ, VGSIM_LIB=lib, LD_PRELOAD=rt[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = _run_child([os.path.join(ROOT, "tests", "test_abi.py")], env)
        assert " passed" in r.stdout
