"""Host AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only).

* The C part of the oracle, built with both sanitizers, runs every exported
  routine on small exact problems (tests/asan/oracle_check.c).
* The host code that checks the C ABI's arguments (runtime.hip and
  batched.hip, built with the sanitizers on the host side only) is linked
  with the library's other objects and driven by tests/asan/abi_check.c:
  invalid arguments must give the documented statuses, and valid calls must
  fail cleanly without a GPU.

Skipped on a machine with a GPU: abi_check.c's valid calls use dummy
pointers and would reach the device there.
"""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
CSRC = os.path.join(ROOT, "paper_2303_04353_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")

pytestmark = pytest.mark.skipif(os.path.exists("/dev/kfd"),
                                reason="host sanitizer runs are for machines without a GPU")

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def _clean(r):
    text = r.stdout + r.stderr
    return r.returncode == 0 and "AddressSanitizer" not in text and "runtime error" not in text


def test_oracle_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.run([CLANG, "-O1", "-std=c99", "-ffp-contract=off", "-fopenmp", *SAN,
                    os.path.join(ROOT, "oracle", "ddgemm_ref.c"), os.path.join(ROOT, "tests", "asan", "oracle_check.c"),
                    "-o", exe, "-lm", "-L/opt/rocm/llvm/lib", "-Wl,-rpath,/opt/rocm/llvm/lib"], check=True)
    r = subprocess.run([exe], env=_env(), capture_output=True, text=True, timeout=300)
    assert _clean(r), r.stdout + r.stderr
    assert "oracle checks passed" in r.stdout


def test_abi_argument_checks_under_host_sanitizers(tmp_path):
    from paper_2303_04353_amd import build as hb
    flags = [f for f in hb.HIPCC_FLAGS if f != "-shared"]
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        host_san += ["-Xarch_host", f]
    objs = []
    for src in ("runtime.hip", "batched.hip"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run(["hipcc", *flags, *host_san, "-c", os.path.join(CSRC, src), "-o", o], check=True,
                       capture_output=True)
        objs.append(o)
    others = [o for o in sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
              if os.path.basename(o) not in ("runtime.hip.o", "batched.hip.o")]
    if len(others) + 2 != len(hb.sources()):
        hb.build()   # the other objects come from the ordinary build
        others = [o for o in sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
                  if os.path.basename(o) not in ("runtime.hip.o", "batched.hip.o")]
    lib = str(tmp_path / "libddgemm_san.so")
    subprocess.run(["hipcc", *hb.HIPCC_FLAGS, *objs, *others, "-o", lib, "-lrocblas"], check=True, capture_output=True)
    exe = str(tmp_path / "abi_check")
    subprocess.run([CLANG, "-O1", "-std=c99", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(ROOT, "tests", "asan", "abi_check.c"), lib, "-o", exe,
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath," + str(tmp_path)],
                   check=True)
    r = subprocess.run([exe], env=_env(), capture_output=True, text=True, timeout=300)
    assert _clean(r), r.stdout + r.stderr
    assert "abi checks passed" in r.stdout
