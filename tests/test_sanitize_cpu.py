"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer.

The host sources (plans and argument checks, template responses, statistics,
sifting) are compiled with g++ and the sanitizers, linked with the unsanitized
HIP objects of the normal build, and the CPU tests of the C ABI and of the
sifting run against that library in a child process (the sanitizer runtime
must be the first library of the process). Any report aborts the child.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1912_12807_amd", "csrc")
HOST_SOURCES = ("fdas_api.cpp", "response.cpp", "stats.cpp", "sift.cpp")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    from paper_1912_12807_amd import build
    out = tmp_path_factory.mktemp("san")
    hip_obj = os.path.join(str(out), "hip")
    # the HIP objects of the normal build (device code is not instrumented)
    build.build(out=os.path.join(str(out), "libfdas_plain.so"), obj_dir=hip_obj)
    objs = []
    for src in HOST_SOURCES:
        o = os.path.join(str(out), src + ".o")
        _run(["g++", *SAN, "-g", "-O1", "-fPIC", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
              "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    hip = sorted(os.path.join(hip_obj, f) for f in os.listdir(hip_obj) if f.endswith(".hip.o"))
    lib = os.path.join(str(out), "libfdas_san.so")
    _run(["g++", "-shared", *SAN, "-o", lib, *objs, *hip, "-L/opt/rocm/lib", "-lamdhip64", "-lpthread",
          "-Wl,-rpath,/opt/rocm/lib"])
    return lib


def test_host_code_under_address_and_undefined_sanitizers(sanitized_lib):
    pre = [subprocess.run(["g++", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
           for n in ("libasan.so", "libubsan.so")]
    assert all(os.path.isabs(p) and os.path.exists(p) for p in pre), pre
    env = dict(os.environ, FDAS_LIB_PATH=sanitized_lib, LD_PRELOAD=":".join(pre),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    probe = ("import ctypes, paper_1912_12807_amd as F; lib = F.load(); "
             "assert lib._name == __import__('os').environ['FDAS_LIB_PATH']; "
             "assert hasattr(ctypes.CDLL(None), '__asan_init'); print('sanitized library loaded')")
    r = _run([sys.executable, "-c", probe], env=env, cwd=ROOT)
    assert "sanitized library loaded" in r.stdout
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
              "tests/test_abi_cpu.py", "tests/test_sift_cpu.py"], env=env, cwd=ROOT, timeout=900)
    assert " passed" in r.stdout and "failed" not in r.stdout, r.stdout[-2000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
