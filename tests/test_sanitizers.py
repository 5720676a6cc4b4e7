"""CPU: the oracle and the host paths of the library built with AddressSanitizer
and UndefinedBehaviorSanitizer (host code only), with CPU tests run against
those builds in child processes.  Any sanitizer report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0704_3573_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-O1", "-g"]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def run_tests(tests, extra_env, tmp):
    env = dict(os.environ, **ENV, **extra_env)
    log = os.path.join(tmp, "log.txt")
    with open(log, "w") as f:
        rc = subprocess.call([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                              "-m", "not gpu"] + tests, cwd=ROOT, env=env, stdout=f,
                             stderr=subprocess.STDOUT)
    text = open(log).read()
    assert rc == 0 and "Sanitizer" not in text and "runtime error" not in text, text[-4000:]


def test_oracle_under_asan_and_ubsan(tmp_path):
    so = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-std=c11", "-fPIC", "-shared", "-pthread"] + SAN +
                          ["-o", str(so), os.path.join(ROOT, "oracle", "sg_oracle.c"), "-lm"])
    runtime = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.isfile(runtime), runtime
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    run_tests(tests, {"SG_ORACLE_LIBRARY": str(so), "LD_PRELOAD": runtime}, str(tmp_path))


def test_library_host_paths_under_asan_and_ubsan(tmp_path):
    kernels = os.path.join(CSRC, "sg_kernels.o")
    if not os.path.exists(kernels):
        pytest.skip("the library has not been built (sg_kernels.o missing)")
    clang = "/opt/rocm/llvm/bin/clang++"
    objs = []
    for src in ("sg_host.cpp", "sg_seed.cpp"):
        obj = tmp_path / (src + ".o")
        subprocess.check_call([clang, "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}",
                               f"-I{CSRC}", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + SAN +
                              ["-c", os.path.join(CSRC, src), "-o", str(obj)])
        objs.append(str(obj))
    so = tmp_path / "libsg_san.so"
    subprocess.check_call([clang, "-shared", "-fsanitize=address,undefined", "-o", str(so), kernels] +
                          objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    runtime = subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                      text=True).strip()
    assert os.path.isfile(runtime), runtime
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_lib_host.py", "test_lib_tables.py", "test_serving_logic.py")]
    run_tests(tests, {"SG_LIBRARY": str(so), "LD_PRELOAD": runtime}, str(tmp_path))
