"""The oracle's C code and the library's host code (argument validation,
planning, the tuning cache) built with AddressSanitizer and
UndefinedBehaviorSanitizer, and their CPU tests run against those builds in
a child process with the sanitizer runtime preloaded: any invalid access or
undefined operation stops the child with an error."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run_child(args, env_extra, timeout=600):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def _check_child(r):
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert r.returncode == 0, text[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not installed")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-std=gnu11", "-Wall", "-fPIC", "-shared", "-pthread",
                    "-o", lib, os.path.join(ROOT, "oracle", "oracle_cgemm.c")], check=True)
    env = {"LD_PRELOAD": asan, "ORACLE_LIBRARY": lib}
    probe = _run_child(["-c", "import ctypes, oracle; L = oracle.lib(); print(L._name); "
                              "ctypes.CDLL(None).__asan_init"], env, timeout=120)
    _check_child(probe)
    assert probe.stdout.strip() == lib
    r = _run_child(["-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                    "tests/test_oracle.py", "tests/test_oracle_acc.py"], env)
    _check_child(r)
    assert " passed" in r.stdout


def test_host_code_under_sanitizers(tmp_path):
    """The library's host sources rebuilt with the sanitizers (device code
    unchanged) and linked with the device objects of the regular build; the
    ABI tests, which drive argument validation, the planner's error paths and
    the tuning cache without a GPU, run against it."""
    from paper_2307_06072_amd import build as b
    hipcc = b.HIPCC
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not installed")
    dev_objs = [os.path.join(b.BUILD, s + ".o") for s in b.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in dev_objs):
        pytest.skip("the library's device objects are not built (run __graft_entry__.build())")
    rt = subprocess.run([os.path.join(os.path.dirname(hipcc), "..", "llvm", "bin", "clang"),
                         "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    asan = os.path.realpath(rt.stdout.strip()) if rt.returncode == 0 else ""
    if not os.path.isabs(asan) or not os.path.exists(asan):
        found = [os.path.join(d, f) for d, _, fs in os.walk("/opt/rocm/llvm/lib/clang")
                 for f in fs if f == "libclang_rt.asan-x86_64.so"]
        if not found:
            pytest.skip("clang's AddressSanitizer runtime is not installed")
        asan = found[0]
    host_objs = []
    for s in b.SOURCES:
        if s.endswith(".hip"):
            continue
        obj = str(tmp_path / (s + ".o"))
        cmd = [hipcc, *b.FLAGS, "-O1", "-g",
               "-Xarch_host", "-fsanitize=address",
               "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=undefined",
               "-Xarch_host", "-fno-omit-frame-pointer",
               "-c", os.path.join(b.CSRC, s), "-o", obj]
        subprocess.run(cmd, check=True, capture_output=True)
        host_objs.append(obj)
    lib = str(tmp_path / "libmpcgemm_san.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-o", lib, *host_objs, *dev_objs, *b.LINK], check=True)
    env = {"LD_PRELOAD": asan, "MPCG_LIBRARY": lib}
    probe = _run_child(["-c", "import ctypes, paper_2307_06072_amd as mp; print(mp.LIB_PATH); "
                              "ctypes.CDLL(None).__asan_init"], env, timeout=300)
    _check_child(probe)
    assert probe.stdout.strip().splitlines()[-1] == lib
    r = _run_child(["-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", "tests/test_abi.py"],
                   env)
    _check_child(r)
    assert " passed" in r.stdout
