"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds made for this test alone, each run in a child Python process with
its sanitizer runtime preloaded, so that any report fails the test:

* the C part of the oracle (``oracle/csrc``), built by gcc with
  -fsanitize=address and -fsanitize=undefined, running the oracle tests that
  call it (direct sums, per-pixel w-stacking, binning statistics);
* the host side of librick (argument checks, plan set-up and the no-device
  path in ``plan.cpp``), built by hipcc with the sanitizers on the host pass
  only and linked with the library's own device objects, running the ABI
  tests (every declared symbol, invalid descriptors, NULL pointers and bad
  handles).

Device code is never instrumented: the GPU sanitizers are not used here.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC_ORACLE = os.path.join(ROOT, "oracle", "csrc")
PKG = os.path.join(ROOT, "paper_2504_00959_amd")


def _gcc_runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc has no {name}")
    return path


def _clang_asan_runtime():
    base = "/opt/rocm/llvm/lib/clang"
    if os.path.isdir(base):
        for ver in sorted(os.listdir(base), reverse=True):
            p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
            if os.path.exists(p):
                return p
    pytest.skip("no clang AddressSanitizer runtime")


def _run_child(env_extra, args):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONDONTWRITEBYTECODE"] = "1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + args,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for bad in ("AddressSanitizer", "runtime error:", "LeakSanitizer"):
        assert bad not in out, out[-4000:]
    assert " passed" in out, out[-2000:]
    return out


def test_oracle_c_code_under_asan_and_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    lib = str(tmp_path / "liboracle_san.so")
    srcs = [os.path.join(CSRC_ORACLE, f) for f in ("dft.c", "pixels.c", "binstats.c")]
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
           "-shared", "-fPIC", "-I", CSRC_ORACLE, "-o", lib] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    _run_child({"ORACLE_LIB": lib, "LD_PRELOAD": asan, "OMP_NUM_THREADS": "4"},
               ["tests/test_oracle.py", "-k", "dft or pixel or bin_stats or off_centre"])


def test_librick_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2504_00959_amd import _build
    asan = _clang_asan_runtime()
    obj_dir = os.path.join(PKG, "_build")
    dev = [os.path.join(obj_dir, os.path.splitext(s)[0] + ".o") for s in _build.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in dev):
        _build.build()
    plan_o = str(tmp_path / "plan_san.o")
    # the sanitizers go to the host pass only (device code is not instrumented)
    flags = [f for f in _build.COMMON if f != "-O3"]
    compile_cmd = [_build.HIPCC] + flags + ["-O1", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
                                            "-Xarch_host", "-fsanitize=address",
                                            "-Xarch_host", "-fsanitize=undefined",
                                            "-c", os.path.join(PKG, "csrc", "plan.cpp"), "-o", plan_o]
    r = subprocess.run(compile_cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    lib = str(tmp_path / "librick_san.so")
    # the runtime's symbols come from the preloaded library at load time
    link_cmd = [_build.HIPCC, "-shared", "-fPIC", f"--offload-arch={_build.ARCH}", "-o", lib, plan_o] + dev
    r = subprocess.run(link_cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    _run_child({"RICK_LIB": lib, "LD_PRELOAD": asan}, ["tests/test_abi.py"])
