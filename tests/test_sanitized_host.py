"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The float64 oracle is rebuilt by gcc with both sanitizers and runs its pins;
the library is rebuilt by hipcc with both sanitizers on its host side only
and runs the host-validation tests.  Each runs in a child process with the
sanitizer runtime preloaded (the interpreter itself is not instrumented);
any report aborts that process and fails the test.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(extra_env, tests):
    env = dict(os.environ)
    env.update(ENV)
    env.update(extra_env)
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    return tail


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.exists(asan) and os.path.isabs(ubsan) and os.path.exists(ubsan)):
        pytest.skip("gcc sanitizer runtimes not installed")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", so, "-lm"], check=True)
    tail = _run({"ORACLE_LIB": so, "LD_PRELOAD": f"{asan} {ubsan}"},
                ["tests/test_oracle_neighbours.py", "tests/test_oracle_gnn.py", "tests/test_oracle_components.py",
                 "tests/test_oracle_triplets.py", "tests/test_oracle_int8.py", "tests/test_oracle_embed.py"])
    print(tail.strip().splitlines()[-1])


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang AddressSanitizer runtime not installed")
    objs = []
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2407_12119_amd", "csrc", "*.hip")))
    procs = []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        # sanitizers on the host pass only (each flag after -Xarch_host)
        procs.append(subprocess.Popen(
            ["hipcc", "-c", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2407_12119_amd", "csrc"),
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", src, "-o", obj],
            stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err[-2000:]
    so = str(tmp_path / "libvelognn_san.so")
    subprocess.run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", so], check=True)
    tail = _run({"VELO_LIB": so, "LD_PRELOAD": rt[-1]}, ["tests/test_abi_host.py", "tests/test_abi.py"])
    print(tail.strip().splitlines()[-1])
