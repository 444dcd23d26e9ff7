"""Address and undefined-behaviour sanitizer builds, on the CPU.

- The oracle, built by g++ with -fsanitize=address,undefined, runs every
  entry point on Figure 1, small random trees, an overflowing chain and a
  cyclic natural join, and must agree with the regular build.
- The runtime's host code, built by hipcc with the sanitizers on the host
  side only (-Xarch_host) and without device code (--offload-host-only; each
  translation unit's code-object symbol is a placeholder, as no kernel is
  launched), runs graph validation, the junction tree, the expansion's launch
  shapes and the stored-summary file check on good and damaged inputs.

Each runs in a child process that preloads the matching sanitizer runtime;
an invalid access or undefined behaviour aborts it and fails the test."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(script, args, preload, tmp_path):
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload)
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, script), *args], env=env, cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    asan = subprocess.check_output([gxx, "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("g++ has no address sanitizer runtime")
    from oracle import oracle as O

    O.build()  # the regular build the results are compared with
    lib = str(tmp_path / "liboracle_san.so")
    srcs = sorted(glob.glob(os.path.join(ROOT, "oracle", "*.cpp")))
    subprocess.check_call([gxx, "-O1", "-g", "-std=c++17", "-shared", "-fPIC", "-pthread",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           *srcs, "-o", lib])
    out = _run("sanitized_oracle_run.py", [lib], asan, tmp_path)
    assert "sanitized oracle ok" in out


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_runtime_host_code_under_address_and_ub_sanitizers(tmp_path):
    if os.path.exists("/dev/kfd"):
        pytest.skip("the host-only build carries placeholder code objects: run it where no GPU is visible")
    hipcc, gxx, rt = shutil.which("hipcc"), shutil.which("g++"), _clang_asan_runtime()
    if not (hipcc and gxx and rt):
        pytest.skip("hipcc, g++ or the clang address sanitizer runtime not found")
    from paper_2206_10435_amd import build as B

    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g", "--offload-host-only", "-fno-omit-frame-pointer",
                                                  "-Xarch_host", "-fsanitize=address",
                                                  "-Xarch_host", "-fsanitize=undefined",
                                                  "-Xarch_host", "-fno-sanitize-recover=all"]

    def comp(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([hipcc, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj], capture_output=True,
                           text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with cf.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(comp, B.SOURCES))
    # one placeholder per translation unit's code-object symbol
    undef = subprocess.check_output(["nm", "-u", *objs], text=True).split()
    syms = sorted({s for s in undef if s.startswith("__hip_fatbin_")})
    stub = tmp_path / "placeholders.cpp"
    stub.write_text("".join(f'extern "C" const char {s}[64] = {{0}};\n' for s in syms))
    subprocess.check_call([gxx, "-c", "-fPIC", str(stub), "-o", str(tmp_path / "placeholders.o")])
    lib = str(tmp_path / "libgj_host_san.so")
    subprocess.check_call([gxx, "-shared", "-fPIC", *objs, str(tmp_path / "placeholders.o"), "-o", lib,
                           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", rt])
    out = _run("sanitized_runtime_run.py", [lib, str(tmp_path)], rt, tmp_path)
    assert "sanitized runtime host paths ok" in out
