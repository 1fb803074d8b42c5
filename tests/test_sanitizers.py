"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU (no GPU):
the oracle's C sources under every entry point (tests/c/oracle_sanitize.c),
and the library's host code, rebuilt with the sanitizers on the host side
only, under the ABI's host paths (tests/c/host_sanitize.c).  Leaks count as
failures."""
import concurrent.futures as cf
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1611_00298_amd", "csrc")
LLVM = "/opt/rocm/llvm/bin"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle_sanitize: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(os.path.join(LLVM, "clang")), reason="ROCm clang is not installed")
def test_library_host_code_under_sanitizers(tmp_path):
    # device code is compiled as usual; the sanitizers instrument host code only
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{ROOT}/include", f"-I{CSRC}"] + san
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(["/opt/rocm/bin/hipcc", *flags, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libeofa_san.so")
    rt = _run([f"{LLVM}/clang", "-print-resource-dir"]).stdout.strip() + "/lib/linux"
    _run([f"{LLVM}/clang++", "-shared", "-fsanitize=address,undefined", "-shared-libsan", "-o", lib, *objs,
          "-L/opt/rocm/lib", "-lamdhip64"])
    exe = str(tmp_path / "host_sanitize")
    _run([f"{LLVM}/clang", "-std=c99", "-O1", "-g", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
          "-fsanitize=address,undefined", "-shared-libsan", "-fno-omit-frame-pointer",
          f"-I{ROOT}/include", "-I/opt/rocm/include", os.path.join(ROOT, "tests", "c", "host_sanitize.c"),
          "-o", exe, f"-L{tmp_path}", "-leofa_san", "-L/opt/rocm/lib", "-lamdhip64",
          f"-Wl,-rpath,{tmp_path}:/opt/rocm/lib:{rt}", "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "host_sanitize: ok" in r.stdout
