"""The C ABI used from plain C99 (tests/c/abi_check.c): it must compile and
link with warnings as errors against include/eofa.h, libeofa.so and the
oracle, and (on a GPU) pass its checks against the oracle."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_check.c")
PKG = os.path.join(ROOT, "paper_1611_00298_amd")
ORC = os.path.join(ROOT, "oracle")


def _compile(out):
    import oracle
    oracle.build(force=False)
    if not os.path.exists(os.path.join(PKG, "libeofa.so")):
        pytest.skip("libeofa.so is not built")
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROOT}/include", "-I/opt/rocm/include", SRC, "-o", out,
           f"-L{PKG}", "-leofa", f"-L{ORC}", "-loracle", "-L/opt/rocm/lib", "-lamdhip64",
           f"-Wl,-rpath,{PKG}:{ORC}:/opt/rocm/lib", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_c_abi_compiles_and_links(tmp_path):
    _compile(str(tmp_path / "abi_check"))


@pytest.mark.gpu
def test_c_abi_runs_on_the_gpu(tmp_path):
    exe = str(tmp_path / "abi_check")
    _compile(exe)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240,
                       env=dict(os.environ, OMP_WAIT_POLICY="PASSIVE"))
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "abi_check: ok" in r.stdout, r.stderr
