"""The C ABI from plain C: tests/c/abi_dimer.c is compiled against
include/aqs.h and linked with libaqs.so and the HIP runtime only (no Python
binding, no torch); on the GPU it minimises a dimer to the analytic minimum
of Eq. (13) and steps it (see the program's header)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2507_20802_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def compile_program(out_dir: str) -> str:
    if not os.path.exists(os.path.join(PKG, "libaqs.so")):
        pytest.skip("libaqs.so is not built")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = os.path.join(out_dir, "abi_dimer")
    cmd = [cc, "-std=c11", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c", "abi_dimer.c"), "-o", exe,
           "-L", PKG, "-laqs", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


def test_c_program_compiles_and_links_against_the_abi(tmp_path):
    assert os.access(compile_program(str(tmp_path)), os.X_OK)


@pytest.mark.gpu
def test_c_program_minimises_a_dimer_through_the_abi(tmp_path):
    exe = compile_program(str(tmp_path))
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr)
    assert res.returncode == 0 and "abi ok" in res.stdout
