"""The C-ABI library loads and exports every function include/*.h declares,
and the Python binding covers exactly those names (CPU only: no compute)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(aqs_[a-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("aqs_create", "aqs_affine_shear", "aqs_minimize_batch", "aqs_compare_configs", "aqs_stress"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2507_20802_amd import _lib
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    assert declared_functions() <= exported


def test_binding_signatures_cover_the_header():
    from paper_2507_20802_amd import _lib
    assert set(_lib.SIGNATURES) == declared_functions()


def test_struct_sizes_match_the_header_layout():
    from paper_2507_20802_amd import _lib
    assert ctypes.sizeof(_lib.aqs_potential) == 8 + 32 + 32 + 8
    assert ctypes.sizeof(_lib.aqs_fire_params) == 9 * 8 + 4 * 4 + 8
    assert ctypes.sizeof(_lib.aqs_step_record) == 8 * 4 + 8
    assert ctypes.sizeof(_lib.aqs_cg_params) == 5 * 8 + 2 * 4 + 8
    n_params = 64 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3
    assert ctypes.sizeof(_lib.aqs_mlp) == 8 + 4 * (n_params + 64 + 64 + 3 + 3)


def test_struct_sizes_match_a_c_compiler(tmp_path):
    """sizeof of every ABI struct as gcc lays it out from include/aqs.h."""
    import shutil
    import subprocess
    from paper_2507_20802_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    names = ["aqs_potential", "aqs_fire_params", "aqs_tuning", "aqs_step_record", "aqs_counters",
             "aqs_mlp", "aqs_train_params", "aqs_check", "aqs_cg_params"]
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "aqs.h"\nint main(void){' +
                   "".join(f'printf("%zu\\n", sizeof({n}));' for n in names) + "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                            text=True).stdout.split()]
    assert sizes == [ctypes.sizeof(getattr(_lib, n)) for n in names]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2507_20802_amd import _lib
    monkeypatch.setattr(_lib, "_LIB", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libaqs.so"))
    with pytest.raises(ImportError):
        _lib.load()
