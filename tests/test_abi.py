"""The C ABI: librbws.so loads on a machine without a GPU and exports every
function that include/rbws.h declares (no compute calls are made here)."""
import ctypes
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbws.h")
LIB = os.path.join(ROOT, "paper_2311_13862_amd", "librbws.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(rbws_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rbws_problem_create", "rbws_rb_build", "rbws_rb_coeffs", "rbws_rb_lift", "rbws_solve",
              "rbws_mlp_create", "rbws_mlp_train", "rbws_mlp_predict", "rbws_spmv", "rbws_exact_dots"):
        assert n in names, n
    assert len(names) >= 35, names


def _lib():
    """The library as the binding loads it (after torch, on torch's HIP runtime)."""
    if not os.path.exists(LIB):
        from paper_2311_13862_amd import build
        build.build()
    from paper_2311_13862_amd import rbws
    return rbws.lib()


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.rbws_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.rbws_version()


def test_tuning_knobs_validate_without_a_gpu():
    """rbws_set_tuning checks its arguments on the host (no device call)."""
    lib = _lib()
    RBWS_TUNE_TZ, EINVAL = 2, -1
    assert lib.rbws_set_tuning(RBWS_TUNE_TZ, 12) == EINVAL
    assert lib.rbws_set_tuning(RBWS_TUNE_TZ, 128) == EINVAL
    assert lib.rbws_set_tuning(RBWS_TUNE_TZ, 32) == 0
    assert lib.rbws_set_tuning(RBWS_TUNE_TZ, 0) == 0
    RBWS_TUNE_MG_PZ = 3
    assert lib.rbws_set_tuning(RBWS_TUNE_MG_PZ, 2) == EINVAL
    assert lib.rbws_set_tuning(RBWS_TUNE_MG_PZ, 1) == 0
    assert lib.rbws_set_tuning(99, 0) == EINVAL


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must leave one HIP and one HSA runtime
    mapped (torch's): with two, the library's runtime sees no device."""
    _lib()
    code = ("from paper_2311_13862_amd import rbws\n"
            "import torch\n"
            "m = rbws.mapped_runtimes()\n"
            "print({k: len(v) for k, v in m.items()})\n"
            "assert all(len(v) == 1 for v in m.values()), m\n"
            "tl = os.path.dirname(torch.__file__)\n"
            "assert all(p.startswith(tl) for v in m.values() for p in v), m\n")
    r = subprocess.run([sys.executable, "-c", "import os\n" + code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
