"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "phicomb.h")).read()
    return re.findall(r"^\s*(?:int|int64_t|const char \*)\s*\**(phicomb_\w+)\(", src, re.M)


def test_header_declares_the_api():
    names = set(_declared())
    for n in ("phicomb_op_create_csr", "phicomb_op_create_stencil", "phicomb_op_create_dense",
              "phicomb_params", "phicomb_solve", "phicomb_submit", "phicomb_poll",
              "phicomb_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2509_26475_amd as pc
    lib = pc._lib()
    for n in _declared():
        assert hasattr(lib, n), n
    assert pc.phicomb_strerror(pc.EOVERFLOW).startswith("power basis")


def test_no_oracle_in_product_path():
    """The HIP library and its binding never reach the oracle."""
    pkg = os.path.join(ROOT, "paper_2509_26475_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "phicomb_oracle" not in txt, f
