"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1706_00037_amd import ubqp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_boundary():
    names = ubqp.declared_functions()
    for want in ("ubqp_diversify", "ubqp_eval", "ubqp_screen", "ubqp_ascent", "ubqp_multistart",
                 "ubqp_create", "ubqp_destroy", "ubqp_problem_create", "ubqp_problem_destroy",
                 "ubqp_last_error"):
        assert want in names


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(ubqp.LIB_PATH):
        pytest.skip("libubqp.so not built")
    L = ctypes.CDLL(ubqp.LIB_PATH)
    for name in ubqp.declared_functions():
        assert hasattr(L, name), name


def test_library_exports_nothing_undeclared():
    if not os.path.exists(ubqp.LIB_PATH):
        pytest.skip("libubqp.so not built")
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", ubqp.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ubqp_\w+)", out))
    assert exported == set(ubqp.declared_functions())


def test_null_arguments_are_rejected_without_a_device():
    L = ubqp.load()
    assert L.ubqp_create(None, 0, None) == ubqp.UBQP_EINVAL
    assert L.ubqp_sync(None) == ubqp.UBQP_EINVAL
    assert L.ubqp_problem_destroy(None) == ubqp.UBQP_EINVAL
    assert L.ubqp_last_error(None) == b"null context"


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_1706_00037_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "ubqp_oracle" not in text, f
