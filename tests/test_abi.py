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


def test_request_footprint_host_logic():
    """ubqp_request_footprint is host arithmetic: invalid requests give -1; the
    footprint grows with n and M, two planes (int16 / int32 coefficients) cost more
    than one, and it covers the resident Q planes, the ascent matrix, the population
    and the Delta workspace."""
    if not os.path.exists(ubqp.LIB_PATH):
        pytest.skip("libubqp.so not built")
    fp = ubqp.request_footprint
    base = dict(M=4096, H=10, lam_num=1, lam_den=2, G=10)
    assert fp(0, 1, base) == -1 and fp(8193, 1, base) == -1 and fp(100, 3, base) == -1
    assert fp(100, 1, dict(base, G=0)) == -1 and fp(100, 1, dict(base, M=0)) == -1
    assert fp(100, 1, dict(base, lam_num=3, lam_den=2)) == -1
    prev = 0
    assert fp(129, 1, base) > fp(128, 1, base)                 # next padding step
    for n in (1, 64, 65, 500, 1000, 4000, 7000, 8192):
        f1, f2, f4 = fp(n, 1, base), fp(n, 2, base), fp(n, 4, base)
        assert f1 >= prev and f2 > f1 and f4 >= f2       # equal within one 128-column padding
        prev = f1
        n_pad = -(-n // 128) * 128
        ncol = -(-n_pad // 1024) * 1024
        W = -(-n // 64)
        need = n_pad * n_pad + n_pad * ncol + 4096 * W * 8 + 4096 * 8 + 4096 * n_pad * 4
        assert f1 >= need, (n, f1, need)
        assert f2 >= 2 * n_pad * n_pad + 2 * n_pad * ncol + 2 * 4096 * n_pad * 4
    assert fp(2000, 1, dict(base, M=8192)) > fp(2000, 1, base)
    assert fp(2000, 1, dict(base, G=100)) > fp(2000, 1, base)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message before
    touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_flip_limit_rejects_null_problem_without_a_device():
    L = ubqp.load()
    assert L.ubqp_problem_set_flip_limit(None, 5) == ubqp.UBQP_EINVAL


def test_bench_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    """bench.py reports a kernel's counter traffic only while the kernel's source
    still has the SHA-256 recorded with the counters."""
    import hashlib
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    table = {"k<1>": {"source": "k.hip", "source_sha256": sha, "gb": 1.5},
             "k<2>": {"source": "k.hip", "source_sha256": "0" * 64, "gb": 2.5},
             "k<3>": {"source": "missing.hip", "source_sha256": sha, "gb": 3.5}}
    md = tmp_path / "counters.md"
    md.write_text("# counters\n\n```json\n" + json.dumps(table) + "\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(md))
    monkeypatch.setattr(bench, "CSRC", str(tmp_path))
    t = bench.load_traffic()
    assert t["k<1>"]["gb"] == 1.5 and t["k<2>"] is None and t["k<3>"] is None
    src.write_text("kernel v2\n")                     # the kernel changed since the counters
    assert bench.load_traffic()["k<1>"] is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.load_traffic() == {}
