"""Benchmark-file ingestion (ubqp_read_instance) and time-to-target, on the CPU.

The paper's test problems (OR-Library bqp sets, Palubeckis instances) are not
in this repository; the files here are written by the tests, in the same text
formats, from seeded synthetic matrices, so every read is checked against the
matrix it was written from."""
import ctypes
import os

import numpy as np
import pytest

from paper_1706_00037_amd import ubqp
from paper_1706_00037_amd.inputs import make_instance

pytestmark = pytest.mark.skipif(not os.path.exists(ubqp.LIB_PATH), reason="libubqp.so not built")


def _entries(Q, rng, both=False):
    """(i, j, q) 1-based triples of the nonzeros with i <= j (and the mirror
    entry too with `both`), in a shuffled order."""
    n = Q.shape[0]
    iu, ju = np.nonzero(np.triu(Q))
    t = [(int(i) + 1, int(j) + 1, int(Q[i, j])) for i, j in zip(iu, ju)]
    if both:
        t += [(j, i, q) for i, j, q in t if i != j]
    rng.shuffle(t)
    return t


def _write(path, blocks, orlib=True, seps=(" ", "\t", "  ")):
    rng = np.random.default_rng(7)
    lines = [str(len(blocks))] if orlib else []
    for n, t in blocks:
        lines.append(f"{n} {len(t)}")
        for i, j, q in t:
            s = seps[int(rng.integers(len(seps)))]
            lines.append(f"{i}{s}{j}{s}{q}")
    path.write_text("\n".join(lines) + "\n")


def test_orlib_round_trip(tmp_path):
    rng = np.random.default_rng(1)
    Qs = [make_instance(7, 0.5, -100, 100, 11), make_instance(50, 0.1, -100, 100, 12),
          make_instance(129, 0.9, -100, 100, 13)]
    p = tmp_path / "bqp_like.txt"
    _write(p, [(Q.shape[0], _entries(Q, rng)) for Q in Qs])
    for k, Q in enumerate(Qs):
        R, count = ubqp.read_instance(str(p), ubqp.UBQP_FMT_ORLIB, k)
        assert count == 3
        assert R.dtype == np.int32 and R.shape == Q.shape
        assert np.array_equal(R, Q)
        assert np.array_equal(R, R.T)


def test_both_triangles_listed_and_crlf(tmp_path):
    rng = np.random.default_rng(2)
    Q = make_instance(40, 0.3, -100, 100, 21)
    t = _entries(Q, rng, both=True)
    p = tmp_path / "both.txt"
    p.write_bytes(("1\r\n40 %d\r\n" % len(t) + "".join(f"{i} {j} {q}\r\n" for i, j, q in t)).encode())
    R, count = ubqp.read_instance(str(p), ubqp.UBQP_FMT_ORLIB, 0)
    assert count == 1 and np.array_equal(R, Q)


def test_triplets_round_trip_no_trailing_newline(tmp_path):
    rng = np.random.default_rng(3)
    Q = make_instance(300, 0.5, -100, 100, 31)
    t = _entries(Q, rng)
    p = tmp_path / "p_like.txt"
    p.write_text(f"300 {len(t)}\n" + "\n".join(f"{i} {j} {q}" for i, j, q in t))
    R, count = ubqp.read_instance(str(p), ubqp.UBQP_FMT_TRIPLETS, 0)
    assert count == 1 and np.array_equal(R, Q)


def test_empty_matrix_and_diagonal_only(tmp_path):
    p = tmp_path / "e.txt"
    p.write_text("2\n3 0\n4 2\n2 2 -5\n4 4 9\n")
    R, _ = ubqp.read_instance(str(p), ubqp.UBQP_FMT_ORLIB, 0)
    assert np.array_equal(R, np.zeros((3, 3), np.int32))
    R, _ = ubqp.read_instance(str(p), ubqp.UBQP_FMT_ORLIB, 1)
    assert np.array_equal(R, np.diag([0, -5, 0, 9]).astype(np.int32))


@pytest.mark.parametrize("text,fmt,index,code,words", [
    ("1\n3 1\n1 2 5\n", ubqp.UBQP_FMT_ORLIB, 1, ubqp.UBQP_EINVAL, "holds 1 problems"),
    ("1\n3 2\n1 2 5\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "file ends"),
    ("1\n3 1\n1 2 x\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "not an integer"),
    ("1\n3 1\n1 2 5x\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "not an integer"),
    ("1\n3 1\n0 2 5\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "outside 1..3"),
    ("1\n3 1\n1 4 5\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "outside 1..3"),
    ("1\n3 2\n1 2 5\n2 1 6\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EASYM, "listed with 5 and 6"),
    ("1\n3 1\n1 2 3000000000\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_ERANGE, "outside int32"),
    ("1\n9000 0\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_ERANGE, "> 8192"),
    ("1\n0 0\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "n = 0"),
    ("1\n2 5\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "5 entries for n = 2"),
    ("0\n", ubqp.UBQP_FMT_ORLIB, 0, ubqp.UBQP_EINVAL, "0 problems"),
    ("", ubqp.UBQP_FMT_TRIPLETS, 0, ubqp.UBQP_EINVAL, "file ends"),
    ("3 0\n", 3, 0, ubqp.UBQP_EINVAL, "unknown format"),
    ("3 0\n", ubqp.UBQP_FMT_TRIPLETS, 1, ubqp.UBQP_EINVAL, "holds 1 problems"),
])
def test_malformed_files_are_rejected_with_a_reason(tmp_path, text, fmt, index, code, words):
    p = tmp_path / "bad.txt"
    p.write_text(text)
    with pytest.raises(ubqp.UbqpError) as e:
        ubqp.read_instance(str(p), fmt, index)
    assert e.value.code == code
    assert words in str(e.value)


def test_missing_file_and_small_buffer(tmp_path):
    with pytest.raises(ubqp.UbqpError) as e:
        ubqp.read_instance(str(tmp_path / "none.txt"), ubqp.UBQP_FMT_ORLIB, 0)
    assert e.value.code == ubqp.UBQP_EINVAL and "cannot open" in str(e.value)
    p = tmp_path / "s.txt"
    p.write_text("1\n3 1\n1 2 5\n")
    L = ubqp.load()
    buf = np.zeros(8, np.int32)                          # needs 9
    err = ctypes.create_string_buffer(256)
    count, n = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = L.ubqp_read_instance(os.fsencode(str(p)), ubqp.UBQP_FMT_ORLIB, 0, ctypes.byref(count), ctypes.byref(n),
                              buf.ctypes.data_as(ctypes.c_void_p), buf.size, err, len(err))
    assert rc == ubqp.UBQP_EINVAL and b"q_cap = 8" in err.value
    assert np.all(buf == 0)                              # nothing written
    rc = L.ubqp_read_instance(os.fsencode(str(p)), ubqp.UBQP_FMT_ORLIB, 0, None, ctypes.byref(n), None, 0, None, 0)
    assert rc == ubqp.UBQP_EINVAL                        # null count pointer, no message buffer


def test_time_to_target():
    stats = np.zeros((4, 5), np.int64)
    stats[:, 4] = [10, 10, 25, 40]
    r = dict(generations=4, stats=stats, gen_ms=np.array([1.0, 2.0, 3.5, 5.0]))
    assert ubqp.time_to_target(r, 10) == (0, 1.0)
    assert ubqp.time_to_target(r, 11) == (2, 3.5)
    assert ubqp.time_to_target(r, 40) == (3, 5.0)
    assert ubqp.time_to_target(r, 41) is None
    r["generations"] = 3
    assert ubqp.time_to_target(r, 40) is None
