"""Stored fixtures under tests/golden/.

* splitmix64.txt: published first outputs of SplitMix64; the input generator
  must reproduce them.
* stream_chains.txt: written by tests/golden/make_golden.py from the oracle.
  Each line is checked twice: the oracle must still reproduce it (a change to
  the oracle's arithmetic shows up here), and an independent computation must
  agree with it (exact rational arithmetic rounded once per operation,
  tests/exact.py, or the exact integer closed form).
"""
import os
import struct

import numpy as np

import exact
import tsgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def _bits(v) -> str:
    return "0x%016x" % struct.unpack("<Q", struct.pack("<d", float(v)))[0]


def test_splitmix64_published_outputs():
    for state, k, out in _rows("splitmix64.txt"):
        assert int(tsgen.raw(int(state), 0, [int(k) - 1])[0]) == int(out)


def _exact_copyb(k):
    a, b, c = 1.0, 2.0, 0.0
    for _ in range(k):
        a = b
        b = exact.mul(3.0, c, "f64")
        c = exact.add(a, b, "f64")
        a = exact.fma(3.0, c, b, "f64")
    return a, b, c


def test_stream_chains_fixture(oracle_lib):
    rows = _rows("stream_chains.txt")
    assert len(rows) > 20
    n, k_rand = 1000, 3
    rand = [tsgen.uniform_array(2, s, n) for s in range(3)]
    oracle_lib.stream_run(oracle_lib.F64, rand[0], rand[1], rand[2], 3.0, k_rand)
    init = [tsgen.uniform_array(2, s, n) for s in range(3)]
    for row in rows:
        if row[0] == "constant":
            order, k, want = row[1], int(row[2]), row[3:6]
            if order == "listing":
                got = oracle_lib.stream_scalar_f64(1.0, 2.0, 0.0, 3.0, k)
                ind = exact.stream_scalar(1.0, 2.0, 0.0, 3.0, k, "f64", fused=True)
            else:
                s = [np.array([v]) for v in (1.0, 2.0, 0.0)]
                oracle_lib.stream_run_copyb_f64(*s, 3.0, k)
                got = tuple(float(x[0]) for x in s)
                ind = _exact_copyb(k)
            assert [_bits(v) for v in got] == want, row
            assert [_bits(v) for v in ind] == want, row
        else:
            k, name, j, want = int(row[1]), row[2], int(row[3]), row[4]
            assert k == k_rand
            idx = "abc".index(name)
            assert _bits(rand[idx][j]) == want, row
            a, b, c = (float(v[j]) for v in init)
            for _ in range(k):
                c = a
                b = exact.mul(3.0, c, "f64")
                c = exact.add(a, b, "f64")
                a = exact.fma(3.0, c, b, "f64")
            assert _bits((a, b, c)[idx]) == want, row
