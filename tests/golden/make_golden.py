"""Write tests/golden/stream_chains.txt from the CPU oracle alone.

The file records binary64 bit patterns of STREAM chains (Section 5,
Listing 4): constant initial values (1, 2, 0) with q = 3 in the listing's
order and in the copy a = b variant, and a seeded random start.  It is a
regression fixture: tests/test_golden.py checks that the oracle still
reproduces it.  Inputs come from tsgen; every value comes from oracle/.

    python tests/golden/make_golden.py
"""
import os
import struct
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import tsgen  # noqa: E402


def bits(v: float) -> str:
    return "0x%016x" % struct.unpack("<Q", struct.pack("<d", float(v)))[0]


def main() -> None:
    import numpy as np

    lines = ["# STREAM chains computed by the CPU oracle (tests/golden/make_golden.py).",
             "# constant: order k a b c   (from a = 1, b = 2, c = 0, q = 3)",
             "# random:   k array index value   (tsgen seed 2, streams a = 0, b = 1, c = 2, n = 1000, q = 3)"]
    for k in (1, 10, 13, 14, 21, 33, 50, 51, 80):
        a, b, c = oracle.stream_scalar_f64(1.0, 2.0, 0.0, 3.0, k)
        lines.append(f"constant listing {k} {bits(a)} {bits(b)} {bits(c)}")
    for k in (1, 10, 21, 25, 40):
        s = [np.array([v]) for v in (1.0, 2.0, 0.0)]
        oracle.stream_run_copyb_f64(*s, 3.0, k)
        lines.append(f"constant copy_b {k} {bits(s[0][0])} {bits(s[1][0])} {bits(s[2][0])}")
    n, k = 1000, 3
    arr = [tsgen.uniform_array(2, stream, n) for stream in range(3)]
    oracle.stream_run(oracle.F64, arr[0], arr[1], arr[2], 3.0, k)
    for name, x in zip("abc", arr):
        for j in (0, 1, 2, 3, 499, 998, 999):
            lines.append(f"random {k} {name} {j} {bits(x[j])}")
    with open(os.path.join(HERE, "stream_chains.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
