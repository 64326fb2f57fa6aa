"""Generic transforms: a user expression compiled at run time for the GPU
(the paper's executor runs any device callable; its hello-world example
upper-cases a vector of chars).  Results are compared with the oracle for
the STREAM maps written as expressions, and with numpy's IEEE evaluation
of the same expression otherwise."""
import numpy as np
import pytest

import oracle
import tsgen
from gpu_util import assert_same_bits, device_array, empty_array, say

pytestmark = pytest.mark.gpu

TO_UPPER = "(x >= 'a' && x <= 'z') ? x - ('a' - 'A') : x"


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    yield ts, torch, tgt
    tgt.synchronize()
    tgt.close()


def test_hello_world_to_upper(env):
    """Listing 3: transform the characters of "hello world" to upper case."""
    ts, torch, tgt = env
    text = b"hello world"
    s = device_array(ts, torch, tgt, np.frombuffer(text, np.uint8).copy(), "u8")
    up = ts.Transform(tgt, TO_UPPER, 1, "u8")
    up(tgt, s, s)  # in place, as transform(par.on(exec), s.begin(), s.end(), to_upper)
    assert s.to_host().tobytes() == b"HELLO WORLD"
    rng = np.random.default_rng(1)
    big = rng.integers(32, 127, (1 << 20) + 3).astype(np.uint8)
    B = device_array(ts, torch, tgt, big, "u8", 1)
    D = empty_array(ts, torch, tgt, big.size, "u8")
    up(tgt, B, D)
    assert D.to_host().tobytes() == big.tobytes().upper()
    up.close()


@pytest.mark.parametrize("offset", [0, 1])
def test_fused_triad_expression_equals_oracle(env, offset):
    ts, torch, tgt = env
    n = (1 << 20) + 7
    x = tsgen.uniform_array(3, 0, n)
    y = tsgen.uniform_array(3, 1, n)
    X = device_array(ts, torch, tgt, x, "f64", offset)
    Y = device_array(ts, torch, tgt, y, "f64", offset)
    D = empty_array(ts, torch, tgt, n, "f64", offset)
    tr = ts.Transform(tgt, "__builtin_fma(q, y, x)", 2, "f64")
    say(f"[transform triad off={offset}]")
    tr(tgt, X, D, Y, 3.0)
    ref = np.zeros(n)
    oracle.op(oracle.F64, oracle.TRIAD, x, y, ref, 3.0)
    assert_same_bits(D.to_host(), ref, "f64", "fma expression")
    tr.close()


@pytest.mark.parametrize("dtype,expr,op", [("f32", "q * x", "scale"), ("bf16", "x + y", "add"),
                                           ("f16", "__builtin_fmaf(q, y, x)", "triad"), ("bf16", "x", "copy")])
def test_reduced_expressions_equal_oracle(env, dtype, expr, op):
    ts, torch, tgt = env
    n = 100003
    x = tsgen.uniform_array(4, 0, n, dtype)
    y = tsgen.uniform_array(4, 1, n, dtype)
    X = device_array(ts, torch, tgt, x, dtype)
    Y = device_array(ts, torch, tgt, y, dtype)
    D = empty_array(ts, torch, tgt, n, dtype)
    two = op in ("add", "triad")
    tr = ts.Transform(tgt, expr, 2 if two else 1, dtype)
    tr(tgt, X, D, Y if two else None, 3.0)
    ref = np.zeros_like(x)
    oracle.op(oracle.DTYPES[dtype], oracle.OPS[op], x, y if two else None, ref, 3.0)
    assert_same_bits(D.to_host(), ref, dtype, f"{dtype} {expr}")
    tr.close()


def test_general_expression_matches_numpy(env):
    """x*x - q*y with separate roundings (nothing is contracted), as numpy
    evaluates it in binary64."""
    ts, torch, tgt = env
    n = 300007
    x = tsgen.uniform_array(6, 0, n)
    y = tsgen.uniform_array(6, 1, n)
    X, Y = device_array(ts, torch, tgt, x, "f64"), device_array(ts, torch, tgt, y, "f64")
    D = empty_array(ts, torch, tgt, n, "f64")
    tr = ts.Transform(tgt, "x * x - q * y", 2, "f64")
    tr(tgt, X, D, Y, 0.75)
    ref = x * x - 0.75 * y
    assert_same_bits(D.to_host(), ref, "f64", "x*x - q*y")
    tr2 = ts.Transform(tgt, "x * x - q * y", 2, "f64")  # served from the compile cache
    tr2(tgt, X, D, Y, 0.75)
    assert_same_bits(D.to_host(), ref, "f64", "cached")
    tr.close(), tr2.close()


def test_bad_expressions_and_rules(env):
    ts, torch, tgt = env
    with pytest.raises(ts.TSError) as e:
        ts.Transform(tgt, "x +* y", 2, "f64")
    assert e.value.status == -1 and "error" in e.value.message
    with pytest.raises(ts.TSError):
        ts.Transform(tgt, "x", 3, "f64")
    tr = ts.Transform(tgt, "x + 1.0", 1, "f64")
    a = empty_array(ts, torch, tgt, 100, "f64")
    f = empty_array(ts, torch, tgt, 100, "f32")
    with pytest.raises(ts.TSError) as e:
        tr(tgt, f, f)
    assert e.value.status == -3
    short = empty_array(ts, torch, tgt, 99, "f64")
    with pytest.raises(ts.TSError) as e:
        tr(tgt, a, short)
    assert e.value.status == -2
    tr.close()


@pytest.mark.parametrize("offs", [(0, 0, 0), (1, 1, 1), (1, 0, 0), (0, 1, 1), (1, 1, 0)])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 4099, 100003])
def test_vector_and_elementwise_paths(env, offs, n):
    """Operands sharing their misalignment run the 16-byte vector kernel with
    an element-wise head and tail; others run the element-wise kernel.  Both
    give numpy's IEEE result of the expression."""
    ts, torch, tgt = env
    x = tsgen.uniform_array(8, 0, n)
    y = tsgen.uniform_array(8, 1, n)
    X = device_array(ts, torch, tgt, x, "f64", offs[0])
    Y = device_array(ts, torch, tgt, y, "f64", offs[1])
    D = empty_array(ts, torch, tgt, n, "f64", offs[2])
    tr = ts.Transform(tgt, "x * x - q * y", 2, "f64")
    say(f"[transform paths n={n} offs={offs}]")
    tr(tgt, X, D, Y, 0.75)
    assert_same_bits(D.to_host(), x * x - 0.75 * y, "f64", f"offs={offs}")
    tr(tgt, X, X, Y, 0.75)  # in place
    assert_same_bits(X.to_host(), x * x - 0.75 * y, "f64", "in place")
    tr.close()


@pytest.mark.parametrize("off_in,off_out", [(0, 0), (3, 3), (5, 0), (15, 15)])
@pytest.mark.parametrize("n", [1, 15, 16, 33, 65537])
def test_bytes_to_upper_offsets(env, off_in, off_out, n):
    """1-byte elements: 16 per vector, heads of up to 15 bytes."""
    ts, torch, tgt = env
    rng = np.random.default_rng(n + off_in)
    text = rng.integers(32, 127, n).astype(np.uint8)
    S = device_array(ts, torch, tgt, text, "u8", off_in)
    D = empty_array(ts, torch, tgt, n, "u8", off_out)
    up = ts.Transform(tgt, TO_UPPER, 1, "u8")
    up(tgt, S, D)
    assert D.to_host().tobytes() == text.tobytes().upper()
    up.close()
