"""Pins for the inclusive-scan oracle (Sec. III, "Scan Operator": every element
becomes the sum of all elements from the first up to itself)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs


def pin_closed_forms(scan):
    n = 100
    assert np.array_equal(scan(np.ones((1, n), np.int32))[0], np.arange(1, n + 1))
    ar = np.arange(n, dtype=np.int32)[None]
    assert np.array_equal(scan(ar)[0], np.arange(n) * (np.arange(n) + 1) // 2)
    alt = np.array([[1, -1] * 8], dtype=np.int32)
    assert np.array_equal(scan(alt)[0], np.array([1, 0] * 8))
    imp = np.zeros((1, 16), np.int32)
    imp[0, 5] = 7
    assert np.array_equal(scan(imp)[0], np.where(np.arange(16) >= 5, 7, 0))


def pin_invariants(scan):
    x = np.random.default_rng(5).integers(-1000, 1000, (4, 257), dtype=np.int32)
    y = scan(x)
    assert np.array_equal(y[:, -1], x.astype(np.int64).sum(1))
    assert np.array_equal(np.diff(y.astype(np.int64), axis=1), x[:, 1:])
    assert np.array_equal(y[:, 0], x[:, 0])
    perm = np.array([2, 0, 3, 1])
    assert np.array_equal(scan(x[perm]), y[perm])


def pin_brute_force_01(scan):
    # Every 0/1 vector of length 10, against the sum written as a Python loop.
    vecs = np.array(list(itertools.product([0, 1], repeat=10)), dtype=np.int32)
    y = scan(vecs)
    for v, yy in zip(vecs[::37], y[::37]):
        acc, ref = 0, []
        for e in v:
            acc += int(e)
            ref.append(acc)
        assert list(yy) == ref
    assert np.array_equal(y, np.cumsum(vecs, axis=1))


def pin_numpy_int64(scan):
    x = inputs.scan_input(8192, 4, np.int32, seed=3)
    assert np.array_equal(scan(x), np.cumsum(x.astype(np.int64), axis=1))


def pin_float_exact(scan):
    # float32 uniform[0,1) values are multiples of 2^-24; 2^14 of them sum
    # exactly in float64, so the float oracle must equal the integer sum.
    x = inputs.scan_input(1 << 14, 2, np.float32, seed=7)
    k = (x.astype(np.float64) * 2.0 ** 24).astype(np.int64)
    assert np.array_equal(k.astype(np.float64) * 2.0 ** -24, x.astype(np.float64))
    y = scan(x)
    assert np.array_equal(y * 2.0 ** 24, np.cumsum(k, axis=1).astype(np.float64))


PINS = [pin_closed_forms, pin_invariants, pin_brute_force_01, pin_numpy_int64,
        pin_float_exact]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_scan_pins(pin):
    pin(oracle.scan)


def test_int32_wraps_modulo_2_32():
    x = np.array([[2 ** 31 - 1, 1, 5, -(2 ** 31), -(2 ** 31)]], dtype=np.int32)
    y = oracle.scan(x)[0]
    acc, ref = 0, []
    for e in x[0]:
        acc = (acc + int(e)) % (1 << 32)
        ref.append(acc - (1 << 32) if acc >= (1 << 31) else acc)
    assert y.dtype == np.int32 and list(y) == ref


def _shift(y):
    z = np.zeros_like(y)
    z[:, 1:] = y[:, :-1]
    return z


MUTANTS = {
    "exclusive_instead_of_inclusive": lambda x: _shift(oracle.scan(x)),
    "dropped_first_element": lambda x: oracle.scan(np.asarray(x)) - np.asarray(x)[:, :1],
    "scanned_right_to_left": lambda x: oracle.scan(np.asarray(x)[:, ::-1])[:, ::-1],
    "includes_next_element": lambda x: oracle.scan(x) + np.concatenate(
        [np.asarray(x)[:, 1:], np.zeros_like(np.asarray(x)[:, :1])], 1),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    failed = 0
    for pin in PINS:
        try:
            pin(MUTANTS[name])
        except AssertionError:
            failed += 1
    assert failed >= 1, f"no pin caught mutant {name}"


# ------------------------------------------------------------ exclusive form
# Each output is the sum of the elements strictly before it (0 first).

def _excl(x):
    return oracle.scan(x, exclusive=True)


def test_exclusive_closed_forms():
    n = 100
    assert np.array_equal(_excl(np.ones((1, n), np.int32))[0], np.arange(n))
    ar = np.arange(n, dtype=np.int32)[None]
    assert np.array_equal(_excl(ar)[0], np.arange(n) * (np.arange(n) - 1) // 2)
    imp = np.zeros((1, 16), np.int32)
    imp[0, 5] = 7
    assert np.array_equal(_excl(imp)[0], np.where(np.arange(16) > 5, 7, 0))
    x = np.random.default_rng(2).integers(-9, 9, (3, 33), dtype=np.int32)
    assert np.all(_excl(x)[:, 0] == 0)
    assert np.all(_excl(x.astype(np.float64))[:, 0] == 0.0)


def test_exclusive_brute_force_01():
    vecs = np.array(list(itertools.product([0, 1], repeat=10)), dtype=np.int32)
    y = _excl(vecs)
    for v, yy in zip(vecs[::29], y[::29]):
        ref, before = [], 0
        for e in v:
            ref.append(before)
            before += int(e)
        assert list(yy) == ref


def test_exclusive_against_numpy_with_wrap():
    x = np.random.default_rng(4).integers(-2 ** 31, 2 ** 31, (5, 1000), dtype=np.int32)
    want = np.zeros((5, 1000), dtype=np.int64)
    want[:, 1:] = np.cumsum(x.astype(np.int64), axis=1)[:, :-1]
    want = (want % (1 << 32)).astype(np.uint32).view(np.int32)
    assert np.array_equal(_excl(x), want)


def test_exclusive_in_place_buffer_semantics():
    # the exclusive output at i never depends on x[i]: changing the last
    # element of a row changes no output of that row
    x = inputs.scan_input(64, 3, np.int32, seed=8)
    x2 = x.copy()
    x2[:, -1] += 5
    assert np.array_equal(_excl(x), _excl(x2))


# ------------------------------------------------------------ float64 inputs

@pytest.mark.parametrize("exclusive", [False, True])
def test_float64_exact_on_dyadic_values(exclusive):
    k, x = inputs.scan_input_dyadic(4096, 3, seed=12)
    s = np.cumsum(k, axis=1)
    if exclusive:
        s = np.concatenate([np.zeros((3, 1), np.int64), s[:, :-1]], axis=1)
    assert np.array_equal(oracle.scan(x, exclusive=exclusive), s.astype(np.float64) * 2.0 ** -20)


def test_float64_within_recursive_summation_bound():
    # Left-to-right summation of i+1 terms is within i * u / (1 - i u) of
    # the exact sum, relative to the sum of |x| (Higham, Accuracy and
    # Stability of Numerical Algorithms, Sec. 4.2); math.fsum gives the
    # correctly rounded exact sum.
    import math
    x = np.random.default_rng(13).standard_normal((2, 600))
    y = oracle.scan(x)
    u = 2.0 ** -53
    for b in range(2):
        for i in range(0, 600, 7):
            exact = math.fsum(x[b, :i + 1])
            s_abs = math.fsum(np.abs(x[b, :i + 1]))
            assert abs(y[b, i] - exact) <= (i * u / (1 - i * u)) * s_abs + u * abs(exact)
