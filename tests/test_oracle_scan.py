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
