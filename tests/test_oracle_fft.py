"""Pins for the DFT oracle (Sec. III, complex FFT) against values fixed by the
mathematics, independent of the oracle's own code.

Each pin set is a function of the implementation under test; it runs on the
oracle (must pass) and on planted mistakes (each must fail at least one pin).
"""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs

RNG = np.random.default_rng(1234)


def _rand(n, batch=3):
    return (RNG.uniform(-1, 1, (batch, n)) + 1j * RNG.uniform(-1, 1, (batch, n)))


def pin_explicit_matrices(dft):
    # N = 1: identity.  N = 2: [[1, 1], [1, -1]].  N = 4: rows of powers of -i.
    x1 = np.array([[0.3 - 0.7j]])
    assert np.allclose(dft(x1), x1, atol=1e-15)
    x2 = np.array([[1.5 + 0.25j, -0.5 + 2.0j]])
    m2 = np.array([[1, 1], [1, -1]])
    assert np.allclose(dft(x2), x2 @ m2.T, atol=1e-14)
    m4 = np.array([[1, 1, 1, 1],
                   [1, -1j, -1, 1j],
                   [1, -1, 1, -1],
                   [1, 1j, -1, -1j]])
    x4 = _rand(4, 2)
    assert np.allclose(dft(x4), x4 @ m4.T, atol=1e-14)
    assert np.allclose(dft(x4, inverse=True), x4 @ m4.conj().T, atol=1e-14)


def pin_impulses(dft, n=16):
    eye = np.eye(n, dtype=np.complex128)
    X = dft(eye)  # row m = DFT of delta_m
    k = np.arange(n)
    assert np.allclose(X[0], np.ones(n), atol=1e-14)
    for m in (1, 3, n - 1):
        assert np.allclose(X[m], np.exp(-2j * np.pi * m * k / n), atol=1e-13)


def pin_constant_and_tone(dft, n=32):
    X = dft(np.ones((1, n)))[0]
    ref = np.zeros(n, dtype=np.complex128)
    ref[0] = n
    assert np.allclose(X, ref, atol=1e-12)
    f = 5
    tone = np.exp(2j * np.pi * f * np.arange(n) / n)[None, :]
    X = dft(tone)[0]
    ref = np.zeros(n, dtype=np.complex128)
    ref[f] = n
    assert np.allclose(X, ref, atol=1e-11)


def pin_parseval_linearity_shift(dft, n=64):
    x, y = _rand(n, 2), _rand(n, 2)
    X, Y = dft(x), dft(y)
    assert np.allclose(np.sum(np.abs(X) ** 2, 1), n * np.sum(np.abs(x) ** 2, 1),
                       rtol=1e-12)
    al, be = 0.7 - 0.2j, -1.3 + 0.4j
    assert np.allclose(dft(al * x + be * y), al * X + be * Y, atol=1e-11)
    s = 3
    k = np.arange(n)
    assert np.allclose(dft(np.roll(x, s, axis=1)), X * np.exp(-2j * np.pi * s * k / n),
                       atol=1e-11)


def pin_real_symmetry_and_inverse(dft, n=64):
    xr = RNG.uniform(-1, 1, (2, n)).astype(np.complex128)
    X = dft(xr)
    k = np.arange(1, n)
    assert np.allclose(X[:, n - k], np.conj(X[:, k]), atol=1e-12)
    x = _rand(n, 2)
    assert np.allclose(dft(dft(x), inverse=True), n * x, atol=1e-11)


def pin_numpy_cross_check(dft):
    for n in (16, 128, 1024):
        x = _rand(n, 2)
        ref = np.fft.fft(x, axis=1)
        err = np.max(np.abs(dft(x) - ref)) / np.max(np.abs(ref))
        assert err < 1e-12
        ref_i = np.fft.ifft(x, axis=1) * n
        assert np.max(np.abs(dft(x, inverse=True) - ref_i)) / np.max(np.abs(ref_i)) < 1e-12


PINS = [pin_explicit_matrices, pin_impulses, pin_constant_and_tone,
        pin_parseval_linearity_shift, pin_real_symmetry_and_inverse,
        pin_numpy_cross_check]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_dft_pins(pin):
    pin(oracle.dft)


# Planted mistakes: each models a plausible slip in a DFT implementation.
MUTANTS = {
    "wrong_sign": lambda x, inverse=False: oracle.dft(x, inverse=not inverse),
    "dropped_last_term": lambda x, inverse=False: oracle.dft(
        np.concatenate([np.asarray(x)[:, :-1], 0 * np.asarray(x)[:, -1:]], 1), inverse),
    "output_off_by_one": lambda x, inverse=False: np.roll(oracle.dft(x, inverse), 1, axis=1),
    "normalised": lambda x, inverse=False: oracle.dft(x, inverse) / np.asarray(x).shape[-1],
    "input_reversed": lambda x, inverse=False: oracle.dft(np.asarray(x)[:, ::-1], inverse),
    "bit_reversed_output": lambda x, inverse=False: _bitrev(oracle.dft(x, inverse)),
}


def _bitrev(X):
    n = X.shape[1]
    bits = max(1, int(np.log2(n)))
    idx = np.array([int(format(i, f"0{bits}b")[::-1], 2) for i in range(n)]) if n > 1 else [0]
    return X[:, idx]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    mutant = MUTANTS[name]
    failed = 0
    for pin in PINS:
        try:
            pin(mutant)
        except AssertionError:
            failed += 1
    assert failed >= 1, f"no pin caught mutant {name}"


def test_oracle_on_workload_recipe_matches_numpy():
    # The GPU parity case at the smallest benchmark size: 64 signals of 1024.
    x = inputs.fft_input(1024, 64, seed=0)
    X = oracle.dft(x)
    ref = np.fft.fft(x.astype(np.complex128), axis=1)
    assert np.max(oracle.rel_l2(X, ref)) < 1e-12
    assert x.dtype == np.complex64 and x.shape == (64, 1024)


def test_rel_l2_pins():
    ref = np.array([[3.0 + 4.0j, 0.0]])
    assert oracle.rel_l2(ref, ref)[0] == 0.0
    assert np.isclose(oracle.rel_l2(np.array([[3.0 + 4.0j, 5.0]]), ref)[0], 1.0)


# ---------------------------------------------------------------- per-bin DFT
# Pins of oracle.dft_bins, the check for sizes whose full O(N^2) transform is
# too slow: closed forms (an impulse at j0 gives exp(-2 pi i j0 k / N) in every
# bin, a constant gives N at bin 0 and 0 elsewhere), numpy's FFT at a few
# bins of a large random input, and the direction sign.

def test_dft_bins_closed_forms():
    n, j0 = 1 << 15, 12345
    ks = np.array([0, 1, 2, 777, n // 2, n - 1])
    x = np.zeros((2, n), np.complex128)
    x[0, j0] = 1.0
    x[1, :] = 1.0
    X = oracle.dft_bins(x, ks)
    assert np.allclose(X[0], np.exp(-2j * np.pi * j0 * ks / n), atol=1e-12)
    ref = np.where(ks == 0, float(n), 0.0)
    assert np.allclose(X[1], ref, atol=1e-7)


def test_dft_bins_match_numpy_and_direction():
    n = 1 << 16
    x = inputs.fft_input(n, 2, seed=5).astype(np.complex128)
    ks = np.array([0, 3, 4096, 31337, n - 1])
    X = oracle.dft_bins(x, ks)
    F = np.fft.fft(x, axis=1)[:, ks]
    assert np.max(np.abs(X - F)) <= 1e-9 * np.max(np.abs(F))
    Xi = oracle.dft_bins(x, ks, inverse=True)
    Fi = np.fft.ifft(x, axis=1)[:, ks] * n
    assert np.max(np.abs(Xi - Fi)) <= 1e-9 * np.max(np.abs(Fi))
    # a wrong sign would be caught: forward and inverse differ at these bins
    assert np.max(np.abs(X - Xi)) > 1.0


def test_dft_bins_reject_out_of_range_bins():
    with pytest.raises(RuntimeError):
        oracle.dft_bins(np.zeros((1, 16), np.complex64), [16])
