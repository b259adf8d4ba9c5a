"""Pins for the tridiagonal oracle (Sec. III: a_i x_{i-1} + b_i x_i +
c_i x_{i+1} = d_i, with the absent unknowns x_{-1} = x_N = 0)."""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs


def _dense(a, b, c):
    n = b.shape[0]
    m = np.diag(b.astype(np.float64))
    if n > 1:
        m += np.diag(a[1:].astype(np.float64), -1) + np.diag(c[:-1].astype(np.float64), 1)
    return m


def pin_diagonal(solve):
    rng = np.random.default_rng(0)
    b = rng.uniform(1, 2, (3, 32))
    d = rng.uniform(-1, 1, (3, 32))
    z = np.zeros_like(b)
    assert np.allclose(solve(z, b, z, d), d / b, rtol=1e-15)


def pin_tiny_systems(solve):
    # N = 1: b x = d.  N = 2: Cramer's rule.
    assert np.allclose(solve([[9.0]], [[4.0]], [[9.0]], [[2.0]]), [[0.5]], rtol=0)
    a, b, c, d = [0.0, 2.0], [3.0, 5.0], [1.0, 0.0], [4.0, 7.0]
    det = b[0] * b[1] - c[0] * a[1]
    x0 = (d[0] * b[1] - c[0] * d[1]) / det
    x1 = (b[0] * d[1] - a[1] * d[0]) / det
    assert np.allclose(solve([a], [b], [c], [d])[0], [x0, x1], rtol=1e-15)


def pin_known_solution(solve):
    a, b, c, d, x = inputs.tridiag_input(1024, 8, np.float64, seed=11)
    xs = solve(a, b, c, d)
    assert np.max(np.abs(xs - x)) < 1e-13


def pin_toeplitz_141(solve):
    n = 64
    ones = np.ones((1, n))
    d = np.full((1, n), 6.0)
    d[0, 0] = d[0, -1] = 5.0
    # The elimination ratios are not exact binary fractions, so agreement is
    # to a few ulps rather than bitwise.
    assert np.max(np.abs(solve(ones, 4 * ones, ones, d) - ones)) < 4e-16


def pin_dense_solve(solve):
    rng = np.random.default_rng(3)
    for n in (3, 7, 16):
        a, c = rng.uniform(-1, 1, (2, n))
        b = np.abs(a) + np.abs(c) + rng.uniform(1, 2, n)
        d = rng.uniform(-1, 1, n)
        ref = np.linalg.solve(_dense(a, b, c), d)
        assert np.allclose(solve(a[None], b[None], c[None], d[None])[0], ref, rtol=1e-13,
                           atol=1e-14)


def pin_row_scaling_and_boundaries(solve):
    a, b, c, d, _ = inputs.tridiag_input(64, 2, np.float64, seed=4)
    x = solve(a, b, c, d)
    s = np.random.default_rng(8).uniform(0.5, 4.0, a.shape)
    assert np.allclose(solve(a * s, b * s, c * s, d * s), x, rtol=1e-13, atol=1e-14)
    a2, c2 = a.copy(), c.copy()
    a2[:, 0] = np.nan
    c2[:, -1] = np.nan
    assert np.array_equal(solve(a2, b, c2, d), x)


PINS = [pin_diagonal, pin_tiny_systems, pin_known_solution, pin_toeplitz_141,
        pin_dense_solve, pin_row_scaling_and_boundaries]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_thomas_pins(pin):
    pin(oracle.thomas)


MUTANTS = {
    "swapped_sub_and_super": lambda a, b, c, d: oracle.thomas(c, b, a, d),
    "reversed_system": lambda a, b, c, d: oracle.thomas(
        *[np.asarray(v, dtype=float)[:, ::-1] for v in (a, b, c, d)]),
    "dropped_subdiagonal": lambda a, b, c, d: oracle.thomas(
        np.zeros_like(np.asarray(a, dtype=float)), b, c, d),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    failed = 0
    for pin in PINS:
        try:
            pin(MUTANTS[name])
        except (AssertionError, FloatingPointError):
            failed += 1
    assert failed >= 1, f"no pin caught mutant {name}"


def test_residual_pins():
    a, b, c, d, x = inputs.tridiag_input(256, 4, np.float64, seed=2)
    assert np.max(oracle.tridiag_residual(a, b, c, d, x)) < 1e-15
    xs = oracle.thomas(a, b, c, d)
    assert np.max(oracle.tridiag_residual(a, b, c, d, xs)) < 1e-15
    # A perturbation of one unknown by e gives a residual of exactly the
    # column of A scaled by e.
    x2 = x.copy()
    x2[0, 10] += 1e-3
    col = np.array([c[0, 9], b[0, 10], a[0, 11]]) * 1e-3
    r = oracle.tridiag_residual(a[:1], b[:1], c[:1], d[:1], x2[:1])[0]
    assert np.isclose(r, np.linalg.norm(col) / np.linalg.norm(d[0]), rtol=1e-9)


def test_inputs_recipe_is_diagonally_dominant():
    for dt in (np.float32, np.float64):
        a, b, c, d, x = inputs.tridiag_input(128, 16, dt, seed=0)
        assert a.dtype == dt and d.dtype == dt
        assert np.all(np.abs(b) >= np.abs(a) + np.abs(c) + 1.0 - 1e-6)
        assert np.all(np.abs(x) <= 1.0)


def test_phi_pins():
    assert oracle.phi([1.0, 1.0, 1.0]) == 1.0
    assert np.isclose(oracle.phi([1.0, 0.5]), 2.0 / 3.0)
    e = [0.9, 0.5, 0.75, 1.0]
    assert oracle.phi(e) <= np.mean(e) and min(e) <= oracle.phi(e) <= 1.0
    with pytest.raises(ValueError):
        oracle.phi([1.0, 0.0])
