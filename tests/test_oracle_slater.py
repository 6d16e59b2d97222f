"""Pins of the oracle's Sherman-Morrison update (Sec. VI.D, the inverse of
the Slater matrix of Eq. (5) after accepted moves) by things other than the
update itself: a 2x2 case worked in exact rational arithmetic, explicit
inverses and determinants (numpy.linalg) of the moved matrices, and the
invariants the sequential update must keep.  Each pin is a function of the
update under test, so planted mistakes in copies of it can be shown to fail."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import slater


def well_conditioned(rng, n):
    return 2.0 * np.eye(n) + rng.normal(0, 1.0 / np.sqrt(n), (n, n))


def moves(rng, D, k):
    """k distinct electrons, each given a new orbital row close to its old
    one (as a small trial move would), in a shuffled order."""
    n = D.shape[0]
    cols = rng.permutation(n)[:k]
    u = D[cols] + rng.normal(0, 0.5, (k, n))
    return cols, u


def apply_rows(D, cols, u):
    D = D.copy()
    for c, row in zip(cols, u):
        D[c] = row
    return D


# --- pins, each a check of an update function fn(inv_t, u, cols) ---------

def pin_2x2_exact(fn):
    """D = [[3, 1], [4, 2]] (electron rows), electron 0 moves to (5, 7):
    D' = [[5, 7], [4, 2]], det D = 2, det D' = -18, ratio -9, and
    inv(D')^T = [[2, -4], [-7, 5]] / -18, all exact."""
    D = [[Fraction(3), Fraction(1)], [Fraction(4), Fraction(2)]]
    det = D[0][0] * D[1][1] - D[0][1] * D[1][0]
    inv_t = [[D[1][1] / det, -D[1][0] / det], [-D[0][1] / det, D[0][0] / det]]
    u = [Fraction(5), Fraction(7)]
    det1 = u[0] * D[1][1] - u[1] * D[1][0]
    want_ratio = det1 / det
    want_t = [[D[1][1] / det1, -D[1][0] / det1], [-u[1] / det1, u[0] / det1]]
    b, r = fn(np.array(inv_t, dtype=float), np.array([u], dtype=float), [0])
    assert float(want_ratio) == -9.0
    np.testing.assert_allclose(r, [float(want_ratio)], rtol=1e-15)
    np.testing.assert_allclose(b, np.array(want_t, dtype=float), rtol=1e-15, atol=1e-16)


def pin_explicit_inverse(fn, seed=0, n=12, k=7):
    rng = np.random.default_rng(seed)
    D = well_conditioned(rng, n)
    cols, u = moves(rng, D, k)
    b, _ = fn(np.linalg.inv(D).T, u, cols)
    want = np.linalg.inv(apply_rows(D, cols, u)).T
    np.testing.assert_allclose(b, want, rtol=0, atol=1e-11 * np.abs(want).max())


def pin_ratios_are_determinant_ratios(fn, seed=1, n=10, k=6):
    rng = np.random.default_rng(seed)
    D = well_conditioned(rng, n)
    cols, u = moves(rng, D, k)
    _, r = fn(np.linalg.inv(D).T, u, cols)
    prev = np.linalg.det(D)
    for m in range(k):
        cur = np.linalg.det(apply_rows(D, cols[: m + 1], u[: m + 1]))
        assert r[m] == pytest.approx(cur / prev, rel=1e-11), m
        prev = cur


def pin_unmoved_electron(fn, seed=2, n=9):
    """A 'move' that gives electron c its own orbital row back: ratio 1 and
    the inverse unchanged."""
    rng = np.random.default_rng(seed)
    D = well_conditioned(rng, n)
    inv_t = np.linalg.inv(D).T
    b, r = fn(inv_t, D[[4]], [4])
    assert r[0] == pytest.approx(1.0, abs=1e-13)
    np.testing.assert_allclose(b, inv_t, rtol=0, atol=1e-13)


def pin_order_and_repeats(fn, seed=3, n=11):
    """The final matrix fixes the final inverse and the product of the ratios,
    whatever the order of the moves; moving an electron twice equals moving it
    once to the second position."""
    rng = np.random.default_rng(seed)
    D = well_conditioned(rng, n)
    inv_t = np.linalg.inv(D).T
    cols, u = moves(rng, D, 5)
    b1, r1 = fn(inv_t, u, cols)
    rev = np.arange(5)[::-1]
    b2, r2 = fn(inv_t, u[rev], cols[rev])
    np.testing.assert_allclose(b1, b2, rtol=0, atol=1e-12 * np.abs(b1).max())
    assert np.prod(r1) == pytest.approx(np.prod(r2), rel=1e-12)
    c = cols[0]
    mid = D[c] + rng.normal(0, 0.5, n)
    b3, r3 = fn(inv_t, np.stack([mid, u[0]]), [c, c])
    b4, r4 = fn(inv_t, u[:1], [c])
    np.testing.assert_allclose(b3, b4, rtol=0, atol=1e-12 * np.abs(b4).max())
    assert np.prod(r3) == pytest.approx(r4[0], rel=1e-12)


PINS = (pin_2x2_exact, pin_explicit_inverse, pin_ratios_are_determinant_ratios,
        pin_unmoved_electron, pin_order_and_repeats)


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    pin(slater.sm_update)


# --- planted mistakes: copies of the update, each with one error ----------

def _variant(kind):
    def fn(inv_t, u, cols):
        b = np.array(inv_t, dtype=np.float64, copy=True)
        u = np.atleast_2d(np.asarray(u, dtype=np.float64))
        n = b.shape[0]
        rs = []
        for m, c in enumerate(np.atleast_1d(cols)):
            v = (b.T @ u[m]) if kind == "transposed" else (b @ u[m])
            r = v[c] - 1.0 if kind == "ratio_off_by_one" else v[c]
            rs.append(r)
            old_c = b[c].copy()
            for i in range(n):
                if i == c:
                    b[i] = old_c if kind == "row_not_scaled" else old_c / r
                else:
                    sgn = -1.0 if kind == "sign" else 1.0
                    b[i] = b[i] - sgn * (v[i] / r) * old_c
        return b, np.array(rs)
    return fn


def _reads_new_row(inv_t, u, cols):
    """Row c is overwritten first and the other rows then subtract the new
    row c instead of the old one."""
    b = np.array(inv_t, dtype=np.float64, copy=True)
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    rs = []
    for m, c in enumerate(np.atleast_1d(cols)):
        v = b @ u[m]
        r = v[c]
        rs.append(r)
        b[c] = b[c] / r
        for i in range(b.shape[0]):
            if i != c:
                b[i] = b[i] - (v[i] / r) * b[c]
    return b, np.array(rs)


def _uses_first_ratio(inv_t, u, cols):
    """Every move divided by the ratio against the original inverse (the
    quasi-simultaneous ratio) instead of the current one."""
    b0 = np.array(inv_t, dtype=np.float64)
    b = b0.copy()
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    rs = []
    for m, c in enumerate(np.atleast_1d(cols)):
        v = b @ u[m]
        r = (b0 @ u[m])[c]
        rs.append(r)
        old_c = b[c].copy()
        for i in range(b.shape[0]):
            b[i] = old_c / r if i == c else b[i] - (v[i] / r) * old_c
    return b, np.array(rs)


MUTANTS = {
    "transposed": _variant("transposed"),
    "ratio_off_by_one": _variant("ratio_off_by_one"),
    "row_not_scaled": _variant("row_not_scaled"),
    "sign": _variant("sign"),
    "reads_new_row": _reads_new_row,
    "uses_first_ratio": _uses_first_ratio,
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    caught = []
    for pin in PINS:
        try:
            pin(MUTANTS[name])
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
