"""Pins of the oracle's Monte Carlo steps (oracle/vmc.py) by determinants and
inverses computed with numpy.linalg on the Slater matrices themselves, by
finite differences of the determinant for the kinetic energy, and by the
special cases where quasi-simultaneous and particle-by-particle
updating must coincide."""
import zlib

import numpy as np
import pytest

from oracle import vmc

A = np.array([[6.0, 0.3, 0.0], [0.2, 5.0, 0.4], [0.0, -0.3, 5.5]])
NG = (10, 9, 8)
L = 4


@pytest.fixture(scope="module")
def system(oracle_lib):
    rng = np.random.default_rng(zlib.crc32(b"vmc-oracle"))
    coef = rng.uniform(-1, 1, NG + (L,)).astype(np.float32)
    pos = rng.uniform(0, 1, (2 * L, 3)) @ A
    D = vmc.slater_matrices(A, NG, coef, pos)
    inv_t = np.stack([np.linalg.inv(D[0]).T, np.linalg.inv(D[1]).T])
    return coef, pos, inv_t, rng


def det_pair(coef, pos):
    D = vmc.slater_matrices(A, NG, coef, pos)
    return np.linalg.det(D[0]) * np.linalg.det(D[1])


def test_qs_step_ratios_decisions_and_inverse(system):
    coef, pos, inv_t, rng = system
    eta = rng.normal(0, 0.4, pos.shape)
    uni = rng.uniform(0, 1, 2 * L)
    new_pos, new_inv, acc, ratio, seq, e = vmc.qs_step(A, NG, coef, pos, inv_t, eta, uni)
    d0 = det_pair(coef, pos)
    for g in range(2 * L):
        p = pos.copy()
        p[g] = pos[g] + eta[g]
        assert ratio[g] == pytest.approx(det_pair(coef, p) / d0, rel=1e-9, abs=1e-12)
    np.testing.assert_array_equal(acc, uni < ratio * ratio)
    np.testing.assert_array_equal(new_pos[acc], (pos + eta)[acc])
    np.testing.assert_array_equal(new_pos[~acc], pos[~acc])
    D = vmc.slater_matrices(A, NG, coef, new_pos)
    for s in range(2):
        want = np.linalg.inv(D[s]).T
        np.testing.assert_allclose(new_inv[s], want, rtol=0, atol=1e-9 * np.abs(want).max())
    # the sequential ratios multiply to the change of the determinants
    prod = np.prod(seq[0]) * np.prod(seq[1])
    assert prod == pytest.approx(det_pair(coef, new_pos) / d0, rel=1e-9)


def test_qs_step_all_rejected_and_all_accepted(system):
    coef, pos, inv_t, rng = system
    eta = rng.normal(0, 0.3, pos.shape)
    p1, b1, a1, _, _, _ = vmc.qs_step(A, NG, coef, pos, inv_t, eta, np.full(2 * L, np.inf))
    assert not a1.any()
    np.testing.assert_array_equal(p1, pos)
    np.testing.assert_allclose(b1, inv_t, rtol=0, atol=0)
    p2, b2, a2, _, _, _ = vmc.qs_step(A, NG, coef, pos, inv_t, eta, np.zeros(2 * L))
    assert a2.all()
    D = vmc.slater_matrices(A, NG, coef, pos + eta)
    for s in range(2):
        want = np.linalg.inv(D[s]).T
        np.testing.assert_allclose(b2[s], want, rtol=0, atol=1e-8 * np.abs(want).max())


def test_local_kinetic_by_finite_differences(system):
    """-1/2 sum_j lap_j Psi / Psi by central finite differences of the
    product of the two determinants (numpy.linalg.det)."""
    coef, pos, inv_t, _ = system
    e = vmc.local_kinetic(A, NG, coef, pos, inv_t)
    h = 1e-3
    psi0 = det_pair(coef, pos)
    lap = 0.0
    for g in range(2 * L):
        for c in range(3):
            p = pos.copy()
            p[g, c] += h
            fp = det_pair(coef, p)
            p[g, c] -= 2 * h
            fm = det_pair(coef, p)
            lap += (fp - 2 * psi0 + fm) / (h * h)
    assert e == pytest.approx(-0.5 * lap / psi0, rel=2e-4, abs=1e-6 * abs(lap / psi0))


def test_single_moving_electron_qs_equals_pbp(system):
    """With only electron 5 proposing a move, both schemes make the same
    decision and reach the same state."""
    coef, pos, inv_t, rng = system
    eta = np.zeros(pos.shape)
    eta[5] = rng.normal(0, 0.5, 3)
    for u in (0.0, 1.0, 0.37):
        uni = np.full(2 * L, np.inf)   # the others are never accepted (and do not move)
        uni[5] = u
        q = vmc.qs_step(A, NG, coef, pos, inv_t, eta, uni)
        b = vmc.pbp_sweep(A, NG, coef, pos, inv_t, eta, uni)
        np.testing.assert_array_equal(q[2], b[2])
        np.testing.assert_array_equal(q[0], b[0])
        np.testing.assert_allclose(q[1], b[1], rtol=0, atol=1e-12 * np.abs(b[1]).max())
        assert q[5] == pytest.approx(b[3], rel=1e-12)


def test_pbp_sweep_judges_against_the_updated_configuration(system):
    """Every decision of a sweep uses the ratio against the configuration
    holding the earlier decisions: replay it with numpy determinants."""
    coef, pos, inv_t, rng = system
    eta = rng.normal(0, 0.4, pos.shape)
    uni = rng.uniform(0, 1, 2 * L)
    new_pos, new_inv, acc, _ = vmc.pbp_sweep(A, NG, coef, pos, inv_t, eta, uni)
    cur = pos.copy()
    for g in range(2 * L):
        trial = cur.copy()
        trial[g] = cur[g] + eta[g]
        r = det_pair(coef, trial) / det_pair(coef, cur)
        assert acc[g] == (uni[g] < r * r), g
        if acc[g]:
            cur = trial
    np.testing.assert_array_equal(new_pos, cur)
