"""Pins of the FP64 oracle against facts fixed by the mathematics.

The paper prints no worked orbital values, so the oracle is pinned by:
  * textbook values of the cubic B-spline (tests/golden/bspline3_values.txt);
  * identities of the 4-point stencil (partition of unity, polynomial
    reproduction) that any slip in a weight, sign or offset breaks;
  * closed forms in 3-D: node stencils, constant / linear / quadratic /
    bilinear coefficient fields through a skewed lattice (pins the metric
    M = n G and g = M^T M including mixed second derivatives);
  * a separable field against scipy's BSpline (a library routine);
  * brute force over every coefficient and its periodic images
    (oracle.brute, truncated-power spline) on tiny grids;
  * finite differences (gradient vs value, Laplacian vs gradient);
  * lattice-translation invariance and the Bloch relation at a k-point.
"""
import math
import os
import zlib

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

SKEW = np.array([[5.0, 0.3, 0.1], [0.2, 4.5, 0.4], [0.1, -0.3, 6.0]])


def _rel(a, b):
    """Normwise relative error max|a-b| / max|b| (absolute if b == 0)."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    num = np.max(np.abs(a - b))
    return num / den if den > 0 else num


# ---------------------------------------------------------------------------
# 1-D basis


def test_phi_golden_values(oracle_lib):
    rows = np.loadtxt(os.path.join(HERE, "golden", "bspline3_values.txt"))
    for x, pn, pd, dn, dd, sn, sd in rows:
        assert oracle_lib.phi(x, 0) == pytest.approx(pn / pd, abs=1e-15)
        assert oracle_lib.phi(x, 1) == pytest.approx(dn / dd, abs=1e-15)
        assert oracle_lib.phi(x, 2) == pytest.approx(sn / sd, abs=1e-15)


def test_phi_stencil_identities(oracle_lib):
    """For the 4 sites i0-1..i0+2 (x = f+1-m): sum w = 1, sum w' = 0,
    sum w'' = 0; sum (m-1) w = f; sum (m-1)^2 w = f^2 + 1/3;
    sum (m-1) w' = 1; sum (m-1)^2 w'' = 2."""
    f = np.random.default_rng(0).uniform(0.0, 1.0, 200)
    f = np.concatenate([f, [0.0, 0.5, 1.0 - 2.0 ** -52]])
    m = np.arange(4)
    x = f[:, None] + 1.0 - m[None, :]
    w = oracle_lib.phi(x, 0)
    w1 = oracle_lib.phi(x, 1)
    w2 = oracle_lib.phi(x, 2)
    k = (m - 1.0)[None, :]
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-15)
    np.testing.assert_allclose(w1.sum(1), 0.0, atol=1e-15)
    np.testing.assert_allclose(w2.sum(1), 0.0, atol=1e-14)
    np.testing.assert_allclose((k * w).sum(1), f, atol=1e-15)
    np.testing.assert_allclose((k * k * w).sum(1), f * f + 1.0 / 3.0, atol=1e-15)
    np.testing.assert_allclose((k * w1).sum(1), 1.0, atol=1e-15)
    np.testing.assert_allclose((k * k * w2).sum(1), 2.0, atol=1e-14)
    # support: the fifth site on either side is exactly zero
    assert np.all(oracle_lib.phi(f + 2.0, 0) == 0.0)
    assert np.all(oracle_lib.phi(f - 3.0, 0) == 0.0)


def test_phi_derivatives_by_finite_difference(oracle_lib):
    x = np.random.default_rng(1).uniform(-2.2, 2.2, 300)
    x = x[np.min(np.abs(x[:, None] - np.arange(-2, 3)[None, :]), axis=1) > 1e-3]
    h = 1e-6
    d1 = (oracle_lib.phi(x + h) - oracle_lib.phi(x - h)) / (2 * h)
    np.testing.assert_allclose(oracle_lib.phi(x, 1), d1, atol=1e-8)
    d2 = (oracle_lib.phi(x + h, 1) - oracle_lib.phi(x - h, 1)) / (2 * h)
    np.testing.assert_allclose(oracle_lib.phi(x, 2), d2, atol=1e-8)


def test_inverse3_against_numpy(oracle_lib):
    rng = np.random.default_rng(2)
    for _ in range(20):
        A = rng.normal(size=(3, 3)) + 3 * np.eye(3)
        np.testing.assert_allclose(oracle_lib.inverse3(A), np.linalg.inv(A),
                                   rtol=1e-12, atol=1e-14)
    with pytest.raises(ValueError):
        oracle_lib.inverse3(np.zeros((3, 3)))


# ---------------------------------------------------------------------------
# Wrap and site selection (Eq. (7))


def test_wrap_cases(oracle_lib):
    A = np.diag([16.0, 16.0, 8.0])          # power-of-two cell: u exact
    n = (16, 16, 8)
    i0, f, ok = oracle_lib.wrap(A, n, [3.0, 0.0, 7.5])
    assert ok and list(i0) == [3, 0, 7] and np.allclose(f, [0, 0, 0.5])
    i0, f, ok = oracle_lib.wrap(A, n, [-0.0, 16.0, -8.0])   # -0 and faces
    assert ok and list(i0) == [0, 0, 0] and np.all(f == 0.0)
    i0, f, ok = oracle_lib.wrap(A, n, [-1e-18, 35.25, -0.5])
    # -1e-18/16 - floor(..) rounds to 1.0 -> 0;  35.25 = 2*16 + 3.25
    assert ok and list(i0) == [0, 3, 7] and np.allclose(f, [0, 0.25, 0.5])
    i0, f, ok = oracle_lib.wrap(A, n, [1e300, -1e300, 3.0])
    assert ok and i0[2] == 3 and np.all((f >= 0) & (f < 1))
    for bad in ([np.nan, 0, 0], [0, np.inf, 0], [0, 0, -np.inf]):
        _, _, ok = oracle_lib.wrap(A, n, bad)
        assert not ok


def test_nonfinite_positions_give_nan_rows(oracle_lib):
    A = np.diag([10.0, 10.0, 10.0])
    c = np.random.default_rng(3).uniform(-1, 1, (6, 6, 6, 3))
    pos = np.array([[1.0, 2.0, 3.0], [np.nan, 1.0, 1.0], [1.0, np.inf, 1.0]])
    o = oracle_lib.evaluate(A, (6, 6, 6), c, pos)
    for k in ("val", "grad", "lap"):
        assert np.all(np.isfinite(o[k][0]))
        assert np.all(np.isnan(o[k][1])) and np.all(np.isnan(o[k][2]))


# ---------------------------------------------------------------------------
# 3-D closed forms


def test_node_stencils(oracle_lib):
    """At a grid node (f = 0): value stencil [1,4,1]/6, first-derivative
    stencil [-1,0,1]/2 and second-derivative stencil [1,-2,1] in each
    direction, scaled by n_d/L_d per derivative (orthorhombic cell)."""
    A = np.diag([8.0, 4.0, 16.0])
    n = (8, 8, 8)
    c = np.random.default_rng(4).uniform(-1, 1, (8, 8, 8, 2))
    s0 = np.array([1.0, 4.0, 1.0]) / 6.0
    s1 = np.array([-1.0, 0.0, 1.0]) / 2.0
    s2 = np.array([1.0, -2.0, 1.0])
    scale = np.array([8 / 8.0, 8 / 4.0, 8 / 16.0])
    nodes = [(0, 0, 0), (3, 7, 5), (7, 1, 0)]
    pos = np.array([[i * 8.0 / 8, j * 4.0 / 8, k * 16.0 / 8] for i, j, k in nodes])
    o = oracle_lib.evaluate(A, n, c, pos)
    for p, (i, j, k) in enumerate(nodes):
        blk = np.empty((3, 3, 3, 2))
        for a in range(3):
            for b in range(3):
                for cc in range(3):
                    blk[a, b, cc] = c[(i + a - 1) % 8, (j + b - 1) % 8, (k + cc - 1) % 8]
        val = np.einsum("a,b,c,abcl->l", s0, s0, s0, blk)
        gx = np.einsum("a,b,c,abcl->l", s1, s0, s0, blk) * scale[0]
        gy = np.einsum("a,b,c,abcl->l", s0, s1, s0, blk) * scale[1]
        gz = np.einsum("a,b,c,abcl->l", s0, s0, s1, blk) * scale[2]
        lap = (np.einsum("a,b,c,abcl->l", s2, s0, s0, blk) * scale[0] ** 2
               + np.einsum("a,b,c,abcl->l", s0, s2, s0, blk) * scale[1] ** 2
               + np.einsum("a,b,c,abcl->l", s0, s0, s2, blk) * scale[2] ** 2)
        np.testing.assert_allclose(o["val"][p], val, atol=1e-14)
        np.testing.assert_allclose(o["grad"][p], np.stack([gx, gy, gz]), atol=1e-14)
        np.testing.assert_allclose(o["lap"][p], lap, atol=1e-13)


def test_constant_field(oracle_lib):
    rng = np.random.default_rng(5)
    c = np.full((5, 6, 7, 3), 1.0)
    c[..., 1] = -2.5
    c[..., 2] = 0.125
    pos = rng.uniform(-20, 20, (40, 3))
    o = oracle_lib.evaluate(SKEW, (5, 6, 7), c, pos)
    np.testing.assert_allclose(o["val"], np.broadcast_to(c[0, 0, 0], (40, 3)), atol=1e-14)
    np.testing.assert_allclose(o["grad"], 0.0, atol=1e-13)
    np.testing.assert_allclose(o["lap"], 0.0, atol=1e-12)


def _interior_positions(A, n, count, seed, margin=2.0):
    """Positions whose stencil stays inside 0..n-1 without wrapping."""
    rng = np.random.default_rng(seed)
    n = np.asarray(n, dtype=float)
    t = rng.uniform(margin, n - margin - 1.0, (count, 3))
    return (t / n) @ A, t


def test_polynomial_fields_pin_metric(oracle_lib):
    """c = i_d  -> psi = t_d, grad psi = M[:, d], lap = 0
       c = i_d^2 -> psi = t_d^2 + 1/3, lap = 2 g_dd
       c = i_d i_e (d != e) -> psi = t_d t_e, lap = 2 g_de
    with M = n_d (A^{-1})_{cd} from numpy and g = M^T M (skewed cell)."""
    n = (12, 13, 14)
    A = SKEW
    M = np.linalg.inv(A) * np.asarray(n, dtype=float)[None, :]
    g = M.T @ M
    pos, t = _interior_positions(A, n, 25, 6)
    idx = np.stack(np.meshgrid(*[np.arange(v, dtype=float) for v in n],
                               indexing="ij"), axis=-1)
    fields, vals, grads, laps = [], [], [], []
    for d in range(3):
        fields.append(idx[..., d])
        vals.append(t[:, d])
        grads.append(np.broadcast_to(M[:, d], (25, 3)))
        laps.append(np.zeros(25))
        fields.append(idx[..., d] ** 2)
        vals.append(t[:, d] ** 2 + 1.0 / 3.0)
        grads.append(2.0 * t[:, d][:, None] * M[:, d][None, :])
        laps.append(np.full(25, 2.0 * g[d, d]))
    for d, e in ((0, 1), (0, 2), (1, 2)):
        fields.append(idx[..., d] * idx[..., e])
        vals.append(t[:, d] * t[:, e])
        grads.append(t[:, e][:, None] * M[:, d][None, :] + t[:, d][:, None] * M[:, e][None, :])
        laps.append(np.full(25, 2.0 * g[d, e]))
    c = np.stack(fields, axis=-1)
    o = oracle_lib.evaluate(A, n, c, pos)
    for l in range(c.shape[-1]):
        np.testing.assert_allclose(o["val"][:, l], vals[l], rtol=1e-12, atol=1e-11)
        np.testing.assert_allclose(o["grad"][:, :, l], grads[l], rtol=1e-12, atol=1e-11)
        np.testing.assert_allclose(o["lap"][:, l], laps[l], rtol=1e-12, atol=1e-11)


def test_separable_field_against_scipy(oracle_lib):
    """c = p(i1) q(i2) r(i3): psi = P(t1) Q(t2) R(t3) with each factor a
    periodic cubic spline evaluated by scipy.interpolate.BSpline."""
    from scipy.interpolate import BSpline
    rng = np.random.default_rng(7)
    n = (7, 9, 6)
    Ls = np.array([7.0, 4.5, 3.0])
    A = np.diag(Ls)
    p = [rng.uniform(-1, 1, v) for v in n]
    c = np.einsum("i,j,k->ijk", *p)[..., None]
    pos = rng.uniform(-10, 10, (30, 3))
    o = oracle_lib.evaluate(A, n, c, pos)

    def factor(d, tt, der):
        nd = n[d]
        # B-spline with knots j..j+4 is centred at j+2: coefficient of the
        # basis centred at integer i is p[i mod n]; cover t in [-3, nd+3].
        ii = np.arange(-4, nd + 5)
        knots = np.arange(ii[0] - 2, ii[-1] + 3, dtype=float)
        spl = BSpline(knots, p[d][ii % nd], 3, extrapolate=False)
        if der:
            spl = spl.derivative(der)
        return spl(tt)

    t = np.mod(pos / Ls, 1.0) * np.asarray(n, float)
    F = [[factor(d, t[:, d], k) for k in range(3)] for d in range(3)]
    sc = np.asarray(n, float) / Ls
    val = F[0][0] * F[1][0] * F[2][0]
    gx = F[0][1] * F[1][0] * F[2][0] * sc[0]
    gy = F[0][0] * F[1][1] * F[2][0] * sc[1]
    gz = F[0][0] * F[1][0] * F[2][1] * sc[2]
    lap = (F[0][2] * F[1][0] * F[2][0] * sc[0] ** 2 + F[0][0] * F[1][2] * F[2][0] * sc[1] ** 2
           + F[0][0] * F[1][0] * F[2][2] * sc[2] ** 2)
    np.testing.assert_allclose(o["val"][:, 0], val, atol=1e-13)
    np.testing.assert_allclose(o["grad"][:, :, 0], np.stack([gx, gy, gz], 1), atol=1e-13)
    np.testing.assert_allclose(o["lap"][:, 0], lap, atol=1e-12)


@pytest.mark.parametrize("case", ["ortho_4x5x6", "cube_5", "skew_4x5x6",
                                  "skew_complex_k", "ortho_complex_gamma"])
def test_brute_force_every_site(oracle_lib, case):
    from oracle import brute
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    if case == "ortho_4x5x6":
        A, n = np.diag([4.0, 5.5, 6.0]), (4, 5, 6)
    elif case == "cube_5":
        A, n = np.diag([3.0, 3.0, 3.0]), (5, 5, 5)
    else:
        A, n = SKEW, (4, 5, 6)
    cplx = "complex" in case
    shape = tuple(n) + (3,)
    c = rng.uniform(-1, 1, shape)
    if cplx:
        c = c + 1j * rng.uniform(-1, 1, shape)
    k = np.array([0.31, -0.17, 0.52]) if case.endswith("_k") else None
    pos = rng.uniform(-12, 15, (16, 3))
    o = oracle_lib.evaluate(A, n, c, pos, kvec=k)
    b = brute.evaluate(A, n, c, pos, kvec=k)
    for key in ("val", "grad", "lap"):
        assert _rel(o[key], b[key]) < 1e-12, key


def test_brute_force_float32_table(oracle_lib):
    """FP32 and complex64 tables are read exactly (widened to FP64)."""
    from oracle import brute
    rng = np.random.default_rng(11)
    A, n = np.diag([4.0, 4.0, 4.0]), (4, 4, 4)
    c = rng.uniform(-1, 1, (4, 4, 4, 5)).astype(np.float32)
    pos = rng.uniform(0, 4, (8, 3))
    o = oracle_lib.evaluate(A, n, c, pos)
    b = brute.evaluate(A, n, c.astype(np.float64), pos)
    assert _rel(o["val"], b["val"]) < 1e-12
    cc = (c + 1j * c[..., ::-1]).astype(np.complex64)
    o = oracle_lib.evaluate(A, n, cc, pos, kvec=[0.1, 0.2, 0.3])
    b = brute.evaluate(A, n, cc.astype(np.complex128), pos, kvec=[0.1, 0.2, 0.3])
    assert _rel(o["lap"], b["lap"]) < 1e-12


# ---------------------------------------------------------------------------
# Derivatives and symmetries


def _away_from_nodes(A, n, pos, gap):
    t = np.mod(pos @ np.linalg.inv(A), 1.0) * np.asarray(n, float)
    fr = t - np.floor(t)
    return np.all(np.minimum(fr, 1.0 - fr) > gap, axis=1)


def test_finite_differences(oracle_lib):
    rng = np.random.default_rng(8)
    A, n = SKEW, (9, 8, 11)
    c = rng.uniform(-1, 1, (9, 8, 11, 4))
    pos = rng.uniform(-5, 10, (60, 3))
    h = 1e-4
    pos = pos[_away_from_nodes(A, n, pos, 0.01)][:30]
    o = oracle_lib.evaluate(A, n, c, pos)
    fd_grad = np.zeros_like(o["grad"])
    fd_lap = np.zeros_like(o["lap"])
    for cdir in range(3):
        e = np.zeros(3)
        e[cdir] = h
        op = oracle_lib.evaluate(A, n, c, pos + e)
        om = oracle_lib.evaluate(A, n, c, pos - e)
        fd_grad[:, cdir] = (op["val"] - om["val"]) / (2 * h)
        fd_lap += (op["grad"][:, cdir] - om["grad"][:, cdir]) / (2 * h)
    assert _rel(o["grad"], fd_grad) < 1e-7
    assert _rel(o["lap"], fd_lap) < 1e-7


def test_lattice_translation_invariance(oracle_lib):
    rng = np.random.default_rng(9)
    A, n = SKEW, (6, 7, 8)
    c = rng.uniform(-1, 1, (6, 7, 8, 3))
    pos = rng.uniform(0, 5, (20, 3))
    o = oracle_lib.evaluate(A, n, c, pos)
    for m in ([1, 0, 0], [0, -2, 0], [3, 1, -1], [-7, 5, 2]):
        T = np.asarray(m, float) @ A
        ot = oracle_lib.evaluate(A, n, c, pos + T)
        for k in ("val", "grad", "lap"):
            assert _rel(ot[k], o[k]) < 1e-12


def test_bloch_relation(oracle_lib):
    """psi(r + T) = exp(i k.T) psi(r) for complex orbitals at a k-point;
    grad and lap transform the same way."""
    rng = np.random.default_rng(10)
    A, n = np.diag([6.0, 6.0, 4.0]), (6, 6, 4)
    c = (rng.standard_normal((6, 6, 4, 3)) + 1j * rng.standard_normal((6, 6, 4, 3)))
    k = np.array([math.pi / 6.0, math.pi / 6.0, math.pi / 4.0])
    pos = rng.uniform(0, 4, (15, 3))
    o = oracle_lib.evaluate(A, n, c, pos, kvec=k)
    for m in ([1, 0, 0], [0, 1, 1], [2, -1, 3]):
        T = np.asarray(m, float) @ A
        ot = oracle_lib.evaluate(A, n, c, pos + T, kvec=k)
        ph = np.exp(1j * (k @ T))
        for key in ("val", "grad", "lap"):
            assert _rel(ot[key], ph * o[key]) < 1e-12
    # the periodic part is the Gamma-point evaluation
    g = oracle_lib.evaluate(A, n, c, pos)
    ph = np.exp(1j * (pos @ k))
    assert _rel(o["val"], ph[:, None] * g["val"]) < 1e-13


def test_positions_are_independent(oracle_lib):
    """Quasi-simultaneous updating evaluates each moved electron against the
    same table independently (Eq. (11.12.23.1)): a block equals its parts."""
    rng = np.random.default_rng(12)
    A, n = SKEW, (5, 6, 7)
    c = rng.uniform(-1, 1, (5, 6, 7, 4))
    pos = rng.uniform(-3, 9, (12, 3))
    o = oracle_lib.evaluate(A, n, c, pos, nthreads=4)
    for j in (0, 5, 11):
        oj = oracle_lib.evaluate(A, n, c, pos[j:j + 1])
        for k in ("val", "grad", "lap"):
            np.testing.assert_array_equal(oj[k][0], o[k][j])


def test_bloch_values_only_equals_full_call(oracle_lib):
    """With a k-point, asking for values only gives exactly the values of the
    full call (the Bloch factor of the value uses the value alone), and a
    gradient without the value is refused."""
    rng = np.random.default_rng(zlib.crc32(b"bloch-values-only"))
    n = (6, 7, 5)
    L = 4
    A = np.array([[5.0, 0.4, 0.0], [0.1, 4.0, 0.3], [0.0, -0.2, 6.0]])
    coef = (rng.uniform(-1, 1, n + (L,)) + 1j * rng.uniform(-1, 1, n + (L,))).astype(np.complex128)
    k = np.array([0.3, -0.2, 0.5])
    pos = rng.uniform(-3, 9, (11, 3))
    full = oracle_lib.evaluate(A, n, coef, pos, kvec=k)
    vo = oracle_lib.evaluate(A, n, coef, pos, kvec=k, want=("val",))
    np.testing.assert_array_equal(vo["val"], full["val"])
    with pytest.raises(ValueError):
        oracle_lib.evaluate(A, n, coef, pos, kvec=k, want=("grad",))
