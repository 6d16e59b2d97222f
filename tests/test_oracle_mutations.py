"""Planted mistakes in the oracle are caught by its pins (CPU only).

Each mutation is a plausible slip -- a dropped term, a wrong sign or index,
a transposed operand -- applied to a temporary copy of oracle/blip_oracle.c.
The copy is compiled and run through a battery of the same kinds of pins as
tests/test_oracle_pins.py (textbook spline values, stencil identities, brute
force over every site, finite differences, translation and Bloch relations);
at least one pin must fail for every mutation, and all must pass for the
unmodified source.
"""
import math
import os
import shutil
import tempfile

import numpy as np
import pytest

import oracle
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "blip_oracle.c")
SKEW = np.array([[5.0, 0.3, 0.1], [0.2, 4.5, 0.4], [0.1, -0.3, 6.0]])

MUTATIONS = [
    ("phi inner cubic coefficient", "0.5 * ax * ax * ax", "0.25 * ax * ax * ax"),
    ("phi' outer sign", "return -sg * 0.5 * q * q;", "return sg * 0.5 * q * q;"),
    ("phi'' inner slope", "return -2.0 + 3.0 * ax;", "return -2.0 + 2.0 * ax;"),
    ("stencil offset by one", "double x = f[d] + 1.0 - (double)m[d];",
     "double x = f[d] - (double)m[d];"),
    ("metric transposed", "M[c * 3 + d] = (double)n[d] * G[c * 3 + d];",
     "M[c * 3 + d] = (double)n[d] * G[d * 3 + c];"),
    ("mixed second derivative dropped", "h[1] = h[3] = dp[0] * dp[1] * p[2];",
     "h[1] = h[3] = 0.0;"),
    ("wrong site index", "+ pmod(i0[2] - 1 + m3, n[2]);", "+ pmod(i0[2] - 1 + m2, n[2]);"),
    ("wrap by truncation", "u = u - floor(u);", "u = u - trunc(u);"),
    ("Bloch Laplacian cross-term sign", "double lr = lap[2 * l] - 2.0 * kgi - k2 * ur;",
     "double lr = lap[2 * l] + 2.0 * kgi - k2 * ur;"),
    ("Bloch phase sign", "double cr = cos(kr), ci = sin(kr);",
     "double cr = cos(kr), ci = -sin(kr);"),
    ("cofactor typo", "G[4] = (A[0] * A[8] - A[2] * A[6]) / det;",
     "G[4] = (A[0] * A[8] - A[2] * A[7]) / det;"),
    ("gradient uses the wrong factor", "dt[1] = p[0] * dp[1] * p[2];",
     "dt[1] = p[0] * p[1] * dp[2];"),
    ("Laplacian metric diagonal only", "for (e = 0; e < 3; ++e) lth += g[d * 3 + e] * h[d * 3 + e];",
     "lth += g[d * 3 + d] * h[d * 3 + d];"),
]


def _rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / den if den > 0 else np.max(np.abs(a - b))


def battery(orc):
    """Run the pins against an Oracle; returns the names of the failing ones."""
    fails = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            fails.append(name)

    rows = np.loadtxt(os.path.join(HERE, "golden", "bspline3_values.txt"))
    check("golden", lambda: all(
        abs(orc.phi(x, 0) - a / b) < 1e-15 and abs(orc.phi(x, 1) - c / d) < 1e-15
        and abs(orc.phi(x, 2) - e / f) < 1e-15 for x, a, b, c, d, e, f in rows))
    def wrap_ok():
        Aw, nw = np.diag([16.0, 16.0, 8.0]), (16, 16, 8)
        for r, want in (([3.0, 0.0, 7.5], [3, 0, 7]), ([-0.5, -17.0, -0.25], [15, 15, 7]),
                        ([-1e-18, 35.25, -8.0], [0, 3, 0])):
            i0, f, ok = orc.wrap(Aw, nw, r)
            if not ok or list(i0) != want or not np.all((f >= 0) & (f < 1)):
                return False
        return True
    check("wrap", wrap_ok)
    rng = np.random.default_rng(0)
    fs = rng.uniform(0, 1, 50)
    m = np.arange(4)
    xx = fs[:, None] + 1.0 - m[None, :]
    check("stencil", lambda: np.allclose(orc.phi(xx, 0).sum(1), 1.0, atol=1e-14)
          and np.allclose(orc.phi(xx, 1).sum(1), 0.0, atol=1e-14)
          and np.allclose(((m - 1.0) * orc.phi(xx, 1)).sum(1), 1.0, atol=1e-14))
    for label, A, n, cplx, k in (("ortho", np.diag([4.0, 5.5, 6.0]), (4, 5, 6), False, None),
                                 ("skew", SKEW, (4, 5, 6), False, None),
                                 ("skew-k", SKEW, (4, 5, 6), True, np.array([0.31, -0.17, 0.52]))):
        c = rng.uniform(-1, 1, n + (3,))
        if cplx:
            c = c + 1j * rng.uniform(-1, 1, n + (3,))
        pos = rng.uniform(-9, 14, (10, 3))

        def bf(A=A, n=n, c=c, pos=pos, k=k):
            o = orc.evaluate(A, n, c, pos, kvec=k)
            b = brute.evaluate(A, n, c, pos, kvec=k)
            return all(_rel(o[q], b[q]) < 1e-12 for q in o)
        check(f"brute-{label}", bf)
    A, n = SKEW, (9, 8, 11)
    c = rng.uniform(-1, 1, n + (2,))
    pos = rng.uniform(0, 5, (10, 3))

    def fd():
        h = 1e-4
        o = orc.evaluate(A, n, c, pos)
        g = np.zeros_like(o["grad"])
        lp = np.zeros_like(o["lap"])
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            op, om = orc.evaluate(A, n, c, pos + e), orc.evaluate(A, n, c, pos - e)
            g[:, d] = (op["val"] - om["val"]) / (2 * h)
            lp += (op["grad"][:, d] - om["grad"][:, d]) / (2 * h)
        return _rel(o["grad"], g) < 1e-6 and _rel(o["lap"], lp) < 1e-5
    check("finite-differences", fd)

    def shift():
        o = orc.evaluate(A, n, c, pos)
        T = np.array([2.0, -1.0, 3.0]) @ A
        ot = orc.evaluate(A, n, c, pos + T)
        return all(_rel(ot[q], o[q]) < 1e-12 for q in o)
    check("translation", shift)

    def bloch():
        Ab, nb = np.diag([6.0, 6.0, 4.0]), (6, 6, 4)
        cb = rng.standard_normal(nb + (2,)) + 1j * rng.standard_normal(nb + (2,))
        k = np.array([math.pi / 6, math.pi / 6, math.pi / 4])
        p = rng.uniform(0, 4, (8, 3))
        o = orc.evaluate(Ab, nb, cb, p, kvec=k)
        T = np.array([1.0, 1.0, 2.0]) @ Ab
        ot = orc.evaluate(Ab, nb, cb, p + T, kvec=k)
        ph = np.exp(1j * (k @ T))
        g = orc.evaluate(Ab, nb, cb, p)
        return (all(_rel(ot[q], ph * o[q]) < 1e-12 for q in o)
                and _rel(o["val"], np.exp(1j * (p @ k))[:, None] * g["val"]) < 1e-13)
    check("bloch", bloch)
    return fails


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _variant(workdir, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique or missing: {old}"
    path = os.path.join(workdir, name.replace(" ", "_").replace("'", "p") + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = oracle.build(path, path[:-2] + ".so")
    return oracle.load_variant(lib)


def test_unmodified_oracle_passes_the_battery():
    assert battery(oracle._oracle()) == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(workdir, name, old, new):
    fails = battery(_variant(workdir, name, old, new))
    assert fails, f"mutation '{name}' passed every pin"
