"""Brute-force blip evaluation over every coefficient -- TEST INFRASTRUCTURE ONLY.

An independent second formulation used to pin the C oracle on tiny grids.
Instead of selecting the 4x4x4 site subset (Eq. (7)) it sums Eq.
(11.12.24.1) over *all* S grid sites and over enough periodic images of each
that every non-zero Theta is included, without wrapping the position.

The cubic B-spline here is written in truncated-power form,
    phi(x) = (1/6) sum_{k=0..4} (-1)^k C(4,k) (x + 2 - k)_+^3,
with derivatives from differentiating the truncated powers; the C oracle
writes it by cases of |x|.  The Jacobian dt/dr comes from numpy.linalg.inv.
"""
from __future__ import annotations

import numpy as np

_BINOM4 = np.array([1.0, -4.0, 6.0, -4.0, 1.0])   # (-1)^k C(4,k)


def _tp(x, p):
    """(x)_+^p elementwise (with (x)_+^0 the unit step)."""
    xp = np.where(x > 0.0, x, 0.0)
    if p == 0:
        return (x > 0.0).astype(np.float64)
    return xp ** p


def bspline3(x, deriv=0):
    """Cardinal cubic B-spline centred at 0, or its first/second derivative."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros_like(x)
    for k in range(5):
        y = x + 2.0 - k
        if deriv == 0:
            acc = acc + _BINOM4[k] * _tp(y, 3) / 6.0
        elif deriv == 1:
            acc = acc + _BINOM4[k] * 3.0 * _tp(y, 2) / 6.0
        else:
            acc = acc + _BINOM4[k] * 6.0 * _tp(y, 1) / 6.0
    # Outside (-2, 2) the truncated powers cancel exactly in real arithmetic;
    # in floating point they leave a residue of order (x+2)^3 eps, so the
    # identically-zero region is set to zero explicitly.
    return np.where(np.abs(x) < 2.0, acc, 0.0)


def evaluate(lattice, n, coef, pos, kvec=None):
    """Value, Cartesian gradient and Laplacian by summing over every site.

    Same argument conventions as :func:`oracle.evaluate`; intended for grids
    of a few hundred sites and a few dozen positions.
    """
    A = np.asarray(lattice, dtype=np.float64).reshape(3, 3)
    n = np.asarray(n, dtype=np.int64)
    coef = np.asarray(coef)
    cplx = np.iscomplexobj(coef)
    c = coef.astype(np.complex128 if cplx else np.float64)
    L = c.shape[3]
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    G = np.linalg.inv(A)
    J = G * n[None, :]            # J[c, d] = d t_d / d r_c
    npos = pos.shape[0]
    val = np.zeros((npos, L), dtype=c.dtype)
    grad = np.zeros((npos, 3, L), dtype=c.dtype)
    lap = np.zeros((npos, L), dtype=c.dtype)
    cflat = c.reshape(-1, L)
    for j in range(npos):
        r = pos[j]
        t = (r @ G) * n           # grid coordinates, not wrapped
        # every grid site i plus periodic images i + k*n with |t - i - k n| < 2
        axes = []
        for d in range(3):
            lo = int(np.floor((t[d] - 2.0) / n[d])) - 1
            hi = int(np.floor((t[d] + 2.0) / n[d])) + 1
            img = np.arange(lo, hi + 1)
            ii = np.arange(n[d])
            # x = t - (i + k n) for all (i, k): shape [n_d, nimg]
            x = t[d] - (ii[:, None] + img[None, :] * n[d])
            axes.append((bspline3(x, 0).sum(axis=1),
                         bspline3(x, 1).sum(axis=1),
                         bspline3(x, 2).sum(axis=1)))
        # tensor products over all sites: [n1, n2, n3]
        P = [ax[0] for ax in axes]
        D = [ax[1] for ax in axes]
        D2 = [ax[2] for ax in axes]

        def outer(a, b, cc):
            return np.einsum("i,j,k->ijk", a, b, cc).reshape(-1)

        theta = outer(P[0], P[1], P[2])
        dth = [outer(D[0], P[1], P[2]), outer(P[0], D[1], P[2]),
               outer(P[0], P[1], D[2])]
        hess = {}
        for d in range(3):
            for e in range(3):
                fac = [P[0], P[1], P[2]]
                if d == e:
                    fac[d] = D2[d]
                else:
                    fac[d] = D[d]
                    fac[e] = D[e]
                hess[(d, e)] = outer(*fac)
        u = theta @ cflat
        du = np.stack([dth[d] @ cflat for d in range(3)])          # [3(t), L]
        gu = J @ du                                                # [3(r), L]
        lu = np.zeros(L, dtype=c.dtype)
        for d in range(3):
            for e in range(3):
                gde = float(J[:, d] @ J[:, e])
                lu = lu + gde * (hess[(d, e)] @ cflat)
        if kvec is not None:
            k = np.asarray(kvec, dtype=np.float64)
            ph = np.exp(1j * float(k @ r))
            val[j] = ph * u
            grad[j] = ph * (gu + 1j * k[:, None] * u[None, :])
            lap[j] = ph * (lu + 2j * (k @ gu) - float(k @ k) * u)
        else:
            val[j], grad[j], lap[j] = u, gu, lu
    return {"val": val, "grad": grad, "lap": lap}
