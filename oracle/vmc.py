"""FP64 variational Monte Carlo steps on a synthetic blip Slater determinant
-- TEST INFRASTRUCTURE ONLY (same rules as the rest of :mod:`oracle`).

The trial function is the Slater part of Eq. (6), two determinants of Eq. (5)
(one per spin) of the same L real blip orbitals, with n = L electrons per
spin; the Jastrow factor is left out, so p(R) = |Psi_D(R)|^2.  Each step
follows the sequence of Sec. II.B: a trial move, the probability ratio, the
accept/reject decision, then the local energy (here the kinetic part,
-1/2 sum_j lap_j Psi / Psi, the synthetic system having no potential).

* :func:`qs_step` -- quasi-simultaneous updating (Sec. IV.A, Eq.
  (11.12.23.1)): every electron proposes a move; each is judged against the
  *old* configuration; the accepted ones are then applied, the inverse
  Slater matrices brought up to date one accepted electron at a time in
  electron order (Sec. VI.D).
* :func:`pbp_sweep` -- the particle-by-particle (sequential) updating the
  paper compares with (Eq. (11.12.23.0b)): the same proposals, applied one
  electron at a time, each judged against the configuration holding all
  earlier decisions.

Random numbers are inputs: eta[j] (Gaussian displacements, bohr) and
uniform[j] in [0, 1).  A move is accepted when uniform < ratio^2.

State for one walker: pos [2n, 3] (electrons 0..n-1 spin up, n..2n-1 spin
down), inv_t [2, n, n] transposed inverses (row j of inv_t[s] = column j of
D_s^{-1}, D_s[j, l] = psi_l(r_j) for the electrons of spin s).
"""
from __future__ import annotations

import numpy as np

from . import evaluate
from .slater import sm_update


def slater_matrices(lattice, n_grid, coef, pos):
    """D_s[j, l] = psi_l(r_j) for both spins, FP64 [2, n, n]."""
    val = evaluate(lattice, n_grid, coef, pos, want=("val",))["val"]
    ne = pos.shape[0] // 2
    return np.stack([val[:ne], val[ne:]])


def local_kinetic(lattice, n_grid, coef, pos, inv_t):
    """-1/2 sum_j (lap_j Psi_D)/Psi_D: for electron j of spin s,
    lap_j det(D_s)/det(D_s) = sum_l lap psi_l(r_j) Dinv_s[l, j]."""
    o = evaluate(lattice, n_grid, coef, pos, want=("val", "grad", "lap"))
    ne = pos.shape[0] // 2
    lap = o["lap"]
    s = np.einsum("jl,jl->", lap[:ne], inv_t[0]) + np.einsum("jl,jl->", lap[ne:], inv_t[1])
    return -0.5 * s


def qs_step(lattice, n_grid, coef, pos, inv_t, eta, uniform):
    """One quasi-simultaneous step.  Returns (new pos, new inv_t, accepted
    mask [2n], quasi-simultaneous ratios [2n], sequential ratios per spin
    (list of 2 arrays), local kinetic energy at the new configuration)."""
    pos = np.asarray(pos, dtype=np.float64)
    ne = pos.shape[0] // 2
    trial = pos + eta
    # ratios of every trial move against the old configuration
    val = evaluate(lattice, n_grid, coef, trial, want=("val",))["val"]
    ratio = np.empty(2 * ne)
    for s in range(2):
        for j in range(ne):
            ratio[s * ne + j] = val[s * ne + j] @ inv_t[s][j]
    accept = uniform < ratio * ratio
    new_pos = pos.copy()
    new_pos[accept] = trial[accept]
    new_inv = []
    seq = []
    for s in range(2):
        cols = np.nonzero(accept[s * ne:(s + 1) * ne])[0]
        b, r = sm_update(inv_t[s], val[s * ne + cols], cols)
        new_inv.append(b)
        seq.append(r)
    new_inv = np.stack(new_inv)
    e = local_kinetic(lattice, n_grid, coef, new_pos, new_inv)
    return new_pos, new_inv, accept, ratio, seq, e


def pbp_sweep(lattice, n_grid, coef, pos, inv_t, eta, uniform):
    """One sweep of single-electron moves in electron order: electron j's
    proposal is judged against the configuration that already holds the
    decisions for electrons 0..j-1.  Returns (new pos, new inv_t, accepted
    mask [2n], local kinetic energy after the sweep)."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    inv = np.array(inv_t, dtype=np.float64, copy=True)
    ne = pos.shape[0] // 2
    accept = np.zeros(2 * ne, dtype=bool)
    for g in range(2 * ne):
        s, j = divmod(g, ne)
        trial = pos[g] + eta[g]
        u = evaluate(lattice, n_grid, coef, trial[None, :], want=("val",))["val"][0]
        r = u @ inv[s][j]
        if uniform[g] < r * r:
            accept[g] = True
            pos[g] = trial
            inv[s], _ = sm_update(inv[s], u[None, :], [j])
    e = local_kinetic(lattice, n_grid, coef, pos, inv)
    return pos, inv, accept, e
