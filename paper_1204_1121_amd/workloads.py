"""Seeded synthetic workloads shaped like the paper's benchmark systems.

This module only draws random numbers.  It holds none of the method's
arithmetic (no wrapping, no spline weights, no sums) and is the single place
both the GPU path and the FP64 oracle get their inputs from.

The paper's systems (Si and TiO2 supercells, Sec. II.C and Table
"system_size") need CASINO inputs and DFT orbitals that are not available;
these generators stand in for them with the same shapes: S ~ 250,000 grid
sites, N = 1,536 electrons, L = 768 real (or 384 complex) orbitals.

Every generator uses NumPy's PCG64 with seed 12041121 + config index.
Coefficients are drawn first, in C order [n1][n2][n3][L]; positions after.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SEED_BASE = 12041121


@dataclass
class TableSpec:
    """A periodic blip table: lattice rows (bohr), grid, orbitals, k-point."""
    name: str
    lattice: np.ndarray                 # [3, 3] rows a_1, a_2, a_3
    n: tuple                            # (n1, n2, n3)
    norb: int
    complex_: bool = False
    kvec: np.ndarray | None = None
    seed: int = SEED_BASE

    @property
    def sites(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


# ---------------------------------------------------------------------------
# Table specifications


def spec_small() -> TableSpec:
    """Cubic 10 bohr cell, 16^3 grid, 8 real orbitals (oracle-sized case)."""
    return TableSpec("cubic10_16cubed_L8", np.diag([10.0, 10.0, 10.0]),
                     (16, 16, 16), 8, seed=SEED_BASE + 0)


def spec_tio2() -> TableSpec:
    """TiO2-supercell-shaped table: 18x18x12 bohr, 72x72x48 grid, 768 orbitals."""
    return TableSpec("tio2_72x72x48_L768", np.diag([18.0, 18.0, 12.0]),
                     (72, 72, 48), 768, seed=SEED_BASE + 1)


def spec_tio2_complex() -> TableSpec:
    """The TiO2 geometry with 384 complex orbitals at k = half of each b_d."""
    k = np.array([math.pi / 18.0, math.pi / 18.0, math.pi / 12.0])
    return TableSpec("tio2_72x72x48_L384c", np.diag([18.0, 18.0, 12.0]),
                     (72, 72, 48), 384, complex_=True, kvec=k,
                     seed=SEED_BASE + 3)


def spec_serving():
    """The three resident systems of the serving workload (grid spacing 0.25 bohr)."""
    a = spec_tio2()
    a = TableSpec("tio2_72x72x48_L768", a.lattice, a.n, a.norb, seed=SEED_BASE + 4)
    b = TableSpec("cubic12_48cubed_L256", np.diag([12.0, 12.0, 12.0]),
                  (48, 48, 48), 256, seed=SEED_BASE + 40)
    c = TableSpec("cell24x24x16_96x96x64_L1024", np.diag([24.0, 24.0, 16.0]),
                  (96, 96, 64), 1024, seed=SEED_BASE + 41)
    return [a, b, c]


# ---------------------------------------------------------------------------
# Coefficients


def coefficients(spec: TableSpec, dist: str = "normal") -> np.ndarray:
    """The coefficient table a[i1, i2, i3, l] for a spec.

    dist="uniform": U[-1, 1] float64 (the small oracle case).
    dist="normal":  N(0, 1)/sqrt(S) float32 (complex64 with independent
                    real and imaginary parts for complex specs), drawn one
                    i1-slab at a time so no float64 copy is ever held.
    """
    rng = np.random.default_rng(spec.seed)
    n1, n2, n3 = spec.n
    L = spec.norb
    if dist == "uniform":
        shape = (n1, n2, n3, L, 2) if spec.complex_ else (n1, n2, n3, L)
        a = rng.uniform(-1.0, 1.0, size=shape)
        if spec.complex_:
            a = a[..., 0] + 1j * a[..., 1]
        return a
    scale = np.float32(1.0 / math.sqrt(spec.sites))
    if spec.complex_:
        out = np.empty((n1, n2, n3, L), dtype=np.complex64)
        fv = out.view(np.float32).reshape(n1, n2, n3, L, 2)
        for i in range(n1):
            fv[i] = rng.standard_normal((n2, n3, L, 2), dtype=np.float32) * scale
        return out
    out = np.empty((n1, n2, n3, L), dtype=np.float32)
    for i in range(n1):
        out[i] = rng.standard_normal((n2, n3, L), dtype=np.float32) * scale
    return out


# ---------------------------------------------------------------------------
# Positions


def uniform_positions(spec: TableSpec, npos: int, seed) -> np.ndarray:
    """npos points uniform in the cell (fractional U[0,1)^3 times the lattice)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=(npos, 3))
    return u @ spec.lattice


def move_block(spec: TableSpec, npos: int, block: int = 0,
               sigma: float = 0.5) -> np.ndarray:
    """A quasi-simultaneous move block (Eq. (11.12.23.2)): npos electron sites
    uniform in the cell, each displaced by N(0, sigma^2) per component.

    The result is *not* wrapped into the cell.  ``block`` selects an
    independent configuration (a different walker).
    """
    rng = np.random.default_rng([spec.seed, 1, block])
    sites = rng.uniform(0.0, 1.0, size=(npos, 3)) @ spec.lattice
    return sites + rng.normal(0.0, sigma, size=(npos, 3))


@dataclass
class WalkerBatch:
    """Ragged per-walker move blocks, concatenated, with offsets[nw+1]."""
    pos: np.ndarray
    offsets: np.ndarray
    sizes: np.ndarray = field(default=None)


def walker_batch(spec: TableSpec, nwalkers: int = 512, max_block: int = 256,
                 batch: int = 0, sigma: float = 0.5) -> WalkerBatch:
    """nwalkers walkers, each with a move block of size U[1, max_block]."""
    rng = np.random.default_rng([spec.seed, 2, batch])
    sizes = rng.integers(1, max_block + 1, size=nwalkers)
    offsets = np.zeros(nwalkers + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    sites = rng.uniform(0.0, 1.0, size=(total, 3)) @ spec.lattice
    pos = sites + rng.normal(0.0, sigma, size=(total, 3))
    return WalkerBatch(pos=pos, offsets=offsets, sizes=sizes)


@dataclass
class Request:
    rid: int
    system: int
    arrival: float          # scheduled arrival time, seconds from start
    pos: np.ndarray


def serving_requests(nsys: int, nreq: int, rate: float, specs, seed: int = 0,
                     max_pos: int = 1536, sigma: float = 0.5):
    """Poisson arrivals at ``rate`` req/s; each request picks a system
    uniformly and brings round(exp(U(0, ln max_pos))) positions."""
    rng = np.random.default_rng([SEED_BASE + 4, 3, seed])
    gaps = rng.exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps)
    out = []
    for i in range(nreq):
        s = int(rng.integers(0, nsys))
        k = int(np.rint(math.exp(rng.uniform(0.0, math.log(max_pos)))))
        k = max(1, min(max_pos, k))
        sp = specs[s]
        p = rng.uniform(0.0, 1.0, size=(k, 3)) @ sp.lattice
        p = p + rng.normal(0.0, sigma, size=(k, 3))
        out.append(Request(i, s, float(t[i]), p))
    return out
