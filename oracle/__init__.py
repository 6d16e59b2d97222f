"""FP64 CPU oracle for blip orbital evaluation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it; the two meet only at the seeded input generators.

Two independent formulations live here:

* :func:`evaluate` -- the plain definition of Eq. (11.12.24.1)/(11.12.24.2)
  in C (``blip_oracle.c``): wrap, select the 4x4x4 site subset of Eq. (7),
  sum a_{l,s} Theta_s with Theta_s and its derivatives from the cubic
  B-spline written by cases of |x|.
* :mod:`oracle.brute` -- a NumPy brute force over *every* coefficient of a
  tiny grid and its periodic images, with the spline written in
  truncated-power form.  It pins the C oracle.
* :func:`ratio` -- the quasi-simultaneous acceptance ratio of the Slater part,
  the FP64 dot product of the orbitals with a column of the old inverse.
* :mod:`oracle.slater` -- the sequential Sherman-Morrison update of the
  inverse Slater matrix after accepted moves, in NumPy.
* :mod:`oracle.vmc` -- Monte Carlo steps on a synthetic Slater determinant:
  a quasi-simultaneous step and a particle-by-particle sweep.

Inputs are NumPy arrays; outputs are float64 (complex128 for complex tables).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "blip_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_KIND = {np.dtype(np.float64): 0, np.dtype(np.float32): 1,
         np.dtype(np.complex128): 2, np.dtype(np.complex64): 3}

_lib = None


def build(src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compile the C oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    for name in ("oracle_phi", "oracle_dphi", "oracle_d2phi"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_double
        fn.argtypes = [ctypes.c_double]
    lib.oracle_inverse3.restype = ctypes.c_int
    lib.oracle_inverse3.argtypes = [dp, dp]
    lib.oracle_wrap.restype = ctypes.c_int
    lib.oracle_wrap.argtypes = [dp, ip, dp, ip, dp]
    lib.oracle_eval.restype = ctypes.c_int
    lib.oracle_eval.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                dp, dp, ctypes.c_int64, dp, dp, dp,
                                ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """The C oracle bound to one compiled library (the default build, or a
    variant compiled from a modified source by the mutation tests)."""

    def __init__(self, lib):
        self._lib = lib

    def phi(self, x, deriv: int = 0) -> np.ndarray:
        """The 1-D cubic B-spline phi (deriv 0), phi' (1) or phi'' (2)."""
        lib = self._lib
        fn = (lib.oracle_phi, lib.oracle_dphi, lib.oracle_d2phi)[deriv]
        xs = np.asarray(x, dtype=np.float64)
        return np.vectorize(lambda v: fn(float(v)), otypes=[np.float64])(xs)


    def inverse3(self, lattice) -> np.ndarray:
        """A^{-1} by cofactors, as the oracle forms it (raises if singular)."""
        lib = self._lib
        A = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
        G = np.zeros(9)
        if lib.oracle_inverse3(_dptr(A), _dptr(G)) != 0:
            raise ValueError("singular lattice")
        return G.reshape(3, 3)


    def wrap(self, lattice, n, r):
        """Cell index i0 and offset f of position r (the subset selection, Eq. (7))."""
        lib = self._lib
        G = np.ascontiguousarray(self.inverse3(lattice).reshape(9))
        nn = (ctypes.c_int * 3)(*[int(v) for v in n])
        rr = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(3))
        i0 = (ctypes.c_int * 3)()
        f = np.zeros(3)
        rc = lib.oracle_wrap(_dptr(G), nn, _dptr(rr), i0, _dptr(f))
        return np.array(list(i0), dtype=np.int64), f, rc == 0


    def evaluate(self, lattice, n, coef, pos, kvec=None, want=("val", "grad", "lap"),
                 nthreads: int = 1):
        """Orbitals (and gradients, Laplacians) at every position, in FP64.

        lattice: 3x3 rows a_1..a_3 (bohr); n: (n1, n2, n3);
        coef: array [n1, n2, n3, L] of float64/float32/complex128/complex64;
        pos: [npos, 3] Cartesian bohr; kvec: k-point (complex tables only).
        Returns a dict with ``val`` [npos, L], ``grad`` [npos, 3, L] and
        ``lap`` [npos, L] for the requested keys.
        """
        lib = self._lib
        coef = np.ascontiguousarray(coef)
        if coef.dtype not in _KIND:
            raise TypeError(f"unsupported coefficient dtype {coef.dtype}")
        n1, n2, n3 = (int(v) for v in n)
        if coef.ndim != 4 or coef.shape[:3] != (n1, n2, n3):
            raise ValueError("coef must be [n1, n2, n3, L]")
        L = int(coef.shape[3])
        cplx = np.iscomplexobj(coef)
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        npos = pos.shape[0]
        A = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
        odt = np.complex128 if cplx else np.float64
        out = {}
        if "val" in want:
            out["val"] = np.zeros((npos, L), dtype=odt)
        if "grad" in want:
            out["grad"] = np.zeros((npos, 3, L), dtype=odt)
        if "lap" in want:
            out["lap"] = np.zeros((npos, L), dtype=odt)
        k = None
        if kvec is not None:
            k = np.ascontiguousarray(np.asarray(kvec, dtype=np.float64).reshape(3))
        null = ctypes.POINTER(ctypes.c_double)()
        rc = lib.oracle_eval(
            _dptr(A), n1, n2, n3, L, coef.ctypes.data_as(ctypes.c_void_p),
            _KIND[coef.dtype], _dptr(k) if k is not None else null,
            _dptr(pos), npos,
            _dptr(out["val"]) if "val" in out else null,
            _dptr(out["grad"]) if "grad" in out else null,
            _dptr(out["lap"]) if "lap" in out else null,
            int(nthreads))
        if rc != 0:
            raise ValueError("oracle_eval rejected its arguments")
        return out


_default = None


def _oracle() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(_load())
    return _default


def load_variant(path: str) -> Oracle:
    """An Oracle bound to another compiled build of blip_oracle.c."""
    return Oracle(_bind(ctypes.CDLL(path)))


def phi(x, deriv: int = 0) -> np.ndarray:
    """The 1-D cubic B-spline phi (deriv 0), phi' (1) or phi'' (2)."""
    return _oracle().phi(x, deriv)


def inverse3(lattice) -> np.ndarray:
    """A^{-1} by cofactors, as the oracle forms it (raises if singular)."""
    return _oracle().inverse3(lattice)


def wrap(lattice, n, r):
    """Cell index i0 and offset f of position r (the subset selection, Eq. (7))."""
    return _oracle().wrap(lattice, n, r)


def evaluate(lattice, n, coef, pos, kvec=None, want=("val", "grad", "lap"),
             nthreads: int = 1):
    """Orbitals (and gradients, Laplacians) at every position, in FP64;
    see Oracle.evaluate."""
    return _oracle().evaluate(lattice, n, coef, pos, kvec=kvec, want=want, nthreads=nthreads)


def ratio(lattice, n, coef, pos, inv_t, cols, want=("ratio", "grad", "lap"), nthreads: int = 1):
    """Quasi-simultaneous acceptance ratios of the Slater part (Eq.
    (11.12.23.1)) against the old inverse, for real orbitals, in FP64:

        r_j      = sum_l psi_l(r'_j)      Dinv[l, c_j]
        g_j      = sum_l grad psi_l(r'_j) Dinv[l, c_j]
        lambda_j = sum_l lap psi_l(r'_j)  Dinv[l, c_j]

    inv_t is the transposed inverse, inv_t[c, l] = Dinv[l, c] (the column of
    electron c stored contiguously); cols[j] is the electron whose move
    position j is.  r_j is det(D')/det(D) for D' = D with row c_j replaced by
    the orbitals at r'_j; g_j / r_j and lambda_j / r_j are the gradient and
    Laplacian of that ratio with respect to r'_j.
    """
    o = evaluate(lattice, n, coef, pos, want=tuple(
        k for k in ("val", "grad", "lap") if (k == "val") or (k in want)), nthreads=nthreads)
    cols = np.asarray(cols, dtype=np.int64)
    w = np.asarray(inv_t, dtype=np.float64)[cols]              # [npos, L]
    out = {"ratio": np.einsum("jl,jl->j", o["val"], w)}
    if "grad" in want:
        out["grad"] = np.einsum("jcl,jl->jc", o["grad"], w)
    if "lap" in want:
        out["lap"] = np.einsum("jl,jl->j", o["lap"], w)
    return out
