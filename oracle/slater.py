"""FP64 Sherman-Morrison update of the inverse Slater matrix -- TEST
INFRASTRUCTURE ONLY (same rules as the rest of :mod:`oracle`).

Sec. VI.D ("Acceleration of Slater determinant updating"): once the moves of a
step have been accepted or rejected, the inverse of the Slater matrix of
Eq. (5) is brought up to date one accepted electron at a time.  Each update
changes a single electron's orbital row of the matrix.  So the new determinant
follows from a Laplace expansion along that row, and the inverse from a rank-1
correction: O(N^2) work, a dot product per column of the inverse (ddot) and
a scaled row addition per column (daxpy).  The stored new orbital rows are
read in order.

Conventions (shared with the acceptance ratio of Eq. (11.12.23.1)):

* D[i, l] = psi_l(r_i), electron i by orbital l, an N x N matrix per spin
  (the paper arranges electrons as columns; the transpose has the same
  determinant, and a moved electron's row here is its column there).
* ``inv_t`` is the transposed inverse: inv_t[c, l] = Dinv[l, c], so column
  c of the inverse (the one electron c's row of D pairs with) is stored
  contiguously.
* Moving electron c to r'_c replaces row c of D by u[l] = psi_l(r'_c).  The
  determinant changes by the factor R = sum_l u[l] Dinv[l, c] (the matrix
  determinant lemma), and

      Dinv'[l, i] = Dinv[l, i] - Dinv[l, c] (v_i - delta_ic) / R,
      v_i = sum_l u[l] Dinv[l, i],   R = v_c,

  i.e. in rows of inv_t:  row c is divided by R and every other row i has
  (v_i / R) times the old row c subtracted.
"""
from __future__ import annotations

import numpy as np


def sm_update(inv_t, u, cols, return_rows: bool = False):
    """Apply accepted moves one after another with Sherman-Morrison.

    inv_t  [N, N] transposed inverse before the moves (not modified).
    u      [N] or [k, N]: the new orbital row of each accepted move, in order
           (u[m, l] = psi_l(r'_{cols[m]})).
    cols   [k] electron (row of D) of each move, in order.

    Returns (inv_t after all moves, ratios[k]), where ratios[m] is
    det(D^(m)) / det(D^(m-1)) for the matrix after m moves: the ratio of move
    m against the configuration that already holds moves 0..m-1.  With
    return_rows, also the row cols[m] of inv_t just before move m ([k, N]),
    the row that move m's ratio is the dot product with.
    """
    b = np.array(inv_t, dtype=np.float64, copy=True)
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    cols = np.atleast_1d(np.asarray(cols, dtype=np.int64))
    n = b.shape[0]
    if b.shape != (n, n) or u.shape != (cols.shape[0], n):
        raise ValueError("inv_t must be N x N and u k x N")
    ratios = np.empty(cols.shape[0], dtype=np.float64)
    before = np.empty((cols.shape[0], n)) if return_rows else None
    for m, c in enumerate(cols):
        v = b @ u[m]                   # ddot of the new row with every column
        r = v[c]
        ratios[m] = r
        old_c = b[c].copy()
        if return_rows:
            before[m] = old_c
        for i in range(n):             # daxpy per column of the inverse
            if i == c:
                b[i] = old_c / r
            else:
                b[i] = b[i] - (v[i] / r) * old_c
    return (b, ratios, before) if return_rows else (b, ratios)
