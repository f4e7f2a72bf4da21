"""Plain CPU full-Stokes formation from visibilities, the reference for the
GPU Stokes kernel.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may load it.  It shares no code with the GPU library.

What it computes (paper, Section 1: the correlator delivers full-Stokes
output for 96 dual-polarisation feeds; Section 3.3 names the two linear
polarisations, X north-south and Y east-west).  Readings where the paper is
silent:
  * input 2 f + pol is feed f's polarisation pol (0 = X, 1 = Y);
  * for feeds a >= b the four polarisation products are XX = V(2a, 2b),
    YY = V(2a+1, 2b+1), XY = V(2a, 2b+1) and YX = V(2a+1, 2b), with
    V(i, j) = sum_t x_i conj(x_j); for a = b, XY = conj V(2a+1, 2a), the
    stored lower-triangle entry;
  * Stokes parameters of linear feeds: I = XX + YY, Q = XX - YY,
    U = XY + YX, V = -i (XY - YX);
  * exact integer arithmetic (int64) on the exact integer visibilities.
Output: int64 [F][Nf (Nf + 1) / 2][4 (I, Q, U, V)][2 (re, im)], feed pairs
in row-major lower-triangle order, index a (a + 1) / 2 + b.
"""
from __future__ import annotations

import numpy as np


def _vis(V: np.ndarray, i: int, j: int) -> np.ndarray:
    """Complex visibility V(i, j) (any order) from the lower triangle, as int64
    (re, im) pairs over channels: [F][2]."""
    if i >= j:
        return V[:, i * (i + 1) // 2 + j, :].astype(np.int64)
    v = V[:, j * (j + 1) // 2 + i, :].astype(np.int64)
    return np.stack([v[:, 0], -v[:, 1]], axis=-1)


def stokes(V: np.ndarray, n_inputs: int) -> np.ndarray:
    """Full-Stokes visibilities of every feed pair from input visibilities V
    [F][P][2] (P = N (N + 1) / 2, N = 2 Nf)."""
    if n_inputs % 2:
        raise ValueError("dual-polarisation feeds need an even input count")
    nf = n_inputs // 2
    F = V.shape[0]
    out = np.zeros((F, nf * (nf + 1) // 2, 4, 2), dtype=np.int64)
    for a in range(nf):
        for b in range(a + 1):
            xx = _vis(V, 2 * a, 2 * b)
            yy = _vis(V, 2 * a + 1, 2 * b + 1)
            xy = _vis(V, 2 * a, 2 * b + 1)
            yx = _vis(V, 2 * a + 1, 2 * b)
            p = a * (a + 1) // 2 + b
            out[:, p, 0] = xx + yy
            out[:, p, 1] = xx - yy
            out[:, p, 2] = xy + yx
            d = xy - yx
            out[:, p, 3, 0] = d[:, 1]          # -i (dr + i di) = di - i dr
            out[:, p, 3, 1] = -d[:, 0]
    return out
