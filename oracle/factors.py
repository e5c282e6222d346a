"""Dense factors of eq. (6) and eq. (9), built literally from Section III.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every factor is a real 2N x 2N matrix acting on the interleaved vector
x_2N = [x0r, x0i, x1r, x1i, ...] of Section III.  They are assembled with
``numpy.kron`` exactly as the paper writes them, with two readings:

* the leading identity of W^(i) and D^(i) has order 2^(m-i), as in the
  worked N = 8 example (the general formula prints 2^(m-1), which does not
  give a 2N x 2N matrix for i > 1);
* omega^(i,q) is taken from its formula, not from the printed omega^(3,3) of
  eq. (8), which repeats omega^(3,1).

Only small N (up to 64) is meant: the matrices are dense.
"""
from __future__ import annotations

import numpy as np

from . import bit_reverse, omega


def H2() -> np.ndarray:
    return np.array([[1.0, 1.0], [1.0, -1.0]])


def omega_block(i: int, q: int) -> np.ndarray:
    """omega^(i,q)_2 = [[cos t, sin t], [-sin t, cos t]], t = 2 pi q / 2^i."""
    c, s = omega(q, i)
    return np.array([[c, s], [-s, c]])


def bitrev_matrix(m: int) -> np.ndarray:
    """S_(2^m): row k has its single 1 in column rev_m(k) (0-based)."""
    n = 1 << m
    p = np.zeros((n, n))
    for k in range(n):
        p[k, bit_reverse(k, m)] = 1.0
    return p


def S_pairwise(m: int) -> np.ndarray:
    """S_(2^(m+1)) = S_(2^m) (x) I_2."""
    return np.kron(bitrev_matrix(m), np.eye(2))


def D_block(i: int) -> np.ndarray:
    """D_(2^(i+1)) = diag(I_(2R), omega^(i,0), ..., omega^(i,R-1)), R = 2^(i-1)."""
    R = 1 << (i - 1)
    size = 1 << (i + 1)
    d = np.zeros((size, size))
    d[: 2 * R, : 2 * R] = np.eye(2 * R)
    for q in range(R):
        o = 2 * R + 2 * q
        d[o:o + 2, o:o + 2] = omega_block(i, q)
    return d


def D_factor(m: int, i: int) -> np.ndarray:
    """D^(i)_(2^(m+1)) = I_(2^(m-i)) (x) D_(2^(i+1))."""
    return np.kron(np.eye(1 << (m - i)), D_block(i))


def W_factor(m: int, i: int) -> np.ndarray:
    """W^(i)_(2^(m+1)) = I_(2^(m-i)) (x) H_2 (x) I_(2^i)."""
    return np.kron(np.kron(np.eye(1 << (m - i)), H2()), np.eye(1 << i))


def dit_product(m: int) -> np.ndarray:
    """W^(m) D^(m) ... W^(1) D^(1) S_(2^(m+1)) of eq. (6)."""
    acc = S_pairwise(m)
    for i in range(1, m + 1):
        acc = W_factor(m, i) @ (D_factor(m, i) @ acc)
    return acc


def dif_product(m: int) -> np.ndarray:
    """S_(2^(m+1)) D^(1) W^(1) ... D^(m) W^(m) of eq. (9)."""
    n2 = 2 << m
    acc = np.eye(n2)
    for i in range(m, 0, -1):
        acc = D_factor(m, i) @ (W_factor(m, i) @ acc)
    return S_pairwise(m) @ acc


def E2N_planar(n: int) -> np.ndarray:
    """E_2N = [[C, S], [-S, C]] of eq. (5), c_kn = cos(2 pi k n/N), s_kn = sin(2 pi k n/N)."""
    k = np.arange(n)
    t = 2.0 * np.pi * ((np.outer(k, k)) % n) / n
    C, S = np.cos(t), np.sin(t)
    return np.block([[C, S], [-S, C]])


def perfect_shuffle(n: int) -> np.ndarray:
    """Q with x_2N = Q [xr; xi]: interleaved index 2k <- k, 2k+1 <- N+k."""
    q = np.zeros((2 * n, 2 * n))
    for k in range(n):
        q[2 * k, k] = 1.0
        q[2 * k + 1, n + k] = 1.0
    return q


def E2N_interleaved(n: int) -> np.ndarray:
    """E_2N of eq. (5) expressed on the interleaved vectors of Section III."""
    Q = perfect_shuffle(n)
    return Q @ E2N_planar(n) @ Q.T
