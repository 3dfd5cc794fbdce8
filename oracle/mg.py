"""Plain geometric multigrid for the implicit step matrix M = I - a L_h, a = dt^2/2.

Test infrastructure only (see ``oracle/__init__``).

The paper solves each implicit step with its own multigrid solver (Sec. "O(N)
scaling") and names only its ingredients: red-black Gauss-Seidel smoothing on
Cartesian grids and convergence to a relative residual tolerance.  The
remaining choices are this project's readings, stated here once:

* vertex-centred coarsening by two: n_c = (n - 1) / 2 per dimension, while
  every n_d is odd and at least 3; h_c = 2 h.  The same operator M (same a,
  same order, same boundary closure) is rediscretised on every level.
* colour of an interior point = parity of the sum of its 0-based indices;
  colour 0 ("red") is relaxed first.  One half-sweep updates every point of
  one colour simultaneously from the current values,
  x_i <- x_i + (b - M x)_i / M_ii,
  where M_ii is the true diagonal of M (order 4: the odd-reflection ghost of
  the first and last interior point folds into it).  For order 2 this is
  exact red-black Gauss-Seidel; for order 4 the +-2 neighbours share the
  point's colour and enter with their values from before the half-sweep.
  With a relaxation weight w the correction is scaled,
  x_i <- x_i + w (b - M x)_i / M_ii (w = 1: the plain sweep; w > 1:
  over-relaxed red-black Gauss-Seidel, a standard variant of the same
  smoother family).  The finest level may take its own weight (``relax``)
  and every coarser level another (``relax_coarse``).
* restriction: full weighting, tensor product of [1 2 1]/4.
* prolongation: multilinear interpolation (the transpose of full weighting
  up to the factor 2^dim), zero boundary values.
* coarsest level: exact when it has a single point, otherwise
  ``coarse_sweeps`` red-black sweeps from the incoming iterate (zero on every
  level below the finest).
* V(nu1, nu2) cycle; the solve stops when ||b - M x||_2 <= tol ||b||_2.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .discrete import apply_laplacian


def level_sizes(n: Sequence[int], max_levels: int = 64) -> List[Tuple[int, ...]]:
    """Interior sizes of all levels, finest first."""
    sizes = [tuple(int(k) for k in n)]
    while len(sizes) < max_levels:
        cur = sizes[-1]
        if all(k % 2 == 1 and k >= 3 for k in cur):
            sizes.append(tuple((k - 1) // 2 for k in cur))
        else:
            break
    return sizes


def apply_M(x: np.ndarray, h: Sequence[float], order: int, a: float) -> np.ndarray:
    """M x = x - a L_h x."""
    return x - a * apply_laplacian(x, h, order)


def diag_M(shape: Tuple[int, ...], h: Sequence[float], order: int, a: float) -> np.ndarray:
    """Diagonal of M on a grid of numpy shape ``shape`` (x last)."""
    ndim = len(shape)
    diag = np.ones(shape)
    for d in range(ndim):
        k = shape[ndim - 1 - d]
        if order == 2:
            line = np.full(k, -2.0 / (h[d] * h[d]))
        else:
            c = np.full(k, -30.0)
            c[0] += 1.0
            c[k - 1] += 1.0
            line = c / (12.0 * h[d] * h[d])
        bshape = [1] * ndim
        bshape[ndim - 1 - d] = k
        diag = diag - a * line.reshape(bshape)
    return diag


def colour_mask(shape: Tuple[int, ...], colour: int) -> np.ndarray:
    """True where the sum of 0-based indices has parity ``colour``."""
    s = np.zeros(shape, dtype=np.int64)
    for ax, k in enumerate(shape):
        bshape = [1] * len(shape)
        bshape[ax] = k
        s = s + np.arange(k).reshape(bshape)
    return (s % 2) == colour


def residual(x: np.ndarray, b: np.ndarray, h, order: int, a: float) -> np.ndarray:
    """b - M x."""
    return b - apply_M(x, h, order, a)


def rb_half_sweep(x: np.ndarray, b: np.ndarray, h, order: int, a: float, colour: int,
                  relax: float = 1.0) -> np.ndarray:
    """Relax every point of one colour simultaneously with weight ``relax``;
    returns the new x."""
    r = residual(x, b, h, order, a)
    d = diag_M(x.shape, h, order, a)
    m = colour_mask(x.shape, colour)
    out = x.copy()
    out[m] = x[m] + relax * r[m] / d[m]
    return out


def rb_sweep(x, b, h, order, a, relax: float = 1.0):
    """One red-black Gauss-Seidel sweep (red, then black)."""
    x = rb_half_sweep(x, b, h, order, a, 0, relax)
    return rb_half_sweep(x, b, h, order, a, 1, relax)


def restrict_full_weighting(r: np.ndarray) -> np.ndarray:
    """Coarse value at fine index 2I+1 (0-based) = [1 2 1]/4 tensor weights."""
    out = r
    for ax in range(r.ndim):
        k = out.shape[ax]
        kc = (k - 1) // 2
        left = np.take(out, 2 * np.arange(kc), axis=ax)
        mid = np.take(out, 2 * np.arange(kc) + 1, axis=ax)
        right = np.take(out, 2 * np.arange(kc) + 2, axis=ax)
        out = 0.25 * left + 0.5 * mid + 0.25 * right
    return out


def prolong_linear(xc: np.ndarray, fine_shape: Tuple[int, ...]) -> np.ndarray:
    """Multilinear interpolation: fine index 2I+1 takes coarse I, fine index 2I
    averages coarse I-1 and I (zero outside the interior)."""
    out = xc
    for ax in range(xc.ndim):
        kf = fine_shape[ax]
        kc = out.shape[ax]
        pad_shape = list(out.shape)
        pad_shape[ax] = 1
        z = np.zeros(pad_shape)
        padded = np.concatenate([z, out, z], axis=ax)   # coarse index I -> I+1
        new_shape = list(out.shape)
        new_shape[ax] = kf
        fine = np.zeros(new_shape)
        idx_f = np.arange(kf)
        odd = idx_f % 2 == 1
        even = ~odd
        I_odd = (idx_f[odd] - 1) // 2
        I_even = idx_f[even] // 2
        sl_odd = [slice(None)] * xc.ndim
        sl_odd[ax] = np.nonzero(odd)[0]
        sl_even = [slice(None)] * xc.ndim
        sl_even[ax] = np.nonzero(even)[0]
        fine[tuple(sl_odd)] = np.take(padded, I_odd + 1, axis=ax)
        fine[tuple(sl_even)] = 0.5 * (np.take(padded, I_even, axis=ax) + np.take(padded, I_even + 1, axis=ax))
        out = fine
    return out


class Hierarchy:
    """Level sizes and spacings for one grid and one implicit step size."""

    def __init__(self, n: Sequence[int], h: Sequence[float], order: int, a: float,
                 nu1: int = 2, nu2: int = 1, coarse_sweeps: int = 8, max_levels: int = 64,
                 relax: float = 1.0, relax_coarse: float = None):
        self.sizes = level_sizes(n, max_levels)
        self.h = [tuple(hd * (2 ** l) for hd in h) for l in range(len(self.sizes))]
        self.order = order
        self.a = a
        self.nu1 = nu1
        self.nu2 = nu2
        self.coarse_sweeps = coarse_sweeps
        self.relax = relax
        self.relax_coarse = relax if relax_coarse is None else relax_coarse

    def weight(self, level: int) -> float:
        """Relaxation weight of the red-black sweeps on ``level``: ``relax`` on
        the finest level, ``relax_coarse`` below it."""
        return self.relax if level == 0 else self.relax_coarse

    def shape(self, level: int) -> Tuple[int, ...]:
        return self.sizes[level][::-1]


def coarse_solve(x: np.ndarray, b: np.ndarray, hier: Hierarchy, level: int) -> np.ndarray:
    """Coarsest level: exact for a single point, otherwise ``coarse_sweeps``
    red-black sweeps from the incoming iterate (zero below the finest level)."""
    h = hier.h[level]
    if b.size == 1:
        return b / diag_M(b.shape, h, hier.order, hier.a)
    for _ in range(hier.coarse_sweeps):
        x = rb_sweep(x, b, h, hier.order, hier.a, hier.weight(level))
    return x


def vcycle(x: np.ndarray, b: np.ndarray, hier: Hierarchy, level: int = 0) -> np.ndarray:
    """One V(nu1, nu2) cycle on ``level``; returns the new x."""
    h = hier.h[level]
    if level == len(hier.sizes) - 1:
        return coarse_solve(x, b, hier, level)
    for _ in range(hier.nu1):
        x = rb_sweep(x, b, h, hier.order, hier.a, hier.weight(level))
    r = residual(x, b, h, hier.order, hier.a)
    bc = restrict_full_weighting(r)
    xc = vcycle(np.zeros_like(bc), bc, hier, level + 1)
    x = x + prolong_linear(xc, x.shape)
    for _ in range(hier.nu2):
        x = rb_sweep(x, b, h, hier.order, hier.a, hier.weight(level))
    return x


def solve(b: np.ndarray, hier: Hierarchy, tol: float, x0=None, max_cycles: int = 100):
    """V-cycles until ||b - M x||_2 <= tol ||b||_2.  Returns (x, cycles, rel_res)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    h = hier.h[0]
    rel = np.linalg.norm(residual(x, b, h, hier.order, hier.a)) / bn
    cycles = 0
    while rel > tol and cycles < max_cycles:
        x = vcycle(x, b, hier)
        cycles += 1
        rel = np.linalg.norm(residual(x, b, h, hier.order, hier.a)) / bn
    return x, cycles, rel
