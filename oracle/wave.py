"""One wave-solve plus time filter: the WaveHoltz operator S applied to v.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

from typing import Callable, Optional, Sequence

import numpy as np
import scipy.fft

from .discrete import TimePlan, apply_laplacian, laplacian_matrix, mu_all


def implicit_matrix_eigenvalues(n: Sequence[int], h: Sequence[float], order: int, dt: float) -> np.ndarray:
    """Eigenvalues 1 + (dt^2/2) mu of M = I - (dt^2/2) L_h (eq. impMatrix), one
    per sine mode, laid out like :func:`mu_all`."""
    return 1.0 + 0.5 * dt * dt * mu_all(n, h, order)


def solve_implicit_exact(b: np.ndarray, h: Sequence[float], order: int, dt: float) -> np.ndarray:
    """Exact solve of M x = b by diagonalisation in the sine basis.

    The sampled sines are the eigenvectors of L_h for both stencils with the
    Dirichlet/odd-reflection closure, and the orthonormal type-I discrete sine
    transform is the change of basis to them (and its own inverse), so
    x = DST(DST(b) / eig(M)).  A library FFT does the transform.
    """
    n = b.shape[::-1]
    lam = implicit_matrix_eigenvalues(n, h, order, dt)
    bh = scipy.fft.dstn(b, type=1, norm="ortho")
    return scipy.fft.idstn(bh / lam, type=1, norm="ortho")


def solve_implicit_dense(b: np.ndarray, h: Sequence[float], order: int, dt: float) -> np.ndarray:
    """Exact solve of M x = b with an assembled dense M (tiny grids only)."""
    n = b.shape[::-1]
    L = laplacian_matrix(n, h, order)
    M = np.eye(L.shape[0]) - 0.5 * dt * dt * L
    return np.linalg.solve(M, b.ravel()).reshape(b.shape)


def apply_filter(v: np.ndarray, h: Sequence[float], order: int, plan: TimePlan,
                 solve: Optional[Callable[[np.ndarray], np.ndarray]] = None,
                 return_levels: bool = False):
    """S v: solve the wave equation from W^0 = v, dW/dt(0) = 0, over N_t steps
    and accumulate the trapezoidal time filter (eq. filterQuadrature).

    Explicit (eq. explicitScheme, first step eq. explicitStep1):
        W^1     = W^0 + (dt^2/2) L W^0
        W^{n+1} = 2 W^n - W^{n-1} + dt^2 L W^n
    Implicit (eq. implicitScheme, first step eq. implicitStep1), with
    M = I - (dt^2/2) L:
        M W^1     = W^0
        M W^{n+1} = 2 W^n - M W^{n-1}, computed as M S = 2 W^n, W^{n+1} = S - W^{n-1}
    The filter V = sum_n c_n W^n is accumulated inside the loop (Alg. 1 note).

    ``solve(b)`` returns M^{-1} b for the implicit scheme; by default the exact
    sine-transform solve.  With ``return_levels`` the list of all W^n is also
    returned (small cases only).
    """
    v = np.asarray(v, dtype=np.float64)
    dt = plan.dt
    c = plan.c
    levels = [v.copy()] if return_levels else None
    if plan.ts == "explicit":
        w_prev = v.copy()
        acc = c[0] * w_prev
        w_cur = w_prev + 0.5 * dt * dt * apply_laplacian(w_prev, h, order)
        acc = acc + c[1] * w_cur
        if return_levels:
            levels.append(w_cur.copy())
        for k in range(1, plan.n_t):
            w_next = 2.0 * w_cur - w_prev + dt * dt * apply_laplacian(w_cur, h, order)
            acc = acc + c[k + 1] * w_next
            w_prev, w_cur = w_cur, w_next
            if return_levels:
                levels.append(w_cur.copy())
    else:
        if solve is None:
            def solve(b):
                return solve_implicit_exact(b, h, order, dt)
        w_prev = v.copy()
        acc = c[0] * w_prev
        w_cur = solve(w_prev)
        acc = acc + c[1] * w_cur
        if return_levels:
            levels.append(w_cur.copy())
        for k in range(1, plan.n_t):
            s = solve(2.0 * w_cur)
            w_next = s - w_prev
            acc = acc + c[k + 1] * w_next
            w_prev, w_cur = w_cur, w_next
            if return_levels:
                levels.append(w_cur.copy())
    if return_levels:
        return acc, levels
    return acc
