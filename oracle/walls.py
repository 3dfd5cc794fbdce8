"""Boxes with Neumann walls: the discrete Laplacian with even-reflection
ghosts, its closed-form eigenpairs, the weights that make it symmetric, and
one wave-solve with the explicit scheme.

Test infrastructure only (see ``oracle/__init__``).

A wall is Dirichlet ("D", the walls of ``discrete``) or Neumann ("N", zero
normal derivative).  The paper states the boundary operator may be
Dirichlet, Neumann or Robin (Sec. "Problem specification and the EigenWave
algorithm"), reports that Neumann results are like the Dirichlet ones (Sec.
"Numerical results"), and uses a Neumann wall as a symmetry plane (Sec.
"Eigenmodes of a double ellipsoid"); it does not print the discrete closure.
Reading for a vertex-centred grid:

* Neumann: the wall point is active and the ghosts mirror the interior evenly
  about it, u_{-k} = u_{k} (central difference of the normal derivative; for
  order 4 the even extension, which makes every odd normal derivative vanish,
  the counterpart of the odd reflection used for Dirichlet walls).
* Dirichlet: as in ``discrete``, the wall is not active, its value is 0, and
  the order-4 ghost is the odd reflection u_{-1-k} = -u_{-1+k}.

Per axis, with n active points on [0, L] (index i = 0 .. n-1):

  D-D  x_i = (i+1) h,  h = L/(n+1)
  D-N  x_i = (i+1) h,  h = L/n        (x_{n-1} = L is the Neumann wall)
  N-D  x_i = i h,      h = L/n        (x_0 = 0 is the Neumann wall)
  N-N  x_i = i h,      h = L/(n-1)

``walls`` is a sequence with one (lo, hi) pair per dimension, x first.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

from .discrete import TimePlan

Walls = Sequence[Tuple[str, str]]


def _check(walls: Walls, dim: int):
    if len(walls) != dim:
        raise ValueError("one (lo, hi) wall pair per dimension")
    for lo, hi in walls:
        if lo not in ("D", "N") or hi not in ("D", "N"):
            raise ValueError("walls are 'D' or 'N'")


def spacing(n: Sequence[int], length: Sequence[float], walls: Walls) -> Tuple[float, ...]:
    """h_d = L_d / (n_d + 1 - number of Neumann walls of dimension d)."""
    _check(walls, len(n))
    return tuple(float(L) / (int(k) + 1 - (lo == "N") - (hi == "N")) for k, L, (lo, hi) in zip(n, length, walls))


def _ghost(j: int, n: int, lo: str, hi: str):
    """(index, sign) of the value at line index j, or None for a zero
    Dirichlet wall value.  Reflections as in the module docstring."""
    if 0 <= j < n:
        return j, 1.0
    if j < 0:
        if lo == "N":
            return -j, 1.0          # u_{-k} = u_{k}
        if j == -1:
            return None             # the wall, value 0
        return -2 - j, -1.0         # u_{-1-k} = -u_{-1+k}
    if hi == "N":
        return 2 * (n - 1) - j, 1.0  # u_{n-1+k} = u_{n-1-k}
    if j == n:
        return None
    return 2 * n - j, -1.0          # u_{n+k} = -u_{n-k}


def line_matrix(n: int, h: float, order: int, lo: str, hi: str) -> np.ndarray:
    """Dense n x n matrix of the second difference along one axis, ghosts
    folded in: order 2 (u_{i-1} - 2u_i + u_{i+1})/h^2, order 4
    (-u_{i-2} + 16u_{i-1} - 30u_i + 16u_{i+1} - u_{i+2})/(12 h^2)."""
    if order == 2:
        st = {-1: 1.0, 0: -2.0, 1: 1.0}
        scale = 1.0 / (h * h)
    elif order == 4:
        st = {-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}
        scale = 1.0 / (12.0 * h * h)
    else:
        raise ValueError("order must be 2 or 4")
    A = np.zeros((n, n))
    for i in range(n):
        for o, c in st.items():
            g = _ghost(i + o, n, lo, hi)
            if g is not None:
                A[i, g[0]] += c * g[1]
    return A * scale


def _apply_along(A: np.ndarray, u: np.ndarray, d: int) -> np.ndarray:
    ax = u.ndim - 1 - d
    return np.moveaxis(np.tensordot(A, np.moveaxis(u, ax, 0), axes=([1], [0])), 0, ax)


def apply_laplacian(u: np.ndarray, h: Sequence[float], order: int, walls: Walls) -> np.ndarray:
    """L_h u: the sum over dimensions of the line operators."""
    _check(walls, u.ndim)
    n = u.shape[::-1]
    out = np.zeros_like(u, dtype=np.float64)
    for d in range(u.ndim):
        out += _apply_along(line_matrix(n[d], h[d], order, *walls[d]), u, d)
    return out


def laplacian_matrix(n: Sequence[int], h: Sequence[float], order: int, walls: Walls) -> np.ndarray:
    """Dense L_h (tiny grids): Kronecker sum of the line matrices, x fastest."""
    mats = [line_matrix(int(k), hd, order, *w) for k, hd, w in zip(n, h, walls)]
    N = int(np.prod(n))
    A = np.zeros((N, N))
    for d, M in enumerate(mats):
        left = int(np.prod(n[d + 1:])) if d + 1 < len(n) else 1
        right = int(np.prod(n[:d])) if d > 0 else 1
        A += np.kron(np.eye(left), np.kron(M, np.eye(right)))
    return A


def line_theta(n: int, lo: str, hi: str) -> np.ndarray:
    """Angle per grid step of each mode of one axis: m pi/(n+1) (D-D),
    (m + 1/2) pi/n (mixed), m pi/(n-1) (N-N), m = 0.. in increasing order
    (m >= 1 for D-D)."""
    m = np.arange(n, dtype=np.float64)
    if lo == "D" and hi == "D":
        return (m + 1.0) * np.pi / (n + 1)
    if lo != hi:
        return (m + 0.5) * np.pi / n
    return m * np.pi / (n - 1)


def line_modes(n: int, lo: str, hi: str) -> np.ndarray:
    """Columns = sampled modes of one axis: sin((i+1) theta) when the low wall
    is Dirichlet (x = (i+1) h), cos(i theta) when it is Neumann (x = i h)."""
    th = line_theta(n, lo, hi)
    i = np.arange(n, dtype=np.float64)[:, None]
    if lo == "D":
        return np.sin((i + 1.0) * th[None, :])
    return np.cos(i * th[None, :])


def line_mu(n: int, h: float, order: int, lo: str, hi: str) -> np.ndarray:
    """Closed-form eigenvalues of minus the line operator, in the order of
    :func:`line_theta`: (4/h^2)(s^2 [+ s^4/3 for order 4]), s = sin(theta/2)."""
    s = np.sin(0.5 * line_theta(n, lo, hi))
    t = s * s if order == 2 else s * s + s ** 4 / 3.0
    return 4.0 / (h * h) * t


def mu_all(n: Sequence[int], h: Sequence[float], order: int, walls: Walls) -> np.ndarray:
    """Closed-form mu for every mode, laid out like a grid function (entry
    [.., j, i] belongs to mode indices (i, j, ..) of :func:`line_theta`)."""
    shape = tuple(int(k) for k in n)[::-1]
    mu = np.zeros(shape)
    for d, (k, hd, w) in enumerate(zip(n, h, walls)):
        b = [1] * len(shape)
        b[len(shape) - 1 - d] = k
        mu = mu + line_mu(k, hd, order, *w).reshape(b)
    return mu


def mode(idx: Sequence[int], n: Sequence[int], walls: Walls) -> np.ndarray:
    """Grid function of the mode with per-axis indices ``idx`` (0-based, in the
    order of :func:`line_theta`)."""
    shape = tuple(int(k) for k in n)[::-1]
    out = np.ones(shape)
    for d, (m, k, w) in enumerate(zip(idx, n, walls)):
        b = [1] * len(shape)
        b[len(shape) - 1 - d] = k
        out = out * line_modes(k, *w)[:, m].reshape(b)
    return out


def weights(n: Sequence[int], walls: Walls) -> np.ndarray:
    """Trapezoid weights that make L_h symmetric: the product over dimensions
    of 1/2 on a Neumann wall point and 1 elsewhere (a grid function)."""
    shape = tuple(int(k) for k in n)[::-1]
    out = np.ones(shape)
    for d, (k, (lo, hi)) in enumerate(zip(n, walls)):
        line = np.ones(k)
        if lo == "N":
            line[0] *= 0.5
        if hi == "N":
            line[-1] *= 0.5
        b = [1] * len(shape)
        b[len(shape) - 1 - d] = k
        out = out * line.reshape(b)
    return out


def apply_filter_explicit(v: np.ndarray, h: Sequence[float], order: int, walls: Walls, plan: TimePlan) -> np.ndarray:
    """S v with the explicit scheme (eqs. explicitStep1, explicitScheme) and
    the trapezoidal filter (eq. filterQuadrature), L_h with these walls."""
    if plan.ts != "explicit":
        raise ValueError("explicit plan expected")
    dt, c = plan.dt, plan.c
    w_prev = np.asarray(v, dtype=np.float64).copy()
    acc = c[0] * w_prev
    w_cur = w_prev + 0.5 * dt * dt * apply_laplacian(w_prev, h, order, walls)
    acc = acc + c[1] * w_cur
    for k in range(1, plan.n_t):
        w_next = 2.0 * w_cur - w_prev + dt * dt * apply_laplacian(w_cur, h, order, walls)
        acc = acc + c[k + 1] * w_next
        w_prev, w_cur = w_cur, w_next
    return acc


def solve_implicit_exact(b: np.ndarray, h: Sequence[float], order: int, walls: Walls, dt: float) -> np.ndarray:
    """Exact solve of M x = b, M = I - (dt^2/2) L_h (eq. impMatrix), by
    diagonalisation: L_h is a Kronecker sum of line operators, each of which
    the sampled modes diagonalise, so x = P (P^{-1} b / (1 + (dt^2/2) mu))
    with P the tensor product of the line mode matrices (a library solve with
    each line's mode matrix does the change of basis)."""
    n = b.shape[::-1]
    mats = [line_modes(int(k), *w) for k, w in zip(n, walls)]
    c = np.asarray(b, dtype=np.float64)
    for d, P in enumerate(mats):
        c = _apply_along(np.linalg.inv(P), c, d)
    c = c / (1.0 + 0.5 * dt * dt * mu_all(n, h, order, walls))
    for d, P in enumerate(mats):
        c = _apply_along(P, c, d)
    return c


def apply_filter_implicit(v: np.ndarray, h: Sequence[float], order: int, walls: Walls, plan: TimePlan) -> np.ndarray:
    """S v with the implicit scheme (eqs. implicitStep1, implicitScheme: M W^1
    = W^0, M S = 2 W^n, W^{n+1} = S - W^{n-1}) and the trapezoidal filter,
    exact solves."""
    if plan.ts != "implicit":
        raise ValueError("implicit plan expected")
    c, dt = plan.c, plan.dt
    w_prev = np.asarray(v, dtype=np.float64).copy()
    acc = c[0] * w_prev
    w_cur = solve_implicit_exact(w_prev, h, order, walls, dt)
    acc = acc + c[1] * w_cur
    for k in range(1, plan.n_t):
        w_next = solve_implicit_exact(2.0 * w_cur, h, order, walls, dt) - w_prev
        acc = acc + c[k + 1] * w_next
        w_prev, w_cur = w_cur, w_next
    return acc
