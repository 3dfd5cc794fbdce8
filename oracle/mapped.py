"""A single curvilinear grid by the mapping method: the order-2 Laplacian in
conservative form with the metric terms of a mapping x = G(r) of the unit
square, its symmetrising weights, the explicit time plan, and one wave-solve
with the explicit scheme or with the implicit scheme (exact sparse solves).

Test infrastructure only (see ``oracle/__init__``).

The paper (Sec. "Discrete approximations") transforms the equations to the
unit-square coordinates r by the chain rule and discretises them with
standard centred or conservative differences; it prints no discrete form.
Reading (second order, 2D, Dirichlet walls).  With J = x_r y_s - x_s y_r and
the contravariant metric a^{mn} = grad r_m . grad r_n,

    Laplacian u = (1/J) sum_{m,n} d/dr_m ( J a^{mn} du/dr_n ),

    J a^{11} = (x_s^2 + y_s^2) / J,   J a^{22} = (x_r^2 + y_r^2) / J,
    J a^{12} = J a^{21} = -(x_r x_s + y_r y_s) / J.

At an active point (i, j):

    J L_h u = D+r (A11 D-r u) + D+s (A22 D-s u) + D0r (B D0s u) + D0s (B D0r u)

with A11 at the half point i - 1/2 the mean of J a^{11} at nodes i - 1 and i
(A22 likewise along s), B = J a^{12} at the nodes, and the metric derivatives
x_r, x_s, y_r, y_s taken by centred differences of the grid coordinates at
every node, walls included (hence one layer of coordinates beyond each
wall).  Dirichlet walls hold u = 0.  Summation by parts makes J L_h
symmetric: L_h is self-adjoint in the inner product weighted by J.

Index conventions as in ``discrete``: a grid function has shape (n2, n1),
x (r) fastest; active point (i, j), i in [0, n1), has r = (i + 1)/(n1 + 1).
Coordinates come as an array of shape (2, n2 + 4, n1 + 4) (x, then y) holding
node (i, j) for i in [-2, n1 + 1], j in [-2, n2 + 1] at [., j + 2, i + 2]
(``synthetic.mapped_coords``).
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import discrete
from .discrete import TimePlan


def _sizes(xy: np.ndarray):
    if xy.ndim != 3 or xy.shape[0] != 2:
        raise ValueError("coordinates must have shape (2, n2 + 4, n1 + 4)")
    n2, n1 = xy.shape[1] - 4, xy.shape[2] - 4
    if n1 < 1 or n2 < 1:
        raise ValueError("need at least one active point per direction")
    return n1, n2


def metrics(xy: np.ndarray) -> Dict[str, np.ndarray]:
    """Metric terms at every node i in [-1, n1], j in [-1, n2] (arrays of
    shape (n2 + 2, n1 + 2), node (i, j) at [j + 1, i + 1]): centred
    differences x_r = (x_{i+1} - x_{i-1}) / (2 dr), dr = 1/(n1 + 1), and so
    on; J and the products J a^{mn}."""
    n1, n2 = _sizes(xy)
    dr, ds = 1.0 / (n1 + 1), 1.0 / (n2 + 1)
    X, Y = np.asarray(xy[0], dtype=np.float64), np.asarray(xy[1], dtype=np.float64)
    x_r = (X[1:-1, 2:] - X[1:-1, :-2]) / (2.0 * dr)
    y_r = (Y[1:-1, 2:] - Y[1:-1, :-2]) / (2.0 * dr)
    x_s = (X[2:, 1:-1] - X[:-2, 1:-1]) / (2.0 * ds)
    y_s = (Y[2:, 1:-1] - Y[:-2, 1:-1]) / (2.0 * ds)
    J = x_r * y_s - x_s * y_r
    return {"J": J,
            "a11J": (x_s * x_s + y_s * y_s) / J,
            "a22J": (x_r * x_r + y_r * y_r) / J,
            "a12J": -(x_r * x_s + y_r * y_s) / J,
            "dr": dr, "ds": ds}


def _at(F: np.ndarray, di: int, dj: int) -> np.ndarray:
    """Values of a node array (offset 1) at (i + di, j + dj) for every active (i, j)."""
    n2, n1 = F.shape[0] - 2, F.shape[1] - 2
    return F[1 + dj:n2 + 1 + dj, 1 + di:n1 + 1 + di]


def stencil(xy: np.ndarray) -> Dict[tuple, np.ndarray]:
    """The nine weights of J L_h at every active point, keyed by the offset
    (di, dj) of the neighbour they multiply (the formula of the module
    docstring, expanded)."""
    m = metrics(xy)
    dr, ds = m["dr"], m["ds"]
    a11, a22, B = m["a11J"], m["a22J"], m["a12J"]
    Ap = 0.5 * (_at(a11, 0, 0) + _at(a11, 1, 0))    # A11 at i + 1/2
    Am = 0.5 * (_at(a11, -1, 0) + _at(a11, 0, 0))   # A11 at i - 1/2
    Cp = 0.5 * (_at(a22, 0, 0) + _at(a22, 0, 1))    # A22 at j + 1/2
    Cm = 0.5 * (_at(a22, 0, -1) + _at(a22, 0, 0))   # A22 at j - 1/2
    q = 1.0 / (4.0 * dr * ds)
    Be, Bw, Bn, Bs = _at(B, 1, 0), _at(B, -1, 0), _at(B, 0, 1), _at(B, 0, -1)
    return {(0, 0): -(Ap + Am) / dr ** 2 - (Cp + Cm) / ds ** 2,
            (1, 0): Ap / dr ** 2, (-1, 0): Am / dr ** 2,
            (0, 1): Cp / ds ** 2, (0, -1): Cm / ds ** 2,
            # D0r(B D0s u): +B_e u_{i+1,j+1} - B_e u_{i+1,j-1} - B_w u_{i-1,j+1} + B_w u_{i-1,j-1}
            # D0s(B D0r u): +B_n u_{i+1,j+1} - B_n u_{i-1,j+1} - B_s u_{i+1,j-1} + B_s u_{i-1,j-1}
            (1, 1): q * (Be + Bn), (1, -1): -q * (Be + Bs),
            (-1, 1): -q * (Bw + Bn), (-1, -1): q * (Bw + Bs)}


def apply_laplacian_full(U: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """L_h at the active points from node values U of shape (n2 + 2, n1 + 2)
    that include the walls (node (i, j) at [j + 1, i + 1]), written as the
    conservative differences of the module docstring."""
    m = metrics(xy)
    dr, ds = m["dr"], m["ds"]
    a11, a22, B, J = m["a11J"], m["a22J"], m["a12J"], m["J"]
    U = np.asarray(U, dtype=np.float64)
    u = lambda di, dj: _at(U, di, dj)
    Ap = 0.5 * (_at(a11, 0, 0) + _at(a11, 1, 0))
    Am = 0.5 * (_at(a11, -1, 0) + _at(a11, 0, 0))
    Cp = 0.5 * (_at(a22, 0, 0) + _at(a22, 0, 1))
    Cm = 0.5 * (_at(a22, 0, -1) + _at(a22, 0, 0))
    rr = (Ap * (u(1, 0) - u(0, 0)) - Am * (u(0, 0) - u(-1, 0))) / dr ** 2
    ss = (Cp * (u(0, 1) - u(0, 0)) - Cm * (u(0, 0) - u(0, -1))) / ds ** 2
    # D0r (B D0s u): B D0s u at nodes i +- 1, then the centred difference in r
    rs = (_at(B, 1, 0) * (u(1, 1) - u(1, -1)) - _at(B, -1, 0) * (u(-1, 1) - u(-1, -1))) / (4.0 * dr * ds)
    # D0s (B D0r u)
    sr = (_at(B, 0, 1) * (u(1, 1) - u(-1, 1)) - _at(B, 0, -1) * (u(1, -1) - u(-1, -1))) / (4.0 * dr * ds)
    return (rr + ss + rs + sr) / _at(J, 0, 0)


def apply_laplacian(u: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """L_h u for a grid function on the active points (Dirichlet walls: 0)."""
    n1, n2 = _sizes(xy)
    u = np.asarray(u, dtype=np.float64)
    if u.shape != (n2, n1):
        raise ValueError("grid function shape must be (n2, n1)")
    U = np.zeros((n2 + 2, n1 + 2))
    U[1:-1, 1:-1] = u
    return apply_laplacian_full(U, xy)


def laplacian_matrix(xy: np.ndarray) -> np.ndarray:
    """Dense L_h (tiny grids), column k = L_h applied to unit vector k (x fastest)."""
    n1, n2 = _sizes(xy)
    N = n1 * n2
    A = np.empty((N, N))
    e = np.zeros(N)
    for k in range(N):
        e[k] = 1.0
        A[:, k] = apply_laplacian(e.reshape(n2, n1), xy).ravel()
        e[k] = 0.0
    return A


def weights(xy: np.ndarray) -> np.ndarray:
    """J at the active points: the weights in which L_h is self-adjoint."""
    return _at(metrics(xy)["J"], 0, 0).copy()


def spectral_radius_bound(xy: np.ndarray) -> float:
    """Gershgorin bound on the spectrum of -L_h: the largest, over active
    points, of (1/J) times the sum of the absolute values of the nine weights
    of J L_h (the weights of wall neighbours included, which only loosens
    it).  For an affine map of a rectangle it equals the box bound
    4 (1/h_x^2 + 1/h_y^2)."""
    w = stencil(xy)
    total = sum(np.abs(v) for v in w.values())
    return float(np.max(total / weights(xy)))


def time_plan(xy: np.ndarray, omega: float, cfl: float = 0.5, n_p: int = 1,
              filter_const: str = "alpha_d") -> TimePlan:
    """Explicit plan with dt_max = 2 / sqrt(spectral_radius_bound) (the box
    plan of ``discrete.time_plan`` with this grid's bound)."""
    return discrete.time_plan((1.0, 1.0), 2, omega, "explicit", cfl=cfl, n_p=n_p,
                              filter_const=filter_const, rho=spectral_radius_bound(xy))


def apply_filter_explicit(v: np.ndarray, xy: np.ndarray, plan: TimePlan) -> np.ndarray:
    """S v with the explicit scheme (eqs. explicitStep1, explicitScheme) and
    the trapezoidal filter (eq. filterQuadrature) on the mapped grid."""
    if plan.ts != "explicit":
        raise ValueError("explicit plan expected")
    dt, c = plan.dt, plan.c
    w_prev = np.asarray(v, dtype=np.float64).copy()
    acc = c[0] * w_prev
    w_cur = w_prev + 0.5 * dt * dt * apply_laplacian(w_prev, xy)
    acc = acc + c[1] * w_cur
    for k in range(1, plan.n_t):
        w_next = 2.0 * w_cur - w_prev + dt * dt * apply_laplacian(w_cur, xy)
        acc = acc + c[k + 1] * w_next
        w_prev, w_cur = w_cur, w_next
    return acc


def laplacian_sparse(xy: np.ndarray):
    """L_h as a sparse matrix (rows and columns x fastest), assembled from the
    nine weights of :func:`stencil` divided by J; wall neighbours dropped."""
    from scipy import sparse
    n1, n2 = _sizes(xy)
    w = stencil(xy)
    iJ = 1.0 / weights(xy)
    jj, ii = np.meshgrid(np.arange(n2), np.arange(n1), indexing="ij")
    rows, cols, vals = [], [], []
    for (di, dj), wk in w.items():
        ti, tj = ii + di, jj + dj
        ok = (ti >= 0) & (ti < n1) & (tj >= 0) & (tj < n2)
        rows.append((jj * n1 + ii)[ok])
        cols.append((tj * n1 + ti)[ok])
        vals.append((wk * iJ)[ok])
    N = n1 * n2
    return sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def solve_implicit_exact(b: np.ndarray, xy: np.ndarray, dt: float) -> np.ndarray:
    """Exact solve of M x = b, M = I - (dt^2/2) L_h (eq. impMatrix), by a
    library sparse direct solve."""
    from scipy import sparse
    from scipy.sparse.linalg import spsolve
    n1, n2 = _sizes(xy)
    M = sparse.identity(n1 * n2, format="csc") - 0.5 * dt * dt * laplacian_sparse(xy).tocsc()
    return spsolve(M, np.asarray(b, dtype=np.float64).ravel()).reshape(n2, n1)


def implicit_plan(xy: np.ndarray, omega: float, n_its: int = 10, n_p: int = 1, adjust_omega: bool = True,
                  filter_const: str = "alpha_d") -> TimePlan:
    """Implicit plan: N_t = N_p N_its (it does not depend on the grid)."""
    return discrete.time_plan((1.0, 1.0), 2, omega, "implicit", n_its=n_its, n_p=n_p,
                              adjust_omega=adjust_omega, filter_const=filter_const)


def apply_filter_implicit(v: np.ndarray, xy: np.ndarray, plan: TimePlan) -> np.ndarray:
    """S v with the implicit scheme (eqs. implicitStep1, implicitScheme:
    M W^1 = W^0, M S = 2 W^n, W^{n+1} = S - W^{n-1}) and the trapezoidal
    filter, exact solves, on the mapped grid."""
    if plan.ts != "implicit":
        raise ValueError("implicit plan expected")
    c, dt = plan.c, plan.dt
    w_prev = np.asarray(v, dtype=np.float64).copy()
    acc = c[0] * w_prev
    w_cur = solve_implicit_exact(w_prev, xy, dt)
    acc = acc + c[1] * w_cur
    for k in range(1, plan.n_t):
        w_next = solve_implicit_exact(2.0 * w_cur, xy, dt) - w_prev
        acc = acc + c[k + 1] * w_next
        w_prev, w_cur = w_cur, w_next
    return acc
