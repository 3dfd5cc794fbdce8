"""Grids, the discrete Dirichlet Laplacian, closed forms and the filter plan.

Test infrastructure only (see ``oracle/__init__``).

Conventions.  A grid has ``n[d]`` interior (active) points in dimension d
(x first) on a box of side ``length[d]``; ``h[d] = length[d] / (n[d] + 1)``.
Grid functions are numpy arrays of shape ``n[::-1]`` so that the flattened
C-order vector is lexicographic with x fastest (the active-point vector of the
paper's matrix-vector routine, Alg. "WaveHoltz matrix-vector product").
Boundary points carry the homogeneous Dirichlet value 0 and are not stored.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Sequence, Tuple

import numpy as np


def spacing(n: Sequence[int], length: Sequence[float]) -> Tuple[float, ...]:
    """Grid spacing per dimension, h_d = L_d / (n_d + 1)."""
    return tuple(float(L) / (int(k) + 1) for k, L in zip(n, length))


def _axis(u: np.ndarray, d: int) -> int:
    """numpy axis that holds dimension d (x is the last axis)."""
    return u.ndim - 1 - d


def _padded_line_values(u: np.ndarray, d: int, order: int) -> np.ndarray:
    """Extend u along dimension d with boundary values and, for order 4, ghosts.

    Order 2: one boundary point with value 0 at each end.
    Order 4: additionally one ghost beyond each boundary point, set by odd
    reflection about the wall, u_{-1} = -u_{1} and u_{n+2} = -u_{n}.  The paper
    suppresses the details of its compatibility conditions (Sec. "Discrete
    approximations"); for a flat Dirichlet wall of the constant-coefficient
    Laplacian they make every even normal derivative vanish, which is exactly
    odd reflection.
    """
    ax = _axis(u, d)
    zero = np.zeros_like(np.take(u, [0], axis=ax))
    if order == 2:
        return np.concatenate([zero, u, zero], axis=ax)
    if order == 4:
        first = np.take(u, [0], axis=ax)
        last = np.take(u, [u.shape[ax] - 1], axis=ax)
        return np.concatenate([-first, zero, u, zero, -last], axis=ax)
    raise ValueError("order must be 2 or 4")


def apply_laplacian(u: np.ndarray, h: Sequence[float], order: int) -> np.ndarray:
    """L_h u on the interior points (the operator L_ph of eq. eigBVPdiscrete).

    Order 2: sum_d (u_{i+1} - 2 u_i + u_{i-1}) / h_d^2.
    Order 4: sum_d (-u_{i-2} + 16 u_{i-1} - 30 u_i + 16 u_{i+1} - u_{i+2}) / (12 h_d^2).
    """
    out = np.zeros_like(u, dtype=np.float64)
    for d in range(u.ndim):
        ax = _axis(u, d)
        p = _padded_line_values(u, d, order)
        n = u.shape[ax]
        g = 1 if order == 2 else 2

        def sl(shift: int) -> np.ndarray:
            return np.take(p, np.arange(g + shift, g + shift + n), axis=ax)

        if order == 2:
            out += (sl(1) - 2.0 * sl(0) + sl(-1)) / (h[d] * h[d])
        else:
            out += (-sl(-2) + 16.0 * sl(-1) - 30.0 * sl(0) + 16.0 * sl(1) - sl(2)) / (12.0 * h[d] * h[d])
    return out


def laplacian_matrix(n: Sequence[int], h: Sequence[float], order: int) -> np.ndarray:
    """Dense matrix of L_h on the active points (tiny grids only), built by
    applying L_h to every unit vector."""
    shape = tuple(int(k) for k in n)[::-1]
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = apply_laplacian(e.reshape(shape), h, order).ravel()
    return A


def mu_closed_form(modes: Sequence[int], n: Sequence[int], h: Sequence[float], order: int) -> float:
    """Eigenvalue mu = lambda_h^2 of -L_h for the sampled sine mode ``modes``.

    With s_d = sin(m_d pi / (2 (n_d + 1))):
      order 2: mu = sum_d (4 / h_d^2) s_d^2
      order 4: mu = sum_d (4 / h_d^2) (s_d^2 + s_d^4 / 3)
    (the symbols of the stencils above on e^{i theta j}, theta = m pi/(n+1)).
    """
    mu = 0.0
    for m, k, hd in zip(modes, n, h):
        s = math.sin(m * math.pi / (2.0 * (k + 1)))
        t = s * s if order == 2 else s * s + s ** 4 / 3.0
        mu += 4.0 / (hd * hd) * t
    return mu


def mu_all(n: Sequence[int], h: Sequence[float], order: int) -> np.ndarray:
    """Closed-form mu for every mode; entry [.., j, i] belongs to modes (i+1, j+1, ..)."""
    shape = tuple(int(k) for k in n)[::-1]
    mu = np.zeros(shape)
    for d, (k, hd) in enumerate(zip(n, h)):
        s = np.sin(np.arange(1, k + 1) * np.pi / (2.0 * (k + 1)))
        t = s * s if order == 2 else s * s + s ** 4 / 3.0
        line = 4.0 / (hd * hd) * t
        bshape = [1] * len(shape)
        bshape[len(shape) - 1 - d] = k
        mu = mu + line.reshape(bshape)
    return mu


def sine_mode(modes: Sequence[int], n: Sequence[int]) -> np.ndarray:
    """Grid function prod_d sin(m_d pi x_d / L_d) sampled at the interior points."""
    shape = tuple(int(k) for k in n)[::-1]
    out = np.ones(shape)
    for d, (m, k) in enumerate(zip(modes, n)):
        line = np.sin(m * np.pi * np.arange(1, k + 1) / (k + 1))
        bshape = [1] * len(shape)
        bshape[len(shape) - 1 - d] = k
        out = out * line.reshape(bshape)
    return out


def spectral_radius_bound(h: Sequence[float], order: int) -> float:
    """Upper bound rho on the spectrum of -L_h: sum_d c / h_d^2 with c = 4 for
    order 2 (the s = 1 value of the symbol) and c = 16/3 for order 4."""
    c = 4.0 if order == 2 else 16.0 / 3.0
    rho = 0.0
    for hd in h:
        rho += c / (hd * hd)
    return rho


def omega_adjusted(omega: float, n_its: int) -> float:
    """Adjusted target frequency (eq. adjustedOmega): the frequency whose
    time-corrected implicit filter peaks at lambda = omega,
    omega~ = (omega pi / N_its) sqrt((1 - 2 sin^2(pi/N_its)) / sin^2(pi/N_its))."""
    s2 = math.sin(math.pi / n_its) ** 2
    return omega * math.pi / n_its * math.sqrt((1.0 - 2.0 * s2) / s2)


def alpha_d(omega: float, dt: float) -> float:
    """Filter constant alpha_d = tan(omega dt / 2) / tan(omega dt) (eq. alphad)."""
    return math.tan(omega * dt / 2.0) / math.tan(omega * dt)


@dataclass
class TimePlan:
    """Everything one wave-solve needs besides the grid."""

    omega: float          # frequency actually used in the filter (adjusted or not)
    t_final: float        # T_f = N_p 2 pi / omega
    n_t: int              # number of time steps N_t
    dt: float             # dt = T_f / N_t
    alpha_d: float
    c: np.ndarray         # filter weights c_n, n = 0..N_t (eq. filterQuadrature)
    ts: str


def time_plan(h: Sequence[float], order: int, omega: float, ts: str, cfl: float = 0.5,
              n_its: int = 10, n_p: int = 1, adjust_omega: bool = False,
              filter_const: str = "alpha_d", rho: float = None) -> TimePlan:
    """Time step, step count and trapezoidal filter weights of one wave-solve.

    * T_f = N_p * 2 pi / omega (Sec. "Continuous algorithm").
    * Implicit: N_t = N_p * N_its, dt = T_f / N_t.
    * Explicit (the paper only says a CFL-type restriction applies): the
      leapfrog scheme is stable for dt * sqrt(rho) <= 2 with rho the spectral
      radius bound of -L_h, so dt_max = 2 / sqrt(rho),
      N_t = ceil(T_f / (cfl * dt_max)) and dt = T_f / N_t, which lands on T_f
      exactly.  ``rho`` replaces the box bound (a mapped grid passes its own).
    * Trapezoid weights sigma_0 = sigma_{N_t} = dt/2, sigma_n = dt otherwise;
      c_n = (2/T_f) sigma_n (cos(omega t^n) - alpha_d/2) (eq. filterQuadrature),
      or with 1/4 in place of alpha_d/2 when ``filter_const == "quarter"``
      (the continuous filter of eq. waveHoltzFilterStep).
    * ``adjust_omega`` replaces omega by the adjusted frequency everywhere
      (eq. adjustedOmega); omega dt and alpha_d are unchanged by it.
    """
    om = omega_adjusted(omega, n_its) if adjust_omega else float(omega)
    t_final = n_p * 2.0 * math.pi / om
    if ts == "implicit":
        n_t = n_p * n_its
    elif ts == "explicit":
        dt_max = 2.0 / math.sqrt(spectral_radius_bound(h, order) if rho is None else rho)
        n_t = int(math.ceil(t_final / (cfl * dt_max)))
    else:
        raise ValueError("ts must be 'explicit' or 'implicit'")
    dt = t_final / n_t
    ad = alpha_d(om, dt)
    shift = ad / 2.0 if filter_const == "alpha_d" else 0.25
    c = np.empty(n_t + 1)
    for k in range(n_t + 1):
        sigma = dt / 2.0 if (k == 0 or k == n_t) else dt
        c[k] = (2.0 / t_final) * sigma * (math.cos(om * k * dt) - shift)
    return TimePlan(omega=om, t_final=t_final, n_t=n_t, dt=dt, alpha_d=ad, c=c, ts=ts)


def beta_continuous(lam, omega: float, n_p: int = 1):
    """Continuous filter function in three-sinc form (eq. filterThreeSincs),
    beta = sinc((omega-lam) T_f) + sinc((omega+lam) T_f) - sinc(lam T_f)/2,
    sinc(x) = sin(x)/x."""
    t_f = n_p * 2.0 * np.pi / omega
    lam = np.asarray(lam, dtype=np.float64)

    def sinc(x):
        x = np.asarray(x, dtype=np.float64)
        out = np.ones_like(x)
        nz = x != 0.0
        out[nz] = np.sin(x[nz]) / x[nz]
        return out

    return sinc((omega - lam) * t_f) + sinc((omega + lam) * t_f) - 0.5 * sinc(lam * t_f)


def lambda_tilde_implicit(lam, dt: float):
    """Implicit time correction (eq. discreteCorr):
    (2/dt) asin((lam dt / 2) / sqrt(1 + (lam dt)^2 / 2))."""
    lam = np.asarray(lam, dtype=np.float64)
    x = lam * dt
    return (2.0 / dt) * np.arcsin(0.5 * x / np.sqrt(1.0 + 0.5 * x * x))


def lambda_tilde_explicit(lam, dt: float):
    """Explicit time correction (eq. discreteExplicitLambdaTilde): (2/dt) asin(lam dt / 2)."""
    lam = np.asarray(lam, dtype=np.float64)
    return (2.0 / dt) * np.arcsin(lam * dt / 2.0)


def beta_discrete(lam_t, plan: TimePlan):
    """Discrete filter (eq. betad): sum_n c_n cos(lam~ t^n)."""
    lam_t = np.asarray(lam_t, dtype=np.float64)
    t = np.arange(plan.n_t + 1) * plan.dt
    return np.tensordot(np.cos(np.multiply.outer(lam_t, t)), plan.c, axes=([-1], [0]))


def beta_corrected(mu, plan: TimePlan):
    """Time-corrected discrete filter (eq. correctedBeta) at mu = lambda_h^2:
    the value by which one wave-solve multiplies that eigenvector."""
    lam = np.sqrt(np.asarray(mu, dtype=np.float64))
    if plan.ts == "implicit":
        lt = lambda_tilde_implicit(lam, plan.dt)
    else:
        lt = lambda_tilde_explicit(lam, plan.dt)
    return beta_discrete(lt, plan)


def box_eigenvalues(length: Sequence[float], lam_max: float) -> np.ndarray:
    """Frequencies lambda = pi sqrt(sum_d (m_d / L_d)^2), m_d >= 1, of the
    continuous Dirichlet Laplacian on the box, all those <= lam_max (with
    multiplicity), ascending."""
    ranges = [np.arange(1, int(np.floor(lam_max * L / np.pi)) + 1) for L in length]
    if any(r.size == 0 for r in ranges):
        return np.zeros(0)
    grids = np.meshgrid(*ranges, indexing="ij")
    s = np.zeros_like(grids[0], dtype=np.float64)
    for g, L in zip(grids, length):
        s = s + (g / L) ** 2
    lam = np.pi * np.sqrt(s.ravel())
    return np.sort(lam[lam <= lam_max])


def lobe_count(length: Sequence[float], omega: float, n_p: int, beta_r: float) -> int:
    """Number of box eigenvalues (with multiplicity) whose continuous filter
    value beta(lambda; omega, N_p) (eq. filterThreeSincs) is at least beta_r.
    For beta_r >= 0.5 only the main lobe, |lambda - omega| < omega / 2, qualifies."""
    lam = box_eigenvalues(length, 1.5 * omega)
    return int(np.sum(beta_continuous(lam, omega, n_p) >= beta_r))


def choose_periods(length: Sequence[float], omega: float, k: int, beta_r: float = 0.8, np_max: int = 256):
    """Number of filter periods for k wanted eigenpairs (Sec. "Changing the
    number of filter periods", Sec. "Estimating the EigenWave convergence
    rate"): the main lobe narrows like 1/N_p, the simultaneous-iteration rate
    beta(1 + 2 dw)/beta(1 + dw) at the lobe's edge beta_r hardly depends on
    N_p, and the best runs keep about the wanted eigenvalues above beta ~ 0.8.
    Reading: the largest N_p <= np_max whose lobe {beta >= beta_r} still holds
    at least k eigenvalues (1 if even N_p = 1 holds fewer).  Returns
    (N_p, eigenvalues in that lobe)."""
    best = 1
    for n_p in range(1, np_max + 1):
        if lobe_count(length, omega, n_p, beta_r) >= k:
            best = n_p
        else:
            break
    return best, lobe_count(length, omega, best, beta_r)
