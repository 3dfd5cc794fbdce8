"""Pins of oracle/discrete.py: closed forms, dense eigensolves, printed paper values."""
import math

import numpy as np
import pytest

from oracle import discrete as D
from tests.conftest import load_golden


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("n,length,modes", [
    ((9, 7), (1.0, 1.3), (2, 3)),
    ((16, 11), (0.7, 1.9), (5, 1)),
    ((6, 5, 7), (1.0, 0.8, 1.2), (1, 2, 3)),
])
def test_laplacian_symbol_on_sine_modes(order, n, length, modes):
    """L_h phi = -mu phi with mu from the stencil symbol (not from the oracle's
    own closed-form routine: the symbol is re-derived here with cosines)."""
    h = D.spacing(n, length)
    phi = D.sine_mode(modes, n)
    Lphi = D.apply_laplacian(phi, h, order)
    mu = 0.0
    for m, k, hd in zip(modes, n, h):
        th = m * math.pi / (k + 1)
        if order == 2:
            mu += (2.0 - 2.0 * math.cos(th)) / hd ** 2
        else:
            mu += (30.0 - 32.0 * math.cos(th) + 2.0 * math.cos(2 * th)) / (12.0 * hd ** 2)
    assert np.max(np.abs(Lphi + mu * phi)) <= 1e-12 * mu
    assert abs(D.mu_closed_form(modes, n, h, order) - mu) <= 1e-13 * mu


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("n", [(6, 6), (5, 7), (4, 4, 4), (1, 3), (2, 5)])
def test_dense_eigh_matches_closed_form(order, n):
    length = tuple(1.0 + 0.1 * d for d in range(len(n)))
    h = D.spacing(n, length)
    A = D.laplacian_matrix(n, h, order)
    assert np.allclose(A, A.T, atol=0, rtol=0) or np.max(np.abs(A - A.T)) < 1e-9 * np.max(np.abs(A))
    ev = np.sort(np.linalg.eigvalsh(-0.5 * (A + A.T)))
    cf = np.sort(D.mu_all(n, h, order).ravel())
    assert np.max(np.abs(ev - cf)) <= 1e-11 * cf.max()


def test_order4_stencil_brute_force_small():
    """Order 4 with odd-reflection ghosts, written out for one row of a 1-D-like grid."""
    n = (5, 1)
    h = (0.25, 0.5)
    u = np.array([[1.0, -2.0, 0.5, 3.0, -1.0]])
    Lu = D.apply_laplacian(u, h, 4)
    ext = [-u[0, 0], 0.0] + list(u[0]) + [0.0, -u[0, -1]]
    for i in range(5):
        j = i + 2
        want = (-ext[j - 2] + 16 * ext[j - 1] - 30 * ext[j] + 16 * ext[j + 1] - ext[j + 2]) / (12 * h[0] ** 2)
        # y direction: single interior point, neighbours are the wall (0) and ghosts (-u)
        want += (-(-u[0, i]) + 0 - 30 * u[0, i] + 0 - (-u[0, i])) / (12 * h[1] ** 2)
        assert abs(Lu[0, i] - want) < 1e-12 * max(1.0, abs(want))


def _closed_form_lambdas(n, order, lo, hi):
    h = D.spacing(n, (1.0,) * len(n))
    lam = np.sqrt(np.sort(D.mu_all(n, h, order).ravel()))
    return lam[(lam >= lo) & (lam <= hi)]


def test_paper_square128_eigenvalues():
    """Table tab:square128Order2 lists 27 eigenvalues with multiplicity; the
    closed-form discrete eigenvalues in the same range are exactly that list."""
    printed = np.array(load_golden("square128_order2_lambda.txt"))
    lam = _closed_form_lambdas((127, 127), 2, 7.0, 20.1052)
    assert lam.size == printed.size == 27
    assert np.max(np.abs(lam - printed)) < 6e-7


def test_paper_box2_eigenvalues():
    """Table tab:box2Order2: all but the last printed value carry their full
    multiplicity; the last (multiplicity 6) is printed once."""
    printed = np.array(load_golden("box2_order2_lambda.txt"))
    lam = _closed_form_lambdas((19, 19, 19), 2, 5.0, 14.2053)
    assert lam.size == 26 + 6
    assert np.max(np.abs(lam[:26] - printed[:26])) < 6e-7
    assert np.max(np.abs(lam[26:] - printed[26])) < 6e-7


def test_continuous_beta_sinc_form_vs_quadrature():
    """eq. filterThreeSincs equals the integral of eq. filterFunction."""
    omega = 15.0
    for n_p in (1, 2):
        tf = n_p * 2 * math.pi / omega
        t = np.linspace(0.0, tf, 400001)
        for lam in (0.0, 3.0, 7.0, 14.0, 15.0, 22.0, 40.0):
            f = (np.cos(omega * t) - 0.25) * np.cos(lam * t)
            quad = 2.0 / tf * np.trapezoid(f, t)
            assert abs(quad - D.beta_continuous(lam, omega, n_p)) < 1e-9
    lam = np.linspace(0, 200, 20001)
    b = D.beta_continuous(lam, omega)
    assert b.min() >= -0.5 - 1e-12 and b.max() <= 1.0 + 1e-12
    assert abs(D.beta_continuous(0.0, omega) + 0.5) < 1e-15
    assert abs(D.beta_continuous(omega, omega) - 1.0) < 1e-15


@pytest.mark.parametrize("n_its", [5, 10, 15])
def test_alpha_d_makes_discrete_filter_peak_at_omega(n_its):
    """With alpha_d (eq. alphad) the discrete filter of eq. betad, as a
    function of a continuous lambda, is 1 with zero slope at lambda = omega."""
    omega = 12.0
    plan = D.time_plan((0.01, 0.01), 2, omega, "implicit", n_its=n_its)
    f = lambda lam: float(D.beta_discrete(lam, plan))
    assert abs(f(omega) - 1.0) < 1e-13
    d = 1e-4
    slope = (f(omega + d) - f(omega - d)) / (2 * d)
    assert abs(slope) < 1e-8
    plan_q = D.time_plan((0.01, 0.01), 2, omega, "implicit", n_its=n_its, filter_const="quarter")
    fq = lambda lam: float(D.beta_discrete(lam, plan_q))
    assert abs((fq(omega + d) - fq(omega - d)) / (2 * d)) > 1e-3


def test_alpha_d_value_at_ten_steps():
    plan = D.time_plan((0.01, 0.01), 2, 7.0, "implicit", n_its=10)
    assert abs(plan.alpha_d - 1.0 / math.sqrt(5.0)) < 1e-15


def test_adjusted_omega_peaks_corrected_filter_at_omega():
    """eq. adjustedOmega: with omega~ the time-corrected implicit filter
    (eq. correctedBeta) reaches its maximum 1 at lambda = omega."""
    omega = 12.0
    assert abs(D.omega_adjusted(1.0, 10) - 0.91442129) < 1e-8
    plan = D.time_plan((0.01, 0.01), 2, omega, "implicit", n_its=10, adjust_omega=True)
    lam = np.linspace(0.8 * omega, 1.2 * omega, 40001)
    b = D.beta_corrected(lam ** 2, plan)
    assert abs(lam[np.argmax(b)] - omega) < 2e-4
    assert abs(b.max() - 1.0) < 1e-9
    # Without the adjustment the peak sits above omega (the paper's observation).
    plan0 = D.time_plan((0.01, 0.01), 2, omega, "implicit", n_its=10)
    assert lam[np.argmax(D.beta_corrected(lam ** 2, plan0))] > 1.05 * omega


def test_time_plan_small_explicit_square():
    """64x64 interior, h = 1/65, order 2, CFL 0.5, omega = 15."""
    h = D.spacing((64, 64), (1.0, 1.0))
    plan = D.time_plan(h, 2, 15.0, "explicit", cfl=0.5)
    assert plan.n_t == 78
    assert abs(plan.dt - 5.370244e-3) < 1e-9
    assert abs(plan.alpha_d / 2 - 0.249594) < 1e-6
    # stability: dt * sqrt(rho) <= 2 * CFL
    assert plan.dt * math.sqrt(D.spectral_radius_bound(h, 2)) <= 1.0 + 1e-15
    # trapezoid weights sum to T_f
    w = plan.c / (2.0 / plan.t_final) / (np.cos(plan.omega * np.arange(79) * plan.dt) - plan.alpha_d / 2)
    assert abs(w.sum() - plan.t_final) < 1e-12


def test_lambda_tilde_matches_mode_recurrences():
    """eqs. discreteCorr and discreteExplicitLambdaTilde: the scalar mode
    recurrences of the two schemes produce cos(lambda~ t^n)."""
    dt = 0.07
    for lam in (0.5, 3.0, 11.0, 25.0):
        # implicit: (1 + a l^2) (w+ + w-) = 2 w, a = dt^2/2, w1 = w0 / (1 + a l^2)
        a = 0.5 * dt * dt * lam * lam
        w = [1.0, 1.0 / (1 + a)]
        for n in range(1, 30):
            w.append(2 * w[n] / (1 + a) - w[n - 1])
        lt = D.lambda_tilde_implicit(lam, dt)
        assert max(abs(w[n] - math.cos(lt * n * dt)) for n in range(31)) < 1e-12
        if lam * dt < 2:
            w = [1.0, 1.0 - 0.5 * (lam * dt) ** 2]
            for n in range(1, 30):
                w.append(2 * w[n] - w[n - 1] - (lam * dt) ** 2 * w[n])
            lt = D.lambda_tilde_explicit(lam, dt)
            assert max(abs(w[n] - math.cos(lt * n * dt)) for n in range(31)) < 1e-11


def test_box_eigenvalues_match_brute_force_and_weyl():
    """Enumeration of pi sqrt(sum (m/L)^2) against a plain double loop, and the
    two-term Weyl law N(L) ~ A L^2/(4 pi) - P L/(4 pi) for a rectangle."""
    import itertools
    length = (1.0, 0.7)
    lam = D.box_eigenvalues(length, 60.0)
    brute = sorted(np.pi * np.hypot(m / length[0], n / length[1])
                   for m, n in itertools.product(range(1, 40), range(1, 40))
                   if np.pi * np.hypot(m / length[0], n / length[1]) <= 60.0)
    assert np.allclose(lam, brute, rtol=0, atol=1e-12)
    big = D.box_eigenvalues(length, 400.0)
    A, P = length[0] * length[1], 2 * (length[0] + length[1])
    weyl = A * 400.0 ** 2 / (4 * np.pi) - P * 400.0 / (4 * np.pi)
    assert abs(big.size - weyl) / weyl < 0.01
    cube = D.box_eigenvalues((1.0, 1.0, 1.0), 20.0)
    assert cube[0] == pytest.approx(np.pi * np.sqrt(3)) and np.sum(np.isclose(cube, np.pi * np.sqrt(6))) == 3


def test_filter_lobe_width_and_rate_are_those_of_the_convergence_estimate():
    """beta(1 + dw) = 0.8 gives dw N_p nearly independent of N_p, and the
    simultaneous-iteration rate beta(1 + 2 dw) / beta(1 + dw) about 0.4 (the
    values the convergence-rate estimate quotes for beta_r ~ 0.8)."""
    from scipy.optimize import brentq
    widths, rates = [], []
    for n_p in (1, 2, 4, 8):
        dw = brentq(lambda d: D.beta_continuous(1 + d, 1.0, n_p) - 0.8, 1e-9, 0.3 / n_p)
        widths.append(dw * n_p)
        rates.append(float(D.beta_continuous(1 + 2 * dw, 1.0, n_p)) / 0.8)
    assert max(widths) - min(widths) < 0.02 * widths[0]
    assert all(0.38 < r < 0.45 for r in rates)


def test_choose_periods_keeps_k_eigenvalues_in_the_lobe():
    length = (1.0, 1.0)
    omega = 36.5769
    n_p, n_lobe = D.choose_periods(length, omega, 8)
    assert n_lobe >= 8
    assert D.lobe_count(length, omega, n_p + 1, 0.8) < 8
    assert 4 <= n_p <= 16
    # more wanted eigenpairs -> fewer periods; too many for any N_p -> 1
    assert D.choose_periods(length, omega, 24)[0] < n_p
    assert D.choose_periods(length, omega, 10 ** 6)[0] == 1
