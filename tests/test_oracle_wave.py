"""Pins of oracle/wave.py: S on sine modes equals the discrete filter function,
dense S is symmetric with the predicted spectrum, exact solves agree."""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from oracle import wave as W


CASES = [
    # n, length, omega, ts, n_p, filter_const
    ((12, 12), (1.0, 1.0), 9.0, "explicit", 1, "alpha_d"),
    ((12, 12), (1.0, 1.0), 9.0, "implicit", 1, "alpha_d"),
    ((10, 13), (0.8, 1.5), 14.0, "explicit", 2, "quarter"),
    ((10, 13), (0.8, 1.5), 14.0, "implicit", 2, "quarter"),
    ((6, 7, 5), (1.0, 1.1, 0.9), 8.0, "explicit", 1, "alpha_d"),
    ((6, 7, 5), (1.0, 1.1, 0.9), 8.0, "implicit", 1, "alpha_d"),
]


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("case", CASES)
def test_filter_on_sine_modes_equals_corrected_beta(order, case):
    """S phi_m = beta~_d(mu_m) phi_m (eqs. betad, correctedBeta with the
    explicit or implicit time correction), for several modes."""
    n, length, omega, ts, n_p, fc = case
    h = D.spacing(n, length)
    plan = D.time_plan(h, order, omega, ts, cfl=0.5, n_its=10, n_p=n_p,
                       adjust_omega=(ts == "implicit"), filter_const=fc)
    modes_list = [tuple(1 + (j * (d + 2)) % k for d, k in enumerate(n)) for j in range(4)]
    for modes in modes_list:
        phi = D.sine_mode(modes, n)
        Sphi = W.apply_filter(phi, h, order, plan)
        mu = D.mu_closed_form(modes, n, h, order)
        beta = float(D.beta_corrected(mu, plan))
        assert np.max(np.abs(Sphi - beta * phi)) <= 2e-14 * max(1.0, np.max(np.abs(phi)))


@pytest.mark.parametrize("ts", ["explicit", "implicit"])
@pytest.mark.parametrize("order", [2, 4])
def test_dense_filter_operator_spectrum(ts, order):
    """Brute force on a 5x4 grid: the assembled S is symmetric and its
    eigenvalues are beta~_d over all closed-form mu."""
    n = (5, 4)
    h = D.spacing(n, (1.0, 0.9))
    plan = D.time_plan(h, order, 7.0, ts, cfl=0.7, n_its=8)
    N = 20
    S = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        S[:, j] = W.apply_filter(e.reshape(n[::-1]), h, order, plan).ravel()
    assert np.max(np.abs(S - S.T)) < 1e-14
    ev = np.sort(np.linalg.eigvalsh(0.5 * (S + S.T)))
    want = np.sort(D.beta_corrected(D.mu_all(n, h, order).ravel(), plan))
    assert np.max(np.abs(ev - want)) < 1e-13
    assert ev.min() >= -0.5 - 0.2 and ev.max() <= 1.0 + 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_exact_solve_equals_dense_solve(order):
    n = (7, 5)
    h = D.spacing(n, (1.0, 1.2))
    b = synthetic.uniform_pm1(11, 35).reshape(5, 7)
    dt = 0.05
    x1 = W.solve_implicit_exact(b, h, order, dt)
    x2 = W.solve_implicit_dense(b, h, order, dt)
    assert np.max(np.abs(x1 - x2)) < 1e-13
    # and it solves M x = b with M applied by the stencil
    from oracle.mg import apply_M
    assert np.max(np.abs(apply_M(x1, h, order, 0.5 * dt * dt) - b)) < 1e-12


def test_explicit_first_steps_written_out():
    """First two levels of the explicit scheme, against eqs. explicitStep1 and
    explicitScheme written out with the dense L."""
    n = (4, 3)
    h = D.spacing(n, (1.0, 1.0))
    plan = D.time_plan(h, 2, 6.0, "explicit", cfl=0.4)
    v = synthetic.uniform_pm1(3, 12)
    L = D.laplacian_matrix(n, h, 2)
    _, levels = W.apply_filter(v.reshape(3, 4), h, 2, plan, return_levels=True)
    w1 = v + 0.5 * plan.dt ** 2 * (L @ v)
    w2 = 2 * w1 - v + plan.dt ** 2 * (L @ w1)
    assert np.allclose(levels[1].ravel(), w1, atol=1e-14)
    assert np.allclose(levels[2].ravel(), w2, atol=1e-14)


def test_implicit_scheme_written_out():
    """Levels of the implicit scheme satisfy M W^{n+1} = 2 W^n - M W^{n-1}
    and M W^1 = W^0 (eqs. implicitScheme, implicitStep1)."""
    n = (4, 3)
    h = D.spacing(n, (1.0, 1.0))
    plan = D.time_plan(h, 4, 6.0, "implicit", n_its=6)
    v = synthetic.uniform_pm1(4, 12)
    L = D.laplacian_matrix(n, h, 4)
    M = np.eye(12) - 0.5 * plan.dt ** 2 * L
    _, lv = W.apply_filter(v.reshape(3, 4), h, 4, plan, return_levels=True)
    lv = [x.ravel() for x in lv]
    assert np.allclose(M @ lv[1], lv[0], atol=1e-13)
    for k in range(1, plan.n_t):
        assert np.allclose(M @ lv[k + 1], 2 * lv[k] - M @ lv[k - 1], atol=1e-12)
    acc = sum(plan.c[k] * lv[k] for k in range(plan.n_t + 1))
    assert np.allclose(W.apply_filter(v.reshape(3, 4), h, 4, plan).ravel(), acc, atol=1e-14)
