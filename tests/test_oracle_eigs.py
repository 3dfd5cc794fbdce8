"""Pins of oracle/eigs.py: Arnoldi relation, and eigenpairs against the
closed-form discrete spectrum (with multiplicity)."""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from oracle import eigs as E
from oracle import wave as W


def _ops(P):
    h = D.spacing(P.n, P.length)
    plan = D.time_plan(h, P.order, P.omega, P.ts, cfl=P.cfl, n_its=P.n_its, n_p=P.n_p,
                       adjust_omega=P.adjust_omega, filter_const=P.filter_const)
    shape = P.n[::-1]
    S = lambda v: W.apply_filter(v.reshape(shape), h, P.order, plan).ravel()
    L = lambda v: D.apply_laplacian(v.reshape(shape), h, P.order).ravel()
    return h, plan, S, L


def wanted_closed_form(P, plan, h, k):
    """Closed-form mu of the k largest beta~_d, plus the k-th beta."""
    mu = D.mu_all(P.n, h, P.order).ravel()
    beta = D.beta_corrected(mu, plan)
    idx = np.argsort(-np.abs(beta), kind="stable")
    return mu[idx[:k]], np.abs(beta[idx[k - 1]]), mu, beta


def test_arnoldi_relation_and_orthogonality():
    rng_v = synthetic.uniform_pm1(5, 40)
    A = np.diag(np.linspace(1, 3, 40)) + 0.01 * np.outer(np.arange(40) % 3, np.arange(40) % 5)
    V, H = E.arnoldi(lambda x: A @ x, rng_v, 10)
    # plain MGS loses orthogonality in proportion to the conditioning of the Krylov basis
    assert np.max(np.abs(V.T @ V - np.eye(11))) < 1e-9
    assert np.max(np.abs(A @ V[:, :10] - V @ H)) < 1e-12
    assert np.max(np.abs(np.tril(H, -2))) == 0.0


def test_arnoldi_on_filter_operator_is_symmetric_lanczos():
    """S is symmetric, so the Arnoldi matrix is tridiagonal up to rounding."""
    P = synthetic.config_small_explicit()
    h, plan, S, L = _ops(P)
    V, H = E.arnoldi(S, synthetic.start_vector(1, P.n_active), 8)
    assert np.max(np.abs(np.triu(H[:8, :8], 2))) < 1e-12
    assert np.max(np.abs(np.diag(H, 1) - np.diag(H, -1)[:7])) < 1e-12


def test_eigs_small_explicit_square_matches_closed_form():
    """64^2, order 2, explicit, omega = 15, k = 4, m = 16: the 4 wanted are two
    double eigenvalues; the solver must return both copies of each."""
    P = synthetic.config_small_explicit()
    h, plan, S, L = _ops(P)
    r = E.eigs(S, L, synthetic.start_vector(P.seed, P.n_active), P.k, P.m,
               lambda p: synthetic.start_vector(P.seed + p, P.n_active))
    want, beta_k, mu_all, beta_all = wanted_closed_form(P, plan, h, P.k)
    got = np.sort(r.mu[:P.k])
    assert np.max(np.abs(got - np.sort(want)) / np.sort(want)) < 1e-10
    # every returned pair is a true discrete eigenpair
    for mu in r.mu:
        assert np.min(np.abs(mu_all - mu)) / mu < 1e-10
    assert np.all(r.res <= 1e-8)
    # all eigenvalues with beta at least the k-th are present with multiplicity
    band = np.sort(mu_all[np.abs(beta_all) >= beta_k * (1 - 1e-10)])
    for mu in band:
        assert np.sum(np.abs(r.mu - mu) < 1e-8 * mu) == np.sum(np.abs(band - mu) < 1e-8 * mu)
    # eigenvectors: unit norm, orthogonal, and beta matches the closed form
    assert np.max(np.abs(r.Y.T @ r.Y - np.eye(r.Y.shape[1]))) < 1e-10
    b_cf = D.beta_corrected(r.mu, plan)
    assert np.max(np.abs(b_cf - r.beta)) < 1e-10


def test_eigs_cube_triple_eigenvalues_implicit():
    """11^3 cube, order 2, implicit: the wanted band holds 3-fold eigenvalues."""
    P = synthetic.Problem(n=(11, 11, 11), length=(1.0, 1.0, 1.0), order=2, omega=8.0,
                          ts="implicit", n_its=10, adjust_omega=True, k=4, m=12, seed=9)
    h, plan, S, L = _ops(P)
    r = E.eigs(S, L, synthetic.start_vector(P.seed, P.n_active), P.k, P.m,
               lambda p: synthetic.start_vector(P.seed + p, P.n_active))
    want, beta_k, mu_all, beta_all = wanted_closed_form(P, plan, h, P.k)
    band = np.sort(mu_all[np.abs(beta_all) >= beta_k * (1 - 1e-10)])
    assert band.size >= 4
    for mu in band:
        assert np.sum(np.abs(r.mu - mu) < 1e-8 * mu) == np.sum(np.abs(band - mu) < 1e-8 * mu)
    assert np.all(r.res <= 1e-8)


def test_power_iteration_top_pair():
    """Alg. 1 on a case whose largest beta is simple: 12 x 9 rectangle."""
    P = synthetic.Problem(n=(12, 9), length=(1.0, 0.77), order=4, omega=5.0, ts="explicit",
                          cfl=0.5, k=1, m=8, seed=3)
    h, plan, S, L = _ops(P)
    mu_all = D.mu_all(P.n, h, P.order).ravel()
    beta = D.beta_corrected(mu_all, plan)
    idx = np.argsort(-np.abs(beta))
    assert abs(beta[idx[0]]) > abs(beta[idx[1]]) * 1.5
    mu, b, v, its = E.power_iteration(S, L, synthetic.start_vector(3, P.n_active), 1e-11)
    assert abs(mu - mu_all[idx[0]]) / mu_all[idx[0]] < 1e-9
    assert abs(b - beta[idx[0]]) < 1e-9


def test_rayleigh_ritz_separates_mixed_vectors():
    """Two exact eigenvectors with different mu, mixed by a rotation: the
    Stage-2 projection recovers both eigenvalues exactly."""
    n = (9, 8)
    h = D.spacing(n, (1.0, 1.0))
    L = lambda v: D.apply_laplacian(v.reshape(8, 9), h, 2).ravel()
    p1 = D.sine_mode((2, 3), n).ravel()
    p2 = D.sine_mode((4, 1), n).ravel()
    p1 /= np.linalg.norm(p1)
    p2 /= np.linalg.norm(p2)
    c, s = np.cos(0.4), np.sin(0.4)
    Y = np.column_stack([c * p1 + s * p2, -s * p1 + c * p2])
    mu, Z, res = E.rayleigh_ritz_L(L, Y)
    want = np.sort([D.mu_closed_form((2, 3), n, h, 2), D.mu_closed_form((4, 1), n, h, 2)])
    assert np.max(np.abs(np.sort(mu) - want) / want) < 1e-13
    assert np.all(res < 1e-12)
