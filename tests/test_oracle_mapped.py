"""Pins of the curvilinear-grid oracle (oracle/mapped.py) against what the
mathematics fixes: the box operator for a rotated rectangle, exactness on
quadratics for affine maps (cross terms included), second-order convergence
to the continuous Laplacian and to the Dirichlet spectrum of an annulus
sector (Bessel cross-product roots), self-adjointness in the J-weighted inner
product, and S phi = beta(lambda) phi for discrete eigenvectors."""
import math

import numpy as np
import pytest
from scipy import linalg, optimize, special

import synthetic as syn
from oracle import discrete as D
from oracle import mapped as Mp
from oracle import wave as Wv


def _nodes(xy):
    """Node coordinates incl. walls (shape (n2 + 2, n1 + 2))."""
    return xy[0][1:-1, 1:-1], xy[1][1:-1, 1:-1]


def test_rotated_rectangle_is_the_box_operator():
    n, L = (7, 5), (1.3, 0.8)
    xy = syn.mapped_coords("affine", *n, len1=L[0], len2=L[1], phi=0.7)
    h = D.spacing(n, L)
    A = Mp.laplacian_matrix(xy)
    B = D.laplacian_matrix(n, h, 2)
    assert np.max(np.abs(A - B)) <= 1e-12 * np.max(np.abs(B))
    rho_box = D.spectral_radius_bound(h, 2)
    assert abs(Mp.spectral_radius_bound(xy) - rho_box) <= 1e-12 * rho_box
    assert np.allclose(Mp.weights(xy), L[0] * L[1], rtol=1e-13)
    plan = Mp.time_plan(xy, 11.0, cfl=0.5)
    ref = D.time_plan(h, 2, 11.0, "explicit", cfl=0.5)
    assert plan.n_t == ref.n_t and abs(plan.dt - ref.dt) <= 1e-15 * ref.dt


@pytest.mark.parametrize("shear,phi", [(0.4, 0.3), (-0.6, 1.1)])
def test_affine_maps_exact_on_quadratics(shear, phi):
    # second differences are exact for quadratics, so L_h q = Laplacian q
    xy = syn.mapped_coords("affine", 9, 6, len1=1.2, len2=0.7, phi=phi, shear=shear)
    X, Y = _nodes(xy)
    for (a, b, c, d, e), lap in [((0.3, -0.2, 0.7, 1.0, -2.0), 2.0), ((0.0, 1.0, 0.0, 0.0, 0.0), 0.0),
                                 ((1.0, 0.0, -1.0, 0.5, 0.25), 0.0)]:
        U = a * X * X + b * X * Y + c * Y * Y + d * X + e * Y + 0.5
        got = Mp.apply_laplacian_full(U, xy)
        assert np.max(np.abs(got - lap)) <= 1e-9, (a, b, c)


def test_nine_weights_reproduce_the_operator():
    xy = syn.mapped_coords("skew", 8, 7, eps=0.2)
    rng = np.random.default_rng(3)
    U = rng.standard_normal((9, 10))
    w = Mp.stencil(xy)
    acc = sum(wk * Mp._at(U, di, dj) for (di, dj), wk in w.items())
    got = Mp.apply_laplacian_full(U, xy)
    assert np.max(np.abs(acc / Mp.weights(xy) - got)) <= 1e-11 * np.max(np.abs(got))


@pytest.mark.parametrize("kind,params", [("skew", {"eps": 0.15, "len1": 1.1}),
                                         ("annulus", {"a": 0.5, "b": 1.0, "theta0": 0.5 * math.pi})])
def test_second_order_convergence_to_the_laplacian(kind, params):
    errs = []
    for n in (33, 67, 135):
        xy = syn.mapped_coords(kind, n, n, **params)
        X, Y = _nodes(xy)
        U = np.sin(1.3 * X + 0.4) * np.cos(0.7 * Y - 0.2)
        exact = -(1.3 ** 2 + 0.7 ** 2) * U[1:-1, 1:-1]
        errs.append(np.max(np.abs(Mp.apply_laplacian_full(U, xy) - exact)))
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.4 < r < 4.6 for r in rates), (errs, rates)


def test_self_adjoint_in_the_J_weighted_product():
    xy = syn.mapped_coords("skew", 9, 7, eps=0.2, len2=0.8)
    A = Mp.laplacian_matrix(xy)
    K = Mp.weights(xy).ravel()[:, None] * A
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))
    ev = linalg.eigh(-K, np.diag(Mp.weights(xy).ravel()), eigvals_only=True)
    assert ev[0] > 0.0
    assert ev[-1] <= Mp.spectral_radius_bound(xy) * (1 + 1e-12)
    # the plain eigenvalues of L_h are the same (real) numbers
    plain = np.sort(-np.linalg.eigvals(A).real)
    assert np.allclose(plain, ev, rtol=1e-9)


def _sector_eigenvalues(a, b, th0, count):
    """Lowest Dirichlet eigenvalues k^2 of the annulus sector a < rho < b,
    0 < theta < th0: modes sin(m pi theta / th0) Z_nu(k rho), nu = m pi / th0,
    with J_nu(k a) Y_nu(k b) - J_nu(k b) Y_nu(k a) = 0."""
    out = []
    for m in range(1, 8):
        nu = m * math.pi / th0
        f = lambda k: special.jv(nu, k * a) * special.yv(nu, k * b) - special.jv(nu, k * b) * special.yv(nu, k * a)
        ks = np.linspace(0.5, 40.0, 8000)
        vals = f(ks)
        for i in range(len(ks) - 1):
            if vals[i] * vals[i + 1] < 0:
                out.append(optimize.brentq(f, ks[i], ks[i + 1], xtol=1e-14) ** 2)
    out.sort()
    return np.array(out[:count])


def test_annulus_sector_spectrum_converges():
    a, b, th0 = 0.5, 1.0, 0.5 * math.pi
    exact = _sector_eigenvalues(a, b, th0, 4)
    errs = []
    for n in (15, 31):
        xy = syn.mapped_coords("annulus", n, n, a=a, b=b, theta0=th0)
        A = Mp.laplacian_matrix(xy)
        Wt = Mp.weights(xy).ravel()
        mu = linalg.eigh(-(Wt[:, None] * A), np.diag(Wt), eigvals_only=True, subset_by_index=[0, 3])
        errs.append(np.abs(mu - exact) / exact)
    assert np.all(errs[1] < 1e-2), errs
    ratio = errs[0] / errs[1]
    assert np.all((ratio > 3.6) & (ratio < 4.4)), (errs, ratio)


def test_filter_on_rotated_rectangle_matches_box_oracle():
    n, L = (9, 7), (1.0, 0.75)
    xy = syn.mapped_coords("affine", *n, len1=L[0], len2=L[1], phi=-0.4)
    h = D.spacing(n, L)
    plan = Mp.time_plan(xy, 10.0, cfl=0.5)
    v = syn.start_vector(5, n[0] * n[1]).reshape(n[1], n[0])
    got = Mp.apply_filter_explicit(v, xy, plan)
    ref = Wv.apply_filter(v, h, 2, plan)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_filter_on_discrete_eigenvectors():
    xy = syn.mapped_coords("skew", 10, 8, eps=0.2)
    A = Mp.laplacian_matrix(xy)
    Wt = Mp.weights(xy).ravel()
    mu, V = linalg.eigh(-(Wt[:, None] * A), np.diag(Wt))
    plan = Mp.time_plan(xy, 9.0, cfl=0.5)
    for k in (0, 3, 17, len(mu) - 1):
        phi = V[:, k].reshape(8, 10)
        got = Mp.apply_filter_explicit(phi, xy, plan)
        beta = float(D.beta_corrected(mu[k], plan))
        assert np.max(np.abs(got - beta * phi)) <= 1e-11 * np.max(np.abs(phi)), k


def test_sparse_operator_equals_the_stencil_form():
    xy = syn.mapped_coords("annulus", 11, 9, a=0.4, b=1.0, theta0=1.3)
    A = Mp.laplacian_sparse(xy).toarray()
    assert np.max(np.abs(A - Mp.laplacian_matrix(xy))) <= 1e-12 * np.max(np.abs(A))


def test_implicit_on_rotated_rectangle_matches_box_oracle():
    n, L = (9, 7), (1.0, 0.75)
    xy = syn.mapped_coords("affine", *n, len1=L[0], len2=L[1], phi=0.9)
    h = D.spacing(n, L)
    plan = Mp.implicit_plan(xy, 12.0)
    ref_plan = D.time_plan(h, 2, 12.0, "implicit", n_its=10, adjust_omega=True)
    assert plan.n_t == ref_plan.n_t and plan.dt == ref_plan.dt
    b = syn.start_vector(7, n[0] * n[1]).reshape(n[1], n[0])
    x = Mp.solve_implicit_exact(b, xy, plan.dt)
    assert np.max(np.abs(x - Wv.solve_implicit_exact(b, h, 2, plan.dt))) <= 1e-12 * np.max(np.abs(x))
    got = Mp.apply_filter_implicit(b, xy, plan)
    ref = Wv.apply_filter(b, h, 2, plan)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_implicit_filter_on_discrete_eigenvectors():
    xy = syn.mapped_coords("skew", 10, 8, eps=0.2)
    A = Mp.laplacian_matrix(xy)
    Wt = Mp.weights(xy).ravel()
    mu, V = linalg.eigh(-(Wt[:, None] * A), np.diag(Wt))
    plan = Mp.implicit_plan(xy, 9.0)
    # M phi = (1 + a mu) phi
    phi = V[:, 4].reshape(8, 10)
    x = Mp.solve_implicit_exact(phi, xy, plan.dt)
    assert np.max(np.abs(x - phi / (1 + 0.5 * plan.dt ** 2 * mu[4]))) <= 1e-12 * np.max(np.abs(phi))
    for k in (0, 4, 30, len(mu) - 1):
        phi = V[:, k].reshape(8, 10)
        got = Mp.apply_filter_implicit(phi, xy, plan)
        beta = float(D.beta_corrected(mu[k], plan))
        assert np.max(np.abs(got - beta * phi)) <= 1e-11 * np.max(np.abs(phi)), k
