"""Pins of the Neumann-wall oracle (oracle/walls.py) against what the
mathematics fixes: the dense line operators' spectra equal the closed-form
symbols, the sampled sine/cosine modes are exact eigenvectors, the weighted
operator is symmetric, a hand-written boundary row, the continuum limit, the
constant mode of an all-Neumann box, and S phi = beta(lambda~) phi for the
explicit scheme on modes."""
import itertools
import math

import numpy as np
import pytest

from oracle import discrete as D
from oracle import walls as Wl

PAIRS = [("D", "D"), ("D", "N"), ("N", "D"), ("N", "N")]


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("lo,hi", PAIRS)
@pytest.mark.parametrize("n", [5, 12, 33])
def test_line_spectrum_and_modes(order, lo, hi, n):
    h = 0.37
    A = Wl.line_matrix(n, h, order, lo, hi)
    w = np.ones(n)
    if lo == "N":
        w[0] = 0.5
    if hi == "N":
        w[-1] = 0.5
    # weighted symmetry: diag(w) A is symmetric, so A is self-adjoint in <., .>_w
    WA = w[:, None] * A
    assert np.max(np.abs(WA - WA.T)) <= 1e-12 * np.max(np.abs(A))
    # spectrum of the symmetrised operator equals the closed form
    S = np.sqrt(w)[:, None] * A / np.sqrt(w)[None, :]
    ev = np.sort(-np.linalg.eigvalsh(0.5 * (S + S.T)))
    mu = np.sort(Wl.line_mu(n, h, order, lo, hi))
    assert np.max(np.abs(ev - mu)) <= 1e-10 * mu.max()
    # modes are eigenvectors
    P = Wl.line_modes(n, lo, hi)
    mu_u = Wl.line_mu(n, h, order, lo, hi)
    assert np.max(np.abs(A @ P + P * mu_u[None, :])) <= 1e-10 * mu.max()


def test_handwritten_neumann_rows_order4():
    # rows 0 and 1 at a Neumann wall with ghosts u_{-1} = u_1, u_{-2} = u_2
    n, h = 8, 1.0
    A = Wl.line_matrix(n, h, 4, "N", "D") * 12.0
    assert np.allclose(A[0, :3], [-30.0, 32.0, -2.0]) and np.all(A[0, 3:] == 0)
    assert np.allclose(A[1, :4], [16.0, -31.0, 16.0, -1.0]) and np.all(A[1, 4:] == 0)
    # the Dirichlet end keeps the odd-reflection closure of discrete.py
    assert np.allclose(A[-1, -3:], [-1.0, 16.0, -29.0])
    # order 2 at a Neumann wall: (2 u_1 - 2 u_0) / h^2
    B = Wl.line_matrix(n, h, 2, "N", "N")
    assert np.allclose(B[0, :2], [-2.0, 2.0]) and np.allclose(B[-1, -2:], [2.0, -2.0])


@pytest.mark.parametrize("order", [2, 4])
def test_dirichlet_walls_match_discrete(order):
    rng = np.random.default_rng(0)
    n = (7, 5, 4)
    h = D.spacing(n, (1.0, 0.8, 0.6))
    u = rng.standard_normal(n[::-1])
    walls = [("D", "D")] * 3
    assert np.allclose(Wl.apply_laplacian(u, h, order, walls), D.apply_laplacian(u, h, order), atol=1e-12,
                       rtol=0)
    assert Wl.spacing(n, (1.0, 0.8, 0.6), walls) == h


@pytest.mark.parametrize("walls", [[("N", "D"), ("D", "N")], [("N", "N"), ("D", "D")], [("D", "N"), ("N", "N")]])
@pytest.mark.parametrize("order", [2, 4])
def test_box_operator_and_modes(walls, order):
    n = (6, 5)
    h = Wl.spacing(n, (1.0, 0.7), walls)
    A = Wl.laplacian_matrix(n, h, order, walls)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(n[::-1])
    assert np.allclose(A @ u.ravel(), Wl.apply_laplacian(u, h, order, walls).ravel(), atol=1e-10, rtol=0)
    mu = Wl.mu_all(n, h, order, walls)
    for idx in itertools.product(range(n[0]), range(n[1])):
        phi = Wl.mode(idx, n, walls)
        r = Wl.apply_laplacian(phi, h, order, walls) + mu[idx[1], idx[0]] * phi
        assert np.max(np.abs(r)) <= 1e-10 * mu.max()
    wt = Wl.weights(n, walls).ravel()
    WA = wt[:, None] * A
    assert np.max(np.abs(WA - WA.T)) <= 1e-12 * np.max(np.abs(A))


def test_positions_and_spacing():
    # D-N on [0, 1] with 4 points: x = h, 2h, 3h, 4h = 1 (the Neumann wall)
    assert Wl.spacing((4,), (1.0,), [("D", "N")]) == (0.25,)
    assert Wl.spacing((5,), (1.0,), [("N", "N")]) == (0.25,)
    assert Wl.spacing((3,), (1.0,), [("D", "D")]) == (0.25,)


@pytest.mark.parametrize("lo,hi,k", [("N", "N", lambda m: m * math.pi), ("D", "N", lambda m: (m + 0.5) * math.pi),
                                     ("N", "D", lambda m: (m + 0.5) * math.pi)])
@pytest.mark.parametrize("order,rate", [(2, 2.0), (4, 4.0)])
def test_continuum_limit(lo, hi, k, order, rate):
    # mu_h of the first modes approaches the continuous (k_m / L)^2 at O(h^order)
    errs = []
    for n in (33, 65, 129):
        h = Wl.spacing((n,), (1.0,), [(lo, hi)])[0]
        mu = Wl.line_mu(n, h, order, lo, hi)[:4]
        errs.append(max(abs(mu[m] - k(m) ** 2) for m in range(4)))
    slope = math.log(errs[1] / errs[2]) / math.log(2.0)
    assert abs(slope - rate) < 0.15


def test_constant_mode_all_neumann():
    n = (6, 4)
    walls = [("N", "N"), ("N", "N")]
    h = Wl.spacing(n, (1.0, 1.0), walls)
    for order in (2, 4):
        assert np.max(np.abs(Wl.apply_laplacian(np.ones(n[::-1]), h, order, walls))) < 1e-12
        assert Wl.mu_all(n, h, order, walls)[0, 0] == 0.0


@pytest.mark.parametrize("walls", [[("N", "D"), ("D", "D")], [("D", "N"), ("N", "N")]])
@pytest.mark.parametrize("order", [2, 4])
def test_explicit_filter_on_modes(walls, order):
    n = (12, 10)
    h = Wl.spacing(n, (1.0, 0.9), walls)
    plan = D.time_plan(h, order, 9.0, "explicit", cfl=0.5)
    mu = Wl.mu_all(n, h, order, walls)
    for idx in ((0, 0), (2, 3), (5, 1), (11, 9)):
        phi = Wl.mode(idx, n, walls)
        got = Wl.apply_filter_explicit(phi, h, order, walls, plan)
        beta = float(D.beta_corrected(mu[idx[1], idx[0]], plan))
        assert np.max(np.abs(got - beta * phi)) <= 1e-12


@pytest.mark.parametrize("walls", [[("N", "D"), ("D", "N")], [("N", "N"), ("N", "D")], [("D", "D"), ("D", "N")]])
@pytest.mark.parametrize("order", [2, 4])
def test_implicit_exact_solve_and_filter(walls, order):
    n = (7, 6)
    h = Wl.spacing(n, (1.0, 0.8), walls)
    dt = 0.05
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n[::-1])
    A = Wl.laplacian_matrix(n, h, order, walls)
    M = np.eye(A.shape[0]) - 0.5 * dt * dt * A
    want = np.linalg.solve(M, b.ravel())
    got = Wl.solve_implicit_exact(b, h, order, walls, dt).ravel()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    plan = D.time_plan(h, order, 11.0, "implicit", n_its=10, adjust_omega=True)
    mu = Wl.mu_all(n, h, order, walls)
    for idx in ((0, 0), (3, 2), (6, 5)):
        phi = Wl.mode(idx, n, walls)
        got = Wl.apply_filter_implicit(phi, h, order, walls, plan)
        beta = float(D.beta_corrected(mu[idx[1], idx[0]], plan))
        assert np.max(np.abs(got - beta * phi)) <= 1e-12
