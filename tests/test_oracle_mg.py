"""Pins of oracle/mg.py: Gauss-Seidel properties, transfer operators, and
convergence to the exact implicit solve."""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from oracle import mg
from oracle import wave as W


def test_level_sizes():
    assert mg.level_sizes((2047, 2047))[-1] == (1, 1)
    assert len(mg.level_sizes((2047, 2047))) == 11
    assert mg.level_sizes((255, 255, 255))[1] == (127, 127, 127)
    assert mg.level_sizes((64, 64)) == [(64, 64)]
    assert mg.level_sizes((9, 13)) == [(9, 13), (4, 6)]


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("n", [(7, 9), (5, 3, 7), (2, 5)])
def test_diag_matches_dense_matrix(order, n):
    h = D.spacing(n, (1.0,) * len(n))
    a = 0.003
    M = np.eye(int(np.prod(n))) - a * D.laplacian_matrix(n, h, order)
    assert np.allclose(mg.diag_M(n[::-1], h, order, a).ravel(), np.diag(M), rtol=1e-14, atol=0)


def test_order2_red_black_is_gauss_seidel():
    """Order 2: after the red half-sweep the red residual is zero, after the
    black one the black residual is zero (exact GS within each colour), and
    the sweep equals point GS in red-then-black order done one point at a time."""
    n = (7, 6)
    h = D.spacing(n, (1.0, 1.0))
    a = 2e-3
    b = synthetic.uniform_pm1(21, 42).reshape(6, 7)
    x = synthetic.uniform_pm1(22, 42).reshape(6, 7)
    xr = mg.rb_half_sweep(x, b, h, 2, a, 0)
    red = mg.colour_mask(x.shape, 0)
    assert np.max(np.abs(mg.residual(xr, b, h, 2, a)[red])) < 1e-13
    xb = mg.rb_half_sweep(xr, b, h, 2, a, 1)
    assert np.max(np.abs(mg.residual(xb, b, h, 2, a)[~red])) < 1e-13
    # scalar Gauss-Seidel, lexicographic within colours, with the dense matrix
    M = np.eye(42) - a * D.laplacian_matrix(n, h, 2)
    y = x.ravel().copy()
    for colour in (0, 1):
        for idx in range(42):
            i, j = idx % 7, idx // 7
            if (i + j) % 2 == colour:
                y[idx] = (b.ravel()[idx] - M[idx] @ y + M[idx, idx] * y[idx]) / M[idx, idx]
    assert np.max(np.abs(y - xb.ravel())) < 1e-13


def test_order4_half_sweep_uses_old_same_colour_values():
    """Order 4: one half-sweep equals x_i <- (b_i - sum_{j != i} M_ij x_j) / M_ii
    with all x_j taken before the half-sweep, for the points of that colour."""
    n = (6, 5)
    h = D.spacing(n, (1.0, 1.0))
    a = 1e-3
    b = synthetic.uniform_pm1(31, 30).reshape(5, 6)
    x = synthetic.uniform_pm1(32, 30).reshape(5, 6)
    M = np.eye(30) - a * D.laplacian_matrix(n, h, 4)
    for colour in (0, 1):
        got = mg.rb_half_sweep(x, b, h, 4, a, colour).ravel()
        xf = x.ravel()
        for idx in range(30):
            i, j = idx % 6, idx // 6
            if (i + j) % 2 == colour:
                want = (b.ravel()[idx] - M[idx] @ xf + M[idx, idx] * xf[idx]) / M[idx, idx]
            else:
                want = xf[idx]
            assert abs(got[idx] - want) < 1e-13


@pytest.mark.parametrize("n", [(7, 9), (5, 3, 7)])
def test_prolongation_is_scaled_transpose_of_restriction(n):
    coarse = tuple((k - 1) // 2 for k in n)
    rf = synthetic.uniform_pm1(41, int(np.prod(n))).reshape(n[::-1])
    xc = synthetic.uniform_pm1(42, int(np.prod(coarse))).reshape(coarse[::-1])
    lhs = np.sum(mg.restrict_full_weighting(rf) * xc)
    rhs = np.sum(rf * mg.prolong_linear(xc, n[::-1])) / 2 ** len(n)
    assert abs(lhs - rhs) < 1e-13


def test_transfer_operators_exact_on_linear_functions():
    """Full weighting and linear interpolation reproduce linear functions at
    interior points away from the walls (values sampled at x = ih)."""
    nf = (15, 15)
    xs = np.arange(1, 16) / 16.0
    f = xs[None, :] * 2.0 + xs[:, None] * 3.0 + 1.0
    c = mg.restrict_full_weighting(f)
    xc = np.arange(1, 8) / 8.0
    fc = xc[None, :] * 2.0 + xc[:, None] * 3.0 + 1.0
    assert np.max(np.abs(c - fc)) < 1e-14
    p = mg.prolong_linear(fc, nf[::-1])
    assert np.max(np.abs(p[1:-1, 1:-1] - f[1:-1, 1:-1])) < 1e-14


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("n", [(63, 63), (31, 31, 31)])
def test_mg_converges_to_exact_solution(order, n):
    h = D.spacing(n, (1.0,) * len(n))
    plan = D.time_plan(h, order, 30.0, "implicit", n_its=10, adjust_omega=True)
    a = 0.5 * plan.dt ** 2
    hier = mg.Hierarchy(n, h, order, a)
    b = synthetic.uniform_pm1(51, int(np.prod(n))).reshape(n[::-1])
    x, cycles, rel = mg.solve(b, hier, 1e-10)
    assert rel <= 1e-10 and cycles <= 12
    xe = W.solve_implicit_exact(b, h, order, plan.dt)
    # ||x - xe|| <= ||M^{-1}|| ||r|| <= ||r|| (eigenvalues of M are >= 1)
    assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(b) * 1.0000001
    # per-cycle contraction of the residual
    xs = np.zeros_like(b)
    r_prev = np.linalg.norm(b)
    for _ in range(4):
        xs = mg.vcycle(xs, b, hier)
        r = np.linalg.norm(mg.residual(xs, b, h, order, a))
        assert r / r_prev < 0.1
        r_prev = r


def test_single_point_coarsest_is_exact():
    hier = mg.Hierarchy((1, 1), (0.5, 0.5), 4, 0.01)
    b = np.array([[0.7]])
    x = mg.vcycle(np.zeros_like(b), b, hier)
    assert abs(mg.residual(x, b, (0.5, 0.5), 4, 0.01)[0, 0]) < 1e-15


@pytest.mark.parametrize("w", [0.8, 1.15, 1.4])
def test_order2_weighted_red_black_is_point_sor(w):
    """Order 2 with relaxation weight w: the red-black sweep equals point
    successive over-relaxation (SOR) in red-then-black order done one point at
    a time with the dense matrix, y_i <- y_i + w (b_i - (M y)_i) / M_ii."""
    n = (7, 6)
    h = D.spacing(n, (1.0, 1.0))
    a = 2e-3
    b = synthetic.uniform_pm1(23, 42).reshape(6, 7)
    x = synthetic.uniform_pm1(24, 42).reshape(6, 7)
    got = mg.rb_sweep(x, b, h, 2, a, w).ravel()
    M = np.eye(42) - a * D.laplacian_matrix(n, h, 2)
    y = x.ravel().copy()
    for colour in (0, 1):
        for idx in range(42):
            i, j = idx % 7, idx // 7
            if (i + j) % 2 == colour:
                y[idx] = y[idx] + w * (b.ravel()[idx] - M[idx] @ y) / M[idx, idx]
    assert np.max(np.abs(y - got)) < 1e-13


def test_order4_weighted_half_sweep_with_old_values():
    """Order 4, weight w: the half-sweep gives x_i + w (b - M x)_i / M_ii from
    the values before it on its colour, and leaves the other colour alone."""
    n = (6, 5)
    h = D.spacing(n, (1.0, 1.0))
    a = 1e-3
    w = 1.15
    b = synthetic.uniform_pm1(33, 30).reshape(5, 6)
    x = synthetic.uniform_pm1(34, 30).reshape(5, 6)
    M = np.eye(30) - a * D.laplacian_matrix(n, h, 4)
    xf = x.ravel()
    for colour in (0, 1):
        got = mg.rb_half_sweep(x, b, h, 4, a, colour, w).ravel()
        for idx in range(30):
            i, j = idx % 6, idx // 6
            want = xf[idx] + (w * (b.ravel()[idx] - M[idx] @ xf) / M[idx, idx] if (i + j) % 2 == colour else 0.0)
            assert abs(got[idx] - want) < 1e-13


@pytest.mark.parametrize("order,w", [(2, 1.1), (4, 1.15)])
def test_weighted_mg_converges_to_exact_solution(order, w):
    """The over-relaxed V(2,1) cycle reaches the exact implicit solve and
    needs no more cycles than the plain one on a 63^2 grid with a/h^2 = 15."""
    n = (63, 63)
    h = D.spacing(n, (1.0, 1.0))
    plan = D.time_plan(h, order, 8.0, "implicit", n_its=10, adjust_omega=True)
    a = 0.5 * plan.dt ** 2
    b = synthetic.uniform_pm1(52, 63 * 63).reshape(63, 63)
    xw, cw, rel = mg.solve(b, mg.Hierarchy(n, h, order, a, relax=w), 1e-10)
    x1, c1, _ = mg.solve(b, mg.Hierarchy(n, h, order, a), 1e-10)
    assert rel <= 1e-10 and cw <= c1
    xe = W.solve_implicit_exact(b, h, order, plan.dt)
    assert np.linalg.norm(xw - xe) <= 1e-10 * np.linalg.norm(b) * 1.0000001


@pytest.mark.parametrize("n,order", [((63, 63), 2), ((63, 63), 4), ((15, 15, 15), 2)])
def test_level_weights_converge_to_exact_solution(n, order):
    """Weight 1.2 on the finest level and 1.05 below it: the V(2,1) solve
    still reaches the exact implicit solve (dense / sine-transform), so the
    per-level weights change the smoother, never the fixed point."""
    h = D.spacing(n, (1.0,) * len(n))
    plan = D.time_plan(h, order, 8.0, "implicit", n_its=10, adjust_omega=True)
    a = 0.5 * plan.dt ** 2
    b = synthetic.uniform_pm1(53, int(np.prod(n))).reshape(n[::-1])
    hier = mg.Hierarchy(n, h, order, a, relax=1.2, relax_coarse=1.05)
    assert hier.weight(0) == 1.2 and all(hier.weight(l) == 1.05 for l in range(1, len(hier.sizes)))
    x, c, rel = mg.solve(b, hier, 1e-10)
    assert rel <= 1e-10
    xe = W.solve_implicit_exact(b, h, order, plan.dt)
    assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(b) * 1.0000001


def test_equal_level_weights_reproduce_single_weight_cycle():
    n = (31, 31)
    h = D.spacing(n, (1.0, 1.0))
    a = 0.002
    b = synthetic.uniform_pm1(54, 31 * 31).reshape(31, 31)
    x = synthetic.uniform_pm1(55, 31 * 31).reshape(31, 31)
    one = mg.vcycle(x, b, mg.Hierarchy(n, h, 4, a, relax=1.1))
    two = mg.vcycle(x, b, mg.Hierarchy(n, h, 4, a, relax=1.1, relax_coarse=1.1))
    assert np.array_equal(one, two)
