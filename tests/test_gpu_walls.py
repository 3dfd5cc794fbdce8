"""Boxes with Neumann walls on the GPU against the oracle (oracle/walls.py),
element by element through the C ABI, and eigensolves against the
closed-form spectrum.

Tolerances as in test_gpu_parity.py: L_h v to 1e-13 relative, one explicit
wave-solve to 1e-11 (FP64; rounding order only), 2e-5 for FP32 state; modes
S phi = beta phi to 1e-13.  Eigenvalues within 1e-10 relative of the closed
form, the wanted band present with multiplicity, eig-res <= 1e-8, and the
returned vectors satisfy L_h u = -mu u on the grid (they are grid functions,
converted back from the eigensolver's weighted coordinates).
"""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from oracle import walls as Wl
from tests.gpu_helpers import assert_signs, rel_err, say, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [
    # (n, length, walls, order, omega, cfl)
    ((40, 30), (1.0, 0.8), (("N", "D"), ("D", "N")), 2, 12.0, 0.5),      # one workgroup (k_wave_small)
    ((40, 30), (1.0, 0.8), (("N", "N"), ("D", "D")), 4, 12.0, 0.5),
    ((64, 48), (1.0, 0.7), (("D", "D"), ("N", "D")), 4, 15.0, 0.7),      # symmetry plane at y = 0
    ((100, 90), (1.0, 0.9), (("N", "N"), ("N", "D")), 2, 10.0, 0.5),    # several steps per launch
    ((100, 90), (1.0, 0.9), (("D", "N"), ("N", "N")), 4, 10.0, 0.5),
    ((150, 70), (1.2, 0.6), (("N", "N"), ("N", "N")), 4, 11.0, 0.9),    # ragged tiles, Neumann all round
    ((13, 11, 9), (1.0, 0.9, 1.1), (("N", "D"), ("D", "D"), ("D", "N")), 2, 8.0, 0.5),
    ((13, 11, 9), (1.0, 0.9, 1.1), (("N", "N"), ("N", "D"), ("N", "N")), 4, 8.0, 0.5),
]


def _op(n, length, walls, order, omega, cfl, precision="fp64"):
    from paper_2507_18282_amd import Operator
    return Operator(n=n, length=length, order=order, omega=omega, ts="explicit", cfl=cfl, walls=walls,
                    precision=precision)


def _plan(n, length, walls, order, omega, cfl):
    h = Wl.spacing(n, length, walls)
    return h, D.time_plan(h, order, omega, "explicit", cfl=cfl)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[2]}-o{c[3]}")
def test_laplacian_and_filter_match_oracle(case):
    n, length, walls, order, omega, cfl = case
    op = _op(*case)
    h, plan = _plan(*case)
    assert op.n_t == plan.n_t and abs(op.dt - plan.dt) <= 1e-15 * plan.dt
    N = int(np.prod(n))
    v = synthetic.uniform_pm1(31, N)
    say("walls laplacian", n, walls, order)
    got = to_host(op.apply_laplacian(to_dev(v)))
    want = Wl.apply_laplacian(v.reshape(n[::-1]), h, order, walls).ravel()
    assert rel_err(got, want) < 1e-13
    say("walls filter", n, walls, order)
    got = to_host(op.apply_filter(to_dev(v)))
    want = Wl.apply_filter_explicit(v.reshape(n[::-1]), h, order, walls, plan).ravel()
    assert rel_err(got, want) < 1e-11


@pytest.mark.parametrize("case", CASES[:1] + CASES[3:4] + CASES[5:6], ids=lambda c: f"{c[0]}-o{c[3]}")
def test_filter_mixed_precision(case):
    n, length, walls, order, omega, cfl = case
    op = _op(*case, precision="mixed")
    h, plan = _plan(*case)
    v = synthetic.uniform_pm1(32, int(np.prod(n)))
    got = to_host(op.apply_filter(to_dev(v)))
    want = Wl.apply_filter_explicit(v.reshape(n[::-1]), h, order, walls, plan).ravel()
    assert rel_err(got, want) < max(2e-5, 4 * plan.n_t * 2.0 ** -24)


@pytest.mark.parametrize("case", CASES[1:3] + CASES[4:5], ids=lambda c: f"{c[0]}-o{c[3]}")
def test_filter_on_modes_is_beta(case):
    n, length, walls, order, omega, cfl = case
    op = _op(*case)
    h, plan = _plan(*case)
    mu = Wl.mu_all(n, h, order, walls)
    for idx in ((0, 0), (3, 2), (n[0] - 1, 1), (7, n[1] - 1)):
        phi = Wl.mode(idx, n, walls)
        beta = float(D.beta_corrected(mu[idx[1], idx[0]], plan))
        got = to_host(op.apply_filter(to_dev(phi.ravel())))
        assert np.max(np.abs(got - beta * phi.ravel())) < 1e-13, idx


EIG_CASES = [
    # (n, length, walls, order, omega, cfl, k, m): a square with a symmetry plane,
    # a box with Neumann on three sides (no zero mode), and an order-4 rectangle
    ((48, 48), (1.0, 1.0), (("D", "D"), ("N", "D")), 2, 15.0, 0.5, 6, 16),
    ((40, 36), (1.0, 0.9), (("N", "N"), ("N", "D")), 2, 12.0, 0.5, 6, 16),
    ((50, 40), (1.0, 0.8), (("N", "D"), ("D", "N")), 4, 14.0, 0.5, 8, 20),
]


@pytest.mark.parametrize("case", EIG_CASES, ids=lambda c: f"{c[0]}-{c[2]}-o{c[3]}")
def test_eigs_match_closed_form(case):
    n, length, walls, order, omega, cfl, k, m = case
    op = _op(n, length, walls, order, omega, cfl)
    h, plan = _plan(n, length, walls, order, omega, cfl)
    say("walls eigs", n, walls, order)
    r = op.eigs(k, m, seed=4)
    mu_all = Wl.mu_all(n, h, order, walls).ravel()
    beta_all = D.beta_corrected(mu_all, plan)
    order_b = np.argsort(-np.abs(beta_all), kind="stable")
    beta_k = np.abs(beta_all[order_b[k - 1]])
    mu = np.array(r.mu)
    assert r.n_conv >= k
    for x in mu:
        assert np.min(np.abs(mu_all - x)) / x < 1e-10
    band = np.sort(mu_all[np.abs(beta_all) >= beta_k * (1 - 1e-10)])
    for x in band:
        want = np.sum(np.abs(band - x) <= 1e-9 * x)
        assert np.sum(np.abs(mu - x) <= 1e-9 * x) >= want, (x, mu)
    assert max(r.res) <= 1e-8
    assert np.max(np.abs(D.beta_corrected(mu, plan) - np.array(r.beta))) < 1e-8
    # returned vectors are grid functions with L_h u = -mu u
    Y = r.Y.cpu().numpy()
    assert_signs(Y)
    for c in range(Y.shape[1]):
        u = Y[:, c].reshape(n[::-1])
        assert abs(np.linalg.norm(u) - 1.0) < 1e-12
        res = Wl.apply_laplacian(u, h, order, walls) + mu[c] * u
        assert np.linalg.norm(res) / mu[c] < 1e-7


# ---------------------------------------------------------------------------
# Implicit scheme: multigrid with the walls' points kept on every level.
# Tolerances as in test_gpu_parity.py: a solve stops at ||r|| <= tau ||b||
# and M's eigenvalues are >= 1, so ||x - x*|| <= tau ||b||; ten steps of the
# stable recurrence and the filter sum stay below 1e-8 relative.
# ---------------------------------------------------------------------------
IMPLICIT_CASES = [
    # (n, length, walls, order, omega)
    ((63, 64), (1.0, 1.0), (("D", "D"), ("N", "D")), 2, 20.0),         # symmetry plane
    ((65, 31), (1.0, 0.5), (("N", "N"), ("D", "D")), 4, 25.0),
    ((64, 64), (1.0, 1.0), (("D", "N"), ("N", "D")), 4, 30.0),
    ((17, 16, 15), (1.0, 0.9, 1.0), (("N", "N"), ("N", "D"), ("D", "D")), 2, 10.0),
    ((16, 17, 16), (1.0, 1.0, 1.0), (("D", "N"), ("N", "N"), ("N", "D")), 4, 12.0),
    # wide enough for the 64 x 16 tiles of the finest level: tiles near the
    # Neumann wall run its closures, tiles inside the grid the test-free path
    ((2047, 512), (1.0, 0.25), (("D", "D"), ("N", "D")), 4, 60.0),
]


def _iop(n, length, walls, order, omega, **kw):
    from paper_2507_18282_amd import Operator
    return Operator(n=n, length=length, order=order, omega=omega, ts="implicit", n_its=10, adjust_omega=True,
                    mg_tol=1e-10, walls=walls, **kw)


def _iplan(n, length, walls, order, omega):
    h = Wl.spacing(n, length, walls)
    return h, D.time_plan(h, order, omega, "implicit", n_its=10, adjust_omega=True)


@pytest.mark.parametrize("case", IMPLICIT_CASES, ids=lambda c: f"{c[0]}-{c[2]}-o{c[3]}")
def test_implicit_solve_and_filter_match_oracle(case):
    n, length, walls, order, omega = case
    op = _iop(*case)
    h, plan = _iplan(*case)
    assert op.mg_levels >= 3
    N = int(np.prod(n))
    b = synthetic.uniform_pm1(41, N)
    say("walls mg solve", n, walls, order, op.mg_levels)
    x, cycles, rel = op.mg_solve(to_dev(b), to_dev(np.zeros(N)))
    xe = Wl.solve_implicit_exact(b.reshape(n[::-1]), h, order, walls, plan.dt).ravel()
    assert rel <= 1e-10 and cycles <= 20, (cycles, rel)
    assert np.linalg.norm(to_host(x) - xe) <= 1e-10 * np.linalg.norm(b) * 1.0001
    say("walls implicit filter", n, walls, order)
    v = synthetic.uniform_pm1(42, N)
    got = to_host(op.apply_filter(to_dev(v)))
    want = Wl.apply_filter_implicit(v.reshape(n[::-1]), h, order, walls, plan).ravel()
    assert rel_err(got, want) < 1e-8


@pytest.mark.parametrize("case", IMPLICIT_CASES[:2] + IMPLICIT_CASES[3:4], ids=lambda c: f"{c[0]}-o{c[3]}")
def test_implicit_modes_and_mixed_precision(case):
    n, length, walls, order, omega = case
    h, plan = _iplan(*case)
    mu = Wl.mu_all(n, h, order, walls)
    op = _iop(*case)
    idxs = [(0,) * len(n), tuple(min(3, k - 1) for k in n), tuple(k - 1 for k in n)]
    for idx in idxs:
        phi = Wl.mode(idx, n, walls)
        beta = float(D.beta_corrected(mu[idx[::-1]], plan))
        got = to_host(op.apply_filter(to_dev(phi.ravel())))
        assert np.max(np.abs(got - beta * phi.ravel())) < 1e-8, idx
    mixed = _iop(*case, precision="mixed")
    v = synthetic.uniform_pm1(43, int(np.prod(n)))
    want = Wl.apply_filter_implicit(v.reshape(n[::-1]), h, order, walls, plan).ravel()
    assert rel_err(to_host(mixed.apply_filter(to_dev(v))), want) < 4 * plan.n_t * 2.0 ** -24 + 1e-8


def test_implicit_eigs_symmetry_plane_match_closed_form():
    """127 x 128 unit square, Neumann wall at y = 0 (the symmetry-plane case),
    order 4, implicit, omega 30, automatic multigrid depth: the wanted band of
    the closed-form spectrum with multiplicity."""
    n, length, walls, order, omega, k, m = (127, 128), (1.0, 1.0), (("D", "D"), ("N", "D")), 4, 30.0, 6, 16
    op = _iop(n, length, walls, order, omega, mg_max_levels=-1, mg_coarse_sweeps=4)
    h, plan = _iplan(n, length, walls, order, omega)
    say("walls implicit eigs", n, op.mg_levels)
    r = op.eigs(k, m, seed=5)
    mu_all = Wl.mu_all(n, h, order, walls).ravel()
    beta_all = D.beta_corrected(mu_all, plan)
    beta_k = np.abs(beta_all[np.argsort(-np.abs(beta_all), kind="stable")[k - 1]])
    mu = np.array(r.mu)
    assert r.n_conv >= k
    for x in mu:
        assert np.min(np.abs(mu_all - x)) / x < 1e-10
    band = np.sort(mu_all[np.abs(beta_all) >= beta_k * (1 - 1e-10)])
    for x in band:
        assert np.sum(np.abs(mu - x) <= 1e-9 * x) >= np.sum(np.abs(band - x) <= 1e-9 * x), (x, mu)
    assert max(r.res) <= 1e-8
