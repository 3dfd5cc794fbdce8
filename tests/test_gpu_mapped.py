"""Single curvilinear grids (mapping method) on the GPU against the oracle
(oracle/mapped.py), element by element through the C ABI.

Tolerances: L_h v to 1e-12 relative to max |L_h v| (the library folds
1/dr^2, 1/ds^2 and 1/(4 dr ds) into its coefficients, the oracle divides
after summing: rounding order only); one explicit wave-solve to 1e-10 (a few
hundred FP64 steps of the same recurrence); S phi = beta phi to 1e-12 for
discrete eigenvectors.  Eigensolves: every returned mu within 1e-9 relative
of the dense spectrum, the wanted band present with multiplicity, eig-res <=
1e-8, and the returned grid functions satisfy L_h u = -mu u.  At 2047^2 the
Laplacian is compared everywhere, and S is checked for self-adjointness in
the J-weighted product, which holds at any size.
"""
import numpy as np
import pytest
from scipy import linalg

import synthetic
from oracle import discrete as D
from oracle import mapped as Mp
from tests.gpu_helpers import assert_signs, rel_err, say, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [
    # (kind, n, params, omega, cfl)
    ("skew", (70, 45), dict(eps=0.2, len1=1.1), 12.0, 0.5),                      # ragged tiles both ways
    ("annulus", (130, 67), dict(a=0.5, b=1.0, theta0=1.2), 15.0, 0.5),
    ("affine", (64, 33), dict(len1=1.0, len2=0.6, phi=0.5, shear=0.3), 10.0, 0.7),  # parallelogram
    ("skew", (5, 3), dict(eps=0.1), 6.0, 0.5),                                    # smaller than one tile
    ("annulus", (1, 4), dict(a=0.3, b=1.0, theta0=2.0), 4.0, 0.5),                # one column
]


def _op(kind, n, params, omega, cfl):
    from paper_2507_18282_amd import Operator
    xy = synthetic.mapped_coords(kind, *n, **params)
    return xy, Operator(n=n, length=(1.0, 1.0), order=2, omega=omega, ts="explicit", cfl=cfl, coords=xy)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_laplacian_and_filter_match_oracle(case):
    kind, n, params, omega, cfl = case
    say("mapped create", kind, n)
    xy, op = _op(*case)
    plan = Mp.time_plan(xy, omega, cfl=cfl)
    rho = Mp.spectral_radius_bound(xy)
    assert abs(op.mapped_rho() - rho) <= 1e-13 * rho
    assert op.n_t == plan.n_t and abs(op.dt - plan.dt) <= 1e-15 * plan.dt
    N = n[0] * n[1]
    v = synthetic.uniform_pm1(51, N)
    say("mapped laplacian", kind, n)
    got = to_host(op.apply_laplacian(to_dev(v)))
    want = Mp.apply_laplacian(v.reshape(n[::-1]), xy).ravel()
    assert rel_err(got, want) < 1e-12
    say("mapped filter", kind, n, plan.n_t)
    got = to_host(op.apply_filter(to_dev(v)))
    want = Mp.apply_filter_explicit(v.reshape(n[::-1]), xy, plan).ravel()
    assert rel_err(got, want) < 1e-10


def test_filter_on_discrete_eigenvectors():
    case = ("skew", (20, 16), dict(eps=0.2), 9.0, 0.5)
    xy, op = _op(*case)
    plan = Mp.time_plan(xy, 9.0, cfl=0.5)
    A = Mp.laplacian_matrix(xy)
    Wt = Mp.weights(xy).ravel()
    mu, V = linalg.eigh(-(Wt[:, None] * A), np.diag(Wt))
    for k in (0, 5, 60, len(mu) - 1):
        phi = V[:, k] / np.max(np.abs(V[:, k]))
        beta = float(D.beta_corrected(mu[k], plan))
        got = to_host(op.apply_filter(to_dev(phi)))
        assert np.max(np.abs(got - beta * phi)) < 1e-12, k


BLOCKED_CASES = [
    # (kind, n, params, omega, cfl): grids of at most 2^18 points advance 8
    # steps per launch in tiles with 8-point halos
    ("annulus", (255, 255), dict(a=0.5, b=1.0, theta0=0.5 * np.pi), 40.0, 0.5),  # the benchmark's annulus, N_t = 191
    ("skew", (40, 24), dict(eps=0.2), 10.1, 0.5),                                  # N_t = 120, a multiple of 8
]


@pytest.mark.parametrize("case", BLOCKED_CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_blocked_steps_match_oracle(case):
    kind, n, params, omega, cfl = case
    xy, op = _op(*case)
    plan = Mp.time_plan(xy, omega, cfl=cfl)
    v = synthetic.uniform_pm1(52, n[0] * n[1])
    say("mapped blocked filter", kind, n, plan.n_t)
    op.profile_begin("leapfrog")
    got = to_host(op.apply_filter(to_dev(v)))
    prof = op.profile_end()
    assert prof["launches"] == (plan.n_t + 7) // 8
    want = Mp.apply_filter_explicit(v.reshape(n[::-1]), xy, plan).ravel()
    assert rel_err(got, want) < 1e-10
    # a second wave-solve on the same operator reuses its state buffers
    got2 = to_host(op.apply_filter(to_dev(v)))
    assert np.array_equal(got, got2)


EIG_CASES = [
    # (kind, n, params, omega, cfl, k, m)
    ("annulus", (48, 40), dict(a=0.5, b=1.0, theta0=0.5 * np.pi), 20.0, 0.5, 6, 16),
    ("skew", (44, 36), dict(eps=0.2, len2=0.9), 14.0, 0.5, 6, 16),
]


@pytest.mark.parametrize("case", EIG_CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_eigs_match_dense_spectrum(case):
    kind, n, params, omega, cfl, k, m = case
    xy, op = _op(kind, n, params, omega, cfl)
    plan = Mp.time_plan(xy, omega, cfl=cfl)
    A = Mp.laplacian_matrix(xy)
    Wt = Mp.weights(xy).ravel()
    mu_all = linalg.eigh(-(Wt[:, None] * A), np.diag(Wt), eigvals_only=True)
    beta_all = D.beta_corrected(mu_all, plan)
    beta_k = np.sort(np.abs(beta_all))[::-1][k - 1]
    say("mapped eigs", kind, n)
    r = op.eigs(k, m, seed=4)
    mu = np.array(r.mu)
    assert r.n_conv >= k
    for x in mu:
        assert np.min(np.abs(mu_all - x)) / x < 1e-9
    band = np.sort(mu_all[np.abs(beta_all) >= beta_k * (1 - 1e-10)])
    for x in band:
        want = np.sum(np.abs(band - x) <= 1e-9 * x)
        assert np.sum(np.abs(mu - x) <= 1e-9 * x) >= want, (x, mu)
    assert max(r.res) <= 1e-8
    Y = r.Y.cpu().numpy()
    assert_signs(Y)
    for c in range(Y.shape[1]):
        u = Y[:, c].reshape(n[::-1])
        assert abs(np.linalg.norm(u) - 1.0) < 1e-12
        res = Mp.apply_laplacian(u, xy) + mu[c] * u
        assert np.linalg.norm(res) / mu[c] < 1e-7


def test_full_size_laplacian_and_weighted_symmetry():
    import torch
    n = (2047, 2047)
    xy = synthetic.mapped_coords("skew", *n, eps=0.15)
    from paper_2507_18282_amd import Operator
    say("mapped full size create", n)
    op = Operator(n=n, length=(1.0, 1.0), order=2, omega=60.0, ts="explicit", cfl=0.9, coords=xy)
    N = n[0] * n[1]
    v = synthetic.uniform_pm1(61, N)
    say("mapped full size laplacian", n)
    got = to_host(op.apply_laplacian(to_dev(v)))
    want = Mp.apply_laplacian(v.reshape(n[::-1]), xy).ravel()
    assert rel_err(got, want) < 1e-12
    # <S u, w>_J = <u, S w>_J at any size (S is a polynomial in L_h, self-adjoint in it)
    say("mapped full size symmetry", n, op.n_t)
    J = to_dev(Mp.weights(xy).ravel())
    u = to_dev(synthetic.uniform_pm1(62, N))
    w = to_dev(synthetic.uniform_pm1(63, N))
    Su, Sw = op.apply_filter(u), op.apply_filter(w)
    a = float(torch.sum(J * Su * w))
    b = float(torch.sum(J * u * Sw))
    scale = float(torch.sqrt(torch.sum(J * Su * Su) * torch.sum(J * w * w)))
    assert abs(a - b) <= 1e-10 * scale


# ---------------------------------------------------------------------------
# Implicit scheme: multigrid on mapped levels against exact sparse solves.
# A solve stops at ||r||_2 <= tau ||b||_2; M is self-adjoint and >= I in the
# J-weighted product, so ||x - x*||_2 <= sqrt(J_max / J_min) tau ||b||_2.
# ---------------------------------------------------------------------------
IMPLICIT_CASES = [
    # (kind, n, params, omega)
    ("skew", (127, 127), dict(eps=0.15), 30.0),
    ("annulus", (127, 63), dict(a=0.5, b=1.0, theta0=1.2), 25.0),
    ("affine", (63, 31), dict(len1=1.0, len2=0.5, phi=0.3, shear=0.2), 20.0),
]


def _iop(kind, n, params, omega, **kw):
    from paper_2507_18282_amd import Operator
    xy = synthetic.mapped_coords(kind, *n, **params)
    return xy, Operator(n=n, length=(1.0, 1.0), order=2, omega=omega, ts="implicit", n_its=10, adjust_omega=True,
                        mg_tol=1e-10, mg_max_levels="auto", mg_coarse_sweeps=4, coords=xy, **kw)


@pytest.mark.parametrize("case", IMPLICIT_CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_implicit_solve_and_filter_match_oracle(case):
    kind, n, params, omega = case
    say("mapped implicit create", kind, n)
    xy, op = _iop(*case)
    plan = Mp.implicit_plan(xy, omega)
    assert op.n_t == plan.n_t and abs(op.dt - plan.dt) <= 1e-15 * plan.dt
    assert op.mg_levels >= (3 if kind != "affine" else 2)
    N = n[0] * n[1]
    b = synthetic.uniform_pm1(71, N)
    say("mapped mg solve", kind, n, op.mg_levels)
    x, cycles, rel = op.mg_solve(to_dev(b), to_dev(np.zeros(N)))
    assert rel <= 1e-10 and cycles <= 60, (cycles, rel)
    xe = Mp.solve_implicit_exact(b.reshape(n[::-1]), xy, plan.dt).ravel()
    Jw = Mp.weights(xy)
    bound = np.sqrt(Jw.max() / Jw.min()) * 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(to_host(x) - xe) <= bound * 1.0001
    say("mapped implicit filter", kind, n)
    v = synthetic.uniform_pm1(72, N)
    got = to_host(op.apply_filter(to_dev(v)))
    want = Mp.apply_filter_implicit(v.reshape(n[::-1]), xy, plan).ravel()
    assert rel_err(got, want) < 1e-8


HALF_SWEEP_CASES = IMPLICIT_CASES[:2] + [
    ("skew", (301, 9), dict(eps=0.15), 30.0),     # two points per thread of the line scan
    ("skew", (1, 7), dict(eps=0.15), 30.0),       # lines of one point
    ("skew", (2901, 3), dict(eps=0.15), 30.0),    # lines longer than the LDS holds: point rule
]


@pytest.mark.parametrize("case", HALF_SWEEP_CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_mapped_half_sweep_and_vcycle(case):
    """A half-sweep relaxes whole lines j of one parity (the block
    Gauss-Seidel step: M restricted to those lines solved exactly, lines
    j +- 1 held), or points of one colour on grids too wide for that."""
    from scipy import sparse
    from scipy.sparse import linalg as spl
    kind, n, params, omega = case
    xy, op = _iop(*case)
    plan = Mp.implicit_plan(xy, omega)
    N = n[0] * n[1]
    M = (sparse.identity(N) - 0.5 * plan.dt ** 2 * Mp.laplacian_sparse(xy)).tocsr()
    b = synthetic.uniform_pm1(73, N)
    x0 = synthetic.uniform_pm1(74, N)
    ii = np.tile(np.arange(n[0]), n[1])
    jj = np.repeat(np.arange(n[1]), n[0])
    lines = n[0] <= 2816
    for colour in (0, 1):
        say("mapped half sweep", kind, n, colour)
        got = to_host(op.mg_half_sweep(to_dev(b), to_dev(x0), colour))
        if lines:
            sel = np.flatnonzero((jj & 1) == colour)
            want = x0.copy()
            want[sel] += spl.spsolve(M[sel][:, sel].tocsc(), (b - M @ x0)[sel])
            assert np.array_equal(got[(jj & 1) != colour], x0[(jj & 1) != colour])
            assert np.max(np.abs((b - M @ got)[sel])) <= 1e-12 * np.max(np.abs(b))
        else:
            want = x0 + (b - M @ x0) / M.diagonal()
            want = np.where(((ii + jj) & 1) == colour, want, x0)
        assert rel_err(got, want) < 1e-12
    # one V-cycle from zero contracts the residual (a property at any size)
    say("mapped vcycle", kind, n)
    x = to_host(op.mg_vcycle(to_dev(b), to_dev(np.zeros(N))))
    assert np.linalg.norm(b - M @ x) < 0.6 * np.linalg.norm(b)


def test_implicit_eigs_match_dense_spectrum():
    case = ("annulus", (63, 47), dict(a=0.5, b=1.0, theta0=0.5 * np.pi), 25.0)
    kind, n, params, omega = case
    xy, op = _iop(*case)
    plan = Mp.implicit_plan(xy, omega)
    A = Mp.laplacian_matrix(xy)
    Wt = Mp.weights(xy).ravel()
    mu_all = linalg.eigh(-(Wt[:, None] * A), np.diag(Wt), eigvals_only=True)
    beta_all = D.beta_corrected(mu_all, plan)
    k, m = 6, 16
    beta_k = np.sort(np.abs(beta_all))[::-1][k - 1]
    say("mapped implicit eigs", kind, n)
    r = op.eigs(k, m, seed=5)
    mu = np.array(r.mu)
    assert r.n_conv >= k
    for x in mu:
        assert np.min(np.abs(mu_all - x)) / x < 1e-8
    band = np.sort(mu_all[np.abs(beta_all) >= beta_k * (1 - 1e-8)])
    for x in band:
        want = np.sum(np.abs(band - x) <= 1e-8 * x)
        assert np.sum(np.abs(mu - x) <= 1e-8 * x) >= want, (x, mu)
    assert max(r.res) <= 1e-8
    Y = r.Y.cpu().numpy()
    assert_signs(Y)
    for c in range(Y.shape[1]):
        u = Y[:, c].reshape(n[::-1])
        res = Mp.apply_laplacian(u, xy) + mu[c] * u
        assert np.linalg.norm(res) / mu[c] < 1e-7


@pytest.mark.parametrize("case", [HALF_SWEEP_CASES[0], HALF_SWEEP_CASES[4]], ids=lambda c: f"{c[0]}-{c[1]}")
def test_mapped_over_relaxed_half_sweep_and_solve(case):
    """With mg_relax = w the half-sweep moves the relaxed lines (or points)
    from x to x + w (relaxed value - x) (successive line over-relaxation);
    mapped grids default to w = 1 on every level.  A solve with the weights
    still reaches the exact solution within the stopping bound."""
    from scipy import sparse
    from scipy.sparse import linalg as spl
    kind, n, params, omega = case
    xy, op0 = _iop(*case)
    assert (op0.mg_relax, op0.mg_relax_coarse) == (1.0, 1.0)
    xy, op = _iop(*case, mg_relax=1.3, mg_relax_coarse=1.2)
    assert (op.mg_relax, op.mg_relax_coarse) == (1.3, 1.2)
    plan = Mp.implicit_plan(xy, omega)
    N = n[0] * n[1]
    M = (sparse.identity(N) - 0.5 * plan.dt ** 2 * Mp.laplacian_sparse(xy)).tocsr()
    b = synthetic.uniform_pm1(75, N)
    x0 = synthetic.uniform_pm1(76, N)
    ii = np.tile(np.arange(n[0]), n[1])
    jj = np.repeat(np.arange(n[1]), n[0])
    for colour in (0, 1):
        say("mapped over-relaxed half sweep", kind, n, colour)
        got = to_host(op.mg_half_sweep(to_dev(b), to_dev(x0), colour))
        if n[0] <= 2816:
            sel = np.flatnonzero((jj & 1) == colour)
            want = x0.copy()
            want[sel] += 1.3 * spl.spsolve(M[sel][:, sel].tocsc(), (b - M @ x0)[sel])
        else:
            want = x0 + 1.3 * (b - M @ x0) / M.diagonal()
            want = np.where(((ii + jj) & 1) == colour, want, x0)
        assert rel_err(got, want) < 1e-12
    if n[1] > 3:
        say("mapped over-relaxed solve", kind, n)
        x, cycles, rel = op.mg_solve(to_dev(b), to_dev(np.zeros(N)))
        xe = Mp.solve_implicit_exact(b.reshape(n[::-1]), xy, plan.dt).ravel()
        Jw = Mp.weights(xy)
        assert rel <= 1e-10
        assert np.linalg.norm(to_host(x) - xe) <= np.sqrt(Jw.max() / Jw.min()) * 1e-10 * np.linalg.norm(b) * 1.0001
