"""Eigensolver on the GPU against the closed-form discrete spectrum.

Bar (FP64): every returned eigenvalue within 1e-10 relative of a closed-form
mu_h, every eigenvalue whose beta reaches the k-th largest present with its
multiplicity, and L_h residuals <= 1e-8.  Mixed precision: 1e-5 relative.
"""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from tests.gpu_helpers import assert_signs, make_op, oracle_plan, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def closed_form(P):
    h, plan = oracle_plan(P)
    mu = D.mu_all(P.n, h, P.order).ravel()
    beta = D.beta_corrected(mu, plan)
    order = np.argsort(-np.abs(beta), kind="stable")
    return mu, beta, np.abs(beta[order[P.k - 1]])


def check_result(P, r, rel_tol=1e-10, res_tol=1e-8):
    mu_all, beta_all, beta_k = closed_form(P)
    mu = np.array(r.mu)
    if res_tol is not None:
        assert r.n_conv >= P.k
    else:
        assert len(mu) >= P.k
    for x in mu:
        assert np.min(np.abs(mu_all - x)) / x < rel_tol
    band = np.sort(mu_all[np.abs(beta_all) >= beta_k * (1 - 1e-10)])
    for x in band:
        want = np.sum(np.abs(band - x) <= 1e-9 * x)
        assert np.sum(np.abs(mu - x) <= max(rel_tol, 1e-9) * x) >= want, (x, mu)
    if res_tol is not None:
        assert max(r.res) <= res_tol
    # beta of each pair matches the closed form at its mu
    h, plan = oracle_plan(P)
    assert np.max(np.abs(D.beta_corrected(mu, plan) - np.array(r.beta))) < max(1e-8, 10 * rel_tol)


def test_eigs_small_explicit_square():
    """64^2 interior, order 2, explicit CFL 0.5, omega 15, k = 4, m = 16."""
    P = synthetic.config_small_explicit()
    op = make_op(P)
    say("eigs small explicit")
    r = op.eigs(P.k, P.m, seed=P.seed)
    check_result(P, r)
    # eigenvectors: unit norm and orthogonal
    Y = to_host(r.Y.contiguous()).reshape(P.n_active, -1) if False else r.Y.cpu().numpy()
    assert np.max(np.abs(Y.T @ Y - np.eye(Y.shape[1]))) < 1e-9
    assert_signs(Y)
    # four wanted: the two double eigenvalues (3,4)/(4,3) and (2,4)/(4,2)
    want = sorted([D.mu_closed_form(mm, P.n, D.spacing(P.n, P.length), 2) for mm in ((3, 4), (4, 3), (2, 4), (4, 2))])
    got = sorted(r.mu[:4])
    assert np.max(np.abs(np.array(got) - np.array(want)) / np.array(want)) < 1e-10


def test_eigs_start_vector_from_caller_matches_seeded():
    P = synthetic.config_small_explicit()
    op = make_op(P)
    r1 = op.eigs(P.k, P.m, seed=P.seed)
    v0 = synthetic.start_vector(P.seed, P.n_active)
    r2 = op.eigs(P.k, P.m, seed=P.seed, v0=to_dev(v0))
    assert r1.wave_solves == r2.wave_solves
    assert np.array_equal(np.array(r1.mu), np.array(r2.mu))


def test_eigs_repeatable_bitwise():
    P = synthetic.config_small_explicit()
    op = make_op(P)
    r1 = op.eigs(P.k, P.m, seed=3)
    r2 = op.eigs(P.k, P.m, seed=3)
    assert np.array_equal(np.array(r1.mu), np.array(r2.mu))
    assert np.array_equal(r1.Y.cpu().numpy(), r2.Y.cpu().numpy())


@pytest.mark.parametrize("order", [2, 4])
def test_eigs_implicit_square(order):
    P = synthetic.Problem(n=(63, 63), length=(1.0, 1.0), order=order, omega=20.0, ts="implicit",
                          adjust_omega=True, k=6, m=16, seed=7)
    op = make_op(P)
    say("eigs implicit", order)
    r = op.eigs(P.k, P.m, seed=P.seed)
    check_result(P, r)


def test_eigs_cube_multiplicity_three():
    P = synthetic.Problem(n=(15, 15, 15), length=(1.0, 1.0, 1.0), order=2, omega=8.0, ts="implicit",
                          adjust_omega=True, k=4, m=12, seed=9)
    op = make_op(P)
    say("eigs cube")
    r = op.eigs(P.k, P.m, seed=P.seed)
    check_result(P, r)


# Mixed precision: S v carries the FP32 accumulation error of the filter,
# about 4 N_t 2^-24 relative (2.4e-6 at N_t = 10), so Ritz pairs are screened
# at 1e-7 and the eigenvectors carry errors of that order; the L_h residual of
# such a vector is that error amplified by at most mu_max / mu of the grid
# (a few hundred here), which bounds eig-res by 1e-4.  Eigenvalues, Rayleigh
# quotients of those vectors, are quadratically accurate: 1e-5 relative is the
# stated bar.
MIXED_RES = 1e-4


def test_eigs_mixed_precision_rectangle():
    P = synthetic.Problem(n=(63, 47), length=(1.0, 0.75), order=2, omega=18.0, ts="implicit",
                          adjust_omega=True, precision="mixed", k=4, m=12, seed=5)
    op = make_op(P)
    say("eigs mixed")
    r = op.eigs(P.k, P.m, seed=P.seed, tol_ritz=1e-7, tol_res=MIXED_RES)
    say("mixed rectangle: max eig-res", max(r.res))
    check_result(P, r, rel_tol=1e-5, res_tol=MIXED_RES)


def test_eigs_mixed_precision_cube_against_fp64():
    """The cube workload's eigenproblem (unit cube, order 2, implicit, omega 40
    adjusted, k = 8, N_p from the lobe rule) on a 31^3 grid, mixed precision
    and FP64 with the same solver settings: every mixed eigenvalue within 1e-5
    of the closed form and of the FP64 solve's, the wanted band complete with
    multiplicity, eig-res within MIXED_RES; the FP64 run meets the FP64 bar."""
    import dataclasses
    from paper_2507_18282_amd import choose_periods
    base = synthetic.Problem(n=(31, 31, 31), length=(1.0, 1.0, 1.0), order=2, omega=40.0, ts="implicit",
                             adjust_omega=True, precision="mixed", k=8, m=17, seed=3)
    n_p, _ = choose_periods(base.length, base.omega, base.k)
    P = dataclasses.replace(base, n_p=n_p)
    rs = {}
    for prec in ("mixed", "fp64"):
        Pp = dataclasses.replace(P, precision=prec)
        say("eigs cube", prec, n_p)
        rs[prec] = make_op(Pp).eigs(P.k, P.m, seed=P.seed, tol_ritz=1e-7, tol_res=MIXED_RES,
                                    max_wave_solves=1000, want_vectors=False)
    rm, rf = rs["mixed"], rs["fp64"]
    say("cube mixed: pairs", len(rm.mu), "max eig-res", max(rm.res), "| fp64: pairs", len(rf.mu),
        "max eig-res", max(rf.res))
    check_result(P, rm, rel_tol=1e-5, res_tol=MIXED_RES)
    for x in rm.mu:
        assert np.min(np.abs(np.array(rf.mu) - x)) / x < 1e-5
    mu_all = closed_form(P)[0]
    for x in rf.mu:
        assert np.min(np.abs(mu_all - x)) / x < 1e-10


def test_eigs_lucky_breakdown_sine_start():
    """Start vector = an exact eigenvector: the Krylov space is invariant after
    one step; the solver must continue from a fresh direction and still find
    the wanted set."""
    P = synthetic.Problem(n=(31, 23), length=(1.0, 0.8), order=2, omega=14.0, ts="explicit", cfl=0.5,
                          k=2, m=8, seed=2)
    op = make_op(P)
    v0 = D.sine_mode((3, 2), P.n).ravel()
    r = op.eigs(P.k, P.m, v0=to_dev(v0), seed=P.seed)
    check_result(P, r)


def test_eigs_with_periods_from_the_lobe_rule():
    """A dense-spectrum case (127^2, order 2, implicit, omega 30): with N_p from
    the lobe rule the complete solve converges to the closed-form wanted set."""
    import dataclasses
    from paper_2507_18282_amd import choose_periods
    base = synthetic.Problem(n=(127, 127), length=(1.0, 1.0), order=2, omega=30.0, ts="implicit",
                             adjust_omega=True, k=4, m=9, seed=7)
    n_p, n_lobe = choose_periods(base.length, base.omega, base.k)
    assert n_p > 1 and n_lobe >= base.k
    P = dataclasses.replace(base, n_p=n_p)
    op = make_op(P)
    say("eigs periods rule", n_p)
    r = op.eigs(P.k, P.m, seed=P.seed, max_wave_solves=2000)
    check_result(P, r)
