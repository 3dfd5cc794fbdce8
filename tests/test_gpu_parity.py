"""HIP path vs the CPU oracle, element by element, through the C ABI.

Tolerances (FP64): the stencils and one leapfrog step differ from the oracle
only in the order of rounding (a few ulp per operation), so L_h v agrees to
1e-13 relative and one explicit wave-solve (N_t up to ~100 steps, each
perturbation carried forward with unit amplification since |beta| <= 1 and
the scheme is stable) to 1e-11.  Multigrid results are compared against the
exact solve within the stopping tolerance: ||x - x*|| <= ||M^{-1}|| ||r|| and
every eigenvalue of M is >= 1.  Mixed precision: each of the N_t steps adds
at most a few FP32 roundings (unit roundoff 2^-24) of values bounded by the
output's scale to the accumulated filter, and a stable scheme carries them
forward without growth, so the filter error is below 4 N_t 2^-24 relative
(1.9e-5 for the 78 explicit steps of 64^2, 2.4e-6 for 10 implicit steps; the
implicit solves add the multigrid tolerance as in FP64).
"""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from oracle import mg as OMG
from oracle import wave as W
from tests.gpu_helpers import make_op, oracle_S, oracle_plan, rel_err, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_device_start_vector_is_bitwise_splitmix():
    from paper_2507_18282_amd import fill_uniform
    for seed, n in ((1, 4096), (12345, 1000003), (2 ** 63 + 5, 777)):
        say("splitmix", seed, n)
        got = to_host(fill_uniform(n, seed))
        want = synthetic.uniform_pm1(seed, n)
        assert np.array_equal(got, want)


LAP_CASES = [
    ((67, 45), (1.0, 0.7), 2), ((67, 45), (1.0, 0.7), 4),
    ((130, 7), (1.3, 0.4), 4), ((1, 5), (1.0, 1.0), 4), ((2, 3), (1.0, 1.0), 4),
    ((13, 11, 9), (1.0, 0.9, 1.1), 2), ((13, 11, 9), (1.0, 0.9, 1.1), 4), ((70, 5, 3), (2.0, 1.0, 1.0), 4),
]


@pytest.mark.parametrize("n,length,order", LAP_CASES)
def test_laplacian_matches_oracle(n, length, order):
    P = synthetic.Problem(n=n, length=length, order=order, omega=5.0, ts="explicit")
    op = make_op(P)
    v = synthetic.uniform_pm1(7, P.n_active)
    say("laplacian", n, order)
    got = to_host(op.apply_laplacian(to_dev(v)))
    want = D.apply_laplacian(v.reshape(n[::-1]), D.spacing(n, length), order).ravel()
    assert rel_err(got, want) < 1e-13


EXPLICIT_CASES = [
    synthetic.Problem(n=(67, 45), length=(1.0, 0.7), order=2, omega=12.0, ts="explicit", cfl=0.5),
    synthetic.Problem(n=(67, 45), length=(1.0, 0.7), order=4, omega=12.0, ts="explicit", cfl=0.9,
                      filter_const="quarter"),
    synthetic.Problem(n=(64, 64), length=(1.0, 1.0), order=2, omega=15.0, ts="explicit", cfl=0.5),
    synthetic.Problem(n=(130, 9), length=(1.3, 0.5), order=4, omega=9.0, ts="explicit", cfl=0.7, n_p=2),
    # 9000 points: above the single-workgroup wave-solve, through the tiled leapfrog
    synthetic.Problem(n=(100, 90), length=(1.0, 0.9), order=4, omega=10.0, ts="explicit", cfl=0.5),
    synthetic.Problem(n=(13, 11, 9), length=(1.0, 0.9, 1.1), order=2, omega=8.0, ts="explicit", cfl=0.5),
    synthetic.Problem(n=(13, 11, 9), length=(1.0, 0.9, 1.1), order=4, omega=8.0, ts="explicit", cfl=0.5),
]


@pytest.mark.parametrize("P", EXPLICIT_CASES, ids=lambda P: f"{P.n}-o{P.order}-{P.filter_const}-np{P.n_p}")
def test_explicit_filter_matches_oracle(P):
    op = make_op(P)
    h, plan = oracle_plan(P)
    assert op.n_t == plan.n_t
    assert abs(op.dt - plan.dt) <= 1e-15 * plan.dt
    v = synthetic.uniform_pm1(11, P.n_active)
    say("explicit filter", P.n, P.order)
    got = to_host(op.apply_filter(to_dev(v)))
    want = oracle_S(P, v)
    assert rel_err(got, want) < 1e-11


BLOCKED_CASES = [
    # 2D FP64 boxes above the single-workgroup wave-solve advance 8 / R steps
    # per launch (R the stencil radius) in 16 x 16 tiles with 8-point halos;
    # ragged tiles both ways and step counts that leave a shorter last launch
    synthetic.Problem(n=(211, 150), length=(1.0, 0.8), order=2, omega=12.0, ts="explicit", cfl=0.5),
    synthetic.Problem(n=(150, 97), length=(1.1, 0.7), order=4, omega=11.0, ts="explicit", cfl=0.9,
                      filter_const="quarter"),
]


@pytest.mark.parametrize("P", BLOCKED_CASES, ids=lambda P: f"{P.n}-o{P.order}")
def test_explicit_blocked_steps_match_oracle(P):
    op = make_op(P)
    h, plan = oracle_plan(P)
    v = synthetic.uniform_pm1(12, P.n_active)
    say("explicit blocked filter", P.n, P.order, plan.n_t)
    op.profile_begin("leapfrog")
    got = to_host(op.apply_filter(to_dev(v)))
    prof = op.profile_end()
    per = 8 // (P.order // 2)
    assert prof["launches"] == -(-plan.n_t // per)
    assert rel_err(got, oracle_S(P, v)) < 1e-11
    # a second wave-solve reuses the operator's state buffers
    assert np.array_equal(got, to_host(op.apply_filter(to_dev(v))))


def test_explicit_filter_on_sine_mode_is_beta_d():
    """S phi = beta~_d phi on the GPU (closed form of the discrete filter)."""
    P = synthetic.config_small_explicit()
    op = make_op(P)
    h, plan = oracle_plan(P)
    for modes in ((3, 4), (1, 1), (17, 5)):
        phi = D.sine_mode(modes, P.n).ravel()
        beta = float(D.beta_corrected(D.mu_closed_form(modes, P.n, h, P.order), plan))
        got = to_host(op.apply_filter(to_dev(phi)))
        assert np.max(np.abs(got - beta * phi)) < 1e-13


@pytest.mark.parametrize("P", EXPLICIT_CASES[:5] + EXPLICIT_CASES[5:6], ids=lambda P: f"{P.n}-o{P.order}")
def test_explicit_filter_mixed_precision(P):
    import dataclasses
    Pm = dataclasses.replace(P, precision="mixed")
    op = make_op(Pm)
    v = synthetic.uniform_pm1(13, P.n_active)
    say("explicit mixed", P.n, P.order)
    n_t = oracle_plan(P)[1].n_t
    got = to_host(op.apply_filter(to_dev(v)))
    want = oracle_S(P, v)
    assert rel_err(got, want) < 4 * n_t * 2.0 ** -24


IMPLICIT_CASES = [
    synthetic.Problem(n=(63, 63), length=(1.0, 1.0), order=2, omega=30.0, ts="implicit", adjust_omega=True),
    synthetic.Problem(n=(127, 95), length=(1.0, 0.75), order=4, omega=50.0, ts="implicit", adjust_omega=True),
    synthetic.Problem(n=(31, 15, 31), length=(1.0, 0.5, 1.0), order=2, omega=15.0, ts="implicit"),
    synthetic.Problem(n=(63, 31), length=(1.0, 0.5), order=4, omega=30.0, ts="implicit", adjust_omega=True),
    synthetic.Problem(n=(95, 47), length=(1.0, 0.5), order=4, omega=40.0, ts="implicit", n_p=2),
    synthetic.Problem(n=(15, 15, 15), length=(1.0, 1.0, 1.0), order=2, omega=12.0, ts="implicit",
                      adjust_omega=True),
    synthetic.Problem(n=(15, 7, 15), length=(1.0, 0.5, 1.0), order=4, omega=12.0, ts="implicit"),
    synthetic.Problem(n=(20, 12), length=(1.0, 0.6), order=2, omega=10.0, ts="implicit"),
]


def _mg_hierarchy(P, a, op):
    return OMG.Hierarchy(P.n, D.spacing(P.n, P.length), P.order, a, nu1=2, nu2=1, coarse_sweeps=8,
                         relax=op.mg_relax, relax_coarse=op.mg_relax_coarse)


def test_default_relaxation_weights():
    """mg_relax = mg_relax_coarse = 0 select the documented defaults (1.2 on
    the finest level, 1.05 below); given weights are kept."""
    for P in IMPLICIT_CASES[:3]:
        op = make_op(P)
        assert (op.mg_relax, op.mg_relax_coarse) == (1.2, 1.05)
    op = make_op(IMPLICIT_CASES[1], mg_relax=1.0, mg_relax_coarse=1.3)
    assert (op.mg_relax, op.mg_relax_coarse) == (1.0, 1.3)


# mg_coarse_points: 0 lets the single-workgroup kernel take every level that
# fits in LDS; 40 sends all but the last levels through the tiled kernels.
# (mg_relax, mg_relax_coarse): the defaults, plain red-black Gauss-Seidel, and
# a coarse weight above the finest one.
@pytest.mark.parametrize("relax", [(0.0, 0.0), (1.0, 1.0), (1.1, 1.3)], ids=str)
@pytest.mark.parametrize("coarse_points", [0, 40])
@pytest.mark.parametrize("P", IMPLICIT_CASES, ids=lambda P: f"{P.n}-o{P.order}")
def test_mg_half_sweep_and_vcycle_match_oracle(P, coarse_points, relax):
    op = make_op(P, mg_coarse_points=coarse_points, mg_relax=relax[0], mg_relax_coarse=relax[1])
    h, plan = oracle_plan(P)
    a = 0.5 * plan.dt ** 2
    hier = _mg_hierarchy(P, a, op)
    assert op.mg_levels == len(hier.sizes)
    shape = P.n[::-1]
    b = synthetic.uniform_pm1(21, P.n_active)
    x = synthetic.uniform_pm1(22, P.n_active)
    for colour in (0, 1):
        say("half sweep", P.n, P.order, colour)
        got = to_host(op.mg_half_sweep(to_dev(b), to_dev(x), colour))
        want = OMG.rb_half_sweep(x.reshape(shape), b.reshape(shape), h, P.order, a, colour, op.mg_relax).ravel()
        assert rel_err(got, want) < 1e-13
    say("vcycle", P.n, P.order)
    got = to_host(op.mg_vcycle(to_dev(b), to_dev(x)))
    want = OMG.vcycle(x.reshape(shape), b.reshape(shape), hier).ravel()
    assert rel_err(got, want) < 1e-12


@pytest.mark.parametrize("max_levels", [2, 3])
@pytest.mark.parametrize("P", IMPLICIT_CASES[:2] + IMPLICIT_CASES[4:5], ids=lambda P: f"{P.n}-o{P.order}")
def test_truncated_hierarchy_vcycle_and_solve_match_oracle(P, max_levels):
    """mg_max_levels stops the coarsening early; the last level then gets
    mg_coarse_sweeps sweeps, as in the oracle hierarchy with the same limit."""
    op = make_op(P, mg_max_levels=max_levels)
    h, plan = oracle_plan(P)
    a = 0.5 * plan.dt ** 2
    hier = OMG.Hierarchy(P.n, D.spacing(P.n, P.length), P.order, a, nu1=2, nu2=1, coarse_sweeps=8,
                         max_levels=max_levels, relax=op.mg_relax, relax_coarse=op.mg_relax_coarse)
    assert op.mg_levels == len(hier.sizes) == max_levels
    shape = P.n[::-1]
    b = synthetic.uniform_pm1(23, P.n_active)
    x = synthetic.uniform_pm1(24, P.n_active)
    say("truncated vcycle", P.n, P.order, max_levels)
    got = to_host(op.mg_vcycle(to_dev(b), to_dev(x)))
    want = OMG.vcycle(x.reshape(shape), b.reshape(shape), hier).ravel()
    assert rel_err(got, want) < 1e-12
    xd, cycles, rel = op.mg_solve(to_dev(b), to_dev(np.zeros(P.n_active)))
    xe = W.solve_implicit_exact(b.reshape(shape), h, P.order, plan.dt).ravel()
    assert rel <= P.mg_tol
    assert np.linalg.norm(to_host(xd) - xe) <= P.mg_tol * np.linalg.norm(b) * 1.0001
    _, oc, _ = OMG.solve(b.reshape(shape), hier, P.mg_tol)
    assert abs(cycles - oc) <= 1


def _auto_levels(P, a, sweeps):
    """Depth the automatic rule documented for EW_MG_LEVELS_AUTO keeps: the
    first level whose red-black Gauss-Seidel bound (Gershgorin ratio of M,
    squared) to the power `sweeps` is <= 0.1, else the full hierarchy."""
    h0 = D.spacing(P.n, P.length)
    n = list(P.n)
    levels = 1
    while True:
        s = sum(1.0 / (hd * 2.0 ** (levels - 1)) ** 2 for hd in h0)
        off = (2.0 if P.order == 2 else 34.0 / 12.0) * a * s
        diag = 1.0 + (2.0 if P.order == 2 else 30.0 / 12.0) * a * s
        if off < diag and (off / diag) ** (2 * sweeps) <= 0.1:
            return levels
        if not all(k % 2 == 1 and k >= 3 for k in n):
            return levels
        n = [(k - 1) // 2 for k in n]
        levels += 1


AUTO_CASES = IMPLICIT_CASES[:3] + [
    synthetic.config_many_pairs(k=16),                                          # ends on 15^2
    synthetic.config_square_order4_implicit(n=255),                              # ends on 127^2
    synthetic.config_learned(n=255, omega=40.0),
]


@pytest.mark.parametrize("P", AUTO_CASES, ids=lambda P: f"{P.n}-o{P.order}-w{P.omega:g}")
def test_auto_depth_vcycle_and_solve_match_oracle(P):
    """mg_max_levels = -1 picks the depth by its documented bound; the V-cycle
    then matches the oracle hierarchy of that depth (4 sweeps on the last
    level) and solves reach the exact solution to mg_tol."""
    op = make_op(P, mg_max_levels=-1, mg_coarse_sweeps=4)
    h, plan = oracle_plan(P)
    a = 0.5 * plan.dt ** 2
    want_levels = _auto_levels(P, a, 4)
    assert op.mg_levels == want_levels
    hier = OMG.Hierarchy(P.n, D.spacing(P.n, P.length), P.order, a, nu1=2, nu2=1, coarse_sweeps=4,
                         max_levels=want_levels, relax=op.mg_relax, relax_coarse=op.mg_relax_coarse)
    shape = P.n[::-1]
    b = synthetic.uniform_pm1(25, P.n_active)
    x = synthetic.uniform_pm1(26, P.n_active)
    say("auto depth vcycle", P.n, P.order, want_levels)
    got = to_host(op.mg_vcycle(to_dev(b), to_dev(x)))
    want = OMG.vcycle(x.reshape(shape), b.reshape(shape), hier).ravel()
    assert rel_err(got, want) < 1e-12
    xd, cycles, rel = op.mg_solve(to_dev(b), to_dev(np.zeros(P.n_active)))
    xe = W.solve_implicit_exact(b.reshape(shape), h, P.order, plan.dt).ravel()
    assert rel <= P.mg_tol
    assert np.linalg.norm(to_host(xd) - xe) <= P.mg_tol * np.linalg.norm(b) * 1.0001


@pytest.mark.parametrize("coarse_points", [0, 40])
@pytest.mark.parametrize("P", IMPLICIT_CASES, ids=lambda P: f"{P.n}-o{P.order}")
def test_mg_solve_reaches_exact_solution(P, coarse_points):
    op = make_op(P, mg_coarse_points=coarse_points)
    h, plan = oracle_plan(P)
    b = synthetic.uniform_pm1(31, P.n_active)
    x0 = np.zeros(P.n_active)
    say("mg solve", P.n, P.order)
    xd, cycles, rel = op.mg_solve(to_dev(b), to_dev(x0))
    x = to_host(xd)
    xe = W.solve_implicit_exact(b.reshape(P.n[::-1]), h, P.order, plan.dt).ravel()
    assert rel <= P.mg_tol
    assert np.linalg.norm(x - xe) <= P.mg_tol * np.linalg.norm(b) * 1.0001
    # same cycle count as the oracle solver from the same start
    hier = _mg_hierarchy(P, 0.5 * plan.dt ** 2, op)
    _, oc, _ = OMG.solve(b.reshape(P.n[::-1]), hier, P.mg_tol)
    assert abs(cycles - oc) <= 1


@pytest.mark.parametrize("P", IMPLICIT_CASES, ids=lambda P: f"{P.n}-o{P.order}")
def test_implicit_filter_matches_oracle(P):
    """Each of the N_t solves stops at ||r|| <= tau ||b||, so the error of S v
    against the exact-solve oracle is bounded by sum_n |c_n| N_t tau ||W||,
    well under 100 tau relative."""
    op = make_op(P)
    v = synthetic.uniform_pm1(41, P.n_active)
    say("implicit filter", P.n, P.order)
    got = to_host(op.apply_filter(to_dev(v)))
    want = oracle_S(P, v)
    assert rel_err(got, want) < 100 * P.mg_tol * np.sqrt(P.n_active)


@pytest.mark.parametrize("pred", ["zero", "scaled"])
def test_implicit_filter_predictors_agree(pred):
    P = IMPLICIT_CASES[3]
    op = make_op(P, predictor=pred)
    v = synthetic.uniform_pm1(43, P.n_active)
    got = to_host(op.apply_filter(to_dev(v)))
    assert rel_err(got, oracle_S(P, v)) < 100 * P.mg_tol * np.sqrt(P.n_active)


@pytest.mark.parametrize("P", [IMPLICIT_CASES[0], IMPLICIT_CASES[2], IMPLICIT_CASES[5]], ids=lambda P: f"{P.n}")
def test_implicit_filter_mixed_precision(P):
    import dataclasses
    Pm = dataclasses.replace(P, precision="mixed")
    op = make_op(Pm)
    v = synthetic.uniform_pm1(45, P.n_active)
    say("implicit mixed", P.n)
    got = to_host(op.apply_filter(to_dev(v)))
    n_t = oracle_plan(P)[1].n_t
    assert rel_err(got, oracle_S(P, v)) < 4 * n_t * 2.0 ** -24 + 100 * P.mg_tol * np.sqrt(P.n_active)


# An order-2 3D level large enough for the z-marching sweep (64 x 8 column
# tiles marched through chunks of 8 planes): ragged in every direction (129 =
# 2 x 64 + 1, 67 = 8 x 8 + 3, 151 = 18 x 8 + 7); its coarser levels take the
# block-tiled sweep.
Z3D_CASE = synthetic.Problem(n=(129, 67, 151), length=(1.0, 0.5, 1.2), order=2, omega=20.0, ts="implicit",
                             adjust_omega=True)


def test_zmarch_sweep_vcycle_and_solve_match_oracle():
    P = Z3D_CASE
    op = make_op(P)
    h, plan = oracle_plan(P)
    a = 0.5 * plan.dt ** 2
    hier = _mg_hierarchy(P, a, op)
    assert op.mg_levels == len(hier.sizes)
    shape = P.n[::-1]
    b = synthetic.uniform_pm1(41, P.n_active)
    x = synthetic.uniform_pm1(42, P.n_active)
    say("z-march vcycle", P.n)
    got = to_host(op.mg_vcycle(to_dev(b), to_dev(x)))
    want = OMG.vcycle(x.reshape(shape), b.reshape(shape), hier).ravel()
    assert rel_err(got, want) < 1e-12
    say("z-march solve from zero", P.n)
    xd, cycles, rel = op.mg_solve(to_dev(b), to_dev(np.zeros(P.n_active)))
    xe = W.solve_implicit_exact(b.reshape(shape), h, P.order, plan.dt).ravel()
    assert rel <= P.mg_tol
    assert np.linalg.norm(to_host(xd) - xe) <= P.mg_tol * np.linalg.norm(b) * 1.0001


def test_zmarch_sweep_mixed_filter_matches_oracle():
    """The FP32 instance of the z-marching sweep inside mixed-precision
    implicit S v, within the FP32 bound 4 N_t 2^-24."""
    import dataclasses
    P = dataclasses.replace(Z3D_CASE, precision="mixed")
    op = make_op(P)
    v = synthetic.uniform_pm1(43, P.n_active)
    n_t = oracle_plan(P)[1].n_t
    say("z-march mixed S v", P.n)
    got = to_host(op.apply_filter(to_dev(v)))
    assert rel_err(got, oracle_S(P, v)) < 4 * n_t * 2.0 ** -24


# 2D levels of at least 1024 tiles of 64 x 16 run the two pre-smoothing sweeps
# as one fused pass, the restriction on its own tiles and the prolongation
# sweep on 64 x 16 tiles; smaller levels run the pre-smoothing fused with the
# restriction.  Tiles whose staged halo lies inside the grid take the code
# path without bounds, ghost or wall-diagonal tests.  2047 x 513 has 32 x 33
# such tiles (ragged: 513 = 32 x 16 + 1), most of them inside; its second and
# last level, 1023 x 256, takes eight sweeps as four fused passes on 64 x 8
# tiles.  2047 x 511 (32 x 32 tiles, ragged in y) coarsens to nine levels, the
# second of which (1023 x 255) takes the fused pre-smoothing and restriction.
WIDE_CASES = [
    synthetic.Problem(n=(2047, 513), length=(1.0, 0.25), order=4, omega=60.0, ts="implicit", adjust_omega=True),
    synthetic.Problem(n=(2047, 513), length=(1.0, 0.25), order=2, omega=60.0, ts="implicit", adjust_omega=True),
    synthetic.Problem(n=(2047, 511), length=(1.0, 0.25), order=4, omega=60.0, ts="implicit", adjust_omega=True),
]


@pytest.mark.parametrize("P", WIDE_CASES, ids=lambda P: f"{P.n}-o{P.order}")
def test_wide_tiles_vcycle_matches_oracle(P):
    op = make_op(P)
    h, plan = oracle_plan(P)
    hier = _mg_hierarchy(P, 0.5 * plan.dt ** 2, op)
    assert op.mg_levels == len(hier.sizes) == (2 if P.n[1] == 513 else 9)
    shape = P.n[::-1]
    b = synthetic.uniform_pm1(51, P.n_active)
    x = synthetic.uniform_pm1(52, P.n_active)
    say("wide vcycle", P.n, P.order)
    got = to_host(op.mg_vcycle(to_dev(b), to_dev(x)))
    want = OMG.vcycle(x.reshape(shape), b.reshape(shape), hier).ravel()
    assert rel_err(got, want) < 1e-12


def test_wide_tiles_solve_reaches_exact_solution():
    """The residual-norm pass of the convergence tests on wide tiles: the solve
    stops at ||r|| <= tau ||b|| and reaches the exact solve within that bound."""
    P = WIDE_CASES[2]
    op = make_op(P)
    h, plan = oracle_plan(P)
    b = synthetic.uniform_pm1(54, P.n_active)
    say("wide solve", P.n, P.order)
    xd, cycles, rel = op.mg_solve(to_dev(b), to_dev(np.zeros(P.n_active)))
    xe = W.solve_implicit_exact(b.reshape(P.n[::-1]), h, P.order, plan.dt).ravel()
    assert rel <= P.mg_tol
    assert np.linalg.norm(to_host(xd) - xe) <= P.mg_tol * np.linalg.norm(b) * 1.0001


def test_wide_tiles_mixed_filter_matches_oracle():
    """The FP32 instances of the same kernels inside mixed-precision implicit
    S v, within the FP32 bound 4 N_t 2^-24 plus the multigrid tolerance, on
    2047 x 511 (the two-level hierarchy of 2047 x 513 would not converge: its
    1023 x 256 coarsest level gets only eight sweeps)."""
    import dataclasses
    P = dataclasses.replace(WIDE_CASES[2], precision="mixed")
    op = make_op(P)
    v = synthetic.uniform_pm1(53, P.n_active)
    n_t = oracle_plan(P)[1].n_t
    say("wide mixed S v", P.n)
    got = to_host(op.apply_filter(to_dev(v)))
    assert rel_err(got, oracle_S(P, v)) < 4 * n_t * 2.0 ** -24 + 100 * P.mg_tol


# Grids on which the inside-tile test holds with equality: a tile's staged
# halo ends on the last grid point.  131 x 75: the prolongation sweep of the
# finest level (halo R + 1 = 3 for order 4 on 64 x 8 tiles: 131 = 64 + 64 +
# 3, 75 = 64 + 8 + 3).  133 x 77 with one level: eight sweeps as fused
# two-sweep passes, whose halo R + 3 ends on the last point (133 = 64 + 64 +
# 5, 77 = 64 + 8 + 5).
EDGE_CASES = [
    (synthetic.Problem(n=(131, 75), length=(1.0, 0.6), order=4, omega=40.0, ts="implicit", adjust_omega=True), 0),
    (synthetic.Problem(n=(133, 77), length=(1.0, 0.6), order=4, omega=40.0, ts="implicit", adjust_omega=True), 1),
]


@pytest.mark.parametrize("case", EDGE_CASES, ids=lambda c: f"{c[0].n}-levels{c[1]}")
def test_inside_tile_edges_vcycle_matches_oracle(case):
    P, max_levels = case
    op = make_op(P, mg_max_levels=max_levels, mg_coarse_points=40)
    h, plan = oracle_plan(P)
    a = 0.5 * plan.dt ** 2
    hier = OMG.Hierarchy(P.n, D.spacing(P.n, P.length), P.order, a, nu1=2, nu2=1, coarse_sweeps=8,
                         max_levels=max_levels if max_levels > 0 else 64, relax=op.mg_relax,
                         relax_coarse=op.mg_relax_coarse)
    assert op.mg_levels == len(hier.sizes)
    shape = P.n[::-1]
    b = synthetic.uniform_pm1(61, P.n_active)
    x = synthetic.uniform_pm1(62, P.n_active)
    say("inside-tile edge vcycle", P.n, max_levels)
    got = to_host(op.mg_vcycle(to_dev(b), to_dev(x)))
    want = OMG.vcycle(x.reshape(shape), b.reshape(shape), hier).ravel()
    assert rel_err(got, want) < 1e-12
