"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times.

* 2047^2 order-4 implicit (the headline, multigrid of 5 levels, which ends
  on 127^2 with one sweep there): S v against the oracle's exact
  (sine-transform) implicit solves, and S phi = beta~(mu) phi for sine modes
  (closed form).
* 255^3 order-2 implicit in mixed precision: sine modes against the closed
  form, and mixed against FP64 on a random vector.
* the 96-rectangle batch: one sine mode per problem against the closed form.
* the learned guess on 1023^2: windows of the whole-grid guess against the
  oracle network evaluated on the same windows (valid convolutions make a
  window with a 3-cell halo exact).

Tolerances: the multigrid stops at relative residual 1e-10 per implicit
solve and M = I - a L has eigenvalues >= 1, so each solve's error is below
1e-10 relative; 10 steps of the (stable) recurrence and the filter sum stay
below 1e-8.  FP32 state: 4 N_t 2^-24 (implicit mixed, N_t = 10: 2.4e-6), and
max(2e-5, 4 N_t 2^-24) for the FP32 leapfrog of the batch.
"""
import numpy as np
import pytest

import synthetic
from oracle import cnn as C
from oracle import discrete as D
from oracle import wave as W
from tests.gpu_helpers import oracle_plan, rel_err, say, to_dev, to_host

pytestmark = pytest.mark.gpu

HEADLINE_MG = dict(mg_max_levels=5, mg_coarse_sweeps=1)  # the benchmark's hierarchy for 2047^2


def _op(P, **kw):
    from paper_2507_18282_amd import Operator
    args = dict(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its, n_p=P.n_p,
                adjust_omega=P.adjust_omega, precision=P.precision, mg_tol=P.mg_tol)
    args.update(kw)
    return Operator(**args)


def test_headline_filter_full_size_matches_oracle():
    P = synthetic.config_square_order4_implicit()
    say("full size 2047^2 S v")
    op = _op(P, **HEADLINE_MG)
    assert op.mg_levels == 5  # 2047^2 .. 127^2
    h, plan = oracle_plan(P)
    v = synthetic.uniform_pm1(P.seed, P.n_active)
    got = to_host(op.apply_filter(to_dev(v)))
    want = W.apply_filter(v.reshape(P.n[::-1]), h, P.order, plan).ravel()
    assert rel_err(got, want) < 1e-8


@pytest.mark.parametrize("modes", [(1, 1), (33, 14), (1500, 700)])
def test_headline_sine_modes_full_size(modes):
    P = synthetic.config_square_order4_implicit()
    op = _op(P, **HEADLINE_MG)
    h, plan = oracle_plan(P)
    phi = D.sine_mode(modes, P.n).ravel()
    beta = float(D.beta_corrected(D.mu_closed_form(modes, P.n, h, P.order), plan))
    got = to_host(op.apply_filter(to_dev(phi)))
    assert np.max(np.abs(got - beta * phi)) < 1e-8


def test_mixed_cube_full_size():
    P = synthetic.config_cube_mixed()
    say("full size 255^3 mixed")
    mixed = _op(P)
    h, plan = oracle_plan(P)
    for modes in ((1, 1, 1), (9, 7, 6), (200, 3, 100)):
        phi = D.sine_mode(modes, P.n).ravel()
        beta = float(D.beta_corrected(D.mu_closed_form(modes, P.n, h, P.order), plan))
        got = to_host(mixed.apply_filter(to_dev(phi)))
        assert np.max(np.abs(got - beta * phi)) < 4 * plan.n_t * 2.0 ** -24, modes
    import dataclasses
    fp64 = _op(dataclasses.replace(P, precision="fp64"))
    v = to_dev(synthetic.uniform_pm1(P.seed, P.n_active))
    assert rel_err(to_host(mixed.apply_filter(v)), to_host(fp64.apply_filter(v))) < 4 * plan.n_t * 2.0 ** -24


def test_batch_full_config_sine_modes():
    from paper_2507_18282_amd import Batch
    Ps = synthetic.batch_problems()
    say("full batch", len(Ps))
    bt = Batch([{"n": P.n, "length": P.length, "order": 2, "omega": P.omega, "cfl": 0.5} for P in Ps])
    vs, want = [], []
    for i, P in enumerate(Ps):
        h, plan = oracle_plan(P)
        modes = (1 + i % 5, 2 + i % 3)
        phi = D.sine_mode(modes, P.n).ravel()
        vs.append(to_dev(phi))
        want.append(float(D.beta_corrected(D.mu_closed_form(modes, P.n, h, 2), plan)) * phi)
        assert bt.n_t[i] == plan.n_t
    outs = bt.apply_filter(vs)
    for i, P in enumerate(Ps):
        tol = max(2e-5, 4.0 * bt.n_t[i] * 2.0 ** -24)
        assert np.max(np.abs(to_host(outs[i]) - want[i])) < tol, (i, P.n, bt.n_t[i])


def test_learned_guess_full_size_windows():
    """The learned correction on the 1023^2 grid from a zero base (empty
    projection window): windows of s y against the oracle network on the
    whole-grid planes (b / s, b / s, c2, c3), within s times the BF16 bound."""
    from paper_2507_18282_amd import Cnn
    from tests.test_gpu_cnn import _effective, _forward_with_bound, _params
    P = synthetic.config_learned()
    say("full size 1023^2 guess")
    op = _op(P, mg_max_levels=5, mg_coarse_sweeps=4, predictor="cnn")
    net = Cnn(0)
    params = _params(21)
    net.set_params(params)
    op.set_cnn(net)
    n = P.n[0]
    b = synthetic.uniform_pm1(501, n * n).reshape(n, n)
    got = to_host(op.cnn_guess(to_dev(b))).reshape(n, n)
    h, plan = oracle_plan(P)
    a = 0.5 * plan.dt ** 2
    s = float(np.sqrt(np.mean(b * b)))
    c2, c3 = C.step_planes(a, plan.omega, h[0])
    x = C.make_input_residual(b, b, s, s, np.float32(c2), np.float32(c3))  # whole grid plus the zero halo
    theta = _effective(params)
    win = 48
    for (r0, c0) in ((0, 0), (n - win, n - win), (0, n - win), (500, 333), (n - win, 17)):
        y, bound = _forward_with_bound(theta, x[:, r0:r0 + win + 6, c0:c0 + win + 6])
        ref = s * y
        assert np.all(np.abs(got[r0:r0 + win, c0:c0 + win] - ref) <= s * bound + 1e-14), (r0, c0)
