"""Batched form on the GPU: every problem of a batch gives what the same
problem gives alone, and what the oracle gives.

With FP32 state the batched path keeps W and the filter accumulator in FP32
(as the standalone mixed-precision explicit operator does), so both are
compared with the FP64 oracle at fp32_tol(N_t) = max(2e-5, 4 N_t 2^-24)
relative -- the FP32 unit roundoff accumulated over N_t steps of a stable
recurrence -- and with each other at 1e-5.  With FP64 state the batched step
does the standalone FP64 step's arithmetic, so the two agree to rounding
(1e-12) and the oracle to 1e-11; its eigensolves are held to eig-res 1e-8.
"""
import numpy as np
import pytest

import synthetic
from oracle import discrete as D
from tests.gpu_helpers import make_op, oracle_S, oracle_plan, rel_err, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def fp32_tol(n_t):
    return max(2e-5, 4.0 * n_t * 2.0 ** -24)


def _problems(order, sizes, seed=17, precision="mixed"):
    u = synthetic.uniform01(seed, 3 * len(sizes))
    out = []
    for i, n in enumerate(sizes):
        a = 0.5 + 1.5 * u[3 * i]
        b = 0.5 + 1.5 * u[3 * i + 1]
        om = 10.0 + 30.0 * u[3 * i + 2]
        out.append(synthetic.Problem(n=(n, n + (i % 3)), length=(a, b), order=order, omega=om, ts="explicit",
                                     cfl=0.5, precision=precision, k=3, m=12, seed=100 + i))
    return out


def _batch(Ps):
    from paper_2507_18282_amd import Batch
    return Batch([{"n": P.n, "length": P.length, "order": P.order, "omega": P.omega, "cfl": P.cfl,
                   "precision": P.precision} for P in Ps])


@pytest.mark.parametrize("order", [2, 4])
def test_batch_apply_matches_standalone_and_oracle(order):
    # sizes straddle the single-workgroup limit (128) and span several tiles
    Ps = _problems(order, [13, 40, 126, 128, 129, 200, 333])
    say("batch apply", order)
    bt = _batch(Ps)
    assert bt.info["n_small"] >= 3 and bt.info["n_large"] >= 3
    vs = [to_dev(synthetic.uniform_pm1(500 + i, P.n_active)) for i, P in enumerate(Ps)]
    outs = bt.apply_filter(vs)
    for i, P in enumerate(Ps):
        h, plan = oracle_plan(P)
        assert bt.n_t[i] == plan.n_t
        op = make_op(P)
        alone = to_host(op.apply_filter(vs[i]))
        got = to_host(outs[i])
        assert rel_err(got, alone) < 1e-5, (i, P.n)
        assert rel_err(got, oracle_S(P, to_host(vs[i]))) < fp32_tol(plan.n_t), (i, P.n)


def test_batch_apply_repeated_calls_and_partial_reuse():
    """The captured graph is replayed: a second call with other vectors gives
    the standalone results again (nothing of the first call leaks)."""
    Ps = _problems(2, [50, 150, 260])
    bt = _batch(Ps)
    for rep in range(3):
        vs = [to_dev(synthetic.uniform_pm1(900 + 10 * rep + i, P.n_active)) for i, P in enumerate(Ps)]
        outs = bt.apply_filter(vs)
        for i, P in enumerate(Ps):
            assert rel_err(to_host(outs[i]), oracle_S(P, to_host(vs[i]))) < fp32_tol(bt.n_t[i])


def test_batch_autotuner_reports_candidates():
    Ps = _problems(2, [300, 500])
    bt = _batch(Ps)
    tu = bt.info["tune_us"]
    assert all(t > 0 for t in tu)
    assert bt.info["step_rows_per_thread"] in (1, 2, 4, 8) and bt.info["steps_per_launch"] == 1
    assert tu[[1, 2, 4, 8].index(bt.info["step_rows_per_thread"])] == min(tu)


def test_batch_eigs_match_closed_form_and_standalone():
    Ps = _problems(2, [30, 64, 140, 170], seed=23)
    bt = _batch(Ps)
    say("batch eigs")
    res, st = bt.eigs(k=3, m=12, seeds=[P.seed for P in Ps], tol_ritz=1e-7, tol_res=1e-4)
    assert st["status"] == 0
    for i, P in enumerate(Ps):
        h, plan = oracle_plan(P)
        mu_all = D.mu_all(P.n, h, P.order).ravel()
        beta_all = D.beta_corrected(mu_all, plan)
        kth = np.sort(np.abs(beta_all))[::-1][P.k - 1]
        got = np.array(res[i]["mu"])
        assert res[i]["n_conv"] >= P.k
        for x in got:
            assert np.min(np.abs(mu_all - x)) / x < 1e-5
        band = np.sort(mu_all[np.abs(beta_all) >= kth * (1 - 1e-10)])
        for x in band:
            assert np.sum(np.abs(got - x) <= 1e-5 * x) >= np.sum(np.abs(band - x) <= 1e-9 * x)
        # the same problem alone
        op = make_op(P)
        r = op.eigs(P.k, P.m, seed=P.seed, tol_ritz=1e-7, tol_res=1e-4)
        assert np.allclose(np.sort(r.mu[:P.k]), np.sort(got[:P.k]), rtol=1e-5)


@pytest.mark.parametrize("order", [2, 4])
def test_batch_fp64_apply_matches_standalone_and_oracle(order):
    """FP64 state: every problem takes the batched launches of several steps
    each (none runs in one workgroup; sizes from below one tile to ragged
    multi-tile grids, step counts that end inside a launch); repeated calls
    with other vectors leave v untouched."""
    Ps = _problems(order, [13, 40, 128, 129, 333], precision="fp64")
    say("batch fp64 apply", order)
    bt = _batch(Ps)
    assert bt.info["state_fp64"] and bt.info["n_small"] == 0 and bt.info["n_large"] == len(Ps)
    # 8 / R steps per launch (R the stencil's radius), no tile-height tuning
    assert bt.info["steps_per_launch"] == 8 // (order // 2) and bt.info["step_rows_per_thread"] == 0
    for rep in range(2):
        hv = [synthetic.uniform_pm1(700 + 10 * rep + i, P.n_active) for i, P in enumerate(Ps)]
        vs = [to_dev(x) for x in hv]
        outs = bt.apply_filter(vs)
        for i, P in enumerate(Ps):
            assert np.array_equal(to_host(vs[i]), hv[i])
            alone = to_host(make_op(P).apply_filter(vs[i]))
            got = to_host(outs[i])
            assert rel_err(got, alone) < 1e-12, (i, P.n)
            assert rel_err(got, oracle_S(P, hv[i])) < 1e-11, (i, P.n)


def test_batch_fp64_eigs_at_1e8():
    Ps = _problems(2, [30, 64, 140, 170], seed=23, precision="fp64")
    bt = _batch(Ps)
    say("batch fp64 eigs")
    res, st = bt.eigs(k=3, m=12, seeds=[P.seed for P in Ps], tol_res=1e-8)
    assert st["status"] == 0
    for i, P in enumerate(Ps):
        h, plan = oracle_plan(P)
        mu_all = D.mu_all(P.n, h, P.order).ravel()
        beta_all = D.beta_corrected(mu_all, plan)
        kth = np.sort(np.abs(beta_all))[::-1][P.k - 1]
        got = np.array(res[i]["mu"])
        assert res[i]["n_conv"] >= P.k
        assert sum(1 for x in res[i]["res"] if x <= 1e-8) >= P.k
        for x in got:
            assert np.min(np.abs(mu_all - x)) / x < 1e-9
        band = np.sort(mu_all[np.abs(beta_all) >= kth * (1 - 1e-10)])
        for x in band:
            assert np.sum(np.abs(got - x) <= 1e-9 * x) >= np.sum(np.abs(band - x) <= 1e-9 * x)
        r = make_op(P).eigs(P.k, P.m, seed=P.seed, tol_res=1e-8)
        assert np.allclose(np.sort(r.mu[:P.k]), np.sort(got[:P.k]), rtol=1e-9)


def test_batch_rejects_mixed_precisions():
    from paper_2507_18282_amd import Batch, EigenwaveError
    Ps = _problems(2, [20, 30])
    with pytest.raises(EigenwaveError, match="one precision"):
        Batch([{"n": P.n, "length": P.length, "order": 2, "omega": P.omega, "cfl": P.cfl,
                "precision": pr} for P, pr in zip(Ps, ("mixed", "fp64"))])
