"""Error paths of the C ABI forced from the host with ordinary inputs: a
multigrid cycle cap that is too small, a NaN in a vector, a wave-solve budget
that is too small.  Each test checks the status code, the message of
ew_last_error(), and that a valid call on the same object succeeds afterwards
with the result of an untouched object."""
import ctypes

import numpy as np
import pytest

import synthetic
from gpu_helpers import make_op, rel_err, say, to_dev, to_host

pytestmark = pytest.mark.gpu

IMPLICIT = synthetic.Problem(n=(63, 63), length=(1.0, 1.0), order=4, omega=30.0, ts="implicit",
                             adjust_omega=True)
EXPLICIT = synthetic.config_small_explicit()


def _raw_apply(op, v, out):
    """ew_op_apply_filter through the raw ABI: (status, ew_last_error())."""
    from paper_2507_18282_amd import _lib
    lib = _lib.load()
    st = lib.ew_op_apply_filter(op._h, ctypes.c_void_p(int(v.data_ptr())), ctypes.c_void_p(int(out.data_ptr())))
    msg = lib.ew_last_error()
    return st, (msg.decode() if msg else "")


def test_mg_not_converged_then_recovers():
    from paper_2507_18282_amd import _lib
    v = to_dev(synthetic.uniform_pm1(5, IMPLICIT.n_active))
    say("errors: mg_max_cycles=1")
    op = make_op(IMPLICIT, mg_max_cycles=1)
    out = to_dev(np.zeros(IMPLICIT.n_active))
    st, msg = _raw_apply(op, v, out)
    assert st == -4 and _lib.STATUS_NAMES[st] == "EW_ERR_MG_NOT_CONVERGED"
    assert "mg_max_cycles" in msg
    # the same operator still answers valid calls: its Laplacian equals a fresh operator's
    ref = make_op(IMPLICIT)
    assert rel_err(to_host(op.apply_laplacian(v)), to_host(ref.apply_laplacian(v))) == 0.0
    # and a fresh operator with a normal cap converges on the same input
    w = ref.apply_filter(v)
    assert np.all(np.isfinite(to_host(w)))


def test_nonfinite_vector_in_apply_filter():
    vv = synthetic.uniform_pm1(6, IMPLICIT.n_active)
    vv[1234] = np.nan
    bad = to_dev(vv)
    say("errors: NaN in apply_filter")
    op = make_op(IMPLICIT)
    out = to_dev(np.zeros(IMPLICIT.n_active))
    st, msg = _raw_apply(op, bad, out)
    assert st == -5
    assert "non-finite" in msg
    good = to_dev(synthetic.uniform_pm1(7, IMPLICIT.n_active))
    got = to_host(op.apply_filter(good))
    want = to_host(make_op(IMPLICIT).apply_filter(good))
    assert rel_err(got, want) < 1e-9   # both solves stop at mg_tol = 1e-10


@pytest.mark.parametrize("P", [EXPLICIT, IMPLICIT], ids=["explicit", "implicit"])
def test_nonfinite_start_vector_in_eigs(P):
    from paper_2507_18282_amd import EigenwaveError
    vv = synthetic.uniform_pm1(8, P.n_active)
    vv[17] = np.inf
    say("errors: Inf in eigs v0", P.ts)
    op = make_op(P)
    with pytest.raises(EigenwaveError) as e:
        op.eigs(4, 12, v0=to_dev(vv), max_wave_solves=50)
    assert e.value.status == -5
    assert "non-finite" in str(e.value)
    # a valid eigensolve on the same operator equals one on a fresh operator
    r1 = op.eigs(2, 8, seed=3, max_wave_solves=6, want_vectors=False, raise_on_error=False)
    r2 = make_op(P).eigs(2, 8, seed=3, max_wave_solves=6, want_vectors=False, raise_on_error=False)
    assert r1.wave_solves == r2.wave_solves == 6
    assert r1.status == r2.status


def test_not_converged_reports_partial_stats():
    from paper_2507_18282_amd import _lib
    P = EXPLICIT
    say("errors: max_wave_solves=2")
    op = make_op(P)
    r = op.eigs(P.k, P.m, seed=P.seed, max_wave_solves=2, raise_on_error=False)
    assert r.status == -6 and _lib.STATUS_NAMES[r.status] == "EW_ERR_NOT_CONVERGED"
    assert "max_wave_solves" in _lib.load().ew_last_error().decode()
    assert r.wave_solves == 2 and r.n_conv == 0 and r.mu == []
    assert r.time_steps == 2 * op.n_t and r.pt_updates == 2 * op.n_t * op.n_active
    # the full solve on the same operator then converges as usual
    full = op.eigs(P.k, P.m, seed=P.seed)
    assert full.status == 0 and len(full.mu) >= P.k and max(full.res) <= 1e-8
