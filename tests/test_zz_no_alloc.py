"""ew_apply_filter_noalloc (the entry point for callers that cannot allocate)
against ew_op_apply_filter, called through the raw C ABI: two calls in a row,
the second on a smaller grid, FP64 and mixed precision, and the size limit."""
import ctypes

import numpy as np
import pytest

import synthetic
from gpu_helpers import make_op, rel_err, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _descs(P):
    from paper_2507_18282_amd import _lib
    g = _lib.GridDesc()
    g.dim = len(P.n)
    for d in range(3):
        g.n[d] = P.n[d] if d < len(P.n) else 1
        g.len[d] = P.length[d] if d < len(P.n) else 1.0
    g.order = P.order
    d = _lib.OpDesc()
    d.omega, d.ts, d.cfl, d.n_its, d.n_p = P.omega, _lib.TS[P.ts], P.cfl, P.n_its, P.n_p
    d.filter_const, d.precision = _lib.FILTER[P.filter_const], _lib.PRECISION[P.precision]
    d.mg_tol, d.mg_nu1, d.mg_nu2, d.mg_max_cycles, d.mg_coarse_sweeps = 1e-10, 2, 1, 100, 8
    return g, d


def _noalloc(P, v):
    """S v by the no-allocation entry point on torch's current stream."""
    import torch
    from paper_2507_18282_amd import _lib
    lib = _lib.load()
    g, d = _descs(P)
    out = torch.full_like(v, float("nan"))
    st = lib.ew_apply_filter_noalloc(ctypes.byref(g), ctypes.byref(d), ctypes.c_void_p(int(v.data_ptr())),
                                     ctypes.c_void_p(int(out.data_ptr())),
                                     ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream)))
    return st, out


BIG = synthetic.Problem(n=(300, 200), length=(1.0, 0.7), order=4, omega=25.0, ts="explicit", cfl=0.5)
SMALL = synthetic.config_small_explicit()       # 64^2, order 2, omega 15, CFL 0.5 (78 steps)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_apply_filter_twice_smaller_second(precision):
    import dataclasses
    first = dataclasses.replace(BIG, precision=precision)
    second = dataclasses.replace(SMALL, precision=precision)
    for P, seed in ((first, 41), (second, 42)):
        say("noalloc", P.n, P.order, P.precision)
        v = to_dev(synthetic.uniform_pm1(seed, P.n_active))
        st, out = _noalloc(P, v)
        assert st == 0
        got = to_host(out)
        want = to_host(make_op(P).apply_filter(v))
        n_t = make_op(P).n_t
        # FP64: the same kernels and weights (1e-13; the one-workgroup path of
        # small grids sums in another order, 1e-11 as for the oracle);
        # mixed: the FP32 unit roundoff accumulated over N_t steps
        tol = (1e-11 if P.precision == "fp64" else max(2e-5, 4 * n_t * 2.0 ** -24))
        assert np.all(np.isfinite(got))
        assert rel_err(got, want) < tol, (P.n, P.precision, rel_err(got, want))


def test_noalloc_3d_neumann_and_limits():
    from paper_2507_18282_amd import _lib
    P = synthetic.Problem(n=(40, 30, 20), length=(1.0, 0.75, 0.5), order=2, omega=12.0, ts="explicit", cfl=0.5)
    say("noalloc 3d", P.n)
    v = to_dev(synthetic.uniform_pm1(43, P.n_active))
    st, out = _noalloc(P, v)
    assert st == 0
    assert rel_err(to_host(out), to_host(make_op(P).apply_filter(v))) < 1e-13
    # beyond the scratch limit (2^22 points): refused on the host, nothing launched
    big = synthetic.Problem(n=(2049, 2049), length=(1.0, 1.0), order=2, omega=30.0, ts="explicit", cfl=0.5)
    g, d = _descs(big)
    lib = _lib.load()
    st = lib.ew_apply_filter_noalloc(ctypes.byref(g), ctypes.byref(d), ctypes.c_void_p(8), ctypes.c_void_p(16), None)
    assert st == -1 and b"scratch limit" in lib.ew_last_error()
    # implicit stepping is not offered
    imp = synthetic.Problem(n=(63, 63), length=(1.0, 1.0), order=2, omega=30.0, ts="implicit")
    g, d = _descs(imp)
    st = lib.ew_apply_filter_noalloc(ctypes.byref(g), ctypes.byref(d), ctypes.c_void_p(8), ctypes.c_void_p(16), None)
    assert st == -7
