"""The C-ABI library loads and exports every function include/eigenwave.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(ew_[a-z0-9_]+)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for want in ("ew_op_create", "ew_op_apply_filter", "ew_eigs", "ew_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2507_18282_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libeigenwave.so is not built (run python -m paper_2507_18282_amd.build)")
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding declares a signature for exactly the header's functions
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_version_and_last_error_need_no_gpu():
    from paper_2507_18282_amd import _lib
    lib = _lib.load()
    assert b"gfx950" in lib.ew_version()
    assert lib.ew_last_error() is not None


def test_invalid_arguments_rejected_on_host():
    """Argument validation happens before any device call."""
    from paper_2507_18282_amd import _lib
    lib = _lib.load()
    g = _lib.GridDesc()
    g.dim = 2
    g.n[0] = g.n[1] = 8
    g.len[0] = g.len[1] = 1.0
    g.order = 3
    d = _lib.OpDesc()
    d.omega = 10.0
    d.ts = 0
    d.cfl = 0.5
    d.n_p = 1
    h = ctypes.c_void_p()
    assert lib.ew_op_create(ctypes.byref(g), ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert b"order" in lib.ew_last_error()
    g.order = 2
    d.cfl = 1.5
    assert lib.ew_op_create(ctypes.byref(g), ctypes.byref(d), None, ctypes.byref(h)) == -1
    d.cfl = 0.5
    d.ts = 1
    d.n_its = 4
    d.mg_tol = 1e-10
    d.mg_nu1, d.mg_nu2, d.mg_max_cycles, d.mg_coarse_sweeps = 2, 1, 50, 8
    assert lib.ew_op_create(ctypes.byref(g), ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert b"n_its" in lib.ew_last_error()
    d.n_its = 10
    for field, bad in (("mg_relax", 2.0), ("mg_relax", -0.5), ("mg_relax_coarse", 2.5)):
        setattr(d, field, bad)
        assert lib.ew_op_create(ctypes.byref(g), ctypes.byref(d), None, ctypes.byref(h)) == -1
        assert field.encode() in lib.ew_last_error()
        setattr(d, field, 0.0)
    d.omega = -1.0
    assert lib.ew_op_create(ctypes.byref(g), ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert lib.ew_op_apply_filter(None, None, None) == -1


def test_single_hip_runtime_in_process():
    """The library binds to the HIP runtime PyTorch already loaded (a second
    runtime in the process would not see the same devices and streams)."""
    from paper_2507_18282_amd import _lib
    _lib.load()
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    assert len(paths) == 1, paths


def test_neumann_walls_rejected_where_not_implemented():
    """Validation runs before any device work, so it is checked here through
    the raw ABI: with Neumann walls the implicit projection and network
    guesses are rejected (EW_ERR_UNSUPPORTED; both assume a symmetric M), and
    an axis with a Neumann wall needs at least 3 points."""
    import ctypes
    from paper_2507_18282_amd import _lib
    lib = _lib.load()

    def create(n0, ts, predictor="zero"):
        g = _lib.GridDesc()
        g.dim = 2
        g.n[0], g.n[1], g.n[2] = n0, 15, 1
        g.len[0], g.len[1], g.len[2] = 1.0, 1.0, 1.0
        g.order = 2
        g.walls[0][0] = _lib.WALL_NEUMANN
        d = _lib.OpDesc()
        d.omega, d.ts, d.cfl, d.n_its, d.n_p = 10.0, _lib.TS[ts], 0.5, 10, 1
        d.mg_tol, d.mg_nu1, d.mg_nu2, d.mg_max_cycles, d.mg_coarse_sweeps = 1e-10, 2, 1, 100, 8
        d.predictor = _lib.PREDICTOR[predictor]
        h = ctypes.c_void_p()
        return lib.ew_op_create(ctypes.byref(g), ctypes.byref(d), None, ctypes.byref(h))

    assert create(15, "implicit", "proj") == -7  # EW_ERR_UNSUPPORTED
    assert b"symmetric" in lib.ew_last_error()
    assert create(15, "implicit", "cnn") == -7
    assert create(2, "explicit") == -1  # EW_ERR_INVALID_ARG


def test_mapped_grid_validation():
    """ew_op_create_mapped validates the combination and the coordinates on
    the host before any device work: 3D, order 4, Neumann walls, mixed
    precision and the implicit PROJ and CNN guesses are EW_ERR_UNSUPPORTED;
    null coordinates, non-finite coordinates and a map whose Jacobian is not
    positive at some node (walls included) are EW_ERR_INVALID_ARG."""
    import ctypes

    import numpy as np

    import synthetic
    from paper_2507_18282_amd import _lib
    lib = _lib.load()
    n = (12, 9)
    good = synthetic.mapped_coords("skew", *n, eps=0.15)

    def create(xy, order=2, ts="explicit", precision="fp64", neumann=False, dim=2, predictor="zero"):
        g = _lib.GridDesc()
        g.dim = dim
        g.n[0], g.n[1], g.n[2] = n[0], n[1], 5
        g.len[0], g.len[1], g.len[2] = 1.0, 1.0, 1.0
        g.order = order
        if neumann:
            g.walls[1][0] = _lib.WALL_NEUMANN
        d = _lib.OpDesc()
        d.omega, d.ts, d.cfl, d.n_its, d.n_p = 10.0, _lib.TS[ts], 0.5, 10, 1
        d.precision = _lib.PRECISION[precision]
        d.mg_tol, d.mg_nu1, d.mg_nu2, d.mg_max_cycles, d.mg_coarse_sweeps = 1e-10, 2, 1, 100, 8
        d.predictor = _lib.PREDICTOR[predictor]
        h = ctypes.c_void_p()
        p = None if xy is None else np.ascontiguousarray(xy).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return lib.ew_op_create_mapped(ctypes.byref(g), ctypes.byref(d), p, None, ctypes.byref(h))

    assert create(good, order=4) == -7
    assert create(good, ts="implicit", predictor="proj") == -7
    assert create(good, ts="implicit", predictor="cnn") == -7
    assert create(good, precision="mixed") == -7
    assert create(good, neumann=True) == -7
    assert create(good, dim=3) == -7
    assert create(None) == -1
    flipped = good.copy()
    flipped[0] = -flipped[0]  # mirror image: x_r < 0, so J < 0
    assert create(flipped) == -1
    assert b"Jacobian" in lib.ew_last_error()
    bad = good.copy()
    bad[1, 3, 4] = np.nan
    assert create(bad) == -1


def test_allocator_hooks_validated_on_host():
    from paper_2507_18282_amd import _lib
    lib = _lib.load()
    hook = _lib.ALLOC_FN(lambda nbytes, dev, stream, ctx: None)
    free = _lib.FREE_FN(lambda p, c: None)
    assert lib.ew_set_allocator(ctypes.cast(hook, ctypes.c_void_p), None, None) == -1
    assert b"both" in lib.ew_last_error()
    assert lib.ew_set_allocator(None, ctypes.cast(free, ctypes.c_void_p), None) == -1
    # restoring the default needs no device and succeeds while nothing is live
    assert lib.ew_set_allocator(None, None, None) == 0
