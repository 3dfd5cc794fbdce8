"""Learned warm start on the GPU against the FP64 network oracle.

The kernels round the input planes and both activation layers to BF16 and
use BF16 weights with FP32 accumulation.  The oracle runs in FP64 with the
same BF16-rounded weights, and forward results are compared elementwise
against a running error bound carried through the network by the oracle
itself: every BF16 rounding contributes u |value| (u = 2^-8, twice the unit
roundoff 2^-9 of round-to-nearest BF16, covering the rounding of the
perturbed value and FP32 accumulation) and propagates through |W| (ReLU is
1-Lipschitz).  Gradients carry several such roundings per product, summed
over many points; they are compared in relative 2-norm per parameter block
at 2e-2 (about ten BF16 unit roundoffs).
"""
import numpy as np
import pytest

import synthetic
from oracle import cnn as C
from oracle import discrete as D
from oracle import wave as W
from tests.gpu_helpers import oracle_plan, say, to_dev, to_host

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8


def _params(seed, bias_scale=0.1):
    th = C.init_params(synthetic.uniform_pm1(seed, C.N_PARAMS), last_layer_zero=False)
    b = synthetic.uniform_pm1(seed + 1, 64) * bias_scale
    p = C.unpack(th)
    p["b1"][...] = b[:16]
    p["b2"][...] = b[16:32]
    p["b3"][...] = b[32:33]
    return C.pack(p).astype(np.float32)


def _effective(params32):
    """The network the kernels evaluate: BF16-rounded weights, FP32 biases."""
    th = params32.astype(np.float64)
    p = C.unpack(th.copy())
    for name in ("W1", "W2", "W3"):
        p[name][...] = C.round_bf16(p[name])
    return C.pack(p)


def _forward_with_bound(theta, x):
    y, (x, z1, a1, z2, a2) = C.forward(theta, x)
    p = C.unpack(theta)
    zb = np.zeros(16)

    def conv_abs(inp, w):
        return C.conv_valid(inp, np.abs(w), zb[:w.shape[0]])

    e0 = U_BF16 * np.abs(x)
    e1 = conv_abs(e0, p["W1"]) + U_BF16 * np.abs(a1) + 1e-6 * conv_abs(np.abs(x), p["W1"])
    e2 = conv_abs(e1, p["W2"]) + U_BF16 * np.abs(a2) + 1e-6 * conv_abs(a1, p["W2"])
    ey = conv_abs(e2, p["W3"])[0] + 1e-6 * conv_abs(a2, p["W3"])[0] + 1e-7
    return y, ey


# Window geometries of test crops: (grid shape (ny, nx), origin (oy, ox)) for a
# crop of side c; interior, top wall, right wall, bottom-left corner.
def _geometry(i, c):
    g = (c + 20, c + 20)
    return g, [(10, 10), (0, 10), (10, 20), (20, 0)][i % 4]


def _rect(grid, origin, c):
    """The padded window's rectangle inside the grid, as the collection writes it."""
    (ny, nx), (oy, ox) = grid, origin
    cp = c + 6
    return [max(0, 3 - oy), min(cp, ny - oy + 3), max(0, 3 - ox), min(cp, nx - ox + 3)]


AH = (0.75, 0.5)   # a / h_x^2, a / h_y^2 of the test crops (exact in FP32)


def _random_crops(n, crop, seed):
    """Random fields and targets on windows of the _geometry cases, zero outside
    their grids; planes (c2, c3, a/h_x^2, a/h_y^2)."""
    cp = crop + 6
    fields = synthetic.uniform_pm1(seed, n * 2 * cp * cp).reshape(n, 2, cp, cp).astype(np.float32)
    target = (0.3 * synthetic.uniform_pm1(seed + 1, n * crop * crop)).reshape(n, crop, crop).astype(np.float32)
    u = synthetic.uniform01(seed + 2, 2 * n)
    planes = np.stack([0.05 + 0.3 * u[:n], 0.9 * u[n:], np.full(n, AH[0]), np.full(n, AH[1])],
                      axis=1).astype(np.float32)
    rects = np.zeros((n, 4), dtype=np.int32)
    for i in range(n):
        rects[i] = _rect(*_geometry(i, crop), crop)
        r0, r1, c0, c1 = rects[i]
        mask = np.zeros((cp, cp), dtype=bool)
        mask[r0:r1, c0:c1] = True
        fields[i, :, ~mask] = 0.0
    return fields, target, planes, rects


def _oracle_input(fields, planes, rect):
    cp = fields.shape[-1]
    x = np.zeros((4, cp, cp))
    x[0] = fields[0]
    x[1] = fields[1]
    r0, r1, c0, c1 = rect
    x[2, r0:r1, c0:c1] = planes[0]
    x[3, r0:r1, c0:c1] = planes[1]
    return x


def _oracle_loss_grad(theta, fields, target, planes, rects, ids, crop, order):
    """Mean residual loss over the crops ids and its gradient (oracle): h = 1 per
    axis scaled so that a / h^2 are the crops' values."""
    n = len(ids)
    loss, g = 0.0, np.zeros(C.N_PARAMS)
    for i in ids:
        grid, origin = _geometry(i, crop)
        ahx, ahy = float(planes[i, 2]), float(planes[i, 3])
        h = (1.0, np.sqrt(ahx / ahy))          # a = ahx with h_x = 1 gives a / h_y^2 = ahy
        li, gi = C.residual_loss_and_grad(theta, _oracle_input(fields[i], planes[i], rects[i]),
                                          target[i].astype(np.float64), grid, origin, h, order, ahx,
                                          npix=n * crop * crop)
        loss += li
        g += gi
    return loss, g


def _store(fields, target, planes, rects, crop, capacity=None, order=4):
    from paper_2507_18282_amd import CropStore
    st = CropStore(capacity or len(planes), crop, order)
    st.append(to_dev(fields.ravel()).float(), to_dev(target.ravel()).float(), planes, rects)
    return st


def test_init_matches_oracle_draws():
    from paper_2507_18282_amd import Cnn
    for seed in (0, 5, 12345):
        got = Cnn(seed).get_params()
        ref = C.init_params(synthetic.uniform_pm1(seed, C.N_PARAMS)).astype(np.float32)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("crop", [16, 48])
def test_forward_on_crops_within_bf16_bound(crop):
    from paper_2507_18282_amd import Cnn
    say("cnn forward crops", crop)
    params = _params(3)
    n = 5
    fields, target, planes, rects = _random_crops(n, crop, 40 + crop)
    st = _store(fields, target, planes, rects, crop)
    net = Cnn(0)
    net.set_params(params)
    y = to_host(net.forward(st, 0, n))
    theta = _effective(params)
    for i in range(n):
        ref, bound = _forward_with_bound(theta, _oracle_input(fields[i], planes[i], rects[i]))
        err = np.abs(y[i] - ref)
        assert np.all(err <= bound), (i, float(np.max(err / bound)))
        # the bound is not vacuous: typical errors are far below it and below 1% of the output scale
        assert np.median(err) <= 1e-2 * np.std(ref)


def test_forward_subrange_and_repeatability():
    from paper_2507_18282_amd import Cnn
    params = _params(4)
    fields, target, planes, rects = _random_crops(6, 32, 77)
    st = _store(fields, target, planes, rects, 32)
    net = Cnn(0)
    net.set_params(params)
    y_all = to_host(net.forward(st, 0, 6))
    y_sub = to_host(net.forward(st, 2, 3))
    assert np.array_equal(y_all[2:5], y_sub)
    assert np.array_equal(y_all, to_host(net.forward(st, 0, 6)))


@pytest.mark.parametrize("order", [4, 2])
def test_residual_loss_and_gradient_match_oracle(order):
    from paper_2507_18282_amd import Cnn
    say("cnn residual loss/grad", order)
    params = _params(8)
    crop, n = 32, 4
    fields, target, planes, rects = _random_crops(n, crop, 91)
    st = _store(fields, target, planes, rects, crop, order=order)
    net = Cnn(0)
    net.set_params(params)
    loss, g = net.loss_grad(st, 0, n)
    g = to_host(g).astype(np.float64)
    theta = _effective(params)
    loss_ref, g_ref = _oracle_loss_grad(theta, fields, target, planes, rects, range(n), crop, order)
    assert abs(loss - loss_ref) <= 2e-2 * loss_ref
    gp, rp = C.unpack(g), C.unpack(g_ref)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        rel = np.linalg.norm(gp[name] - rp[name]) / np.linalg.norm(rp[name])
        assert rel <= 2e-2, (name, rel)
    # bitwise repeatable (fixed reduction order)
    loss2, g2 = net.loss_grad(st, 0, n)
    assert loss2 == loss and np.array_equal(to_host(g2), g.astype(np.float32))


def test_adam_first_step_matches_oracle():
    from paper_2507_18282_amd import Cnn
    params = _params(9)
    crop, n = 16, 6
    fields, target, planes, rects = _random_crops(n, crop, 123)
    st = _store(fields, target, planes, rects, crop)
    net = Cnn(0)
    net.set_params(params)
    lr, batch, seed = 1e-3, 4, 99
    net.train(st, steps=1, batch=batch, lr=lr, seed=seed)
    after = net.get_params().astype(np.float64)
    ids = np.minimum(np.floor(synthetic.uniform01(seed, batch) * n).astype(int), n - 1)
    theta = _effective(params)
    _, g_ref = _oracle_loss_grad(theta, fields, target, planes, rects, ids, crop, 4)
    th1, _, _ = C.adam_step(params.astype(np.float64), np.zeros(C.N_PARAMS), np.zeros(C.N_PARAMS), g_ref, 1, lr)
    step = after - params.astype(np.float64)
    assert np.all(np.abs(step) <= lr * (1 + 1e-5) + 1e-7)
    big = np.abs(g_ref) > 0.1 * np.max(np.abs(g_ref))
    assert big.sum() > 50
    assert np.allclose(step[big], (th1 - params)[big], rtol=2e-3, atol=1e-7)


def _implicit_op(n, order, omega, predictor="zero"):
    from paper_2507_18282_amd import Operator
    return Operator(n, (1.0, 1.0), order, omega, "implicit", n_its=10, mg_tol=1e-10, predictor=predictor)


def test_grid_guess_ragged_within_bound():
    """The correction on a ragged grid (tiles of 32 do not divide it) from a zero
    base (an empty projection window): the guess equals the oracle's s y, y the
    network on (r / s, b / s_b, c2, c3) with r = b, within s times the bound."""
    from paper_2507_18282_amd import Cnn
    say("cnn grid guess")
    nx, ny = 70, 45
    op = _implicit_op((nx, ny), 4, 25.0, predictor="cnn")
    net = Cnn(0)
    params = _params(12)
    net.set_params(params)
    op.set_cnn(net)
    b = 0.37 * synthetic.uniform_pm1(201, nx * ny)
    base = to_dev(np.full(nx * ny, 5.0))
    got = to_host(op.cnn_guess(to_dev(b), base=base)).reshape(ny, nx)
    assert np.all(to_host(base) == 0.0)
    a = 0.5 * op.dt ** 2
    h = (1.0 / (nx + 1), 1.0 / (ny + 1))
    theta = _effective(params)
    B = b.reshape(ny, nx)
    s = float(np.sqrt(np.mean(B * B)))
    c2, c3 = C.step_planes(a, op.omega_used, h[0])
    y, bound = _forward_with_bound(theta, C.make_input_residual(B, B, s, s, np.float32(c2), np.float32(c3)))
    ref = s * y
    assert np.all(np.abs(got - ref) <= s * bound + 1e-14)
    assert np.allclose(ref, C.predict_correction(theta, np.zeros_like(B), B, h, 4, a, op.omega_used), rtol=1e-6,
                       atol=1e-6 * s)
    assert op.stats()["cnn_guesses"] == 1


def _origin(n, crop, u):
    rng = n - crop + 1
    extra = rng // 8
    o = int(np.floor(u * (rng + 2 * extra))) - extra
    return min(max(o, 0), rng - 1)


def test_collect_crops_match_oracle_levels():
    """Crops recorded during a wave-solve of an operator whose base guess is the
    extrapolation x0 = b: fields (r / s, b / s_b) with b = 2 W^n from the
    oracle's time levels and r = b - M b, at the documented window origins
    (draws oy, ox per crop from the SplitMix64 stream)."""
    from paper_2507_18282_amd import CropStore
    from oracle import mg as OMG
    say("cnn collect")
    nx, ny, crop, per = 80, 64, 32, 2
    P = synthetic.Problem(n=(nx, ny), length=(1.0, 1.0), order=4, omega=20.0, ts="implicit", n_its=10,
                          k=1, m=4, seed=3)
    op = _implicit_op((nx, ny), 4, 20.0, predictor="extrap")
    h, plan = oracle_plan(P)
    v = synthetic.uniform_pm1(55, nx * ny)
    store = CropStore(64, crop, 4)
    seed = 17
    out = to_host(store.collect(op, to_dev(v), crops_per_step=per, seed=seed))
    acc, levels = W.apply_filter(v.reshape(ny, nx), h, 4, plan, return_levels=True)
    assert np.max(np.abs(out - acc.ravel())) <= 1e-8 * np.max(np.abs(acc))
    n_steps = plan.n_t - 1
    assert store.count == per * n_steps
    fields, target, planes, rects = store.read(0, store.count)
    fields, target = to_host(fields), to_host(target)
    u = synthetic.uniform01(seed, 2 * per * n_steps)
    a = 0.5 * plan.dt ** 2
    c2, c3 = C.step_planes(a, plan.omega, h[0])
    cp = crop + 6
    j = 0
    for n in range(1, plan.n_t):
        b = 2.0 * levels[n]
        r = b - OMG.apply_M(b, h, 4, a)
        s, sb = np.sqrt(np.mean(r * r)), np.sqrt(np.mean(b * b))
        pad_r, pad_b = np.pad(r / s, 3), np.pad(b / sb, 3)
        for _ in range(per):
            oy, ox = _origin(ny, crop, u[2 * j]), _origin(nx, crop, u[2 * j + 1])
            np.testing.assert_allclose(fields[j, 0], pad_r[oy:oy + cp, ox:ox + cp], rtol=0, atol=2e-6 * np.max(np.abs(pad_r)))
            np.testing.assert_allclose(fields[j, 1], pad_b[oy:oy + cp, ox:ox + cp], rtol=0, atol=2e-6 * np.max(np.abs(pad_b)))
            np.testing.assert_array_equal(target[j], fields[j, 0, 3:3 + crop, 3:3 + crop])
            assert planes[j, 0] == np.float32(c2) and planes[j, 1] == np.float32(c3)
            assert planes[j, 2] == np.float32(a / h[0] ** 2) and planes[j, 3] == np.float32(a / h[1] ** 2)
            assert list(rects[j]) == [max(0, 3 - oy), min(cp, ny - oy + 3), max(0, 3 - ox), min(cp, nx - ox + 3)]
            j += 1


def test_training_lowers_loss_and_is_deterministic():
    from paper_2507_18282_amd import Cnn, CropStore
    say("cnn train")
    nx = ny = 127
    op = _implicit_op((nx, ny), 4, 30.0, predictor="proj")
    store = CropStore(256, 32, 4)
    for r in range(4):
        v = to_dev(synthetic.uniform_pm1(300 + r, nx * ny))
        store.collect(op, v, crops_per_step=6, seed=400)
    assert store.count == 4 * 6 * (op.n_t - 1)
    runs = []
    for _ in range(2):
        net = Cnn(7)
        st = net.train(store, steps=150, batch=8, lr=2e-3, seed=5)
        runs.append((st, net.get_params()))
    assert runs[0][0]["last_loss"] < 0.5 * runs[0][0]["first_loss"]
    assert np.array_equal(runs[0][1], runs[1][1])
    assert runs[0][0]["last_loss"] == runs[1][0]["last_loss"]


@pytest.mark.parametrize("predictor", ["cnn", "scaled", "extrap", "proj"])
def test_warm_started_eigenpairs_equal_cold_start(predictor):
    """Whatever the initial guess (here an untrained network), multigrid runs
    to the same tolerance, so the eigenpairs agree with the cold start and with
    the closed form."""
    from paper_2507_18282_amd import Cnn
    say("warm start eigs", predictor)
    n, order, omega = 63, 4, 30.0
    cold = _implicit_op((n, n), order, omega)
    warm = _implicit_op((n, n), order, omega, predictor=predictor)
    if predictor == "cnn":
        net = Cnn(11)
        warm.set_cnn(net)
    rc = cold.eigs(4, 16, seed=3, tol_res=1e-8, want_vectors=False)
    rw = warm.eigs(4, 16, seed=3, tol_res=1e-8, want_vectors=False)
    mu_all = D.mu_all((n, n), (1.0 / (n + 1),) * 2, order).ravel()
    for x in rw.mu[:4]:
        assert np.min(np.abs(mu_all - x)) / x < 1e-9
    assert np.allclose(np.sort(rw.mu[:4]), np.sort(rc.mu[:4]), rtol=1e-9)
    if predictor == "cnn":
        assert warm.stats()["cnn_guesses"] > 0


def test_trained_network_lowers_initial_residual_on_held_out_solves():
    """Trained on the projection residuals of wave-solves from some start
    vectors, the network's guesses on wave-solves from other start vectors
    leave a smaller initial residual ||b - M x0|| / ||b|| than the projection
    guess they correct (both measured inside the solves), and the multigrid,
    iterated to the same tolerance, needs fewer V-cycles than from the zero
    guess on the same wave-solves."""
    from paper_2507_18282_amd import Cnn, CropStore
    say("cnn held-out residuals")
    nx = ny = 127
    store = CropStore(1200, 32, 4)
    for r in range(4):
        op = _implicit_op((nx, ny), 4, 30.0 + 10.0 * r, predictor="proj")
        w = to_dev(synthetic.uniform_pm1(600 + r, nx * ny))
        for _ in range(3):
            w = store.collect(op, w / w.norm(), crops_per_step=10, seed=601)
    net = Cnn(21)
    net.train(store, steps=600, batch=16, lr=2e-3, seed=8)
    net.train(store, steps=600, batch=16, lr=5e-4, seed=9)
    op = _implicit_op((nx, ny), 4, 35.0, predictor="cnn")
    op.set_cnn(net)
    op.probe_guesses(True)
    w = to_dev(synthetic.uniform_pm1(777, nx * ny))
    for _ in range(4):
        w = op.apply_filter(w / w.norm())
    st = op.stats()
    assert st["guess_probes"] == 4 * (op.n_t - 1) and st["cnn_guesses"] == st["guess_probes"]
    base, guess = st["base_rel_res_sum"], st["guess_rel_res_sum"]
    say("held-out mean relative residual: base", base / st["guess_probes"], "network", guess / st["guess_probes"])
    assert guess < 0.8 * base
    cold = _implicit_op((nx, ny), 4, 35.0, predictor="zero")
    w = to_dev(synthetic.uniform_pm1(777, nx * ny))
    for _ in range(4):
        w = cold.apply_filter(w / w.norm())
    warm_cycles, cold_cycles = st["mg_cycles"], cold.stats()["mg_cycles"]
    say("V-cycles over 4 wave-solves: learned", warm_cycles, "zero guess", cold_cycles)
    assert warm_cycles < cold_cycles
