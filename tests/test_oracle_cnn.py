"""Pins of the FP64 network oracle (oracle/cnn.py) against things other than
itself: scipy's 2D correlation for the forward pass, central finite
differences for every parameter of the backward pass, crop/whole-grid
consistency of the valid convolutions, and torch's bfloat16 rounding."""
import numpy as np
import pytest
import scipy.signal
import torch

import synthetic
from oracle import cnn as C


def _theta(seed, scale=1.0):
    u = synthetic.uniform_pm1(seed, C.N_PARAMS)
    th = C.init_params(u, last_layer_zero=False) * scale
    # non-zero biases so that their gradients are exercised
    b = synthetic.uniform_pm1(seed + 1, C.N_PARAMS) * 0.1
    p = C.unpack(th.copy())
    for name in ("b1", "b2", "b3"):
        n = p[name].size
        p[name][...] = b[:n]
    return C.pack(p)


def _input(seed, h, w):
    return synthetic.uniform_pm1(seed, 4 * (h + 6) * (w + 6)).reshape(4, h + 6, w + 6)


def _forward_scipy(theta, x):
    """The same network written with scipy.signal.correlate2d, channel by channel."""
    p = C.unpack(theta)

    def layer(inp, w, b, relu):
        out = []
        for o in range(w.shape[0]):
            acc = np.full((inp.shape[1] - 2, inp.shape[2] - 2), b[o])
            for i in range(w.shape[1]):
                acc = acc + scipy.signal.correlate2d(inp[i], w[o, i], mode="valid")
            out.append(np.maximum(acc, 0.0) if relu else acc)
        return np.array(out)

    a1 = layer(x, p["W1"], p["b1"], True)
    a2 = layer(a1, p["W2"], p["b2"], True)
    return layer(a2, p["W3"], p["b3"], False)[0]


def test_param_count_and_layout():
    assert C.N_PARAMS == 16 * 4 * 9 + 16 + 16 * 16 * 9 + 16 + 16 * 9 + 1 == 3057
    th = np.arange(C.N_PARAMS, dtype=np.float64)
    assert np.array_equal(C.pack(C.unpack(th)), th)
    p = C.unpack(th)
    assert p["W1"][0, 0, 0, 1] == 1 and p["b1"][0] == 576 and p["W2"][0, 0, 0, 0] == 592
    assert p["b3"][0] == C.N_PARAMS - 1


@pytest.mark.parametrize("hw", [(5, 7), (12, 9)])
def test_forward_matches_scipy_correlate(hw):
    th = _theta(11)
    x = _input(21, *hw)
    y, _ = C.forward(th, x)
    assert y.shape == hw
    ref = _forward_scipy(th, x)
    assert np.max(np.abs(y - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_single_tap_kernel_is_a_shift():
    """A network whose only non-zero weights pick input channel 0 at tap
    (ky, kx) in each layer returns that channel shifted by the summed offsets
    (inputs kept positive so that ReLU is the identity)."""
    p = C.unpack(np.zeros(C.N_PARAMS))
    p["W1"][0, 0, 2, 0] = 1.0   # offset (+1, -1)
    p["W2"][0, 0, 1, 2] = 1.0   # offset (0, +1)
    p["W3"][0, 0, 0, 0] = 1.0   # offset (-1, -1)
    th = C.pack(p)
    h, w = 6, 5
    x = np.zeros((4, h + 6, w + 6))
    x[0] = 1.0 + np.arange((h + 6) * (w + 6)).reshape(h + 6, w + 6)
    y, _ = C.forward(th, x)
    # output (p, q) reads input (p + 3 + dy, q + 3 + dx) with dy = 0, dx = -1
    assert np.array_equal(y, x[0, 3:3 + h, 2:2 + w])


def test_gradient_matches_central_differences_all_parameters():
    th = _theta(31)
    x = _input(41, 4, 5)
    t = synthetic.uniform_pm1(51, 20).reshape(4, 5)
    loss, g = C.loss_and_grad(th, x, t)
    eps = 1e-6
    fd = np.zeros(C.N_PARAMS)
    for i in range(C.N_PARAMS):
        tp = th.copy()
        tp[i] += eps
        tm = th.copy()
        tm[i] -= eps
        lp = np.mean((C.forward(tp, x)[0] - t) ** 2)
        lm = np.mean((C.forward(tm, x)[0] - t) ** 2)
        fd[i] = (lp - lm) / (2 * eps)
    assert loss == pytest.approx(np.mean((C.forward(th, x)[0] - t) ** 2), rel=1e-14)
    err = np.abs(fd - g)
    assert np.max(err) <= 1e-6 * max(1.0, np.max(np.abs(g))), np.argmax(err)
    # every layer's weights and biases actually receive gradient
    p = C.unpack(g)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert np.max(np.abs(p[name])) > 0, name


def test_crop_with_halo_reproduces_whole_grid_output():
    """Valid convolutions: a crop that carries three extra cells on each side
    gives exactly the whole-grid output on its interior."""
    th = _theta(61)
    h, w = 20, 17
    x = _input(71, h, w)
    y, _ = C.forward(th, x)
    r0, c0, hh, ww = 5, 3, 9, 11
    yc, _ = C.forward(th, x[:, r0:r0 + hh + 6, c0:c0 + ww + 6])
    assert np.array_equal(yc, y[r0:r0 + hh, c0:c0 + ww])


def test_guess_residual_form():
    """With W3 = 0 and b3 = 0 the guess is the scaled guess 2 W^n / (1 + a w^2);
    with the exact target added it is the solution itself."""
    th = _theta(81)
    p = C.unpack(th.copy())
    p["W3"][...] = 0.0
    p["b3"][...] = 0.0
    th0 = C.pack(p)
    wn = synthetic.uniform_pm1(91, 12 * 10).reshape(12, 10)
    wp = synthetic.uniform_pm1(92, 12 * 10).reshape(12, 10)
    a, om, h = 2e-4, 30.0, 1.0 / 11
    g = C.predict_guess(th0, wn, wp, a, om, h)
    assert np.allclose(g, 2 * wn / (1 + a * om * om), rtol=0, atol=1e-15)
    assert np.all(C.predict_guess(th, np.zeros_like(wn), wp, a, om, h) == 0.0)
    c2, c3 = C.step_planes(a, om, h)
    assert c2 == pytest.approx(a * om * om / (1 + a * om * om)) and 0 < c3 <= 1
    x = C.make_input(wn, wp, 2.0, c2, c3)
    assert x.shape == (4, 18, 16)
    assert np.all(x[:, :3] == 0) and np.all(x[:, :, -3:] == 0)
    assert np.all(x[2, 3:-3, 3:-3] == c2) and np.array_equal(x[0, 3:-3, 3:-3], wn / 2.0)


def test_round_bf16_matches_torch():
    v = np.concatenate([synthetic.uniform_pm1(101, 4000) * 10.0 ** np.arange(-20, 20, 0.01),
                        [0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e38, 1e-40]])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.round_bf16(v), ref)


def test_adam_first_step_and_constant_gradient():
    """Adam's first step from zero moments is -lr g / (|g| + eps) (the bias
    corrections cancel the (1 - beta) factors); under a constant gradient
    every later step has the same size."""
    g = synthetic.uniform_pm1(111, 50)
    th0 = synthetic.uniform_pm1(112, 50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = C.adam_step(th0, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    assert np.allclose(th1, th0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    th = th1
    for t in range(2, 6):
        th_new, m, v = C.adam_step(th, m, v, g, t, lr, eps=eps)
        assert np.allclose(th_new - th, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)
        th = th_new


# ---------------------------------------------------------------------------
# The residual form: loss points, the crop operator, the residual loss and its
# gradient, and the corrected guess.
# ---------------------------------------------------------------------------
from oracle import discrete as D  # noqa: E402
from oracle import wave as W  # noqa: E402


def test_crop_loss_points_interior_and_walls():
    """Order 4 reaches two cells: an interior crop loses two rows and columns
    on every side; a crop at the grid's corner keeps the rows and columns on
    its wall sides (the closure replaces the neighbours beyond a wall)."""
    m = C.crop_loss_points((40, 50), (10, 12), 16, 4)
    assert m.shape == (16, 16) and m.sum() == 12 * 12
    assert m[2:14, 2:14].all() and not m[:2].any() and not m[:, 14:].any()
    m = C.crop_loss_points((40, 50), (0, 34), 16, 4)      # top wall, right wall (34 + 16 = 50)
    assert m[0:14, 2:16].all() and not m[14:].any() and not m[:, :2].any()
    assert C.crop_loss_points((40, 50), (10, 12), 16, 2).sum() == 14 * 14


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("origin", [(3, 5), (0, 0), (13, 11)])
def test_residual_loss_matches_dense_operator(order, origin):
    """The residual loss equals sum over the loss points of (t - M y)^2 / npix
    with M = I - a L_h assembled as a dense matrix on the whole grid and y
    placed in the window (zero elsewhere)."""
    ny, nx, crop = 20, 18, 7
    shape = (ny, nx)
    h = D.spacing((nx, ny), (1.0, 1.1))
    a = 3e-4
    th = _theta(121)
    x = _input(122, crop, crop)
    t = synthetic.uniform_pm1(123, crop * crop).reshape(crop, crop)
    loss, _ = C.residual_loss_and_grad(th, x, t, shape, origin, h, order, a)
    y, _ = C.forward(th, x)
    M = np.eye(nx * ny) - a * D.laplacian_matrix((nx, ny), h, order)
    full = np.zeros(shape)
    oy, ox = origin
    full[oy:oy + crop, ox:ox + crop] = y
    My = (M @ full.ravel()).reshape(shape)[oy:oy + crop, ox:ox + crop]
    mask = C.crop_loss_points(shape, origin, crop, order)
    want = np.sum(np.where(mask, t - My, 0.0) ** 2) / crop ** 2
    assert loss == pytest.approx(want, rel=1e-13)
    # and on the loss points M y does not depend on values outside the window
    full2 = full.copy()
    full2[:oy] = 7.0
    full2[oy + crop:] = -3.0
    My2 = (M @ full2.ravel()).reshape(shape)[oy:oy + crop, ox:ox + crop]
    assert np.max(np.abs(np.where(mask, My - My2, 0.0))) == 0.0


@pytest.mark.parametrize("origin", [(4, 6), (0, 11)])
def test_residual_loss_gradient_matches_central_differences(origin):
    ny, nx, crop = 16, 16, 5
    shape = (ny, nx)
    h = D.spacing((nx, ny), (1.0, 1.0))
    a = 5e-3
    th = _theta(131)
    x = _input(132, crop, crop)
    t = synthetic.uniform_pm1(133, crop * crop).reshape(crop, crop)
    loss, g = C.residual_loss_and_grad(th, x, t, shape, origin, h, 4, a)
    idx = np.concatenate([np.arange(0, C.N_PARAMS, 7), [C.N_PARAMS - 1, 575, 591, 2911]])
    eps = 1e-6
    for i in idx:
        tp = th.copy()
        tp[i] += eps
        tm = th.copy()
        tm[i] -= eps
        lp, _ = C.residual_loss_and_grad(tp, x, t, shape, origin, h, 4, a)
        lm, _ = C.residual_loss_and_grad(tm, x, t, shape, origin, h, 4, a)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.max(np.abs(g))), (i, fd, g[i])
    p = C.unpack(g)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert np.max(np.abs(p[name])) > 0, name


def test_corrected_guess_degenerate_cases():
    """A network that outputs the constant beta (all weights zero, b3 = beta)
    moves the base guess by s * beta with s the RMS of its residual; an exact
    base guess has no residual and is returned unchanged."""
    n = (12, 10)
    h = D.spacing(n, (1.0, 1.0))
    a, om = 4e-4, 20.0
    p = C.unpack(np.zeros(C.N_PARAMS))
    p["b3"][0] = 0.25
    th = C.pack(p)
    b = synthetic.uniform_pm1(141, 120).reshape(10, 12)
    x0 = synthetic.uniform_pm1(142, 120).reshape(10, 12) * 0.1
    r = b - C.apply_M(x0, h, 4, a)
    s = np.sqrt(np.mean(r * r))
    g = C.predict_correction(th, x0, b, h, 4, a, om)
    assert np.allclose(g, x0 + 0.25 * s, rtol=0, atol=1e-14)
    xe = W.solve_implicit_exact(b, h, 4, np.sqrt(2 * a))
    ge = C.predict_correction(_theta(143), xe, b, h, 4, a, om)
    assert np.max(np.abs(ge - xe)) <= 1e-12 * np.max(np.abs(xe))
    xin = C.make_input_residual(r, b, s, 2.0, 0.5, 0.25)
    assert np.array_equal(xin[0, 3:-3, 3:-3], r / s) and np.array_equal(xin[1, 3:-3, 3:-3], b / 2.0)
    assert np.all(xin[:, :3] == 0) and np.all(xin[3, 3:-3, 3:-3] == 0.25)


def test_default_init_returns_the_base_guess():
    """The default initialisation zeroes the last layer: the untrained network
    outputs 0, so the corrected guess is the base guess; the hidden layers are
    the He-scaled draws."""
    u = synthetic.uniform_pm1(151, C.N_PARAMS)
    th = C.init_params(u)
    p, q = C.unpack(th), C.unpack(C.init_params(u, last_layer_zero=False))
    assert np.all(p["W3"] == 0) and np.all(p["b3"] == 0) and np.any(q["W3"] != 0)
    assert np.array_equal(p["W1"], q["W1"]) and np.array_equal(p["W2"], q["W2"])
    n = (9, 8)
    h = D.spacing(n, (1.0, 1.0))
    b = synthetic.uniform_pm1(152, 72).reshape(8, 9)
    x0 = 0.1 * synthetic.uniform_pm1(153, 72).reshape(8, 9)
    assert np.array_equal(C.predict_correction(th, x0, b, h, 4, 1e-3, 10.0), x0)
