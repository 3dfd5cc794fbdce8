"""The small convolutional network used as the initial guess of each implicit
solve, in FP64: forward, losses and backward.

Test infrastructure only (see ``oracle/__init__``).  This network is not in
the paper; it is this project's learned warm start.  The paper solves each
implicit step M x = b (eqs. implicitScheme, impMatrix) with multigrid to a
relative residual tolerance (Sec. "An optimal O(N) eigenvalue solver"), so a
guess saves cycles only through its residual b - M x0.  The network therefore
corrects a base guess x0 (the projection on earlier solves, or zero) from that
base's residual, and is trained on the residual norm:

* input planes (4): r / s, b / s_b, and two constant planes
  c2 = a w^2 / (1 + a w^2) and c3 = min(a / h^2, 100) / 100 that tell the
  network which step it is looking at (a = dt^2/2, w the frequency used in the
  filter, h the grid spacing); r = b - M x0 is the base guess's residual, s
  its RMS over the grid and s_b the RMS of b;
* conv 3x3, 4 -> 16 channels, bias, ReLU; conv 3x3, 16 -> 16, bias, ReLU;
  conv 3x3, 16 -> 1, bias; zero values outside the domain (the Dirichlet wall);
* the guess is  x0 + s y;
* loss on a crop (a window of the grid, its network input carrying a
  three-cell halo): the mean over the window's points of e^2, where
  e = r / s - M y on the points whose stencil lies inside the window or
  reaches beyond a wall (M with the grid's wall closure), and e = 0 on the
  other points near the window's edges.  Minimising it minimises the initial
  residual that the multigrid solve has to remove.

The earlier form of the same network (planes W^n / s, W^{n-1} / s; target
(S - 2 W^n / (1 + a w^2)) / s; mean squared error) is kept below as
``loss_and_grad`` and ``predict_guess``: it is the plain regression the
residual form replaced.

Parameters are one flat vector in the order W1[16][4][3][3], b1[16],
W2[16][16][3][3], b2[16], W3[1][16][3][3], b3[1] (3057 values); a kernel
index [o][i][ky][kx] multiplies the input at offset (ky - 1, kx - 1).
Convolutions here are "valid" (an input of size H+6 gives an output of size H)
so that a crop carrying a three-cell halo reproduces the whole-grid network
exactly on its interior.
"""
from __future__ import annotations

import numpy as np

from .mg import apply_M

SHAPES = [("W1", (16, 4, 3, 3)), ("b1", (16,)), ("W2", (16, 16, 3, 3)), ("b2", (16,)),
          ("W3", (1, 16, 3, 3)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed_values: np.ndarray, last_layer_zero: bool = True) -> np.ndarray:
    """He-style initialisation from given uniform[-1,1) draws (one per parameter):
    weight ~ u * sqrt(6 / fan_in), biases zero; with last_layer_zero the last
    layer's weights start at zero too, so that the untrained network returns
    the base guess unchanged (a He-scaled last layer starts from a guess whose
    residual M y is hundreds of times that of the base, and Adam on the
    residual loss then settles on y = 0 instead of a correction)."""
    theta = np.zeros(N_PARAMS)
    off = 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        if name.startswith("W") and not (last_layer_zero and name == "W3"):
            fan_in = shape[1] * 9
            theta[off:off + n] = seed_values[off:off + n] * np.sqrt(6.0 / fan_in)
        off += n
    return theta


def conv_valid(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[o, p, q] = b[o] + sum_{i,ky,kx} w[o,i,ky,kx] x[i, p+ky, q+kx]."""
    C, H, W = x.shape
    O = w.shape[0]
    out = np.zeros((O, H - 2, W - 2))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oi,ipq->opq", w[:, :, ky, kx], x[:, ky:ky + H - 2, kx:kx + W - 2])
    return out + b[:, None, None]


def forward(theta: np.ndarray, x: np.ndarray):
    """x: (4, H+6, W+6) -> y (H, W) and the cache for backward."""
    p = unpack(theta)
    z1 = conv_valid(x, p["W1"], p["b1"])
    a1 = np.maximum(z1, 0.0)
    z2 = conv_valid(a1, p["W2"], p["b2"])
    a2 = np.maximum(z2, 0.0)
    y = conv_valid(a2, p["W3"], p["b3"])[0]
    return y, (x, z1, a1, z2, a2)


def conv_valid_backward(x: np.ndarray, w: np.ndarray, dout: np.ndarray):
    """Gradients of conv_valid with respect to w, b and x."""
    C, H, W = x.shape
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for ky in range(3):
        for kx in range(3):
            xs = x[:, ky:ky + H - 2, kx:kx + W - 2]
            dw[:, :, ky, kx] = np.einsum("opq,ipq->oi", dout, xs)
            dx[:, ky:ky + H - 2, kx:kx + W - 2] += np.einsum("oi,opq->ipq", w[:, :, ky, kx], dout)
    db = dout.sum(axis=(1, 2))
    return dw, db, dx


def backward_from_dy(theta: np.ndarray, cache, dy: np.ndarray) -> np.ndarray:
    """Gradient of a loss with respect to the parameters, given dL/dy."""
    x, z1, a1, z2, a2 = cache
    p = unpack(theta)
    dW3, db3, da2 = conv_valid_backward(a2, p["W3"], dy[None])
    dz2 = da2 * (z2 > 0)
    dW2, db2, da1 = conv_valid_backward(a1, p["W2"], dz2)
    dz1 = da1 * (z1 > 0)
    dW1, db1, _ = conv_valid_backward(x, p["W1"], dz1)
    return pack({"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3})


def loss_and_grad(theta: np.ndarray, x: np.ndarray, target: np.ndarray):
    """Mean squared error of y against target and its gradient (backpropagation)."""
    y, cache = forward(theta, x)
    npix = y.size
    r = y - target
    loss = float(np.sum(r * r) / npix)
    return loss, backward_from_dy(theta, cache, (2.0 / npix) * r)


def crop_loss_points(grid_shape, origin, crop: int, order: int) -> np.ndarray:
    """Mask over a crop x crop window at `origin` (row, col) of a grid of numpy
    shape `grid_shape`: True where every stencil neighbour (reach order / 2
    per direction) lies inside the window or beyond a wall of the grid."""
    R = order // 2
    ny, nx = grid_shape
    oy, ox = origin
    rows = np.arange(crop)
    cols = np.arange(crop)
    ok_r = ((rows >= R) | (oy == 0)) & ((rows <= crop - 1 - R) | (oy + crop == ny))
    ok_c = ((cols >= R) | (ox == 0)) & ((cols <= crop - 1 - R) | (ox + crop == nx))
    return ok_r[:, None] & ok_c[None, :]


def crop_M(y: np.ndarray, grid_shape, origin, h, order: int, a: float) -> np.ndarray:
    """M applied to the grid function that equals y on the window and zero
    elsewhere (the oracle's M with its wall closures), read on the window."""
    ny, nx = grid_shape
    oy, ox = origin
    c = y.shape[0]
    full = np.zeros((ny, nx))
    full[oy:oy + c, ox:ox + c] = y
    return apply_M(full, h, order, a)[oy:oy + c, ox:ox + c]


def residual_loss_and_grad(theta: np.ndarray, x: np.ndarray, target: np.ndarray, grid_shape, origin, h,
                           order: int, a: float, npix: int = None):
    """Residual loss of one crop: y = network(x) on the window, e = target -
    M y on the loss points (crop_loss_points), 0 elsewhere; loss = sum e^2 /
    npix (npix defaults to the window's point count) and its gradient: dL/dy
    = -(2 / npix) M^T e, and M is symmetric (its closures keep L_h
    symmetric), so M^T e is crop_M applied to e."""
    y, cache = forward(theta, x)
    crop = y.shape[0]
    npix = crop * crop if npix is None else npix
    mask = crop_loss_points(grid_shape, origin, crop, order)
    e = np.where(mask, target - crop_M(y, grid_shape, origin, h, order, a), 0.0)
    loss = float(np.sum(e * e) / npix)
    dy = -(2.0 / npix) * crop_M(e, grid_shape, origin, h, order, a)
    return loss, backward_from_dy(theta, cache, dy)


def step_planes(a: float, omega: float, h: float):
    """The two constant input planes of one implicit step."""
    c2 = a * omega * omega / (1.0 + a * omega * omega)
    c3 = min(a / (h * h), 100.0) / 100.0
    return c2, c3


def make_input(wn: np.ndarray, wprev: np.ndarray, s: float, c2: float, c3: float, halo: int = 3) -> np.ndarray:
    """Network input over the whole grid with `halo` zero cells outside the walls."""
    H, W = wn.shape
    x = np.zeros((4, H + 2 * halo, W + 2 * halo))
    x[0, halo:halo + H, halo:halo + W] = wn / s
    x[1, halo:halo + H, halo:halo + W] = wprev / s
    # the constant planes are zero outside the domain, like the fields
    x[2, halo:halo + H, halo:halo + W] = c2
    x[3, halo:halo + H, halo:halo + W] = c3
    return x


def make_input_residual(r: np.ndarray, b: np.ndarray, s: float, s_b: float, c2: float, c3: float,
                        halo: int = 3) -> np.ndarray:
    """Planes r / s, b / s_b, c2, c3 over the whole grid with `halo` zero cells
    outside the walls (a zero residual gives a zero first plane)."""
    H, W = r.shape
    x = np.zeros((4, H + 2 * halo, W + 2 * halo))
    if s > 0.0:
        x[0, halo:halo + H, halo:halo + W] = r / s
    if s_b > 0.0:
        x[1, halo:halo + H, halo:halo + W] = b / s_b
    x[2, halo:halo + H, halo:halo + W] = c2
    x[3, halo:halo + H, halo:halo + W] = c3
    return x


def predict_correction(theta: np.ndarray, x0: np.ndarray, b: np.ndarray, h, order: int, a: float, omega: float):
    """Guess x0 + s y for M x = b from the base guess x0 (residual form)."""
    r = b - apply_M(x0, h, order, a)
    s = float(np.sqrt(np.mean(r * r)))
    s_b = float(np.sqrt(np.mean(b * b)))
    c2, c3 = step_planes(a, omega, h[0])
    y, _ = forward(theta, make_input_residual(r, b, s, s_b, c2, c3))
    return x0 + s * y


def predict_guess(theta: np.ndarray, wn: np.ndarray, wprev: np.ndarray, a: float, omega: float, h: float):
    """Initial guess S0 = 2 W^n / (1 + a w^2) + s y for the solve of M S = 2 W^n."""
    s = float(np.sqrt(np.mean(wn * wn)))
    if s == 0.0:
        return np.zeros_like(wn)
    c2, c3 = step_planes(a, omega, h)
    y, _ = forward(theta, make_input(wn, wprev, s, c2, c3))
    return 2.0 * wn / (1.0 + a * omega * omega) + s * y


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def adam_step(theta: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015), step number t >= 1: moment
    estimates, their bias corrections 1/(1 - beta^t), and the scaled step."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
