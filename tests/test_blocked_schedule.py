"""The multi-step explicit launches as a schedule, on the CPU (eqs.
explicitStep1, explicitScheme and filterQuadrature; the same schedule drives
the box, mapped-grid and FP64-batch kernels).

A launch advances up to 8 / R steps (R the stencil's radius): every 16 x 16
output tile loads a region with an 8-point halo, and after step s only the
points at least R (s + 1) from the region's edge are current.  Values a
region cannot know spread inward by R per step, so the halo bounds the
steps per launch (one step more fails these tests); updating only the
current points keeps every read inside the region, which the kernels' LDS
holds, and saves the rest.  Points beyond a wall read 0 in the region and
the wall closures replace them as in one step per launch.  Each update then
uses exactly the values one launch per step would use, so the two schedules
agree bit for bit (numpy evaluates the same expression elementwise in
both); both agree with the oracle's wall operator to rounding.  Sizes cover
a grid smaller than one tile, ragged tiles, Neumann and mixed walls, and
step counts that end inside a launch.
"""
import numpy as np
import pytest

from oracle import walls as Wl

TILE, HALO = 16, 8
SIDE = TILE + 2 * HALO
PAD = 2  # zero cells around a frame so that shifts by +-2 stay inside


def d2_framed(F, gidx, n, uc, nlo, nhi, order, axis):
    """Second difference along `axis` of the frame F (PAD zero cells around
    the positions of uc) with the Dirichlet (odd) and Neumann (even) wall
    closures, written as the kernels' d2_framed."""
    def sh(o):
        if axis == 1:
            return F[PAD:F.shape[0] - PAD, PAD + o:F.shape[1] - PAD + o]
        return F[PAD + o:F.shape[0] - PAD + o, PAD:F.shape[1] - PAD]
    l1, r1 = sh(-1), sh(1)
    l1 = np.where((gidx == 0) & nlo, r1, l1)
    r1 = np.where((gidx == n - 1) & nhi, l1, r1)
    if order == 2:
        return l1 + r1 - 2.0 * uc
    l2, r2 = sh(-2), sh(2)
    l2n = np.where(gidx == 0, r2 if nlo else -uc, np.where((gidx == 1) & nlo, uc, l2))
    r2n = np.where(gidx == n - 1, l2 if nhi else -uc, np.where((gidx == n - 2) & nhi, uc, r2))
    return 16.0 * (l1 + r1) - (l2n + r2n) - 30.0 * uc


def lap_frame(U, gx, gy, nx, ny, order, cx, cy, wall):
    F = np.pad(U, PAD)
    s = d2_framed(F, gx, nx, U, bool(wall & 1), bool(wall & 2), order, 1) * cx
    s = s + d2_framed(F, gy, ny, U, bool(wall & 4), bool(wall & 8), order, 0) * cy
    return s


def lap_mapped(U, gx, gy, nx, ny, cw, cs, cb, ij):
    """The mapped-grid operator as the kernels form it: conservative A11 and
    A22 differences at half points plus the two cross terms, scaled by 1/J;
    coefficients beyond the walls read 0."""
    F = np.pad(U, 1)
    sh = lambda ox, oy: F[1 + oy:F.shape[0] - 1 + oy, 1 + ox:F.shape[1] - 1 + ox]
    uc, uW, uE, uS, uN = U, sh(-1, 0), sh(1, 0), sh(0, -1), sh(0, 1)
    uSW, uSE, uNW, uNE = sh(-1, -1), sh(1, -1), sh(-1, 1), sh(1, 1)

    def at(A, x, y, xmax, ymax):
        ok = (x >= 0) & (x < xmax) & (y >= 0) & (y < ymax)
        return np.where(ok, A[np.clip(y, 0, ymax - 1), np.clip(x, 0, xmax - 1)], 0.0)
    inside = (gx >= 0) & (gx < nx) & (gy >= 0) & (gy < ny)
    wl = np.where(inside, at(cw, gx, gy, nx + 1, ny), 0.0)
    wr = np.where(inside, at(cw, gx + 1, gy, nx + 1, ny), 0.0)
    ss = np.where(inside, at(cs, gx, gy, nx, ny + 1), 0.0)
    sn = np.where(inside, at(cs, gx, gy + 1, nx, ny + 1), 0.0)
    bE, bW = at(cb, gx + 1, gy, nx, ny), at(cb, gx - 1, gy, nx, ny)
    bN, bS = at(cb, gx, gy + 1, nx, ny), at(cb, gx, gy - 1, nx, ny)
    t = wr * (uE - uc) - wl * (uc - uW)
    t = t + (sn * (uN - uc) - ss * (uc - uS))
    t = t + (bE * (uNE - uSE) - bW * (uNW - uSW))
    t = t + (bN * (uNE - uNW) - bS * (uSE - uSW))
    return at(ij, gx, gy, nx, ny) * t


def per_step(v, lap_at, dt2, cf, n_t):
    ny, nx = v.shape
    gy, gx = np.mgrid[0:ny, 0:nx]
    lap = lambda U: lap_at(U, gx, gy)
    cur = v + (0.5 * dt2) * lap(v)
    acc = cf[0] * v + cf[1] * cur
    prev = v
    for k in range(1, n_t):
        nxt = 2.0 * cur - prev + dt2 * lap(cur)
        acc = acc + cf[k + 1] * nxt
        prev, cur = cur, nxt
    return acc


def blocked(v, R, lap_at, dt2, cf, n_t):
    """The launches of 8 / R steps: R is the stencil's reach (1 for order 2
    and the nine-point mapped operator, 2 for order 4)."""
    ny, nx = v.shape
    per = HALO // R
    yy, xx = np.mgrid[0:SIDE, 0:SIDE]
    depth = np.minimum(np.minimum(xx, SIDE - 1 - xx), np.minimum(yy, SIDE - 1 - yy))
    src_cur, src_prev = v, None
    acc = np.full((ny, nx), np.nan)
    for k0 in range(0, n_t, per):
        ns = min(per, n_t - k0)
        first = k0 == 0
        dst_cur = np.full((ny, nx), np.nan)
        dst_prev = np.full((ny, nx), np.nan)
        for by in range(-(-ny // TILE)):
            for bx in range(-(-nx // TILE)):
                gx = bx * TILE - HALO + xx
                gy = by * TILE - HALO + yy
                inside = (gx >= 0) & (gx < nx) & (gy >= 0) & (gy < ny)
                cx_, cy_ = np.clip(gx, 0, nx - 1), np.clip(gy, 0, ny - 1)
                cur = np.where(inside, src_cur[cy_, cx_], 0.0)
                prev = np.zeros_like(cur) if first else np.where(inside, src_prev[cy_, cx_], 0.0)
                out = inside & (depth >= HALO)
                fsum = np.zeros_like(cur) if first else np.where(out, acc[cy_, cx_], 0.0)
                for s in range(ns):
                    active = inside & (depth >= R * (s + 1))
                    assert not np.any(active & (depth < R))  # reads stay in the region
                    lap = lap_at(cur, gx, gy)
                    if first and s == 0:
                        wn = cur + (0.5 * dt2) * lap
                        fn = cf[0] * cur + cf[1] * wn
                    else:
                        wn = 2.0 * cur - prev + dt2 * lap
                        fn = fsum + cf[k0 + s + 1] * wn
                    # a point no longer current keeps a value no current point reads
                    fsum = np.where(active, fn, fsum)
                    prev, cur = np.where(active, cur, prev), np.where(active, wn, cur)
                dst_cur[gy[out], gx[out]] = cur[out]
                dst_prev[gy[out], gx[out]] = prev[out]
                acc[gy[out], gx[out]] = fsum[out]
        src_cur, src_prev = dst_cur, dst_prev
    return acc


CASES = [
    # (nx, ny, order, walls bits: x low/high, y low/high Neumann; N_t)
    (5, 3, 4, 0b1111, 5),       # smaller than one tile, Neumann all round
    (37, 21, 2, 0b0000, 17),    # ragged tiles, a last launch of one step
    (37, 21, 4, 0b0000, 9),
    (20, 33, 4, 0b0101, 6),     # Neumann low walls
    (33, 18, 2, 0b1010, 8),     # Neumann high walls, N_t a multiple of 8
    (19, 17, 4, 0b0110, 13),    # mixed walls
]


@pytest.mark.parametrize("nx,ny,order,wall,n_t", CASES)
def test_blocked_schedule_equals_one_step_per_launch(nx, ny, order, wall, n_t):
    rng = np.random.default_rng(1000 + nx * ny + order)
    v = rng.uniform(-1.0, 1.0, (ny, nx))
    cf = rng.uniform(0.0, 1.0, n_t + 1)
    lap_at = lambda U, gx, gy: lap_frame(U, gx, gy, nx, ny, order, 1.3, 0.7, wall)
    a = per_step(v, lap_at, 0.01, cf, n_t)
    b = blocked(v, order // 2, lap_at, 0.01, cf, n_t)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("nx,ny,n_t", [(5, 3, 3), (1, 4, 9), (37, 21, 17), (16, 16, 8), (33, 17, 11)])
def test_blocked_schedule_on_the_mapped_operator(nx, ny, n_t):
    """The same for the nine-point operator of a mapped grid (random
    positive conservative coefficients, random cross terms)."""
    rng = np.random.default_rng(2000 + nx * ny)
    cw = rng.uniform(0.5, 1.5, (ny, nx + 1))
    cs = rng.uniform(0.5, 1.5, (ny + 1, nx))
    cb = rng.uniform(-0.2, 0.2, (ny, nx))
    ij = rng.uniform(0.5, 1.5, (ny, nx))
    v = rng.uniform(-1.0, 1.0, (ny, nx))
    cf = rng.uniform(0.0, 1.0, n_t + 1)
    lap_at = lambda U, gx, gy: lap_mapped(U, gx, gy, nx, ny, cw, cs, cb, ij)
    a = per_step(v, lap_at, 0.05, cf, n_t)
    b = blocked(v, 1, lap_at, 0.05, cf, n_t)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("nx,ny,order,wall,n_t", CASES[1:4])
def test_one_step_schedule_is_the_oracle_operator(nx, ny, order, wall, n_t):
    """The framed closures are the oracle's Dirichlet / Neumann wall operator
    (h = 1, so cx = cy = 1 at order 2 and 1/12 at order 4)."""
    rng = np.random.default_rng(7 + nx)
    U = rng.uniform(-1.0, 1.0, (ny, nx))
    gy, gx = np.mgrid[0:ny, 0:nx]
    c = 1.0 if order == 2 else 1.0 / 12.0
    got = lap_frame(U, gx, gy, nx, ny, order, c, c, wall)
    side = lambda b: "N" if b else "D"
    walls = ((side(wall & 1), side(wall & 2)), (side(wall & 4), side(wall & 8)))
    want = Wl.apply_laplacian(U, (1.0, 1.0), order, walls)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
