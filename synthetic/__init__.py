"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module holds no arithmetic of the eigensolver: only the counter-based
random generator used for start vectors and batch draws, and the workload
presets (grid sizes, target frequencies, Krylov sizes) of the synthetic
problems.  Both the oracle (``oracle/``) and the GPU binding take their inputs
from here, and from nowhere else, so that they see identical data.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the finaliser constants are Vigna's public
version).  Element ``i`` of stream ``seed`` is the finaliser applied to
``seed + (i + 1) * 0x9E3779B97F4A7C15`` (mod 2**64), i.e. the value the
sequential generator returns on its ``(i+1)``-th call, so any element can be
produced independently.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Return ``count`` SplitMix64 outputs (uint64) of stream ``seed`` from ``offset``."""
    idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each SplitMix64 output times 2**-53."""
    z = splitmix64(seed, count, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_pm1(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [-1, 1): ``2 u - 1`` with ``u`` from :func:`uniform01`."""
    return 2.0 * uniform01(seed, count, offset) - 1.0


def start_vector(seed: int, n_active: int) -> np.ndarray:
    """Seeded uniform[-1,1] start vector over the active points, lexicographic
    with x fastest.  It is *not* normalised here: normalising is the first step
    of the Arnoldi process and belongs to each implementation."""
    return uniform_pm1(seed, n_active)


# --------------------------------------------------------------------------
# Workload presets.  Sizes count interior (active) points per dimension.
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Problem:
    """One synthetic Dirichlet box eigenproblem (all fields are inputs)."""

    n: Tuple[int, ...]            # interior points per dimension (x first)
    length: Tuple[float, ...]     # box side lengths (x first)
    order: int                    # 2 or 4
    omega: float                  # requested target frequency
    ts: str                       # "explicit" or "implicit"
    cfl: float = 0.5              # explicit only
    n_its: int = 10               # implicit only: steps per period
    n_p: int = 1                  # number of periods
    adjust_omega: bool = False    # use the adjusted target frequency
    filter_const: str = "alpha_d"  # "alpha_d" or "quarter"
    precision: str = "fp64"       # "fp64" or "mixed"
    mg_tol: float = 1e-10
    k: int = 4                    # eigenpairs requested
    m: int = 16                   # Krylov dimension
    seed: int = 1

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def n_active(self) -> int:
        return int(np.prod(self.n))


def config_small_explicit() -> Problem:
    """64x64 interior unit square, order 2, explicit leapfrog at CFL 0.5,
    omega = 15, Krylov dimension 16, 4 eigenpairs, seed 1."""
    return Problem(n=(64, 64), length=(1.0, 1.0), order=2, omega=15.0, ts="explicit",
                   cfl=0.5, k=4, m=16, seed=1)


def config_square_order4_implicit(n: int = 2047, omega: float = 120.0, n_p: int = 1,
                                  k: int = 16, m: int = 32, seed: int = 2) -> Problem:
    """Unit square with 2049x2049 total points (2047^2 interior, h = 1/2048),
    order 4, implicit 10 steps per period with multigrid to 1e-10, omega = 120
    (adjusted), Krylov dimension 32 for 16 eigenpairs."""
    return Problem(n=(n, n), length=(1.0, 1.0), order=4, omega=omega, ts="implicit",
                   n_its=10, n_p=n_p, adjust_omega=True, mg_tol=1e-10, k=k, m=m, seed=seed)


def config_cube_mixed(n: int = 255, omega: float = 40.0, k: int = 8, m: int = 17,
                      seed: int = 3) -> Problem:
    """Unit cube with 257^3 total points (255^3 interior), order 2, implicit 10
    steps per period, mixed precision, omega = 40 (adjusted), 8 eigenpairs."""
    return Problem(n=(n, n, n), length=(1.0, 1.0, 1.0), order=2, omega=omega,
                   ts="implicit", n_its=10, adjust_omega=True, precision="mixed",
                   mg_tol=1e-10, k=k, m=m, seed=seed)


def config_learned(n: int = 1023, omega: float = 90.0, k: int = 16, m: int = 32,
                   seed: int = 5) -> Problem:
    """Unit square with 1025^2 total points (1023^2 interior), order 4,
    implicit 10 steps per period, multigrid to 1e-10."""
    return Problem(n=(n, n), length=(1.0, 1.0), order=4, omega=omega, ts="implicit",
                   n_its=10, adjust_omega=True, mg_tol=1e-10, k=k, m=m, seed=seed)


def config_many_pairs(k: int = 256, n: int = 127, omega: float = 12.0, seed: int = 6) -> Problem:
    """The square128 grid (h = 1/128, 127^2 interior), order 2, implicit 10
    steps per period with multigrid to 1e-10, omega = 12 (adjusted), one
    period; k eigenpairs with a Krylov dimension of 2k + 1."""
    return Problem(n=(n, n), length=(1.0, 1.0), order=2, omega=omega, ts="implicit",
                   n_its=10, adjust_omega=True, mg_tol=1e-10, k=k, m=2 * k + 1, seed=seed)


def batch_problems(count: int = 96, seed: int = 4, n_lo: int = 65, n_hi: int = 1025,
                   len_lo: float = 0.5, len_hi: float = 2.0, om_lo: float = 10.0,
                   om_hi: float = 80.0) -> List[Problem]:
    """Batch of independent Dirichlet rectangles.  Per problem, four draws from
    stream ``seed`` in the order (a, b, n, omega): side lengths a, b uniform in
    [len_lo, len_hi], an n x n interior grid with n uniform over the integers
    [n_lo, n_hi], and omega uniform in [om_lo, om_hi].  Order 2, explicit
    leapfrog at CFL 0.5, mixed precision, 4 eigenpairs, Krylov dimension 16;
    the start-vector seed of problem i is 1000 + i."""
    u = uniform01(seed, 4 * count)
    out = []
    for i in range(count):
        a = len_lo + (len_hi - len_lo) * u[4 * i]
        b = len_lo + (len_hi - len_lo) * u[4 * i + 1]
        n = n_lo + min(int(math.floor(u[4 * i + 2] * (n_hi - n_lo + 1))), n_hi - n_lo)
        om = om_lo + (om_hi - om_lo) * u[4 * i + 3]
        out.append(Problem(n=(n, n), length=(float(a), float(b)), order=2, omega=float(om),
                           ts="explicit", cfl=0.5, precision="mixed", k=4, m=16,
                           seed=1000 + i))
    return out


def cnn_input_planes(seed: int, count: int) -> np.ndarray:
    """Uniform[-1,1] values for tiny network test inputs (brute-force checks)."""
    return uniform_pm1(seed, count)


# ---------------------------------------------------------------------------
# Mapped grids: coordinates x = G(r) of a single curvilinear grid, sampled at
# r_i = (i + 1) / (n_1 + 1), s_j = (j + 1) / (n_2 + 1) for i in [-2, n_1 + 1],
# j in [-2, n_2 + 1]: the active points are i in [0, n_1), the walls i = -1
# and i = n_1, plus one layer beyond each wall.  Returned as an array of shape
# (2, n_2 + 4, n_1 + 4): [0] holds x, [1] holds y, entry [., j + 2, i + 2].
# Pure geometry (the mapping evaluated at the parameter points); the
# discretisation lives in the oracle and in the library.
# ---------------------------------------------------------------------------
def _param_points(n: int) -> np.ndarray:
    return (np.arange(-2, n + 2, dtype=np.float64) + 1.0) / (n + 1)


def mapped_coords(kind: str, n1: int, n2: int, **p) -> np.ndarray:
    """Coordinates of one of the synthetic mappings of the unit square:

    * ``affine``: x = R(phi) (len1 r, len2 s) + shear * len2 s e_x (a
      rotated rectangle, or a parallelogram with ``shear`` != 0);
    * ``annulus``: sector of an annulus, radius a + (b - a) r, angle theta0 s;
    * ``skew``: the smooth non-orthogonal map x = len1 (r + eps r sin(pi s)),
      y = len2 (s + eps sin(pi r)).
    """
    r = _param_points(n1)[None, :]
    s = _param_points(n2)[:, None]
    if kind == "affine":
        l1, l2 = p.get("len1", 1.0), p.get("len2", 1.0)
        phi, shear = p.get("phi", 0.0), p.get("shear", 0.0)
        u = l1 * r + shear * l2 * s
        v = l2 * s + 0.0 * r
        x = math.cos(phi) * u - math.sin(phi) * v
        y = math.sin(phi) * u + math.cos(phi) * v
    elif kind == "annulus":
        a, b, th0 = p.get("a", 0.5), p.get("b", 1.0), p.get("theta0", 0.5 * math.pi)
        rho = a + (b - a) * r
        th = th0 * s
        x = rho * np.cos(th)
        y = rho * np.sin(th)
    elif kind == "skew":
        l1, l2, eps = p.get("len1", 1.0), p.get("len2", 1.0), p.get("eps", 0.15)
        x = l1 * (r + eps * r * np.sin(math.pi * s))
        y = l2 * (s + eps * np.sin(math.pi * r))
    else:
        raise ValueError(f"unknown mapping {kind!r}")
    out = np.empty((2, n2 + 4, n1 + 4))
    out[0] = np.broadcast_to(x, (n2 + 4, n1 + 4))
    out[1] = np.broadcast_to(y, (n2 + 4, n1 + 4))
    return out
