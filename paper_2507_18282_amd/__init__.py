"""MI355X-native WaveHoltz-filter eigensolver (EigenWave): Python binding.

Every step of the computation runs in the HIP library libeigenwave.so
(include/eigenwave.h); this module only marshals arguments.  PyTorch supplies
device memory (tensors) and the stream.  There is no CPU fallback: without the
built library, or without a GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

from . import _lib
from ._lib import EigenwaveError, check, load

__all__ = ["Operator", "Batch", "EigsResult", "Cnn", "CropStore", "fill_uniform", "choose_periods",
           "EigenwaveError", "load", "use_torch_allocator", "version"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t, n: int) -> int:
    torch = _torch()
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < n:
        raise ValueError("expected a contiguous float64 CUDA tensor with at least n_active elements")
    return int(t.data_ptr())


def version() -> str:
    return load().ew_version().decode()


@dataclass
class EigsResult:
    mu: list            # lambda_h^2 per returned pair, |beta| descending
    beta: list          # eigenvalues of S
    res: list           # ||L y + mu y|| / (mu ||y||)
    Y: object           # torch tensor (n_active, n_returned) on the device, or None
    n_conv: int
    wave_solves: int
    restarts: int
    probes: int
    time_steps: int
    pt_updates: int
    mg_cycles: int
    seconds: float
    status: int


def _set_walls(g, walls, dim: int) -> None:
    """walls: None (all Dirichlet) or one (lo, hi) pair per dimension of 'D'/'N'."""
    if walls is None:
        return
    if len(walls) != dim:
        raise ValueError("one (lo, hi) wall pair per dimension")
    code = {"D": _lib.WALL_DIRICHLET, "N": _lib.WALL_NEUMANN}
    for d, (lo, hi) in enumerate(walls):
        g.walls[d][0] = code[lo]
        g.walls[d][1] = code[hi]


class Operator:
    """The WaveHoltz operator S on one box (see ew_op_create); walls default to
    Dirichlet, ``walls=(("N", "D"), ("D", "D"))`` makes the low x wall Neumann.
    ``coords`` (an array of shape (2, n[1] + 4, n[0] + 4): x and y of the
    nodes i in [-2, n[0] + 1], j in [-2, n[1] + 1]) makes it an explicit
    operator on that curvilinear grid (see ew_op_create_mapped)."""

    def __init__(self, n: Sequence[int], length: Sequence[float], order: int, omega: float, ts: str,
                 cfl: float = 0.5, n_its: int = 10, n_p: int = 1, adjust_omega: bool = False,
                 filter_const: str = "alpha_d", precision: str = "fp64", mg_tol: float = 1e-10,
                 mg_nu1: int = 2, mg_nu2: int = 1, mg_max_cycles: int = 100, mg_coarse_sweeps: int = 8,
                 mg_coarse_points: int = 0, predictor: str = "zero", proj_window: int = 0,
                 mg_max_levels: int = 0, mg_relax: float = 0.0, mg_relax_coarse: float = 0.0, walls=None,
                 coords=None, stream=None):
        lib = load()
        self._lib = lib
        g = _lib.GridDesc()
        g.dim = len(n)
        for d in range(3):
            g.n[d] = int(n[d]) if d < len(n) else 1
            g.len[d] = float(length[d]) if d < len(n) else 1.0
        g.order = int(order)
        _set_walls(g, walls, len(n))
        d = _lib.OpDesc()
        d.omega = float(omega)
        d.ts = _lib.TS[ts]
        d.cfl = float(cfl)
        d.n_its = int(n_its)
        d.n_p = int(n_p)
        d.adjust_omega = int(bool(adjust_omega))
        d.filter_const = _lib.FILTER[filter_const]
        d.precision = _lib.PRECISION[precision]
        d.mg_tol = float(mg_tol)
        d.mg_nu1 = int(mg_nu1)
        d.mg_nu2 = int(mg_nu2)
        d.mg_max_cycles = int(mg_max_cycles)
        d.mg_coarse_sweeps = int(mg_coarse_sweeps)
        d.mg_coarse_points = int(mg_coarse_points)
        d.predictor = _lib.PREDICTOR[predictor]
        d.proj_window = int(proj_window)
        d.mg_max_levels = -1 if mg_max_levels == "auto" else int(mg_max_levels)
        d.mg_relax = float(mg_relax)
        d.mg_relax_coarse = float(mg_relax_coarse)
        self._stream = stream
        self._h = ctypes.c_void_p()
        if coords is None:
            check(lib.ew_op_create(ctypes.byref(g), ctypes.byref(d), ctypes.c_void_p(_stream_handle(stream)),
                                   ctypes.byref(self._h)))
        else:
            import numpy as np
            xy = np.ascontiguousarray(coords, dtype=np.float64)
            if len(n) != 2 or xy.shape != (2, int(n[1]) + 4, int(n[0]) + 4):
                raise ValueError("coords must have shape (2, n[1] + 4, n[0] + 4)")
            check(lib.ew_op_create_mapped(ctypes.byref(g), ctypes.byref(d),
                                          xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(self._h)))
        self.mapped = coords is not None
        self.n = tuple(int(x) for x in n)
        info = _lib.OpInfo()
        check(lib.ew_op_get_info(self._h, ctypes.byref(info)))
        self.n_active = int(info.n_active)
        self.n_t = int(info.n_t)
        self.dt = float(info.dt)
        self.omega_used = float(info.omega_used)
        self.t_final = float(info.t_final)
        self.alpha_d = float(info.alpha_d)
        self.mg_levels = int(info.mg_levels)
        self.mg_relax = float(info.mg_relax)
        self.mg_relax_coarse = float(info.mg_relax_coarse)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ew_op_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self):
        torch = _torch()
        return torch.empty(self.n_active, dtype=torch.float64, device="cuda")

    def mapped_rho(self) -> float:
        """Gershgorin bound on the spectrum of -L_h of a mapped operator."""
        r = ctypes.c_double()
        check(self._lib.ew_op_mapped_rho(self._h, ctypes.byref(r)))
        return float(r.value)

    def stats(self) -> dict:
        s = _lib.OpStats()
        check(self._lib.ew_op_get_stats(self._h, ctypes.byref(s)))
        return {f: (float(getattr(s, f)) if t is ctypes.c_double else int(getattr(s, f)))
                for f, t in _lib.OpStats._fields_}

    def probe_guesses(self, on: bool = True) -> None:
        """Measure the initial residuals of the guesses (see ew_op_probe_guesses)."""
        check(self._lib.ew_op_probe_guesses(self._h, int(bool(on))))

    def reset_stats(self) -> None:
        check(self._lib.ew_op_reset_stats(self._h))

    def profile_begin(self, kclass: str, level: int = -1) -> None:
        """Start timing every launch of one kernel class with hipEvents (see ew_op_profile_begin)."""
        check(self._lib.ew_op_profile_begin(self._h, _lib.KCLASS[kclass], int(level)))

    def profile_end(self) -> dict:
        p = _lib.KernelProfile()
        check(self._lib.ew_op_profile_end(self._h, ctypes.byref(p)))
        return {"launches": int(p.launches), "total_ms": float(p.total_ms), "bytes_alg": float(p.bytes_alg)}

    def apply_filter(self, v, out=None):
        out = self._new() if out is None else out
        check(self._lib.ew_op_apply_filter(self._h, _dev_ptr(v, self.n_active), _dev_ptr(out, self.n_active)))
        return out

    def apply_laplacian(self, v, out=None):
        out = self._new() if out is None else out
        check(self._lib.ew_op_apply_laplacian(self._h, _dev_ptr(v, self.n_active), _dev_ptr(out, self.n_active)))
        return out

    def mg_solve(self, b, x):
        cyc = ctypes.c_int()
        rel = ctypes.c_double()
        check(self._lib.ew_op_mg_solve(self._h, _dev_ptr(b, self.n_active), _dev_ptr(x, self.n_active),
                                       ctypes.byref(cyc), ctypes.byref(rel)))
        return x, int(cyc.value), float(rel.value)

    def mg_vcycle(self, b, x):
        check(self._lib.ew_op_mg_vcycle(self._h, _dev_ptr(b, self.n_active), _dev_ptr(x, self.n_active)))
        return x

    def mg_half_sweep(self, b, x, colour: int):
        check(self._lib.ew_op_mg_half_sweep(self._h, _dev_ptr(b, self.n_active), _dev_ptr(x, self.n_active),
                                            int(colour)))
        return x

    def set_cnn(self, cnn: Optional["Cnn"]) -> None:
        """Attach the network used by predictor="cnn" (kept alive by this object)."""
        check(self._lib.ew_op_set_cnn(self._h, cnn._h if cnn is not None else None))
        self._cnn = cnn

    def cnn_guess(self, b, base=None, out=None):
        """The learned guess for M x = b (see ew_op_cnn_guess); with `base` a
        tensor, it also receives the base guess."""
        out = self._new() if out is None else out
        check(self._lib.ew_op_cnn_guess(self._h, _dev_ptr(b, self.n_active),
                                        _dev_ptr(base, self.n_active) if base is not None else None,
                                        _dev_ptr(out, self.n_active)))
        return out

    def eigs(self, k: int, m: int, tol_ritz: float = 1e-12, tol_res: float = 1e-8,
             max_wave_solves: int = 100000, seed: int = 1, v0=None, n_keep: int = 0, max_probes: int = 16,
             k_cap: Optional[int] = None, want_vectors: bool = True, raise_on_error: bool = True) -> EigsResult:
        torch = _torch()
        d = _lib.EigsDesc()
        d.k, d.m = int(k), int(m)
        d.tol_ritz, d.tol_res = float(tol_ritz), float(tol_res)
        d.max_wave_solves = int(max_wave_solves)
        d.seed = int(seed)
        d.v0_dev = _dev_ptr(v0, self.n_active) if v0 is not None else None
        d.n_keep = int(n_keep)
        d.max_probes = int(max_probes)
        cap = int(k_cap) if k_cap is not None else 3 * m + k
        mu = (ctypes.c_double * cap)()
        beta = (ctypes.c_double * cap)()
        res = (ctypes.c_double * cap)()
        Y = torch.zeros((cap, self.n_active), dtype=torch.float64, device="cuda") if want_vectors else None
        st = _lib.EigsStats()
        status = self._lib.ew_eigs(self._h, ctypes.byref(d), cap, mu, beta, res,
                                   ctypes.c_void_p(int(Y.data_ptr())) if Y is not None else None,
                                   ctypes.byref(st))
        if status != _lib.EW_OK and raise_on_error:
            check(status)
        nret = int(st.n_returned)
        return EigsResult(mu=list(mu[:nret]), beta=list(beta[:nret]), res=list(res[:nret]),
                          Y=(Y[:nret].T if Y is not None else None), n_conv=int(st.n_conv),
                          wave_solves=int(st.wave_solves), restarts=int(st.restarts), probes=int(st.probes),
                          time_steps=int(st.time_steps), pt_updates=int(st.pt_updates),
                          mg_cycles=int(st.mg_cycles), seconds=float(st.seconds), status=int(status))


def _grid_desc(n, length, order):
    g = _lib.GridDesc()
    g.dim = len(n)
    for d in range(3):
        g.n[d] = int(n[d]) if d < len(n) else 1
        g.len[d] = float(length[d]) if d < len(n) else 1.0
    g.order = int(order)
    return g


def _op_desc(omega, ts, cfl=0.5, n_its=10, n_p=1, adjust_omega=False, filter_const="alpha_d", precision="fp64",
             mg_tol=1e-10, mg_nu1=2, mg_nu2=1, mg_max_cycles=100, mg_coarse_sweeps=8, mg_coarse_points=0,
             predictor="zero", proj_window=0, mg_max_levels=0, mg_relax=0.0, mg_relax_coarse=0.0):
    d = _lib.OpDesc()
    d.omega, d.ts, d.cfl, d.n_its, d.n_p = float(omega), _lib.TS[ts], float(cfl), int(n_its), int(n_p)
    d.adjust_omega, d.filter_const = int(bool(adjust_omega)), _lib.FILTER[filter_const]
    d.precision, d.mg_tol = _lib.PRECISION[precision], float(mg_tol)
    d.mg_nu1, d.mg_nu2, d.mg_max_cycles = int(mg_nu1), int(mg_nu2), int(mg_max_cycles)
    d.mg_coarse_sweeps, d.mg_coarse_points, d.predictor = int(mg_coarse_sweeps), int(mg_coarse_points), \
        _lib.PREDICTOR[predictor]
    d.proj_window = int(proj_window)
    d.mg_max_levels = int(mg_max_levels)
    d.mg_relax = float(mg_relax)
    d.mg_relax_coarse = float(mg_relax_coarse)
    return d


class Batch:
    """Many independent 2D explicit problems solved together (see ew_batch_create).

    ``problems`` is a list of dicts with keys n, length, order, omega and the
    optional operator keywords (cfl, n_p, filter_const, precision); every
    problem uses explicit stepping, with FP32 state (precision "mixed", the
    default) or FP64 state (precision "fp64", the same for all problems)."""

    def __init__(self, problems, stream=None):
        lib = load()
        self._lib = lib
        n = len(problems)
        G = (_lib.GridDesc * n)()
        D = (_lib.OpDesc * n)()
        for i, p in enumerate(problems):
            G[i] = _grid_desc(p["n"], p["length"], p["order"])
            kw = {k: v for k, v in p.items() if k not in ("n", "length", "order", "omega")}
            kw.setdefault("precision", "mixed")
            D[i] = _op_desc(p["omega"], "explicit", **kw)
        self._h = ctypes.c_void_p()
        check(lib.ew_batch_create(n, G, D, ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(self._h)))
        self.nprob = n
        self.n_active = []
        self.n_t = []
        for i in range(n):
            na, nt = ctypes.c_int64(), ctypes.c_int()
            check(lib.ew_batch_n_active(self._h, i, ctypes.byref(na), ctypes.byref(nt)))
            self.n_active.append(int(na.value))
            self.n_t.append(int(nt.value))
        info = _lib.BatchInfo()
        check(lib.ew_batch_get_info(self._h, ctypes.byref(info)))
        self.info = {"n_small": info.n_small, "n_large": info.n_large, "max_steps_large": info.max_steps_large,
                     "step_rows_per_thread": info.step_rows_per_thread, "tune_us": list(info.tune_us),
                     "total_steps": int(info.total_steps),
                     "pt_updates_per_wave_solve": int(info.pt_updates_per_wave_solve),
                     "state_fp64": bool(info.state_fp64), "steps_per_launch": info.steps_per_launch}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ew_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_filter(self, vs, outs=None):
        torch = _torch()
        if outs is None:
            outs = [torch.empty(n, dtype=torch.float64, device="cuda") for n in self.n_active]
        V = (ctypes.c_void_p * self.nprob)(*[_dev_ptr(v, n) for v, n in zip(vs, self.n_active)])
        O = (ctypes.c_void_p * self.nprob)(*[_dev_ptr(o, n) for o, n in zip(outs, self.n_active)])
        check(self._lib.ew_batch_apply_filter(self._h, V, O))
        return outs

    def eigs(self, k: int, m: int, tol_ritz: float = 1e-12, tol_res: float = 1e-8, max_wave_solves: int = 100000,
             seeds=None, n_keep: int = 0, max_probes: int = 16, k_cap: Optional[int] = None,
             want_vectors: bool = False, raise_on_error: bool = True):
        torch = _torch()
        n = self.nprob
        D = (_lib.EigsDesc * n)()
        for i in range(n):
            D[i].k, D[i].m = int(k), int(m)
            D[i].tol_ritz, D[i].tol_res = float(tol_ritz), float(tol_res)
            D[i].max_wave_solves = int(max_wave_solves)
            D[i].seed = int(seeds[i]) if seeds is not None else 1 + i
            D[i].v0_dev = None
            D[i].n_keep, D[i].max_probes = int(n_keep), int(max_probes)
        cap = int(k_cap) if k_cap is not None else 3 * m + k
        mu = (ctypes.c_double * (cap * n))()
        beta = (ctypes.c_double * (cap * n))()
        res = (ctypes.c_double * (cap * n))()
        nconv = (ctypes.c_int * n)()
        Ys = None
        Yp = None
        if want_vectors:
            Ys = [torch.zeros((cap, na), dtype=torch.float64, device="cuda") for na in self.n_active]
            Yp = (ctypes.c_void_p * n)(*[int(y.data_ptr()) for y in Ys])
        st = _lib.EigsStats()
        status = self._lib.ew_batch_eigs(self._h, D, cap, mu, beta, res, nconv, Yp, ctypes.byref(st))
        if status != _lib.EW_OK and raise_on_error:
            check(status)
        out = []
        for i in range(n):
            nc = int(nconv[i])
            # returned pairs: every pair Stage 2 produced, up to k_cap (converged or not)
            rows = [j for j in range(cap) if mu[i * cap + j] != 0.0]
            out.append({"mu": [mu[i * cap + j] for j in rows], "beta": [beta[i * cap + j] for j in rows],
                        "res": [res[i * cap + j] for j in rows], "n_conv": nc,
                        "Y": (Ys[i][:len(rows)].T if Ys is not None else None)})
        return out, {"wave_solves": int(st.wave_solves), "restarts": int(st.restarts), "probes": int(st.probes),
                     "pt_updates": int(st.pt_updates), "seconds": float(st.seconds), "n_conv": int(st.n_conv),
                     "max_res": float(st.max_res), "status": int(status)}


_alloc_hooks = None   # the ctypes callbacks must outlive their registration


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device buffers through PyTorch's caching allocator
    (``enable=False`` restores hipMalloc/hipFree).  Only while no operator,
    batch or network exists: the library refuses otherwise."""
    global _alloc_hooks
    torch = _torch()
    lib = load()
    if not enable:
        check(lib.ew_set_allocator(None, None, None))
        _alloc_hooks = None
        return

    def _alloc(nbytes, device, stream, _ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0)))
        except Exception:
            return None   # the library reports EW_ERR_OOM

    def _free(ptr, _ctx):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    hooks = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    check(lib.ew_set_allocator(ctypes.cast(hooks[0], ctypes.c_void_p), ctypes.cast(hooks[1], ctypes.c_void_p), None))
    _alloc_hooks = hooks


def fill_uniform(n: int, seed: int, stream=None):
    """SplitMix64 uniform[-1,1) vector of stream ``seed`` generated on the device."""
    torch = _torch()
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    check(load().ew_fill_uniform(ctypes.c_void_p(int(x.data_ptr())), int(n), int(seed),
                                 ctypes.c_void_p(_stream_handle(stream))))
    return x


def _f32_ptr(t, n: int) -> int:
    torch = _torch()
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or t.numel() < n:
        raise ValueError("expected a contiguous float32 CUDA tensor with at least %d elements" % n)
    return int(t.data_ptr())


class Cnn:
    """The learned warm-start network (see ew_cnn_create)."""

    n_params = _lib.CNN_PARAMS

    def __init__(self, seed: int = 0, stream=None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        check(self._lib.ew_cnn_create(int(seed), ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(self._h)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ew_cnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        buf = (ctypes.c_float * self.n_params)()
        check(self._lib.ew_cnn_get_params(self._h, buf))
        return np.frombuffer(buf, dtype=np.float32).copy()

    def set_params(self, params) -> None:
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError("expected %d parameters" % self.n_params)
        check(self._lib.ew_cnn_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def forward(self, store: "CropStore", first: int, count: int, out=None):
        torch = _torch()
        n = count * store.crop * store.crop
        out = torch.empty(n, dtype=torch.float32, device="cuda") if out is None else out
        check(self._lib.ew_cnn_forward(self._h, store._h, int(first), int(count), _f32_ptr(out, n)))
        return out.view(count, store.crop, store.crop)

    def loss_grad(self, store: "CropStore", first: int, count: int):
        torch = _torch()
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = ctypes.c_double()
        check(self._lib.ew_cnn_loss_grad(self._h, store._h, int(first), int(count), ctypes.byref(loss),
                                         _f32_ptr(g, self.n_params)))
        return float(loss.value), g

    def train(self, store: "CropStore", steps: int, batch: int, lr: float = 1e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, seed: int = 0) -> dict:
        d = _lib.CnnTrainDesc(int(steps), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(seed))
        st = _lib.CnnTrainStats()
        check(self._lib.ew_cnn_train(self._h, store._h, ctypes.byref(d), ctypes.byref(st)))
        return {"steps": int(st.steps), "first_loss": float(st.first_loss), "last_loss": float(st.last_loss),
                "seconds": float(st.seconds)}


class CropStore:
    """Training crops for the network (see ew_cnn_data_create)."""

    def __init__(self, capacity: int, crop: int = 128, order: int = 4):
        self._lib = load()
        self._h = ctypes.c_void_p()
        check(self._lib.ew_cnn_data_create(int(capacity), int(crop), int(order), ctypes.byref(self._h)))
        self.capacity = int(capacity)
        self.crop = int(crop)
        self.order = int(order)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ew_cnn_data_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def count(self) -> int:
        c = ctypes.c_int()
        check(self._lib.ew_cnn_data_count(self._h, ctypes.byref(c)))
        return int(c.value)

    def append(self, fields, target, planes, rects) -> None:
        import numpy as np
        n = len(planes)
        cp = self.crop + 2 * _lib.CNN_HALO
        pl = np.ascontiguousarray(planes, dtype=np.float32).reshape(n, 4)
        rc = np.ascontiguousarray(rects, dtype=np.int32).reshape(n, 4)
        check(self._lib.ew_cnn_data_append(self._h, n, _f32_ptr(fields, n * 2 * cp * cp),
                                           _f32_ptr(target, n * self.crop * self.crop),
                                           pl.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                           rc.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))

    def read(self, first: int, count: int):
        """(fields, target, planes, rects) of crops first..first+count-1; tensors on the device."""
        import numpy as np
        torch = _torch()
        cp = self.crop + 2 * _lib.CNN_HALO
        fields = torch.empty((count, 2, cp, cp), dtype=torch.float32, device="cuda")
        target = torch.empty((count, self.crop, self.crop), dtype=torch.float32, device="cuda")
        planes = np.zeros((count, 4), dtype=np.float32)
        rects = np.zeros((count, 4), dtype=np.int32)
        check(self._lib.ew_cnn_data_read(self._h, int(first), int(count), int(fields.data_ptr()),
                                         int(target.data_ptr()), planes.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         rects.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return fields, target, planes, rects

    def collect(self, op: Operator, v, out=None, crops_per_step: int = 4, seed: int = 0):
        """out = S v by op (implicit FP64 2D) while recording crops at every step."""
        out = op._new() if out is None else out
        check(self._lib.ew_cnn_data_collect(self._h, op._h, _dev_ptr(v, op.n_active), _dev_ptr(out, op.n_active),
                                            int(crops_per_step), int(seed)))
        return out


def choose_periods(length: Sequence[float], omega: float, k: int, ts: str = "implicit", n_its: int = 10,
                   adjust_omega: bool = True, beta_r: float = 0.8, np_max: int = 256):
    """(N_p, eigenvalues in the lobe) for k wanted eigenpairs (see ew_choose_periods)."""
    lib = load()
    g = _grid_desc([1] * len(length), length, 2)
    d = _op_desc(omega, ts, n_its=n_its, adjust_omega=adjust_omega)
    n_p, n_lobe = ctypes.c_int(), ctypes.c_int()
    check(lib.ew_choose_periods(ctypes.byref(g), ctypes.byref(d), int(k), float(beta_r), int(np_max),
                                ctypes.byref(n_p), ctypes.byref(n_lobe)))
    return int(n_p.value), int(n_lobe.value)


def sym_eig(a):
    """(w, Q) with a = Q diag(w) Q^T for a symmetric float64 matrix (host
    routine of the eigensolver's projected problems; see ew_sym_eig)."""
    import numpy as np
    lib = load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix expected")
    w = np.empty(n)
    q = np.empty((n, n))
    check(lib.ew_sym_eig(int(n), a.ctypes.data, w.ctypes.data, q.ctypes.data))
    return w, q
