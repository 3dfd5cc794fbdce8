"""Benchmark of the WaveHoltz-filter eigensolver on one MI355X.

A step is one Arnoldi step of the eigensolver on the headline workload: one
wave-solve (S v: 10 implicit steps over one period, each solved by FP64
multigrid V(2,1) cycles to relative residual 1e-10, filter accumulated in the
same loop) plus the modified Gram-Schmidt orthogonalisation against the basis,
with the Krylov-Schur restarts that fall inside the timed steps.

Headline workload: unit square, 2049 x 2049 grid points (2047^2 interior
unknowns, h = 1/2048), 4th-order Laplacian, implicit stepping with 10 steps
per period, omega = 120 (adjusted to 109.7306), Krylov dimension 32 for 16
eigenpairs, SplitMix64 start vector (seed 2).  Inputs are synthetic and
resident in HBM before the timed region starts.

value = grid-point updates per second (active points x time steps advanced)
over the K timed steps.  Eigenpairs per second at residual <= 1e-8 are
measured on complete solves of the headline eigenproblem (with the number of
filter periods from the lobe rule; about 1000 eigenvalues lie in the main lobe
at one period) and of the 64^2 explicit workload, and reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LEARN_CHAINS = 40          # wave-solve chains that generate training crops
LEARN_CROPS_PER_STEP = 19  # 40 chains x 3 wave-solves x 9 steps x 19 crops = 20520 crops
LEARN_STEPS = 3000         # Adam steps per phase (one phase at 2e-3, one at 5e-4)
LEARN_BATCH = 32
LEARN_OMEGA_SEED = 4242
LEARN_CROP_SEED = 777
LEARN_BUDGET = 32          # wave-solves per predictor in the one-period comparisons
LEARN_OMEGAS = (40.0, 90.0, 140.0)
LEARN_COMPLETE_OMEGA = 90.0  # complete eigensolves (N_p from the lobe rule) for every predictor
CUBE_N = 63                # side of the mixed-vs-FP64 cube eigensolve (--cube-n: 127, 255)
MIXED_TOL_RITZ = 1e-7      # Ritz tolerance above the FP32 accumulation noise of S v
CUBE_BUDGET = 400          # wave-solves per precision in the cube eigensolves
PERIODS_BUDGET_NP1 = 400   # wave-solves allowed to N_p = 1 in the periods-rule comparison
METRIC = "grid-pt updates/s + eigenpairs/s at resid 1e-8; learned/batched vs plain"
SMOOTH_SRC = os.path.join(ROOT, "paper_2507_18282_amd", "csrc", "sweep2d.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_smooth_square2047_order4.txt")


# Multigrid depth of the implicit workloads: the library's automatic rule
# (EW_MG_LEVELS_AUTO) ends the hierarchy on the first level that
# MG_COARSE_SWEEPS red-black sweeps contract by 0.1 (on 2047^2 at omega 120 that
# is 127^2, on 1023^2 at omega 90 it is 63^2); coarser levels only add
# latency-bound launches there.
MG_LEVELS = -1
MG_COARSE_SWEEPS = 4
# line over-relaxation weights (finest, coarser levels) for the skew map: the
# fewest cycles in a CPU model of the same multigrid on a 511^2 skew map with
# the same a / h^2 (9 cycles against 12 with weight 1); an annulus sector
# wants weight 1, the mapped default
MAPPED_SLOR = (1.3, 1.2)
# The 2047^2 headline (and its complete eigensolve) stops on 127^2 as above but
# relaxes that level with a single sweep: the V-cycles per solve stay at 8.99
# and the step takes 14.1 ms instead of 14.8 ms (4 sweeps; measured in an
# Arnoldi sequence).  One sweep is not better everywhere (the 127^2
# many-pairs workload needs 9.9 cycles with it against 7.2), so the other
# workloads keep the rule above.
HEADLINE_MG_LEVELS = 5
HEADLINE_COARSE_SWEEPS = 1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the smoother from the committed rocprofv3 counter
    summary, or None when the counters were taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != source_digest(SMOOTH_SRC):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """Logical CPUs and model name of the host the bench runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(P, n_solves: int):
    """The oracle, as it stands, on a bounded sample: n_solves wave-solves of the
    headline grid (exact sine-transform implicit solves, numpy and scipy.fft),
    once on one core and once with scipy.fft's transforms on every host core
    (scipy.fft.set_workers); the faster is `value`."""
    import numpy as np
    import scipy.fft
    import synthetic
    from oracle import discrete as D
    from oracle import wave as W
    h = D.spacing(P.n, P.length)
    plan = D.time_plan(h, P.order, P.omega, P.ts, n_its=P.n_its, n_p=P.n_p, adjust_omega=P.adjust_omega)
    ncpu, model = host_cpu()
    runs = {}
    for cores in (1, ncpu):
        v = synthetic.start_vector(P.seed, P.n_active).reshape(P.n[::-1])
        t0 = time.perf_counter()
        with scipy.fft.set_workers(cores):
            for _ in range(n_solves):
                v = W.apply_filter(v, h, P.order, plan)
                v = v / np.linalg.norm(v)
        runs[cores] = time.perf_counter() - t0
        log(f"cpu baseline: {n_solves} wave-solves on {cores} cores in {runs[cores]:.1f} s")
    best = min(runs, key=runs.get)
    rate = {c: P.n_active * plan.n_t * n_solves / t for c, t in runs.items()}
    return {"value": rate[best], "unit": "grid-pt updates/s", "cores": best, "kind": "oracle",
            "sample": f"{n_solves} wave-solves of the 2047^2 order-4 implicit grid ({plan.n_t} steps each, "
                      f"exact DST solves instead of multigrid), {runs[best]:.1f} s",
            "host": {"logical_cpus": ncpu, "model": model},
            "per_cores": {str(c): {"value": rate[c], "seconds": runs[c]} for c in runs}}

def vcycle_roofline(op, n_cycles: int = 20):
    """Time whole V-cycles of the headline operator (ew_op_mg_vcycle, the
    kernels of the solves, without convergence tests) and each finest-level
    pass, against the algorithmic bytes of a V(2,1) cycle: 144 B per
    finest-level point (13.5 FP64 arrays: 3 per red-black sweep, 2.25 for the
    residual and restriction, 2.25 for the prolongation and correction, times
    4/3 for the coarser levels)."""
    import torch
    from paper_2507_18282_amd import fill_uniform
    n = op.n_active
    b = fill_uniform(n, 71)
    x = fill_uniform(n, 72)
    op.mg_vcycle(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_cycles):
        op.mg_vcycle(b, x)
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) / n_cycles * 1e6
    bytes_cycle = 144.0 * n
    out = {"us_per_cycle": round(us, 2), "bytes_alg_per_cycle": bytes_cycle,
           "achieved_GBs": round(bytes_cycle / (us * 1e-6) / 1e9, 1), "peak_GBs": HBM_PEAK_GBS,
           "frac": round(bytes_cycle / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), "finest_level": {}}
    for cls, what in (("smooth", "two pre-smoothing sweeps in one pass"),
                      ("prolong", "prolongation + post-smoothing sweep"),
                      ("restrict", "residual + full-weighting restriction")):
        op.profile_begin(cls, level=0)
        for _ in range(n_cycles):
            op.mg_vcycle(b, x)
        torch.cuda.synchronize()
        p = op.profile_end()
        if p["launches"]:
            avg = p["total_ms"] / p["launches"] * 1e3
            gbs = p["bytes_alg"] / p["launches"] / (avg * 1e-6) / 1e9
            out["finest_level"][cls] = {"kernel": what, "avg_us": round(avg, 2), "alg_GBs": round(gbs, 1),
                                        "frac": round(gbs / HBM_PEAK_GBS, 4),
                                        "share_of_cycle": round(avg / us, 3)}
    log(f"V-cycle: {us:.1f} us, {out['achieved_GBs']:.0f} GB/s algorithmic ({out['frac']:.2f} of peak)")
    return out


def _batch_run(Ps, precision: str, tol_ritz: float, tol_res: float, budget: int):
    """One batched eigensolve of every problem against the same problems solved
    one after the other, same budget of wave-solves per problem; pairs counted
    at eig-res <= tol_res."""
    import torch
    from paper_2507_18282_amd import Batch, Operator
    bt = Batch([{"n": P.n, "length": P.length, "order": 2, "omega": P.omega, "cfl": 0.5, "precision": precision}
                for P in Ps])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, st = bt.eigs(k=4, m=16, seeds=[P.seed for P in Ps], tol_ritz=tol_ritz, tol_res=tol_res,
                      max_wave_solves=budget, raise_on_error=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    nb = sum(sum(1 for x in r["res"] if x <= tol_res) for r in res)
    info = bt.info
    bt.close()
    log(f"batched {precision}: {nb} pairs at eig-res <= {tol_res:g} in {tb:.2f} s")
    t0 = time.perf_counter()
    npl, wsp, ptp = 0, 0, 0
    for P in Ps:
        op = Operator(n=P.n, length=P.length, order=2, omega=P.omega, ts="explicit", cfl=0.5, precision=precision)
        r = op.eigs(4, 16, seed=P.seed, tol_ritz=tol_ritz, tol_res=tol_res, max_wave_solves=budget,
                    want_vectors=False, raise_on_error=False)
        npl += sum(1 for x in r.res if x <= tol_res)
        wsp += r.wave_solves
        ptp += r.pt_updates
        op.close()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    log(f"plain {precision}: {npl} pairs at eig-res <= {tol_res:g} in {tp:.2f} s")
    return {"state": "FP64" if precision == "fp64" else "FP32", "tol_ritz": tol_ritz, "eig_res_tol": tol_res,
            "batched": {"eigenpairs_per_s": nb / tb, "pairs": nb, "seconds": tb, "wave_solves": st["wave_solves"],
                        "pt_updates_per_s": st["pt_updates"] / tb, "small_problems": info["n_small"],
                        "step_rows_per_thread": info["step_rows_per_thread"], "tune_us": info["tune_us"],
                        "steps_per_launch": info["steps_per_launch"]},
            "plain": {"eigenpairs_per_s": npl / tp, "pairs": npl, "seconds": tp, "wave_solves": wsp,
                      "pt_updates_per_s": ptp / tp},
            "speedup_eigenpairs_per_s": (nb / tb) / (npl / tp) if npl > 0 else None}


def batched_vs_plain(budget: int):
    """96 independent rectangles (sides U[0.5,2], n^2 grids with n U[65,1025],
    omega U[10,80], order 2, explicit CFL 0.5, FP64 Arnoldi, k = 4, m = 16).
    With FP64 state at eig-res <= 1e-8; with FP32 state at eig-res <= 5e-3,
    above the floor that the FP32 time levels leave in the residual (rounding
    of about 2^-24 N_t in every mode of S v, which L_h amplifies by up to
    lambda_max / mu, some 1e4 on the finest grids here)."""
    import synthetic
    Ps = synthetic.batch_problems()
    return {"workload": "96 Dirichlet rectangles, sides U[0.5,2], n^2 grids n U[65,1025], omega U[10,80], order 2, "
                        "explicit CFL 0.5, FP64 Arnoldi, k=4, m=16",
            "budget_wave_solves_per_problem": budget,
            "fp64_state": _batch_run(Ps, "fp64", 1e-12, 1e-8, budget),
            "fp32_state": _batch_run(Ps, "mixed", MIXED_TOL_RITZ, 5e-3, budget)}


def learned_vs_plain():
    """1023^2 unit square, order 4, implicit 10 steps/period, FP64 multigrid to
    1e-10, k = 16, m = 32.  Training: 20520 crops of 128^2 (40 chains of 3
    wave-solves from SplitMix64 starts 5000.., omega U[30, 150], projection
    guesses; 19 crops per step) at the projection guess's residual, Adam on the
    residual loss.  Then: complete eigensolves at omega 90 with N_p from the
    lobe rule for the zero, projection and learned guesses (multigrid always to
    the same tolerance, so the eigenpairs agree), eigenpairs/s at eig-res <=
    1e-8; the initial residuals of the guesses measured inside the solves; and
    one-period runs of LEARN_BUDGET wave-solves at omega 40, 90, 140."""
    import torch
    import synthetic
    from paper_2507_18282_amd import Cnn, CropStore, Operator, choose_periods, fill_uniform
    P = synthetic.config_learned()
    n = P.n[0]

    def make(omega, predictor, n_p=1):
        return Operator(n=P.n, length=P.length, order=P.order, omega=omega, ts=P.ts, n_its=P.n_its, n_p=n_p,
                        adjust_omega=P.adjust_omega, mg_tol=P.mg_tol, predictor=predictor,
                        mg_max_levels=MG_LEVELS, mg_coarse_sweeps=MG_COARSE_SWEEPS)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    store = CropStore(LEARN_CHAINS * 3 * 9 * LEARN_CROPS_PER_STEP, 128, P.order)
    u = synthetic.uniform01(LEARN_OMEGA_SEED, LEARN_CHAINS)
    for c in range(LEARN_CHAINS):
        op = make(30.0 + 120.0 * u[c], "proj")
        v = fill_uniform(op.n_active, 5000 + c)
        for _ in range(3):
            w = store.collect(op, v, crops_per_step=LEARN_CROPS_PER_STEP, seed=LEARN_CROP_SEED)
            v = w / w.norm()
        op.close()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = Cnn(1)
    tr1 = net.train(store, steps=LEARN_STEPS, batch=LEARN_BATCH, lr=2e-3, seed=11)
    tr2 = net.train(store, steps=LEARN_STEPS, batch=LEARN_BATCH, lr=5e-4, seed=12)
    log(f"learned: {store.count} crops in {t_data:.2f} s, training {tr1['seconds'] + tr2['seconds']:.2f} s, "
        f"loss {tr1['first_loss']:.4g} -> {tr2['last_loss']:.4g}")
    out = {"workload": "unit square 1025^2 points (1023^2 interior), order 4, implicit 10 steps/period, FP64 "
                       "multigrid to 1e-10 (automatic depth, 4 sweeps on the coarsest level), k=16, m=32",
           "data": {"crops": store.count, "crop": 128, "seconds": t_data, "base_guess": "projection"},
           "training": {"steps": 2 * LEARN_STEPS, "batch": LEARN_BATCH, "seconds": tr1["seconds"] + tr2["seconds"],
                        "first_loss": tr1["first_loss"], "last_loss": tr2["last_loss"],
                        "loss": "mean over window points of (r/s - M y)^2; 1.0 = the base guess's residual"}}
    preds = ("zero", "proj", "cnn")
    # complete eigensolves at the rule's N_p
    omega = LEARN_COMPLETE_OMEGA
    n_p, n_lobe = choose_periods(P.length, omega, P.k)
    comp = {"omega": omega, "n_p": n_p, "eigenvalues_in_lobe": n_lobe}
    for pred in preds:
        op = make(omega, pred, n_p)
        if pred == "cnn":
            op.set_cnn(net)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = op.eigs(P.k, P.m, seed=P.seed, tol_res=1e-8, want_vectors=False, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ok = sum(1 for x in r.res if x <= 1e-8)
        comp[pred] = {"pairs": ok, "wave_solves": r.wave_solves, "seconds": dt, "eigenpairs_per_s": ok / dt,
                      "ms_per_wave_solve": dt / max(1, r.wave_solves) * 1e3,
                      "mg_cycles_per_implicit_solve": r.mg_cycles / max(1, r.time_steps),
                      "max_res": max(r.res) if r.res else None, "status": r.status, "mu": list(r.mu)}
        log(f"learned form complete omega {omega} N_p {n_p} {pred}: {ok} pairs, {r.wave_solves} wave-solves, "
            f"{dt:.1f} s, {comp[pred]['mg_cycles_per_implicit_solve']:.2f} cycles/solve")
        op.close()
    for pred in preds[1:]:
        c = comp[pred]
        c["speedup_eigenpairs_per_s_vs_zero"] = c["eigenpairs_per_s"] / comp["zero"]["eigenpairs_per_s"] \
            if comp["zero"]["eigenpairs_per_s"] else None
        c["vcycles_saved_per_implicit_solve"] = comp["zero"]["mg_cycles_per_implicit_solve"] - \
            c["mg_cycles_per_implicit_solve"]
        if comp["zero"]["mu"] and c["mu"]:
            # each returned eigenvalue against the nearest one of the cold start (the
            # two solves may return a different number of extra pairs)
            c["max_mu_rel_diff_vs_zero"] = max(min(abs(a - b) / b for b in comp["zero"]["mu"]) for a in c["mu"])
    comp["cnn"]["speedup_eigenpairs_per_s_vs_proj"] = comp["cnn"]["eigenpairs_per_s"] / \
        comp["proj"]["eigenpairs_per_s"] if comp["proj"]["eigenpairs_per_s"] else None
    out["complete_solves"] = comp
    # one-period runs: wave-solve cost and cycles, and the guesses' initial residuals (separate probed runs)
    for omega in LEARN_OMEGAS:
        res = {}
        for pred in preds:
            op = make(omega, pred)
            if pred == "cnn":
                op.set_cnn(net)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = op.eigs(P.k, P.m, seed=P.seed, tol_res=1e-8, max_wave_solves=LEARN_BUDGET, want_vectors=False,
                        raise_on_error=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            res[pred] = {"ms_per_wave_solve": dt / r.wave_solves * 1e3, "wave_solves": r.wave_solves,
                         "mg_cycles_per_implicit_solve": r.mg_cycles / max(1, r.time_steps)}
            if pred != "zero":
                op.reset_stats()
                op.probe_guesses(True)
                w = fill_uniform(op.n_active, 99)
                for _ in range(2):
                    w = op.apply_filter(w / w.norm())
                st = op.stats()
                res[pred]["guess_rel_res"] = st["guess_rel_res_sum"] / max(1, st["guess_probes"])
                res[pred]["base_rel_res"] = st["base_rel_res_sum"] / max(1, st["guess_probes"])
            log(f"learned form omega {omega} {pred}: {r.wave_solves} wave-solves in {dt:.2f} s, "
                f"{res[pred]['mg_cycles_per_implicit_solve']:.2f} cycles/solve"
                + (f", initial residual {res[pred]['guess_rel_res']:.3g} (base {res[pred]['base_rel_res']:.3g})"
                   if pred != "zero" else ""))
            op.close()
        z = res["zero"]
        for pred in preds[1:]:
            o = res[pred]
            o["vcycles_saved_per_implicit_solve"] = z["mg_cycles_per_implicit_solve"] - o["mg_cycles_per_implicit_solve"]
            o["speedup_wave_solve_vs_zero"] = z["ms_per_wave_solve"] / o["ms_per_wave_solve"]
        out[f"one_period_omega_{omega:g}"] = res
    return out

def periods_rule():
    """255^2 unit square, order 4, implicit 10 steps/period, omega 40 (adjusted),
    FP64 multigrid to 1e-10, k = 8, m = 17: complete eigensolves with the number
    of filter periods from the lobe rule (ew_choose_periods) against N_p = 1,
    which on this dense spectrum (about 70 eigenvalues with beta >= 0.8) does not
    converge within PERIODS_BUDGET_NP1 wave-solves."""
    import torch
    from paper_2507_18282_amd import Operator, choose_periods
    n, omega, k = 255, 40.0, 8
    n_p, n_lobe = choose_periods((1.0, 1.0), omega, k)
    out = {"workload": "unit square 257^2 points (255^2 interior), order 4, implicit 10 steps/period, omega 40 "
                       "(adjusted), FP64 multigrid to 1e-10 (automatic depth), k=8, m=17, eig-res <= 1e-8",
           "rule": {"n_p": n_p, "eigenvalues_in_lobe": n_lobe}}
    for label, npp, budget in (("np1", 1, PERIODS_BUDGET_NP1), ("rule", n_p, 100000)):
        op = Operator(n=(n, n), length=(1.0, 1.0), order=4, omega=omega, ts="implicit", n_its=10, n_p=npp,
                      adjust_omega=True, mg_tol=1e-10, mg_max_levels=MG_LEVELS, mg_coarse_sweeps=MG_COARSE_SWEEPS)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.eigs(k, 2 * k + 1, seed=3, tol_res=1e-8, max_wave_solves=budget, want_vectors=False,
                    raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(1 for x in r.res if x <= 1e-8)
        res = out.setdefault(label, {})
        res.update({"n_p": npp, "pairs": ok, "wave_solves": r.wave_solves, "seconds": dt,
                    "eigenpairs_per_s": ok / dt, "time_steps_per_eigenpair": r.time_steps / ok if ok else None,
                    "status": r.status})
        log(f"periods rule: N_p {npp}: {ok} pairs, {r.wave_solves} wave-solves, {dt:.2f} s")
        op.close()
    return out


# Requested-eigenpairs table of the paper (Sec. "Changing the number of
# requested eigenpairs"; square128, omega 12, N_a = 2 N_r + 1): requested ->
# (converged, wave-solves), measured on CPUs with SLEPc.
MANY_PAIRS_PAPER = {16: (16, 64), 64: (65, 209), 256: (285, 675), 512: (571, 1325)}


def walls_form():
    """Neumann walls beside Dirichlet ones on the same work: the headline grid
    with a symmetry plane (2047 x 2048 points, Neumann wall at y = 0, order 4,
    implicit, omega 120, automatic multigrid depth) against the all-Dirichlet
    2047^2, two wave-solves each; and the small explicit eigensolve on a 64 x
    65 square with a Neumann wall at y = 0 against the Dirichlet 64^2 one."""
    import torch
    import synthetic
    from paper_2507_18282_amd import Operator, fill_uniform
    out = {"workload": "implicit: 2047 x 2048 (Neumann y=0) vs 2047^2 (Dirichlet), order 4, omega 120 (adjusted), "
                       "multigrid to 1e-10, 2 wave-solves; explicit: 64 x 65 (Neumann y=0) vs 64^2, order 2, "
                       "CFL 0.5, omega 15, k=4, m=16, eig-res <= 1e-8"}
    P = synthetic.config_square_order4_implicit()
    for label, n, walls in (("implicit_dirichlet", (2047, 2047), None),
                            ("implicit_neumann_y0", (2047, 2048), (("D", "D"), ("N", "D")))):
        op = Operator(n=n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its,
                      adjust_omega=P.adjust_omega, mg_tol=P.mg_tol, mg_max_levels=MG_LEVELS,
                      mg_coarse_sweeps=MG_COARSE_SWEEPS, walls=walls)
        v = fill_uniform(op.n_active, 3)
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        op.reset_stats()
        t0 = time.perf_counter()
        w = op.apply_filter(v)
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = op.stats()
        out[label] = {"pt_updates_per_s": st["pt_updates"] / dt, "ms_per_wave_solve": dt / 2 * 1e3,
                      "mg_levels": op.mg_levels, "mg_cycles_per_implicit_solve": st["mg_cycles"] / max(1, st["mg_solves"])}
        log(f"walls form: {label}: {dt / 2 * 1e3:.1f} ms per wave-solve, {op.mg_levels} levels")
        op.close()
    for label, n, walls in (("explicit_dirichlet", (64, 64), None),
                            ("explicit_neumann_y0", (64, 65), (("D", "D"), ("N", "D")))):
        op = Operator(n=n, length=(1.0, 1.0), order=2, omega=15.0, ts="explicit", cfl=0.5, walls=walls)
        r = op.eigs(4, 16, seed=1, want_vectors=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.eigs(4, 16, seed=1, want_vectors=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(1 for x in r.res if x <= 1e-8)
        out[label] = {"pairs": ok, "wave_solves": r.wave_solves, "seconds": dt, "eigenpairs_per_s": ok / dt,
                      "max_res": max(r.res)}
        log(f"walls form: {label}: {ok} pairs, {r.wave_solves} wave-solves, {dt * 1e3:.1f} ms")
        op.close()
    return out


def mapped_form():
    """A single curvilinear grid beside the box: one explicit wave-solve on a
    2047^2 grid mapped by the smooth non-orthogonal skew map (order 2,
    omega 60, CFL 0.9) against the 2047^2 unit square with the same settings,
    the leapfrog kernels timed with hipEvents (8 steps per launch on both;
    one step as one launch would stream it moves 40 B per point on the box
    and 72 B on the mapped grid, the state plus four coefficient arrays);
    and an eigensolve on a 255^2
    quarter annulus (radii 0.5 to 1, omega 40, k = 8, m = 20)."""
    import torch
    import synthetic
    from paper_2507_18282_amd import Operator, fill_uniform
    out = {"workload": "explicit order 2, omega 60, CFL 0.9: 2047^2 skew-mapped grid (eps 0.15) vs 2047^2 unit "
                       "square, 2 wave-solves each; eigensolve: 255^2 quarter annulus (radii 0.5..1), omega 40, "
                       "CFL 0.5, k=8, m=20, eig-res <= 1e-8"}
    n = (2047, 2047)
    xy = synthetic.mapped_coords("skew", *n, eps=0.15)
    for label, coords in (("box", None), ("mapped", xy)):
        op = Operator(n=n, length=(1.0, 1.0), order=2, omega=60.0, ts="explicit", cfl=0.9, coords=coords)
        v = fill_uniform(op.n_active, 3)
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        op.reset_stats()
        t0 = time.perf_counter()
        w = op.apply_filter(v)
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = op.stats()
        # kernel timing in a separate wave-solve: the events would add gaps to the timed ones
        op.profile_begin("leapfrog")
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        prof = op.profile_end()
        avg = prof["total_ms"] / max(1, prof["launches"])
        gbs = prof["bytes_alg"] / max(1, prof["launches"]) / (avg * 1e-3) / 1e9
        # several steps per launch: the bytes one launch per step would move
        # (40 B per point-step on the box, 72 B on the mapped grid) over the
        # time per step can exceed what HBM streams, since the blocked kernels
        # read each point once per launch
        out[label] = {"n_t": op.n_t, "pt_updates_per_s": st["pt_updates"] / dt, "ms_per_wave_solve": dt / 2 * 1e3,
                      "steps_per_launch": round(op.n_t / max(1, prof["launches"]), 2),
                      "launch_avg_us": round(avg * 1e3, 3),
                      "us_per_step": round(prof["total_ms"] * 1e3 / op.n_t, 3),
                      "per_step_form_GBs": round(gbs, 1)}
        log(f"mapped form: {label}: n_t {op.n_t}, {dt / 2 * 1e3:.1f} ms per wave-solve, {prof['launches']} launches "
            f"of {avg * 1e3:.1f} us")
        op.close()
    # implicit (10 steps per period, adjusted omega, multigrid to 1e-10, automatic depth)
    out["implicit_workload"] = ("implicit order 2, omega 60 (adjusted), 10 steps, multigrid V(2,1) to 1e-10 "
                                "(automatic depth, 4 sweeps on the coarsest level): 2047^2 skew map vs unit square, "
                                "2 wave-solves each; the skew map with the default line weights 1 and with line "
                                "over-relaxation (1.3 on the finest level, 1.2 below)")
    for label, coords, relax in (("implicit_box", None, (0.0, 0.0)), ("implicit_mapped", xy, (0.0, 0.0)),
                                 ("implicit_mapped_slor", xy, MAPPED_SLOR)):
        op = Operator(n=n, length=(1.0, 1.0), order=2, omega=60.0, ts="implicit", n_its=10, adjust_omega=True,
                      mg_tol=1e-10, mg_max_levels=MG_LEVELS, mg_coarse_sweeps=MG_COARSE_SWEEPS, coords=coords,
                      mg_relax=relax[0], mg_relax_coarse=relax[1])
        v = fill_uniform(op.n_active, 3)
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        op.reset_stats()
        t0 = time.perf_counter()
        w = op.apply_filter(v)
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = op.stats()
        out[label] = {"pt_updates_per_s": st["pt_updates"] / dt, "ms_per_wave_solve": dt / 2 * 1e3,
                      "mg_levels": op.mg_levels,
                      "mg_cycles_per_implicit_solve": st["mg_cycles"] / max(1, st["mg_solves"])}
        log(f"mapped form: {label}: {dt / 2 * 1e3:.1f} ms per wave-solve, {op.mg_levels} levels, "
            f"{st['mg_cycles'] / max(1, st['mg_solves']):.1f} cycles per solve")
        op.close()
    na = (255, 255)
    xa = synthetic.mapped_coords("annulus", *na, a=0.5, b=1.0, theta0=0.5 * math.pi)
    op = Operator(n=na, length=(1.0, 1.0), order=2, omega=40.0, ts="explicit", cfl=0.5, coords=xa)
    r = op.eigs(8, 20, seed=2, want_vectors=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = op.eigs(8, 20, seed=2, want_vectors=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = sum(1 for x in r.res if x <= 1e-8)
    out["annulus_eigs"] = {"pairs": ok, "wave_solves": r.wave_solves, "n_t": op.n_t, "seconds": dt,
                           "eigenpairs_per_s": ok / dt, "max_res": max(r.res)}
    log(f"mapped form: annulus eigs: {ok} pairs, {r.wave_solves} wave-solves, {dt:.2f} s")
    op.close()
    return out


def headline_np_rule(budget: int = 400):
    """The headline eigenproblem (2047^2, order 4, implicit, omega 120, k = 16)
    as a complete eigensolve, with N_p from the lobe rule and m = 2k + 1: at
    N_p = 1 the lobe holds about 1000 eigenvalues above beta 0.8 and the solve
    does not finish; the rule's N_p narrows it to about k.  Eigenpairs/s at
    eig-res <= 1e-8, every eigenvalue checked against the closed form."""
    import numpy as np
    import torch
    import synthetic
    from oracle import discrete as D
    from paper_2507_18282_amd import Operator, choose_periods
    P = synthetic.config_square_order4_implicit()
    n_p, n_lobe = choose_periods(P.length, P.omega, P.k)
    op = Operator(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its, n_p=n_p,
                  adjust_omega=P.adjust_omega, mg_tol=P.mg_tol, mg_max_levels=HEADLINE_MG_LEVELS,
                  mg_coarse_sweeps=HEADLINE_COARSE_SWEEPS)
    log(f"headline with the N_p rule: N_p {n_p} ({n_lobe} eigenvalues in the lobe), budget {budget} wave-solves")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = op.eigs(P.k, 2 * P.k + 1, seed=P.seed, want_vectors=False, max_wave_solves=budget, raise_on_error=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = sum(1 for x in r.res if x <= 1e-8)
    h = D.spacing(P.n, P.length)
    mu_cf = np.sort(D.mu_all(P.n, h, P.order).ravel())
    errs = [float(np.min(np.abs(mu_cf - m)) / m) for m in r.mu]
    log(f"headline with the N_p rule: {ok} pairs, {r.wave_solves} wave-solves, {r.restarts} restarts, "
        f"{r.probes} runs, {dt:.1f} s")
    out = {"workload": "unit square 2049^2 points (2047^2 interior), order 4, implicit 10 steps/period, omega 120 "
                       "(adjusted), FP64 multigrid to 1e-10 (automatic depth), k=16, m=33",
           "value": ok / dt, "unit": "eigenpairs/s",
           "n_p": n_p, "eigenvalues_in_lobe": n_lobe, "pairs": ok, "wave_solves": r.wave_solves,
           "restarts": r.restarts, "runs": r.probes, "seconds": dt, "max_res": max(r.res) if r.res else None,
           "max_mu_rel_err_vs_closed_form": max(errs) if errs else None,
           "pt_updates_per_s": r.pt_updates / dt,
           "mg_cycles_per_implicit_solve": r.mg_cycles / max(1, r.time_steps), "status": r.status,
           "mu": list(r.mu)}
    op.close()
    return out

def many_pairs(ks=None):
    """The square128 grid (127^2 interior), order 2, implicit 10 steps/period,
    omega 12 (adjusted), FP64 multigrid to 1e-10, one period: k eigenpairs at
    once with a Krylov dimension of 2k + 1, for k = 16, 64, 256, 512.  The
    Ritz tolerance equals the multigrid tolerance: S is applied to that
    accuracy, so a smaller one cannot be met reliably (with 1e-12 the counts
    of wave-solves follow the rounding of the multigrid)."""
    import torch
    import synthetic
    from paper_2507_18282_amd import Operator
    out = {"workload": "unit square 129^2 points (127^2 interior, h=1/128), order 2, implicit 10 steps/period, "
                       "omega 12 (adjusted), FP64 multigrid to 1e-10 (automatic depth: 127^2..15^2), N_p 1, "
                       "Krylov dimension 2k+1, "
                       "tol_ritz 1e-10 (= the multigrid tolerance), eig-res <= 1e-8"}
    for k in (ks or sorted(MANY_PAIRS_PAPER)):
        P = synthetic.config_many_pairs(k=k)
        op = Operator(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its,
                      adjust_omega=P.adjust_omega, mg_tol=P.mg_tol, mg_max_levels=MG_LEVELS,
                      mg_coarse_sweeps=MG_COARSE_SWEEPS)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.eigs(P.k, P.m, seed=P.seed, tol_ritz=P.mg_tol, want_vectors=False, k_cap=3 * k,
                    raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        conv, ws = MANY_PAIRS_PAPER.get(k, (None, None))
        out[f"k_{k}"] = {"m": P.m, "converged": r.n_conv, "wave_solves": r.wave_solves, "restarts": r.restarts,
                         "probes": r.probes, "wave_solves_per_eigenpair": r.wave_solves / max(1, r.n_conv),
                         "seconds": dt, "eigenpairs_per_s": r.n_conv / dt, "max_res": max(r.res) if r.res else None,
                         "status": r.status,
                         "paper": ({"converged": conv, "wave_solves": ws, "wave_solves_per_eigenpair": ws / conv}
                                   if conv else None)}
        log(f"many pairs: k {k} m {P.m}: {r.n_conv} converged, {r.wave_solves} wave-solves "
            f"({r.wave_solves / max(1, r.n_conv):.2f} per pair" + (f"; paper {ws / conv:.2f}" if conv else "") +
            f"), {dt:.2f} s")
        op.close()
    return out


def mixed_cube(n_cube: int = CUBE_N, precs=("mixed", "fp64")):
    """Unit cube, order 2, implicit 10 steps/period, omega 40 (adjusted), k = 8,
    m = 17, N_p from the lobe rule: complete eigensolves in mixed precision
    (FP32 inner multigrid + FP64 defect correction, FP32 filter accumulation)
    and in FP64 with the same solver settings (Ritz tolerance MIXED_TOL_RITZ,
    deflation probes for the repeated eigenvalues, CUBE_BUDGET wave-solves),
    each eigenvalue compared with the closed form and with the FP64 solve's,
    eig-res stated; and the cost of one period on the 255^3 grid in both
    precisions (S^2 v compared).  `precs` selects the complete solves that run
    (a 255^3 solve takes minutes in each precision)."""
    import numpy as np
    import torch
    import synthetic
    from oracle import discrete as D
    from paper_2507_18282_amd import Operator, choose_periods, fill_uniform
    P = synthetic.config_cube_mixed(n=n_cube)
    n_p, n_lobe = choose_periods(P.length, P.omega, P.k)
    h = D.spacing(P.n, P.length)
    mu_cf = np.sort(D.mu_all(P.n, h, P.order).ravel())
    out = {"workload": f"unit cube {n_cube + 2}^3 points ({n_cube}^3 interior), order 2, implicit 10 steps/period, "
                       f"omega 40 (adjusted), N_p {n_p} (lobe rule), k=8, m=17, multigrid to 1e-10",
           "n_p": n_p, "eigenvalues_in_lobe": n_lobe}
    res = {}
    for prec in precs:
        op = Operator(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its, n_p=n_p,
                      adjust_omega=True, precision=prec, mg_tol=P.mg_tol, mg_max_levels=MG_LEVELS,
                      mg_coarse_sweeps=MG_COARSE_SWEEPS)
        # the same solver settings for both precisions: a Ritz tolerance above the
        # FP32 noise of the mixed S v, and the same wave-solve budget
        tol_ritz = MIXED_TOL_RITZ
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.eigs(P.k, P.m, seed=P.seed, tol_ritz=tol_ritz, tol_res=1e-4, want_vectors=False,
                    raise_on_error=False, max_wave_solves=CUBE_BUDGET)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        errs = [float(np.min(np.abs(mu_cf - m)) / m) for m in r.mu]
        res[prec] = r
        ok = sum(1 for e in errs if e <= (1e-5 if prec == "mixed" else 1e-10))
        out[prec] = {"pairs_returned": len(r.mu), "pairs_within_tolerance": ok,
                     "tolerance_vs_closed_form": 1e-5 if prec == "mixed" else 1e-10,
                     "wave_solves": r.wave_solves, "seconds": dt, "eigenpairs_per_s": ok / dt,
                     "ms_per_wave_solve": dt / max(1, r.wave_solves) * 1e3,
                     "mg_cycles_per_implicit_solve": r.mg_cycles / max(1, r.time_steps), "status": r.status,
                     "tol_ritz": tol_ritz, "max_res": max(r.res) if r.res else None,
                     "per_pair": [{"mu": m, "rel_err_vs_closed_form": e, "eig_res": q}
                                  for m, e, q in zip(r.mu, errs, r.res)]}
        log(f"mixed cube {n_cube}^3 {prec}: {len(r.mu)} pairs, {r.wave_solves} wave-solves, {dt:.1f} s, "
            f"max err vs closed form {max(errs) if errs else float('nan'):.2e}, "
            f"max eig-res {max(r.res) if r.res else float('nan'):.2e}")
        op.close()
    a, b = (sorted(res[p].mu) if p in res else [] for p in ("mixed", "fp64"))
    if a and b and len(a) == len(b):
        out["mixed_vs_fp64_mu_rel_diff"] = [abs(x - y) / y for x, y in zip(a, b)]
    # one period on 255^3: cost of each precision, S^2 v compared
    Pb = synthetic.config_cube_mixed()
    Sv, cost = {}, {}
    for prec in ("mixed", "fp64"):
        op = Operator(n=Pb.n, length=Pb.length, order=Pb.order, omega=Pb.omega, ts=Pb.ts, n_its=Pb.n_its,
                      adjust_omega=True, precision=prec, mg_tol=Pb.mg_tol, mg_max_levels=MG_LEVELS,
                      mg_coarse_sweeps=MG_COARSE_SWEEPS)
        v = fill_uniform(op.n_active, Pb.seed)
        w = op.apply_filter(v)
        torch.cuda.synchronize()
        op.reset_stats()
        t0 = time.perf_counter()
        w = op.apply_filter(v)
        w2 = op.apply_filter(w)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = op.stats()
        Sv[prec] = w2
        cost[prec] = {"pt_updates_per_s": st["pt_updates"] / dt, "ms_per_wave_solve": dt / 2 * 1e3,
                      "mg_cycles_per_implicit_solve": st["mg_cycles"] / max(1, st["mg_solves"])}
        op.close()
    cost["mixed_vs_fp64_rel_err_S2v"] = (Sv["mixed"] - Sv["fp64"]).abs().max().item() / Sv["fp64"].abs().max().item()
    cost["speedup"] = cost["mixed"]["pt_updates_per_s"] / cost["fp64"]["pt_updates_per_s"]
    out["one_period_255"] = cost
    return out

def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solves", type=int, default=4)
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and mixed-precision comparisons")
    ap.add_argument("--batch-budget", type=int, default=150, help="wave-solves per problem in the batch comparison")
    ap.add_argument("--many-k", type=int, nargs="*", default=None,
                    help="requested counts of the many-pairs form (default: the paper's table rows)")
    ap.add_argument("--only-many-pairs", action="store_true",
                    help="run only the many-pairs form and print its JSON (for profiling)")
    ap.add_argument("--only-walls", action="store_true",
                    help="run only the Neumann-walls form and print its JSON (for profiling)")
    ap.add_argument("--only-mapped", action="store_true",
                    help="run only the curvilinear-grid form (mapped vs box wave-solve, annulus eigensolve)")
    ap.add_argument("--headline-np-rule", action="store_true",
                    help="run only the complete headline eigensolve with the N_p of the lobe rule and print its JSON")
    ap.add_argument("--only-learned", action="store_true", help="run only the learned-guess form and print its JSON")
    ap.add_argument("--only-cube", action="store_true", help="run only the mixed-vs-FP64 cube form and print its JSON")
    ap.add_argument("--only-batch", action="store_true", help="run only the batched form and print its JSON")
    ap.add_argument("--cube-n", type=int, default=CUBE_N,
                    help="cube side of the mixed-vs-FP64 eigensolves (63 by default; 127 and 255 are longer runs)")
    ap.add_argument("--cube-prec", choices=("mixed", "fp64", "both"), default="both",
                    help="which complete cube eigensolves run (one precision per call keeps a 255^3 run shorter)")
    ap.add_argument("--no-headline-eigs", action="store_true",
                    help="skip the complete headline eigensolve (the eigenpairs/s of the headline workload)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); a multi-GPU decomposition "
              "(slabs with a halo exchange per half-sweep) is not built", file=sys.stderr)
        return 2
    import torch
    import synthetic
    from paper_2507_18282_amd import Operator

    torch.cuda.set_device(0)
    if a.only_many_pairs:
        print(json.dumps({"form": "many_pairs", "result": many_pairs(a.many_k)}), flush=True)
        return 0
    if a.only_walls:
        print(json.dumps({"form": "walls", "result": walls_form()}), flush=True)
        return 0
    if a.only_mapped:
        print(json.dumps({"form": "mapped", "result": mapped_form()}), flush=True)
        return 0
    if a.headline_np_rule:
        print(json.dumps({"form": "headline_np_rule", "result": headline_np_rule()}), flush=True)
        return 0
    if a.only_learned:
        print(json.dumps({"form": "learned_vs_plain", "result": learned_vs_plain()}), flush=True)
        return 0
    if a.only_cube:
        precs = ("mixed", "fp64") if a.cube_prec == "both" else (a.cube_prec,)
        print(json.dumps({"form": "mixed_cube", "result": mixed_cube(a.cube_n, precs)}), flush=True)
        return 0
    if a.only_batch:
        print(json.dumps({"form": "batched_vs_plain", "result": batched_vs_plain(a.batch_budget)}), flush=True)
        return 0
    P = synthetic.config_square_order4_implicit()
    op = Operator(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its, n_p=P.n_p,
                  adjust_omega=P.adjust_omega, precision=P.precision, mg_tol=P.mg_tol,
                  mg_max_levels=HEADLINE_MG_LEVELS, mg_coarse_sweeps=HEADLINE_COARSE_SWEEPS)
    coarsest = P.n[0]
    for _ in range(op.mg_levels - 1):
        coarsest = (coarsest - 1) // 2
    log(f"workload {P.n} order {P.order} n_t {op.n_t} omega_used {op.omega_used:.4f} levels {op.mg_levels} "
        f"(coarsest {coarsest}^2)")
    if a.warmup > 0:
        op.eigs(P.k, P.m, seed=P.seed, max_wave_solves=a.warmup, want_vectors=False, raise_on_error=False)
    log("warmup done")
    torch.cuda.synchronize()
    op.profile_begin("smooth", level=0)
    t0 = time.perf_counter()
    r = op.eigs(P.k, P.m, seed=P.seed, max_wave_solves=a.steps, want_vectors=False, raise_on_error=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = op.profile_end()
    elapsed = t1 - t0
    assert r.wave_solves == a.steps, (r.wave_solves, a.steps)
    value = r.pt_updates / elapsed
    log(f"timed {a.steps} steps in {elapsed:.3f} s; MG cycles per implicit solve "
        f"{r.mg_cycles / max(1, r.time_steps):.2f}")

    avg_ms = prof["total_ms"] / max(1, prof["launches"])
    bytes_per_launch = prof["bytes_alg"] / max(1, prof["launches"])
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    # The dominant kernel runs the two pre-smoothing sweeps of the finest level in
    # one pass.  Algorithmic bytes are counted per point-sweep (x and b read, x
    # written: 3 x 8 B), two sweeps per launch; the pass itself moves each array
    # once, so its minimum traffic is half of that (frac_min_traffic).
    roofline = {"bound": "hbm",
                "kernel": "two red-black Gauss-Seidel sweeps in one pass, finest level "
                          "(k_sweep2x_tile2d<double, 4, 16, false, false>)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "launches": prof["launches"], "avg_us": round(avg_ms * 1e3, 3),
                "bytes_alg_per_launch": bytes_per_launch,
                "bytes_alg_unit": "24 B per point-sweep (read x, b; write x), 2 sweeps per launch",
                "frac_min_traffic": round(achieved / 2 / HBM_PEAK_GBS, 4),
                "kernel_share_of_step": round(prof["total_ms"] * 1e-3 / elapsed, 3)}

    vcycle = vcycle_roofline(op)

    # Eigenpairs per second: a complete solve of the 64^2 explicit workload.
    P1 = synthetic.config_small_explicit()
    op1 = Operator(n=P1.n, length=P1.length, order=P1.order, omega=P1.omega, ts=P1.ts, cfl=P1.cfl)
    op1.eigs(P1.k, P1.m, seed=P1.seed, want_vectors=False)  # warm
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    r1 = op1.eigs(P1.k, P1.m, seed=P1.seed, want_vectors=False)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    n_ok = sum(1 for x in r1.res if x <= 1e-8)
    eig = {"value": n_ok / (t3 - t2), "unit": "eigenpairs/s", "pairs": n_ok, "requested": P1.k,
           "wave_solves": r1.wave_solves, "seconds": round(t3 - t2, 4), "max_res": max(r1.res),
           "pt_updates_per_s": r1.pt_updates / (t3 - t2),
           "workload": "unit square 64^2 interior (h = 1/65), order 2, explicit leapfrog CFL 0.5 (78 steps), "
                       "omega 15, Krylov dimension 16, 4 requested, seed 1"}

    headline_eigs = None
    if not a.no_headline_eigs:
        headline_eigs = headline_np_rule()

    forms = {}
    if not a.no_forms:
        forms["batched_vs_plain"] = batched_vs_plain(a.batch_budget)
        forms["mixed_cube"] = mixed_cube(a.cube_n)
        forms["learned_vs_plain"] = learned_vs_plain()
        forms["periods_rule"] = periods_rule()
        forms["many_pairs"] = many_pairs(a.many_k)
        forms["walls"] = walls_form()
        forms["mapped"] = mapped_form()

    cpu = None
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(P, a.cpu_solves)

    out = {
        "metric": METRIC, "value": value, "unit": "grid-pt updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": elapsed / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "unit square 2049^2 points (2047^2 interior, h=1/2048), 4th-order Laplacian, "
                               f"implicit 10 steps/period, FP64 multigrid V(2,1) (levels 2047^2..{coarsest}^2, {HEADLINE_COARSE_SWEEPS} sweep(s) on {coarsest}^2) to rel. "
                               "residual 1e-10, "
                               "omega 120 (adjusted 109.7306), Arnoldi m=32 for k=16, seed 2",
                   "global_batch": 1, "parallelism": "single GPU"},
        "mg_cycles_per_implicit_solve": round(r.mg_cycles / max(1, r.time_steps), 3),
        "eigenpairs_per_s": eig,
        "eigenpairs_per_s_headline": headline_eigs,
        "roofline": roofline,
        "vcycle_roofline": vcycle,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
