"""Workload for rocprofv3 counter runs: one plain device copy of a known size
(the calibration for FETCH_SIZE / WRITE_SIZE) followed by wave-solves of the
headline implicit workload (2047^2 interior, order 4, FP64 multigrid), or
with ``--workload mapped`` explicit wave-solves on the 2047^2 skew-mapped
grid (order 2, omega 60, CFL 0.9), or with ``--workload box-explicit`` the
same on the 2047^2 unit square, or with ``--workload mapped-implicit``
one implicit wave-solve there (omega 60 adjusted, 10 steps, multigrid to
1e-10).  Further workloads for kernel traces:

  cube    implicit wave-solves of the 255^3 cube in mixed precision (FP32
          multigrid sweeps with FP64 defect correction);
  batch   batched wave-solves of the 96 rectangles, FP32 state then FP64 state;
  cnn     crops from one wave-solve of the 1023^2 learned-guess workload, 64
          training steps of the network (batch 32), then wave-solves with the
          learned guess (one network evaluation per implicit step after the
          first).

  rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2507_18282_amd.counters_probe
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 256 * 1024 * 1024


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--wave-solves", type=int, default=1)
    ap.add_argument("--workload", choices=("headline", "mapped", "box-explicit", "mapped-implicit", "cube", "batch",
                                                "cnn"),
                    default="headline")
    a = ap.parse_args(argv)
    import torch
    import synthetic
    from paper_2507_18282_amd import Operator, fill_uniform
    torch.cuda.set_device(0)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    if a.workload in ("cube", "batch", "cnn"):
        _trace_workload(a.workload, a.wave_solves)
        torch.cuda.synchronize()
        print("counters probe done", flush=True)
        return 0
    if a.workload in ("mapped", "box-explicit", "mapped-implicit"):
        n = (2047, 2047)
        xy = synthetic.mapped_coords("skew", *n, eps=0.15)
        if a.workload == "box-explicit":
            op = Operator(n=n, length=(1.0, 1.0), order=2, omega=60.0, ts="explicit", cfl=0.9)
        elif a.workload == "mapped":
            op = Operator(n=n, length=(1.0, 1.0), order=2, omega=60.0, ts="explicit", cfl=0.9, coords=xy)
        else:
            op = Operator(n=n, length=(1.0, 1.0), order=2, omega=60.0, ts="implicit", n_its=10, adjust_omega=True,
                          mg_tol=1e-10, mg_max_levels=-1, mg_coarse_sweeps=4, coords=xy)
        v = fill_uniform(op.n_active, 3)
        for _ in range(a.wave_solves):
            v = op.apply_filter(v)
        torch.cuda.synchronize()
        print("counters probe done", flush=True)
        return 0
    P = synthetic.config_square_order4_implicit()
    # the multigrid settings of the benchmark's headline: 5 levels (down to 127^2), one sweep there
    op = Operator(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its, n_p=P.n_p,
                  adjust_omega=P.adjust_omega, precision=P.precision, mg_tol=P.mg_tol, mg_max_levels=5,
                  mg_coarse_sweeps=1)
    v = fill_uniform(op.n_active, P.seed)
    for _ in range(a.wave_solves):
        v = op.apply_filter(v)
    torch.cuda.synchronize()
    print("counters probe done", flush=True)
    return 0


def _trace_workload(workload: str, wave_solves: int) -> None:
    import torch
    import synthetic
    from paper_2507_18282_amd import Batch, Cnn, CropStore, Operator, fill_uniform
    if workload == "cube":
        P = synthetic.config_cube_mixed()
        op = Operator(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its, n_p=P.n_p,
                      adjust_omega=P.adjust_omega, precision=P.precision, mg_tol=P.mg_tol)
        v = fill_uniform(op.n_active, P.seed)
        for _ in range(wave_solves):
            v = op.apply_filter(v)
            v = v / v.norm()
        return
    if workload == "batch":
        Ps = synthetic.batch_problems()
        for precision in ("mixed", "fp64"):
            bt = Batch([{"n": P.n, "length": P.length, "order": 2, "omega": P.omega, "cfl": 0.5,
                         "precision": precision} for P in Ps])
            vs = [fill_uniform(P.n[0] * P.n[1], P.seed) for P in Ps]
            for _ in range(wave_solves):
                vs = bt.apply_filter(vs)
                vs = [x / x.norm() for x in vs]
            torch.cuda.synchronize()
            bt.close()
            print(f"batch {precision} done", flush=True)
        return
    P = synthetic.config_learned()

    def make(predictor):
        return Operator(n=P.n, length=P.length, order=P.order, omega=90.0, ts=P.ts, n_its=P.n_its, n_p=1,
                        adjust_omega=P.adjust_omega, mg_tol=P.mg_tol, predictor=predictor, mg_max_levels=-1,
                        mg_coarse_sweeps=4)
    store = CropStore(9 * 19, 128, P.order)
    op = make("proj")
    v = fill_uniform(op.n_active, 5000)
    store.collect(op, v, crops_per_step=19, seed=777)
    op.close()
    net = Cnn(1)
    net.train(store, steps=64, batch=32, lr=2e-3, seed=11)
    print(f"cnn trained on {store.count} crops", flush=True)
    op = make("cnn")
    op.set_cnn(net)
    v = fill_uniform(op.n_active, 99)
    for _ in range(wave_solves + 1):  # the first wave-solve fills the projection window
        v = op.apply_filter(v)
        v = v / v.norm()


if __name__ == "__main__":
    sys.exit(main())
