"""Workload for rocprofv3 counter runs: one plain device copy of a known size
(the calibration for FETCH_SIZE / WRITE_SIZE) followed by wave-solves of the
headline implicit workload (2047^2 interior, order 4, FP64 multigrid), or
with ``--workload mapped`` explicit wave-solves on the 2047^2 skew-mapped
grid (order 2, omega 60, CFL 0.9), or with ``--workload mapped-implicit``
one implicit wave-solve there (omega 60 adjusted, 10 steps, multigrid to
1e-10).

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
    ap.add_argument("--workload", choices=("headline", "mapped", "mapped-implicit"), default="headline")
    a = ap.parse_args(argv)
    import torch
    import synthetic
    from paper_2507_18282_amd import Operator, fill_uniform
    torch.cuda.set_device(0)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    if a.workload in ("mapped", "mapped-implicit"):
        n = (2047, 2047)
        xy = synthetic.mapped_coords("skew", *n, eps=0.15)
        if a.workload == "mapped":
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
    # the multigrid settings of the benchmark: automatic depth (down to 127^2), 4 sweeps there
    op = Operator(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, n_its=P.n_its, n_p=P.n_p,
                  adjust_omega=P.adjust_omega, precision=P.precision, mg_tol=P.mg_tol, mg_max_levels=-1,
                  mg_coarse_sweeps=4)
    v = fill_uniform(op.n_active, P.seed)
    for _ in range(a.wave_solves):
        v = op.apply_filter(v)
    torch.cuda.synchronize()
    print("counters probe done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
