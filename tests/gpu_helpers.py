"""Shared helpers for the GPU parity tests (oracle on the CPU, HIP path through the C ABI)."""
import sys

import numpy as np

import synthetic
from oracle import discrete as D
from oracle import wave as W


def say(*a):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print(*a, file=sys.stderr, flush=True)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def make_op(P: synthetic.Problem, **kw):
    from paper_2507_18282_amd import Operator
    args = dict(n=P.n, length=P.length, order=P.order, omega=P.omega, ts=P.ts, cfl=P.cfl, n_its=P.n_its,
                n_p=P.n_p, adjust_omega=P.adjust_omega, filter_const=P.filter_const, precision=P.precision,
                mg_tol=P.mg_tol)
    args.update(kw)
    return Operator(**args)


def oracle_plan(P: synthetic.Problem):
    h = D.spacing(P.n, P.length)
    plan = D.time_plan(h, P.order, P.omega, P.ts, cfl=P.cfl, n_its=P.n_its, n_p=P.n_p,
                       adjust_omega=P.adjust_omega, filter_const=P.filter_const)
    return h, plan


def oracle_S(P: synthetic.Problem, v: np.ndarray) -> np.ndarray:
    h, plan = oracle_plan(P)
    return W.apply_filter(v.reshape(P.n[::-1]), h, P.order, plan).ravel()


def assert_signs(Y):
    """The returned eigenvectors' sign convention: in each column the entry of
    largest magnitude (the first such) is positive."""
    Y = np.asarray(Y)
    for c in range(Y.shape[1]):
        i = int(np.argmax(np.abs(Y[:, c])))
        assert Y[i, c] > 0.0, (c, i, Y[i, c])


def rel_err(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
