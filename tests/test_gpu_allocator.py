"""The device-allocator hook (ew_set_allocator): with PyTorch's caching
allocator supplying the library's buffers, operators, the eigensolver and a
batch give the same results as with hipMalloc, the buffers show up in
PyTorch's accounting while the objects live and are handed back when they
are destroyed, and the hook cannot be swapped while buffers are live."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2507_18282_amd as ew
from paper_2507_18282_amd import _lib
import synthetic
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _run(n, ts):
    op = ew.Operator(n=n, length=(1.0, 1.0), order=2, omega=20.0, ts=ts, n_its=10, mg_tol=1e-10)
    v = torch.from_numpy(synthetic.start_vector(3, op.n_active)).cuda()
    s = op.apply_filter(v)
    r = op.eigs(k=4, m=12, seed=5)
    torch.cuda.synchronize()
    return op, s.cpu().numpy(), np.array(r.mu), r.Y.cpu().numpy()


def _batch():
    probs = [{"n": (31, 31), "length": (1.0, 1.0), "order": 2, "omega": 12.0},
             {"n": (95, 63), "length": (1.5, 1.0), "order": 2, "omega": 15.0}]
    b = ew.Batch(probs)
    vs = [torch.from_numpy(synthetic.start_vector(7 + i, n)).cuda() for i, n in enumerate(b.n_active)]
    outs = b.apply_filter(vs)
    torch.cuda.synchronize()
    return b, [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("ts", ["explicit", "implicit"])
def test_torch_allocator_matches_hipmalloc(ts):
    n = (127, 95)
    say(f"allocator hook, {ts} {n}")
    op, s0, mu0, y0 = _run(n, ts)
    op.close()
    b, outs0 = _batch()
    b.close()
    base = torch.cuda.memory_allocated()
    ew.use_torch_allocator(True)
    op = b = None
    try:
        op, s1, mu1, y1 = _run(n, ts)
        held = torch.cuda.memory_allocated() - base
        assert held >= 2 * op.n_active * 8, held                 # the operator's own vectors
        with pytest.raises(ew.EigenwaveError):
            ew.use_torch_allocator(False)                        # buffers are live
        b, outs1 = _batch()
    finally:
        for obj in (op, b):
            if obj is not None:
                obj.close()
        ew.use_torch_allocator(False)
    assert torch.cuda.memory_allocated() == base
    # same kernels on the same inputs; launch shapes tuned by timing at
    # creation may differ between the runs, so compare to rounding level
    assert np.max(np.abs(s1 - s0)) <= 1e-12 * np.max(np.abs(s0))
    assert np.max(np.abs(mu1 - mu0) / mu0) <= 1e-10
    assert np.max(np.abs(y1 - y0)) <= 1e-6 * np.max(np.abs(y0))
    for a, c in zip(outs0, outs1):
        assert np.max(np.abs(a - c)) <= 1e-5 * np.max(np.abs(a))   # FP32 stepping in the batch


def test_hooks_see_every_buffer_once():
    """A counting hook on the raw C-ABI: the Krylov basis of the eigensolver
    goes through it, every pointer handed out comes back exactly once, and
    the stream argument is the operator's stream."""
    live, peak, streams, bad = {}, [0], set(), []

    def alloc(nbytes, dev, stream, ctx):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), int(dev), int(stream or 0))
        live[int(p)] = int(nbytes)
        peak[0] = max(peak[0], sum(live.values()))
        streams.add(int(stream or 0))
        return int(p)

    def free(p, ctx):
        if live.pop(int(p), None) is None:
            bad.append(int(p))
        torch.cuda.caching_allocator_delete(int(p))

    hooks = (_lib.ALLOC_FN(alloc), _lib.FREE_FN(free))
    lib = ew.load()
    s = torch.cuda.Stream()
    _lib.check(lib.ew_set_allocator(ctypes.cast(hooks[0], ctypes.c_void_p), ctypes.cast(hooks[1], ctypes.c_void_p),
                                    None))
    try:
        with torch.cuda.stream(s):
            op = ew.Operator(n=(127, 95), length=(1.0, 1.0), order=2, omega=20.0, ts="implicit")
            held, na = sum(live.values()), op.n_active
            r = op.eigs(k=4, m=12, seed=5)
            s.synchronize()
            assert r.n_conv >= 4
            op.close()
    finally:
        lib.ew_set_allocator(None, None, None)
    assert not live and not bad
    assert peak[0] >= held + 12 * na * 8, (peak[0], held)
    assert streams == {int(s.cuda_stream)}
