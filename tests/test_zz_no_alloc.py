"""The allocation-free batched step (slbm_batch_step_static) against slbm_batch_step,
through the C ABI: the same members stepped the same number of steps must give the same
state, on two calls in a row (the second with a smaller batch), then once more on the first
batch after the second one has taken over the static array."""
import numpy as np
import pytest

from synth import cases

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _rel(a, b):
    d = np.abs(a - b).max()
    s = np.abs(b).max()
    return d / s if s > 0 else d


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_00535_amd as P
    P.lib()
    return P


def _solves(P, cs, stream):
    out = []
    for c in cs:
        s = P.Solve(c, stream=stream)
        s.init_tanh()
        out.append(s)
    return out


def test_static_batch_step_equals_batch_step(P):
    import torch
    big = [cases.small_flat(60.0, nx=16, ny=8, N=6, Lx=128.0, Ly=64.0, R=24.0),
           cases.small_cyl(120.0), cases.small_sphere(), cases.small_flat(90.0, N=4)]
    small = [cases.c1(), cases.small_flat(75.0, N=5)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ref = {}
        for key, cs, n in (("big", big, 30), ("small", small, 20)):
            ss = _solves(P, cs, stream)
            b = P.Batch(stream)
            for s in ss:
                b.add(s)
            b.step(n)
            ref[key] = [s.get_state()[0] for s in ss]
            b.step(10)
            ref[key + "+10"] = [s.get_state()[0] for s in ss]
            del b
        print("[no-alloc] references stepped", flush=True)
        sb, ss_ = _solves(P, big, stream), _solves(P, small, stream)
        bb, bs = P.Batch(stream), P.Batch(stream)
        for s in sb:
            bb.add(s)
        for s in ss_:
            bs.add(s)
        bb.step_static(30)
        print("[no-alloc] big batch: 30 static steps", flush=True)
        for s, r in zip(sb, ref["big"]):
            f, st = s.get_state()
            assert st == 30 and _rel(f, r) <= TOL
        bs.step_static(20)  # smaller input: the array now holds the small batch's tables
        print("[no-alloc] small batch: 20 static steps", flush=True)
        for s, r in zip(ss_, ref["small"]):
            f, st = s.get_state()
            assert st == 20 and _rel(f, r) <= TOL
        bb.step_static(10)  # the big batch again: its tables are uploaded anew
        print("[no-alloc] big batch: 10 more static steps", flush=True)
        for s, r in zip(sb, ref["big+10"]):
            assert _rel(s.get_state()[0], r) <= TOL
        bs.step(10)  # the regular step on a batch that stepped statically
        for s, r in zip(ss_, ref["small+10"]):
            assert _rel(s.get_state()[0], r) <= TOL
        del bb, bs
