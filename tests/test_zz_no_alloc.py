"""swsph_step_static (the entry point for callers that cannot allocate device
memory) against swsph_step with a caller workspace, through the C ABI.

Both run the same kernels on the same particles, so every output must be
bitwise identical: integer counts and float fields alike.  Two calls in a row
on one plan, the second with a smaller particle set (the library's scratch
keeps the first call's contents), then the reverse order on a fresh plan.
"""
import sys

import numpy as np
import pytest

from paper_2505_14538_amd import workloads as W

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_14538_amd import swsph
    return swsph


def _host_all(S, d, g, f):
    out = {}
    for pre, dd in (("d", d), ("g", g), ("f", f)):
        for k, v in S.host(dd).items():
            out[pre + "." + k] = np.array(v, copy=True)
    return out


def _compare(a, b, label):
    assert a.keys() == b.keys()
    for k in a:
        x, y = a[k], b[k]
        assert x.shape == y.shape, (label, k)
        assert np.array_equal(x, y), "%s: %s differs (max |diff| %g)" % (
            label, k, float(np.max(np.abs(x.astype(np.float64) - y.astype(np.float64)))))


def _sets():
    # a 16^3 jittered lattice (4,096 particles), then a smaller 12^3 one
    # (1,728) from another seed
    return [W.tiny(nside=16), W.tiny(nside=12, seed=77)]


def test_static_matches_workspace_step(S):
    import torch
    plan_s = S.Plan()
    plan_w = S.Plan()
    for parts in _sets():
        _flush("static step vs workspace step: n=%d" % parts.n)
        dp = S.to_device(parts)
        ds, gs, fs = plan_s.step_static(dp)
        torch.cuda.synchronize()
        st = plan_s.stats(static=True)
        assert st["code"] == 0, st
        a = _host_all(S, ds, gs, fs)
        dw, gw, fw = plan_w.step(dp)
        torch.cuda.synchronize()
        assert plan_w.stats()["code"] == 0
        b = _host_all(S, dw, gw, fw)
        _compare(a, b, "n=%d" % parts.n)
        # sanity: the results are a converged density solve
        assert np.all(a["d.iters"] > 0)
        assert np.all(a["d.nngb"] > 0)


def test_static_small_after_large_fresh_plan(S):
    """Reverse order on a fresh plan: smaller set first, then the larger one,
    each compared with the workspace path."""
    import torch
    plan_s = S.Plan()
    for parts in reversed(_sets()):
        _flush("static step (fresh plan) n=%d" % parts.n)
        dp = S.to_device(parts)
        ds, gs, fs = plan_s.step_static(dp)
        torch.cuda.synchronize()
        assert plan_s.stats(static=True)["code"] == 0
        a = _host_all(S, ds, gs, fs)
        plan_w = S.Plan()
        dw, gw, fw = plan_w.step(dp)
        torch.cuda.synchronize()
        b = _host_all(S, dw, gw, fw)
        _compare(a, b, "fresh n=%d" % parts.n)
