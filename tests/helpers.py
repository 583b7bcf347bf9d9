"""Shared helpers of the GPU tests: host<->device copies and bitwise comparison rules."""
import numpy as np


def dev(a):
    """numpy -> contiguous CUDA tensor (same dtype)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def assert_same_values(got, want, what=""):
    """Every component equal as a binary64 value (+0 == -0; any NaN fails)."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    assert not np.isnan(got).any(), "%s: NaN in GPU result" % what
    assert not np.isnan(want).any(), "%s: NaN in oracle result" % what
    bad = got != want
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError("%s: %d mismatches, first at %s: gpu=%r oracle=%r" % (
            what, int(bad.sum()), idx.tolist(), [got[tuple(i)] for i in idx], [want[tuple(i)] for i in idx]))
