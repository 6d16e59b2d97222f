"""blip_eval_batched_static: the batched launch with the library's fixed
scratch instead of a caller's workspace.  Two calls in a row, the second with
a smaller batch, each equal bit for bit to blip_eval_batched on the same
input; the largest capacity the fixed scratch serves; the capacity limit
refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_util import say, to_np

pytestmark = pytest.mark.gpu

MAX_CAPACITY = 131072


@pytest.fixture(scope="module")
def blip():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    from paper_1204_1121_amd import blip as b
    b.lib()
    return b


def ragged(rng, A, nw, maxb, sigma=0.3):
    sizes = rng.integers(1, maxb + 1, nw)
    off = np.zeros(nw + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    sites = rng.uniform(0, 1, (int(off[-1]), 3)) @ A
    return sites + rng.normal(0, sigma, sites.shape), off


def both(t, pos, off, grad=True):
    """(static result, workspace result) as numpy dicts, same input."""
    p = torch.from_numpy(pos).cuda()
    o = torch.from_numpy(off).cuda()
    out_s = t.alloc_outputs(pos.shape[0], grad)
    t.eval_batched_static(p, o, out_s)
    out_w = t.eval_batched(p, o, grad=grad)
    torch.cuda.synchronize()
    keys = ("val", "grad", "lap")
    return ({k: to_np(v) for k, v in zip(keys, out_s) if v is not None},
            {k: to_np(v) for k, v in zip(keys, out_w) if v is not None})


def test_static_two_calls_equal_workspace_path(blip):
    rng = np.random.default_rng(71)
    A = np.diag([7.0, 6.0, 5.0])
    n = (28, 24, 20)
    c = rng.uniform(-1, 1, n + (300,)).astype(np.float32)
    t = blip.Table(A, n, c, "f32")
    try:
        for nw, maxb in ((60, 64), (9, 20)):         # the second call smaller
            pos, off = ragged(rng, A, nw, maxb)
            say(f"static scratch: {nw} walkers, {off[-1]} positions")
            got, ref = both(t, pos, off)
            for k in ref:
                np.testing.assert_array_equal(got[k], ref[k], err_msg=f"nw {nw} {k}")
        pos, off = ragged(rng, A, 17, 40)
        say(f"static scratch, values only: {off[-1]} positions")
        got, ref = both(t, pos, off, grad=False)
        np.testing.assert_array_equal(got["val"], ref["val"])
    finally:
        t.free()


def test_static_largest_capacity_then_small(blip):
    rng = np.random.default_rng(72)
    A = np.diag([18.0, 18.0, 12.0])
    n = (72, 72, 48)                                 # 3,888 bricks of the sort
    c = (rng.standard_normal(n + (8,)) / np.sqrt(np.prod(n))).astype(np.float32)
    t = blip.Table(A, n, c, "f32")
    try:
        sizes = np.full(512, MAX_CAPACITY // 512, dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        pos = rng.uniform(0, 1, (MAX_CAPACITY, 3)) @ A + rng.normal(0, 0.5, (MAX_CAPACITY, 3))
        say(f"static scratch at its capacity: {MAX_CAPACITY} positions")
        got, ref = both(t, pos, off)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        pos2, off2 = ragged(rng, A, 3, 5)
        say(f"static scratch after the full call: {off2[-1]} positions")
        got, ref = both(t, pos2, off2)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        say("capacity above the fixed scratch is refused on the host")
        p = torch.zeros((MAX_CAPACITY + 1, 3), dtype=torch.float64, device="cuda")
        o = torch.tensor([0, MAX_CAPACITY + 1], dtype=torch.int64, device="cuda")
        out = t.alloc_outputs(1, True)
        rc = blip.lib().blip_eval_batched_static(t.handle, ctypes.c_void_p(p.data_ptr()),
                                                 ctypes.c_void_p(o.data_ptr()), 1,
                                                 MAX_CAPACITY + 1,
                                                 *[ctypes.c_void_p(x.data_ptr()) for x in out],
                                                 None)
        assert rc == -1, rc
        assert b"capacity" in blip.lib().blip_last_error()
    finally:
        t.free()
