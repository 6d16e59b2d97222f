"""The site-parallel kernel (BLIP_KERNEL_SITE) in its particle-by-particle
form: one launch per position gives, bit for bit, the rows of one launch over
the whole block (each (position, orbital) item is summed by the same fixed
butterfly whatever the launch), and so does the captured graph of those
launches that the benchmark replays.  Accuracy against the oracle is in
test_gpu_parity.py."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import group_errors, say, to_np

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def blip():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    torch.cuda.init()
    from paper_1204_1121_amd import blip as b
    b.lib()
    return b


CASES = ("real f32", "complex c64 at k")


def make_case(blip, label):
    """A small ragged table (L = 29 real or 13 complex on a 9x8x7 grid) and
    41 positions, many outside the cell."""
    rng = np.random.default_rng(1204)
    A = np.diag([7.0, 6.0, 5.0])
    n = (9, 8, 7)
    pos = rng.uniform(-9, 17, (41, 3))
    if label == "real f32":
        c = rng.uniform(-1, 1, n + (29,)).astype(np.float32)
        return blip.Table(A, n, c, "f32"), A, n, c, None, pos
    k = np.array([0.3, -0.2, 0.1])
    c = (rng.standard_normal(n + (13,)) + 1j * rng.standard_normal(n + (13,))).astype(np.complex64)
    return blip.Table(A, n, c, "c64", kvec=k), A, n, c, k, pos


@pytest.mark.parametrize("grad", [True, False])
@pytest.mark.parametrize("label", CASES)
def test_per_position_launches_equal_block_launch(blip, label, grad):
    t, A, n, c, k, pos = make_case(blip, label)
    say(f"site kernel, one launch per position vs block launch: {label}, grad={grad}")
    p = torch.from_numpy(pos).cuda()
    blk = t.eval(p, grad=grad, kernel="site")
    one = t.alloc_outputs(p.shape[0], grad=grad)
    for j in range(p.shape[0]):
        t.eval(p[j:j + 1], grad=grad, kernel="site",
               out=tuple(None if x is None else x[j:j + 1] for x in one))
    torch.cuda.synchronize()
    for x, y in zip(blk, one):
        if x is not None:
            np.testing.assert_array_equal(to_np(y), to_np(x))
    ref = oracle.evaluate(A, n, c, pos, kvec=k,
                          want=("val", "grad", "lap") if grad else ("val",))
    got = {"val": to_np(blk[0])}
    if grad:
        got.update(grad=to_np(blk[1]), lap=to_np(blk[2]))
    e = group_errors(got, ref)
    say("  vs oracle: " + " ".join(f"{q}={v:.2e}" for q, v in e.items()))
    assert max(e.values()) <= FP32_TOL
    t.free()


def test_captured_per_position_launches(blip):
    """The benchmark's particle-by-particle timing replays a graph of npos
    single-position launches.  Each of three replays, with eager work and a
    synchronisation between them, must give the block launch's rows."""
    label = CASES[1]
    t, A, n, c, k, pos = make_case(blip, label)
    say(f"site kernel, captured per-position launches: {label}")
    p = torch.from_numpy(pos).cuda()
    blk = t.eval(p, grad=False, kernel="site")
    out = t.alloc_outputs(p.shape[0], grad=False)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        calls = [t.bind(p[j:j + 1], (out[0][j:j + 1], None, None), kernel="site")
                 for j in range(p.shape[0])]
        for call in calls:
            call()
    torch.cuda.synchronize()
    for rep in range(3):
        out[0].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(out[0]), to_np(blk[0]), err_msg=f"replay {rep}")
        t.eval(p, grad=False, kernel="site")   # eager work between replays
        torch.cuda.synchronize()
    t.free()
