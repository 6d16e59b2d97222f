"""The streaming-read probe (blip_stream_read) that gives the bandwidth
denominator: the per-workgroup sums cover every element of the buffer once,
for buffer sizes that are not a multiple of the grid's stride and for
several grid sizes."""
import numpy as np
import pytest
import torch

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def blip():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    from paper_1204_1121_amd import blip as b
    b.lib()
    return b


@pytest.mark.parametrize("n,nblocks", [(4, 1), (1 << 20, 37), ((1 << 22) + 12, 2048),
                                       (3 * 256 * 4 * 7 + 4, 3)])
def test_every_element_read_once(blip, n, nblocks):
    say(f"stream read: {n} floats, {nblocks} workgroups")
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    part = torch.full((nblocks,), -1.0, dtype=torch.float32, device="cuda")
    blip.stream_read(ones, part)
    torch.cuda.synchronize()
    p = part.cpu().numpy().astype(np.float64)
    assert p.sum() == n                      # integers below 2^24 per workgroup: exact
    assert np.all(p >= 0)
    rng = np.random.default_rng(n)
    x = rng.uniform(0.5, 1.5, n).astype(np.float32)
    blip.stream_read(torch.from_numpy(x).cuda(), part)
    torch.cuda.synchronize()
    got = part.cpu().numpy().astype(np.float64).sum()
    want = x.astype(np.float64).sum()
    assert abs(got - want) <= 1e-5 * want


@pytest.mark.parametrize("run_bytes", [4096, 12288, 49152])
def test_runs_read_what_they_name(blip, run_bytes):
    """The scattered form reads exactly the named runs (overlapping runs
    count twice), and skips runs that are misaligned or past the end."""
    n = 1 << 20
    rng = np.random.default_rng(run_bytes)
    x = rng.integers(0, 8, n).astype(np.float32)
    buf = torch.from_numpy(x).cuda()
    nb = n * 4
    good = rng.integers(0, (nb - run_bytes) // 16, 300) * 16
    bad = np.array([-16, 8, nb - run_bytes + 16, nb], dtype=np.int64)
    offs = np.concatenate([good, bad]).astype(np.int64)
    rng.shuffle(offs)
    part = torch.zeros(64, dtype=torch.float32, device="cuda")
    say(f"scattered read: {len(good)} runs of {run_bytes} B and {len(bad)} to skip")
    blip.stream_read_runs(buf, torch.from_numpy(offs).cuda(), run_bytes, part)
    torch.cuda.synchronize()
    w = run_bytes // 4
    want = sum(float(x[o // 4: o // 4 + w].astype(np.float64).sum()) for o in good)
    got = float(part.cpu().numpy().astype(np.float64).sum())
    assert got == want          # integers: every partial below 2^24, exact
