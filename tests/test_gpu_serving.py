"""The serving loop on the GPU: three resident systems, Poisson arrivals,
continuous batching; every request's result in the mix equals the same
request evaluated alone, bit for bit, and agrees with the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_1121_amd import workloads as wl
from paper_1204_1121_amd.serve import GpuBackend, Server, ServeRequest
from tests.gpu_util import group_errors, say, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def systems():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    from paper_1204_1121_amd import blip
    specs = [wl.TableSpec("a", np.diag([6.0, 6.0, 4.0]), (24, 24, 16), 256, seed=11),
             wl.TableSpec("b", np.diag([4.0, 4.0, 4.0]), (16, 16, 16), 64, seed=12),
             wl.TableSpec("c", np.diag([5.0, 5.0, 5.0]), (20, 20, 20), 96, seed=13)]
    coefs = [wl.coefficients(s) for s in specs]
    tables = [blip.Table(s.lattice, s.n, c, "f32") for s, c in zip(specs, coefs)]
    yield specs, coefs, tables
    for t in tables:
        t.free()


@pytest.mark.parametrize("batched,threshold", [(True, 4096), (True, 1), (False, 0)],
                         ids=["batched", "batched-always-sorted", "unbatched-plain"])
def test_serving_mix_equals_alone(systems, batched, threshold):
    specs, coefs, tables = systems
    be = GpuBackend(tables, capacity=4096, max_requests=64, batched=batched,
                    kernel="auto" if batched else "plain", sort_threshold=threshold)
    sv = Server(be, budget_bytes=64 << 20)
    reqs = wl.serving_requests(3, 300, rate=20000.0, specs=specs, seed=1, max_pos=600)
    sreqs = [ServeRequest(r.rid, r.system, r.pos, arrival=r.arrival, keep=True) for r in reqs]
    say(f"serving {len(sreqs)} requests, batched={batched}")
    st = sv.run(sreqs)
    say(f"  {st}")
    assert st["done"] == len(sreqs)
    if batched:
        assert st["launches"] < len(sreqs)        # requests were packed together
    for r in sreqs[::7]:
        t = tables[r.system]
        p = torch.from_numpy(r.pos).cuda()
        alone = t.eval(p, kernel="auto" if batched else "plain")
        torch.cuda.synchronize()
        for k, v in zip(("val", "grad", "lap"), alone):
            np.testing.assert_array_equal(r.result[k], to_np(v), err_msg=f"rid {r.rid} {k}")
    for r in sreqs[::37]:
        s = specs[r.system]
        ref = oracle.evaluate(s.lattice, s.n, coefs[r.system], r.pos)
        e = group_errors(r.result, ref)
        assert max(e.values()) <= 1e-5, e
    be.close()
