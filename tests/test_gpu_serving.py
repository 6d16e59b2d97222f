"""The serving loop on the GPU: three resident systems, Poisson arrivals,
continuous batching; every request's result in the mix equals the same
request evaluated alone, bit for bit, and agrees with the FP64 oracle.

Each moved electron is an independent evaluation against its system's table
(Eq. (11.12.23.1)), so packing requests into one launch changes no result.
The small stand-in tables exercise the scheduler's paths cheaply; the
serving workload's own three tables (the 72x72x48 x 768 table, 48^3 x 256 and
96x96x64 x 1,024, 3.3 GB resident) are checked on a sample of requests."""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_1121_amd import workloads as wl
from paper_1204_1121_amd.serve import GpuBackend, Server, ServeRequest
from tests.gpu_util import error_report, format_report, group_errors, say, to_np

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


def test_serving_workload_tables():
    """The serving workload's three resident tables, served a burst of 300
    requests and then a sparse Poisson stream of 300.  Every fifth request keeps its result: each equals the same
    request evaluated alone, bit for bit; one request in fifty is compared
    with the FP64 oracle, normwise <= 1e-5 per component group, with the
    elementwise 99th percentile reported.  Both launch forms (the sorted
    batched plan and the direct block launch) must have run."""
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    from paper_1204_1121_amd import blip
    specs = wl.spec_serving()
    coefs, tables = [], []
    for sp in specs:
        say(f"loading serving table {sp.name}")
        c = wl.coefficients(sp)
        coefs.append(c)
        tables.append(blip.Table(sp.lattice, sp.n, c, "f32"))
    try:
        be = GpuBackend(tables, capacity=16384, max_requests=512, batched=True)
        sreqs = []
        # a burst (all requests at once: large packs, the sorted plan) and a
        # sparse Poisson stream (requests mostly alone: the direct launch)
        for rate, seed in ((1e9, 7), (2000.0, 8)):
            reqs = wl.serving_requests(3, 300, rate=rate, specs=specs, seed=seed)
            part = [ServeRequest(r.rid + len(sreqs), r.system, r.pos, arrival=r.arrival,
                                 keep=(r.rid % 5 == 0)) for r in reqs]
            say(f"serving {len(part)} requests at {rate:.0f} req/s on the three workload tables")
            sv = Server(be, budget_bytes=2 << 30)
            st = sv.run(part)
            say(f"  {st}")
            assert st["done"] == len(part)
            sreqs += part
        say(f"  sorted launches {be.sorted_launches}, direct {be.direct_launches}")
        assert be.sorted_launches > 0 and be.direct_launches > 0
        kept = [r for r in sreqs if r.keep]
        for r in kept:
            p = torch.from_numpy(r.pos).cuda()
            alone = tables[r.system].eval(p)
            torch.cuda.synchronize()
            for k, v in zip(("val", "grad", "lap"), alone):
                np.testing.assert_array_equal(r.result[k], to_np(v),
                                              err_msg=f"rid {r.rid} system {r.system} {k}")
        for r in sreqs[::50]:
            sp = specs[r.system]
            ref = oracle.evaluate(sp.lattice, sp.n, coefs[r.system], r.pos, nthreads=16)
            rep = error_report(r.result, ref)
            say(f"  rid {r.rid} system {sp.name} npos {r.npos}: {format_report(rep)}")
            for k, v in rep.items():
                assert v["norm"] <= 1e-5, (r.rid, k, v)
        be.close()
    finally:
        for t in tables:
            t.free()


def test_submit_paths_and_errors(systems):
    """blip_submit directly: from pageable and from pinned host memory, the
    direct launch equals blip_eval bit for bit and the event completes; a
    plan given buffers other than its own, or the wrong number of offsets,
    is refused before anything is enqueued."""
    import ctypes
    from paper_1204_1121_amd import blip
    specs, coefs, tables = systems
    t = tables[0]
    rng = np.random.default_rng(21)
    pos = rng.uniform(0, 6, (300, 3))
    L = blip.lib()
    dev_pos = torch.zeros((512, 3), dtype=torch.float64, device="cuda")
    out = t.alloc_outputs(512)
    st = torch.cuda.Stream()
    ev = torch.cuda.Event()
    ev.record(st)
    ref = t.eval(torch.from_numpy(pos).cuda())
    torch.cuda.synchronize()
    pinned = torch.from_numpy(pos).pin_memory()
    for label, host in (("pageable", np.ascontiguousarray(pos)), ("pinned", pinned)):
        say(f"blip_submit from {label} host memory")
        for x in out:
            x.zero_()
        torch.cuda.synchronize()          # the zeros land before the submit's stream runs
        hp = host.ctypes.data if isinstance(host, np.ndarray) else host.data_ptr()
        rc = L.blip_submit(t.handle, None, None, ctypes.c_void_p(hp), 300,
                           ctypes.c_void_p(dev_pos.data_ptr()), None, 0, None,
                           *[ctypes.c_void_p(x.data_ptr()) for x in out],
                           ctypes.c_void_p(st.cuda_stream), ctypes.c_void_p(ev.cuda_event))
        assert rc == 0, L.blip_last_error()
        ev.synchronize()
        assert ev.query()
        for k, a, b in zip(("val", "grad", "lap"), out, ref):
            np.testing.assert_array_equal(to_np(a[:300]), to_np(b), err_msg=f"{label} {k}")
    say("blip_submit argument errors")
    off = torch.zeros(5, dtype=torch.int64, device="cuda")
    ws = t.workspace(512)
    plan = t.plan(dev_pos, off, out, ws, capacity=512)
    other = torch.zeros((512, 3), dtype=torch.float64, device="cuda")
    hoff = np.array([0, 100, 200, 300, 300], dtype=np.int64)
    hp = pinned.data_ptr()
    rc = L.blip_submit(t.handle, plan._h, None, ctypes.c_void_p(hp), 300,
                       ctypes.c_void_p(other.data_ptr()), ctypes.c_void_p(hoff.ctypes.data), 5,
                       ctypes.c_void_p(off.data_ptr()), None, None, None,
                       ctypes.c_void_p(st.cuda_stream), None)
    assert rc == -1 and b"captured buffers" in L.blip_last_error()
    rc = L.blip_submit(t.handle, plan._h, None, ctypes.c_void_p(hp), 300,
                       ctypes.c_void_p(dev_pos.data_ptr()), ctypes.c_void_p(hoff.ctypes.data), 4,
                       ctypes.c_void_p(off.data_ptr()), None, None, None,
                       ctypes.c_void_p(st.cuda_stream), None)
    assert rc == -1 and b"offsets" in L.blip_last_error()
    say("blip_submit through the plan")
    rc = L.blip_submit(t.handle, plan._h, None, ctypes.c_void_p(hp), 300,
                       ctypes.c_void_p(dev_pos.data_ptr()), ctypes.c_void_p(hoff.ctypes.data), 5,
                       ctypes.c_void_p(off.data_ptr()), None, None, None,
                       ctypes.c_void_p(st.cuda_stream), ctypes.c_void_p(ev.cuda_event))
    assert rc == 0, L.blip_last_error()
    ev.synchronize()
    for k, a, b in zip(("val", "grad", "lap"), out, ref):
        np.testing.assert_array_equal(to_np(a[:300]), to_np(b), err_msg=f"plan {k}")
    plan.free()
