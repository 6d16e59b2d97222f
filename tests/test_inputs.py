"""Seeded input generators and the benchmark's distinct-row byte counter (CPU)."""
import numpy as np

import bench
import oracle
from paper_1204_1121_amd import workloads as wl


def test_generators_are_deterministic():
    s = wl.spec_small()
    a = wl.coefficients(s, dist="uniform")
    b = wl.coefficients(s, dist="uniform")
    assert a.dtype == np.float64 and a.shape == (16, 16, 16, 8)
    np.testing.assert_array_equal(a, b)
    assert np.all(np.abs(a) <= 1.0)
    p1 = wl.move_block(wl.spec_tio2(), 64, block=3)
    p2 = wl.move_block(wl.spec_tio2(), 64, block=3)
    p3 = wl.move_block(wl.spec_tio2(), 64, block=4)
    np.testing.assert_array_equal(p1, p2)
    assert not np.array_equal(p1, p3)
    assert p1.shape == (64, 3) and p1.dtype == np.float64


def test_normal_table_shape_and_scale():
    s = wl.TableSpec("t", np.diag([4.0, 4.0, 4.0]), (16, 16, 16), 32)
    c = wl.coefficients(s)
    assert c.dtype == np.float32 and c.shape == (16, 16, 16, 32)
    assert abs(float(c.std()) * np.sqrt(s.sites) - 1.0) < 0.02
    sc = wl.TableSpec("tc", np.diag([4.0, 4.0, 4.0]), (16, 16, 16), 16, complex_=True)
    cc = wl.coefficients(sc)
    assert cc.dtype == np.complex64
    assert abs(float(cc.real.std()) * np.sqrt(sc.sites) - 1.0) < 0.03
    assert abs(float(cc.imag.std()) * np.sqrt(sc.sites) - 1.0) < 0.03


def test_move_blocks_are_displaced_not_wrapped():
    s = wl.spec_tio2()
    p = wl.move_block(s, 20000, block=0)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    assert np.all(lo < 0.0) and np.all(hi > np.diag(s.lattice))


def test_walker_batch_offsets():
    s = wl.spec_tio2()
    b = wl.walker_batch(s, nwalkers=512, max_block=256)
    assert b.offsets[0] == 0 and b.offsets[-1] == b.pos.shape[0]
    assert np.all(np.diff(b.offsets) >= 1) and np.all(np.diff(b.offsets) <= 256)
    assert 40000 < b.pos.shape[0] < 92000


def test_serving_requests():
    specs = wl.spec_serving()
    r = wl.serving_requests(3, 500, rate=1000.0, specs=specs)
    assert len(r) == 500
    t = np.array([q.arrival for q in r])
    assert np.all(np.diff(t) > 0)
    k = np.array([q.pos.shape[0] for q in r])
    assert k.min() >= 1 and k.max() <= 1536
    assert {q.system for q in r} == {0, 1, 2}


def test_distinct_row_counter_matches_brute_force():
    s = wl.spec_tio2()
    pos = wl.move_block(s, 300, block=7)
    rows = set()
    for r in pos:
        i0, f, ok = oracle.wrap(s.lattice, s.n, r)
        for a in range(-1, 3):
            for b in range(-1, 3):
                for c in range(-1, 3):
                    rows.add((((i0[0] + a) % 72) * 72 + (i0[1] + b) % 72) * 48 + (i0[2] + c) % 48)
    assert bench.distinct_rows(s.lattice, s.n, pos) == len(rows)
