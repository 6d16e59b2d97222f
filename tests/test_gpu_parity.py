"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Error metric per component group c in {val, grad, lap}:
    err_c = max|y - y*| / max|y*|            (normwise over the block)
Bars: FP32 tables <= 1e-5; BF16 / FP16 storage <= 1e-2 against the FP32
master (quantisation included) and <= 1e-5 against the oracle run on the
quantised table (arithmetic alone); FP64-accumulate debug kernel <= 1e-12.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1204_1121_amd import workloads as wl
from tests.gpu_util import (error_report, format_report, quantize_bf16,
                            quantize_f16_scaled, say, to_np)

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
HALF_TOL = 1e-2
SKEW = np.array([[5.0, 0.3, 0.1], [0.2, 4.5, 0.4], [0.1, -0.3, 6.0]])


@pytest.fixture(scope="module")
def blip():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    torch.cuda.init()
    from paper_1204_1121_amd import blip as b
    b.lib()
    return b


def gpu_eval(table, pos, grad=True, **kw):
    p = torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float64)).cuda()
    v, g, l = table.eval(p, grad=grad, **kw)
    torch.cuda.synchronize()
    return {"val": to_np(v), "grad": to_np(g), "lap": to_np(l)}


def check(gpu, ref, tol, label, elem=None):
    """Normwise error <= tol per component group; with ``elem``, also the
    99th percentile of the elementwise error <= elem.  Both are printed."""
    rep = error_report(gpu, ref)
    say(f"  {label}: {format_report(rep)}")
    for k, v in rep.items():
        assert v["norm"] <= tol, (label, k, v)
        if elem is not None:
            assert v["elem_p99"] <= elem, (label, k, v)
    return {k: v["norm"] for k, v in rep.items()}


# ---------------------------------------------------------------------------
# Small cubic cell: 16^3 grid, 8 orbitals, 64 positions


@pytest.fixture(scope="module")
def small(blip):
    spec = wl.spec_small()
    c64 = wl.coefficients(spec, dist="uniform")
    c32 = c64.astype(np.float32)
    rng = np.random.default_rng(wl.SEED_BASE)
    pos = rng.uniform(0.0, 10.0, size=(64, 3))
    t = blip.Table(spec.lattice, spec.n, c32, "f32")
    ref = oracle.evaluate(spec.lattice, spec.n, c32, pos, nthreads=4)
    ref64 = oracle.evaluate(spec.lattice, spec.n, c64, pos, nthreads=4)
    yield spec, c32, pos, t, ref, ref64
    t.free()


def test_small_tiled_and_plain(small):
    spec, c32, pos, t, ref, ref64 = small
    say("small cubic 16^3 L=8, 64 positions")
    check(gpu_eval(t, pos), ref, FP32_TOL, "tiled vs oracle(fp32 table)")
    check(gpu_eval(t, pos), ref64, FP32_TOL, "tiled vs oracle(fp64 master)")
    check(gpu_eval(t, pos, kernel="plain"), ref, FP32_TOL, "plain vs oracle")
    check(gpu_eval(t, pos, kernel="site"), ref, FP32_TOL, "site-parallel vs oracle")


def test_small_fp64_accumulate(small):
    spec, c32, pos, t, ref, _ = small
    say("small cubic, FP64-accumulate kernel")
    for vec in (1, 2, 4):
        check(gpu_eval(t, pos, kernel="f64acc", vec=vec), ref, 1e-12, f"f64acc o={vec}")


def test_small_every_tiling(small):
    spec, c32, pos, t, ref, _ = small
    say("small cubic, every (P, o)")
    base = gpu_eval(t, pos, kernel="tiled", tile_pos=1, vec=4)
    for P in (1, 2, 3, 8, 16, 64):
        for vec in (1, 2, 4):
            y = gpu_eval(t, pos, kernel="tiled", tile_pos=P, vec=vec)
            for k in ("val", "grad", "lap"):
                np.testing.assert_array_equal(y[k], base[k], err_msg=f"P={P} o={vec} {k}")


# ---------------------------------------------------------------------------
# Ragged and general-lattice cases


@pytest.mark.parametrize("L", [1, 13, 300])
def test_ragged_orbitals_and_tiles(blip, L):
    """L not a multiple of the lane vector (scalar store path), several
    chunks with a ragged tail (L=300), npos not a multiple of P."""
    rng = np.random.default_rng(100 + L)
    A = np.diag([7.0, 6.0, 5.0])
    n = (9, 8, 7)
    c = rng.uniform(-1, 1, n + (L,)).astype(np.float32)
    pos = rng.uniform(-10, 20, (77, 3))
    say(f"ragged L={L}, npos=77")
    t = blip.Table(A, n, c, "f32")
    ref = oracle.evaluate(A, n, c, pos, nthreads=4)
    base = None
    for P in (1, 5, 16):
        for vec in (1, 2, 4):
            y = gpu_eval(t, pos, kernel="tiled", tile_pos=P, vec=vec)
            check(y, ref, FP32_TOL, f"P={P} o={vec}")
            if base is None:
                base = y
            for k in y:
                np.testing.assert_array_equal(y[k], base[k])
    check(gpu_eval(t, pos, kernel="plain"), ref, FP32_TOL, "plain")
    check(gpu_eval(t, pos, kernel="site"), ref, FP32_TOL, "site-parallel")
    t.free()


def test_general_lattice(blip):
    """Non-orthogonal cell: full metric with mixed second derivatives."""
    rng = np.random.default_rng(7)
    n = (12, 13, 14)
    L = 37
    c = rng.uniform(-1, 1, n + (L,)).astype(np.float32)
    pos = rng.uniform(-15, 25, (100, 3))
    say("skewed lattice 12x13x14, L=37")
    t = blip.Table(SKEW, n, c, "f32")
    ref = oracle.evaluate(SKEW, n, c, pos, nthreads=4)
    check(gpu_eval(t, pos), ref, FP32_TOL, "tiled")
    check(gpu_eval(t, pos, kernel="plain"), ref, FP32_TOL, "plain")
    check(gpu_eval(t, pos, kernel="site"), ref, FP32_TOL, "site-parallel")
    check(gpu_eval(t, pos, kernel="f64acc", vec=1), ref, 1e-12, "f64acc")
    t.free()


def test_values_only_matches_full(small):
    spec, c32, pos, t, ref, _ = small
    say("values-only kernel")
    full = gpu_eval(t, pos)
    vo = gpu_eval(t, pos, grad=False)
    assert vo["grad"] is None and vo["lap"] is None
    np.testing.assert_array_equal(vo["val"], full["val"])


def test_block_equals_parts(small):
    """Quasi-simultaneous evaluation: each position of a block is evaluated
    independently, so the block result equals single-position calls."""
    spec, c32, pos, t, ref, _ = small
    say("block vs single positions")
    blk = gpu_eval(t, pos)
    for j in (0, 17, 63):
        one = gpu_eval(t, pos[j:j + 1])
        for k in blk:
            np.testing.assert_array_equal(one[k][0], blk[k][j])


def test_edge_positions(blip):
    A = np.diag([16.0, 16.0, 8.0])
    n = (16, 16, 8)
    rng = np.random.default_rng(3)
    c = rng.uniform(-1, 1, n + (12,)).astype(np.float32)
    t = blip.Table(A, n, c, "f32")
    say("edge positions")
    pos = np.array([
        [3.0, 0.0, 7.5], [-0.0, 16.0, -8.0], [-1e-18, 35.25, -0.5],
        [16.0, 16.0, 8.0], [1e300, -1e300, 3.0], [0.5, 0.5, 0.5],
        [np.nan, 1.0, 1.0], [1.0, np.inf, 1.0], [1.0, 1.0, -np.inf],
        [1e-300, -1e-300, 4.0]])
    y = gpu_eval(t, pos)
    ref = oracle.evaluate(A, n, c, pos)
    fin = np.all(np.isfinite(pos), axis=1)
    for k in ("val", "grad", "lap"):
        assert np.all(np.isnan(y[k][~fin])), k
        assert np.all(np.isfinite(y[k][fin])), k
    sub = {k: v[fin] for k, v in y.items()}
    check(sub, {k: v[fin] for k, v in ref.items()}, FP32_TOL, "finite edge rows")
    for kern in ("plain", "site"):
        yp = gpu_eval(t, pos, kernel=kern)
        for k in ("val", "grad", "lap"):
            assert np.all(np.isnan(yp[k][~fin])), (kern, k)
        check({k: v[fin] for k, v in yp.items()}, {k: v[fin] for k, v in ref.items()},
              FP32_TOL, f"{kern} finite edge rows")
    # npos = 0 enqueues nothing and succeeds
    p0 = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    v, g, l = t.eval(p0)
    assert v.shape == (0, 12)
    t.free()


def test_misaligned_pointer_rejected(small, blip):
    """Misaligned pointers are rejected on the host, before any launch."""
    spec, c32, pos, t, ref, _ = small
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")
    out = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    L = blip.lib()
    rc = L.blip_eval(t.handle, ctypes.c_void_p(buf.data_ptr() + 4), 4,
                     ctypes.c_void_p(out.data_ptr()), None, None, None)
    assert rc == -5
    rc = L.blip_eval(t.handle, ctypes.c_void_p(buf.data_ptr()), 4,
                     ctypes.c_void_p(out.data_ptr() + 2), None, None, None)
    assert rc == -5
    # an 8-byte aligned slice of positions is fine (per-walker views)
    p = torch.from_numpy(pos).cuda()
    v, g, l = t.eval(p[1:5])
    torch.cuda.synchronize()
    v2, g2, l2 = t.eval(p[1:5].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(v, v2) and torch.equal(l, l2)
    with pytest.raises(blip.BlipError):
        t.eval(torch.zeros((4, 3), dtype=torch.float64, device="cuda"), kernel="tiled",
               tile_pos=65)
    with pytest.raises(blip.BlipError):
        t.eval(torch.zeros((4, 3), dtype=torch.float64, device="cuda"), kernel="tiled",
               vec=8)


# ---------------------------------------------------------------------------
# TiO2-supercell-shaped table: 72x72x48 grid, 768 real orbitals (764 MB)


@pytest.fixture(scope="module")
def tio2(blip):
    spec = wl.spec_tio2()
    say("generating the 72x72x48 x 768 table")
    c = wl.coefficients(spec)
    t = blip.Table(spec.lattice, spec.n, c, "f32")
    yield spec, c, t
    t.free()


@pytest.mark.parametrize("B", [1, 8, 64, 1536])
def test_tio2_blocks(tio2, B):
    """The C1 block sizes against the oracle: the tiled kernel at the
    default shape and at the launch shape the benchmark runs (the package's
    tuning cache; the same arithmetic per element, so bit for bit the same
    outputs), the plain and the site-parallel kernels."""
    from paper_1204_1121_amd.tuning import TuneCache
    spec, c, t = tio2
    pos = wl.move_block(spec, B, block=0)
    say(f"TiO2 block B={B}")
    ref = oracle.evaluate(spec.lattice, spec.n, c, pos, nthreads=8)
    y = gpu_eval(t, pos)
    check(y, ref, FP32_TOL, "default shape")
    e = TuneCache().get(t, B)
    if e is not None:
        yt = gpu_eval(t, pos, kernel="tiled", tile_pos=e["tile_pos"], vec=e["vec"])
        check(yt, ref, FP32_TOL, f"benchmark shape ({e['tile_pos']}, {e['vec']})")
        for k in ("val", "grad", "lap"):
            np.testing.assert_array_equal(yt[k], y[k], err_msg=f"{k}: shapes differ")
    check(gpu_eval(t, pos, kernel="plain"), ref, FP32_TOL, "plain")
    check(gpu_eval(t, pos, kernel="site"), ref, FP32_TOL, "site-parallel")


def test_tio2_values_only(tio2):
    spec, c, t = tio2
    pos = wl.move_block(spec, 1536, block=1)
    say("TiO2 values only, 1536")
    ref = oracle.evaluate(spec.lattice, spec.n, c, pos, want=("val",), nthreads=8)
    check(gpu_eval(t, pos, grad=False), ref, FP32_TOL, "values")


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_tio2_reduced_precision(blip, tio2, storage):
    spec, c, _ = tio2
    say(f"TiO2 {storage} storage, 1536")
    t = blip.Table(spec.lattice, spec.n, c, storage)
    pos = wl.move_block(spec, 1536, block=2)
    y = gpu_eval(t, pos)
    ys = gpu_eval(t, pos, kernel="site")
    t.free()
    ref = oracle.evaluate(spec.lattice, spec.n, c, pos, nthreads=8)
    check(y, ref, HALF_TOL, f"{storage} vs fp32 master")
    q = quantize_bf16(c) if storage == "bf16" else quantize_f16_scaled(c)
    refq = oracle.evaluate(spec.lattice, spec.n, q, pos, nthreads=8)
    check(y, refq, FP32_TOL, f"{storage} vs oracle on quantised table")
    check(ys, refq, FP32_TOL, f"{storage} site-parallel vs oracle on quantised table")


# ---------------------------------------------------------------------------
# Complex orbitals at a k-point: 384 complex orbitals, c64 / bf16 / f16 pairs


@pytest.fixture(scope="module")
def tio2c(blip):
    spec = wl.spec_tio2_complex()
    say("generating the 72x72x48 x 384 complex table")
    c = wl.coefficients(spec)
    pos = wl.move_block(spec, 1536, block=0)
    ref = oracle.evaluate(spec.lattice, spec.n, c, pos, kvec=spec.kvec, nthreads=8)
    return spec, c, pos, ref


@pytest.mark.parametrize("storage", ["c64", "cbf16", "cf16"])
def test_complex_kpoint(blip, tio2c, storage):
    spec, c, pos, ref = tio2c
    say(f"complex k-point, {storage}")
    t = blip.Table(spec.lattice, spec.n, c, storage, kvec=spec.kvec)
    y = gpu_eval(t, pos)
    yp = gpu_eval(t, pos, kernel="plain")
    ys = gpu_eval(t, pos, kernel="site")
    t.free()
    tol = FP32_TOL if storage == "c64" else HALF_TOL
    check(y, ref, tol, f"{storage} tuned vs c64 master")
    check(yp, ref, tol, f"{storage} plain vs c64 master")
    check(ys, ref, tol, f"{storage} site-parallel vs c64 master")
    if storage != "c64":
        q = quantize_bf16(c) if storage == "cbf16" else quantize_f16_scaled(c)
        refq = oracle.evaluate(spec.lattice, spec.n, q, pos, kvec=spec.kvec, nthreads=8)
        check(y, refq, FP32_TOL, f"{storage} vs oracle on quantised table")


def test_complex_gamma_and_bloch_relation(blip):
    """Complex table at Gamma (no phase), and psi(r+T) = e^{ik.T} psi(r)."""
    rng = np.random.default_rng(21)
    A = np.diag([6.0, 6.0, 4.0])
    n = (12, 12, 8)
    c = (rng.standard_normal(n + (10,)) + 1j * rng.standard_normal(n + (10,))).astype(np.complex64)
    pos = rng.uniform(0, 4, (40, 3))
    say("complex gamma + Bloch relation")
    tg = blip.Table(A, n, c, "c64")
    check(gpu_eval(tg, pos), oracle.evaluate(A, n, c, pos), FP32_TOL, "gamma")
    tg.free()
    k = np.array([np.pi / 6, np.pi / 6, np.pi / 4])
    tk = blip.Table(A, n, c, "c64", kvec=k)
    y0 = gpu_eval(tk, pos)
    T = np.array([1.0, -2.0, 3.0]) @ A
    y1 = gpu_eval(tk, pos + T)
    tk.free()
    ph = np.exp(1j * (k @ T))
    for key in y0:
        ref = ph * y0[key]
        assert np.max(np.abs(y1[key] - ref)) <= FP32_TOL * np.max(np.abs(ref)), key


def test_values_only_complex_and_skewed(blip):
    """Values-only kernels on a complex k-point table in a skewed cell, in
    every storage dtype: equal to the values of the full kernel."""
    rng = np.random.default_rng(41)
    n = (10, 11, 12)
    c = (rng.standard_normal(n + (20,)) + 1j * rng.standard_normal(n + (20,))).astype(np.complex64)
    k = np.array([0.2, -0.3, 0.15])
    pos = rng.uniform(-8, 12, (50, 3))
    ref = oracle.evaluate(SKEW, n, c, pos, kvec=k, nthreads=4)
    say("values-only, complex k-point, skewed cell")
    for storage in ("c64", "cbf16", "cf16"):
        t = blip.Table(SKEW, n, c, storage, kvec=k)
        full = gpu_eval(t, pos)
        vo = gpu_eval(t, pos, grad=False)
        np.testing.assert_array_equal(vo["val"], full["val"])
        tol = FP32_TOL if storage == "c64" else HALF_TOL
        check(full, ref, tol, f"{storage} full")
        pl = gpu_eval(t, pos, kernel="plain", grad=False)
        check({"val": pl["val"]}, {"val": ref["val"]}, tol, f"{storage} plain values")
        sv = gpu_eval(t, pos, kernel="site", grad=False)
        sf = gpu_eval(t, pos, kernel="site")
        np.testing.assert_array_equal(sv["val"], sf["val"])
        check(sf, ref, tol, f"{storage} site-parallel full")
        t.free()


def test_concurrent_streams_share_a_table(small):
    """Evaluations on two streams at once read the same immutable table; each
    result equals the one computed alone."""
    spec, c32, pos, t, ref, _ = small
    rng = np.random.default_rng(5)
    p1 = torch.from_numpy(rng.uniform(0, 10, (3000, 3))).cuda()
    p2 = torch.from_numpy(rng.uniform(0, 10, (2000, 3))).cuda()
    say("two streams on one table")
    a1 = t.eval(p1)
    a2 = t.eval(p2)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    o1 = t.alloc_outputs(3000)
    o2 = t.alloc_outputs(2000)
    for _ in range(3):
        with torch.cuda.stream(s1):
            t.eval(p1, out=o1, stream=s1)
        with torch.cuda.stream(s2):
            t.eval(p2, out=o2, stream=s2)
    torch.cuda.synchronize()
    for x, y in zip(o1, a1):
        assert torch.equal(x, y)
    for x, y in zip(o2, a2):
        assert torch.equal(x, y)
