"""Fused acceptance ratios (blip_eval_ratio) against the oracle's ratio, and
against an FP64 dot of blip_eval's own FP32 orbitals with the inverse."""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_1121_amd import workloads as wl
from tests.gpu_util import say, to_np

pytestmark = pytest.mark.gpu

SKEW = np.array([[5.0, 0.3, 0.1], [0.2, 4.5, 0.4], [0.1, -0.3, 6.0]])


@pytest.fixture(scope="module")
def blip():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    from paper_1204_1121_amd import blip as b
    b.lib()
    return b


def setup(A, n, c, nel, seed, sigma=0.4):
    rng = np.random.default_rng(seed)
    R = rng.uniform(0, 1, (nel, 3)) @ A
    D = oracle.evaluate(A, n, c, R, want=("val",), nthreads=8)["val"]
    Dinv = np.linalg.inv(D)
    moves = R + rng.normal(0, sigma, R.shape)
    return R, Dinv.T.copy(), moves


def check_ratio(got, ref, vals, inv_rows, rows, tol, label):
    """|y - y*| <= tol * sum_l |y_l| |Dinv[l, c]| per position (the sum's
    own scale), for ratio, gradient and Laplacian."""
    w = np.abs(inv_rows[rows])
    for key, part in (("ratio", "val"), ("grad", "grad"), ("lap", "lap")):
        if got.get(key) is None:
            continue
        if key == "grad":
            scale = np.einsum("jcl,jl->jc", np.abs(vals[part]), w)
        else:
            scale = np.einsum("jl,jl->j", np.abs(vals[part]), w)
        err = np.max(np.abs(got[key] - ref[key]) / scale)
        say(f"  {label} {key}: max error / scale = {err:.2e}")
        assert err <= tol, (label, key, err)


def test_small_skewed_ratio(blip):
    rng = np.random.default_rng(3)
    n = (9, 10, 11)
    L = 37
    c = rng.uniform(-1, 1, n + (L,)).astype(np.float32)
    R, inv_rows, moves = setup(SKEW, n, c, L, 1)
    t = blip.Table(SKEW, n, c, "f32")
    say("ratio: skewed cell, L=37")
    ref = oracle.ratio(SKEW, n, c, moves, inv_rows, np.arange(L), nthreads=4)
    vals = oracle.evaluate(SKEW, n, c, moves, nthreads=4)
    p = torch.from_numpy(moves).cuda()
    inv = torch.from_numpy(inv_rows).cuda()
    r, g, l = t.ratio(p, inv)
    torch.cuda.synchronize()
    got = {"ratio": to_np(r), "grad": to_np(g), "lap": to_np(l)}
    check_ratio(got, ref, vals, inv_rows, np.arange(L), 1e-5, "vs oracle")
    # the epilogue itself: FP64 dot of the kernel's own FP32 orbitals
    v, gg, ll = t.eval(p)
    torch.cuda.synchronize()
    mine = {"ratio": np.einsum("jl,jl->j", to_np(v).astype(np.float64), inv_rows),
            "grad": np.einsum("jcl,jl->jc", to_np(gg).astype(np.float64), inv_rows),
            "lap": np.einsum("jl,jl->j", to_np(ll).astype(np.float64), inv_rows)}
    check_ratio(got, mine, vals, inv_rows, np.arange(L), 1e-13, "vs dot of blip_eval")
    # values-only kernel and a row map (reversed electrons)
    r2, g2, l2 = t.ratio(p, inv, grad=False)
    torch.cuda.synchronize()
    assert g2 is None and torch.equal(r2, r)
    rows = torch.arange(L - 1, -1, -1, dtype=torch.int64, device="cuda")
    r3, _, _ = t.ratio(p, inv, row_of=rows)
    torch.cuda.synchronize()
    ref3 = oracle.ratio(SKEW, n, c, moves, inv_rows, np.arange(L - 1, -1, -1))
    check_ratio({"ratio": to_np(r3)}, ref3, vals, inv_rows, np.arange(L - 1, -1, -1), 1e-5,
                "row map")
    t.free()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_tio2_one_spin_ratios(blip, storage):
    """768 electrons of one spin on the 768-orbital table: D from the old
    configuration, its inverse, and a quasi-simultaneous move of every
    electron."""
    spec = wl.spec_tio2()
    say(f"ratio: 72x72x48 x 768 table, 768 moves, {storage}")
    c = wl.coefficients(spec)
    R, inv_rows, moves = setup(spec.lattice, spec.n, c, 768, 7)
    t = blip.Table(spec.lattice, spec.n, c, storage)
    p = torch.from_numpy(moves).cuda()
    r, g, l = t.ratio(p, torch.from_numpy(inv_rows).cuda())
    torch.cuda.synchronize()
    got = {"ratio": to_np(r), "grad": to_np(g), "lap": to_np(l)}
    ref = oracle.ratio(spec.lattice, spec.n, c, moves, inv_rows, np.arange(768), nthreads=8)
    vals = oracle.evaluate(spec.lattice, spec.n, c, moves, nthreads=8)
    check_ratio(got, ref, vals, inv_rows, np.arange(768), 1e-5 if storage == "f32" else 1e-2,
                storage)
    t.free()


def test_complex_table_rejected(blip):
    c = np.zeros((4, 4, 4, 2), dtype=np.complex64)
    t = blip.Table(np.eye(3) * 4.0, (4, 4, 4), c, "c64")
    p = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    inv = torch.zeros((2, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(blip.BlipError) as ei:
        t.ratio(p, inv)
    assert ei.value.status == -4
    t.free()


def test_batched_ratio_equals_per_walker(blip):
    """Walkers with their own inverses and ragged move blocks in one sorted
    persistent launch: equal bit for bit to blip_eval_ratio per walker."""
    rng = np.random.default_rng(11)
    n = (12, 11, 10)
    L = 37
    c = rng.uniform(-1, 1, n + (L,)).astype(np.float32)
    t = blip.Table(SKEW, n, c, "f32")
    nwalk = 8
    invs, blocks, rows = [], [], []
    for w in range(nwalk):
        R, inv_rows, moves = setup(SKEW, n, c, L, 100 + w)
        k = int(rng.integers(1, L + 1))
        who = rng.choice(L, k, replace=False)          # electrons this walker moves
        invs.append(inv_rows)
        blocks.append(moves[who])
        rows.append(w * L + who)
    pos = np.concatenate(blocks)
    off = np.zeros(nwalk + 1, dtype=np.int64)
    off[1:] = np.cumsum([b.shape[0] for b in blocks])
    allinv = torch.from_numpy(np.concatenate(invs)).cuda()
    row_of = torch.from_numpy(np.concatenate(rows).astype(np.int64)).cuda()
    p = torch.from_numpy(pos).cuda()
    say(f"batched ratio: {nwalk} walkers, {pos.shape[0]} moves")
    rb, gb, lb = t.ratio_batched(p, torch.from_numpy(off).cuda(), allinv, row_of=row_of)
    torch.cuda.synchronize()
    for w in range(nwalk):
        a, b = int(off[w]), int(off[w + 1])
        r, g, l = t.ratio(p[a:b].contiguous(), allinv, row_of=row_of[a:b].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(rb[a:b], r) and torch.equal(gb[a:b], g) and torch.equal(lb[a:b], l)
    ref = oracle.ratio(SKEW, n, c, pos, np.concatenate(invs), np.concatenate(rows))
    vals = oracle.evaluate(SKEW, n, c, pos)
    check_ratio({"ratio": to_np(rb), "grad": to_np(gb), "lap": to_np(lb)}, ref, vals,
                np.concatenate(invs), np.concatenate(rows), 1e-5, "batched vs oracle")
    t.free()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_ratio_values_one_pass(blip, storage):
    """blip_eval_ratio_values: the ratios equal blip_eval_ratio's and the
    values equal values-only blip_eval's, bit for bit, with aligned outputs
    (whole-vector stores) and with a value array offset by one float."""
    rng = np.random.default_rng(11)
    n = (9, 10, 11)
    L = 64
    c = rng.uniform(-1, 1, n + (L,)).astype(np.float32)
    R, inv_rows, moves = setup(SKEW, n, c, L, 2)
    t = blip.Table(SKEW, n, c, storage)
    p = torch.from_numpy(moves).cuda()
    inv = torch.from_numpy(inv_rows).cuda()
    want_r = to_np(t.ratio(p, inv, grad=False)[0])
    want_v = to_np(t.eval(p, grad=False)[0])
    r, v = t.ratio_values(p, inv)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(r), want_r)
    np.testing.assert_array_equal(to_np(v), want_v)
    buf = torch.full((L * L + 1,), 7.0, dtype=torch.float32, device="cuda")
    v_off = buf[1:].view(L, L)                       # 4-byte aligned, not 16
    r2 = torch.empty(L, dtype=torch.float64, device="cuda")
    t.ratio_values(p, inv, out=(r2, v_off))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(r2), want_r)
    np.testing.assert_array_equal(to_np(v_off), want_v)
    assert to_np(buf)[0] == 7.0
    # the full form: ratios with gradient and Laplacian, the values and the
    # Laplacian rows, bit for bit those of blip_eval_ratio and blip_eval
    wr, wg, wl = (to_np(x) for x in t.ratio(p, inv, grad=True))
    _, _, wlap = t.eval(p, grad=True)
    r3, g3, l3, v3, lap3 = t.ratio_values(p, inv, lap=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(r3), wr)
    np.testing.assert_array_equal(to_np(g3), wg)
    np.testing.assert_array_equal(to_np(l3), wl)
    np.testing.assert_array_equal(to_np(v3), want_v)
    np.testing.assert_array_equal(to_np(lap3), to_np(wlap))
    t.free()


@pytest.mark.parametrize("o", [1, 2])
def test_ratio_values_batched(blip, o):
    """blip_eval_ratio_values_batched: ragged walker blocks (one of them
    empty) in one sorted persistent launch.  Values and Laplacian rows equal
    blip_eval's bit for bit; with the block launch held to the same orbitals
    per lane, the ratios equal blip_eval_ratio_values' bit for bit; rows past
    offsets[nw] are not written; and the ratios agree with the oracle."""
    rng = np.random.default_rng(29)
    n = (12, 11, 10)
    L = 100
    c = rng.uniform(-1, 1, n + (L,)).astype(np.float32)
    t = blip.Table(SKEW, n, c, "f32")
    nwalk = 6
    invs, blocks, rows = [], [], []
    for w in range(nwalk):
        R, inv_rows, moves = setup(SKEW, n, c, L, 300 + w)
        k = 0 if w == 2 else int(rng.integers(1, L + 1))
        who = rng.choice(L, k, replace=False)
        invs.append(inv_rows)
        blocks.append(moves[who])
        rows.append(w * L + who)
    pos = np.concatenate(blocks)
    total = pos.shape[0]
    cap = total + 5
    off = np.zeros(nwalk + 1, dtype=np.int64)
    off[1:] = np.cumsum([b.shape[0] for b in blocks])
    allinv_np = np.concatenate(invs)
    allrows = np.concatenate(rows).astype(np.int64)
    allinv = torch.from_numpy(allinv_np).cuda()
    row_of = torch.from_numpy(np.concatenate([allrows, np.zeros(5, np.int64)])).cuda()
    p = torch.from_numpy(np.concatenate([pos, np.zeros((5, 3))])).cuda()
    offs = torch.from_numpy(off).cuda()
    t.set_shape(total, 8, o, ratio=True)
    t.set_shape(cap, 8, o, batched=True, ratio=True)
    say(f"batched ratio values: {nwalk} walkers, {total} moves, L={L}, o={o}")
    out = (torch.full((cap,), 7.0, dtype=torch.float64, device="cuda"),
           torch.full((cap, 3), 7.0, dtype=torch.float64, device="cuda"),
           torch.full((cap,), 7.0, dtype=torch.float64, device="cuda"),
           torch.full((cap, L), 7.0, dtype=torch.float32, device="cuda"),
           torch.full((cap, L), 7.0, dtype=torch.float32, device="cuda"))
    r, g, lr, v, lap = t.ratio_values_batched(p, offs, allinv, row_of=row_of, out=out, lap=True)
    rb, gb, lrb, vb, lapb = t.ratio_values(p[:total], allinv, row_of=row_of[:total], lap=True)
    ev, _, elap = t.eval(p[:total])
    torch.cuda.synchronize()
    for x in out:
        assert bool((x[total:] == 7.0).all()), "a row past offsets[nw] was written"
    assert torch.equal(v[:total], ev) and torch.equal(lap[:total], elap)
    assert torch.equal(r[:total], rb) and torch.equal(g[:total], gb)
    assert torch.equal(lr[:total], lrb)
    # the values-only form gives the same ratios and values
    r2, v2 = t.ratio_values_batched(p, offs, allinv, row_of=row_of, capacity=cap)
    torch.cuda.synchronize()
    assert torch.equal(r2[:total], r[:total]) and torch.equal(v2[:total], v[:total])
    ref = oracle.ratio(SKEW, n, c, pos, allinv_np, allrows)
    vals = oracle.evaluate(SKEW, n, c, pos)
    check_ratio({"ratio": to_np(r[:total]), "grad": to_np(g[:total]), "lap": to_np(lr[:total])},
                ref, vals, allinv_np, allrows, 1e-5, "batched values vs oracle")
    t.free()


def test_ratio_at_the_orbital_limit(blip):
    """The largest table the ratio epilogue takes in FP32 (4,096 orbitals: 16
    chunks of 64 lanes x 4 elements, 16 KB rows), against the oracle and the
    FP64 dot of blip_eval's own orbitals; one orbital more is refused."""
    rng = np.random.default_rng(41)
    A = np.diag([4.0, 4.5, 5.0])
    n = (8, 8, 8)
    L = 4096
    c = rng.uniform(-1, 1, n + (L,)).astype(np.float32)
    t = blip.Table(A, n, c, "f32")
    try:
        npos = 24
        moves = rng.uniform(-2, 7, (npos, 3))
        inv_rows = rng.normal(0, 1, (npos, L))
        say(f"ratio at L={L}")
        p = torch.from_numpy(moves).cuda()
        inv = torch.from_numpy(inv_rows).cuda()
        r, g, l = t.ratio(p, inv)
        v, gg, ll = t.eval(p)
        torch.cuda.synchronize()
        got = {"ratio": to_np(r), "grad": to_np(g), "lap": to_np(l)}
        vals = oracle.evaluate(A, n, c, moves, nthreads=8)
        ref = oracle.ratio(A, n, c, moves, inv_rows, np.arange(npos), nthreads=8)
        check_ratio(got, ref, vals, inv_rows, np.arange(npos), 1e-5, "vs oracle")
        mine = {"ratio": np.einsum("jl,jl->j", to_np(v).astype(np.float64), inv_rows),
                "grad": np.einsum("jcl,jl->jc", to_np(gg).astype(np.float64), inv_rows),
                "lap": np.einsum("jl,jl->j", to_np(ll).astype(np.float64), inv_rows)}
        check_ratio(got, mine, vals, inv_rows, np.arange(npos), 1e-13, "vs dot of blip_eval")
        for k, a in (("val", v), ("grad", gg), ("lap", ll)):
            err = np.max(np.abs(to_np(a) - vals[k])) / np.max(np.abs(vals[k]))
            say(f"  blip_eval {k} at L={L}: {err:.2e}")
            assert err <= 1e-5
    finally:
        t.free()
    c2 = rng.uniform(-1, 1, n + (L + 1,)).astype(np.float32)
    t2 = blip.Table(A, n, c2, "f32")
    try:
        inv2 = torch.zeros((4, L + 1), dtype=torch.float64, device="cuda")
        with pytest.raises(blip.BlipError, match="too large"):
            t2.ratio(torch.zeros((4, 3), dtype=torch.float64, device="cuda"), inv2)
    finally:
        t2.free()
