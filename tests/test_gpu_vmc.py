"""Quasi-simultaneous and particle-by-particle Monte Carlo steps on
the GPU (paper_1204_1121_amd/vmc.py) against the FP64 oracle (oracle/vmc.py)
with the same random numbers.

Both sides take the same accept decisions unless a uniform lies within
rounding of ratio^2; the test asserts that no decision is that close, so the
positions must then agree bit for bit (the trial positions are the same FP64
sums).  The GPU's orbital rows are FP32, so its inverses and energies differ
from the oracle's by the FP32 rounding of the rows amplified by the
condition number: bar 64 * cond * 2^-24 relative to max |B| (and for the
kinetic energy, relative to the sum of |lap ratio| terms)."""
import zlib

import numpy as np
import pytest
import torch

from oracle import vmc as ovmc
from tests.gpu_util import say, to_np

pytestmark = pytest.mark.gpu

A = np.array([[6.0, 0.3, 0.0], [0.2, 5.0, 0.4], [0.0, -0.3, 5.5]])
NG = (12, 11, 10)
L = 8
W = 3
TIE = 1e-5


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import vmc
    rng = np.random.default_rng(zlib.crc32(b"gpu-vmc"))
    coef = rng.uniform(-1, 1, NG + (L,)).astype(np.float32)
    t = blip.Table(A, NG, coef, "f32")
    pos = rng.uniform(0, 1, (W, 2 * L, 3)) @ A
    inv = np.stack([np.stack([np.linalg.inv(D).T for D in ovmc.slater_matrices(A, NG, coef, p)])
                    for p in pos])
    yield blip, vmc, t, coef, pos, inv, rng
    t.free()


def cond_bar(coef, pos_w):
    D = ovmc.slater_matrices(A, NG, coef, pos_w)
    return 64 * max(np.linalg.cond(D[0]), np.linalg.cond(D[1])) * 2.0 ** -24


def lap_scale(coef, pos_w, inv_w):
    o = ovmc.evaluate(A, NG, coef, pos_w, want=("val", "grad", "lap"))
    return 0.5 * (np.abs(o["lap"][:L] * inv_w[0]).sum() + np.abs(o["lap"][L:] * inv_w[1]).sum())


@pytest.mark.parametrize("sort_moves", [False, True])
def test_qs_steps_match_oracle(setup, sort_moves):
    blip, vmc, t, coef, pos, inv, rng = setup
    wk = vmc.Walkers(t, torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(inv.copy()).cuda(),
                     sort_moves=sort_moves)
    assert wk.sorted == sort_moves
    cur_pos, cur_inv = pos.copy(), inv.copy()
    for step in range(3):
        eta = rng.normal(0, 0.5, pos.shape)
        uni = rng.uniform(0, 1, (W, 2 * L))
        cnt, e = wk.step(torch.from_numpy(eta).cuda(), torch.from_numpy(uni).cuda())
        torch.cuda.synchronize()
        g_pos, g_inv, g_e = to_np(wk.pos), to_np(wk.inv).reshape(W, 2, L, L), to_np(e)
        g_cnt = to_np(cnt).reshape(W, 2)
        for w in range(W):
            npos, ninv, acc, ratio, _, ek = ovmc.qs_step(A, NG, coef, cur_pos[w], cur_inv[w],
                                                          eta[w], uni[w])
            assert np.min(np.abs(uni[w] - ratio * ratio)) > TIE, "a decision is within rounding"
            assert [acc[:L].sum(), acc[L:].sum()] == list(g_cnt[w]), (step, w)
            np.testing.assert_array_equal(g_pos[w], npos, err_msg=f"step {step} walker {w}")
            bar = cond_bar(coef, npos)
            eb = np.abs(g_inv[w] - ninv).max() / np.abs(ninv).max()
            ee = abs(g_e[w] - ek) / lap_scale(coef, npos, ninv)
            say(f"step {step} walker {w}: accepted {g_cnt[w].tolist()}, inverse err {eb:.1e}, "
                f"energy err {ee:.1e} (bar {bar:.1e})")
            assert eb <= bar and ee <= bar
            cur_pos[w], cur_inv[w] = npos, ninv


def test_pbp_sweep_matches_oracle(setup):
    blip, vmc, t, coef, pos, inv, rng = setup
    wk = vmc.Walkers(t, torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(inv.copy()).cuda())
    eta = rng.normal(0, 0.5, pos.shape)
    uni = rng.uniform(0, 1, (W, 2 * L))
    e = wk.pbp_sweep(torch.from_numpy(eta).cuda(), torch.from_numpy(uni).cuda())
    torch.cuda.synchronize()
    g_pos, g_inv, g_e = to_np(wk.pos), to_np(wk.inv).reshape(W, 2, L, L), to_np(e)
    for w in range(W):
        npos, ninv, acc, ek = ovmc.pbp_sweep(A, NG, coef, pos[w], inv[w], eta[w], uni[w])
        np.testing.assert_array_equal(g_pos[w], npos, err_msg=f"walker {w}")
        bar = cond_bar(coef, npos)
        eb = np.abs(g_inv[w] - ninv).max() / np.abs(ninv).max()
        ee = abs(g_e[w] - ek) / lap_scale(coef, npos, ninv)
        say(f"PbP walker {w}: accepted {int(acc.sum())} of {2 * L}, inverse err {eb:.1e}, "
            f"energy err {ee:.1e} (bar {bar:.1e})")
        assert eb <= bar and ee <= bar


def test_setup_inverse_and_kinetic_of_fresh_walkers(setup):
    """Walkers built without inverses invert their Slater matrices once; the
    kinetic energy at the start matches the oracle's."""
    blip, vmc, t, coef, pos, inv, rng = setup
    wk = vmc.Walkers(t, torch.from_numpy(pos.copy()).cuda())
    e = to_np(wk.kinetic())
    for w in range(W):
        ek = ovmc.local_kinetic(A, NG, coef, pos[w], inv[w])
        assert abs(e[w] - ek) <= cond_bar(coef, pos[w]) * lap_scale(coef, pos[w], inv[w])


def test_kept_laplacian_rows_and_helpers(setup):
    """Energies from the kept Laplacian rows equal a fresh evaluation at the
    same positions and inverses (FP64 sums of the same FP32 rows, in another
    order); blip_qs_copy_rows copies exactly the listed rows;
    blip_qs_lap_ratios equals an FP64 dot of the rows."""
    blip, vmc, t, coef, pos, inv, rng = setup
    wk = vmc.Walkers(t, torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(inv.copy()).cuda())
    for _ in range(3):
        eta = torch.from_numpy(rng.normal(0, 0.5, pos.shape)).cuda()
        uni = torch.from_numpy(rng.uniform(0, 1, (W, 2 * L))).cuda()
        _, e = wk.step(eta, uni)
    assert wk.lap_ok
    kept = to_np(e).copy()
    kept_rows = to_np(wk.lap).copy()
    wk.lap_ok = False
    fresh = to_np(wk.kinetic())
    say(f"kept-row energies {kept} against fresh {fresh}")
    np.testing.assert_allclose(kept, fresh, rtol=1e-12, atol=1e-12 * np.abs(fresh).max())
    np.testing.assert_array_equal(kept_rows, to_np(wk.lap))   # same FP32 rows either way
    # the helpers alone
    nmat, n = 2 * W, L
    src = torch.from_numpy(rng.standard_normal((nmat * n, n)).astype(np.float32)).cuda()
    dst0 = rng.standard_normal((nmat * n, n)).astype(np.float32)
    dst = torch.from_numpy(dst0.copy()).cuda()
    counts = rng.integers(0, n + 1, nmat).astype(np.int32)
    cols = np.zeros((nmat, n), dtype=np.int32)
    want = dst0.copy()
    for q in range(nmat):
        c = np.sort(rng.permutation(n)[: counts[q]])
        cols[q, : len(c)] = c
        want[q * n + c] = to_np(src)[q * n + c]
    lib = blip.lib()
    dcols, dcounts = torch.from_numpy(cols).cuda(), torch.from_numpy(counts).cuda()
    assert lib.blip_qs_copy_rows(nmat, n, n, dcols.data_ptr(), n, dcounts.data_ptr(),
                                 src.data_ptr(), n, dst.data_ptr(), n, None) == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(dst), want)
    a = rng.standard_normal((37, 50)).astype(np.float32)
    b = rng.standard_normal((37, 61))
    out = torch.empty(37, dtype=torch.float64, device="cuda")
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    assert lib.blip_qs_lap_ratios(37, 50, ta.data_ptr(), 50, tb.data_ptr(), 61,
                                  out.data_ptr(), None) == 0
    torch.cuda.synchronize()
    want = np.einsum("rl,rl->r", a.astype(np.float64), b[:, :50])
    scale = np.einsum("rl,rl->r", np.abs(a.astype(np.float64)), np.abs(b[:, :50]))
    assert np.all(np.abs(to_np(out) - want) <= 64 * np.finfo(np.float64).eps * scale)


def test_sorted_ratio_pass_same_chain(setup):
    """40 walkers of 2 x 64 electrons (5,120 moves a step, enough for the
    sorted persistent ratio pass by default): three steps with the sorted pass
    and with the block pass, from the same start and random numbers, take the
    same decisions (none within 1e-9 of a tie), reach the same positions and
    inverses bit for bit (the same FP32 orbital rows, the same updates), and
    energies equal to 1e-12."""
    blip, vmc = setup[0], setup[1]
    rng = np.random.default_rng(zlib.crc32(b"gpu-vmc-sorted"))
    n, nw = 64, 40
    coef = rng.uniform(-1, 1, NG + (n,)).astype(np.float32)
    t = blip.Table(A, NG, coef, "f32")
    pos = torch.from_numpy(rng.uniform(0, 1, (nw, 2 * n, 3)) @ A).cuda()
    a = vmc.Walkers(t, pos.clone())
    b = vmc.Walkers(t, pos.clone(), inv_t=a.inv.clone(), sort_moves=False)
    assert a.sorted and not b.sorted
    say(f"sorted vs block ratio pass: {nw} walkers x {2 * n} electrons")
    # kept rows current from the start, so every step runs the full ratio
    # pass and leaves the trial moves' ratios in place for the tie check
    ka, kb = a.kinetic(), b.kinetic()
    torch.cuda.synchronize()
    np.testing.assert_allclose(to_np(ka), to_np(kb), rtol=1e-12,
                               atol=1e-12 * float(np.abs(to_np(kb)).max()))
    for step in range(3):
        eta = torch.from_numpy(rng.normal(0, 0.3, (nw, 2 * n, 3))).cuda()
        uni = torch.from_numpy(rng.uniform(0, 1, (nw, 2 * n))).cuda()
        ca, ea = a.step(eta, uni)
        cb, eb = b.step(eta, uni)
        torch.cuda.synchronize()
        r2 = to_np(b.ratio) ** 2
        # the two passes' ratios differ by FP64 rounding only (different
        # orbitals per lane are summed in another order)
        assert np.min(np.abs(to_np(uni).ravel() - r2)) > 1e-9, "a decision is within rounding"
        assert torch.equal(ca, cb), step
        assert torch.equal(a.pos, b.pos) and torch.equal(a.inv, b.inv), step
        np.testing.assert_allclose(to_np(ea), to_np(eb), rtol=1e-12,
                                   atol=1e-12 * float(np.abs(to_np(eb)).max()))
        say(f"  step {step}: accepted {int(to_np(ca).sum())} of {nw * 2 * n}")
    t.free()


def test_walkers_on_side_streams(setup):
    """Walkers stepped on their own (non-default) streams: the first inverses
    set up from scratch, quasi-simultaneous steps and a particle-by-particle
    sweep give bit for bit what the same walkers give on the default stream,
    with two walker sets stepping concurrently on two streams."""
    blip, vmc, t, coef, pos, inv, rng = setup
    p0 = torch.from_numpy(pos.copy()).cuda()
    ref = vmc.Walkers(t, p0.clone())
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = vmc.Walkers(t, p0.clone(), stream=s1)
    b = vmc.Walkers(t, p0.clone(), stream=s2)
    torch.cuda.synchronize()
    say("walkers on side streams: setup inverses")
    assert torch.equal(ref.inv, a.inv) and torch.equal(ref.inv, b.inv)
    for step in range(3):
        eta = torch.from_numpy(rng.normal(0, 0.3, (W, 2 * L, 3))).cuda()
        uni = torch.from_numpy(rng.uniform(0, 1, (W, 2 * L))).cuda()
        torch.cuda.synchronize()
        cr, er = ref.step(eta, uni)
        ca, ea = a.step(eta, uni)
        cb, eb = b.step(eta, uni)
        torch.cuda.synchronize()
        for w in (a, b):
            assert torch.equal(w.pos, ref.pos) and torch.equal(w.inv, ref.inv), step
        assert torch.equal(ea, er) and torch.equal(eb, er), step
    eta = torch.from_numpy(rng.normal(0, 0.3, (W, 2 * L, 3))).cuda()
    uni = torch.from_numpy(rng.uniform(0, 1, (W, 2 * L))).cuda()
    torch.cuda.synchronize()
    say("walkers on side streams: particle-by-particle sweep")
    er = ref.pbp_sweep(eta, uni)
    ea = a.pbp_sweep(eta, uni)
    torch.cuda.synchronize()
    assert torch.equal(a.pos, ref.pos) and torch.equal(a.inv, ref.inv)
    assert torch.equal(ea, er)
