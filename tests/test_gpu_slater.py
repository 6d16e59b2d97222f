"""Sherman-Morrison update of the inverse Slater matrix on the GPU
(blip_sm_update) against the oracle's sequential rank-1 updates (Sec. VI.D).

Both sides compute in FP64 from the same FP32 orbital rows; they differ only
in the order of rounding (one rank-k correction per 32 moves against k
rank-1 corrections).  The bar for B after the moves is

    |B_gpu - B_oracle| <= 64 * n * eps * cond(D_new) * max|B_oracle|,

first-order perturbation of a matrix inverse with O(n) rounding per entry,
and for each sequential ratio the same bound relative to the scale of its
dot product, sum_l |u_l B[c][l]|, since a ratio can cancel (the
2-norm condition number from power iterations on D_new and the oracle's
inverse, with a factor 2 to stay above the true value)."""
import numpy as np
import pytest
import torch

from oracle import slater
from tests.gpu_util import say, to_np

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def blip():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    from paper_1204_1121_amd import blip as b
    b.lib()
    return b


def case(seed, n, k, repeats=False):
    """Well-conditioned D (electron rows), the transposed inverse, and k
    accepted moves: new rows near the old ones, rounded to FP32 (as
    blip_eval writes them), stored one per electron in a [n, n] matrix."""
    rng = np.random.default_rng(seed)
    D = 2.0 * np.eye(n) + rng.normal(0, 1.0 / np.sqrt(n), (n, n))
    inv_t = np.linalg.inv(D).T.copy()
    if repeats:
        cols = rng.integers(0, n, k)
    else:
        cols = rng.permutation(n)[:k]
    U = (D + rng.normal(0, 0.3, (n, n))).astype(np.float32)
    return D, inv_t, cols.astype(np.int64), U


def norm2(M, iters=40):
    """2-norm by power iteration on M^T M, times 2: power iteration
    approaches the norm from below, and the margin keeps the bound an upper
    one (O(n^2) per step, so no factorisation at n = 4096)."""
    x = np.random.default_rng(0).normal(size=M.shape[1])
    for _ in range(iters):
        x = M.T @ (M @ x)
        x /= np.linalg.norm(x)
    return 2.0 * np.linalg.norm(M @ x)


def final_matrix(D, cols, rows):
    D = D.copy()
    for c, r in zip(cols, rows):
        D[c] = r
    return D


def check(blip, D, inv_t, cols, U, u_row=None, label=""):
    n = D.shape[0]
    urow = cols if u_row is None else np.asarray(u_row)
    rows = U[urow].astype(np.float64)
    want_b, want_r, before = slater.sm_update(inv_t, rows, cols, return_rows=True)
    inv = torch.from_numpy(inv_t).cuda()
    u = torch.from_numpy(U).cuda()
    r = blip.sm_update(inv, u, cols, u_row=u_row)
    torch.cuda.synchronize()
    got_b, got_r = to_np(inv), to_np(r)
    cond = norm2(final_matrix(D, cols, rows)) * norm2(want_b)
    tol = 64 * n * EPS * cond
    eb = np.abs(got_b - want_b).max() / np.abs(want_b).max()
    # a ratio is a dot product that can cancel: its error is measured against
    # the dot product's own scale, sum_l |u_l B[c][l]| (>= |ratio|)
    scale = np.einsum("ml,ml->m", np.abs(rows), np.abs(before))
    er = np.max(np.abs(got_r - want_r) / scale) if len(cols) else 0.0
    say(f"{label} n={n} k={len(cols)} cond={cond:.1e}: B err {eb:.1e}, ratio err {er:.1e} "
        f"(bar {tol:.1e})")
    assert eb <= tol and er <= tol
    return got_b, got_r


def test_small_several_chunks_ragged(blip):
    """n = 101 (ragged last row tile), 70 moves: chunks of 32, 32 and 6."""
    check(blip, *case(0, 101, 70), label="chunks")


def test_repeated_electrons(blip):
    """Electrons moved more than once in one call: chunks split at repeats;
    u_row gives each move its own new row."""
    D, inv_t, cols, U = case(1, 64, 90, repeats=True)
    assert len(set(cols.tolist())) < len(cols)
    rng = np.random.default_rng(11)
    Ubig = np.concatenate([U, (D + rng.normal(0, 0.3, D.shape)).astype(np.float32)])
    u_row = np.where(rng.random(len(cols)) < 0.5, cols, cols + 64)
    check(blip, D, inv_t, cols, Ubig, u_row=u_row, label="repeats")


def test_one_move_and_no_moves(blip):
    D, inv_t, cols, U = case(2, 40, 1)
    check(blip, D, inv_t, cols, U, label="one move")
    inv = torch.from_numpy(inv_t).cuda()
    r = blip.sm_update(inv, torch.from_numpy(U).cuda(), [])
    torch.cuda.synchronize()
    assert r.numel() == 0
    np.testing.assert_array_equal(to_np(inv), inv_t)


def test_unmoved_electrons_leave_inverse(blip):
    """Moves that give electrons their own rows back: every ratio 1, B kept."""
    rng = np.random.default_rng(3)
    n = 96
    D = (2.0 * np.eye(n) + rng.normal(0, 0.1, (n, n))).astype(np.float32).astype(np.float64)
    inv_t = np.linalg.inv(D).T.copy()
    cols = rng.permutation(n)[:50].astype(np.int64)
    inv = torch.from_numpy(inv_t).cuda()
    r = blip.sm_update(inv, torch.from_numpy(D.astype(np.float32)).cuda(), cols)
    torch.cuda.synchronize()
    np.testing.assert_allclose(to_np(r), 1.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(to_np(inv), inv_t, rtol=0, atol=1e-12 * np.abs(inv_t).max())


@pytest.mark.parametrize("n", [1, 2, 33, 1024, 1025, 2049, 4096])
def test_orders_and_row_tilings(blip, n):
    """The smallest orders, ragged 16-row and 16-column tiles (33, 1025,
    2049), one to four column tiles, and the largest accepted order."""
    k = min(n, 40)
    check(blip, *case(100 + n, n, k), label="order")


@pytest.mark.parametrize("ld,u_ld", [(80, 75), (71, 72)])
def test_padded_leading_dimensions(blip, ld, u_ld):
    """inv and u with row strides above n (views into wider buffers).  An
    odd stride of inv, or a stride of u that is not a multiple of 4, makes
    rows unaligned for 16-byte accesses: those rows take the scalar path."""
    D, inv_t, cols, U = case(4, 70, 45)
    wide = np.full((70, ld), 7.0)
    wide[:, :70] = inv_t
    base = torch.from_numpy(wide).cuda()
    inv = base[:, :70]
    Uw = np.full((70, u_ld), 3.0, dtype=np.float32)
    Uw[:, :70] = U
    u = torch.from_numpy(Uw).cuda()[:, :70]
    want_b, want_r = slater.sm_update(inv_t, U[cols].astype(np.float64), cols)
    r = blip.sm_update(inv, u, cols)
    torch.cuda.synchronize()
    full = base.cpu().numpy()
    assert np.all(full[:, 70:] == 7.0), "columns past n were written"
    np.testing.assert_allclose(full[:, :70], want_b, rtol=0, atol=1e-10 * np.abs(want_b).max())
    np.testing.assert_allclose(to_np(r), want_r, rtol=1e-10)


def test_wide_and_narrow_loads_agree_bitwise(blip):
    """The same update with rows 16-byte aligned (16-byte tile loads) and
    with odd leading dimensions (8- and 4-byte loads): bit for bit equal,
    ratios included, and within the oracle's bar."""
    n, ld = 72, 73
    D, inv_t, cols, U = case(7, n, 50)
    inv_a = torch.from_numpy(inv_t.copy()).cuda()
    r_a = blip.sm_update(inv_a, torch.from_numpy(U).cuda(), cols)
    wide = np.zeros((n, ld))
    wide[:, :n] = inv_t
    base = torch.from_numpy(wide).cuda()
    Uw = np.zeros((n, ld), dtype=np.float32)
    Uw[:, :n] = U
    r_b = blip.sm_update(base[:, :n], torch.from_numpy(Uw).cuda()[:, :n], cols)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(base)[:, :n], to_np(inv_a))
    np.testing.assert_array_equal(to_np(r_b), to_np(r_a))
    check(blip, D, inv_t, cols, U, label="aligned rows")


def test_quasi_simultaneous_step_tio2(blip):
    """One spin of the TiO2 block (768 electrons, 768 orbitals of the
    72x72x48 table): the Slater matrix from blip_eval at the old positions,
    trial moves, acceptance from blip_eval_ratio against the old inverse,
    then the inverse updated for the accepted moves.  The first accepted
    move's sequential ratio is its quasi-simultaneous ratio."""
    from paper_1204_1121_amd import workloads as wl
    spec = wl.spec_tio2()
    c = wl.coefficients(spec)
    t = blip.Table(spec.lattice, spec.n, c, "f32")
    del c
    rng = np.random.default_rng(5)
    n = spec.norb
    old = rng.uniform(0, 1, (n, 3)) @ spec.lattice
    new = old + rng.normal(0, 0.35, old.shape)
    val_old = to_np(t.eval(torch.from_numpy(old).cuda(), grad=False)[0]).astype(np.float64)
    inv_t = np.linalg.inv(val_old).T.copy()
    newd = torch.from_numpy(new).cuda()
    U = t.eval(newd, grad=False)[0]
    inv = torch.from_numpy(inv_t).cuda()
    q, _, _ = t.ratio(newd, inv, grad=False)
    qs = to_np(q)
    accept = rng.random(n) < np.minimum(1.0, qs ** 2)
    cols = np.nonzero(accept)[0].astype(np.int64)
    say(f"TiO2 Q.S. step: {len(cols)} of {n} moves accepted")
    assert 0 < len(cols) < n
    got_b, got_r = check(blip, val_old, inv_t, cols, to_np(U), label="TiO2")
    assert got_r[0] == pytest.approx(qs[cols[0]], rel=1e-10)
    t.free()


def test_batched_equals_single_bitwise(blip):
    """blip_sm_update_batched over matrices with 0, 1, 31, 32, 70 and all 101
    accepted moves equals blip_sm_update on each matrix bit for bit (same
    arithmetic in the same order), ratios included; one matrix against the
    oracle."""
    n = 101
    counts = [0, 1, 31, 32, 70, 101]
    nmat = len(counts)
    rng = np.random.default_rng(21)
    Ds, invs, Us, lists = [], [], [], []
    for q in range(nmat):
        D, inv_t, _, U = case(300 + q, n, 1)
        Ds.append(D)
        invs.append(inv_t)
        Us.append(U)
        lists.append(rng.permutation(n)[: counts[q]].astype(np.int64))
    max_k = max(counts)
    acc = np.zeros((nmat, max_k), dtype=np.int32)
    for q, c in enumerate(lists):
        acc[q, : len(c)] = c
    inv_b = torch.from_numpy(np.stack(invs)).cuda()
    u_b = torch.from_numpy(np.stack(Us)).cuda()
    say(f"batched SM: {nmat} matrices, counts {counts}")
    r_b = blip.sm_update_batched(inv_b, u_b, torch.from_numpy(acc).cuda(),
                                 torch.tensor(counts, dtype=torch.int32, device="cuda"), max_k)
    torch.cuda.synchronize()
    got_inv, got_r = to_np(inv_b), to_np(r_b)
    for q in range(nmat):
        inv1 = torch.from_numpy(invs[q]).cuda()
        r1 = blip.sm_update(inv1, torch.from_numpy(Us[q]).cuda(), lists[q])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got_inv[q], to_np(inv1), err_msg=f"matrix {q}")
        np.testing.assert_array_equal(got_r[q, : counts[q]], to_np(r1), err_msg=f"ratios {q}")
    q = 4
    want_b, want_r = slater.sm_update(invs[q], Us[q][lists[q]].astype(np.float64), lists[q])
    assert np.abs(got_inv[q] - want_b).max() <= 1e-10 * np.abs(want_b).max()
    np.testing.assert_allclose(got_r[q, : counts[q]], want_r, rtol=1e-9)


def test_batched_workspace_offsets_and_reuse(blip):
    """The batched update keeps each chunk's packed u rows in its workspace:
    a workspace that is only 16-byte aligned (a view 16 bytes into a larger
    buffer), reused by a second call with other matrices and counts, gives
    the same bits as a fresh 256-byte-aligned one, and a workspace view 8
    bytes in is refused."""
    n = 136
    counts = [97, 40, 0, 65]
    nmat = len(counts)
    rng = np.random.default_rng(33)
    invs, Us, acc = [], [], np.zeros((nmat, n), dtype=np.int32)
    for q in range(nmat):
        _, inv_t, _, U = case(400 + q, n, 1)
        invs.append(inv_t)
        Us.append(U)
        acc[q, : counts[q]] = rng.permutation(n)[: counts[q]]
    nbytes = blip.lib().blip_sm_batched_workspace_size(nmat, n)
    big = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    cnt = torch.tensor(counts, dtype=torch.int32, device="cuda")
    acc_d = torch.from_numpy(acc).cuda()
    u_b = torch.from_numpy(np.stack(Us)).cuda()
    say(f"batched SM workspace offsets: {nmat} matrices of order {n}, counts {counts}")

    def run(ws, k=max(counts), c=cnt):
        inv_b = torch.from_numpy(np.stack(invs)).cuda()
        r = blip.sm_update_batched(inv_b, u_b, acc_d, c, k, workspace=ws)
        torch.cuda.synchronize()
        return to_np(inv_b), to_np(r)

    want_inv, want_r = run(torch.empty(nbytes, dtype=torch.uint8, device="cuda"))
    # a first call with other counts leaves other packed rows behind
    run(big[16:16 + nbytes], k=n, c=torch.tensor([n, 3, 77, 1], dtype=torch.int32, device="cuda"))
    got_inv, got_r = run(big[16:16 + nbytes])
    np.testing.assert_array_equal(got_inv, want_inv)
    for q in range(nmat):
        np.testing.assert_array_equal(got_r[q, : counts[q]], want_r[q, : counts[q]])
    with pytest.raises(RuntimeError, match="16-byte"):
        run(big[8:8 + nbytes])


@pytest.mark.parametrize("n", [200, 201])
def test_batched_two_row_blocks_equals_single_bitwise(blip, n):
    """Enough matrices for the batched kernel to take two 16-row blocks per
    workgroup (ceil(n/32) * nmat >= 1024): still bit for bit the single-matrix
    result on sampled matrices, with a ragged n and uneven counts.  At
    n = 201 the rows are not 16-byte aligned (8- and 4-byte tile loads)."""
    nmat = 160
    rng = np.random.default_rng(23)
    D0, inv0, _, U0 = case(400, n, 1)
    invs = np.stack([inv0 * (1.0 + 0.01 * q) for q in range(nmat)])
    Us = np.stack([U0] * nmat)
    counts = rng.integers(0, n + 1, nmat)
    counts[:3] = [0, 1, n]
    max_k = int(counts.max())
    acc = np.zeros((nmat, max_k), dtype=np.int32)
    lists = []
    for q in range(nmat):
        c = rng.permutation(n)[: counts[q]].astype(np.int64)
        lists.append(c)
        acc[q, : len(c)] = c
    say(f"batched SM, two row blocks: {nmat} matrices of n = {n}, max_k = {max_k}")
    inv_b = torch.from_numpy(invs).cuda()
    r_b = blip.sm_update_batched(inv_b, torch.from_numpy(Us).cuda(), torch.from_numpy(acc).cuda(),
                                 torch.from_numpy(counts.astype(np.int32)).cuda(), max_k)
    torch.cuda.synchronize()
    got_inv, got_r = to_np(inv_b), to_np(r_b)
    for q in (0, 1, 2, 77, nmat - 1):
        inv1 = torch.from_numpy(invs[q].copy()).cuda()
        r1 = blip.sm_update(inv1, torch.from_numpy(U0).cuda(), lists[q])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got_inv[q], to_np(inv1), err_msg=f"matrix {q}")
        np.testing.assert_array_equal(got_r[q, : counts[q]], to_np(r1), err_msg=f"ratios {q}")


@pytest.mark.parametrize("n", [1, 2, 4096])
def test_batched_extreme_orders(blip, n):
    """The smallest orders and the largest accepted one (four column tiles,
    up to 128 chunks): two matrices, all and half of the electrons moved,
    bit for bit the single-matrix update."""
    counts = [n, n // 2]
    rng = np.random.default_rng(500 + n)
    invs, Us, lists = [], [], []
    for q in range(2):
        D, inv_t, _, U = case(510 + n + q, n, 1)
        invs.append(inv_t)
        Us.append(U)
        lists.append(rng.permutation(n)[: counts[q]].astype(np.int64))
    max_k = max(counts)
    acc = np.zeros((2, max(max_k, 1)), dtype=np.int32)
    for q, c in enumerate(lists):
        acc[q, : len(c)] = c
    say(f"batched SM, order {n}: counts {counts}")
    inv_b = torch.from_numpy(np.stack(invs)).cuda()
    r_b = blip.sm_update_batched(inv_b, torch.from_numpy(np.stack(Us)).cuda(),
                                 torch.from_numpy(acc).cuda(),
                                 torch.tensor(counts, dtype=torch.int32, device="cuda"), max_k)
    torch.cuda.synchronize()
    got_inv, got_r = to_np(inv_b), to_np(r_b)
    for q in range(2):
        inv1 = torch.from_numpy(invs[q]).cuda()
        r1 = blip.sm_update(inv1, torch.from_numpy(Us[q]).cuda(), lists[q])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got_inv[q], to_np(inv1), err_msg=f"matrix {q}")
        np.testing.assert_array_equal(got_r[q, : counts[q]], to_np(r1), err_msg=f"ratios {q}")


@pytest.mark.parametrize("nmat", [12, 60])
def test_batched_ragged_end_bitwise(blip, nmat):
    """Ragged move counts at an order with three column tiles: the later
    launches have few matrices with moves, and there each (row block, column
    tile) gets a workgroup of its own.  Every matrix still equals the
    single-matrix update bit for bit (one and two row blocks per workgroup)."""
    n = 600
    rng = np.random.default_rng(900 + nmat)
    D, inv0, _, U0 = case(901, n, 1)
    invs = np.stack([inv0 * (1.0 + 0.01 * q) for q in range(nmat)])
    counts = rng.integers(0, 120, nmat)
    counts[:4] = [0, 33, 600, 451]          # a long tail: 2, then 1 matrix active
    max_k = int(counts.max())
    acc = np.zeros((nmat, max_k), dtype=np.int32)
    lists = []
    for q in range(nmat):
        c = rng.permutation(n)[: counts[q]].astype(np.int64)
        acc[q, : len(c)] = c
        lists.append(c)
    say(f"batched SM, ragged end: {nmat} matrices of n = {n}, counts up to {max_k}")
    inv_b = torch.from_numpy(invs).cuda()
    U = torch.from_numpy(U0).cuda()
    r_b = blip.sm_update_batched(inv_b, U.unsqueeze(0).expand(nmat, n, n).contiguous(),
                                 torch.from_numpy(acc).cuda(),
                                 torch.from_numpy(counts.astype(np.int32)).cuda(), max_k)
    torch.cuda.synchronize()
    got_inv, got_r = to_np(inv_b), to_np(r_b)
    for q in (0, 1, 2, 3, nmat - 1):
        inv1 = torch.from_numpy(invs[q]).cuda()
        r1 = blip.sm_update(inv1, U, lists[q])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got_inv[q], to_np(inv1), err_msg=f"matrix {q}")
        np.testing.assert_array_equal(got_r[q, : counts[q]], to_np(r1), err_msg=f"ratios {q}")


def test_batched_padded_strides_and_untouched(blip):
    """Matrices with padded rows inside a wider buffer, u with extra rows:
    columns past n and matrices with no moves are left as they were."""
    n, nmat = 40, 3
    counts = [5, 0, 40]
    rng = np.random.default_rng(22)
    base = np.full((nmat, n, 48), 9.0)
    U = np.zeros((nmat, n + 3, 44), dtype=np.float32)
    invs, lists = [], []
    for q in range(nmat):
        D, inv_t, _, Uq = case(400 + q, n, 1)
        base[q, :, :n] = inv_t
        U[q, :n, :n] = Uq
        invs.append((inv_t, Uq))
        lists.append(rng.permutation(n)[: counts[q]].astype(np.int64))
    acc = np.zeros((nmat, 40), dtype=np.int32)
    for q, c in enumerate(lists):
        acc[q, : len(c)] = c
    t = torch.from_numpy(base).cuda()
    inv = t[:, :, :n]
    r = blip.sm_update_batched(inv, torch.from_numpy(U).cuda(), torch.from_numpy(acc).cuda(),
                               torch.tensor(counts, dtype=torch.int32, device="cuda"), 40)
    torch.cuda.synchronize()
    full = t.cpu().numpy()
    assert np.all(full[:, :, n:] == 9.0)
    np.testing.assert_array_equal(full[1, :, :n], invs[1][0])
    for q in (0, 2):
        want_b, want_r = slater.sm_update(invs[q][0], invs[q][1][lists[q]].astype(np.float64),
                                          lists[q])
        assert np.abs(full[q, :, :n] - want_b).max() <= 1e-10 * np.abs(want_b).max()
        np.testing.assert_allclose(to_np(r)[q, : counts[q]], want_r, rtol=1e-9)
