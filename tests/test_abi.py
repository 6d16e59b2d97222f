"""The C-ABI library loads, exports every symbol include/blip.h declares, and
rejects bad arguments on the host before touching a GPU (CPU-only)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blip.h")
LIB = os.path.join(ROOT, "paper_1204_1121_amd", "libblip.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"BLIP_API\s+[\w\s\*]+?\b(blip_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def blip():
    import torch  # noqa: F401  (one HIP runtime for the process)
    from paper_1204_1121_amd import blip as b
    if not os.path.exists(LIB):
        from paper_1204_1121_amd import build
        build.build()
    return b


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("blip_load", "blip_eval", "blip_eval_ex", "blip_free",
                     "blip_last_error", "blip_table_info", "blip_version"):
        assert required in names


def test_every_declared_symbol_is_exported(blip):
    L = blip.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_no_stray_exports(blip):
    """Only the declared C ABI is visible (everything else is hidden)."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert exported <= set(_declared()) | {"_init", "_fini"}, exported - set(_declared())


def _load(blip, lattice=None, n=(4, 4, 4), norb=2, storage=0, kvec=None, coef=True):
    L = blip.lib()
    A = np.ascontiguousarray(np.eye(3) * 4.0 if lattice is None else lattice, dtype=np.float64)
    c = np.zeros(max(1, int(np.prod(n)) * max(norb, 1) * 2), dtype=np.float32)
    h = ctypes.c_void_p()
    k = None if kvec is None else np.ascontiguousarray(kvec, dtype=np.float64)
    rc = L.blip_load(A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n[0], n[1], n[2], norb,
                     c.ctypes.data_as(ctypes.c_void_p) if coef else None, storage,
                     k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if k is not None else None,
                     ctypes.byref(h))
    return rc, h


def test_load_argument_errors(blip):
    assert _load(blip, n=(3, 4, 4))[0] == -1            # grid < 4
    assert _load(blip, norb=0)[0] == -1                  # no orbitals
    assert _load(blip, coef=False)[0] == -1              # NULL coefficients
    assert _load(blip, lattice=np.zeros((3, 3)))[0] == -1   # singular
    sing = np.array([[1.0, 2, 3], [2, 4, 6], [0, 0, 1]])
    assert _load(blip, lattice=sing)[0] == -1
    bad = np.eye(3)
    bad[1, 1] = np.nan
    assert _load(blip, lattice=bad)[0] == -1
    assert _load(blip, storage=9)[0] == -4               # unknown dtype
    assert _load(blip, storage=0, kvec=[0.1, 0, 0])[0] == -4   # k-point on real table
    msg = blip.lib().blip_last_error().decode()
    assert "complex" in msg
    # one (i1, i2) line of n3 rows must stay below 2 GiB: n3 = 4096 rows of
    # 2^20 floats (4 MiB each) is 16 GiB; rejected before any allocation
    L = blip.lib()
    A = np.ascontiguousarray(np.eye(3) * 4.0)
    h = ctypes.c_void_p()
    rc = L.blip_load(A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4, 4, 4096, 1 << 20,
                     ctypes.c_void_p(1), 0, None, ctypes.byref(h))
    assert rc == -1 and "2 GiB" in L.blip_last_error().decode()


def test_eval_rejects_bad_handle(blip):
    L = blip.lib()
    rc = L.blip_eval(None, None, 0, None, None, None, None)
    assert rc == -6
    junk = (ctypes.c_uint32 * 64)()
    rc = L.blip_eval(ctypes.cast(junk, ctypes.c_void_p), None, 1, None, None, None, None)
    assert rc == -6
    rc = L.blip_eval_batched_static(None, None, None, 1, 1, None, None, None, None)
    assert rc == -6
    rc = L.blip_submit(None, None, None, None, 1, None, None, 0, None, None, None, None, None,
                       None)
    assert rc == -6
    assert L.blip_free(None) == 0


def test_version_string(blip):
    assert "gfx950" in blip.version()


def test_sm_update_argument_errors(blip):
    """blip_sm_update validates sizes, indices, alignment and the workspace
    on the host; none of these calls reaches the device (fake pointers)."""
    L = blip.lib()
    n = 64
    ws = L.blip_sm_workspace_size(n)
    assert ws == 4 * 32 * n * 8
    assert L.blip_sm_workspace_size(0) == 0 and L.blip_sm_workspace_size(4097) == 0
    dev = ctypes.c_void_p(0x10000)          # never dereferenced: every call below fails first
    cols = np.array([3, 70], dtype=np.int64)
    cp = cols.ctypes.data_as(ctypes.c_void_p)

    def call(n=n, inv=dev, ld=n, u=dev, u_nrows=n, u_ld=n, c=cp, urow=None, k=2,
             ratios=dev, w=dev, wb=ws):
        return L.blip_sm_update(n, inv, ld, u, u_nrows, u_ld, c, urow, k, ratios, w, wb, None)

    assert call() == -1 and "cols[1]" in L.blip_last_error().decode()
    ok = np.array([3, 5], dtype=np.int64)
    okp = ok.ctypes.data_as(ctypes.c_void_p)
    assert call(n=0, c=okp) == -1
    assert call(n=4097, ld=4097, u_ld=4097, c=okp) == -1
    assert call(ld=n - 1, c=okp) == -1
    assert call(u_ld=n - 1, c=okp) == -1
    assert call(k=-1, c=okp) == -1
    assert call(c=None) == -1
    assert call(inv=None, c=okp) == -1
    assert call(u_nrows=5, c=okp) == -1 and "row 5" in L.blip_last_error().decode()
    bad_row = np.array([0, -1], dtype=np.int64)
    assert call(c=okp, urow=bad_row.ctypes.data_as(ctypes.c_void_p)) == -1
    assert call(c=okp, w=None) == -1
    assert call(c=okp, wb=ws - 1) == -1
    assert call(c=okp, inv=ctypes.c_void_p(0x10004)) == -5
    assert call(c=okp, u=ctypes.c_void_p(0x10002)) == -5
    assert call(c=okp, ratios=ctypes.c_void_p(0x10004)) == -5
    assert call(c=okp, w=ctypes.c_void_p(0x10004)) == -5
    assert call(c=None, k=0, w=None, wb=0) == 0          # k = 0: nothing to do
    # a matrix spanning 2 GiB or more (byte offsets past 31 bits) is refused
    big = (1 << 31) // (8 * (n - 1)) + 1
    assert call(c=okp, ld=big) == -1 and "2 GiB" in L.blip_last_error().decode()
    assert call(c=okp, u_ld=2 * big) == -1 and "2 GiB" in L.blip_last_error().decode()


def test_sm_update_batched_argument_errors(blip):
    """blip_sm_update_batched checks sizes, strides, alignment and the
    workspace on the host; nothing below reaches the device."""
    L = blip.lib()
    n = 64
    ws = L.blip_sm_batched_workspace_size(3, n)
    assert ws > 0 and ws % 256 == 0
    assert L.blip_sm_batched_workspace_size(-1, n) == 0
    assert L.blip_sm_batched_workspace_size(3, 4097) == 0
    dev = ctypes.c_void_p(0x10000)            # never dereferenced

    def call(nmat=3, n=n, inv=dev, ims=n * n, ild=n, u=dev, ums=n * n, uld=n, cols=dev, cld=n,
             cnt=dev, max_k=n, ratios=dev, rld=n, w=dev, wb=ws):
        return L.blip_sm_update_batched(nmat, n, inv, ims, ild, u, ums, uld, cols, cld, cnt, max_k,
                                        ratios, rld, w, wb, None)

    assert call(nmat=-1) == -1
    assert call(nmat=70000) == -1
    assert call(n=0) == -1 and call(n=4097) == -1
    assert call(max_k=n + 1) == -1 and call(max_k=-1) == -1
    assert call(inv=None) == -1 and call(cols=None) == -1 and call(cnt=None) == -1
    assert call(ild=n - 1) == -1 and call(uld=n - 1) == -1
    assert call(cld=n - 1) == -1 and call(rld=n - 1) == -1
    assert call(ims=n * n - 1) == -1 and call(ums=n * n - 1) == -1
    assert call(w=None) == -1 and call(wb=ws - 1) == -1
    assert call(inv=ctypes.c_void_p(0x10004)) == -5
    assert call(cols=ctypes.c_void_p(0x10002)) == -5
    assert call(w=ctypes.c_void_p(0x10004)) == -5 and call(w=ctypes.c_void_p(0x10008)) == -5
    assert call(nmat=0, inv=None, u=None, cols=None, cnt=None, w=None, wb=0) == 0
    assert call(max_k=0, inv=None, u=None, cols=None, cnt=None, w=None, wb=0) == 0
    big = (1 << 31) // (8 * (n - 1)) + 1
    assert call(nmat=1, ild=big) == -1 and "2 GiB" in L.blip_last_error().decode()
    assert call(nmat=1, uld=2 * big) == -1 and "2 GiB" in L.blip_last_error().decode()


def test_qs_helpers_argument_errors(blip):
    """blip_qs_propose / accept / kinetic / copy_rows / lap_ratios reject bad sizes,
    ranges and alignment on the host (fake pointers, never dereferenced)."""
    L = blip.lib()
    dev = ctypes.c_void_p(0x10000)
    odd = ctypes.c_void_p(0x10004)
    assert L.blip_qs_propose(-1, dev, dev, dev, None) == -1
    assert L.blip_qs_propose(0, None, None, None, None) == 0
    assert L.blip_qs_propose(4, None, dev, dev, None) == -1
    assert L.blip_qs_propose(4, odd, dev, dev, None) == -5

    def acc(nmat=2, n=8, j0=0, j1=8, ld=8, ratio=dev, cols=dev):
        return L.blip_qs_accept(nmat, n, j0, j1, ratio, dev, dev, dev, cols, ld, dev, None)

    assert acc(nmat=-1) == -1 and acc(nmat=70000) == -1
    assert acc(n=0) == -1
    assert acc(j0=-1) == -1 and acc(j0=5, j1=4) == -1 and acc(j1=9) == -1
    assert acc(ld=7) == -1
    assert acc(ratio=None) == -1
    assert acc(ratio=odd) == -5
    assert acc(cols=ctypes.c_void_p(0x10002)) == -5
    assert acc(nmat=0) == 0
    assert L.blip_qs_kinetic(-1, 8, dev, dev, None) == -1
    assert L.blip_qs_kinetic(2, 0, dev, dev, None) == -1
    assert L.blip_qs_kinetic(2, 8, odd, dev, None) == -5
    assert L.blip_qs_kinetic(0, 8, None, None, None) == 0

    def copy(nmat=2, n=8, ln=8, ld=8, sld=8, dld=8, src=dev, cols=dev):
        return L.blip_qs_copy_rows(nmat, n, ln, cols, ld, dev, src, sld, dev, dld, None)

    assert copy(nmat=-1) == -1 and copy(nmat=70000) == -1
    assert copy(n=0) == -1 and copy(ln=-1) == -1
    assert copy(ld=7) == -1 and copy(sld=7) == -1 and copy(dld=7) == -1
    assert copy(src=None) == -1
    assert copy(src=ctypes.c_void_p(0x10002)) == -5
    assert copy(nmat=0) == 0 and copy(ln=0) == 0
    assert L.blip_qs_lap_ratios(-1, 8, dev, 8, dev, 8, dev, None) == -1
    assert L.blip_qs_lap_ratios(4, 0, dev, 8, dev, 8, dev, None) == -1
    assert L.blip_qs_lap_ratios(4, 8, dev, 7, dev, 8, dev, None) == -1
    assert L.blip_qs_lap_ratios(4, 8, dev, 8, dev, 7, dev, None) == -1
    assert L.blip_qs_lap_ratios(4, 8, None, 8, dev, 8, dev, None) == -1
    assert L.blip_qs_lap_ratios(4, 8, dev, 8, odd, 8, dev, None) == -5
    assert L.blip_qs_lap_ratios(0, 8, None, 8, None, 8, None, None) == 0
    # blip_eval_ratio_values takes gradient and Laplacian ratios and rows
    # together or not at all (checked before the table handle)
    assert L.blip_eval_ratio_values(None, dev, 4, dev, 8, None, dev, dev, dev, dev, None,
                                    None) == -1
    assert L.blip_eval_ratio_values(None, dev, 4, dev, 8, None, dev, None, None, dev, dev,
                                    None) == -1
    # and so does its batched form, which also needs the values, 4-byte
    # aligned, before it looks at the table
    rvb = L.blip_eval_ratio_values_batched
    assert rvb(None, dev, dev, 1, 4, dev, 8, None, dev, dev, dev, dev, None, dev, 1 << 20,
               None) == -1
    assert rvb(None, dev, dev, 1, 4, dev, 8, None, dev, None, None, None, None, dev, 1 << 20,
               None) == -1
    assert rvb(None, dev, dev, 1, 4, dev, 8, None, dev, None, None, ctypes.c_void_p(0x10002),
               None, dev, 1 << 20, None) == -5
    assert rvb(None, dev, dev, 1, 4, dev, 8, None, dev, None, None, dev, None, dev, 1 << 20,
               None) == -6


def test_stream_read_argument_errors(blip):
    """blip_stream_read checks sizes and alignment on the host (fake pointers,
    never dereferenced)."""
    L = blip.lib()
    dev = ctypes.c_void_p(0x10000)
    assert L.blip_stream_read(dev, 1 << 20, dev, 0, None) == -1
    assert L.blip_stream_read(dev, 1 << 20, dev, 65536, None) == -1
    assert L.blip_stream_read(dev, 0, dev, 8, None) == -1
    assert L.blip_stream_read(dev, 24, dev, 8, None) == -1
    assert L.blip_stream_read(None, 1 << 20, dev, 8, None) == -1
    assert L.blip_stream_read(dev, 1 << 20, None, 8, None) == -1
    assert L.blip_stream_read(ctypes.c_void_p(0x10008), 1 << 20, dev, 8, None) == -5
    assert L.blip_stream_read(dev, 1 << 20, ctypes.c_void_p(0x10002), 8, None) == -5


def test_stream_read_runs_argument_errors(blip):
    """blip_stream_read_runs checks sizes, the run length and alignment on the
    host (fake pointers, never dereferenced)."""
    L = blip.lib()
    dev = ctypes.c_void_p(0x10000)
    MB = 1 << 20

    def call(buf=dev, nbytes=MB, off=dev, nruns=4, rb=12288, part=dev, nb=8):
        return L.blip_stream_read_runs(buf, nbytes, off, nruns, rb, part, nb, None)

    assert call(nb=0) == -1 and call(nb=65536) == -1
    assert call(nruns=-1) == -1
    assert call(nbytes=0) == -1 and call(nbytes=40) == -1
    assert call(rb=4000) == -1 and "run_bytes" in L.blip_last_error().decode()
    assert call(off=None) == -1 and call(buf=None) == -1 and call(part=None) == -1
    assert call(buf=ctypes.c_void_p(0x10008)) == -5
    assert call(off=ctypes.c_void_p(0x10004)) == -5
    assert call(part=ctypes.c_void_p(0x10002)) == -5
