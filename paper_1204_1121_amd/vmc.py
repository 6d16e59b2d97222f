"""Quasi-simultaneous Monte Carlo steps for many walkers, on the device.

A walker is 2n electrons (n of each spin) in the potential-free synthetic
system whose trial function is the Slater part of Eq. (6): one determinant of
Eq. (5) per spin, over the table's L = n real orbitals, p = |Psi_D|^2.  One
quasi-simultaneous step (Sec. IV.A; the sequence of Sec. II.B) runs as:

  blip_qs_propose          trial = pos + eta for every electron
  blip_eval_ratio_values   in one pass: each move's ratio against the old
  (_batched)               configuration, psi_l at every trial position (the
                           new rows) and lap psi_l there; for many moves the
                           sorted persistent launch, in which the moves of all
                           walkers that fall near the same grid sites share
                           the table rows they read
  blip_qs_accept           uniform < ratio^2; accepted positions copied and
                           listed per (walker, spin) in electron order
  blip_sm_update_batched   the inverses brought up to date for those moves
  blip_qs_copy_rows        the accepted electrons' Laplacian rows carried into
                           the rows kept for the current configuration
  blip_qs_lap_ratios +     the local kinetic energy per walker,
  blip_qs_kinetic          -1/2 sum_j lap_j Psi / Psi at the new positions,
                           from the kept rows and the new inverses

The walker keeps the Laplacian rows of the orbitals at its current positions
(lap psi_l(r_j), [2n, n] float32 per walker), so the kinetic energy after a
step costs a pass over those rows and the inverses instead of a second
evaluation of the orbitals.  A step run without the energy leaves the rows
stale; the next kinetic energy then evaluates them afresh
(blip_eval_ratio_values at the current positions).

Random numbers are the caller's (eta Gaussian, uniform in [0, 1)), so a step
can be replayed against the FP64 oracle.  Everything above runs in this
library's kernels on the caller's stream; PyTorch only holds the buffers.
Setting up the first inverses from scratch (``Walkers(..., inv_t=None)``)
uses torch.linalg.inv once: that is setup, not part of a step.

Layout: pos [W, 2n, 3] float64 (electron g of walker w is spin g // n,
index g % n); inverses [W, 2, n, n] float64, row j of [w, s] = column j of
D_{w,s}^{-1} (the layout blip_eval_ratio and blip_sm_update read).
"""
from __future__ import annotations

import torch

from . import blip as _b
from .tuning import TuneCache

# From this many trial moves per step on, the ratio pass runs as one sorted
# persistent launch over all walkers; below it the sort's five small launches
# cost more than the row sharing saves.
SORT_MIN_MOVES = 4096


class Walkers:
    def __init__(self, table: "_b.Table", pos: torch.Tensor, inv_t: torch.Tensor | None = None,
                 stream=None, sort_moves: bool | None = None):
        if table.complex:
            raise ValueError("the synthetic system uses real orbitals")
        W, ne, three = pos.shape
        n = table.norb
        if three != 3 or ne != 2 * n or pos.dtype != torch.float64 or not pos.is_cuda:
            raise ValueError(f"pos must be cuda float64 [W, 2n = {2 * n}, 3]")
        self.t, self.W, self.n, self.stream = table, W, n, stream
        dev = pos.device
        self.pos = pos.contiguous()
        npos = W * 2 * n
        self.trial = torch.empty_like(self.pos)
        self.val = torch.empty((npos, n), dtype=torch.float32, device=dev)
        self.ratio = torch.empty(npos, dtype=torch.float64, device=dev)
        self.rg = torch.empty((npos, 3), dtype=torch.float64, device=dev)
        self.rl = torch.empty(npos, dtype=torch.float64, device=dev)
        self.acc_cols = torch.zeros((2 * W, n), dtype=torch.int32, device=dev)
        self.acc_count = torch.zeros(2 * W, dtype=torch.int32, device=dev)
        self.seq = torch.empty((2 * W, n), dtype=torch.float64, device=dev)
        self.e_kin = torch.empty(W, dtype=torch.float64, device=dev)
        self.lap = torch.empty((npos, n), dtype=torch.float32, device=dev)    # current positions
        self.lapt = torch.empty((npos, n), dtype=torch.float32, device=dev)   # trial positions
        self.lap_ok = False   # whether self.lap holds the rows of the current positions
        nbytes = _b.lib().blip_sm_batched_workspace_size(2 * W, n)
        self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        self.sorted = npos >= SORT_MIN_MOVES if sort_moves is None else bool(sort_moves)
        if self.sorted:
            self.off = torch.tensor([0, npos], dtype=torch.int64, device=dev)
            self.rws = table.workspace(npos, dev)
            # the ratio pass's launch shape measured for this table and step
            # size, if the package's tuning cache holds one (else the default)
            TuneCache().apply(table, npos, batched=True, ratio=True)
        # the first inverses are set up on the walkers' stream (after the
        # evaluation that fills their Slater matrices), where every later
        # kernel reads them
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            if inv_t is None:
                self.t.eval(self.pos.view(npos, 3), grad=False, out=(self.val, None, None),
                            stream=stream)
                D = self.val.view(2 * W, n, n).double()
                inv_t = torch.linalg.inv(D).transpose(1, 2)
            if tuple(inv_t.shape) != (W, 2, n, n) and tuple(inv_t.shape) != (2 * W, n, n):
                raise ValueError(f"inv_t must be [W, 2, n, n] (got {tuple(inv_t.shape)})")
            self.inv = inv_t.reshape(2 * W, n, n).to(torch.float64).contiguous()

    def _call(self, rc):
        _b.check(rc)

    def ratio_values(self, pos_flat: torch.Tensor, out: tuple):
        """Ratios against the current inverses, the orbital values and, with
        five outputs, the gradient and Laplacian ratios and the Laplacian
        rows, at pos_flat [2Wn, 3] (electron j uses inverse row j)."""
        npos, n, s = self.W * 2 * self.n, self.n, self.stream
        lap = len(out) == 5
        inv = self.inv.view(npos, n)
        if self.sorted:
            self.t.ratio_values_batched(pos_flat, self.off, inv, out=out, lap=lap,
                                        workspace=self.rws, stream=s)
        else:
            self.t.ratio_values(pos_flat, inv, out=out, lap=lap, stream=s)

    def step(self, eta: torch.Tensor, uniform: torch.Tensor, energy: bool = True,
             j0: int = 0, j1: int | None = None):
        """One quasi-simultaneous step with the given random numbers
        (eta [W, 2n, 3] bohr, uniform [W, 2n]; cuda float64).  Candidates of
        each (walker, spin) are its electrons j in [j0, j1) (default all).
        Returns (accepted counts [2W] int32, e_kin [W] or None), device
        tensors owned by this object."""
        W, n, s = self.W, self.n, self.stream
        npos = W * 2 * n
        L = _b.lib()
        keep = energy and self.lap_ok   # carry the kept Laplacian rows forward
        eta = eta.contiguous()
        uniform = uniform.contiguous()
        self._call(L.blip_qs_propose(npos, _b._ptr(self.pos), _b._ptr(eta), _b._ptr(self.trial),
                                     _b._stream_ptr(s)))
        tr = self.trial.view(npos, 3)
        if keep:
            self.ratio_values(tr, (self.ratio, self.rg, self.rl, self.val, self.lapt))
        else:
            self.ratio_values(tr, (self.ratio, self.val))
        self._call(L.blip_qs_accept(2 * W, n, j0, n if j1 is None else j1, _b._ptr(self.ratio),
                                    _b._ptr(uniform), _b._ptr(self.trial), _b._ptr(self.pos),
                                    _b._ptr(self.acc_cols), n, _b._ptr(self.acc_count),
                                    _b._stream_ptr(s)))
        _b.sm_update_batched(self.inv, self.val.view(2 * W, n, n), self.acc_cols,
                             self.acc_count, n, ratios=self.seq, workspace=self.ws, stream=s)
        if keep:
            self.carry_rows()
        else:
            self.lap_ok = False
        e = None
        if energy:
            e = self.kinetic()
        return self.acc_count, e

    def carry_rows(self):
        """The accepted electrons' Laplacian rows (at their trial positions,
        now their positions) into the kept rows."""
        W, n, s = self.W, self.n, self.stream
        self._call(_b.lib().blip_qs_copy_rows(2 * W, n, n, _b._ptr(self.acc_cols), n,
                                              _b._ptr(self.acc_count), _b._ptr(self.lapt), n,
                                              _b._ptr(self.lap), n, _b._stream_ptr(s)))

    def kinetic(self):
        """Local kinetic energy of every walker at its current positions:
        from the kept Laplacian rows when they are current, else from a fresh
        evaluation at the current positions (which also refreshes them)."""
        W, n, s = self.W, self.n, self.stream
        npos = W * 2 * n
        if self.lap_ok:
            self._call(_b.lib().blip_qs_lap_ratios(npos, n, _b._ptr(self.lap), n,
                                                   _b._ptr(self.inv), n, _b._ptr(self.rl),
                                                   _b._stream_ptr(s)))
        else:
            self.ratio_values(self.pos.view(npos, 3),
                              (self.ratio, self.rg, self.rl, self.val, self.lap))
            self.lap_ok = True
        self._call(_b.lib().blip_qs_kinetic(W, 2 * n, _b._ptr(self.rl), _b._ptr(self.e_kin),
                                           _b._stream_ptr(s)))
        return self.e_kin

    def pbp_sweep(self, eta: torch.Tensor, uniform: torch.Tensor, energy: bool = True):
        """The particle-by-particle comparison (Eq. (11.12.23.0b)): electron g of every
        walker moves alone, g = 0 .. 2n-1, each judged against the state that
        holds the earlier decisions (one masked step per electron; for
        comparisons on small systems, not a fast path)."""
        W, n = self.W, self.n
        # the masked random numbers are written on the walkers' stream, in
        # order with the steps that read them
        with torch.cuda.stream(self.stream if self.stream is not None
                               else torch.cuda.current_stream()):
            inf = torch.full_like(uniform, float("inf"))
            zero = torch.zeros_like(eta)
            for g in range(2 * n):
                e_g = zero.clone()
                e_g[:, g] = eta[:, g]
                u_g = inf.clone()
                u_g[:, g] = uniform[:, g]
                j = g % n
                self.step(e_g, u_g, energy=False, j0=j, j1=j + 1)
        return self.kinetic() if energy else None
