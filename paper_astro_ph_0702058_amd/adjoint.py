"""Gradients of shared-step Hermite runs through the library's hand-written adjoint.

`HermiteRun.apply(x0, v0, m, runner)` integrates `runner.nsteps` shared steps of size
`runner.dt` from (x0, v0) with masses m (all (3, n) / (n,) float64 CUDA tensors, structure of
arrays) and returns the final positions and velocities.  Its backward pass recomputes the
trajectory from checkpoints kept every `runner.checkpoint_every` steps and applies
nb_step_vjp step by step in reverse, then the VJP of the initial force evaluation
(a0, k0 = F(x0, v0, m)); all arithmetic runs in the library's kernels.  With overlap (the
default) a second context recomputes the next segment on a stream of its own while the
step VJPs of the current one run, which changes no result: the same kernels see the same
inputs.
"""
from __future__ import annotations

import torch

from . import nbody


class SharedRunner:
    """A context and device state for differentiable shared-step runs of n particles."""

    def __init__(self, n, eps, dt, nsteps, checkpoint_every=8, precision="fp32", lmin=0,
                 overlap=True):
        self.n, self.eps, self.dt = int(n), float(eps), float(dt)
        self.nsteps, self.checkpoint_every = int(nsteps), int(checkpoint_every)
        self.ctx = nbody.Context(self.n, self.eps, lmin=lmin, lmax=26, precision=precision)
        z = torch.zeros((self.n, 3), dtype=torch.float64)
        self.state = nbody.DeviceState(z.numpy(), z.numpy(), torch.ones(self.n).numpy())
        self.ctx.nb_bind(self.state)
        self.t0 = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.overlap = bool(overlap)
        if self.overlap:  # the recomputation's own context, state and stream (default priority)
            self.rstream = torch.cuda.Stream()
            self.rctx = nbody.Context(self.n, self.eps, lmin=lmin, lmax=26, precision=precision,
                                      stream=self.rstream)
            self.rstate = nbody.DeviceState(z.numpy(), z.numpy(), torch.ones(self.n).numpy())
            self.rctx.nb_bind(self.rstate)

    def _load(self, x, v):
        st = self.state
        st.x.copy_(x); st.v.copy_(v)

    def _restore(self, snap):
        self.state.xvak.copy_(snap)  # x, v, a, k in one copy

    def _snapshot(self):
        return self.state.xvak.clone()

    def forward(self, x0, v0, m):
        """Run from (x0, v0, m); returns (x, v) at the end and the checkpoints."""
        st = self.state
        st.m.copy_(m)
        self._load(x0, v0)
        self.ctx.nb_init(0.01)           # a0, k0 = F(x0, v0, m); times 0
        checkpoints = []
        done = 0
        while done < self.nsteps:
            checkpoints.append(self._snapshot())
            k = min(self.checkpoint_every, self.nsteps - done)
            self.ctx.nb_shared_step(self.dt, k)
            done += k
        self.ctx.nb_sync()
        return st.x.clone(), st.v.clone(), checkpoints

    def backward(self, x0, v0, m, checkpoints, gx, gv):
        """Adjoints (x0_bar, v0_bar, m_bar) from those of the final positions and velocities."""
        n = self.n
        xb = gx.clone(memory_format=torch.contiguous_format) if gx is not None else torch.zeros((3, n), dtype=torch.float64, device="cuda")
        vb = gv.clone(memory_format=torch.contiguous_format) if gv is not None else torch.zeros((3, n), dtype=torch.float64, device="cuda")
        ab = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        kb = torch.zeros_like(ab)
        mb = torch.zeros(n, dtype=torch.float64, device="cuda")
        self.state.m.copy_(m)
        seg_len = [min(self.checkpoint_every, self.nsteps - s * self.checkpoint_every)
                   for s in range(len(checkpoints))]
        if self.overlap:
            self._backward_overlapped(checkpoints, seg_len, m, xb, vb, ab, kb, mb)
        else:
            for seg in reversed(range(len(checkpoints))):
                # recompute the states before each step of the segment
                self._restore(checkpoints[seg])
                states = [checkpoints[seg]]
                for _ in range(seg_len[seg] - 1):
                    self.ctx.nb_shared_step(self.dt, 1)
                    states.append(self._snapshot())
                for s in reversed(states):
                    self._restore(s)
                    self.ctx.nb_step_vjp(self.dt, xb, vb, ab, kb, mb)
        # the initial force a0, k0 = F(x0, v0, m)
        self._load(x0, v0)
        self.state.tick.zero_()
        self.ctx.nb_predict(self.t0)
        self.ctx.nb_force_vjp(ab, kb, xb, vb, mb)
        self.ctx.nb_sync()
        if self.overlap:
            self.rctx.nb_sync()  # a flag the recomputation latched is reported here
        return xb, vb, mb


    def _backward_overlapped(self, checkpoints, seg_len, m, xb, vb, ab, kb, mb):
        """The segments' step VJPs on the main context's stream, each segment's states
        recomputed by the second context on its stream one segment ahead."""
        cur, rs = torch.cuda.current_stream(), self.rstream
        rs.wait_stream(cur)  # the checkpoints and m are ready
        with torch.cuda.stream(rs):
            self.rstate.m.copy_(m)

        def recompute(seg):
            with torch.cuda.stream(rs):
                checkpoints[seg].record_stream(rs)
                self.rstate.xvak.copy_(checkpoints[seg])
                states = [checkpoints[seg]]
                for _ in range(seg_len[seg] - 1):
                    self.rctx.nb_shared_step(self.dt, 1)
                    states.append(self.rstate.xvak.clone())
                ready = torch.cuda.Event()
                ready.record(rs)
            return states, ready

        order = list(reversed(range(len(checkpoints))))
        ahead = recompute(order[0])
        for i in range(len(order)):
            states, ready = ahead
            if i + 1 < len(order):
                ahead = recompute(order[i + 1])  # overlaps the VJPs below
            cur.wait_event(ready)
            for s in reversed(states):
                s.record_stream(cur)  # made on the recompute stream, read here
                self._restore(s)
                self.ctx.nb_step_vjp(self.dt, xb, vb, ab, kb, mb)


class HermiteRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, m, runner: SharedRunner):
        x, v, cps = runner.forward(x0, v0, m)
        ctx.runner = runner
        ctx.cps = cps
        ctx.save_for_backward(x0, v0, m)
        return x, v

    @staticmethod
    def backward(ctx, gx, gv):
        x0, v0, m = ctx.saved_tensors
        xb, vb, mb = ctx.runner.backward(x0, v0, m, ctx.cps, gx, gv)
        return xb, vb, mb, None
