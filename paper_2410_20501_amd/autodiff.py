"""Differentiable particle-mesh runs: torch.autograd.Function wrappers of the
reverse-mode entry points (argument marshalling and checkpoint bookkeeping only;
every step runs in libhippm.so kernels).

A run from a displacement field psi at lattice points q is
    (x0, v0) = (wrap(q + psi), a0^(1/2) psi)          Zel'dovich state, Sect. 3.3
    (x_{i+1}, v_{i+1}) = KDK(x_i, v_i; a_i -> a_{i+1})    leapfrog, Sect. 3.4
and the gradient of a loss of the final state comes back through the
transposed leapfrog. The forward pass keeps (x, v, acc, phi) only every
`checkpoint_every` steps and at the end; the backward pass re-runs each segment
from its checkpoint but for its last step, whose end state is the next checkpoint
(bitwise identical with the sorted deposit, since the multigrid warm start is part
of the checkpoint), keeping the positions and potentials of the segment, and
reverses it step by step with pm_kdk_adjoint. The second kick
of one reversed step and the first kick of the step before act on the same
positions and cotangent, so they are merged: a run of N steps costs N + 1
transposed force evaluations.
"""
from __future__ import annotations

import torch

from . import hippm as _pm


class Run:
    """Settings of a differentiable run: context, scale factors, step parameters.

    poskind "box" keeps box-unit FP32 positions; "celloff" keeps the in-cell offset
    and an int32 cell index (positions resolved to 2^-24 of a cell instead of 2^-24
    of the box). Gradients are with respect to box-unit quantities in both forms.

    warm: the forward steps' multigrid guess. "warm_rescaled" (the default) keeps the
    warm start inside the checkpointed state, so a recomputed segment replays the forward
    pass bitwise; "extrapolated" also draws on the solves of earlier steps, which a
    recomputation from a checkpoint does not see, so the replay can differ at the level of
    the solver tolerance.
    adj_tol: truncation-error tolerance of the transposed (adjoint) Poisson solves. The
    forward FP32 solves leave potentials accurate to about 1e-6 relative, and the adjoint
    source is built from them; at 1e-5 the gradient moves by about 1e-6 relative from its
    value at 1e-6 and the adjoint solves take one to two V-cycles fewer.
    """

    def __init__(self, n, np_, a_list, mas="tsc", order="sorted", solver="mg", tol=1e-6,
                 max_cycles=40, fixed_cycles=0, checkpoint_every=4, warm="warm_rescaled",
                 poskind="box", adj_tol=1e-5):
        if checkpoint_every < 1:
            raise ValueError("checkpoint_every must be >= 1")
        if poskind not in ("box", "celloff"):
            raise ValueError("poskind must be 'box' or 'celloff'")
        self.n = int(n)
        self.np = int(np_)
        self.a = [float(a) for a in a_list]
        self.k = int(checkpoint_every)
        self.mas = mas
        self.celloff = poskind == "celloff"
        self.ctx = _pm.Context(self.n, self.np)
        common = dict(mas=mas, order=order, solver=solver, tol=tol, max_cycles=max_cycles,
                      fixed_cycles=fixed_cycles)
        self.first = _pm.default_step_params(guess="jacobi", **common)
        self.step = _pm.default_step_params(guess=warm, **common)
        self.adj = _pm.default_step_params(guess="jacobi", **dict(common, tol=adj_tol))
        self.stats = {"forward_steps": 0, "recomputed_steps": 0, "adjoint_evals": 0}

    @property
    def nsteps(self):
        return len(self.a) - 1

    def close(self):
        self.ctx.close()

    def _cell(self, cell):
        return cell if self.celloff else None

    # -- forward pieces -------------------------------------------------------------
    def initial_state(self, psi, q):
        pos = torch.empty_like(psi)
        vel = torch.empty_like(psi)
        cell = torch.empty(psi.shape[0] if self.celloff else 0, dtype=torch.int32,
                           device=psi.device)
        _pm.pm_ic_state(self.ctx, q, psi, self.a[0], pos, vel, cell=self._cell(cell))
        return pos, vel, cell

    def start(self, pos, cell):
        phi = torch.zeros((self.n,) * 3, device=pos.device)
        acc = torch.empty_like(pos)
        _pm.pm_accel(self.ctx, pos, self.a[0], phi, acc, cell=self._cell(cell), params=self.first)
        return phi, acc

    def advance(self, pos, vel, cell, phi, acc, i):
        _pm.pm_kdk(self.ctx, pos, vel, self.a[i], self.a[i + 1], phi, acc, cell=self._cell(cell),
                   params=self.step)

    def loss(self, pos, cell, w, pos_bar=None, want_loss=True):
        return _pm.pm_density_loss(self.ctx, pos, w, pos_bar=pos_bar, cell=self._cell(cell),
                                   mas=self.mas, want_loss=want_loss)


class ZeldovichIC(torch.autograd.Function):
    """psi -> (x0, v0, cell0): x0 = wrap(q + psi), v0 = a0^(1/2) psi (cell0: int32 cell
    indices in the cell-offset form, an empty tensor in the box form)."""

    @staticmethod
    def forward(ctx, psi, q, run: Run):
        pos, vel, cell = run.initial_state(psi.detach().contiguous(), q.contiguous())
        ctx.run = run
        ctx.mark_non_differentiable(cell)
        return pos, vel, cell

    @staticmethod
    def backward(ctx, pos_bar, vel_bar, _cell_bar):
        run = ctx.run
        ref = pos_bar if pos_bar is not None else vel_bar
        pos_bar = torch.zeros_like(ref) if pos_bar is None else pos_bar.contiguous()
        vel_bar = torch.zeros_like(ref) if vel_bar is None else vel_bar.contiguous()
        psi_bar = torch.empty_like(ref)
        _pm.pm_ic_vjp(run.ctx, pos_bar, vel_bar, run.a[0], psi_bar)
        return psi_bar, None, None


class Trajectory(torch.autograd.Function):
    """(x0, v0) -> (x_N, v_N) through N KDK steps, checkpointed every k steps."""

    @staticmethod
    def forward(ctx, pos0, vel0, cell0, run: Run):
        pos = pos0.detach().clone().contiguous()
        vel = vel0.detach().clone().contiguous()
        cell = cell0.clone()
        phi, acc = run.start(pos, cell)
        snap = lambda: tuple(t.clone() for t in (pos, vel, cell, phi, acc))  # noqa: E731
        checkpoints = {0: snap()}
        for i in range(run.nsteps):
            run.advance(pos, vel, cell, phi, acc, i)
            run.stats["forward_steps"] += 1
            # every k-th state, and the final one: the state at the end of a segment is
            # the next checkpoint, so the backward pass recomputes k - 1 steps per segment
            if (i + 1) % run.k == 0 or i + 1 == run.nsteps:
                checkpoints[i + 1] = snap()
        ctx.run = run
        ctx.checkpoints = checkpoints
        ctx.mark_non_differentiable(cell)
        return pos, vel, cell

    @staticmethod
    def backward(ctx, pos_bar, vel_bar, _cell_bar):
        run, cps = ctx.run, ctx.checkpoints
        a = run.a
        nsteps = run.nsteps
        ref = pos_bar if pos_bar is not None else vel_bar
        xbar = torch.zeros_like(ref) if pos_bar is None else pos_bar.detach().clone().contiguous()
        vbar = torch.zeros_like(ref) if vel_bar is None else vel_bar.detach().clone().contiguous()
        starts = sorted(t for t in cps if t < nsteps)
        for seg, s0 in reversed(list(enumerate(starts))):
            s1 = starts[seg + 1] if seg + 1 < len(starts) else nsteps
            states = [(cps[s0][0], cps[s0][2], cps[s0][3])]  # (pos, cell, phi) at s0
            pos, vel, cell, phi, acc = (t.clone() for t in cps[s0])
            for i in range(s0, s1 - 1):
                run.advance(pos, vel, cell, phi, acc, i)
                run.stats["recomputed_steps"] += 1
                states.append((pos.clone(), cell.clone(), phi.clone()))
            # the segment's last step ends at the next checkpoint (bitwise the state the
            # recomputation would give: the sorted deposit and the warm starts replay)
            states.append((cps[s1][0], cps[s1][2], cps[s1][3]))
            for i in reversed(range(s0, s1)):
                # the closing term of step i was merged into the opening term of step i + 1
                # (same positions, same cotangent), except for the last step
                merged = i < nsteps - 1
                x0, c0, phi0 = states[i - s0]
                x1, c1, phi1 = states[i + 1 - s0]
                _pm.pm_kdk_adjoint(run.ctx, x0, phi0, x1, phi1, a[i], a[i + 1], xbar, vbar,
                                   a_prev=a[i - 1] if i > 0 else 0.0, closing_merged=merged,
                                   cell0=run._cell(c0), cell1=run._cell(c1), params=run.adj)
                run.stats["adjoint_evals"] += 1 + (0 if merged else 1)
            del states
        return xbar, vbar, None, None


class DensityLoss(torch.autograd.Function):
    """x -> L = sum_c w_c (rho_c(x) - 1)^2 (FP64 scalar)."""

    @staticmethod
    def forward(ctx, pos, cell, w, run: Run):
        pos = pos.detach().contiguous()
        loss = run.loss(pos, cell, w)
        ctx.save_for_backward(pos, cell, w)
        ctx.run = run
        return torch.tensor(loss, dtype=torch.float64, device=pos.device)

    @staticmethod
    def backward(ctx, grad):
        pos, cell, w = ctx.saved_tensors
        run = ctx.run
        pos_bar = torch.zeros_like(pos)
        run.loss(pos, cell, w, pos_bar=pos_bar, want_loss=False)
        if float(grad) != 1.0:
            pos_bar.mul_(float(grad))  # chain-rule scaling by an upstream factor
        return pos_bar, None, None, None


def density_loss_of_ics(psi, q, w, run: Run):
    """L(psi) for the Zel'dovich run described by `run`; differentiable in psi."""
    x0, v0, c0 = ZeldovichIC.apply(psi, q, run)
    xn, _, cn = Trajectory.apply(x0, v0, c0, run)
    return DensityLoss.apply(xn, cn, w, run)


def loss_and_gradient(psi, q, w, run: Run):
    """(L, dL/dpsi) with the hand-written adjoint."""
    psi = psi.detach().clone().requires_grad_(True)
    loss = density_loss_of_ics(psi, q, w, run)
    loss.backward()
    return float(loss), psi.grad


def loss_only(psi, q, w, run: Run):
    """L(psi) without recording anything for the backward pass."""
    with torch.no_grad():
        pos, vel, cell = run.initial_state(psi.contiguous(), q.contiguous())
        phi, acc = run.start(pos, cell)
        for i in range(run.nsteps):
            run.advance(pos, vel, cell, phi, acc, i)
        return run.loss(pos, cell, w)
