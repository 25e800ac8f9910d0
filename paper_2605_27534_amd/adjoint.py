"""Gradients of a surface-tension-history misfit through libsurf's discrete
adjoint, behind a torch.autograd.Function with checkpointed recomputation.

L(theta, c0) = (1/N) sum_{n=1..N} (<sigma>^n - target^n)^2, theta = (k_a, k_d,
D_b, D_s), F^0 = c0 phi, psi^0 = gamma0 delta.  The forward run keeps the
state every K steps; the backward pass replays each K-step segment from its
checkpoint (storing the K states and, on the 3D plane-marching transport, the
advected state of each step, which the adjoint step then reads instead of
advecting again) and runs the adjoint steps over it in reverse.  Every step,
adjoint step, loss weight and seed is a libsurf kernel; torch only holds the
buffers.
"""
from __future__ import annotations

import torch

from . import surf as S


class Rollout:
    """A static-interface problem set up for adjoint runs."""

    def __init__(self, prob: dict, dt: float, precision=S.SURF_F32, vof=None, chi=None,
                 u=None, gamma0=0.0, nsteps=10, checkpoint=50):
        p = dict(prob)
        p["adjoint"] = 1
        self.s = S.Surf(p, dt, precision)
        if chi is not None:
            self.s.set_levelset(self.s.tensor(chi))
        else:
            self.s.set_geometry(self.s.tensor(vof), full=True)
        self.u = None if u is None else [self.s.tensor(x) for x in u]
        self.gamma0 = float(gamma0)
        self.N = int(nsteps)
        self.K = max(1, int(checkpoint))
        self.bulk = bool(self.s.params.bulk_enabled)
        # whether the recomputation keeps each step's advected state for the
        # adjoint (3D plane-marching transport only; settled on first use)
        self.keep_advected = None
        self._seg = None  # the recomputation's buffers, reused over segments

    # one forward step from (F, P) into fresh buffers
    def _step(self, F, P, tot_row):
        F2 = self.s.empty() if F is not None else None
        P2 = self.s.empty()
        self.s.step(F, P, F2, P2, u=self.u, totals=tot_row)
        return F2, P2

    def _recompute_advected(self, F, P, k, states, scratch):
        """Replays k steps from (F, P), appending the states after steps
        1..k-1 to `states` and returning the advected state of each step;
        None (and nothing appended) where the context has no such step."""
        if self.keep_advected is False:
            return None
        s = self.s
        if self._seg is None or self._seg[0] < k:
            # states after steps 1..k (the last one unused) and the k advected
            # states, allocated once: each segment's adjoint steps are queued
            # before the next segment's recomputation overwrites them
            def block(on):
                return torch.empty((k,) + tuple(s.shape), dtype=s.dtype,
                                   device=s.device) if on else None
            self._seg = (k, block(F is not None), block(True), block(F is not None), block(True))
        _, bF, bP, sF, sP = self._seg
        stars = []
        for i in range(k):
            F2 = bF[i] if F is not None else None
            P2 = bP[i]
            st = (sF[i] if F is not None else None, sP[i])
            try:
                s.step(F, P, F2, P2, u=self.u, totals=scratch, star=st)
            except S.SurfError as e:
                if i or e.code != -1 or self.keep_advected:
                    raise
                self.keep_advected = False
                return None
            self.keep_advected = True
            stars.append(st)
            if i + 1 < k:
                states.append((F2, P2))
            F, P = F2, P2
        return stars

    def forward(self, theta, c0, target, keep=None):
        """Returns (loss [device scalar], totals [N,16], checkpoints dict)."""
        s = self.s
        th = [float(v) for v in theta.detach().cpu().tolist()]
        s.set_kinetics(*th)
        F, P = s.init_state(c0.detach().to(s.dtype).contiguous(), 1.0, self.gamma0)
        tot = torch.zeros((self.N, 16), dtype=torch.float64, device=s.device)
        ck = {0: (F, P)}
        for n in range(self.N):
            F, P = self._step(F, P, tot[n])
            if (n + 1) % self.K == 0 or n + 1 == self.N:
                ck[n + 1] = (F, P)
        w = torch.empty(self.N, dtype=torch.float64, device=s.device)
        loss = torch.empty(1, dtype=torch.float64, device=s.device)
        s.loss_weights(tot, target.to(torch.float64).contiguous(), w, loss)
        return loss[0], tot, w, ck

    def backward(self, w, ck, tot=None):
        """dL/dtheta (4, float64) and dL/dc0 (field) from the checkpoints; tot
        (the forward's totals) restores each segment's starting time, so that
        the recomputed states are the forward's bit for bit."""
        s = self.s
        dth = torch.zeros(4, dtype=torch.float64, device=s.device)
        FN, PN = ck[self.N]
        lF, lP = s.empty(), s.empty()
        nF, nP = s.empty(), s.empty()  # lambda^n, then swapped with lambda^{n+1}
        s.adjoint_seed(PN, w[self.N - 1:self.N], lF, lP)
        scratch = torch.zeros(16, dtype=torch.float64, device=s.device)
        starts = sorted(k for k in ck if k < self.N)
        for s0 in reversed(starts):
            s1 = min(s0 + self.K, self.N)
            states = [ck[s0]]
            F, P = ck[s0]
            s.set_time(tot[s0 - 1, 11:12] if (tot is not None and s0 > 0) else None)
            stars = self._recompute_advected(F, P, s1 - s0, states, scratch)
            if stars is None:
                for n in range(s0, s1 - 1):
                    F, P = self._step(F, P, scratch)
                    states.append((F, P))
            for n in range(s1 - 1, s0 - 1, -1):
                Fn, Pn = states[n - s0]
                wn = w[n - 1:n] if n >= 1 else None
                s.adjoint_step(Fn if self.bulk else None, Pn, lF, lP, nF, nP, dth, u=self.u, w=wn,
                               star=None if stars is None else stars[n - s0])
                lF, lP, nF, nP = nF, nP, lF, lP
        gc0 = s.adjoint_c0(lF)
        return dth, gc0


class SurfRollout(torch.autograd.Function):
    """loss = SurfRollout.apply(theta, c0, rollout, target)."""

    @staticmethod
    def forward(ctx, theta, c0, rollout, target):
        loss, tot, w, ck = rollout.forward(theta, c0, target)
        ctx.rollout = rollout
        ctx.saved = (w, ck, tot)
        ctx.c0_dtype = c0.dtype
        ctx.theta_dtype = theta.dtype
        return loss.clone()

    @staticmethod
    def backward(ctx, g):
        w, ck, tot = ctx.saved
        dth, gc0 = ctx.rollout.backward(w, ck, tot)
        g = g.to(torch.float64)
        return (dth * g).to(ctx.theta_dtype), (gc0.to(torch.float64) * g).to(ctx.c0_dtype), None, None
