"""Berger-Oliger time stepping with subcycling over a refinement hierarchy
(the mesh-refinement part of the Einstein Toolkit paper's framework
section: coarse level first, then two steps of the next finer level, then
the fine solution restricted into the coarse one; fine-grid boundaries
interpolated in space and time).

This module only orders calls: every value is computed by the library
(the RK4 stages of a level's patches, bssn_amr_fill_ghosts for ghost
points, bssn_amr_restrict for the coarse points under a fine patch).
Python keeps the times and rotates the time-level buffers.

A level's stages run either as one batched launch over all of its patches
(batch_patches_stage of a plan per level and time-level rotation, the
default; a level of one patch calls its rk4_stage directly) or as one
rk4_stage per patch (batched=False); both run the same kernel arithmetic,
so the two steppers agree bitwise.

Per level L (spacing h_0 / 2^L, step dt_0 / 2^L) the stepper keeps three
time levels of every patch: the current state and the two before it.  The
ghost points of each RK4 stage input of level L >= 1 are filled at the
stage's time (t, t + dt/2, t + dt/2, t + dt) from the time levels of level
L - 1 (two of them on its first step, three after), and level 0 exchanges
the faces its patches share; level-0 ghosts outside every other patch are
the static physical boundary.  After its step a level's new state gets its
ghosts at the new time, before finer levels interpolate from it.
"""
from . import bssn as B

STAGE_C = (0.0, 0.5, 0.5, 1.0)


class BergerOliger:
    """hier: list of (level, grid); u0: device states (one per patch) at
    t = 0, taken over by the stepper; dt0: the level-0 step."""

    def __init__(self, hier, params, dt0, u0, batched=True):
        import torch
        self.hier = list(hier)
        self.prm = params
        self.dt0 = float(dt0)
        self.nlevel = 1 + max(lv for lv, _ in self.hier)
        self.plan = B.AmrPlan(self.hier)
        self.u = list(u0)
        # static ghosts of level 0 must be the same in every buffer
        self.prev = [t.clone() for t in self.u]
        self.prev2 = [t.clone() for t in self.u]
        self.a = [t.clone() for t in self.u]
        self.b = [t.clone() for t in self.u]
        self.acc = [torch.empty_like(t) for t in self.u]
        self.time = [0.0] * self.nlevel
        self.nsteps = [0] * self.nlevel
        self.batched = batched
        # batch plans per (level, rotation): the three time-level buffers
        # of a patch take turns as u_n and u_{n+1}
        self._plans = {}
        self._rot = [0] * self.nlevel

    def _level(self, L, lst):
        return [t if lv == L else None for (lv, _), t in zip(self.hier, lst)]

    def _coarse_levels(self, L):
        """Time levels of level L - 1 (oldest first) and their times."""
        c = L - 1
        dt = self.dt0 / 2 ** c
        t = self.time[c]
        if self.nsteps[c] >= 2:
            return ([self._level(c, self.prev2), self._level(c, self.prev),
                     self._level(c, self.u)], [t - 2 * dt, t - dt, t])
        return ([self._level(c, self.prev), self._level(c, self.u)],
                [t - dt, t])

    def _fill(self, L, states, t):
        if L == 0:
            self.plan.fill_ghosts(0, states, [], [], t)
        else:
            tabs, ts = self._coarse_levels(L)
            self.plan.fill_ghosts(L, states, tabs, ts, t)

    def _advance(self, L):
        dt = self.dt0 / 2 ** L
        T = self.time[L]
        # rotate: the state at T becomes prev; the oldest buffer is reused
        # for the new state
        for p, (lv, _) in enumerate(self.hier):
            if lv == L:
                self.prev2[p], self.prev[p], self.u[p] = (
                    self.prev[p], self.u[p], self.prev2[p])
        idx = [p for p, (lv, _) in enumerate(self.hier) if lv == L]
        ins = (self.prev, self.a, self.b, self.a)
        outs = (self.a, self.b, self.a, self.u)
        # a level of one patch: its rk4_stage directly (the same kernel
        # arithmetic; a plan's graph launch costs more than it saves there)
        plan = (self._plan(L, idx, dt) if self.batched and len(idx) > 1
                else None)
        for s in range(4):
            self._fill(L, self._level(L, ins[s]), T + STAGE_C[s] * dt)
            if plan is not None:
                B.batch_patches_stage(plan, s)
                continue
            for p in idx:
                g = self.hier[p][1]
                B.rk4_stage(g, self.prm, s, dt, self.prev[p], ins[s][p],
                            self.acc[p], outs[s][p])
        # the new state's ghosts at its time: finer levels interpolate from
        # it (ghosts included) and restriction reads them
        self._fill(L, self._level(L, self.u), T + dt)
        self.time[L] = T + dt
        self.nsteps[L] += 1
        if L + 1 < self.nlevel:
            self._advance(L + 1)
            self._advance(L + 1)
            self.plan.restrict(L + 1, self._level(L + 1, self.u),
                               self._level(L, self.u))

    def _plan(self, L, idx, dt):
        """The batch plan of level L for the current buffer rotation: u_n
        in prev, u_{n+1} into u (stage inputs a, b as the plan's)."""
        key = (L, self._rot[L])
        self._rot[L] = (self._rot[L] + 1) % 3
        plan = self._plans.get(key)
        if plan is None:
            grids = [self.hier[p][1] for p in idx]
            plan = B.batch_patches_plan(
                grids, self.prm, [self.prev[p] for p in idx],
                [self.a[p] for p in idx], [self.b[p] for p in idx],
                [self.acc[p] for p in idx], dt, autotune=0,
                u_new=[self.u[p] for p in idx])
            self._plans[key] = plan
        return plan

    def step(self):
        """One level-0 step (2^L steps of every level L)."""
        self._advance(0)
