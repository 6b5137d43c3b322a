"""Adaptive-mesh driver around PerkSolver: indicator thresholds -> per-leaf flags -> device
adaptation and re-partition (Sec. 6.2: the partition is rebuilt after every mesh change).

The indicator, the flags by threshold, the adaptation with 2:1 balance, the projection and the
re-partition run in libperk, in one call per cycle (pe_amr_cycle); this module schedules the
cycles.  flags_from_indicator is the same threshold rule for callers that take the indicator
values first (PerkSolver.indicator, then PerkSolver.adapt with their own flags).
"""
import numpy as np

from .partition_rule import LevelRule


def flags_from_indicator(eta, refine_above, coarsen_below):
    f = np.zeros(len(eta), np.int8)
    f[np.asarray(eta) > refine_above] = 1
    f[np.asarray(eta) < coarsen_below] = -1
    return f


class AmrDriver:
    def __init__(self, solver, level_min, level_max, member_of_level, refine_above=0.05, coarsen_below=0.01,
                 interval=10):
        self.s = solver
        self.level_min, self.level_max = level_min, level_max
        # an explicit map, or a LevelRule the library applies at the finest level after each cycle
        self.member_of_level = member_of_level if isinstance(member_of_level, LevelRule) else list(member_of_level)
        self.refine_above, self.coarsen_below = refine_above, coarsen_below
        self.interval = interval
        self.n_adapt = 0

    def adapt_once(self):
        """Indicator, flags, adaptation and re-partition (one library call); returns the flags."""
        flags = self.s.amr_cycle(self.refine_above, self.coarsen_below, self.level_min, self.level_max,
                                 self.member_of_level)
        self.n_adapt += 1
        return flags

    def initial_mesh(self, ic_leaf_fn, passes=3):
        """Refine from the initial condition: set, indicate, adapt, re-evaluate, `passes` times."""
        for _ in range(passes):
            self.s.set_state(ic_leaf_fn(self.s.node_coords().cpu().numpy()))
            self.adapt_once()
        self.s.set_state(ic_leaf_fn(self.s.node_coords().cpu().numpy()))

    def run(self, dt, n_steps, on_step=None):
        """n_steps P-ERK steps, adapting every `interval` steps (without a per-step callback the
        steps between adaptations go to the library in one call)."""
        k = 0
        while k < n_steps:
            chunk = 1 if on_step else n_steps - k
            if self.interval:
                chunk = min(chunk, self.interval - k % self.interval)
            self.s.step(dt, chunk)
            k += chunk
            if on_step:
                on_step(k)
            if self.interval and k % self.interval == 0:
                self.adapt_once()
