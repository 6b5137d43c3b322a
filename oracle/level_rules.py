"""Oracle: which P-ERK member integrates the elements of each refinement level.

Test infrastructure only (see oracle/__init__.py).  Written from the paper, independently of
the library's rules:

* paper_rule -- Sec. 6.4.1 (Actual Number of Right-Hand-Side Evaluations): the finest level is
  integrated with the method of most stage evaluations, the second finest with the next one,
  and so on; when there are more levels than methods every remaining coarse level gets the
  method with the fewest evaluations (the paper's example: six levels and E = {3, 6, 12} give
  12, 6, 3, 3, 3, 3 from fine to coarse).
* required_step_rule -- a variant driven by step sizes.  For convection-dominated problems the
  spectrum grows like 1/h (Sec. 3.1), so a method whose optimised step at the finest element size
  h_min is dt_opt admits dt_opt * h / h_min on elements of size h.  All levels advance with the
  common step of the finest level's method of most evaluations; every coarser level takes, among
  the methods that admit that step times a safety margin, the one with the fewest stage
  evaluations (the largest method when none does).  Parity pinned by hand-derived maps and by
  the closed form below (tests/test_oracle_level_rules.py).
"""
from __future__ import annotations


def paper_rule(finest_level: int, n_members: int, n_levels: int | None = None) -> list[int]:
    """Member index (0 = fewest evaluations) per level 0..n_levels-1; levels finer than the
    finest level take the largest member."""
    n_levels = finest_level + 1 if n_levels is None else n_levels
    out = []
    for level in range(n_levels):
        rank_from_finest = finest_level - level        # 0 for the finest level
        if rank_from_finest <= 0:
            out.append(n_members - 1)
        elif rank_from_finest < n_members:
            out.append(n_members - 1 - rank_from_finest)
        else:
            out.append(0)
    return out


def required_step_rule(finest_level: int, E, dt_opt, margin: float = 1.0,
                       n_levels: int | None = None) -> list[int]:
    """Member index per level (E ascending, dt_opt[r] the optimal step of member r at the finest
    element size)."""
    n_levels = finest_level + 1 if n_levels is None else n_levels
    largest = max(range(len(E)), key=lambda r: E[r])
    dt_common = dt_opt[largest]
    out = []
    for level in range(n_levels):
        if level >= finest_level:
            out.append(largest)
            continue
        h_ratio = 2.0 ** (finest_level - level)          # h_level / h_min on a quad/octree
        admissible = [r for r in range(len(E)) if dt_opt[r] * h_ratio >= margin * dt_common * (1 - 1e-12)]
        out.append(min(admissible, key=lambda r: E[r]) if admissible else largest)
    return out
