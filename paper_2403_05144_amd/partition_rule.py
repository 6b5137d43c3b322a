"""Level -> P-ERK member maps.

paper_rule (Sec. 6.3.1): the finest level gets the member with the most stage evaluations,
the next finer level the next member, and so on; when there are more levels than members every
remaining coarse level gets the member with the fewest evaluations.

required_dt_rule: each level gets the cheapest member whose optimal step, scaled with the
level's element size (convection-dominated spectra scale with 1/h, Sec. 3.1), still admits the
common step set by the finest level, times a safety margin.  With margin 1 it coincides with
paper_rule when the optimal step doubles from member to member.  A margin above 1 keeps the
coarser members away from their own stability limit: at the boundaries between members the
partitioned scheme is not monotone (Sec. 5), and for inviscid flow a member running close to its
limit next to a finer level can force the common step down (Sec. 7: the CFL reductions reported
for the hyperbolic cases); the finest level always takes the largest member.
"""
import numpy as np


def paper_rule(level_max, n_members):
    return [max(0, (n_members - 1) - (level_max - l)) for l in range(level_max + 1)]


def required_dt_rule(level_max, dt_opt, E, margin=1.0, rel_tol=1e-12):
    dt_common = dt_opt[-1]                 # finest level, E_max member, element size h_min
    out = []
    for l in range(level_max + 1):
        scale = 2.0 ** (level_max - l)     # element size relative to h_min
        need = dt_common * (margin if l < level_max else 1.0) * (1 - rel_tol)
        r = next((k for k in range(len(E)) if dt_opt[k] * scale >= need), len(E) - 1)
        out.append(r)
    return out
