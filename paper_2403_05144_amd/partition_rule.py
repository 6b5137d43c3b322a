"""Level -> P-ERK member maps.

paper_rule (Sec. 6.3.1): the finest level gets the member with the most stage evaluations,
the next finer level the next member, and so on; when there are more levels than members every
remaining coarse level gets the member with the fewest evaluations.

required_dt_rule: each level gets the cheapest member whose optimal step, scaled with the
level's element size (convection-dominated spectra scale with 1/h, Sec. 3.1), still admits the
common step set by the finest level.  It coincides with paper_rule when the optimal step
doubles from member to member.
"""
import numpy as np


def paper_rule(level_max, n_members):
    return [max(0, (n_members - 1) - (level_max - l)) for l in range(level_max + 1)]


def required_dt_rule(level_max, dt_opt, E, rel_tol=1e-12):
    dt_common = dt_opt[-1]                 # finest level, E_max member, element size h_min
    out = []
    for l in range(level_max + 1):
        scale = 2.0 ** (level_max - l)     # element size relative to h_min
        r = next(k for k in range(len(E)) if dt_opt[k] * scale >= dt_common * (1 - rel_tol))
        out.append(r)
    return out
