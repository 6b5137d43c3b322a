"""Level -> P-ERK member rules: argument marshalling for the library's rules (pe_set_level_rule,
pe_level_map in include/perk.h).  The rules themselves live in libperk:

* PAPER (Sec. 6.4.1): the finest level gets the member with the most stage evaluations, the next
  coarser level the next member, and so on; every level beyond the R finest gets the member with
  the fewest evaluations.
* REQUIRED_STEP: each level gets the cheapest member whose optimal step, scaled with the level's
  element size, still admits the common step of the finest level times a margin.

`LevelRule` is what PerkSolver and the AMR driver accept in place of an explicit map; `level_map`
asks the library for the map of a family at a given finest level (host calls only, no device).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib as L

PAPER = 0
REQUIRED_STEP = 1


@dataclass(frozen=True)
class LevelRule:
    kind: int = PAPER
    dt_opt: tuple | None = None     # [R] optimal steps at a common element size (REQUIRED_STEP)
    margin: float = 1.0

    @staticmethod
    def paper():
        return LevelRule(PAPER)

    @staticmethod
    def required_step(dt_opt, margin=1.0):
        return LevelRule(REQUIRED_STEP, tuple(float(x) for x in dt_opt), float(margin))

    def label(self):
        return "paper rule (Sec. 6.4.1)" if self.kind == PAPER else f"required-step rule, margin {self.margin:g}"


def set_rule(lib, ctx, rule: LevelRule):
    """pe_set_level_rule on an existing context (coefficients already set)."""
    dt = None
    if rule.kind == REQUIRED_STEP:
        arr = np.ascontiguousarray(rule.dt_opt, dtype=np.float64)
        dt = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return lib.pe_set_level_rule(ctx, int(rule.kind), dt, float(rule.margin))


def level_map(family, rule: LevelRule, finest_level, n_levels=None):
    """member_of_level[0..n_levels) of `family` under `rule` for a mesh whose finest level is
    finest_level, computed by the library on a host-only context."""
    lib = L.lib()
    n_levels = finest_level + 1 if n_levels is None else n_levels
    ctx = ctypes.c_void_p()
    phys = L.pe_physics(2, 3, 0, 1.4, 0.0, 0.72)
    st = lib.pe_create(ctypes.byref(ctx), ctypes.byref(phys))
    if st != L.PE_OK:
        raise RuntimeError(f"pe_create: {L.STATUS.get(st, st)}")
    try:
        E = np.ascontiguousarray(np.asarray(family.E, dtype=np.int32))
        c = np.ascontiguousarray(family.c, dtype=np.float64)
        b = np.ascontiguousarray(family.b, dtype=np.float64)
        a = np.ascontiguousarray(np.asarray(family.a_sub, dtype=np.float64).reshape(len(E), -1))
        co = L.pe_perk_coeffs(int(family.order), len(E), int(family.S),
                              E.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        out = np.zeros(n_levels, np.int32)
        for what, st in (("pe_set_perk_coefficients", lambda: lib.pe_set_perk_coefficients(ctx, ctypes.byref(co))),
                         ("pe_set_level_rule", lambda: set_rule(lib, ctx, rule)),
                         ("pe_level_map", lambda: lib.pe_level_map(ctx, int(finest_level), int(n_levels),
                                                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))):
            code = st()
            if code != L.PE_OK:
                raise RuntimeError(f"{what}: {L.STATUS.get(code, code)}: {lib.pe_last_error(ctx).decode()}")
        return [int(x) for x in out]
    finally:
        lib.pe_destroy(ctx)
