"""Writes the P-ERK families used as inputs by the parity tests.  Calls only oracle/.

Families are optimised on the unit disk spectrum {-1 + e^{i theta}} (eq. OptimizationProblem)
and constructed with the oracle's tableau code (Sec. 4.3); any valid family serves parity.
Run: python tests/golden/make_coeffs.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import perk_coeffs as pc  # noqa: E402


def disk():
    th = np.linspace(0, np.pi, 150)
    return -1.0 + np.exp(1j * th)


def write(name, fam, dts):
    d = fam.to_json()
    d["dt_opt_unit_disk"] = [float(x) for x in dts]
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(d, f, indent=1)


if __name__ == "__main__":
    lam = disk()
    for E_list in ([4, 6, 8, 12, 16], [4, 8, 16]):
        res = {E: pc.optimize_alpha(lam, 3, E) for E in E_list}
        fam = pc.perk3_family(E_list, {E: r[1] for E, r in res.items()})
        assert np.max(np.abs(pc.order_condition_residuals(fam))) < 1e-12
        write("perk3_" + "_".join(map(str, E_list)) + "_disk.json", fam, [res[E][0] for E in E_list])
    for E_list in ([4, 8, 16],):
        fam = pc.perk2_family(E_list)
        write("perk2_" + "_".join(map(str, E_list)) + "_disk.json", fam, [E - 1.0 for E in E_list])
