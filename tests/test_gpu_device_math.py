"""GPU: the kernels' own arithmetic routines (node logarithms of the logarithmic means of the
entropy-conserving volume flux, sound-speed square roots of the HLL wave speeds, reciprocals)
against correctly rounded values, through pe_device_math.

The references are computed with Python's decimal module at 40 significant digits from the
exact binary value of each argument, then rounded once to the nearest double.  Bounds: the
square root is correctly rounded, the reciprocal within 1 ulp, the logarithm within 2 ulp."""
import ctypes
import decimal

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ulps(a, b):
    """Distance in units in the last place between doubles of equal sign."""
    ia = np.asarray(a, np.float64).view(np.int64)
    ib = np.asarray(b, np.float64).view(np.int64)
    # map the sign-magnitude bit patterns onto a monotone integer line
    ia = np.where(ia < 0, np.int64(-(2 ** 63)) - ia, ia)
    ib = np.where(ib < 0, np.int64(-(2 ** 63)) - ib, ib)
    return np.abs(ia - ib)


def _reference(x):
    ctx = decimal.Context(prec=40)
    ln, sq, rc = [], [], []
    for v in x.tolist():
        d = decimal.Decimal(v)               # exact value of the double
        ln.append(float(str(d.ln(ctx))))     # one rounding from 40 digits to the nearest double
        sq.append(float(str(d.sqrt(ctx))))
        rc.append(float(str(ctx.divide(1, d))))
    return np.array(ln), np.array(sq), np.array(rc)


def _arguments(seed=2403051440):
    rng = np.random.default_rng(seed)
    parts = [
        2.0 ** rng.uniform(-30, 30, 20000),                       # wide range (densities, 1/T, speeds^2)
        np.sqrt(0.5) * (1 + rng.uniform(-1e-6, 1e-6, 2000)) * 2.0 ** rng.integers(-8, 8, 2000),
        1 + rng.uniform(-1e-3, 1e-3, 2000),                       # near 1: log close to 0
        1 + rng.uniform(-1e-12, 1e-12, 500),
        2.0 ** np.arange(-20, 21, dtype=np.float64),               # exact powers of two
        np.array([1.0, 0.5, 2.0, 3.0, 10.0, 1.4, 71.42857142857143, np.nextafter(1.0, 2.0),
                  np.nextafter(1.0, 0.0), np.sqrt(0.5), np.nextafter(np.sqrt(0.5), 0.0)]),
    ]
    return np.concatenate(parts)


def test_device_math_against_correctly_rounded_values():
    import torch
    from paper_2403_05144_amd import PerkSolver
    import perk_inputs as pin
    from oracle import perk_coeffs as pc
    s = PerkSolver(pin.mesh_vortex_2level(), 3, pc.perk2_family([4, 8]), [0, 1])
    x = _arguments()
    n = x.size
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    out = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    print(f"device_math: {n} arguments", flush=True)
    st = s.lib.pe_device_math(s._ctx, ctypes.c_void_p(xd.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(3, n)
    ln, sq, rc = _reference(x)
    u_ln, u_sq, u_rc = _ulps(got[0], ln), _ulps(got[1], sq), _ulps(got[2], rc)
    print(f"max ulp: log {u_ln.max()}, sqrt {u_sq.max()}, rcp {u_rc.max()}", flush=True)
    # ln 1 = 0 exactly
    assert got[0][x == 1.0].tolist() == [0.0] * int(np.sum(x == 1.0))
    assert u_sq.max() == 0, x[np.argmax(u_sq)]
    assert u_rc.max() <= 1, x[np.argmax(u_rc)]
    assert u_ln.max() <= 2, x[np.argmax(u_ln)]
    # zero and negative arguments of the logarithm give NaN (non-physical states stay visible)
    bad = torch.tensor([0.0, -1.0], dtype=torch.float64, device="cuda")
    ob = torch.empty(6, dtype=torch.float64, device="cuda")
    assert s.lib.pe_device_math(s._ctx, ctypes.c_void_p(bad.data_ptr()), 2, ctypes.c_void_p(ob.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
    torch.cuda.synchronize()
    assert np.all(np.isnan(ob.cpu().numpy()[:2]))
    assert s.lib.pe_device_math(s._ctx, None, -1, None, None) == -1
