"""libperk host side on the CPU: the library loads, exports every symbol of include/perk.h, and
its host-only entry points (mesh build, coefficient validation, call order) behave as
documented.  No device work is started here."""
import ctypes
import os
import re

import numpy as np
import pytest

import perk_inputs as pin
from oracle import perk_coeffs as pc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2403_05144_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libperk.so not built")
    return L, L.lib()


def test_exports_match_header():
    L, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "perk.h")).read()
    declared = set(re.findall(r"\b(pe_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name)


def _ctx(L, lib, dim=2, degree=3, eq=0):
    ctx = ctypes.c_void_p()
    phys = L.pe_physics(dim, degree, eq, 1.4, 1e-3, 0.72)
    assert lib.pe_create(ctypes.byref(ctx), ctypes.byref(phys)) == 0
    return ctx


def _mesh_desc(L, mesh):
    leaves = np.ascontiguousarray(mesh.leaves, dtype=np.int32)
    nr = list(mesh.n_root) + [1] * (3 - mesh.dim)
    lo = list(mesh.lo) + [0.0] * (3 - mesh.dim)
    hi = list(mesh.hi) + [1.0] * (3 - mesh.dim)
    d = L.pe_mesh_desc(mesh.dim, (ctypes.c_int * 3)(*nr), (ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi),
                       leaves.shape[0], leaves.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return d, leaves


def _coeffs(L, fam):
    E = np.ascontiguousarray(np.asarray(fam.E, np.int32))
    c = np.ascontiguousarray(fam.c, dtype=np.float64)
    b = np.ascontiguousarray(fam.b, dtype=np.float64)
    a = np.ascontiguousarray(fam.a_sub, dtype=np.float64)
    co = L.pe_perk_coeffs(fam.order, len(E), fam.S, E.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return co, (E, c, b, a)


def test_mesh_build_and_sizes():
    L, lib = _lib()
    ctx = _ctx(L, lib)
    d, keep = _mesh_desc(L, pin.mesh_vortex_2level())
    assert lib.pe_mesh_build(ctx, ctypes.byref(d)) == 0
    ns, nw, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert lib.pe_query_sizes(ctx, ctypes.byref(ns), ctypes.byref(nw), ctypes.byref(ne)) == 0
    assert ne.value == 304 and ns.value == 304 * 4 * 16
    assert nw.value >= 5 * ns.value * 8
    lib.pe_destroy(ctx)


def test_unbalanced_and_overlapping_meshes_rejected():
    L, lib = _lib()
    ctx = _ctx(L, lib)
    m = pin.uniform_mesh(2, (4, 4), (0, 0), (1, 1), 0)
    m.leaves = pin.refine_leaves(m.leaves, 2, [5])
    # refine one child again -> level 2 next to level 0: not 2:1 balanced
    idx = [r for r, row in enumerate(m.leaves.tolist()) if row[0] == 1][0]
    m.leaves = pin.refine_leaves(m.leaves, 2, [idx])
    d, keep = _mesh_desc(L, m)
    assert lib.pe_mesh_build(ctx, ctypes.byref(d)) == -1
    assert b"2:1" in lib.pe_last_error(ctx)
    m2 = pin.uniform_mesh(2, (2, 2), (0, 0), (1, 1), 0)
    m2.leaves = np.concatenate([m2.leaves, [[1, 0, 0, 0]]]).astype(np.int32)
    d, keep = _mesh_desc(L, m2)
    assert lib.pe_mesh_build(ctx, ctypes.byref(d)) == -1
    m3 = pin.uniform_mesh(2, (2, 2), (0, 0), (1, 1), 0)
    m3.leaves = m3.leaves[:-1]
    d, keep = _mesh_desc(L, m3)
    assert lib.pe_mesh_build(ctx, ctypes.byref(d)) == -1
    lib.pe_destroy(ctx)


def test_coefficient_validation():
    L, lib = _lib()
    ctx = _ctx(L, lib)
    fam = pc.perk2_family([4, 8])
    co, keep = _coeffs(L, fam)
    assert lib.pe_set_perk_coefficients(ctx, ctypes.byref(co)) == 0
    # break b^T c = 1/2
    bad = pc.perk2_family([4, 8]); bad.c = bad.c * 1.01
    co, keep = _coeffs(L, bad)
    assert lib.pe_set_perk_coefficients(ctx, ctypes.byref(co)) == -1
    # nonzero a_{i,i-1} on a stage the E=4 member skips
    bad = pc.perk2_family([4, 8]); bad.a_sub = bad.a_sub.copy(); bad.a_sub[0, 3] = 0.01
    co, keep = _coeffs(L, bad)
    assert lib.pe_set_perk_coefficients(ctx, ctypes.byref(co)) == -1
    # third order: b^T A c = 1/6 is checked per member
    th = np.linspace(0, 2 * np.pi, 100, endpoint=False)
    eigs = -1.0 + np.exp(1j * th)
    fam3 = pc.perk3_family([4, 8], {E: pc.optimize_alpha(eigs, 3, E)[1] for E in (4, 8)})
    co, keep = _coeffs(L, fam3)
    assert lib.pe_set_perk_coefficients(ctx, ctypes.byref(co)) == 0
    bad = pc.perk3_family([4, 8], {E: pc.optimize_alpha(eigs, 3, E)[1] for E in (4, 8)})
    bad.a_sub = bad.a_sub.copy(); bad.a_sub[1, -1] *= 1.1
    co, keep = _coeffs(L, bad)
    assert lib.pe_set_perk_coefficients(ctx, ctypes.byref(co)) == -1
    # descending E
    bad = pc.perk2_family([4, 8]); bad.E = [8, 4]
    co, keep = _coeffs(L, bad)
    assert lib.pe_set_perk_coefficients(ctx, ctypes.byref(co)) == -1
    lib.pe_destroy(ctx)


def test_call_order_errors():
    L, lib = _lib()
    ctx = _ctx(L, lib)
    assert lib.pe_step(ctx, 0.1, 1, None) == -4
    assert lib.pe_bind(ctx, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == -4
    mol = (ctypes.c_int32 * 2)(0, 1)
    assert lib.pe_partition(ctx, mol, 2, None) == -4
    ns = ctypes.c_int64()
    assert lib.pe_query_sizes(ctx, ctypes.byref(ns), None, None) == -4
    # the adaptation cycle and the recorded adjoint step need a partitioned, bound context
    fl = (ctypes.c_int8 * 4)()
    nl = ctypes.c_int64()
    assert lib.pe_amr_cycle(ctx, 0.05, 0.01, 0, 3, mol, 2, fl, ctypes.byref(nl), None) == -4
    assert lib.pe_amr_cycle(ctx, 0.05, 0.01, 0, 3, None, 2, fl, ctypes.byref(nl), None) == -1
    buf = ctypes.c_void_p(256)
    assert lib.pe_step_record(ctx, 0.1, buf, ctypes.c_void_p(512), ctypes.c_void_p(1024), None) == -4
    assert lib.pe_step_adjoint_recorded(ctx, 0.1, buf, ctypes.c_void_p(512), ctypes.c_void_p(1024),
                                        ctypes.c_void_p(2048), None) == -4
    assert lib.pe_adjoint_record_size(ctx, ctypes.byref(ns)) == -4
    assert lib.pe_step_record(None, 0.1, buf, buf, buf, None) == -1
    lib.pe_destroy(ctx)


def test_unsupported_and_invalid_physics():
    L, lib = _lib()
    ctx = ctypes.c_void_p()
    phys = L.pe_physics(4, 3, 0, 1.4, 0.0, 0.72)
    assert lib.pe_create(ctypes.byref(ctx), ctypes.byref(phys)) == -1
    phys = L.pe_physics(2, 3, 0, 0.9, 0.0, 0.72)
    assert lib.pe_create(ctypes.byref(ctx), ctypes.byref(phys)) == -1
