"""ctypes binding of libperk.so: the entry points of include/perk.h under the same names.

Argument marshalling only; every step of the method runs in the HIP library.  Importing this
module fails loudly when the library has not been built.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libperk.so")

PE_OK = 0
STATUS = {0: "PE_OK", -1: "PE_EINVAL", -2: "PE_ENOMEM", -3: "PE_EHIP", -4: "PE_ESTATE",
          -5: "PE_ENONFINITE", -6: "PE_EUNSUPPORTED"}


class pe_physics(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("degree", ctypes.c_int), ("equations", ctypes.c_int),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double)]


class pe_mesh_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_root", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("n_leaves", ctypes.c_int),
                ("leaves", ctypes.POINTER(ctypes.c_int32))]


class pe_perk_coeffs(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("n_members", ctypes.c_int), ("n_stages", ctypes.c_int),
                ("E", ctypes.POINTER(ctypes.c_int32)), ("c", ctypes.POINTER(ctypes.c_double)),
                ("a_sub", ctypes.POINTER(ctypes.c_double)), ("b", ctypes.POINTER(ctypes.c_double)),
                ("coupling", ctypes.POINTER(ctypes.c_int32))]


_lib = None

_SIGS = {
    "pe_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(pe_physics)]),
    "pe_destroy": (None, [ctypes.c_void_p]),
    "pe_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pe_mesh_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(pe_mesh_desc)]),
    "pe_set_perk_coefficients": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(pe_perk_coeffs)]),
    "pe_set_level_rule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_double]),
    "pe_level_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]),
    "pe_query_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "pe_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_partition": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                                    ctypes.c_void_p]),
    "pe_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_element_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "pe_node_coords": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]),
    "pe_counters": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_void_p]),
    "pe_reserve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "pe_amr_indicator": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "pe_adapt": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int8), ctypes.c_int, ctypes.c_int,
                                ctypes.c_void_p]),
    "pe_amr_cycle": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_adjoint_record_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "pe_step_record": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "pe_step_adjoint_recorded": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_get_leaves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "pe_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "pe_batch_destroy": (None, [ctypes.c_void_p]),
    "pe_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pe_batch_set_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "pe_batch_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "pe_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "pe_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]),
    "pe_rhs_vjp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pe_adjoint_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "pe_adjoint_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pe_step_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "pe_max_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "pe_quadrature": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    "pe_mortar_operators": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]),
    "pe_set_graph_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "pe_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "pe_profile_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "pe_max_dt_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "pe_set_amr_indicator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double]),
    "pe_set_shock_capturing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    "pe_rhs_jvp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "pe_rhs_jvp_fd": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "pe_orthogonalize_scratch": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "pe_orthogonalize": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "pe_device_math": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "pe_profile_kernel_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
}

EXPORTS = tuple(_SIGS)


def library_fingerprint():
    """(path, sha256) of the library this process loads."""
    import hashlib
    with open(LIB_PATH, "rb") as f:
        return LIB_PATH, hashlib.sha256(f.read()).hexdigest()


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libperk.so not built at {LIB_PATH}: run __graft_entry__.build() "
                               "(hipcc, gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
