"""PerkSolver: torch-owned device buffers around one libperk context.

Only argument marshalling and buffer ownership live here; the time step, the right-hand side,
the re-partition and the state permutations all run in libperk's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .partition_rule import LevelRule, set_rule


class PerkError(RuntimeError):
    pass


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class PerkSolver:
    """One partitioned P-ERK + DGSEM simulation on a forest mesh.

    mesh: object with dim, n_root, lo, hi, leaves ([n,4] int32 rows (level, i, j, k)).
    family: object with order, S, E, c, b, a_sub (shared c, b; a_{i,i-1} per member).
    member_of_level: int sequence (member index per refinement level), or a LevelRule: the
        library then applies that rule (Sec. 6.4.1, or the required-step variant) at the finest
        level of the current mesh, at this partition and after every adaptation.
    """

    def __init__(self, mesh, degree, family, member_of_level, gamma=1.4, equations=0, mu=0.0,
                 prandtl=0.72, device="cuda", capacity=None):
        if not torch.cuda.is_available():
            raise PerkError("PerkSolver needs a HIP device; there is no CPU path")
        self.lib = L.lib()
        self.device = torch.device(device)
        self.dim = int(mesh.dim)
        self.degree = int(degree)
        self.N = self.degree + 1
        self.nv = self.dim + 2
        self.Nd = self.N ** self.dim
        self._ctx = ctypes.c_void_p()
        phys = L.pe_physics(self.dim, self.degree, int(equations), gamma, mu, prandtl)
        self._check(self.lib.pe_create(ctypes.byref(self._ctx), ctypes.byref(phys)), "pe_create")
        self.mesh = mesh
        self._build_mesh(mesh)
        self.set_family(family)
        self.capacity = int(capacity) if capacity else self.n_elements
        self._check(self.lib.pe_reserve(self._ctx, self.capacity), "pe_reserve")
        self._alloc_and_bind()
        self.partition(member_of_level)

    # ------------------------------------------------------------------ plumbing
    def _check(self, st, what):
        if st != L.PE_OK:
            msg = self.lib.pe_last_error(self._ctx).decode() if self._ctx else ""
            raise PerkError(f"{what}: {L.STATUS.get(st, st)}: {msg}")

    def __del__(self):
        try:
            if self._ctx:
                self.lib.pe_destroy(self._ctx)
                self._ctx = ctypes.c_void_p()
        except Exception:
            pass

    def _build_mesh(self, mesh):
        leaves = np.ascontiguousarray(np.asarray(mesh.leaves, dtype=np.int32).reshape(-1, 4))
        self._leaves = leaves
        nr = list(mesh.n_root) + [1] * (3 - self.dim)
        lo = list(mesh.lo) + [0.0] * (3 - self.dim)
        hi = list(mesh.hi) + [1.0] * (3 - self.dim)
        desc = L.pe_mesh_desc(self.dim, (ctypes.c_int * 3)(*nr), (ctypes.c_double * 3)(*lo),
                              (ctypes.c_double * 3)(*hi), leaves.shape[0],
                              leaves.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(self.lib.pe_mesh_build(self._ctx, ctypes.byref(desc)), "pe_mesh_build")
        self.n_elements = leaves.shape[0]

    def set_family(self, fam):
        self.family = fam
        E = np.ascontiguousarray(np.asarray(fam.E, dtype=np.int32))
        c = np.ascontiguousarray(np.asarray(fam.c, dtype=np.float64))
        b = np.ascontiguousarray(np.asarray(fam.b, dtype=np.float64))
        a = np.ascontiguousarray(np.asarray(fam.a_sub, dtype=np.float64).reshape(len(E), -1))
        # an alternative stage pattern (Sec. 3.2.4) carries its coupling columns
        cp = getattr(fam, "coupling", None)
        cp = None if cp is None else np.ascontiguousarray(np.asarray(cp, dtype=np.int32).reshape(len(E), -1))
        self._coef_keep = (E, c, b, a, cp)
        co = L.pe_perk_coeffs(int(fam.order), len(E), int(fam.S),
                              E.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              None if cp is None else cp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(self.lib.pe_set_perk_coefficients(self._ctx, ctypes.byref(co)),
                    "pe_set_perk_coefficients")

    def _alloc_and_bind(self):
        ns, nw, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.pe_query_sizes(self._ctx, ctypes.byref(ns), ctypes.byref(nw), ctypes.byref(ne)),
                    "pe_query_sizes")
        self.u = torch.empty(ns.value, dtype=torch.float64, device=self.device)
        self.workspace = torch.empty(nw.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._check(self.lib.pe_bind(self._ctx, ctypes.c_void_p(self.u.data_ptr()), ctypes.c_void_p(aligned),
                                     _stream_handle()), "pe_bind")

    # ------------------------------------------------------------------ API
    def partition(self, member_of_level):
        if isinstance(member_of_level, LevelRule):
            self.rule = member_of_level
            self._check(set_rule(self.lib, self._ctx, member_of_level), "pe_set_level_rule")
            self._check(self.lib.pe_partition(self._ctx, None, 0, _stream_handle()), "pe_partition")
            self.member_of_level = self.level_map()
            return
        self.rule = None
        mol = np.ascontiguousarray(np.asarray(member_of_level, dtype=np.int32))
        self.member_of_level = mol
        self._check(self.lib.pe_partition(self._ctx, mol.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          len(mol), _stream_handle()), "pe_partition")

    def level_map(self, finest_level=-1, n_levels=None):
        """The context's level rule as a map (finest level of the current mesh by default)."""
        if n_levels is None:
            n_levels = (int(self._leaves[:, 0].max()) if finest_level < 0 else int(finest_level)) + 1
        out = np.zeros(n_levels, np.int32)
        self._check(self.lib.pe_level_map(self._ctx, int(finest_level), int(n_levels),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "pe_level_map")
        return out

    def element_info(self):
        los = np.zeros(self.n_elements, np.int32)
        mos = np.zeros(self.n_elements, np.int32)
        self._check(self.lib.pe_element_info(self._ctx, los.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             mos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                    "pe_element_info")
        return los, mos

    @property
    def leaf_shape(self):
        return (self.n_elements, self.nv, self.Nd)

    def node_coords(self):
        x = torch.empty((self.n_elements, self.dim, self.Nd), dtype=torch.float64, device=self.device)
        self._check(self.lib.pe_node_coords(self._ctx, ctypes.c_void_p(x.data_ptr()), _stream_handle()),
                    "pe_node_coords")
        return x

    def set_state(self, u_leaf):
        """u_leaf: [n_leaves, n_vars, nodes] (numpy or torch), leaf order of the mesh."""
        t = torch.as_tensor(u_leaf, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != self.leaf_shape:
            raise PerkError(f"set_state: shape {tuple(t.shape)} != {self.leaf_shape}")
        self._check(self.lib.pe_set_state(self._ctx, ctypes.c_void_p(t.data_ptr()), _stream_handle()),
                    "pe_set_state")
        torch.cuda.current_stream().synchronize()

    def get_state(self):
        out = torch.empty(self.leaf_shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.pe_get_state(self._ctx, ctypes.c_void_p(out.data_ptr()), _stream_handle()),
                    "pe_get_state")
        return out

    def step(self, dt, n_steps=1, stream=None):
        self._check(self.lib.pe_step(self._ctx, float(dt), int(n_steps), _stream_handle(stream)), "pe_step")

    def rhs_slot(self, u_slot):
        du = torch.empty_like(u_slot)
        self._check(self.lib.pe_rhs(self._ctx, ctypes.c_void_p(u_slot.data_ptr()), ctypes.c_void_p(du.data_ptr()),
                                    _stream_handle()), "pe_rhs")
        return du

    def rhs_leaf(self, u_leaf):
        """F(u) for a state in leaf layout, returned in leaf layout (uses the bound state buffer)."""
        saved = self.u.clone()
        self.set_state(u_leaf)
        du_slot = self.rhs_slot(self.u)
        self.u.copy_(du_slot)
        out = self.get_state()
        self.u.copy_(saved)
        return out

    # ---------------------------------------------------------------- adjoint (Euler)
    def rhs_vjp_slot(self, u_slot, w_slot):
        """F'(u)^T w in slot layout."""
        out = torch.empty_like(u_slot)
        self._check(self.lib.pe_rhs_vjp(self._ctx, ctypes.c_void_p(u_slot.data_ptr()), ctypes.c_void_p(w_slot.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle()), "pe_rhs_vjp")
        return out

    def jvp_fd_slot(self, u_slot, v_slot, out, eps=1e-7):
        """out = F'(u) v by central differences (pe_rhs_jvp_fd), all slot-layout device arrays."""
        self._check(self.lib.pe_rhs_jvp_fd(self._ctx, ctypes.c_void_p(u_slot.data_ptr()),
                                           ctypes.c_void_p(v_slot.data_ptr()), float(eps),
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle()), "pe_rhs_jvp_fd")
        return out

    def jvp_into(self, u_slot, v_slot, out, f=None):
        """out = F'(u) v exactly (pe_rhs_jvp, Euler) and, if f is given, f = F(u); all
        slot-layout device arrays."""
        self._check(self.lib.pe_rhs_jvp(self._ctx, ctypes.c_void_p(u_slot.data_ptr()), ctypes.c_void_p(v_slot.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(f.data_ptr() if f is not None else 0), _stream_handle()),
                    "pe_rhs_jvp")
        return out

    def vjp_into(self, u_slot, w_slot, out):
        """out = F'(u)^T w (pe_rhs_vjp), all slot-layout device arrays."""
        self._check(self.lib.pe_rhs_vjp(self._ctx, ctypes.c_void_p(u_slot.data_ptr()), ctypes.c_void_p(w_slot.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle()), "pe_rhs_vjp")
        return out

    def orthogonalize(self, V, k, w, scratch):
        """Orthogonalise device vector w against rows 0..k-1 of V (pe_orthogonalize); returns the
        k + 1 coefficients (projections, then the norm w was divided by)."""
        h = np.zeros(k + 1)
        n = w.numel()
        ldv = V.stride(0) if V.dim() == 2 else n
        self._check(self.lib.pe_orthogonalize(self._ctx, ctypes.c_void_p(V.data_ptr()), int(k), int(ldv),
                                              ctypes.c_void_p(w.data_ptr()), int(n), ctypes.c_void_p(scratch.data_ptr()),
                                              h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_handle()),
                    "pe_orthogonalize")
        return h

    def to_slot(self, x_leaf):
        """Leaf-layout array [n_leaves, n_vars, nodes] -> slot-layout tensor (uses the bound state)."""
        saved = self.u.clone()
        self.set_state(x_leaf)
        out = self.u.clone()
        self.u.copy_(saved)
        return out

    def to_leaf(self, x_slot):
        saved = self.u.clone()
        self.u.copy_(x_slot)
        out = self.get_state()
        self.u.copy_(saved)
        return out

    def rhs_vjp_leaf(self, u_leaf, w_leaf):
        return self.to_leaf(self.rhs_vjp_slot(self.to_slot(u_leaf), self.to_slot(w_leaf)))

    def enable_adjoint(self):
        """Allocate and bind the adjoint workspace (stage values and stage cotangents)."""
        nb = ctypes.c_int64()
        self._check(self.lib.pe_adjoint_query(self._ctx, ctypes.byref(nb)), "pe_adjoint_query")
        self._adj_ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._adj_ws.data_ptr() + 255) & ~255
        self._check(self.lib.pe_adjoint_bind(self._ctx, ctypes.c_void_p(aligned)), "pe_adjoint_bind")

    def step_adjoint(self, u_n_slot, lam_slot, dt):
        """Phi'(u_n)^T lam for one step of size dt (slot layout)."""
        if getattr(self, "_adj_ws", None) is None:
            self.enable_adjoint()
        out = torch.empty_like(lam_slot)
        self._check(self.lib.pe_step_adjoint(self._ctx, float(dt), ctypes.c_void_p(u_n_slot.data_ptr()),
                                             ctypes.c_void_p(lam_slot.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             _stream_handle()), "pe_step_adjoint")
        return out

    def step_record(self, u_n_slot, dt):
        """One step from u_n (slot layout) without touching the bound state: (u_next, record),
        the record holding what step_adjoint_recorded reads (K_1 and the stage values)."""
        if getattr(self, "_adj_ws", None) is None:
            self.enable_adjoint()
        nd = ctypes.c_int64()
        self._check(self.lib.pe_adjoint_record_size(self._ctx, ctypes.byref(nd)), "pe_adjoint_record_size")
        u_next = torch.empty_like(u_n_slot)
        record = torch.empty(nd.value, dtype=torch.float64, device=self.device)
        self._check(self.lib.pe_step_record(self._ctx, float(dt), u_n_slot.data_ptr(), u_next.data_ptr(),
                                            record.data_ptr(), _stream_handle()), "pe_step_record")
        return u_next, record

    def step_adjoint_recorded(self, u_n_slot, record, lam_slot, dt):
        """step_adjoint(u_n, lam, dt) from the record of step_record(u_n, dt)."""
        if getattr(self, "_adj_ws", None) is None:
            self.enable_adjoint()
        out = torch.empty_like(lam_slot)
        self._check(self.lib.pe_step_adjoint_recorded(self._ctx, float(dt), u_n_slot.data_ptr(), record.data_ptr(),
                                                      lam_slot.data_ptr(), out.data_ptr(), _stream_handle()),
                    "pe_step_adjoint_recorded")
        return out

    def leaves(self):
        n = ctypes.c_int64()
        self._check(self.lib.pe_get_leaves(self._ctx, None, ctypes.byref(n)), "pe_get_leaves")
        out = np.zeros((n.value, 4), np.int32)
        self._check(self.lib.pe_get_leaves(self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           ctypes.byref(n)), "pe_get_leaves")
        return out

    def indicator(self):
        eta = np.zeros(self.n_elements)
        self._check(self.lib.pe_amr_indicator(self._ctx, eta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              _stream_handle()), "pe_amr_indicator")
        return eta

    def adapt(self, flags, level_min, level_max, member_of_level):
        """Adapt the forest with per-leaf flags, project the state, re-partition."""
        f = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        if f.shape != (self.n_elements,):
            raise PerkError("adapt: one flag per leaf")
        self._check(self.lib.pe_adapt(self._ctx, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), int(level_min),
                                      int(level_max), _stream_handle()), "pe_adapt")
        self._leaves = self.leaves()
        self.n_elements = self._leaves.shape[0]
        self.mesh.leaves = self._leaves
        self.partition(member_of_level)

    def set_indicator(self, kind, variable=1, f_wave=0.2):
        """Refinement indicator of indicator() / amr_cycle(): "density_gradient", "lohner" (on the
        primitive variable `variable`: 0 rho, 1..dim velocity, dim+1 pressure) or
        "hennemann_gassner" (the shock-capturing sigmoid of the density, variable 0)."""
        k = {"density_gradient": 0, "lohner": 1, "hennemann_gassner": 2}[kind]
        self._check(self.lib.pe_set_amr_indicator(self._ctx, k, int(variable), float(f_wave)), "pe_set_amr_indicator")

    def set_shock_capturing(self, on=True, alpha_max=0.5, alpha_min=0.001):
        """Subcell shock capturing (pe_set_shock_capturing, 2D Euler)."""
        self._check(self.lib.pe_set_shock_capturing(self._ctx, int(bool(on)), float(alpha_max), float(alpha_min)),
                    "pe_set_shock_capturing")

    def amr_cycle(self, refine_above, coarsen_below, level_min, level_max, member_of_level):
        """indicator() + threshold flags + adapt() in one library call (the same flags, forest and
        state); returns the flags of the leaves before the call.  Host buffers are kept between
        calls and passed by address: the per-call Python work is a few attribute reads."""
        cap = self.capacity
        if getattr(self, "_cyc", None) is None or self._cyc["cap"] != cap:
            bufs = {"cap": cap, "flags": np.zeros(cap, np.int8), "n": np.zeros(1, np.int64),
                    "leaves": np.zeros((cap, 4), np.int32), "mol_key": None}
            for k in ("flags", "n", "leaves"):
                bufs[k + "_p"] = bufs[k].ctypes.data
            self._cyc = bufs
        c = self._cyc
        if isinstance(member_of_level, LevelRule):
            # the library applies its rule at the finest level of the adapted mesh
            if self.rule != member_of_level:
                self._check(set_rule(self.lib, self._ctx, member_of_level), "pe_set_level_rule")
                self.rule = member_of_level
            mol_p, n_lev = None, 0
        else:
            key = tuple(int(x) for x in member_of_level)
            if c["mol_key"] != key:
                c["mol"] = np.ascontiguousarray(key, dtype=np.int32)
                c["mol_p"], c["mol_key"] = c["mol"].ctypes.data, key
            mol_p, n_lev = c["mol_p"], len(key)
        n_old = self.n_elements
        self._check(self.lib.pe_amr_cycle(self._ctx, float(refine_above), float(coarsen_below), int(level_min),
                                          int(level_max), mol_p, n_lev, c["flags_p"], c["n_p"],
                                          _stream_handle()), "pe_amr_cycle")
        n = int(c["n"][0])
        cnt = ctypes.c_int64(n)
        self._check(self.lib.pe_get_leaves(self._ctx, c["leaves_p"], ctypes.byref(cnt)), "pe_get_leaves")
        self._leaves = c["leaves"][:n].copy()
        self.n_elements = n
        self.mesh.leaves = self._leaves
        if not isinstance(member_of_level, LevelRule):
            self.member_of_level = c["mol"]
        return c["flags"][:n_old].copy()

    def max_dt(self, cfl=1.0):
        """(cfl * min_l beta_l, beta per level) from the current state, eq. (CFL_DG)."""
        dt = ctypes.c_double()
        beta = np.zeros(16)
        self._check(self.lib.pe_max_dt(self._ctx, float(cfl), ctypes.byref(dt),
                                       beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_handle()),
                    "pe_max_dt")
        return dt.value, beta

    def quadrature(self):
        x = np.zeros(self.N)
        w = np.zeros(self.N)
        self._check(self.lib.pe_quadrature(self._ctx, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "pe_quadrature")
        return x, w

    def node_weights(self):
        """Quadrature weight of every node in leaf layout, [n_leaves, nodes] (element volume included)."""
        _, w = self.quadrature()
        W = w
        for _ in range(self.dim - 1):
            W = np.multiply.outer(w, W).reshape(-1)
        lv = self.leaves()[:, 0]
        vol = np.ones(len(lv))
        for d in range(self.dim):
            vol = vol * (self.mesh.hi[d] - self.mesh.lo[d]) / (np.asarray(self.mesh.n_root[d]) * 2.0 ** lv) / 2.0
        return vol[:, None] * W[None, :]

    def set_graph_replay(self, on):
        self._check(self.lib.pe_set_graph_replay(self._ctx, int(bool(on))), "pe_set_graph_replay")

    def set_profiling(self, on):
        self._check(self.lib.pe_set_profiling(self._ctx, int(bool(on))), "pe_set_profiling")

    def profile_stats(self, kernel=0):
        """(milliseconds, launches, elements) of the timed launches of one kernel: 0 the stage
        kernel, 1 the BR1 gradient kernel."""
        ms, nl, es = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.pe_profile_kernel_stats(self._ctx, int(kernel), ctypes.byref(ms), ctypes.byref(nl),
                                                     ctypes.byref(es)), "pe_profile_kernel_stats")
        return ms.value, nl.value, es.value

    def counters(self, reset=False):
        tot = ctypes.c_int64()
        per = (ctypes.c_int64 * 8)()
        self._check(self.lib.pe_counters(self._ctx, ctypes.byref(tot), per, int(reset), _stream_handle()),
                    "pe_counters")
        return tot.value, list(per)[:len(self.family.E)]
