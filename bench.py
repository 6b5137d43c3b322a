"""Benchmark of the partitioned P-ERK + DGSEM hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A step is one P-ERK time step of the whole hot path (every stage's right-hand side on the
active elements, the stage combinations and the final update; for adaptive workloads also the
indicator, mesh adaptation and re-partition every N_AMR steps).  Prints one JSON line.

Metric: DoF-updates/s = steps * n_vars * N^d * n_elements / wall time (inputs resident in HBM
before the timed region).  PID = wall time / N_RHS^Actual (eq. ActualRHSEvals) is reported
beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# what defines the stage kernel (hashed into the counter summaries): its source, the device
# helpers, and the data structures of the internal header (up to its launch declarations)
STAGE_KERNEL_SOURCES = ("perk_stage.hip", "perk_device.h", "perk_internal.h")


def stage_kernel_digest():
    """sha256 of the stage kernel's code (the kernel file, the device helpers, the data
    structures of the internal header) with comments and blank lines left out, so that a
    comment edit does not make recorded counter summaries stale."""
    import hashlib, re
    h = hashlib.sha256()
    for name in STAGE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2403_05144_amd", "csrc", name), encoding="utf-8") as f:
            data = f.read()
        if name == "perk_internal.h":
            cut = data.find("// Kernel launch wrappers")
            data = data[:cut] if cut >= 0 else data
        data = re.sub(r"/\*.*?\*/", "", data, flags=re.S)
        data = re.sub(r"//[^\n]*", "", data)
        h.update("\n".join(l.rstrip() for l in data.splitlines() if l.strip()).encode())
    return h.hexdigest()
FP64_PEAK_TFLOPS = 78.6


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------
def family_for(name, order, E_list, reduced_mesh, degree, ic_fn, h_red, equations=0, mu=0.0, shock_capturing=None):
    """Coefficients from the project's own optimisation on the spectrum of a reduced mesh
    (cached as JSON next to the package); shock_capturing = (alpha_max, alpha_min) takes the
    spectrum of the blended operator."""
    from paper_2403_05144_amd import PerkSolver, coeffs
    path = os.path.join(ROOT, "paper_2403_05144_amd", "data", f"{name}.json")
    if os.path.exists(path):
        return coeffs.Family.load(path)
    _log(f"building coefficient family {name} (spectrum of the reduced mesh, LP optimisation)")
    tmp = coeffs.Family(2, 2, [2], np.array([0.0, 0.5]), np.array([0.0, 1.0]), np.zeros((1, 2)))
    s = PerkSolver(reduced_mesh, degree, tmp, [0] * (int(reduced_mesh.leaves[:, 0].max()) + 1),
                   equations=equations, mu=mu)
    if shock_capturing:
        s.set_shock_capturing(True, *shock_capturing)
    x = s.node_coords().cpu().numpy().transpose(1, 0, 2)
    u = ic_fn(x).transpose(1, 0, 2).copy()
    fam, lam = coeffs.family_from_solver_spectrum(s, u, order, E_list, h_red)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    fam.save(path)
    return fam


def rule_map(fam, rule, finest_level):
    """member_of_level of the library's level rule (pe_level_map) at the given finest level."""
    from paper_2403_05144_amd import partition_rule
    return partition_rule.level_map(fam, rule, int(finest_level))


def stable_dt(fam, mesh, mol, cfl):
    """dt = cfl * min over members of dt_opt(E_r) * h_min(r) / h_ref (spectra scale with 1/h)."""
    levels = mesh.leaves[:, 0]
    h = lambda l: (mesh.hi[0] - mesh.lo[0]) / (mesh.n_root[0] << int(l))
    dts = []
    for l in np.unique(levels):
        r = mol[int(l)]
        dts.append(fam.dt_opt[r] * h(l) / fam.h_ref)
    return cfl * min(dts)


def make_solver(wl, mesh, fam, mol):
    """The workload's solver: capacity, equations and refinement indicator as the workload says."""
    from paper_2403_05144_amd import PerkSolver
    amr = wl.get("amr")
    s = PerkSolver(mesh, wl["degree"], fam, mol, capacity=amr["capacity"] if amr else None,
                   equations=wl.get("equations", 0), mu=wl.get("mu", 0.0))
    if amr and amr.get("indicator"):
        s.set_indicator(*amr["indicator"])
    if wl.get("shock_capturing"):
        s.set_shock_capturing(True, *wl["shock_capturing"])
    return s


def wl_vortex_2level():
    import perk_inputs as pin
    mesh = pin.mesh_vortex_2level()
    red = pin.uniform_mesh(2, (4, 4), (-5, -5), (5, 5), 0)
    ic = lambda x: pin.isentropic_vortex(x[0], x[1])
    fam = family_for("perk2_4_8_vortex_p3", 2, [4, 8], red, 3, ic, 2.5)
    from paper_2403_05144_amd.partition_rule import LevelRule
    rule = LevelRule.paper()
    mol = rule_map(fam, rule, mesh.leaves[:, 0].max())
    return dict(name="vortex_2level", mesh=mesh, degree=3, fam=fam, mol=mol, rule=rule, ic=ic,
                dt=stable_dt(fam, mesh, mol, 0.9), cfl=0.9, t_final=1.0,
                desc="2D Euler isentropic vortex (M=0.5, eps=5) on [-5,5]^2, 16x16 roots with the "
                     "centred 4x4 block refined once (304 elements, 2 levels), p=3, EC volume + HLL "
                     "surface flux, P-ERK2{4,8}")


def wl_kh_amr(n_root=8, level_max=3, name="kh_amr_l3-6", fam=None):
    """Kelvin-Helmholtz shear layer, quadtree AMR between config levels 3 and 6 (forest levels
    0..3 on 8x8 roots), P-ERK3{4,6,8,12,16}, adaptation every 10 steps.

    Level -> member map: the required-step rule with margin 2 ({6,12,16,16} from coarse to
    fine), stable up to CFL 1.0 of the finest member's optimal step over t in [0, 3]; with
    margin 1 ({4,6,12,16}) the family is stable only up to CFL 0.5 (member boundaries at high
    local CFL, Sec. 5).  The timed run uses CFL 0.9."""
    import perk_inputs as pin
    from paper_2403_05144_amd.partition_rule import LevelRule
    mesh = pin.uniform_mesh(2, (n_root, n_root), (-1, -1), (1, 1), 0)
    ic = lambda x: pin.kelvin_helmholtz(x[0], x[1])
    h_red = 2.0 / n_root
    fam_name = f"perk3_4_6_8_12_16_kh_p3_n{n_root}"
    if fam is None:
        fam = family_for(fam_name, 3, [4, 6, 8, 12, 16], pin.uniform_mesh(2, (n_root, n_root), (-1, -1), (1, 1), 0),
                         3, ic, h_red)
    rule = LevelRule.required_step(fam.dt_opt, margin=2.0)
    mol = rule_map(fam, rule, level_max)
    mol1 = rule_map(fam, LevelRule.required_step(fam.dt_opt, margin=1.0), level_max)
    h_min = h_red / 2 ** level_max
    cfl = 0.9
    dt = cfl * fam.dt_opt[-1] * h_min / fam.h_ref
    return dict(name=name, mesh=mesh, degree=3, fam=fam, fam_name=fam_name, mol=mol, rule=rule, ic=ic, dt=dt,
                cfl=cfl, t_final=3.0, spectrum_op="jvp", h_reduced=h_red,
                reduced_mesh=pin.uniform_mesh(2, (n_root, n_root), (-1, -1), (1, 1), 0),
                perk_maps=[("required-step rule, margin 2", mol), ("required-step rule, margin 1", mol1)],
                amr=dict(level_min=0, level_max=level_max, interval=10, refine_above=0.05, coarsen_below=0.01,
                         capacity=(n_root << level_max) ** 2),
                desc=f"2D Euler Kelvin-Helmholtz shear layer on [-1,1]^2 (rho 0.5/1, v_x +-0.5, tanh width "
                     f"0.05, seeded v_y perturbation 0.01), p=3, EC volume + HLL surface flux, quadtree AMR on "
                     f"a density-gradient indicator between levels {int(np.log2(n_root))} and "
                     f"{int(np.log2(n_root)) + level_max} every 10 steps with re-partition after every "
                     f"adaptation, P-ERK3{{4,6,8,12,16}} with levels mapped to E={[fam.E[r] for r in mol]} "
                     f"(required-step rule, margin 2), CFL {cfl} of the finest member's optimised step")


def wl_shear_layer():
    """2D compressible Navier-Stokes doubly periodic shear layer (Sec. 7.1.1, eq. ShearLayerIC):
    kappa 80, delta 0.05, c0 10 (Ma 0.1), Re 2.5e4, Pr 0.72 on [0,1]^2; 8x8 roots (level 3),
    adaptation every 20 steps on Loehner's indicator of v_x (f_wave 0.2) up to six refinements
    (level 9, 512 cells per direction); p = 3, BR1; P-ERK3{3,4,7} from the project's optimisation
    on the spectrum of the 8x8 mesh, levels mapped by the paper's rule (finest E = 7, next E = 4,
    the rest E = 3).  The timed run uses CFL 0.9 of the finest member's optimised step."""
    import perk_inputs as pin
    from paper_2403_05144_amd.partition_rule import LevelRule
    mu = 1.0 / 2.5e4
    mesh = pin.uniform_mesh(2, (8, 8), (0, 0), (1, 1), 0)
    ic = lambda x: pin.shear_layer(x[0], x[1])
    h_red = 1.0 / 8
    fam = family_for("perk3_3_4_7_shear_p3", 3, [3, 4, 7], pin.uniform_mesh(2, (8, 8), (0, 0), (1, 1), 0), 3, ic,
                     h_red, equations=1, mu=mu)
    level_max = 6
    rule = LevelRule.paper()
    mol = rule_map(fam, rule, level_max)
    cfl = 0.9
    dt = cfl * fam.dt_opt[-1] * (h_red / 2 ** level_max) / fam.h_ref
    return dict(name="shear_layer_ns_2d", mesh=mesh, degree=3, fam=fam, mol=mol, rule=rule, ic=ic, dt=dt, cfl=cfl,
                t_final=1.2, eq_t_final=0.1, equations=1, mu=mu,
                amr=dict(level_min=0, level_max=level_max, interval=20, refine_above=0.2, coarsen_below=0.05,
                         capacity=1 << 17, indicator=("lohner", 1, 0.2)),
                perk_maps=[("paper rule", mol)],
                desc="2D compressible Navier-Stokes doubly periodic shear layer (kappa 80, delta 0.05, Ma 0.1, "
                     "Re 2.5e4, Pr 0.72) on [0,1]^2, p=3, EC volume + HLL surface flux, BR1, quadtree AMR on "
                     "Loehner's indicator of v_x between levels 3 and 9 every 20 steps with re-partition after "
                     f"every adaptation, P-ERK3{{3,4,7}} with levels mapped to E={[fam.E[r] for r in mol]} "
                     f"(paper rule), CFL {cfl} of the finest member's optimised step")


def wl_tgv(fam=None):
    """3D compressible Navier-Stokes Taylor-Green vortex, Ma 0.1, Re 1600, Pr 0.72, 16^3 roots
    with a seeded 2-level refined region (7120 elements), p=3, BR1, P-ERK2{4,8,16}.

    Level -> member map: the required-step rule ({8,16,16} from coarse to fine), stable up to
    CFL 0.8 of the finest member's optimal step over 200 steps, like the standalone
    P-ERK2;16; the one-member-per-level map {4,8,16} is stable only up to CFL 0.4.  The timed
    run uses CFL 0.7."""
    import perk_inputs as pin
    from paper_2403_05144_amd.partition_rule import LevelRule
    mesh = pin.mesh_taylor_green()
    mu = 1.0 / 1600
    ic = lambda x: pin.taylor_green(x[0], x[1], x[2])
    red = pin.uniform_mesh(3, (2, 2, 2), (-np.pi,) * 3, (np.pi,) * 3, 0)
    fam_name = "perk2_4_8_16_tgv_p3"
    if fam is None:
        fam = family_for(fam_name, 2, [4, 8, 16], red, 3, ic, np.pi, equations=1, mu=mu)
    rule = LevelRule.required_step(fam.dt_opt, margin=1.0)
    mol = rule_map(fam, rule, 2)
    h_min = 2 * np.pi / 16 / 4
    cfl = 0.7
    dt = cfl * fam.dt_opt[-1] * h_min / fam.h_ref
    return dict(name="tgv_ns_3d", mesh=mesh, degree=3, fam=fam, fam_name=fam_name, mol=mol, rule=rule, ic=ic, dt=dt,
                cfl=cfl, t_final=200 * dt, spectrum_op="fd", reduced_mesh=red, h_reduced=np.pi,
                equations=1, mu=mu,
                perk_maps=[("required-step rule", mol), ("one member per level", [0, 1, 2])],
                desc="3D compressible Navier-Stokes Taylor-Green vortex (Ma 0.1, Re 1600, Pr 0.72) on "
                     "[-pi,pi]^3, 16^3 roots with a seeded 2-level refined region (3880+1512+1728 = 7120 "
                     f"elements), p=3, EC volume + HLL surface flux, BR1, P-ERK2{{4,8,16}} with levels mapped "
                     f"to E={[fam.E[r] for r in mol]} (required-step rule), CFL {cfl} of the finest member's "
                     "optimised step")


def vortex_family(degree, E):
    """P-ERK2 family with stage counts E optimised on the spectrum of the isentropic vortex
    (strength 5) on a 4x4 reduced mesh of [-5,5]^2 at the given degree."""
    import perk_inputs as pin
    red = pin.uniform_mesh(2, (4, 4), (-5, -5), (5, 5), 0)
    ic = lambda x: pin.isentropic_vortex(x[0], x[1])
    return family_for(f"perk2_{'_'.join(str(e) for e in E)}_vortex_p{degree}", 2, list(E), red, degree, ic, 2.5)


def batch_runs(replicas=1, cfl=0.4):
    """The batched workload: 64 seeded isentropic-vortex runs of uneven size (roots per side
    8..64, 1-3 nested refinement disks, strength 1..5, degree 2 or 3, P-ERK2 {4,8} or {4,8,16}),
    each to t = 1 at cfl times its largest stable step, replicated `replicas` times.  (At CFL
    0.6 nine and at 0.8 twenty-seven of the {4,8,16} runs blow up before t = 1; 0.4 keeps all.)"""
    import perk_inputs as pin
    from paper_2403_05144_amd.partition_rule import LevelRule
    runs = []
    for spec in pin.batch_vortex_runs():
        fam = vortex_family(spec["degree"], spec["E"])
        mesh = spec["mesh"]
        lmax = int(mesh.leaves[:, 0].max())
        mol = rule_map(fam, LevelRule.paper(), lmax)
        dt = stable_dt(fam, mesh, mol, cfl)
        n_steps = int(math.ceil(1.0 / dt))
        runs.append(dict(spec, fam=fam, mol=mol, dt=1.0 / n_steps, n_steps=n_steps))
    return runs * replicas


def run_batch(args):
    """Batched independent runs: one stage-tick launch for all runs, against the same runs
    launched one after another through the single-run path (graph replay)."""
    import torch
    import perk_inputs as pin
    from paper_2403_05144_amd import PerkBatch, PerkSolver
    specs = batch_runs(args.batch_replicas)
    solvers, u0s = [], []
    for sp in specs:
        m = sp["mesh"]
        mesh = pin.MeshDesc(m.dim, m.n_root, m.lo, m.hi, np.array(m.leaves, copy=True))
        s = PerkSolver(mesh, sp["degree"], sp["fam"], sp["mol"])
        x = s.node_coords().cpu().numpy().transpose(1, 0, 2)
        u0 = pin.isentropic_vortex(x[0], x[1], eps=sp["eps"]).transpose(1, 0, 2).copy()
        s.set_state(u0)
        solvers.append(s)
        u0s.append(s.u.clone())
    n_runs = len(solvers)
    dofs = [s.n_elements * s.nv * s.Nd for s in solvers]
    work = sum(d * sp["n_steps"] for d, sp in zip(dofs, specs))
    _log(f"batch: {n_runs} runs, {sum(s.n_elements for s in solvers)} elements, {work:.3g} DoF-updates")

    def reset():
        for s, u in zip(solvers, u0s):
            s.u.copy_(u)
            s.counters(reset=True)
        torch.cuda.synchronize()

    # sequential comparator (warm: every run's step graph captured beforehand)
    for s, sp in zip(solvers, specs):
        s.step(sp["dt"], 1)
    reset()
    t0 = time.perf_counter()
    for s, sp in zip(solvers, specs):
        s.step(sp["dt"], sp["n_steps"])
    torch.cuda.synchronize()
    wall_seq = time.perf_counter() - t0
    seq_states = [s.u.clone() for s in solvers]
    seq_es = sum(s.counters()[0] for s in solvers)
    reset()
    b = PerkBatch(solvers)
    b.set_steps([sp["dt"] for sp in specs], [sp["n_steps"] for sp in specs])
    tune = b.autotune()
    n_ticks, es = b.info()
    reset()
    b.run()                                   # warm-up pass
    reset()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    b.run()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    same = all(torch.equal(s.u, ref) for s, ref in zip(solvers, seq_states))
    finite = all(bool(torch.isfinite(s.u[: s.n_elements * s.nv * s.Nd]).all()) for s in solvers)
    if not finite:
        raise RuntimeError("non-finite state after the batched runs")
    # algorithmic bytes and flops of all element-stages (per run: its degree)
    bytes_tot = flops_tot = 0.0
    for s in solvers:
        k = s.counters()[0]
        bytes_tot += k * bytes_per_element_stage(2, s.N)
        flops_tot += k * flops_per_element_stage(2, s.N)
    t_kernel = gpu_ms * 1e-3 / n_ticks          # per tick: launch gaps included (stream events)
    gbs = bytes_tot / n_ticks / t_kernel / 1e9
    tflops = flops_tot / n_ticks / t_kernel / 1e12
    frac_b, frac_f = gbs / HBM_PEAK_GBS, tflops / FP64_PEAK_TFLOPS
    roof = ({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac_b}
            if frac_b >= frac_f else
            {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": frac_f})
    roof.update(traffic=None, kernel="k_stage_batch", avg_launch_us=t_kernel * 1e6,
                element_stages_per_launch=es / n_ticks,
                alt={"hbm_frac": frac_b, "alu_frac": frac_f, "gbs": gbs, "tflops": tflops})
    name = f"batch_vortex64_x{args.batch_replicas}"
    return {
        "metric": "DoF-updates/s & PID; P-ERK vs single-level RK wall time at equal error",
        "value": work / wall, "unit": "DoF-updates/s", "n_gpus": 1, "steps": int(n_ticks), "warmup": 1,
        "ms_per_step": wall / n_ticks * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": name, "runs": n_runs, "elements": int(sum(s.n_elements for s in solvers)),
                   "description": "64 seeded 2D Euler isentropic-vortex runs of uneven size (8..64 roots per side, "
                                  "1-3 nested refinement disks of radii 3/2/1, strength U[1,5], degree 2 or 3, "
                                  "P-ERK2 {4,8} or {4,8,16} optimised on the vortex spectrum, CFL 0.4, t in [0,1]), "
                                  f"replicated x{args.batch_replicas}; one launch per stage tick",
                   "tiling": tune["tiling"], "ticks": int(n_ticks)},
        "pid_s": wall / sum(s.counters()[0] * s.nv * s.Nd for s in solvers),
        "batched_vs_sequential": {"sequential_wall_s": wall_seq, "batched_wall_s": wall,
                                  "speedup": wall_seq / wall, "bitwise_equal": bool(same),
                                  "element_stages": int(es), "element_stages_sequential": int(seq_es)},
        "autotune": tune,
        "roofline": roof,
    }


def run_adjoint(args):
    """Differentiated form: gradient of the final kinetic energy with respect to a seeded initial
    density perturbation through 100 P-ERK2 {4,8} steps on the 2-level band mesh (64^2 roots,
    roots with ||y| - 0.5| < 1/8 refined: 7168 elements, p = 3, Kelvin-Helmholtz state),
    checkpoints every 10 steps; central finite differences on 20 seeded directions."""
    import torch
    import perk_inputs as pin
    from paper_2403_05144_amd import PerkSolver
    from paper_2403_05144_amd.adjoint import kinetic_energy, slot_node_weights, trajectory
    mesh = pin.mesh_band_2level(64)
    ic = lambda x: pin.kelvin_helmholtz(x[0], x[1])
    fam = family_for("perk2_4_8_kh_p3_n8", 2, [4, 8], pin.uniform_mesh(2, (8, 8), (-1, -1), (1, 1), 0), 3, ic, 0.25)
    mol = [0, 1]
    s = PerkSolver(mesh, 3, fam, mol)
    x = s.node_coords().cpu().numpy().transpose(1, 0, 2)
    rho, vx, vy, p = pin.kelvin_helmholtz_prim(x[0], x[1])
    m0 = pin.kh_density_perturbation(x[0], x[1])
    u0_of = lambda m: pin.prim2cons(rho + m, [vx, vy], p, 1.4).transpose(1, 0, 2).copy()
    s.set_state(u0_of(m0))
    ws = slot_node_weights(s)
    n, every = 100, 10
    dt = stable_dt(fam, mesh, mol, 0.5)
    _log(f"adjoint: {s.n_elements} elements, dt={dt:.5g}, {n} steps, checkpoints every {every}")

    def J_of(m):
        s.set_state(u0_of(m))
        s.step(dt, n)
        return float(kinetic_energy(s, s.u, ws))

    J_of(m0)                                          # warm-up (graph capture)
    s.enable_adjoint()
    # warm-up of the reverse sweep too (first launches of its kernels, autograd set-up): one
    # checkpoint interval forward and back, untimed
    uw = s.to_slot(u0_of(m0)).requires_grad_(True)
    kinetic_energy(s, trajectory(uw, s, dt, every, every), ws).backward()
    del uw
    u0 = s.to_slot(u0_of(m0)).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uN = trajectory(u0, s, dt, n, every)
    J = kinetic_energy(s, uN, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lam = s.to_leaf(u0.grad).cpu().numpy()
    g = lam[:, 0] + lam[:, 1] * vx + lam[:, 2] * vy + lam[:, 3] * 0.5 * (vx * vx + vy * vy)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    J_plain = J_of(m0)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t3
    rng = np.random.default_rng(pin.MASTER_SEED + 5)
    errs = []
    for _ in range(20):
        dm = rng.standard_normal(m0.shape)
        eps = 1e-5 / np.max(np.abs(dm))
        fd = (J_of(m0 + eps * dm) - J_of(m0 - eps * dm)) / (2 * eps)
        ad = float(np.sum(g * dm))
        errs.append(abs(fd - ad) / abs(ad))
    errs = np.array(errs)
    dofs = s.n_elements * s.nv * s.Nd
    fwd, bwd = t1 - t0, t2 - t1
    return {
        "metric": "DoF-updates/s & PID; P-ERK vs single-level RK wall time at equal error",
        "value": n * dofs / bwd, "unit": "DoF-updates/s", "n_gpus": 1, "steps": n, "warmup": 1,
        "ms_per_step": bwd / n * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "adjoint_kh_band64", "elements": int(s.n_elements), "degree": 3, "family_E": [4, 8],
                   "dt": dt, "checkpoint_every": every,
                   "description": "discrete adjoint of 100 P-ERK2 {4,8} steps of 2D Euler on the Kelvin-Helmholtz "
                                  "state, 2-level band mesh of 64^2 roots (7168 elements, p=3); objective: total "
                                  "kinetic energy at the final step; control: initial density perturbation; value "
                                  "counts the steps of the reverse sweep (recomputation included) per second"},
        "objective": J_plain, "objective_in_trajectory": float(J.detach()),
        "forward_with_checkpoints_s": fwd, "forward_plain_s": t_plain, "backward_s": bwd,
        "backward_over_forward": bwd / t_plain,
        "finite_differences": {"directions": 20, "step": "1e-5 / max|dm| (relative to the density scale)",
                               "max_rel_err": float(errs.max()), "median_rel_err": float(np.median(errs)),
                               "passed_1e-6": int((errs <= 1e-6).sum())},
    }


PATTERN_CHAINS_S8_E4 = {
    # 0-based evaluated stages of the E = 4 member in an S = 8 family: the classic chain (the last
    # three stages), and the alternating and early-shared chains of Sec. 3.2.4 carried over from
    # the printed S = 6 examples ({1,3,4,6} -> {1,5,6,8}, {1,2,3,6} -> {1,2,3,8}, 1-based)
    "classic": [0, 5, 6, 7],
    "alternating": [0, 4, 5, 7],
    "early_shared": [0, 1, 2, 7],
}


def run_patterns(args):
    """Alternative stage-evaluation patterns (Sec. 3.2.4) on the same kernels: the 2-level band
    mesh (64^2 roots, band refined: 7168 elements, p = 3, Kelvin-Helmholtz state), P-ERK2{4,8}
    from the product's optimisation, the E = 4 member (3072 coarse elements) on each chain of
    PATTERN_CHAINS_S8_E4 in turn, the same polynomials.  Per pattern: DoF-updates/s over the
    timed steps (graph replay) and the stage kernel's event-timed launches (roofline as for the
    main workloads)."""
    import torch
    import perk_inputs as pin
    from paper_2403_05144_amd import PerkSolver, coeffs
    mesh = pin.mesh_band_2level(64)
    ic = lambda x: pin.kelvin_helmholtz(x[0], x[1])
    base = family_for("perk2_4_8_kh_p3_n8", 2, [4, 8], pin.uniform_mesh(2, (8, 8), (-1, -1), (1, 1), 0), 3, ic, 0.25)
    mol = [0, 1]
    dt = stable_dt(base, mesh, mol, 0.5)
    rows = {}
    for kind, chain in PATTERN_CHAINS_S8_E4.items():
        fam = coeffs.with_chains(base, [chain, None])
        s = PerkSolver(mesh, 3, fam, mol)
        x = s.node_coords().cpu().numpy().transpose(1, 0, 2)
        s.set_state(ic(x).transpose(1, 0, 2).copy())
        s.step(dt, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(dt, args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if not np.all(np.isfinite(s.get_state().cpu().numpy())):
            raise RuntimeError(f"patterns: non-finite state ({kind})")
        s.set_profiling(True)
        s.step(dt, min(args.steps, 20))
        torch.cuda.synchronize()
        ms, nl, es = s.profile_stats()
        s.set_profiling(False)
        esl = es / max(1, nl)
        roof = roofline_of("k_stage", ms, nl, esl * bytes_per_element_stage(2, 4), esl * flops_per_element_stage(2, 4))
        roof["element_stages_per_launch"] = esl
        dofs = s.n_elements * s.nv * s.Nd
        rows[kind] = {"chain_E4": chain, "dof_updates_per_s": dofs * args.steps / wall,
                      "ms_per_step": wall / args.steps * 1e3, "roofline": roof}
        _log(f"patterns {kind}: {rows[kind]['dof_updates_per_s']:.3e} DoF-updates/s, "
             f"{roof['avg_launch_us']:.2f} us per launch, frac {roof['frac']:.3f}")
        del s
    c = rows["classic"]
    return {
        "metric": "DoF-updates/s & PID; P-ERK vs single-level RK wall time at equal error",
        "value": c["dof_updates_per_s"], "unit": "DoF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": c["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "patterns_band64", "elements": 7168, "degree": 3, "family_E": [4, 8], "dt": dt,
                   "description": "2D Euler Kelvin-Helmholtz state on the 2-level band mesh (64^2 roots, 7168 "
                                  "elements, p=3), P-ERK2{4,8} with the E=4 member on the classic, alternating "
                                  "and early-shared stage chains (same polynomials); value: classic chain"},
        "roofline": c["roofline"], "patterns": rows,
    }


def spectrum_at_mesh(wl, m):
    """Spectrum estimation at the workload's real mesh (Sec. 4.1, steps 2-4) on the GPU: the hull
    points of the reduced-mesh spectrum, scaled by h_reduced / h, as targets; one Arnoldi
    factorisation of m steps of the Jacobian at the initial state (Euler: exact products from the
    forward-mode kernel; Navier-Stokes: central differences); Ritz values plus the harmonic Ritz
    values nearest to every target; then the P-ERK family optimised on those eigenvalues (h_ref =
    the smallest element size).  Returns (family, report)."""
    import torch
    import perk_inputs as pin
    from paper_2403_05144_amd import coeffs
    from paper_2403_05144_amd.amr import AmrDriver
    fam, mesh, op = wl["fam"], wl["mesh"], wl["spectrum_op"]
    m0 = pin.MeshDesc(mesh.dim, mesh.n_root, mesh.lo, mesh.hi, np.array(mesh.leaves, copy=True))
    s = make_solver(wl, m0, fam, wl["mol"])
    ic_leaf = lambda x: wl["ic"](x.transpose(1, 0, 2)).transpose(1, 0, 2).copy()
    if wl.get("amr"):
        a = wl["amr"]
        AmrDriver(s, a["level_min"], a["level_max"], wl["mol"], a["refine_above"], a["coarsen_below"],
                  a["interval"]).initial_mesh(ic_leaf, passes=3)
    else:
        s.set_state(ic_leaf(s.node_coords().cpu().numpy()))
    # reduced spectrum of the family's own construction (its reduced mesh and element size)
    rs = make_solver(dict(wl, amr=None), wl["reduced_mesh"], fam, [0] * 8)
    rs.set_state(ic_leaf(rs.node_coords().cpu().numpy()))
    t0 = time.perf_counter()
    lam_red = coeffs.fd_spectrum(rs, rs.get_state().cpu().numpy())
    t_red = time.perf_counter() - t0
    del rs
    lv = s.leaves()[:, 0]
    h_min = (mesh.hi[0] - mesh.lo[0]) / (mesh.n_root[0] << int(lv.max()))
    u = s.u.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = coeffs.arnoldi(s, u, m, op=op)
    torch.cuda.synchronize()
    t_arn = time.perf_counter() - t0
    t0 = time.perf_counter()
    shifts = coeffs.hull_points(lam_red) * (fam.h_ref / h_min)
    per = max(1, 1000 // max(1, len(shifts)))
    ritz = np.linalg.eigvals(H[: H.shape[1], : H.shape[1]])
    est = [ritz]
    for sg in shifts:
        th = coeffs.harmonic_ritz(H, sg)
        est.append(th[np.argsort(np.abs(th - sg))[:per]])
    lam = np.concatenate(est)
    lam = lam[np.isfinite(lam) & (lam.imag >= 0)]
    lam.real = np.minimum(lam.real, 0.0)
    t_eig = time.perf_counter() - t0
    full = coeffs.build_family(fam.order, fam.E, coeffs.hull_points(lam), h_ref=h_min)
    scaled_red = [d * h_min / fam.h_ref for d in fam.dt_opt]
    n = int(s.n_elements * s.nv * s.Nd)
    rep = {"elements": int(s.n_elements), "unknowns": n, "arnoldi_steps": int(H.shape[1]),
           "products": {"jvp": "exact J (forward-mode kernel)", "vjp": "exact J^T (adjoint kernel)",
                        "fd": "central differences of F"}[op],
           "targets": int(len(shifts)), "eigenvalue_estimates": int(len(lam)),
           "spectral_radius_estimate": float(np.abs(lam).max()),
           "reduced_spectral_radius_scaled": float(np.abs(lam_red).max() * fam.h_ref / h_min),
           "arnoldi_s": t_arn, "eigen_s": t_eig, "reduced_spectrum_s": t_red,
           "dt_opt_full_mesh": [float(x) for x in full.dt_opt],
           "dt_opt_reduced_scaled": [float(x) for x in scaled_red],
           "E": list(fam.E)}
    _log(f"spectrum {wl['name']}: {H.shape[1]} Arnoldi steps on {n} unknowns in {t_arn:.2f} s, "
         f"{len(lam)} estimates; dt_opt full {np.round(full.dt_opt, 6)} vs reduced {np.round(scaled_red, 6)}")
    del s
    torch.cuda.empty_cache()
    return full, rep


def full_mesh_family(wl, m=200):
    """The workload's family optimised on the spectrum at its real mesh (spectrum_at_mesh), cached
    as JSON next to the reduced-mesh one."""
    from paper_2403_05144_amd import coeffs
    path = os.path.join(ROOT, "paper_2403_05144_amd", "data", f"{wl['fam_name']}_fullmesh.json")
    if os.path.exists(path):
        return coeffs.Family.load(path), None
    _log(f"building coefficient family {wl['fam_name']}_fullmesh (spectrum at the real mesh)")
    fam, rep = spectrum_at_mesh(wl, m)
    fam.save(path)
    return fam, rep


def run_spectrum(args):
    """Spectrum estimation at the real meshes of the KH and TGV workloads (spectrum_at_mesh) and
    the families optimised on them (stored next to the reduced-mesh families when missing).
    Timed: the Arnoldi factorisation (device) and the eigenvalue extraction (host)."""
    out = {}
    for key, mk in (("kh_amr_l3-6", wl_kh_amr), ("tgv_ns_3d", wl_tgv)):
        wl = mk()
        fam, rep = spectrum_at_mesh(wl, args.arnoldi_steps)
        from paper_2403_05144_amd import coeffs
        path = os.path.join(ROOT, "paper_2403_05144_amd", "data", f"{wl['fam_name']}_fullmesh.json")
        if not os.path.exists(path):
            fam.save(path)
        rep["family_file"] = os.path.relpath(path, ROOT)
        out[key] = rep
    k = out["tgv_ns_3d"]
    return {"metric": "DoF-updates/s & PID; P-ERK vs single-level RK wall time at equal error",
            "value": k["unknowns"] * k["arnoldi_steps"] / k["arnoldi_s"], "unit": "DoF-updates/s",
            "n_gpus": 1, "steps": k["arnoldi_steps"], "warmup": 0, "ms_per_step": k["arnoldi_s"] / k["arnoldi_steps"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "spectrum", "description": "Arnoldi spectrum estimation at the real meshes of the "
                       "KH and TGV workloads (value: TGV unknowns x Arnoldi steps per second)"},
            "spectra": out}


def run_sweep(args):
    """Stage-kernel throughput on uniform single-level meshes, every element active at every
    stage: 2D p=3 Euler on 64^2 ... 1024^2 elements (isentropic vortex, P-ERK2;8 alone) and 3D
    p=3 Euler on 16^3 ... 48^3 (Taylor-Green state, P-ERK2;16 alone).  Per size: the stage
    kernel's average launch (HIP events on the launch stream), element-stages per second and the
    roofline fractions of the algorithmic bytes and flops; the line's value is the whole-step
    DoF-update rate (graph replay) of the largest 2D mesh."""
    import torch
    import perk_inputs as pin
    from paper_2403_05144_amd import PerkSolver
    cases = [(2, n) for n in (64, 128, 256, 512, 1024)] + [(3, n) for n in (16, 24, 32, 48)]
    if args.sweep_max:
        cases = [(d, n) for d, n in cases if n ** d <= args.sweep_max]
    rows = []
    value = None
    for dim, n in cases:
        if dim == 2:
            fam = single_member_family(vortex_family(3, (4, 8)), 1)
            mesh = pin.uniform_mesh(2, (n, n), (-5, -5), (5, 5), 0)
            ic = lambda x: pin.isentropic_vortex(x[0], x[1])
        else:
            fam = single_member_family(wl_tgv()["fam"], 2)
            mesh = pin.uniform_mesh(3, (n, n, n), (-np.pi,) * 3, (np.pi,) * 3, 0)
            ic = lambda x: pin.taylor_green(x[0], x[1], x[2])
        s = PerkSolver(mesh, 3, fam, [0])
        x = s.node_coords().cpu().numpy().transpose(1, 0, 2)
        s.set_state(ic(x).transpose(1, 0, 2).copy())
        dt = stable_dt(fam, mesh, [0], 0.5)
        s.step(dt, 2)
        torch.cuda.synchronize()
        steps = max(2, min(50, int(2e6 // (n ** dim))))
        t0 = time.perf_counter()
        s.step(dt, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.set_profiling(True)
        s.step(dt, min(steps, 10))
        torch.cuda.synchronize()
        ms, nl, es = s.profile_stats()
        s.set_profiling(False)
        if not np.all(np.isfinite(s.get_state().cpu().numpy())):
            raise RuntimeError(f"sweep: non-finite state at {dim}D {n}^{dim}")
        launch_s = ms * 1e-3 / nl
        rate = (es / nl) / launch_s
        B, F = bytes_per_element_stage(dim, 4), flops_per_element_stage(dim, 4)
        dofs = s.n_elements * s.nv * s.Nd
        row = {"dim": dim, "elements": int(s.n_elements), "avg_launch_us": launch_s * 1e6,
               "element_stages_per_s": rate, "ns_per_element_stage": 1e9 / rate,
               "hbm_frac": B * rate / (HBM_PEAK_GBS * 1e9), "alu_frac": F * rate / (FP64_PEAK_TFLOPS * 1e12),
               "dof_updates_per_s": dofs * steps / wall}
        rows.append(row)
        _log(f"sweep {dim}D {n}^{dim}: {row['ns_per_element_stage']:.3f} ns/element-stage, "
             f"HBM {row['hbm_frac']:.3f}, ALU {row['alu_frac']:.3f}")
        if dim == 2:
            value = (row["dof_updates_per_s"], steps, wall, int(s.n_elements))
        del s
        torch.cuda.empty_cache()
    big = max((r for r in rows if r["dim"] == 2), key=lambda r: r["elements"])
    roof_b, roof_f = big["hbm_frac"], big["alu_frac"]
    B, F = bytes_per_element_stage(2, 4), flops_per_element_stage(2, 4)
    if roof_b >= roof_f:
        roof = {"bound": "hbm", "achieved": B * big["element_stages_per_s"] / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": roof_b}
    else:
        roof = {"bound": "alu", "achieved": F * big["element_stages_per_s"] / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": roof_f}
    roof.update({"traffic": None, "kernel": "k_stage", "avg_launch_us": big["avg_launch_us"],
                 "element_stages_per_launch": big["elements"]})
    return {
        "metric": "DoF-updates/s & PID; P-ERK vs single-level RK wall time at equal error",
        "value": value[0], "unit": "DoF-updates/s", "n_gpus": 1, "steps": value[1], "warmup": 2,
        "ms_per_step": value[2] / value[1] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "uniform_sweep", "description": "stage kernel on uniform single-level meshes, "
                   "2D p=3 Euler 64^2..1024^2 (P-ERK2;8 alone), 3D p=3 Euler 16^3..48^3 (P-ERK2;16 alone); "
                   "value: the largest 2D mesh"},
        "roofline": roof, "sweep": rows,
    }


def wl_kh_paper(fam=None, refine_above=0.01, coarsen_below=0.001):
    """The paper's inviscid Kelvin-Helmholtz run (Sec. 7.2.1, eq. KelvinHelmholtzIC): Euler on
    [-1,1]^2, 16x16 roots refined up to five times (finest h = 2^-8) where the shock-capturing
    indicator of the density asks for it, subcell shock capturing (alpha_max 0.5, alpha_min 0.001),
    p = 3, EC volume + HLL surface flux, P-ERK3{4,6,11} optimised on the spectrum of the 4x4 mesh
    (1024 unknowns, with shock capturing), levels by the paper's rule (finest E = 11, next E = 6,
    the rest E = 4), adaptation every 10 steps, t in [0, 3]."""
    import perk_inputs as pin
    from paper_2403_05144_amd.partition_rule import LevelRule
    mesh = pin.uniform_mesh(2, (16, 16), (-1, -1), (1, 1), 0)
    ic = lambda x: pin.kelvin_helmholtz_paper(x[0], x[1])
    h_red = 0.5
    red = pin.uniform_mesh(2, (4, 4), (-1, -1), (1, 1), 0)
    sc = (0.5, 0.001)
    fam_name = "perk3_4_6_11_khsc_p3"
    if fam is None:
        fam = family_for(fam_name, 3, [4, 6, 11], red, 3, ic, h_red, shock_capturing=sc)
    level_max = 5
    rule = LevelRule.paper()
    mol = rule_map(fam, rule, level_max)
    # the members' optimised steps on the reduced mesh overestimate what this flow tolerates: at
    # CFL 0.5 of the standalone P-ERK3;11's bound a uniform 128^2 run blows up before t = 1.7, at
    # 0.35 it reaches t = 3; the family on the adaptive mesh runs at 0.3 of its binding member
    cfl = 0.3
    levels = pin.MeshDesc(2, mesh.n_root, mesh.lo, mesh.hi, np.array([[l, 0, 0, 0] for l in range(level_max + 1)]))
    dt = stable_dt(fam, levels, mol, cfl)
    return dict(name="kh_paper_sc", mesh=mesh, degree=3, fam=fam, fam_name=fam_name, mol=mol, rule=rule, ic=ic,
                dt=dt, cfl=cfl, t_final=3.0, shock_capturing=sc, spectrum_op="fd", reduced_mesh=red, h_reduced=h_red,
                amr=dict(level_min=0, level_max=level_max, interval=10, refine_above=refine_above,
                         coarsen_below=coarsen_below, capacity=1 << 18, indicator=("hennemann_gassner", 0, 0.0)),
                perk_maps=[("paper rule", mol)],
                desc="the paper's inviscid Kelvin-Helmholtz instability (eq. KelvinHelmholtzIC) on [-1,1]^2, p=3, EC "
                     "volume + HLL surface flux, subcell shock capturing on the density (alpha_max 0.5), quadtree AMR "
                     "on the same indicator between levels 4 and 9 every 10 steps with re-partition after every "
                     f"adaptation, P-ERK3{{4,6,11}} with levels mapped to E={[fam.E[r] for r in mol]} (paper rule), "
                     f"CFL {cfl} of the binding member's optimised step")


WORKLOADS = {"vortex_2level": wl_vortex_2level, "kh_amr": wl_kh_amr, "tgv": wl_tgv, "batch_vortex64": None,
             "adjoint_kh": None, "uniform_sweep": None, "patterns": None, "shear_layer": wl_shear_layer,
             "spectrum": None, "kh_paper": wl_kh_paper,
             "kh_amr_l4-7": lambda: wl_kh_amr(16, 3, "kh_amr_l4-7")}


# ----------------------------------------------------------------------------------------
def cpu_baseline(wl, u0_leaf, leaves0, budget_s=15.0):
    """The oracle (serial C++, one core) on a bounded number of steps of the same workload
    (the starting mesh; no adaptation inside the sample)."""
    import perk_inputs as pin
    from oracle import dgsem as od
    from oracle import perk_coeffs as pc
    m0 = wl["mesh"]
    mesh = pin.MeshDesc(m0.dim, m0.n_root, m0.lo, m0.hi, leaves0)
    o = od.Oracle(mesh, wl["degree"] + 1, viscous=wl.get("equations", 0) == 1, mu=wl.get("mu", 0.0))
    if wl.get("shock_capturing"):
        o.set_shock_capturing(True, *wl["shock_capturing"])
    fam = wl["fam"]
    ofam = pc.PerkFamily(fam.order, fam.S, list(fam.E), np.asarray(fam.c), np.asarray(fam.b),
                         np.asarray(fam.a_sub))
    member = np.asarray(wl["mol"])[mesh.leaves[:, 0]]
    u = np.array(u0_leaf, copy=True)
    n, t0 = 0, time.perf_counter()
    while True:
        u = o.prk_step(u, wl["dt"], ofam, member)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 1000:
            break
    dofs = mesh.n_elements * (mesh.dim + 2) * (wl["degree"] + 1) ** mesh.dim
    host = host_cpu()
    return {"value": n * dofs / el, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} P-ERK steps of the same workload ({el:.1f} s, serial C++ oracle, dense "
                      f"masked stages: every stage evaluated on every element)",
            "cpu_model": host["model"], "host_cores_total": host["cores_total"],
            "host_cores_available": host["cores_available"]}


def host_cpu():
    """Model name of the host CPU (as lscpu reports it) and its core counts."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"model": model, "cores_total": os.cpu_count(), "cores_available": avail}


# ----------------------------------------------------------------------------------------
# P-ERK against single-level schemes on the same kernels, at equal error
# ----------------------------------------------------------------------------------------
def single_member_family(fam, r):
    """Member r of a family run alone on every element (standalone P-ERK_{p;E_r})."""
    from paper_2403_05144_amd import coeffs
    return coeffs.Family(fam.order, fam.S, [fam.E[r]], np.asarray(fam.c), np.asarray(fam.b),
                         np.asarray(fam.a_sub)[r:r + 1].copy(), [fam.dt_opt[r]], fam.h_ref)


def standard_rk_family(fam):
    """The order's classical low-storage scheme written in P-ERK form with S = E = p: the
    explicit midpoint rule for p = 2, Shu-Osher SSPRK33 for p = 3 (c = (0, 1, 1/2),
    a_{3,2} = a_{3,1} = 1/4, b = (1/6, 1/6, 2/3)).  Its CFL-1 step is the first member's optimal
    step scaled by the stage ratio; the stability scan fixes the usable fraction."""
    from paper_2403_05144_amd import coeffs
    S = fam.order
    a = np.zeros((1, S))
    if S == 3:
        a[0, 2] = 0.25
    return coeffs.Family(fam.order, S, [S], coeffs.abscissae(fam.order, S), coeffs.weights(fam.order, S), a,
                         [fam.dt_opt[0] * S / fam.E[0]], fam.h_ref)


def _dt_cfl1(wl, fam1, mol1, levels):
    m = wl["mesh"]
    h = lambda l: (m.hi[0] - m.lo[0]) / (m.n_root[0] << int(l))
    return min(fam1.dt_opt[mol1[int(l)]] * h(l) / fam1.h_ref for l in levels)


def _steps_per_interval(spi, n_int):
    """Integer step counts of n_int intervals that add up to round(spi * n_int)."""
    edges = np.floor(np.arange(n_int + 1) * spi + 1e-9).astype(int)
    return np.diff(edges)


def _kinetic_energy(u_leaf, w_leaf, dim):
    """Discrete total kinetic energy sum_nodes w |rho v|^2 / (2 rho) of a leaf-layout state."""
    mom2 = np.sum(u_leaf[:, 1:1 + dim] ** 2, axis=1)
    return float(np.sum(w_leaf * 0.5 * mom2 / u_leaf[:, 0]))


def _integrate(wl, fam1, mol1, start, T_int, n_int, spi, flags=None, record=False, reps=1):
    """One run over [0, n_int T_int] with round(spi n_int) steps; the kinetic energy is sampled
    at the end of every interval (its host time is left out of the wall time).  Interval k takes
    its share steps_k of the steps with dt = T_int / steps_k, so that every sample is taken at the
    interval's end exactly (with one dt for the whole run and step counts that do not divide
    evenly, the samples would sit up to a step away from the reference's, and the kinetic
    energy's change over that offset would swamp the error being measured).  An adaptive mesh
    adapts between intervals (recording the flags from the GPU indicator, or replaying recorded
    ones).  Returns the wall time of the stepping and adaptation (graph replay path; the
    smallest of `reps` runs, repeated on the same solver for a static mesh and on a fresh one
    for an adaptive mesh), the final state and mesh, the kinetic-energy history and the
    element-RHS count."""
    import torch
    import perk_inputs as pin
    from paper_2403_05144_amd import PerkError, PerkSolver
    from paper_2403_05144_amd.amr import AmrDriver
    m0 = wl["mesh"]
    amr = wl.get("amr")
    steps = _steps_per_interval(spi, n_int)
    s, walls, rec, ok, ke = None, [], [], True, []
    for rep in range(reps):
        if s is None or amr:
            s = None
            mesh = pin.MeshDesc(m0.dim, m0.n_root, m0.lo, m0.hi, np.array(start["leaves"], copy=True))
            s = make_solver(wl, mesh, fam1, mol1)
        s.set_state(start["u"])
        drv = AmrDriver(s, amr["level_min"], amr["level_max"], mol1, amr["refine_above"], amr["coarsen_below"],
                        0) if (amr and record and rep == 0) else None
        s.counters(reset=True)
        w_static = None if amr else s.node_weights()
        ke_rep, excluded = [], 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            for k in range(n_int):
                dt_k = T_int / steps[k]
                s.step(dt_k, int(steps[k]))
                if rep == 0:
                    torch.cuda.synchronize()
                    ts = time.perf_counter()
                    w = s.node_weights() if amr else w_static
                    ke_rep.append(_kinetic_energy(s.get_state().cpu().numpy(), w, m0.dim))
                    excluded += time.perf_counter() - ts
                if amr and k < n_int - 1:
                    if drv is not None:
                        rec.append(drv.adapt_once())
                    else:
                        s.adapt((flags if flags is not None else rec)[k], amr["level_min"], amr["level_max"], mol1)
            torch.cuda.synchronize()
        except PerkError as e:
            _log(f"run stopped: {e}")
            ok = False
            break
        walls.append(time.perf_counter() - t0 - excluded)
        if rep == 0:
            ke = ke_rep
    out = {"ok": ok, "wall": min(walls) if walls else float("nan"), "steps": int(steps.sum()), "flags": rec,
           "ke": np.array(ke)}
    if ok:
        out["u"] = s.get_state().cpu().numpy()
        out["leaves"] = s.leaves()
        out["w"] = s.node_weights()
        out["element_rhs"] = s.counters()[0]
    del s
    return out


def _stable(run, rho0_max):
    if not run["ok"]:
        return False
    rho = run["u"][:, 0]
    return bool(np.all(np.isfinite(run["u"])) and rho.min() > 0 and rho.max() < 2 * rho0_max)


NORMS = ("L1", "Linf", "KE")


def _errors(run, ref):
    """Errors of a run against the reference: density quadrature L1 (domain mean) and nodal max
    of the final state, and the largest deviation of the kinetic-energy history (sampled at the
    end of every interval) relative to the reference's first sample."""
    if ref.get("exact") is not None:
        r_ref, ke_ref = ref["exact"](run)
    else:
        if not np.array_equal(run["leaves"], ref["leaves"]):
            raise RuntimeError("compared runs ended on different meshes")
        r_ref, ke_ref = ref["u"][:, 0], ref["ke"]
    d = np.abs(run["u"][:, 0] - r_ref)
    ke = np.abs(run["ke"] - ke_ref) / abs(ke_ref[0])
    return {"L1": float(np.sum(run["w"] * d) / np.sum(run["w"])), "Linf": float(d.max()), "KE": float(ke.max())}


def _excess(err, target):
    """Largest ratio of a run's errors to the target errors over the norms."""
    return max(err[n] / target[n] for n in NORMS if target[n] > 0)


CFL_SCAN = (1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2, 0.15, 0.1)


def compare_equal_error(wl, t_final=None, tol=0.05, ref_budget=6e8):
    """Wall time of the P-ERK family against (a) the standalone P-ERK_{p;E_max} on every element
    and (b) the order's classical scheme (explicit midpoint / SSPRK33), all on these kernels.

    Every scheme runs at the largest CFL of CFL_SCAN that keeps the density finite, positive and
    below twice its initial maximum over the horizon.  Errors (three norms: density L1 over the
    domain and nodal max of the final state, and the kinetic-energy history sampled ten times
    over the horizon) are taken against the exact solution where one exists (isentropic vortex)
    and otherwise against the standalone P-ERK_{p;E_max} at an eighth of the finest step used, on
    the same mesh sequence (adaptive meshes replay the P-ERK run's flags).

    Equal error: of each pair, the target in every norm is the smaller of the two errors at the
    largest stable CFLs; each scheme whose error exceeds the target in some norm by more than
    tol has its step shrunk (secant on the log of its largest error/target ratio against the
    log of the step count, then bisection) until its largest ratio is within 1 + tol, so that
    at the end both schemes are at least as accurate as the target in every norm.  Both are then
    timed again.  The P-ERK family is tried with every level -> member map the workload lists;
    the one with the shortest wall time at its largest stable CFL is compared.  A comparator
    whose reference run would exceed ref_budget element-stage evaluations is left out (reported
    as such)."""
    import perk_inputs as pin
    import torch
    from paper_2403_05144_amd import PerkSolver
    from paper_2403_05144_amd.amr import AmrDriver
    fam, mol, m0 = wl["fam"], wl["mol"], wl["mesh"]
    amr = wl.get("amr")
    R = len(fam.E)
    # start state (adaptive workloads: the initial mesh built from the initial condition)
    mesh = pin.MeshDesc(m0.dim, m0.n_root, m0.lo, m0.hi, np.array(m0.leaves, copy=True))
    s = make_solver(wl, mesh, fam, mol)
    ic_leaf = lambda x: wl["ic"](x.transpose(1, 0, 2)).transpose(1, 0, 2).copy()
    if amr:
        AmrDriver(s, amr["level_min"], amr["level_max"], mol, amr["refine_above"], amr["coarsen_below"],
                  amr["interval"]).initial_mesh(ic_leaf, passes=3)
    else:
        s.set_state(ic_leaf(s.node_coords().cpu().numpy()))
    start = {"leaves": s.leaves(), "u": s.get_state().cpu().numpy()}
    torch.cuda.synchronize()
    del s
    rho0_max = float(start["u"][:, 0].max())
    levels = range(amr["level_max"] + 1) if amr else np.unique(start["leaves"][:, 0])
    if amr:
        T_int = amr["interval"] * wl["dt"]
        n_int = int(math.ceil((t_final or wl["t_final"]) / T_int))
    else:
        n_int = 10                      # kinetic-energy samples; one constant step over the horizon
        T_int = (t_final or wl["t_final"] or 200 * wl["dt"]) / n_int
    t_end = n_int * T_int
    Lmax = int(max(levels))
    schemes = {
        "single_level": (single_member_family(fam, R - 1), [0] * (Lmax + 1)),
        "standard_rk": (standard_rk_family(fam), [0] * (Lmax + 1)),
    }
    names = {"p_erk": f"P-ERK{fam.order} E={list(fam.E)}",
             "single_level": f"standalone P-ERK{fam.order};{fam.E[-1]} on every element",
             "standard_rk": "SSPRK33 (Shu-Osher)" if fam.order == 3 else "explicit midpoint RK2"}

    def scan(key, f1, m1, flags, record):
        dt1 = _dt_cfl1(wl, f1, m1, levels)
        for cfl in CFL_SCAN:
            spi = max(1.0, T_int / (cfl * dt1))
            spi = float(math.ceil(spi * n_int - 1e-9)) / n_int
            run = _integrate(wl, f1, m1, start, T_int, n_int, spi, flags=flags, record=record)
            if _stable(run, rho0_max):
                _log(f"equal-error: {key} largest stable CFL {cfl}, {run['steps']} steps")
                return {"cfl_max": cfl, "spi": spi, "run": run}
            _log(f"equal-error: {key} unstable at CFL {cfl}")
        raise RuntimeError(f"{key}: no stable CFL in the scan")

    # P-ERK: every candidate level -> member map at its largest stable CFL (adaptive meshes record
    # their own flags); the fastest one is compared with the single-level schemes
    candidates = []
    for label, m1 in wl.get("perk_maps", [("workload map", list(mol))]):
        c = scan(f"P-ERK ({label})", fam, list(m1), None, bool(amr))
        t2 = _integrate(wl, fam, list(m1), start, T_int, n_int, c["spi"], flags=c["run"]["flags"] or None,
                        reps=2 if amr else 5)
        c.update(label=label, mol=list(m1), wall=min(c["run"]["wall"], t2["wall"]))
        candidates.append(c)
    best = min(candidates, key=lambda c: c["wall"])
    schemes["p_erk"] = (fam, best["mol"])
    flags = best["run"]["flags"] if amr else None
    info = {"p_erk": best}
    for key in ("single_level", "standard_rk"):
        info[key] = scan(key, *schemes[key], flags, False)
    skipped = {}
    n_e0 = len(start["leaves"])
    cost = 8 * max(v["spi"] for v in info.values()) * n_int * fam.E[-1] * n_e0
    if wl["name"] != "vortex_2level" and cost > ref_budget:
        info.pop("standard_rk")
        skipped[names["standard_rk"]] = (f"not compared: a reference at 1/8 of its step would cost about "
                                         f"{cost:.2g} element-stage evaluations")
        _log(f"equal-error: {names['standard_rk']} skipped (reference cost {cost:.2g} element-stages)")
    # reference
    if wl["name"] == "vortex_2level":
        x_cache = {}

        def exact(run):
            key = run["leaves"].tobytes()
            if key not in x_cache:
                mesh = pin.MeshDesc(m0.dim, m0.n_root, m0.lo, m0.hi, run["leaves"])
                sx = PerkSolver(mesh, wl["degree"], fam, mol)
                x = sx.node_coords().cpu().numpy().transpose(1, 0, 2)
                w = sx.node_weights()
                kes = [_kinetic_energy(pin.isentropic_vortex(x[0], x[1], t=(k + 1) * T_int).transpose(1, 0, 2), w, 2)
                       for k in range(n_int)]
                x_cache[key] = (pin.isentropic_vortex(x[0], x[1], t=t_end)[0].copy(), np.array(kes))
                del sx
            return x_cache[key]
        ref = {"exact": exact, "what": "exact solution"}
    else:
        spi_ref = 8 * max(v["spi"] for v in info.values())
        f1, m1 = schemes["single_level"]
        _log(f"equal-error: reference run, {int(round(spi_ref * n_int))} steps")
        rr = _integrate(wl, f1, m1, start, T_int, n_int, spi_ref, flags=flags)
        if not _stable(rr, rho0_max):
            raise RuntimeError("reference run unstable")
        ref = {"u": rr["u"], "leaves": rr["leaves"], "ke": rr["ke"], "what": f"{names['single_level']} with "
               f"{rr['steps']} steps (1/8 of the finest step used), same mesh sequence"}
    for v in info.values():
        v["run"]["err"] = _errors(v["run"], ref)
    for c in candidates:             # other maps: own mesh sequence under adaptation, no common reference
        if c is not best:
            c["run"]["err"] = None if amr else _errors(c["run"], ref)

    def run_at(key, spi):
        f1, m1 = schemes[key]
        r = _integrate(wl, f1, m1, start, T_int, n_int, spi, flags=flags)
        r["err"] = _errors(r, ref)
        return r

    def summary(key, spi, r):
        t2 = _integrate(wl, *schemes[key], start, T_int, n_int, spi, flags=flags, reps=2 if amr else 5)
        return {"scheme": names[key], "steps": r["steps"], "dt_mean": t_end / r["steps"],
                "err": r["err"], "wall_s": min(r["wall"], t2["wall"]), "element_rhs": r["element_rhs"]}

    def shrink(key, spi, run, target):
        """Smallest step count found (up from spi) at which every error of `key` is within
        1 + tol of the target; its (spi, run) and the search history.  The step count grows at
        most 8-fold per try and to at most 64 times the start (an error that stalls against the
        reference's own error would otherwise send it off); (None, None, history) if the target
        is not reached."""
        g = lambda r: _excess(r["err"], target)
        lo, hi = (spi, run), None           # not accurate enough / accurate enough
        hist = [(spi, g(run))]
        if g(run) <= 1 + tol:
            return spi, run, hist
        for _ in range(12):
            if hi is None:
                if len(hist) >= 2 and hist[-1][1] != hist[-2][1]:
                    (s1, e1), (s2, e2) = hist[-2], hist[-1]
                    slope = min(-0.5, (math.log(e2) - math.log(e1)) / (math.log(s2) - math.log(s1)))
                else:
                    slope = -float(fam.order)
                spi_new = min(lo[0] * (1.0 / g(lo[1])) ** (1.0 / slope), 8.0 * lo[0])
                spi_new = max(lo[0] + 1.0 / n_int, float(math.ceil(spi_new * n_int - 1e-9)) / n_int)
                if spi_new > 64.0 * spi:
                    break
            else:
                spi_new = float(round(0.5 * (lo[0] + hi[0]) * n_int)) / n_int
                if spi_new <= lo[0] or spi_new >= hi[0]:
                    break
            r_new = run_at(key, spi_new)
            hist.append((spi_new, g(r_new)))
            _log(f"equal-error:   {key}: {r_new['steps']} steps, largest error/target {g(r_new):.3f}")
            if g(r_new) > 1 + tol:
                lo = (spi_new, r_new)
            else:
                hi = (spi_new, r_new)
                if g(r_new) >= 1 - tol:
                    break
        if hi is None:
            _log(f"equal-error: {key} did not reach the target errors")
            return None, None, hist
        return hi[0], hi[1], hist

    pairs = []
    for other in [k for k in ("single_level", "standard_rk") if k in info]:
        e_p, e_c = info["p_erk"]["run"]["err"], info[other]["run"]["err"]
        target = {n: min(e_p[n], e_c[n]) for n in NORMS}
        res = {}
        for key in ("p_erk", other):
            spi0, run0 = info[key]["spi"], info[key]["run"]
            res[key] = shrink(key, spi0, run0, target)
            if res[key][1] is None:
                break
            _log(f"equal-error: {key} vs {other}: {res[key][1]['steps']} steps (from {run0['steps']}), largest "
                 f"error/target {_excess(res[key][1]['err'], target):.3f}")
        if any(r[1] is None for r in res.values()):
            miss = [k for k, r in res.items() if r[1] is None]
            pairs.append({"comparator_scheme": names[other], "target_err": target, "p_erk_err": e_p,
                          "comparator_err": e_c, "not_reached": miss,
                          "search": {k: [(float(a), float(b)) for a, b in res[k][2]] for k in res}})
            continue
        t_c = _integrate(wl, *schemes[other], start, T_int, n_int, info[other]["spi"], flags=flags,
                         reps=2 if amr else 5)
        wall_c_max = min(info[other]["run"]["wall"], t_c["wall"])
        at_max = {"p_erk_steps": best["run"]["steps"], "comparator_steps": info[other]["run"]["steps"],
                  "p_erk_wall_s": best["wall"], "comparator_wall_s": wall_c_max,
                  "p_erk_err": e_p, "comparator_err": e_c,
                  "wall_ratio_comparator_over_p_erk": wall_c_max / best["wall"]}
        sp, sc = summary("p_erk", res["p_erk"][0], res["p_erk"][1]), summary(other, res[other][0], res[other][1])
        pairs.append({"at_cfl_max": at_max, "target_err": target, "comparator": sc, "p_erk": sp,
                      "comparator_cfl_max": info[other]["cfl_max"],
                      "shrunk": [k for k in ("p_erk", other) if res[k][1] is not info[k]["run"]],
                      "search": {k: [(float(a), float(b)) for a, b in res[k][2]] for k in res},
                      "largest_error_over_target": {"p_erk": _excess(sp["err"], target),
                                                    "comparator": _excess(sc["err"], target)},
                      "wall_ratio_comparator_over_p_erk": sc["wall_s"] / sp["wall_s"],
                      "element_rhs_ratio": sc["element_rhs"] / sp["element_rhs"]})
        _log(f"equal-error: {other}: wall ratio {sc['wall_s'] / sp['wall_s']:.3f} with every error within "
             f"{1 + tol:.2f} of the target {target}")
    cand_out = [{"map": c["label"], "E_of_level": [int(fam.E[r]) for r in c["mol"]], "cfl_max": c["cfl_max"],
                 "steps": c["run"]["steps"], "wall_s_at_cfl_max": c["wall"], "element_rhs": c["run"]["element_rhs"],
                 "err": c["run"]["err"], "chosen": c is best}
                for c in candidates]
    return {"workload": wl["name"], "t_final": t_end, "p_erk_cfl_max": info["p_erk"]["cfl_max"],
            "p_erk_maps": cand_out,
            "cfl": "fraction of the scheme's own largest linearly stable step (optimised stability polynomial, "
                   "element sizes of every level); largest value of the scan without blow-up over the horizon",
            "error": f"density L1 (domain mean) and nodal max of the final state, and the largest deviation of the "
                     f"kinetic-energy history ({n_int} samples) relative to its initial value, against the "
                     f"{ref['what']}",
            "equal_error": f"target per norm = the smaller error of the pair at the largest stable CFLs; each "
                           f"scheme's step shrunk until all its errors are within {1 + tol:.2f} of the target",
            "adaptation": "flags of the P-ERK run replayed in every run" if amr else "static mesh",
            "pairs": pairs, "not_compared": skipped}


# fp64 flops of the kernels' arithmetic routines, counted from their gfx950 instruction sequences
# in this build (FMA = 2 flops; the hardware estimates v_rcp_f64 / v_rsq_f64 = 1; compares,
# exponent/mantissa extraction and conversions = 0): the reciprocal is 1 estimate + 4 FMA, the
# square root 1 estimate + 2 products + 8 FMA, the logarithm 1 estimate + 16 FMA + 4 sums +
# 3 products (29 fp64 instructions in all).  A division is a reciprocal and a product.
RCP_FLOPS, DIV_FLOPS, SQRT_FLOPS, LOG_FLOPS = 9, 10, 19, 40


def flops_per_element_stage(dim, N, viscous=False):
    """Algorithmic fp64 flops of one element-stage of the stage kernel (FMA = 2), from its code
    path with every reciprocal, division, square root and logarithm weighted by the flops of its
    instruction sequence (RCP_FLOPS ...):
      * per unordered node pair of a line (d N^(d-1) N(N-1)/2 pairs, each flux shared by its two
        nodes) one entropy-conserving flux: two logarithmic means on the series branch (34 and
        32 flops, each with one reciprocal) and 24 + 3d flops of products and sums;
      * per node and direction the flux-differencing sum, 2 n_v (N-1) flops;
      * per node the primitive variables (a reciprocal, 3d + 2 flops), two logarithms and one
        division (rho / p);
      * per face node one HLL flux: two sets of primitives, two sound speeds (a division and a
        square root each, 2 products), the Davis speeds (6), the side fluxes (2 (d + 3)), the
        blend (a reciprocal, 7 n_v + 2);
      * per node the lifting, Jacobian and stage combination, 8 n_v flops.
    Navier-Stokes adds in this kernel the divergence of the viscous flux (2 N d n_v per node)
    and its face terms (4 n_v per face node)."""
    nv = dim + 2
    nd = N ** dim
    nfn = 2 * dim * N ** (dim - 1)                 # face nodes of the element
    prim = RCP_FLOPS + 3 * dim + 2
    ec = (34 + 32) + 24 + 3 * dim
    hll = 2 * prim + 2 * (DIV_FLOPS + SQRT_FLOPS + 2) + 6 + 2 * (dim + 3) + RCP_FLOPS + 7 * nv + 2
    pairs = dim * N ** (dim - 1) * N * (N - 1) // 2
    per_node = dim * (N - 1) * 2 * nv + prim + 2 * LOG_FLOPS + DIV_FLOPS + 8 * nv
    f = pairs * ec + nd * per_node + nfn * hll
    if viscous:
        f += nd * 2 * N * dim * nv + nfn * 4 * nv
    return f


def grad_bytes_per_element(dim, N):
    """Algorithmic HBM bytes of one element of the BR1 gradient pass: read the element's stage
    value (one slice of n_v N^d fp64) and its neighbours' face traces (2d faces of n_v N^(d-1)
    values, times 3/2 for neighbours whose stage value is formed from U_n and K_1), write the
    viscous flux at every node (d slices)."""
    nv = dim + 2
    slice_b = nv * N ** dim * 8
    face_b = 2 * dim * nv * N ** (dim - 1) * 8
    return slice_b + 1.5 * face_b + dim * slice_b


def roofline_of(kernel, ms, launches, bytes_per_launch, flops_per_launch):
    """Roofline entry of one kernel from its event-timed launches: achieved algorithmic GB/s
    (and TFLOP/s when a flop count is given) against the MI355X peaks; the bound is the larger
    fraction."""
    avg_s = ms * 1e-3 / max(1, launches)
    gbs = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    out = {"kernel": kernel, "avg_launch_us": avg_s * 1e6, "launches": launches,
           "bytes_per_launch": bytes_per_launch}
    frac_b = gbs / HBM_PEAK_GBS
    if flops_per_launch is None:
        out.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac_b})
        return out
    tflops = flops_per_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    frac_f = tflops / FP64_PEAK_TFLOPS
    out["flops_per_launch"] = flops_per_launch
    if frac_b >= frac_f:
        out.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac_b})
    else:
        out.update({"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": frac_f})
    out["alt"] = {"hbm_frac": frac_b, "alu_frac": frac_f, "gbs": gbs, "tflops": tflops}
    return out


def optimality(fam, wl, finest_steps, dofs_per_elem, rhs_ms, elem_rhs, wall, n_rhs_actual):
    """N_RHS^Opt, N_RHS+^Hyp and kappa of Sec. 6.4.2-6.4.3.  The hypothetical optimal family gives
    the finest level of the mesh E_R stage evaluations and halves them per coarser level
    (E_R / 2^(finest - l)); N_RHS^Opt counts them over the same steps and meshes as the run
    (finest_steps: per run of steps, the finest level and the element-steps per level).  With a
    CFL below the optimisation's (CFL_Opt = 1: the optimised step), the optimal scheme would take
    proportionally fewer steps: N_RHS+^Hyp = N_RHS^Actual - (CFL_Actual / CFL_Opt) N_RHS^Opt
    (eq. AdditionalRHSEvalsIdealDef_CFLReduction).  kappa = tau_Opt / tau with
    tau_Opt = tau - N_RHS+^Hyp tau_RHS/C (eq. HypotheticalSpeedUp), tau_RHS/C the measured
    average cost of one element right-hand side (event-timed stage and gradient kernels over
    the element-stages they evaluated)."""
    E_R = float(fam.E[-1])
    n_opt_elem = 0.0
    for finest, counts in finest_steps:
        for l, c in enumerate(counts):
            if c:
                n_opt_elem += c * E_R / 2.0 ** (finest - l)
    n_rhs_opt = n_opt_elem * dofs_per_elem
    cfl = float(wl.get("cfl", 1.0))
    n_plus = n_rhs_actual - cfl * n_rhs_opt
    tau_rhs_c = rhs_ms * 1e-3 / max(1, elem_rhs)          # seconds per element right-hand side
    tau_opt = wall - (n_plus / dofs_per_elem) * tau_rhs_c
    return {"n_rhs_opt": n_rhs_opt, "n_rhs_plus_hyp": n_plus, "kappa": tau_opt / wall,
            "cfl_actual": cfl, "cfl_opt": 1.0, "tau_rhs_per_element_s": tau_rhs_c, "tau_opt_s": tau_opt,
            "tau_s": wall}


def _lib_fingerprint():
    from paper_2403_05144_amd import _lib
    return _lib.library_fingerprint()


def bytes_per_element_stage(dim, N, viscous=False):
    """Algorithmic HBM bytes of one element-stage: read the stage value, U_n and K_1 and write
    the next stage value of the element (4 element slices of n_v N^d fp64), plus the neighbours'
    face traces (2d faces of n_v N^(d-1) values, times 3/2 for neighbours whose stage value is
    formed from U_n and K_1); Navier-Stokes also reads the element's BR1 viscous flux, written
    by the gradient kernel (d slices), and its neighbours' normal viscous flux on the faces."""
    nv = dim + 2
    slice_b = nv * N ** dim * 8
    face_b = 2 * dim * nv * N ** (dim - 1) * 8
    b = 4 * slice_b + 1.5 * face_b
    if viscous:
        b += dim * slice_b + face_b
    return b


def measured_traffic(workload, es_per_launch):
    """HBM bytes per stage-kernel launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this workload (each counter scaled by its reading for a plain copy of known
    size), at this run's element-stages per launch.  None when there is no summary or the
    kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_stage_{workload}_hbm_counters.txt")
    if not os.path.exists(path):
        return None, "no counter summary for this workload"
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("TRAFFIC "):
                rec = json.loads(line[len("TRAFFIC "):])
    sha = stage_kernel_digest()
    if rec is None or rec.get("kernel_sha256") != sha:
        return None, f"{os.path.relpath(path, ROOT)} was taken on another kernel source"
    per_es = rec["fetch_bytes_per_element_stage"] + rec["write_bytes_per_element_stage"]
    return per_es * es_per_launch, os.path.relpath(path, ROOT)


def run(args):
    import torch
    from paper_2403_05144_amd import PerkSolver

    from paper_2403_05144_amd.amr import AmrDriver

    wl = WORKLOADS[args.workload]()
    if args.family == "full":
        if "fam_name" not in wl:
            raise SystemExit(f"--family full: workload {args.workload} has no full-mesh family")
        fam_full, _ = full_mesh_family(wl)
        wl = WORKLOADS[args.workload](fam=fam_full)
        wl["family_source"] = "spectrum at the real mesh"
    mesh, deg, fam = wl["mesh"], wl["degree"], wl["fam"]
    leaves_init = np.array(mesh.leaves, copy=True)
    N = deg + 1
    amr = wl.get("amr")
    ic_leaf = lambda x: wl["ic"](x.transpose(1, 0, 2)).transpose(1, 0, 2).copy()
    dt = wl["dt"]
    per_elem = (mesh.dim + 2) * N ** mesh.dim

    def setup():
        """Solver at the start of the measured run: initial mesh (and adaptation passes), IC, warmup."""
        import perk_inputs as pin
        m0 = pin.MeshDesc(mesh.dim, mesh.n_root, mesh.lo, mesh.hi, np.array(leaves_init, copy=True))
        # the library applies the workload's level rule (at the finest level of the current mesh)
        rule = wl.get("rule", wl["mol"])
        s = make_solver(wl, m0, fam, rule)
        drv = None
        if amr:
            drv = AmrDriver(s, amr["level_min"], amr["level_max"], rule, amr["refine_above"],
                            amr["coarsen_below"], amr["interval"])
            drv.initial_mesh(ic_leaf, passes=3)
        else:
            s.set_state(ic_leaf(s.node_coords().cpu().numpy()))
        return s, drv

    # The run is a sequence of episodes, each the workload's simulation from t = 0 to its final
    # time (the paper's t_f where it has one); an episode that ends inside the requested steps is
    # followed by a fresh start from the initial mesh and state, set up outside the timed span.
    episode = max(1, int(round(wl["t_final"] / dt))) if wl.get("t_final") else None

    def new_run():
        s, drv = setup()
        return {"s": s, "drv": drv, "k": 0}

    def run_steps(run, n, acc, profiling=False):
        """n steps; returns the seconds spent restarting episodes (untimed work).  Steps go to the
        library in runs up to the next adaptation or episode end (one call per run of steps)."""
        excluded = 0.0
        done = 0
        while done < n:
            if episode and run["k"] == episode:
                torch.cuda.synchronize()
                tr = time.perf_counter()
                old = run["s"]
                counts = old.counters()
                acc["evals"] += counts[0]
                if profiling:
                    for k in range(3):
                        acc["prof"][k] = [x + y for x, y in zip(acc["prof"][k], old.profile_stats(k))]
                del old
                run.clear()
                run.update(new_run())
                if profiling:
                    run["s"].set_profiling(True)
                acc["episodes"] += 1
                torch.cuda.synchronize()
                excluded += time.perf_counter() - tr
            s, drv = run["s"], run["drv"]
            chunk = n - done
            if drv and drv.interval:
                chunk = min(chunk, drv.interval - run["k"] % drv.interval)
            if episode:
                chunk = min(chunk, episode - run["k"])
            if profiling:
                # elements per level over the steps (for N_RHS^Opt, eq. AdditionalRHSEvalsIdealDef);
                # only in the profiled run, outside the timed one
                lv = s.leaves()[:, 0]
                acc["level_steps"] += chunk * np.bincount(lv, minlength=16)[:16]
                acc["finest_steps"].append((int(lv.max()), chunk * np.bincount(lv, minlength=16)[:16]))
            s.step(dt, chunk)
            run["k"] += chunk
            done += chunk
            acc["dof"] += s.n_elements * per_elem * chunk
            if drv and drv.interval and run["k"] % drv.interval == 0:
                # the adaptation's own time: from the finished steps to the return of the cycle
                # (its device work, uploads and re-partition kernels, then overlaps the next
                # step's launch instead of being waited for here)
                torch.cuda.synchronize()
                ta = time.perf_counter()
                drv.adapt_once()
                acc["amr_s"] += time.perf_counter() - ta
                acc["n_adapt"] += 1
        return excluded

    def fresh_acc():
        return {"dof": 0, "amr_s": 0.0, "n_adapt": 0, "evals": 0, "episodes": 0,
                "prof": [[0.0, 0, 0] for _ in range(3)], "level_steps": np.zeros(16, np.int64),
                "finest_steps": []}

    run0 = new_run()
    s = run0["s"]
    u0 = s.get_state().cpu().numpy()
    leaves0 = s.leaves().copy()
    _log(f"workload {wl['name']}: {s.n_elements} elements, dt={dt:.5g}, family E={fam.E}, members/level "
         f"{wl['mol']}, episode {episode} steps")
    run_steps(run0, args.warmup, fresh_acc())
    torch.cuda.synchronize()
    run0["s"].counters(reset=True)
    # timed region: the production path (one captured step replayed as a HIP graph)
    acc = fresh_acc()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    excluded = run_steps(run0, args.steps, acc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s = run0["s"]
    tot_evals = acc["evals"] + s.counters()[0]
    n_elements_end = s.n_elements
    u_end = s.get_state().cpu().numpy()
    if not np.all(np.isfinite(u_end)):
        raise RuntimeError("non-finite state after the timed steps")
    dof_timed, amr_s, n_adapt_timed = acc["dof"], acc["amr_s"], acc["n_adapt"]
    # profiled region: the same run again from the same start, every stage launch bracketed by
    # HIP events on the launch stream
    del s, run0
    run1 = new_run()
    run_steps(run1, args.warmup, fresh_acc())
    torch.cuda.synchronize()
    run1["s"].set_profiling(True)
    pacc = fresh_acc()
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    p_excluded = run_steps(run1, args.steps, pacc, profiling=True)
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - tp0 - p_excluded
    prof = [[x + y for x, y in zip(pacc["prof"][k], run1["s"].profile_stats(k))] for k in range(3)]
    kern_ms, launches, elem_stages = prof[0]
    grad_ms, grad_launches, grad_elems = prof[1]
    part_ms, n_part, part_elems = prof[2]
    run1["s"].set_profiling(False)
    wall = t1 - t0 - excluded
    nv = mesh.dim + 2
    viscous = wl.get("equations", 0) == 1
    value = dof_timed / wall
    n_rhs_actual = tot_evals * nv * N ** mesh.dim
    pid = wall / n_rhs_actual
    es_per_launch = elem_stages / max(1, launches)
    roof = roofline_of("k_stage", kern_ms, launches, es_per_launch * bytes_per_element_stage(mesh.dim, N, viscous),
                       es_per_launch * flops_per_element_stage(mesh.dim, N, viscous))
    roof["traffic"], roof["traffic_source"] = measured_traffic(wl["name"], es_per_launch)
    roof["element_stages_per_launch"] = es_per_launch
    extra = {}
    if grad_launches:
        ge = grad_elems / grad_launches
        rg = roofline_of("k_grad", grad_ms, grad_launches, ge * grad_bytes_per_element(mesh.dim, N), None)
        rg["elements_per_launch"] = ge
        extra["roofline_k_grad"] = rg
        # the whole stage (gradient pass + stage kernel) over the same element-stages
        rs = roofline_of("stage (k_grad + k_stage)", kern_ms + grad_ms, launches,
                         es_per_launch * bytes_per_element_stage(mesh.dim, N, viscous)
                         + ge * grad_bytes_per_element(mesh.dim, N), None)
        extra["roofline_stage_total"] = rs
    # optimality measures of Sec. 6.4.2-6.4.3 on the profiled run's level histogram (the same
    # steps as the timed run)
    opt = optimality(fam, wl, pacc["finest_steps"], nv * N ** mesh.dim, kern_ms + grad_ms, elem_stages, wall,
                     n_rhs_actual)
    lib_path, lib_sha = _lib_fingerprint()
    line = {
        "metric": "DoF-updates/s & PID; P-ERK vs single-level RK wall time at equal error",
        "value": value, "unit": "DoF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "description": wl["desc"], "elements_start": int(leaves0.shape[0]),
                   "elements_end": int(n_elements_end), "degree": deg, "family_E": list(fam.E), "order": fam.order,
                   "dt": dt, "cfl": wl.get("cfl"), "family_dt_opt": [float(x) for x in fam.dt_opt],
                   "family_h_ref": float(fam.h_ref),
                   "family_spectrum": wl.get("family_source", "spectrum of the reduced mesh"),
                   "member_of_level": [int(m) for m in wl["mol"]],
                   "E_of_level": [int(fam.E[m]) for m in wl["mol"]],
                   "adaptations_timed": n_adapt_timed, "episode_steps": episode,
                   "episode_restarts_timed": acc["episodes"], "restart_s_excluded": excluded,
                   "adaptation": ({k: wl["amr"][k] for k in ("level_min", "level_max", "interval", "refine_above",
                                                              "coarsen_below")}
                                  | {"indicator": (wl["amr"].get("indicator") or ("density_gradient",))[0]})
                   if wl.get("amr") else None,
                   "shock_capturing": (dict(zip(("alpha_max", "alpha_min"), wl["shock_capturing"]))
                                       if wl.get("shock_capturing") else None)},
        "pid_s": pid, "pid_per_node_s": pid * nv, "n_rhs_actual": n_rhs_actual,
        "n_rhs_opt": opt["n_rhs_opt"], "n_rhs_plus_hyp": opt["n_rhs_plus_hyp"], "kappa": opt["kappa"],
        "optimality": opt,
        # shares of the profiled run's wall time (every launch timed, re-partitions serialised)
        "stage_kernel_time_frac": (kern_ms + grad_ms) * 1e-3 / prof_wall,
        "adaptation_share": pacc["amr_s"] / prof_wall,
        "repartition_share": (part_ms * 1e-3 / prof_wall) if n_part else 0.0,
        "adaptation_share_timed_run": amr_s / wall,
        "repartition": {"count": n_part, "ms_each": part_ms / n_part if n_part else None,
                        "elements_each": part_elems / n_part if n_part else None,
                        "how": "pe_amr_cycle's re-partition timed on the host from an idle stream to the end of "
                               "its kernels (profiled run), share of the profiled run's wall time"
                        if n_part else "static mesh: partitioned once before the timed region"},
        "roofline": roof,
        **extra,
        "library": {"path": os.path.relpath(lib_path, ROOT), "sha256": lib_sha},
    }
    if not args.no_equal_error:
        _log("P-ERK against single-level schemes at equal error")
        line["p_erk_vs_single_level"] = compare_equal_error(wl, t_final=wl.get("eq_t_final"))
    if not args.no_cpu_baseline:
        _log("timing the oracle on the host (cpu_baseline)")
        line["cpu_baseline"] = cpu_baseline(wl, u0, leaves0, budget_s=args.cpu_seconds)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--workload", default="tgv", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch-replicas", type=int, default=1, help="batch_vortex64: copies of the 64 runs")
    ap.add_argument("--no-equal-error", action="store_true",
                    help="skip the comparison with single-level schemes at equal error")
    ap.add_argument("--sweep-max", type=int, default=0,
                    help="uniform_sweep: largest element count to run (0: all sizes)")
    ap.add_argument("--arnoldi-steps", type=int, default=200, help="spectrum: Arnoldi steps at the real mesh")
    ap.add_argument("--family", default="reduced", choices=["reduced", "full"],
                    help="tgv, kh_amr: coefficients optimised on the spectrum of the reduced mesh (default) or "
                         "of the real mesh (Sec. 4.1 steps 3-4)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device once (calibration of HBM counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch_vortex64":
        line = run_batch(args)
    elif args.workload == "adjoint_kh":
        line = run_adjoint(args)
    elif args.workload == "spectrum":
        line = run_spectrum(args)
    elif args.workload == "patterns":
        line = run_patterns(args)
    elif args.workload == "uniform_sweep":
        line = run_sweep(args)
    else:
        line = run(args)
    if "library" not in line:
        lib_path, lib_sha = _lib_fingerprint()
        line["library"] = {"path": os.path.relpath(lib_path, ROOT), "sha256": lib_sha}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
