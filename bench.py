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
FP64_PEAK_TFLOPS = 78.6


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------
def family_for(name, order, E_list, reduced_mesh, degree, ic_fn, h_red, equations=0, mu=0.0):
    """Coefficients from the project's own optimisation on the spectrum of a reduced mesh
    (cached as JSON next to the package)."""
    from paper_2403_05144_amd import PerkSolver, coeffs
    path = os.path.join(ROOT, "paper_2403_05144_amd", "data", f"{name}.json")
    if os.path.exists(path):
        return coeffs.Family.load(path)
    _log(f"building coefficient family {name} (spectrum of the reduced mesh, LP optimisation)")
    tmp = coeffs.Family(2, 2, [2], np.array([0.0, 0.5]), np.array([0.0, 1.0]), np.zeros((1, 2)))
    s = PerkSolver(reduced_mesh, degree, tmp, [0] * (int(reduced_mesh.leaves[:, 0].max()) + 1),
                   equations=equations, mu=mu)
    x = s.node_coords().cpu().numpy().transpose(1, 0, 2)
    u = ic_fn(x).transpose(1, 0, 2).copy()
    fam, lam = coeffs.family_from_solver_spectrum(s, u, order, E_list, h_red)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    fam.save(path)
    return fam


def member_of_levels(levels, R):
    """Sec. 6.3.1: finest level -> member R-1, next finer -> R-2, remaining coarse levels -> 0."""
    Lmax = int(np.max(levels))
    return [max(0, (R - 1) - (Lmax - l)) for l in range(Lmax + 1)]


def stable_dt(fam, mesh, mol, cfl):
    """dt = cfl * min over members of dt_opt(E_r) * h_min(r) / h_ref (spectra scale with 1/h)."""
    levels = mesh.leaves[:, 0]
    h = lambda l: (mesh.hi[0] - mesh.lo[0]) / (mesh.n_root[0] << int(l))
    dts = []
    for l in np.unique(levels):
        r = mol[int(l)]
        dts.append(fam.dt_opt[r] * h(l) / fam.h_ref)
    return cfl * min(dts)


def wl_vortex_2level():
    import perk_inputs as pin
    mesh = pin.mesh_vortex_2level()
    red = pin.uniform_mesh(2, (4, 4), (-5, -5), (5, 5), 0)
    ic = lambda x: pin.isentropic_vortex(x[0], x[1])
    fam = family_for("perk2_4_8_vortex_p3", 2, [4, 8], red, 3, ic, 2.5)
    mol = member_of_levels(mesh.leaves[:, 0], len(fam.E))
    return dict(name="vortex_2level", mesh=mesh, degree=3, fam=fam, mol=mol, ic=ic,
                dt=stable_dt(fam, mesh, mol, 0.9), t_final=1.0,
                desc="2D Euler isentropic vortex (M=0.5, eps=5) on [-5,5]^2, 16x16 roots with the "
                     "centred 4x4 block refined once (304 elements, 2 levels), p=3, EC volume + HLL "
                     "surface flux, P-ERK2{4,8}")


def wl_kh_amr(n_root=8, level_max=3, name="kh_amr_l3-6"):
    """Kelvin-Helmholtz shear layer, quadtree AMR between config levels 3 and 6 (forest levels
    0..3 on 8x8 roots), P-ERK3{4,6,8,12,16}, adaptation every 10 steps."""
    import perk_inputs as pin
    from paper_2403_05144_amd import partition_rule
    mesh = pin.uniform_mesh(2, (n_root, n_root), (-1, -1), (1, 1), 0)
    ic = lambda x: pin.kelvin_helmholtz(x[0], x[1])
    h_red = 2.0 / n_root
    fam = family_for(f"perk3_4_6_8_12_16_kh_p3_n{n_root}", 3, [4, 6, 8, 12, 16],
                     pin.uniform_mesh(2, (n_root, n_root), (-1, -1), (1, 1), 0), 3, ic, h_red)
    mol = partition_rule.required_dt_rule(level_max, fam.dt_opt, fam.E)
    h_min = h_red / 2 ** level_max
    dt = 0.5 * fam.dt_opt[-1] * h_min / fam.h_ref
    return dict(name=name, mesh=mesh, degree=3, fam=fam, mol=mol, ic=ic, dt=dt, t_final=3.0,
                amr=dict(level_min=0, level_max=level_max, interval=10, refine_above=0.05, coarsen_below=0.01,
                         capacity=(n_root << level_max) ** 2),
                desc=f"2D Euler Kelvin-Helmholtz shear layer on [-1,1]^2 (rho 0.5/1, v_x +-0.5, tanh width "
                     f"0.05, seeded v_y perturbation 0.01), p=3, EC volume + HLL surface flux, quadtree AMR on "
                     f"a density-gradient indicator between levels {int(np.log2(n_root))} and "
                     f"{int(np.log2(n_root)) + level_max} every 10 steps with re-partition after every "
                     f"adaptation, P-ERK3{{4,6,8,12,16}} at 50% of the optimised step (largest of 0.3/0.5/0.7 without blow-up)")


def wl_tgv():
    """3D compressible Navier-Stokes Taylor-Green vortex, Ma 0.1, Re 1600, Pr 0.72, 16^3 roots
    with a seeded 2-level refined region (7120 elements), p=3, BR1, P-ERK2{4,8,16}."""
    import perk_inputs as pin
    mesh = pin.mesh_taylor_green()
    mu = 1.0 / 1600
    ic = lambda x: pin.taylor_green(x[0], x[1], x[2])
    red = pin.uniform_mesh(3, (2, 2, 2), (-np.pi,) * 3, (np.pi,) * 3, 0)
    fam = family_for("perk2_4_8_16_tgv_p3", 2, [4, 8, 16], red, 3, ic, np.pi, equations=1, mu=mu)
    mol = [0, 1, 2]
    dt = stable_dt(fam, mesh, mol, 0.5)
    return dict(name="tgv_ns_3d", mesh=mesh, degree=3, fam=fam, mol=mol, ic=ic, dt=dt, t_final=None,
                equations=1, mu=mu,
                desc="3D compressible Navier-Stokes Taylor-Green vortex (Ma 0.1, Re 1600, Pr 0.72) on "
                     "[-pi,pi]^3, 16^3 roots with a seeded 2-level refined region (3880+1512+1728 = 7120 "
                     "elements), p=3, EC volume + HLL surface flux, BR1, P-ERK2{4,8,16} at 50% of the "
                     "optimised step (largest of 0.9/0.7/0.5 without blow-up over 200 steps)")


WORKLOADS = {"vortex_2level": wl_vortex_2level, "kh_amr": wl_kh_amr, "tgv": wl_tgv,
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
    return {"value": n * dofs / el, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} P-ERK steps of the same workload ({el:.1f} s, serial C++ oracle, dense "
                      f"masked stages: every stage evaluated on every element)"}


def flops_per_element_stage(dim, N):
    """Algorithmic fp64 operations of one element-stage of the stage kernel, counted from its
    code path (divisions, square roots and logarithms as one operation each):
    per node and direction (N-1) two-point fluxes of 53 (2D) / 63 (3D) operations plus 2 n_v
    accumulations; per face node one HLL flux of 95 (2D) / 115 (3D); per node 16 operations for
    primitives and logarithms and 6 n_v for the stage combination."""
    nv = dim + 2
    nd = N ** dim
    ec = 53 if dim == 2 else 63
    hll = 95 if dim == 2 else 115
    per_node = dim * (N - 1) * (ec + 2 * nv) + 16 + 6 * nv
    return nd * per_node + 2 * dim * N ** (dim - 1) * hll


def bytes_per_element_stage(dim, N):
    """Algorithmic HBM bytes of one element-stage: read the stage value, U_n and K_1 and write
    the next stage value of the element (4 element slices of n_v N^d fp64)."""
    return 4 * (dim + 2) * N ** dim * 8


def run(args):
    import torch
    from paper_2403_05144_amd import PerkSolver

    from paper_2403_05144_amd.amr import AmrDriver

    wl = WORKLOADS[args.workload]()
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
        s = PerkSolver(m0, deg, fam, wl["mol"], capacity=amr["capacity"] if amr else None,
                       equations=wl.get("equations", 0), mu=wl.get("mu", 0.0))
        drv = None
        if amr:
            drv = AmrDriver(s, amr["level_min"], amr["level_max"], wl["mol"], amr["refine_above"],
                            amr["coarsen_below"], amr["interval"])
            drv.initial_mesh(ic_leaf, passes=3)
        else:
            s.set_state(ic_leaf(s.node_coords().cpu().numpy()))
        return s, drv

    def run_steps(s, drv, n, acc):
        for k in range(1, n + 1):
            s.step(dt, 1)
            acc["dof"] += s.n_elements * per_elem
            if drv and drv.interval and k % drv.interval == 0:
                torch.cuda.synchronize()
                ta = time.perf_counter()
                drv.adapt_once()
                torch.cuda.synchronize()
                acc["amr_s"] += time.perf_counter() - ta
                acc["n_adapt"] += 1

    s, drv = setup()
    u0 = s.get_state().cpu().numpy()
    leaves0 = s.leaves().copy()
    _log(f"workload {wl['name']}: {s.n_elements} elements, dt={dt:.5g}, family E={fam.E}, members/level {wl['mol']}")
    warm = {"dof": 0, "amr_s": 0.0, "n_adapt": 0}
    run_steps(s, drv, args.warmup, warm)
    torch.cuda.synchronize()
    s.counters(reset=True)
    # timed region: the production path (one captured step replayed as a HIP graph)
    acc = {"dof": 0, "amr_s": 0.0, "n_adapt": 0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(s, drv, args.steps, acc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tot_evals, per_member = s.counters()
    n_elements_end = s.n_elements
    u_end = s.get_state().cpu().numpy()
    if not np.all(np.isfinite(u_end)):
        raise RuntimeError("non-finite state after the timed steps")
    dof_timed, amr_s, n_adapt_timed = acc["dof"], acc["amr_s"], acc["n_adapt"]
    # profiled region: the same run again from the same start, every stage launch bracketed by
    # HIP events on the launch stream
    del s, drv
    s, drv = setup()
    run_steps(s, drv, args.warmup, dict(warm))
    torch.cuda.synchronize()
    s.set_profiling(True)
    run_steps(s, drv, args.steps, {"dof": 0, "amr_s": 0.0, "n_adapt": 0})
    torch.cuda.synchronize()
    kern_ms, launches, elem_stages = s.profile_stats()
    s.set_profiling(False)
    wall = t1 - t0
    nv = mesh.dim + 2
    value = dof_timed / wall
    n_rhs_actual = tot_evals * nv * N ** mesh.dim
    pid = wall / n_rhs_actual
    avg_launch_s = kern_ms * 1e-3 / max(1, launches)
    es_per_launch = elem_stages / max(1, launches)
    B = bytes_per_element_stage(mesh.dim, N) * es_per_launch
    F = flops_per_element_stage(mesh.dim, N) * es_per_launch
    gbs = B / avg_launch_s / 1e9
    tflops = F / avg_launch_s / 1e12
    frac_b, frac_f = gbs / HBM_PEAK_GBS, tflops / FP64_PEAK_TFLOPS
    if frac_b >= frac_f:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac_b}
    else:
        roof = {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": frac_f}
    roof["traffic"] = None
    roof["kernel"] = "k_stage"
    roof["avg_launch_us"] = avg_launch_s * 1e6
    roof["element_stages_per_launch"] = es_per_launch
    roof["alt"] = {"hbm_frac": frac_b, "alu_frac": frac_f, "gbs": gbs, "tflops": tflops}
    line = {
        "metric": "DoF-updates/s & PID; P-ERK vs single-level RK wall time at equal error",
        "value": value, "unit": "DoF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "description": wl["desc"], "elements_start": int(leaves0.shape[0]),
                   "elements_end": int(n_elements_end), "degree": deg, "family_E": list(fam.E), "order": fam.order,
                   "dt": dt, "member_of_level": [int(m) for m in wl["mol"]],
                   "adaptations_timed": n_adapt_timed},
        "pid_s": pid, "n_rhs_actual": n_rhs_actual,
        "stage_kernel_time_frac": kern_ms * 1e-3 / wall,
        "adaptation_share": amr_s / wall,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        _log("timing the oracle on the host (cpu_baseline)")
        line["cpu_baseline"] = cpu_baseline(wl, u0, leaves0, budget_s=args.cpu_seconds)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="kh_amr", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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
    line = run(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
