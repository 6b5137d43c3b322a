"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no arithmetic of the method (no quadrature, no fluxes, no time integration):
only mesh descriptions (leaf lists of a Cartesian forest), analytic initial conditions
evaluated at caller-supplied coordinates, and seeded random numbers.

Leaf lists are int32 arrays of shape [n, 4] with rows (level, i, j, k): a leaf at `level`
covers cell (i, j, k) of the uniform grid with n_root[d] * 2**level cells per direction.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 2403051440


@dataclass
class MeshDesc:
    dim: int
    n_root: tuple
    lo: tuple
    hi: tuple
    leaves: np.ndarray                      # int32 [n, 4]
    meta: dict = field(default_factory=dict)

    @property
    def n_elements(self):
        return int(self.leaves.shape[0])


def _rows(triples):
    return np.array(triples, dtype=np.int32).reshape(-1, 4)


def uniform_mesh(dim, n_root, lo, hi, level=0):
    """Every root refined `level` times."""
    n = [n_root[d] << level for d in range(dim)]
    if dim == 2:
        rows = [(level, i, j, 0) for j in range(n[1]) for i in range(n[0])]
    else:
        rows = [(level, i, j, k) for k in range(n[2]) for j in range(n[1]) for i in range(n[0])]
    return MeshDesc(dim, tuple(n_root), tuple(lo), tuple(hi), _rows(rows))


def refine_leaves(leaves, dim, which):
    """Replace every leaf whose row index is in `which` by its 2^dim children."""
    which = set(int(w) for w in which)
    out = []
    for idx, (l, i, j, k) in enumerate(leaves.tolist()):
        if idx in which:
            for c in range(1 << dim):
                ci, cj, ck = 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), (2 * k + ((c >> 2) & 1)) if dim == 3 else 0
                out.append((l + 1, ci, cj, ck))
        else:
            out.append((l, i, j, k))
    return _rows(out)


# ------------------------------------------------------------------------------------------
# Workload meshes
# ------------------------------------------------------------------------------------------
def mesh_vortex_2level(n_root=16, block=(6, 10)):
    """16 x 16 roots on [-5,5]^2; the roots with i, j in [6, 10) refined once:
    240 coarse + 64 fine leaves."""
    m = uniform_mesh(2, (n_root, n_root), (-5.0, -5.0), (5.0, 5.0), 0)
    sel = [r for r, (l, i, j, k) in enumerate(m.leaves.tolist())
           if block[0] <= i < block[1] and block[0] <= j < block[1]]
    m.leaves = refine_leaves(m.leaves, 2, sel)
    return m


def mesh_taylor_green(seed=MASTER_SEED + 2, n_root=16):
    """16^3 roots on [-pi,pi]^3 (level 4 of a single cube).  A box of 6^3 roots at a seeded
    offset is refined once; inside it a box of 3^3 roots at a seeded offset in {1,2}^3 is
    refined a second time (2:1 by construction): 3880 + 1512 + 1728 = 7120 leaves."""
    rng = np.random.default_rng(seed)
    o = rng.integers(0, n_root - 6 + 1, size=3)
    oi = o + rng.integers(1, 3, size=3)
    rows = []
    for k in range(n_root):
        for j in range(n_root):
            for i in range(n_root):
                r = np.array([i, j, k])
                if np.all((r >= oi) & (r < oi + 3)):
                    for c in range(8):
                        ci, cj, ck = 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1)
                        for g in range(8):
                            rows.append((2, 2 * ci + (g & 1), 2 * cj + ((g >> 1) & 1), 2 * ck + ((g >> 2) & 1)))
                elif np.all((r >= o) & (r < o + 6)):
                    for c in range(8):
                        rows.append((1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1)))
                else:
                    rows.append((0, i, j, k))
    return MeshDesc(3, (n_root,) * 3, (-np.pi,) * 3, (np.pi,) * 3, _rows(rows),
                    {"outer_offset": o.tolist(), "inner_offset": oi.tolist()})


def mesh_band_2level(n_root=64, half_width=0.125):
    """n_root^2 roots on [-1,1]^2; roots whose centre has ||y| - 0.5| < half_width refined once."""
    m = uniform_mesh(2, (n_root, n_root), (-1.0, -1.0), (1.0, 1.0), 0)
    h = 2.0 / n_root
    sel = [r for r, (l, i, j, k) in enumerate(m.leaves.tolist())
           if abs(abs(-1.0 + (j + 0.5) * h) - 0.5) < half_width]
    m.leaves = refine_leaves(m.leaves, 2, sel)
    return m


def random_forest_2d(seed, n_root=4, max_level=2, p_refine=0.35):
    """Small random 2:1-balanced quadtree forest on [0,1]^2 (for parity edge cases): random
    refinement, then balance by refining any leaf that has a face neighbour two levels finer."""
    rng = np.random.default_rng(seed)
    leaves = {(0, i, j) for i in range(n_root) for j in range(n_root)}
    for _ in range(max_level):
        new = set()
        for (l, i, j) in leaves:
            if rng.random() < p_refine and l < max_level:
                for c in range(4):
                    new.add((l + 1, 2 * i + (c & 1), 2 * j + (c >> 1)))
            else:
                new.add((l, i, j))
        leaves = new
    leaves = balance_2d(leaves, n_root)
    rows = sorted(leaves)
    return MeshDesc(2, (n_root, n_root), (0.0, 0.0), (1.0, 1.0),
                    _rows([(l, i, j, 0) for (l, i, j) in rows]))


def _covering_leaf(leaves, l, i, j):
    for lev in range(l, -1, -1):
        s = l - lev
        if (lev, i >> s, j >> s) in leaves:
            return lev
    return None


def balance_2d(leaves, n_root):
    """Refine until every pair of face neighbours differs by at most one level (periodic)."""
    leaves = set(leaves)
    changed = True
    while changed:
        changed = False
        for (l, i, j) in sorted(leaves, key=lambda t: -t[0]):
            n = n_root << l
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ni, nj = (i + di) % n, (j + dj) % n
                lev = _covering_leaf(leaves, l, ni, nj)
                if lev is not None and lev < l - 1:
                    s = l - lev
                    ci, cj = ni >> s, nj >> s
                    leaves.discard((lev, ci, cj))
                    for c in range(4):
                        leaves.add((lev + 1, 2 * ci + (c & 1), 2 * cj + (c >> 1)))
                    changed = True
                    break
            if changed:
                break
    return leaves


def balance_2d_fast(leaves, n_root):
    """Same result class as balance_2d (every pair of face neighbours at most one level apart,
    periodic), refining all offending coarse leaves of a pass together."""
    leaves = set(leaves)
    while True:
        marked = set()
        for (l, i, j) in leaves:
            n = n_root << l
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ni, nj = (i + di) % n, (j + dj) % n
                lev = _covering_leaf(leaves, l, ni, nj)
                if lev is not None and lev < l - 1:
                    s = l - lev
                    marked.add((lev, ni >> s, nj >> s))
        if not marked:
            return leaves
        for (lev, ci, cj) in marked:
            leaves.discard((lev, ci, cj))
            for c in range(4):
                leaves.add((lev + 1, 2 * ci + (c & 1), 2 * cj + (c >> 1)))


def mesh_vortex_disks(n_root, n_levels, radii=(3.0, 2.0, 1.0), box=5.0, centre=(0.0, 0.0)):
    """n_root^2 roots on [-box, box]^2; leaves whose centre lies within radii[l] of the vortex
    centre are refined to level l + 1 (nested disks), for l < n_levels; then 2:1 balanced."""
    h0 = 2.0 * box / n_root
    leaves = {(0, i, j) for i in range(n_root) for j in range(n_root)}
    for l in range(n_levels):
        new = set()
        for (lev, i, j) in leaves:
            h = h0 / (1 << lev)
            cx, cy = -box + (i + 0.5) * h, -box + (j + 0.5) * h
            if lev == l and (cx - centre[0]) ** 2 + (cy - centre[1]) ** 2 < radii[l] ** 2:
                for c in range(4):
                    new.add((lev + 1, 2 * i + (c & 1), 2 * j + (c >> 1)))
            else:
                new.add((lev, i, j))
        leaves = balance_2d_fast(new, n_root)
    rows = sorted(leaves, key=lambda t: (t[0], t[2], t[1]))
    return MeshDesc(2, (n_root, n_root), (-box, -box), (box, box), _rows([(l, i, j, 0) for (l, i, j) in rows]))


def batch_vortex_runs(seed=MASTER_SEED + 3, n_runs=64):
    """Independent isentropic-vortex runs of uneven size for the batched form: per run, roots
    per side n ~ U{8..64}, refinement levels L ~ U{1,2,3} (nested disks of radii 3, 2, 1 around
    the vortex centre), vortex strength eps ~ U[1,5], polynomial degree ~ U{2,3} and stage
    family ~ U{{4,8}, {4,8,16}}; Mach 0.5, t in [0, 1]."""
    rng = np.random.default_rng(seed)
    runs = []
    for k in range(n_runs):
        n = int(rng.integers(8, 65))
        L = int(rng.integers(1, 4))
        eps = float(rng.uniform(1.0, 5.0))
        p = int(rng.integers(2, 4))
        fam = (4, 8) if rng.integers(0, 2) == 0 else (4, 8, 16)
        runs.append(dict(n_root=n, levels=L, eps=eps, degree=p, E=fam, mesh=mesh_vortex_disks(n, L)))
    return runs


# ------------------------------------------------------------------------------------------
# Initial conditions at caller-supplied coordinates.  Conservative output with the variable
# axis first: rho, rho v_1..rho v_d, E.
# ------------------------------------------------------------------------------------------
def prim2cons(rho, vel, p, gamma):
    mom = [rho * v for v in vel]
    E = p / (gamma - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + mom + [E])


def isentropic_vortex(x, y, eps=5.0, mach=0.5, gamma=1.4, center=(0.0, 0.0), t=0.0,
                      box=((-5.0, 5.0), (-5.0, 5.0))):
    """Shu's isentropic vortex: rho_inf = p_inf = 1, background velocity (M c_inf, 0),
    c_inf = sqrt(gamma), centred at `center` advected by the background flow to time t
    (periodic images folded into the box)."""
    cinf = np.sqrt(gamma)
    u0 = mach * cinf
    cx = center[0] + u0 * t
    Lx = box[0][1] - box[0][0]
    cx = box[0][0] + np.mod(cx - box[0][0], Lx)
    dx = x - cx
    dx = dx - Lx * np.round(dx / Lx)
    dy = y - center[1]
    r2 = dx * dx + dy * dy
    dv = eps / (2 * np.pi) * np.exp(0.5 * (1.0 - r2))
    vx = u0 - dv * dy
    vy = dv * dx
    dT = -(gamma - 1.0) * eps * eps / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
    rho = (1.0 + dT) ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return prim2cons(rho, [vx, vy], p, gamma)


def kelvin_helmholtz_prim(x, y, seed=MASTER_SEED + 1, amplitude=0.01, width=0.05):
    """Shear layer on [-1,1]^2 in primitive variables (rho, v_x, v_y, p):
    s(y) = (tanh((y+0.5)/w) - tanh((y-0.5)/w))/2, rho = 0.5 + 0.5 s, v_x = -0.5 + s, p = 1,
    v_y = A sin(2 pi (x + phi)) times Gaussians centred on the two layers; phi from the seed."""
    phi = np.random.default_rng(seed).random()
    s = 0.5 * (np.tanh((y + 0.5) / width) - np.tanh((y - 0.5) / width))
    rho = 0.5 + 0.5 * s
    vx = -0.5 + s
    vy = amplitude * np.sin(2 * np.pi * (x + phi)) * (np.exp(-((y - 0.5) / 0.1) ** 2) +
                                                      np.exp(-((y + 0.5) / 0.1) ** 2))
    return rho, vx, vy, np.ones_like(x)


def kelvin_helmholtz(x, y, seed=MASTER_SEED + 1, gamma=1.4, amplitude=0.01, width=0.05):
    """The shear layer of kelvin_helmholtz_prim in conservative variables."""
    rho, vx, vy, p = kelvin_helmholtz_prim(x, y, seed, amplitude, width)
    return prim2cons(rho, [vx, vy], p, gamma)


def kelvin_helmholtz_paper(x, y, gamma=1.4):
    """The Kelvin-Helmholtz instability of the paper's inviscid run (eq. KelvinHelmholtzIC) on
    [-1,1]^2: B(y) = tanh(15 y + 7.5) - tanh(15 y - 7.5), rho = 0.5 + 0.75 B, v_x = (B - 1)/2,
    v_y = 0.1 sin(2 pi x), p = 1; conservative variables."""
    B = np.tanh(15.0 * y + 7.5) - np.tanh(15.0 * y - 7.5)
    rho = 0.5 + 0.75 * B
    vx = 0.5 * (B - 1.0)
    vy = 0.1 * np.sin(2.0 * np.pi * x)
    return prim2cons(rho, [vx, vy], np.ones_like(x), gamma)


def shear_layer(x, y, kappa=80.0, delta=0.05, c0=10.0, gamma=1.4):
    """Doubly periodic double shear layer on [0,1]^2 (paper eq. ShearLayerIC): rho = 1,
    v_x = tanh(kappa (y - 1/4)) for y <= 1/2 and tanh(kappa (3/4 - y)) above, v_y =
    delta sin(2 pi (x + 1/4)), p = c0^2 rho / gamma; conservative variables."""
    rho = np.ones_like(x)
    vx = np.where(y <= 0.5, np.tanh(kappa * (y - 0.25)), np.tanh(kappa * (0.75 - y)))
    vy = delta * np.sin(2.0 * np.pi * (x + 0.25))
    p = c0 * c0 * rho / gamma
    return prim2cons(rho, [vx, vy], p, gamma)


def kh_density_perturbation(x, y, seed=MASTER_SEED + 4, amplitude=1e-3, n_modes=8):
    """Seeded smooth periodic density perturbation on [-1,1]^2 (the control of the
    differentiated workload): amplitude * sum_k a_k sin(pi (kx_k x + ky_k y) + phi_k), a_k in
    [0,1], integer wave numbers |kx|, |ky| <= 4 not both zero, phases in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    m = np.zeros_like(x)
    for _ in range(n_modes):
        a = rng.random()
        kx, ky = 0, 0
        while kx == 0 and ky == 0:
            kx, ky = (int(v) for v in rng.integers(-4, 5, size=2))
        phi = 2 * np.pi * rng.random()
        m = m + a * np.sin(np.pi * (kx * x + ky * y) + phi)
    return amplitude * m


def taylor_green(x, y, z, mach=0.1, gamma=1.4):
    """Taylor-Green vortex (paper eq. IC_TaylorGreen) with p0 = rho / (M^2 gamma)."""
    rho = np.ones_like(x)
    vx = np.sin(x) * np.cos(y) * np.cos(z)
    vy = -np.cos(x) * np.sin(y) * np.cos(z)
    vz = np.zeros_like(x)
    p = rho / (mach ** 2 * gamma) + rho / 16.0 * ((np.cos(2 * x) + np.cos(2 * y)) * (2 + np.cos(2 * z)))
    return prim2cons(rho, [vx, vy, vz], p, gamma)


def smooth_random_state(coords, dim, seed, gamma=1.4, amp=0.1):
    """Seeded smooth positive state: a few random Fourier modes on top of a constant state.
    coords: [dim, ...] physical coordinates (periodic box assumed of period `period`)."""
    rng = np.random.default_rng(seed)
    shape = coords[0].shape
    def field(base, a):
        f = np.full(shape, base, dtype=float)
        for _ in range(4):
            k = rng.integers(1, 3, size=dim)
            ph = rng.random() * 2 * np.pi
            arg = ph + sum(2 * np.pi * k[d] * coords[d] / 10.0 for d in range(dim))
            f = f + a * rng.standard_normal() * np.sin(arg)
        return f
    rho = field(1.0, amp)
    vel = [field(0.3, amp) for _ in range(dim)]
    p = field(1.0, amp)
    return prim2cons(rho, vel, p, gamma)


def supersonic_state(coords, dim, seed, gamma=1.4, mach=(2.0, -2.0, 1.5), amp=0.05):
    """Seeded smooth supersonic stream: rho = p = 1 plus small random Fourier modes, velocity
    mach[d] times the free-stream sound speed in direction d (positive: every face normal to d
    sees flow faster than sound to +e_d; negative: to -e_d)."""
    rng = np.random.default_rng(seed)
    shape = coords[0].shape
    c0 = np.sqrt(gamma)

    def field(base, a):
        f = np.full(shape, base, dtype=float)
        for _ in range(3):
            k = rng.integers(1, 3, size=dim)
            ph = rng.random() * 2 * np.pi
            arg = ph + sum(2 * np.pi * k[d] * coords[d] / 10.0 for d in range(dim))
            f = f + a * rng.standard_normal() * np.sin(arg)
        return f
    rho = field(1.0, amp)
    vel = [field(mach[d] * c0, amp) for d in range(dim)]
    p = field(1.0, amp)
    return prim2cons(rho, vel, p, gamma)
