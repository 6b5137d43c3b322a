"""Oracle: adaptive refinement of the forest and projection of the DGSEM state.

Test infrastructure only (see oracle/__init__.py).  Plain Python loops over leaves.

The paper refines and coarsens its quad/octree meshes with an indicator every N_AMR steps and
re-flags the elements after every mesh change (Sec. 6.2, Sec. 7); it does not spell out the
indicator of the adaptive Kelvin-Helmholtz workload, the balance rules or the projection.  The
readings implemented here:
  * indicator eta_e = h_e max_nodes |grad rho| / max_nodes rho, grad rho from the LGL derivative
    matrix, h_e the element size in x; or Loehner's indicator on a primitive variable (the
    shear-layer workload, Sec. 7.1.1), the largest normalised second difference of three
    consecutive nodal values along the element's coordinate lines;
  * flags: +1 if eta > refine threshold, -1 if eta < coarsen threshold, else 0;
  * adaptation: flagged leaves below level_max are refined once; then every pair of face
    neighbours whose target levels differ by two or more has the coarser one refined, until no
    such pair is left; a complete family of 2^dim sibling leaves is coarsened when all are
    flagged -1, none is refined, their level exceeds level_min, and no face neighbour outside
    the family has a target level above the family's level;
  * projection: children take the parent polynomial interpolated at their nodes; a parent takes
    the L2 projection of its children with the LGL quadrature (conservative);
  * new leaves are listed in Morton order.
"""
from __future__ import annotations

import numpy as np

from .dgsem import Oracle, lgl


def indicator(o: Oracle, u):
    N, dim = o.N, o.dim
    _, _, D = lgl(N)
    rho = u[:, 0].reshape((o.n_elements,) + (N,) * dim)      # [e, (k,) j, i]
    h = o.element_sizes()
    eta = np.zeros(o.n_elements)
    for e in range(o.n_elements):
        r = rho[e]
        g2 = np.zeros_like(r)
        for d in range(dim):
            axis = dim - 1 - d                                  # node index i is the last axis
            deriv = np.apply_along_axis(lambda line: D @ line, axis, r)
            g2 = g2 + (2.0 / h[e, d] * deriv) ** 2
        eta[e] = h[e, 0] * np.sqrt(g2).max() / r.max()
    return eta


def primitive_variable(u, var, dim, gamma=1.4):
    """Node values of one primitive variable of a state [e, var, node]: 0 rho, 1..dim the velocity
    components, dim+1 the pressure."""
    rho = u[:, 0]
    if var == 0:
        return rho
    if 1 <= var <= dim:
        return u[:, var] / rho
    ke = 0.5 * sum(u[:, 1 + k] ** 2 for k in range(dim)) / rho
    return (gamma - 1.0) * (u[:, dim + 1] - ke)


def lohner_estimate(um, u0, up, f_wave):
    """Loehner's normalised second difference of three consecutive values (Sec. 7.1.1 cites
    Loehner 1987 and the FLASH form): |up - 2 u0 + um| over |up - u0| + |u0 - um|
    + f_wave (|up| + 2 |u0| + |um|); 0 where the denominator vanishes."""
    num = abs(up - 2.0 * u0 + um)
    den = abs(up - u0) + abs(u0 - um) + f_wave * (abs(up) + 2.0 * abs(u0) + abs(um))
    return num / den if den > 0.0 else 0.0


def lohner_indicator(o: Oracle, u, var=1, f_wave=0.2, gamma=1.4):
    """Element indicator: the largest estimate over every interior node of every coordinate line
    of the element's LGL nodes (three consecutive nodal values, as they are; the reading of the
    indicator's adaptation to LGL elements), for the primitive variable `var`."""
    N, dim = o.N, o.dim
    q = primitive_variable(np.asarray(u, float), var, dim, gamma)
    eta = np.zeros(o.n_elements)
    for e in range(o.n_elements):
        v = q[e].reshape((N,) * dim)                         # [(k,) j, i], i fastest
        best = 0.0
        for d in range(dim):
            axis = dim - 1 - d
            lines = np.moveaxis(v, axis, -1).reshape(-1, N)
            for line in lines:
                for i in range(1, N - 1):
                    best = max(best, lohner_estimate(line[i - 1], line[i], line[i + 1], f_wave))
        eta[e] = best
    return eta


def flags_from_indicator(eta, refine_above, coarsen_below):
    f = np.zeros(len(eta), np.int8)
    f[eta > refine_above] = 1
    f[eta < coarsen_below] = -1
    return f


def _key(l, c):
    return (int(l),) + tuple(int(x) for x in c)


def _morton(l, c, dim, top=15):
    sh = top - l
    x = [int(v) << sh for v in c]
    key = 0
    for b in range(21):
        for d in range(dim):
            key |= ((x[d] >> b) & 1) << (dim * b + d)
    return key


def face_neighbours(leaves, dim, n_root):
    """Face-neighbour leaf indices of every leaf (periodic), found by cell lookup."""
    index = {_key(r[0], r[1:1 + dim]): i for i, r in enumerate(leaves)}
    out = []
    for r in leaves:
        l, c = int(r[0]), [int(v) for v in r[1:1 + dim]]
        nb = set()
        for d in range(dim):
            for s in (-1, 1):
                n = n_root[d] << l
                cc = list(c)
                cc[d] = (cc[d] + s) % n
                if _key(l, cc) in index:
                    nb.add(index[_key(l, cc)])
                    continue
                par = [v >> 1 for v in cc]
                if l > 0 and _key(l - 1, par) in index:
                    nb.add(index[_key(l - 1, par)])
                    continue
                # finer neighbours: children of cc touching the shared face
                for m in range(1 << dim):
                    ch = [2 * v + ((m >> q) & 1) for q, v in enumerate(cc)]
                    if ((m >> d) & 1) != (0 if s > 0 else 1):
                        continue
                    k = _key(l + 1, ch)
                    if k in index:
                        nb.add(index[k])
        out.append(sorted(nb))
    return out


def adapt(leaves, flags, level_min, level_max, dim, n_root):
    """New leaf list (Morton order) and a plan per new leaf: ('copy', old), ('child', old, pos)
    or ('parent', [old children by position])."""
    leaves = [tuple(int(v) for v in r[:1 + dim]) for r in np.asarray(leaves)]
    n = len(leaves)
    lev = np.array([r[0] for r in leaves])
    t = lev + ((np.asarray(flags) > 0) & (lev < level_max)).astype(int)
    nbrs = face_neighbours(np.array(leaves), dim, n_root)
    changed = True
    while changed:
        changed = False
        for e in range(n):
            for g in nbrs[e]:
                if t[e] - t[g] >= 2:
                    t[g] = lev[g] + 1
                    changed = True
    families = {}
    for e in range(n):
        if lev[e] > level_min and flags[e] < 0 and t[e] == lev[e]:
            l, c = leaves[e][0], leaves[e][1:]
            families.setdefault((l - 1,) + tuple(v >> 1 for v in c), []).append(e)
    coarsened = {}
    for pkey, mem in families.items():
        if len(mem) != (1 << dim):
            continue
        ok = all(t[g] <= lev[e] for e in mem for g in nbrs[e] if g not in mem)
        if ok:
            for e in mem:
                coarsened[e] = pkey
    new = []
    done = set()
    for e in range(n):
        l, c = leaves[e][0], leaves[e][1:]
        if e in coarsened:
            pkey = coarsened[e]
            if pkey in done:
                continue
            done.add(pkey)
            kids = [None] * (1 << dim)
            for g, pk in coarsened.items():
                if pk == pkey:
                    pos = sum((leaves[g][1 + q] & 1) << q for q in range(dim))
                    kids[pos] = g
            new.append((pkey, ("parent", kids)))
        elif t[e] == l + 1:
            for m in range(1 << dim):
                ch = tuple(2 * v + ((m >> q) & 1) for q, v in enumerate(c))
                new.append(((l + 1,) + ch, ("child", e, m)))
        else:
            new.append((leaves[e], ("copy", e)))
    new.sort(key=lambda x: _morton(x[0][0], x[0][1:], dim))
    out = np.zeros((len(new), 4), np.int32)
    for i, (k, _) in enumerate(new):
        out[i, :1 + dim] = k
    return out, [p for _, p in new]


def project(o_old: Oracle, u_old, plan, N):
    """Apply a plan: interpolation to children, LGL L2 projection to parents."""
    P, R = o_old.mortar_ops()
    dim = o_old.dim
    nv = u_old.shape[1]
    out = np.zeros((len(plan), nv, N ** dim))

    def tensor(mats, f):
        g = f.reshape((nv,) + (N,) * dim)            # axes: v, (k,) j, i
        for d in range(dim):
            ax = 1 + (dim - 1 - d)
            g = np.moveaxis(np.tensordot(mats[d], g, axes=([1], [ax])), 0, ax)
        return g.reshape(nv, -1)

    for i, p in enumerate(plan):
        if p[0] == "copy":
            out[i] = u_old[p[1]]
        elif p[0] == "child":
            pos = p[2]
            out[i] = tensor([P[(pos >> d) & 1] for d in range(dim)], u_old[p[1]])
        else:
            acc = np.zeros((nv, N ** dim))
            for pos, g in enumerate(p[1]):
                acc += tensor([R[(pos >> d) & 1] for d in range(dim)], u_old[g])
            out[i] = acc
    return out
