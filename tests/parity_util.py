"""Shared comparison rules of the GPU-vs-oracle parity tests (fp64, bar 1e-12).

Right-hand sides: every node's du is a sum of terms of size (2/h) |f| (the flux-divergence
scale sigma_v of variable v), so for variable v
    ||du_gpu - du_ora||_inf <= 1e-12 * max(||du_ora_v||_inf, sigma_v).
States after n steps of size dt: U_{n} = U_0 + dt * (sum of stage RHS), so the absolute
rounding floor grows like n * dt * sigma_v; for variable v
    ||U_gpu - U_ora||_inf <= 1e-12 * max(||U_ora_v||_inf, n * dt * sigma_v),
which is the plain relative bar except for components that pass through zero (e.g. the z
momentum of the Taylor-Green vortex)."""
import numpy as np

TOL = 1e-12
GAMMA = 1.4


def flux_scale(o, u, gamma=GAMMA):
    dim = o.dim
    rho = u[:, 0]
    vel = u[:, 1:1 + dim] / rho[:, None]
    p = (gamma - 1) * (u[:, -1] - 0.5 * rho * np.sum(vel * vel, axis=1))
    jmax = np.max(2.0 / o.element_sizes(), axis=1)[:, None]
    out = np.zeros(dim + 2)
    for d in range(dim):
        comps = [u[:, 1 + d]] + [u[:, 1 + k] * vel[:, d] + (p if k == d else 0) for k in range(dim)] + \
                [(u[:, -1] + p) * vel[:, d]]
        out = np.maximum(out, [np.max(jmax * np.abs(c)) for c in comps])
    return out


def rel_err(a, b):
    return max(np.max(np.abs(a[:, v] - b[:, v])) / max(np.max(np.abs(b[:, v])), 1e-300) for v in range(b.shape[1]))


def rhs_close(du_gpu, du_ora, sigma, tol=TOL):
    return all(np.max(np.abs(du_gpu[:, v] - du_ora[:, v])) <= tol * max(np.max(np.abs(du_ora[:, v])), sigma[v])
               for v in range(du_ora.shape[1]))


def state_close(u_gpu, u_ora, sigma, n_steps, dt, tol=TOL):
    return all(np.max(np.abs(u_gpu[:, v] - u_ora[:, v])) <=
               tol * max(np.max(np.abs(u_ora[:, v])), n_steps * dt * sigma[v]) for v in range(u_ora.shape[1]))


def worst(u_gpu, u_ora, sigma, n_steps, dt):
    """Largest ratio error / allowed scale (for messages)."""
    return max(np.max(np.abs(u_gpu[:, v] - u_ora[:, v])) / max(np.max(np.abs(u_ora[:, v])), n_steps * dt * sigma[v])
               for v in range(u_ora.shape[1]))
