"""Independent NumPy references used to pin the oracle (test code only).

- deterministic finite-volume solvers (Burgers / Lax-Friedrichs, 1D Euler /
  Rusanov, 2D Euler / Rusanov or Lax-Friedrichs on a Cartesian grid) advancing
  many samples with a shared or a per-sample time step:
  the special cases N = 1 (deterministic FV) and N = Q (coupled collocation);
- the stochastic-Galerkin Burgers flux with triple products (App. A,
  eq:numFluxAnalytic), with its own high-order quadrature;
- the exact Riemann solution of the Sod tube (textbook, not the paper).
"""
import math

import numpy as np

GAMMA = 1.4


# ---------------------------------------------------------------- Burgers
def burgers_flux(u):
    return 0.5 * u * u


def fv_burgers_lf(u, dx, cfl, t_end=None, steps=None, shared_dt=True):
    """u: [cells][S] states of S independent samples, outflow ghosts.
    shared_dt: one dt for all samples (coupled collocation) or one per sample
    (black-box collocation).  Returns (u, steps taken)."""
    u = np.array(u, dtype=np.float64)
    S = u.shape[1]
    t = np.zeros(S)
    k = 0
    while True:
        if steps is not None and k >= steps:
            break
        active = t < t_end if t_end is not None else np.ones(S, dtype=bool)
        if not active.any():
            break
        a = np.abs(u).max(axis=0)
        if shared_dt:
            a = np.full(S, a.max())
        dt = cfl * dx / a
        last = np.zeros(S, dtype=bool)
        if t_end is not None:
            last = t + dt >= t_end
            dt = np.where(last, t_end - t, dt)
            dt = np.where(active, dt, 0.0)
        ug = np.concatenate([u[:1], u, u[-1:]], axis=0)
        visc = np.where(dt > 0, dx / (2 * np.where(dt > 0, dt, 1.0)), 0.0)
        g = 0.5 * (burgers_flux(ug[:-1]) + burgers_flux(ug[1:])) - visc * (ug[1:] - ug[:-1])
        u = u - dt / dx * (g[1:] - g[:-1])
        t = np.where(last & active, t_end if t_end is not None else 0.0, t + dt)
        k += 1
    return u, k


# ---------------------------------------------------------------- Euler 1D
def euler_flux_1d(U):
    rho, m, E = U[..., 0], U[..., 1], U[..., 2]
    v = m / rho
    p = (GAMMA - 1) * (E - 0.5 * rho * v * v)
    f = np.stack([m, m * v + p, (E + p) * v], axis=-1)
    c = np.sqrt(GAMMA * p / rho)
    return f, np.abs(v) + c


def fv_euler_rusanov(U, dx, cfl, t_end=None, steps=None):
    """U: [cells][S][3], shared dt (coupled collocation), outflow ghosts."""
    U = np.array(U, dtype=np.float64)
    t, k = 0.0, 0
    while True:
        if steps is not None and k >= steps:
            break
        if t_end is not None and t >= t_end:
            break
        f, a = euler_flux_1d(U)
        dt = cfl * dx / a.max()
        last = False
        if t_end is not None and t + dt >= t_end:
            dt, last = t_end - t, True
        Ug = np.concatenate([U[:1], U, U[-1:]], axis=0)
        fg, ag = euler_flux_1d(Ug)
        s = np.maximum(ag[:-1], ag[1:])[..., None]
        g = 0.5 * (fg[:-1] + fg[1:]) - 0.5 * s * (Ug[1:] - Ug[:-1])
        U = U - dt / dx * (g[1:] - g[:-1])
        t = t_end if last else t + dt
        k += 1
    return U, k


# ---------------------------------------------------------------- Euler 2D
def euler_flux_2d(U, direction):
    """Physical flux of the 2D Euler equations in x (direction 0) or y (1) and
    the wave speed |v_n| + c in that direction.  U[..., 4] = (rho, m_x, m_y, E)."""
    rho, mx, my, E = U[..., 0], U[..., 1], U[..., 2], U[..., 3]
    vx, vy = mx / rho, my / rho
    p = (GAMMA - 1) * (E - 0.5 * rho * (vx * vx + vy * vy))
    c = np.sqrt(GAMMA * p / rho)
    vn = vx if direction == 0 else vy
    f = np.stack([rho * vn, mx * vn + (p if direction == 0 else 0.0),
                  my * vn + (p if direction == 1 else 0.0), (E + p) * vn], axis=-1)
    return f, np.abs(vn) + c


def _pad_axis(U, axis, lo_periodic, hi_periodic):
    """One ghost layer on each end of `axis`: periodic wrap or outflow copy."""
    n = U.shape[axis]
    lo = np.take(U, [n - 1 if lo_periodic else 0], axis=axis)
    hi = np.take(U, [0 if hi_periodic else n - 1], axis=axis)
    return np.concatenate([lo, U, hi], axis=axis)


def fv_euler2d(U, dx, dy, cfl, bc, flux="rusanov", t_end=None, steps=None):
    """Deterministic 2D Euler finite volumes for S samples sharing one time step
    (coupled collocation); S = 1 is the plain deterministic scheme.

    U: [ny][nx][S][4], cell (iy, ix).  bc: 4 sides (x-, x+, y-, y+), each
    "periodic" or "outflow" (ghost = the boundary cell).  Unsplit update with
    the normal flux on each of the four faces; per face either Rusanov
    (viscosity 0.5 max(|v_n|+c) of the two states) or Lax-Friedrichs
    (viscosity h/(2 dt), h the cell width across the face).  Time step
    dt = cfl / (a_x/dx + a_y/dy) with a_x, a_y the largest |v_x|+c, |v_y|+c
    over all cells and samples, the last step clipped to t_end.
    Returns (U, steps taken)."""
    U = np.array(U, dtype=np.float64)
    per = [b == "periodic" for b in bc]
    t, k = 0.0, 0
    while True:
        if steps is not None and k >= steps:
            break
        if t_end is not None and t >= t_end:
            break
        _, ax = euler_flux_2d(U, 0)
        _, ay = euler_flux_2d(U, 1)
        dt = cfl / (ax.max() / dx + ay.max() / dy)
        if not np.isfinite(dt) or dt <= 0.0:
            raise FloatingPointError("fv_euler2d: non-finite state at step %d" % k)
        last = False
        if t_end is not None and t + dt >= t_end:
            dt, last = t_end - t, True
        # x faces: pad along axis 1 (ix)
        Ux = _pad_axis(U, 1, per[0], per[1])
        fx, sx = euler_flux_2d(Ux, 0)
        if flux == "rusanov":
            vx = 0.5 * np.maximum(sx[:, :-1], sx[:, 1:])[..., None]
        else:
            vx = dx / (2 * dt)
        Gx = 0.5 * (fx[:, :-1] + fx[:, 1:]) - vx * (Ux[:, 1:] - Ux[:, :-1])
        # y faces: pad along axis 0 (iy)
        Uy = _pad_axis(U, 0, per[2], per[3])
        fy, sy = euler_flux_2d(Uy, 1)
        if flux == "rusanov":
            vy = 0.5 * np.maximum(sy[:-1], sy[1:])[..., None]
        else:
            vy = dy / (2 * dt)
        Gy = 0.5 * (fy[:-1] + fy[1:]) - vy * (Uy[1:] - Uy[:-1])
        U = U - dt / dx * (Gx[:, 1:] - Gx[:, :-1]) - dt / dy * (Gy[1:] - Gy[:-1])
        t = t_end if last else t + dt
        k += 1
    return U, k


# ---------------------------------------------------------------- SG Burgers
def triple_products(M, n_quad=64):
    """C[i][n][k] = <phi_n phi_k phi_i> under U(-1,1), orthonormal Legendre."""
    x, w = np.polynomial.legendre.leggauss(n_quad)
    w = w / 2.0
    P = np.stack([math.sqrt(2 * i + 1) * np.polynomial.legendre.legval(x, np.eye(M + 1)[i])
                  for i in range(M + 1)], axis=1)
    return np.einsum("q,qi,qn,qk->ink", w, P, P, P)


def sg_burgers_lf_step(uh, dx, dt, C):
    """Analytic SG Lax-Friedrichs update (App. A, eq:numFluxAnalytic), outflow ghosts.
    uh: [cells][N]."""
    ug = np.concatenate([uh[:1], uh, uh[-1:]], axis=0)
    quad = np.einsum("cn,ink,ck->ci", ug, C, ug)  # u^T C_i u per cell
    G = 0.25 * (quad[:-1] + quad[1:]) - dx / (2 * dt) * (ug[1:] - ug[:-1])
    return uh - dt / dx * (G[1:] - G[:-1])


# ---------------------------------------------------------------- exact Sod
def exact_riemann(x, t, x0, left, right, gamma=GAMMA):
    """Exact solution (rho, u, p) of the 1D Euler Riemann problem at points x."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)

    def fk(p, rk, pk, ck):
        if p > pk:
            A, B = 2 / ((gamma + 1) * rk), (gamma - 1) / (gamma + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B)), math.sqrt(A / (B + p)) * (1 - (p - pk) / (2 * (B + p)))
        r = (p / pk) ** ((gamma - 1) / (2 * gamma))
        return 2 * ck / (gamma - 1) * (r - 1), 1 / (rk * ck) * (p / pk) ** (-(gamma + 1) / (2 * gamma))

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = fk(p, rl, pl, cl)
        f2, d2 = fk(p, rr, pr, cr)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-14 * p:
            break
    f1, _ = fk(p, rl, pl, cl)
    f2, _ = fk(p, rr, pr, cr)
    us = 0.5 * (ul + ur) + 0.5 * (f2 - f1)
    g = gamma
    out = np.zeros((len(x), 3))
    for j, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:  # left of contact
            if p > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
                if s < sl:
                    out[j] = (rl, ul, pl)
                else:
                    rs = rl * ((p / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pl + 1))
                    out[j] = (rs, us, p)
            else:  # left rarefaction
                cs = cl * (p / pl) ** ((g - 1) / (2 * g))
                if s < ul - cl:
                    out[j] = (rl, ul, pl)
                elif s > us - cs:
                    out[j] = (rl * (p / pl) ** (1 / g), us, p)
                else:
                    uu = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    cc = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rr_ = rl * (cc / cl) ** (2 / (g - 1))
                    out[j] = (rr_, uu, pl * (cc / cl) ** (2 * g / (g - 1)))
        else:
            if p > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
                if s > sr:
                    out[j] = (rr, ur, pr)
                else:
                    rs = rr * ((p / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pr + 1))
                    out[j] = (rs, us, p)
            else:
                cs = cr * (p / pr) ** ((g - 1) / (2 * g))
                if s > ur + cr:
                    out[j] = (rr, ur, pr)
                elif s < us + cs:
                    out[j] = (rr * (p / pr) ** (1 / g), us, p)
                else:
                    uu = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    cc = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    out[j] = (rr * (cc / cr) ** (2 / (g - 1)), uu, pr * (cc / cr) ** (2 * g / (g - 1)))
    return out, p, us
