"""Seeded synthetic initial data for the compact gas-kinetic scheme.

This module holds no arithmetic of the scheme itself: it only turns a
problem description (primitive fields, domain, mesh) into the scheme's input,
the cell averages W of the conservative variables and the cell-averaged
gradients W_x (and W_y), both exact up to quadrature (Sec. 4: the accuracy
test advects exact cell averages; the acoustic test uses exact averages of
values and of derivatives).  Both the HIP library's tests and the CPU oracle
consume what it produces.

Arrays are float64, conservative order (rho, rho U, [rho V], rho E), layout
[nx, nv] in 1-D and [ny, nx, nv] in 2-D.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# 8-point Gauss-Legendre rule on [-1, 1]
_GL_X, _GL_W = np.polynomial.legendre.leggauss(8)


def prim_to_cons(rho, U, p, gamma, V=None):
    """Conservative variables from primitive (pointwise)."""
    rho = np.asarray(rho, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64) * np.ones_like(rho)
    p = np.asarray(p, dtype=np.float64) * np.ones_like(rho)
    if V is None:
        E = p / (gamma - 1.0) + 0.5 * rho * U * U
        return np.stack([rho, rho * U, E], axis=-1)
    V = np.asarray(V, dtype=np.float64) * np.ones_like(rho)
    E = p / (gamma - 1.0) + 0.5 * rho * (U * U + V * V)
    return np.stack([rho, rho * U, rho * V, E], axis=-1)


@dataclass
class Problem:
    """A problem description consumed by the library binding and the oracle."""
    dim: int
    nx: int
    ny: int
    xlo: float
    xhi: float
    ylo: float
    yhi: float
    gamma: float
    mu: float
    cfl: float
    dt_fixed: float
    t_end: float
    order: int
    recon: int  # 0 linear, 1 WENO-Z
    bc: tuple   # (xlo, xhi, ylo, yhi): 0 periodic, 1 extrapolated, 2 reflecting wall
    W: np.ndarray = field(repr=False)
    Wx: np.ndarray = field(repr=False)
    Wy: np.ndarray | None = field(repr=False, default=None)
    name: str = ""
    # boundary data of inflow (3) and split (4) sides: states [side][A/B][4
    # conservative slots], switch position and speed [side][2], kind beyond
    # the switch [side] (3 inflow of state B, 2 reflecting wall)
    bc_state: np.ndarray = field(repr=False, default_factory=lambda: np.zeros((4, 2, 4)))
    bc_split: np.ndarray = field(repr=False, default_factory=lambda: np.zeros((4, 2)))
    bc_beyond: tuple = (2, 2, 2, 2)

    def oracle_kwargs(self):
        return dict(xlo=self.xlo, xhi=self.xhi, ylo=self.ylo, yhi=self.yhi, gamma=self.gamma,
                    mu=self.mu, cfl=self.cfl, dt_fixed=self.dt_fixed, t_end=self.t_end,
                    order=self.order, recon=self.recon, bc=tuple(self.bc),
                    bc_state=np.asarray(self.bc_state, dtype=np.float64).ravel(),
                    bc_split=np.asarray(self.bc_split, dtype=np.float64).ravel(), bc_beyond=tuple(self.bc_beyond))


# ---------------------------------------------------------------- 1-D
def sine_wave_1d(n, *, order=6, recon=0, gamma=1.4, cfl=0.3, dt_fixed=0.0, t_end=2.0, amp=0.2, k=math.pi):
    """rho = 1 + amp sin(k x), U = 1, p = 1 on [0, 2], periodic (Sec. 4.1).
    Exact cell averages and cell-averaged slopes (the conservative variables
    are affine in rho here, so both are closed forms)."""
    xlo, xhi = 0.0, 2.0
    dx = (xhi - xlo) / n
    xf = xlo + dx * np.arange(n + 1)
    # point values at faces and exact cell averages of rho
    rho_f = 1.0 + amp * np.sin(k * xf)
    rho_avg = 1.0 + amp * (np.cos(k * xf[:-1]) - np.cos(k * xf[1:])) / (k * dx)
    W = prim_to_cons(rho_avg, 1.0, 1.0, gamma)          # affine in rho: exact averages
    Wf = prim_to_cons(rho_f, 1.0, 1.0, gamma)
    Wx = (Wf[1:] - Wf[:-1]) / dx
    return Problem(1, n, 1, xlo, xhi, 0.0, 1.0, gamma, 0.0, cfl, dt_fixed, t_end, order, recon,
                   (0, 0, 0, 0), W, Wx, None, name=f"sine1d_n{n}")


def accuracy_dt(n, order, C=0.3, L=2.0):
    """Accuracy-sweep step dt = C dx^(r/4) on n cells of [0, L] (Sec. 4.1); the
    last step is shortened to end at t_end."""
    return C * (L / n) ** (order / 4.0)


def riemann_1d(n, left, right, *, x0=0.5, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=0.14, xlo=0.0, xhi=1.0):
    """Piecewise-constant Riemann data (rho, U, p) with the jump on the face
    nearest x0; zero slopes; extrapolated boundaries."""
    dx = (xhi - xlo) / n
    jface = int(round((x0 - xlo) / dx))
    rho = np.where(np.arange(n) < jface, left[0], right[0])
    U = np.where(np.arange(n) < jface, left[1], right[1])
    p = np.where(np.arange(n) < jface, left[2], right[2])
    W = prim_to_cons(rho, U, p, gamma)
    Wx = np.zeros_like(W)
    return Problem(1, n, 1, xlo, xhi, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (1, 1, 0, 0), W, Wx, None, name="riemann1d")


def blast_wave_1d(n=200, *, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=3.8):
    """Woodward-Colella blast wave (Sec. 4.2): (rho, U, p) = (1, 0, 1000)
    for x < 10, (1, 0, 0.01) for 10 <= x < 90, (1, 0, 100) beyond, on
    [0, 100] between reflecting walls.  With n a multiple of 10 both jumps
    sit on faces; zero slopes."""
    x = (np.arange(n) + 0.5) * 100.0 / n
    p = np.where(x < 10.0, 1000.0, np.where(x < 90.0, 0.01, 100.0))
    W = prim_to_cons(np.ones(n), 0.0, p, gamma)
    return Problem(1, n, 1, 0.0, 100.0, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (2, 2, 0, 0), W, np.zeros_like(W), None, name=f"blast_n{n}")


def acoustic_pulse_1d(n=100, *, bc=(5, 5, 0, 0), order=8, recon=1, gamma=1.4, cfl=0.3, t_end=0.6, amp=1e-3):
    """A right-running acoustic pulse (simple wave to first order: rho' =
    amp exp(-((x - 0.5)/0.06)^2), U' = c rho', p' = c^2 rho' on rho = 1,
    U = 0, p = 1/gamma, c = 1) on [0, 1]; by t = 0.6 it has left through
    x = 1, so what remains measures the reflection of the right boundary.
    Exact cell averages and cell-averaged gradients."""
    c = 1.0

    def fn(x):
        r = amp * np.exp(-(((x - 0.5) / 0.06) ** 2))
        return prim_to_cons(1.0 + r, c * r, 1.0 / gamma + c * c * r, gamma)

    W, Wx = _cell_quadrature_1d(fn, n, 0.0, 1.0)
    return Problem(1, n, 1, 0.0, 1.0, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   tuple(bc), W, Wx, None, name=f"pulse1d_n{n}")


def _cell_quadrature_1d(fn, n, xlo, xhi):
    """Cell averages of fn(x) -> [..., nv] (8-point Gauss-Legendre per cell)
    and the exact cell-averaged gradient (fn at the faces over dx)."""
    dx = (xhi - xlo) / n
    xc = xlo + dx * (np.arange(n) + 0.5)
    pts = xc[:, None] + 0.5 * dx * _GL_X[None, :]
    avg = np.einsum("q,nqk->nk", 0.5 * _GL_W, fn(pts))
    xf = xlo + dx * np.arange(n + 1)
    Wf = fn(xf)
    return avg, (Wf[1:] - Wf[:-1]) / dx


def shu_osher_1d(n=200, *, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=1.8):
    """Shock / density-wave interaction (Sec. 4.2): (rho, U, p) =
    (3.857134, 2.629369, 10.33333) for x <= 1 and (1 + 0.2 sin 5x, 0, 1)
    beyond, on [0, 10]; non-reflecting (extrapolated) ends.  With n a
    multiple of 10 the shock sits on a face."""
    xlo, xhi = 0.0, 10.0
    left = (3.857134, 2.629369, 10.33333)

    def fn(x):
        post = x <= 1.0
        rho = np.where(post, left[0], 1.0 + 0.2 * np.sin(5.0 * x))
        U = np.where(post, left[1], 0.0)
        p = np.where(post, left[2], 1.0)
        return prim_to_cons(rho, U, p, gamma)

    W, Wx = _cell_quadrature_1d(fn, n, xlo, xhi)
    dx = (xhi - xlo) / n
    jshock = int(round((1.0 - xlo) / dx))
    Wx[:jshock] = 0.0  # constant post-shock state
    # the face values at the shock face mix the two sides: the first
    # pre-shock cell's gradient comes from its own (smooth) side only
    xa, xb = xlo + jshock * dx, xlo + (jshock + 1) * dx
    Wa = prim_to_cons(1.0 + 0.2 * np.sin(5.0 * xa), 0.0, 1.0, gamma)
    Wb = prim_to_cons(1.0 + 0.2 * np.sin(5.0 * xb), 0.0, 1.0, gamma)
    Wx[jshock] = (Wb - Wa) / dx
    return Problem(1, n, 1, xlo, xhi, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (1, 1, 0, 0), W, Wx, None, name=f"shu_osher_n{n}")


def titarev_toro_1d(n=1000, *, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=5.0):
    """Shock / high-frequency entropy-wave interaction (Sec. 4.2, after
    Titarev and Toro): (rho, U, p) = (1.515695, 0.523346, 1.805) for
    x <= -4.5 and (1 + 0.1 sin 20 pi x, 0, 1) beyond, on [-5, 5]; a
    characteristic non-reflecting left end and, on the right (where the gas
    stays at rest until t = 5), the extrapolated profile.  With n a multiple
    of 20 the shock sits on a face."""
    xlo, xhi = -5.0, 5.0
    left = (1.515695, 0.523346, 1.805)

    def fn(x):
        post = x <= -4.5
        rho = np.where(post, left[0], 1.0 + 0.1 * np.sin(20.0 * math.pi * x))
        U = np.where(post, left[1], 0.0)
        p = np.where(post, left[2], 1.0)
        return prim_to_cons(rho, U, p, gamma)

    W, Wx = _cell_quadrature_1d(fn, n, xlo, xhi)
    dx = (xhi - xlo) / n
    jshock = int(round((-4.5 - xlo) / dx))
    Wx[:jshock] = 0.0  # constant post-shock state
    # the first pre-shock cell's gradient from its own (smooth) side only
    xa, xb = xlo + jshock * dx, xlo + (jshock + 1) * dx
    Wa = prim_to_cons(1.0 + 0.1 * np.sin(20.0 * math.pi * xa), 0.0, 1.0, gamma)
    Wb = prim_to_cons(1.0 + 0.1 * np.sin(20.0 * math.pi * xb), 0.0, 1.0, gamma)
    Wx[jshock] = (Wb - Wa) / dx
    return Problem(1, n, 1, xlo, xhi, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (5, 1, 0, 0), W, Wx, None, name=f"titarev_toro_n{n}")


def shock_velocity_wave_1d(n=400, *, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=0.8):
    """Mach-10 shock crossing a velocity perturbation (Sec. 4.4): (rho, U,
    p) = (8, 8.25, 116.5) for x <= 1 and (1.4, 0.2 sin 2 pi (x - 1), 1)
    beyond, on [0, 10]; characteristic non-reflecting ends.  With n a
    multiple of 10 the shock sits on a face."""
    xlo, xhi = 0.0, 10.0
    left = (8.0, 8.25, 116.5)

    def fn(x):
        post = x <= 1.0
        rho = np.where(post, left[0], 1.4)
        U = np.where(post, left[1], 0.2 * np.sin(2.0 * math.pi * (x - 1.0)))
        p = np.where(post, left[2], 1.0)
        return prim_to_cons(rho, U, p, gamma)

    W, Wx = _cell_quadrature_1d(fn, n, xlo, xhi)
    dx = (xhi - xlo) / n
    jshock = int(round((1.0 - xlo) / dx))
    Wx[:jshock] = 0.0  # constant post-shock state
    # the first pre-shock cell's gradient from its own (smooth) side only
    xa, xb = xlo + jshock * dx, xlo + (jshock + 1) * dx
    Wa = prim_to_cons(1.4, 0.2 * np.sin(2.0 * math.pi * (xa - 1.0)), 1.0, gamma)
    Wb = prim_to_cons(1.4, 0.2 * np.sin(2.0 * math.pi * (xb - 1.0)), 1.0, gamma)
    Wx[jshock] = (Wb - Wa) / dx
    return Problem(1, n, 1, xlo, xhi, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (5, 5, 0, 0), W, Wx, None, name=f"shock_velocity_wave_n{n}")


ACOUSTIC = dict(eps=1e-5, omega=6.0 * math.pi, rho_inf=1.1771, p_inf=101325.0)


def acoustic_1d(n, *, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=0.01, eps=ACOUSTIC["eps"],
                omega=ACOUSTIC["omega"], rho_inf=ACOUSTIC["rho_inf"], p_inf=ACOUSTIC["p_inf"]):
    """Linear acoustic wave (Sec. 4.3, after Bai et al.): U = eps a cos(w x),
    rho = rho_inf (1 + eps cos 2 w x), p = p_inf (rho/rho_inf)^gamma on
    [0, 1/3], periodic; exact cell averages of the conservative variables and
    of their gradients."""
    a = math.sqrt(gamma * p_inf / rho_inf)

    def fn(x):
        rho = rho_inf * (1.0 + eps * np.cos(2.0 * omega * x))
        return prim_to_cons(rho, eps * a * np.cos(omega * x), p_inf * (rho / rho_inf) ** gamma, gamma)

    W, Wx = _cell_quadrature_1d(fn, n, 0.0, 1.0 / 3.0)
    return Problem(1, n, 1, 0.0, 1.0 / 3.0, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (0, 0, 0, 0), W, Wx, None, name=f"acoustic1d_n{n}")


def acoustic_linear_rho(x, t, *, gamma=1.4, eps=ACOUSTIC["eps"], omega=ACOUSTIC["omega"],
                        rho_inf=ACOUSTIC["rho_inf"], p_inf=ACOUSTIC["p_inf"]):
    """The linear-acoustics solution for the density of acoustic_1d (two
    counter-propagating pairs of waves); exact for the linearised equations."""
    a = math.sqrt(gamma * p_inf / rho_inf)
    xm, xp = x - a * t, x + a * t
    return rho_inf + 0.5 * eps * rho_inf * (np.cos(2 * omega * xm) + np.cos(2 * omega * xp)
                                            + np.cos(omega * xm) - np.cos(omega * xp))


def random_riemann_states(seed):
    """(rho_L, u_L, p_L), (rho_R, u_R, p_R): rho ~ U[0.1, 1], u ~ U[-1, 1],
    p ~ U[0.1, 1], drawn in that order from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    rl, ul, pl, rr, ur, pr = (rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0),
                              rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
    return (rl, ul, pl), (rr, ur, pr)


SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))


def riemann_set_1d(count=32, n=400, base_seed=20190101, order=8, recon=1):
    return [riemann_1d(n, *random_riemann_states(base_seed + k), order=order, recon=recon)
            for k in range(count)]


def batch_1d(count=256, seed=4, nmin=200, nmax=4000, t_end=0.14):
    """Uneven batch: N ~ integer U[nmin, nmax], order 6 or 8 with p = 1/2,
    states as random_riemann_states, jump on the face nearest 0.5."""
    rng = np.random.default_rng(seed)
    probs = []
    for k in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        order = 6 if rng.uniform() < 0.5 else 8
        l, r = random_riemann_states(int(rng.integers(0, 2**31 - 1)))
        probs.append(riemann_1d(n, l, r, order=order, recon=1, t_end=t_end))
    return probs


# ---------------------------------------------------------------- 2-D
def _cell_quadrature_2d(fn, nx, ny, xlo, xhi, ylo, yhi, chunk=128):
    """Cell averages of fn(X, Y) -> [..., nv] and the cell-averaged x/y
    derivatives through face line averages (8-point Gauss-Legendre per cell
    and per face).  fn receives broadcastable coordinate arrays."""
    dx = (xhi - xlo) / nx
    dy = (yhi - ylo) / ny
    xc = xlo + dx * (np.arange(nx) + 0.5)
    yc = ylo + dy * (np.arange(ny) + 0.5)
    gx = 0.5 * dx * _GL_X
    gy = 0.5 * dy * _GL_X
    w = 0.5 * _GL_W
    xf = xlo + dx * np.arange(nx + 1)
    yf = ylo + dy * np.arange(ny + 1)
    avg = np.empty((ny, nx, 0))
    parts_a, parts_l = [], []
    for j0 in range(0, ny, chunk):
        j1 = min(ny, j0 + chunk)
        X = (xc[:, None] + gx[None, :])[None, :, None, :]          # [1, nx, 1, 8]
        Y = (yc[j0:j1, None] + gy[None, :])[:, None, :, None]       # [nj, 1, 8, 1]
        parts_a.append(np.einsum("abijv,i,j->abv", fn(X, Y), w, w))
        Xf = xf[None, :, None]                                       # [1, nx+1, 1]
        Yf = (yc[j0:j1, None] + gy[None, :])[:, None, :]             # [nj, 1, 8]
        parts_l.append(np.einsum("abiv,i->abv", fn(Xf, Yf), w))
    avg = np.concatenate(parts_a, axis=0)
    lx = np.concatenate(parts_l, axis=0)                             # [ny, nx+1, nv]
    Xg = (xc[:, None] + gx[None, :])[None, :, :]                     # [1, nx, 8]
    Yg = yf[:, None, None]                                           # [ny+1, 1, 1]
    ly = np.einsum("abiv,i->abv", fn(Xg, Yg), w)                     # [ny+1, nx, nv]
    Wx = (lx[:, 1:] - lx[:, :-1]) / dx
    Wy = (ly[1:] - ly[:-1]) / dy
    return avg, Wx, Wy


def isentropic_vortex_2d(n, *, ny=None, L=10.0, eps=5.0, mu=1e-4, gamma=1.4, order=8, recon=1, cfl=0.3,
                         t_end=1e9, acoustic_amp=1e-3, nmodes=32, seed=3, periodic_images=True):
    """Isentropic vortex of strength eps at the domain centre on the mean flow
    (1, 1), plus a seeded random-phase acoustic perturbation
    p' = (amp/64) sum_{k=1..nmodes} [cos(2 pi k x/L + phi_k) + cos(2 pi k y/L + chi_k)],
    rho' = p'/gamma; periodic [0, L]^2."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2 * math.pi, nmodes)
    chi = rng.uniform(0.0, 2 * math.pi, nmodes)
    kk = np.arange(1, nmodes + 1)
    xc0 = yc0 = 0.5 * L

    def fn(X, Y):
        X, Y = np.asarray(X, dtype=np.float64), np.asarray(Y, dtype=np.float64)
        shape = np.broadcast_shapes(X.shape, Y.shape)
        # exp((1 - r^2)/2) = e^{1/2} e^{-x'^2/2} e^{-y'^2/2}: the sums over the
        # periodic images factorise into 1-D sums
        shifts = (-L, 0.0, L) if periodic_images else (0.0,)
        sx0 = sx1 = sx2 = 0.0
        sy0 = sy1 = sy2 = 0.0
        for sh in shifts:
            xr = X - xc0 - sh
            yr = Y - yc0 - sh
            ex = np.exp(-0.5 * xr * xr)
            ey = np.exp(-0.5 * yr * yr)
            sx0, sx1, sx2 = sx0 + ex, sx1 + ex * xr, sx2 + ex * ex
            sy0, sy1, sy2 = sy0 + ey, sy1 + ey * yr, sy2 + ey * ey
        c = math.exp(0.5)
        du = -eps / (2 * math.pi) * c * sx0 * sy1
        dv = eps / (2 * math.pi) * c * sx1 * sy0
        dT = -(gamma - 1.0) * eps * eps * math.e / (8 * gamma * math.pi ** 2) * sx2 * sy2
        T = 1.0 + dT
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        pp = np.zeros(shape)
        if acoustic_amp:
            # separable: evaluated on the coordinate arrays, then broadcast
            fx = np.cos(2 * math.pi * X[..., None] * kk / L + phi).sum(-1)
            fy = np.cos(2 * math.pi * Y[..., None] * kk / L + chi).sum(-1)
            pp = pp + acoustic_amp / 64.0 * (fx + fy)
        rho = rho + pp / gamma
        p = p + pp
        return prim_to_cons(rho, 1.0 + du, p, gamma, V=1.0 + dv)

    W, Wx, Wy = _cell_quadrature_2d(fn, n, ny, 0.0, L, 0.0, L)
    return Problem(2, n, ny, 0.0, L, 0.0, L, gamma, mu, cfl, 0.0, t_end, order, recon,
                   (0, 0, 0, 0), W, Wx, Wy, name=f"vortex2d_{n}x{ny}")


def quadrant_states(seed):
    """Four quadrant states (rho, u, v, p): rho ~ U[0.1, 1.5], u, v ~
    U[-0.8, 0.8], p ~ U[0.03, 1.5], quadrants 1..4 = (x>, y>), (x<, y>),
    (x<, y<), (x>, y<)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        out.append((rng.uniform(0.1, 1.5), rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), rng.uniform(0.03, 1.5)))
    return out


def riemann_2d(n, *, ny=None, seed=5, states=None, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=1e9, split=0.5):
    """Four-quadrant Riemann problem on [0, 1]^2, jumps on faces, zero slopes,
    extrapolated boundaries."""
    ny = n if ny is None else ny
    st = states if states is not None else quadrant_states(seed)
    ix = np.arange(n)[None, :] >= int(round(split * n))
    iy = np.arange(ny)[:, None] >= int(round(split * ny))
    q = np.where(ix & iy, 0, np.where(~ix & iy, 1, np.where(~ix & ~iy, 2, 3)))
    arr = np.array(st)
    rho, u, v, p = (arr[q, k] for k in range(4))
    W = prim_to_cons(rho, u, p, gamma, V=v)
    Z = np.zeros_like(W)
    return Problem(2, n, ny, 0.0, 1.0, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (1, 1, 1, 1), W, Z, Z.copy(), name=f"riemann2d_{n}x{ny}")


# Double Mach reflection (Sec. 4.5): Mach 10 shock, 60 degrees to the x axis,
# through (1/6, 0) at t = 0; post-shock and pre-shock (rho, U, V, p)
DMR_POST = (8.0, 4.125 * math.sqrt(3.0), -4.125, 116.5)
DMR_PRE = (1.4, 0.0, 0.0, 1.0)


def dmr_shock_x(y, t):
    """x position of the moving shock at height y and time t."""
    return 1.0 / 6.0 + (y + 20.0 * t) / math.sqrt(3.0)


def double_mach_2d(nx=960, ny=None, *, order=8, recon=1, gamma=1.4, cfl=0.3, t_end=0.2):
    """Double Mach reflection on [0, 4] x [0, 1] (Sec. 4.5).  Cells whose
    centre lies left of the shock take the post-shock state, the others the
    pre-shock state; zero slopes.  Boundaries: post-shock inflow on the left,
    extrapolation on the right; at the bottom the exact post-shock state for
    x < 1/6 and a reflecting wall beyond; at the top the exact shock motion
    (post-shock state left of the shock's crossing of y = 1, pre-shock
    state right of it)."""
    ny = nx // 4 if ny is None else ny
    dx, dy = 4.0 / nx, 1.0 / ny
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    post = np.array(xc[None, :] < dmr_shock_x(yc[:, None], 0.0))
    st = np.where(post[..., None], np.array(DMR_POST), np.array(DMR_PRE))
    W = prim_to_cons(st[..., 0], st[..., 1], st[..., 3], gamma, V=st[..., 2])
    Z = np.zeros_like(W)
    wpost = prim_to_cons(DMR_POST[0], DMR_POST[1], DMR_POST[3], gamma, V=DMR_POST[2])
    wpre = prim_to_cons(DMR_PRE[0], DMR_PRE[1], DMR_PRE[3], gamma, V=DMR_PRE[2])
    bstate = np.zeros((4, 2, 4))
    bsplit = np.zeros((4, 2))
    bstate[0, 0] = wpost                       # left: post-shock inflow
    bstate[2, 0] = wpost                       # bottom: post-shock below x = 1/6
    bsplit[2] = (1.0 / 6.0, 0.0)               #   wall beyond
    bstate[3, 0], bstate[3, 1] = wpost, wpre   # top: shock crossing y = 1
    bsplit[3] = (dmr_shock_x(1.0, 0.0), 20.0 / math.sqrt(3.0))
    return Problem(2, nx, ny, 0.0, 4.0, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon,
                   (3, 1, 4, 4), W, Z, Z.copy(), name=f"dmr_{nx}x{ny}",
                   bc_state=bstate, bc_split=bsplit, bc_beyond=(2, 2, 2, 3))


def pulse_box_2d(n, *, ny=None, bc=(2, 2, 2, 2), mu=0.0, gamma=1.4, order=8, recon=1, cfl=0.3, t_end=1e9,
                 xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0):
    """Smooth off-centre pressure / density pulse with a swirl on the unit
    box (reflecting walls by default, any boundary combination allowed):
    rho = 1 + 0.2 G, p = 1 + 0.5 G, (u, v) = 0.2 G (-(y - 0.55), x - 0.4)/0.15,
    G = exp(-((x - 0.4)^2 + (y - 0.55)^2) / 0.03); exact cell averages and
    cell-averaged gradients."""
    ny = n if ny is None else ny

    def fn(X, Y):
        G = np.exp(-((X - 0.4) ** 2 + (Y - 0.55) ** 2) / 0.03)
        rho = 1.0 + 0.2 * G
        u = -0.2 * G * (Y - 0.55) / 0.15
        v = 0.2 * G * (X - 0.4) / 0.15
        return prim_to_cons(rho, u, 1.0 + 0.5 * G, gamma, V=v)

    W, Wx, Wy = _cell_quadrature_2d(fn, n, ny, xlo, xhi, ylo, yhi)
    return Problem(2, n, ny, xlo, xhi, ylo, yhi, gamma, mu, cfl, 0.0, t_end, order, recon,
                   tuple(bc), W, Wx, Wy, name=f"pulse2d_{n}x{ny}")


def mirror_pair_1d(n, *, gamma=1.4, order=8, recon=1, cfl=0.3, t_end=0.5):
    """Data symmetric about x = 1 on the periodic [0, 2] (2n cells) and the
    same data on [1, 2] (n cells) between two reflecting walls: the walls'
    solution is the right half of the periodic one."""
    def fn(x):
        rho = 1.0 + 0.2 * np.cos(np.pi * x)
        return prim_to_cons(rho, 0.1 * np.sin(np.pi * x), 1.0 + 0.1 * np.cos(np.pi * x), gamma)

    Wf, Wxf = _cell_quadrature_1d(fn, 2 * n, 0.0, 2.0)
    Wh, Wxh = _cell_quadrature_1d(fn, n, 1.0, 2.0)
    full = Problem(1, 2 * n, 1, 0.0, 2.0, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon, (0, 0, 0, 0),
                   Wf, Wxf, None, name=f"mirror_full_n{2 * n}")
    half = Problem(1, n, 1, 1.0, 2.0, 0.0, 1.0, gamma, 0.0, cfl, 0.0, t_end, order, recon, (2, 2, 0, 0),
                   Wh, Wxh, None, name=f"mirror_walls_n{n}")
    return full, half


def axis_wave_2d(n, axis, *, order=8, recon=0, gamma=1.4, amp=0.1, k=math.pi, dt_fixed=1e-7, t_end=None):
    """Entropy wave along one axis of [0, 2]^2 (periodic): rho = 1 + amp sin(k s)
    with s = x and (U, V) = (1, 0) for axis 0, s = y and (0, 1) for axis 1;
    p = 1.  Uniform across the other axis; exact cell averages and gradients
    (the conservative variables are affine in rho)."""
    d = 2.0 / n
    sf = d * np.arange(n + 1)
    rho_f = 1.0 + amp * np.sin(k * sf)
    rho_avg = 1.0 + amp * (np.cos(k * sf[:-1]) - np.cos(k * sf[1:])) / (k * d)
    U, V = (1.0, 0.0) if axis == 0 else (0.0, 1.0)
    wa = prim_to_cons(rho_avg, U, 1.0, gamma, V=V)
    wf = prim_to_cons(rho_f, U, 1.0, gamma, V=V)
    ws = (wf[1:] - wf[:-1]) / d
    if axis == 0:
        W = np.ascontiguousarray(np.broadcast_to(wa[None, :, :], (n, n, 4)))
        Wx = np.ascontiguousarray(np.broadcast_to(ws[None, :, :], (n, n, 4)))
        Wy = np.zeros_like(W)
    else:
        W = np.ascontiguousarray(np.broadcast_to(wa[:, None, :], (n, n, 4)))
        Wy = np.ascontiguousarray(np.broadcast_to(ws[:, None, :], (n, n, 4)))
        Wx = np.zeros_like(W)
    return Problem(2, n, n, 0.0, 2.0, 0.0, 2.0, gamma, 0.0, 0.3, dt_fixed, dt_fixed if t_end is None else t_end,
                   order, recon, (0, 0, 0, 0), W, Wx, Wy, name=f"axis_wave_{axis}_n{n}")


def sine_wave_2d(n, *, order=6, recon=0, gamma=1.4, cfl=0.3, dt_fixed=0.0, t_end=2.0, amp=0.2):
    """2-D analogue of the accuracy test of Sec. 4.1: rho = 1 + amp sin(pi (x + y)),
    U = V = 1, p = 1 on the periodic [0, 2]^2; the exact solution translates
    along the diagonal (period 2 in time).  Exact cell averages and gradients."""
    def fn(X, Y):
        rho = 1.0 + amp * np.sin(np.pi * (X + Y))
        return prim_to_cons(rho, 1.0, 1.0, gamma, V=1.0)

    W, Wx, Wy = _cell_quadrature_2d(fn, n, n, 0.0, 2.0, 0.0, 2.0)
    return Problem(2, n, n, 0.0, 2.0, 0.0, 2.0, gamma, 0.0, cfl, dt_fixed, t_end, order, recon,
                   (0, 0, 0, 0), W, Wx, Wy, name=f"sine2d_n{n}")
