"""Seeded synthetic inputs for the RSST step (shared by tests, smoke and bench).

This module holds initial conditions only: grids, seeded random draws, and
the conversion of (rho, V, P) point values at cell centres to the
conservative state (rho, rho V, E) with E = e(rho, P) + rho|V|^2/2, e the
internal energy density of the gas (ideal: P/(gamma-1); or the van der
Waals gas below).  It contains none of the time-step arithmetic, and imports
neither the oracle nor the GPU library.

Every field is a float64 numpy array laid out [nvar][nz][ny][nx] (x fastest),
nvar = ndim + 2, variables (rho, rho V_1..rho V_ndim, E).  A parameter dict
(`cfg`) carries ndim, n, dx, gamma, xi, cfl, dt_rule, g, bc_lo, bc_hi, form.

Workloads (all in the paper's regime of low Mach number and large density
contrast; the paper's own test problems are defined in its Sec. 4):
  wave1d      1D periodic sound + entropy wave (linear analysis, Sec. 2.1/3.1)
  bubble2d    2D periodic advected dense bubble, contrast 10, Mach 0.01
  strat3d     3D stratified polytropic box, contrast 100, gravity, walls in z
  batch2d     many 2D stratified boxes of uneven size, contrast and xi
  adjoint2d   2D bubble with density noise, for gradients
  random      smooth random states with small-scale noise, for parity
Seeds are 20181211 + k.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 5.0 / 3.0
SEED0 = 20181211

# A van der Waals gas for the general equation of state (the paper reports
# having run such a gas without giving its parameters): attraction a = 0.2
# and co-volume b = 0.1, in units where rho and P are of order one, so that
# a rho^2 is a fifth of P and b rho a tenth at rho = P = 1.  Its internal
# energy density with constant specific heat is
#   e(rho, P) = (P + a rho^2)(1 - b rho)/(gamma-1) - a rho^2.
VDW = {"eos": "vdw", "eos_a": 0.2, "eos_b": 0.1}


def seed(k: int) -> int:
    return SEED0 + k


def internal_energy(rho, P, gamma=GAMMA, gas=None):
    """Internal energy density e(rho, P) of the ideal gas (gas None or
    eos 'ideal') or of a van der Waals gas {eos: 'vdw', eos_a, eos_b}."""
    P = np.asarray(P, dtype=np.float64)
    if gas is None or gas.get("eos", "ideal") == "ideal":
        return P / (gamma - 1.0)
    a, b = float(gas["eos_a"]), float(gas["eos_b"])
    return (P + a * rho * rho) * (1.0 - b * rho) / (gamma - 1.0) - a * rho * rho


def sound_speed(rho, P, gamma=GAMMA, gas=None):
    """Sound speed of the same gases, for setting up linear waves: ideal
    sqrt(gamma P / rho); van der Waals (textbook form)
    sqrt(gamma (P + a rho^2)/(rho (1 - b rho)) - 2 a rho)."""
    if gas is None or gas.get("eos", "ideal") == "ideal":
        return np.sqrt(gamma * P / rho)
    a, b = float(gas["eos_a"]), float(gas["eos_b"])
    return np.sqrt(gamma * (P + a * rho * rho) / (rho * (1.0 - b * rho)) - 2.0 * a * rho)


def with_gas(cfg: dict, gas) -> dict:
    """cfg with the equation-of-state keys of gas (None: unchanged)."""
    if gas is not None:
        cfg = dict(cfg)
        cfg.update(gas)
    return cfg


def conservative(rho, vel, P, gamma=GAMMA, gas=None) -> np.ndarray:
    """Stack (rho, rho V_i, E) from point values; vel is a list of arrays."""
    rho = np.asarray(rho, dtype=np.float64)
    comps = [rho]
    ke = np.zeros_like(rho)
    for v in vel:
        v = np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape)
        comps.append(rho * v)
        ke = ke + v * v
    E = internal_energy(rho, P, gamma, gas) + 0.5 * rho * ke
    comps.append(E)
    return np.ascontiguousarray(np.stack(comps))


def base_cfg(ndim, n, *, xi=1.0, form="pvs", bc_lo=None, bc_hi=None, g=None,
             length=None, gamma=GAMMA, cfl=0.4, dt_rule=0) -> dict:
    n = list(n)
    length = list(length) if length is not None else [1.0] * ndim
    bc_lo = list(bc_lo) if bc_lo is not None else ["periodic"] * ndim
    bc_hi = list(bc_hi) if bc_hi is not None else list(bc_lo)
    g = list(g) if g is not None else [0.0] * ndim
    return {
        "ndim": ndim,
        "n": n + [1] * (3 - ndim),
        "dx": [length[d] / n[d] for d in range(ndim)] + [1.0] * (3 - ndim),
        "gamma": gamma, "xi": float(xi), "cfl": cfl, "dt_rule": dt_rule,
        "g": g + [0.0] * (3 - ndim),
        "bc_lo": bc_lo + ["periodic"] * (3 - ndim),
        "bc_hi": bc_hi + ["periodic"] * (3 - ndim),
        "form": form,
    }


def centres(cfg: dict, d: int) -> np.ndarray:
    return (np.arange(cfg["n"][d]) + 0.5) * cfg["dx"][d]


# --------------------------------------------------------------- 1D wave

def wave1d(xi=1.0, form="pvs", n=256, eps=1e-4, gas=None):
    """Right-going RSST sound wave plus a static entropy wave, one wavelength.

    rho0 = P0 = 1.  Sound: drho = eps sin kx, dP = a0^2 drho,
    dV = xi a0 drho / rho0 (the RSST sound eigenvector: the velocity
    amplitude is xi times the Euler one).  Entropy: drho = eps cos kx.
    Runs to t_end = 2 xi L / a0, two crossings at the reduced speed a0/xi.
    gas: None (ideal) or a van der Waals gas, whose a0 the wave then uses.
    """
    cfg = with_gas(base_cfg(1, [n], xi=xi, form=form), gas)
    x = centres(cfg, 0)
    k = 2 * math.pi
    a0 = float(sound_speed(1.0, 1.0, GAMMA, gas))
    ds = eps * np.sin(k * x)
    de = eps * np.cos(k * x)
    rho = 1.0 + ds + de
    P = 1.0 + a0 * a0 * ds
    V = xi * a0 * ds
    U = conservative(rho, [V], P, gas=gas)
    meta = {"t_end": 2.0 * xi / a0, "a0": a0, "eps": eps, "k": k}
    return cfg, U, meta


# --------------------------------------------------------------- 2D bubble

def _bubble_prims(n, xi, rng, *, contrast=10.0, mach=0.01, vnoise=1e-5):
    cfg = base_cfg(2, [n, n], xi=xi)
    x = centres(cfg, 0)[None, :]
    y = centres(cfg, 1)[:, None]
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
    w = 4.0 * cfg["dx"][0]
    rho = 1.0 + (contrast - 1.0) * 0.5 * (1.0 - np.tanh((r - 0.125) / w))
    a_bub = math.sqrt(GAMMA / contrast)
    v0 = mach * a_bub
    vx = v0 + vnoise * rng.uniform(-1.0, 1.0, size=(n, n))
    vy = vnoise * rng.uniform(-1.0, 1.0, size=(n, n))
    P = np.ones((n, n))
    return cfg, rho, vx, vy, P, v0


def bubble2d(n=512, xi=20.0, form="pvs"):
    """Dense bubble (contrast 10, tanh edge 4 cells) advected at Mach 0.01 of
    the bubble's sound speed, uniform P = 1, velocity noise 1e-5.
    Background for the FP32-perturbation form: the uniform ambient state."""
    rng = np.random.default_rng(seed(2))
    cfg, rho, vx, vy, P, v0 = _bubble_prims(n, xi, rng)
    cfg["form"] = form
    U = conservative(rho, [vx, vy], P)
    bg = conservative(np.ones(1), [np.full(1, v0), np.zeros(1)], np.ones(1))  # [nv][1]
    return cfg, U, {"bg": bg, "bg_axis": -1, "v0": v0}


# --------------------------------------------------------------- stratified

def polytrope(z, contrast=100.0, delta=1e-4, g=1.0):
    """Polytropic hydrostatic layer P = rho T on z in [0,1], gravity g along -z.

    Index m = 1/(nabla_ad + delta) - 1 with nabla_ad = (gamma-1)/gamma,
    T(z) = T_bot - g z/(m+1), T_bot chosen so rho(0)/rho(1) = contrast,
    rho = (T/T_bot)^m, rho(0) = 1."""
    nab = (GAMMA - 1.0) / GAMMA
    m = 1.0 / (nab + delta) - 1.0
    T_bot = g / ((m + 1.0) * (1.0 - contrast ** (-1.0 / m)))
    T = T_bot - g * z / (m + 1.0)
    rho = (T / T_bot) ** m
    return rho, rho * T


def strat3d(n=256, xi=30.0, form="pvs", nz=None, ny=None, gas=None):
    """3D stratified box: polytrope along z (contrast 100, delta 1e-4, g = 1
    along -z), walls in z, periodic in x and y, V = 0, pressure noise
    P <- P (1 + 1e-3 U(-1,1)).  Background: the unperturbed polytrope.
    gas: a van der Waals gas keeps the same rho and P (hydrostatic balance
    does not involve the equation of state) with its own E."""
    nz = nz or n
    ny = ny or n
    cfg = with_gas(base_cfg(3, [n, ny, nz], xi=xi, form=form,
                            bc_lo=["periodic", "periodic", "reflect"], g=[0.0, 0.0, -1.0]), gas)
    z = centres(cfg, 2)
    rho0, P0 = polytrope(z)
    rng = np.random.default_rng(seed(3))
    noise = rng.uniform(-1.0, 1.0, size=(nz, ny, n))
    rho = np.broadcast_to(rho0[:, None, None], (nz, ny, n))
    P = P0[:, None, None] * (1.0 + 1e-3 * noise)
    zero = np.zeros((nz, ny, n))
    U = conservative(rho, [zero, zero, zero], P, gas=gas)
    bg = conservative(rho0, [np.zeros(nz)] * 3, P0, gas=gas)  # [nv][nz]
    return cfg, U, {"bg": bg, "bg_axis": 2}


def stratified(ndim, n, axis, *, xi=30.0, form="pvs", contrast=100.0, seed_k=30, wall_bc=None):
    """A polytrope (as strat3d) along any axis: gravity 1 along -axis, walls
    on that axis, periodic on the others (or wall_bc on the others), V = 0,
    pressure noise 1e-3 relative.  Background: the unperturbed profile
    [nv][n[axis]]."""
    bc = [wall_bc or "periodic"] * ndim
    bc[axis] = "reflect"
    g = [0.0] * ndim
    g[axis] = -1.0
    cfg = base_cfg(ndim, n, xi=xi, form=form, bc_lo=bc, g=g)
    z = centres(cfg, axis)
    rho0, P0 = polytrope(z, contrast=contrast)
    shape = tuple(reversed(list(n)[:ndim]))  # [nz][ny][nx] order
    bshape = [1] * ndim
    bshape[ndim - 1 - axis] = n[axis]
    rng = np.random.default_rng(seed(seed_k))
    noise = rng.uniform(-1.0, 1.0, size=shape)
    rho = np.broadcast_to(rho0.reshape(bshape), shape)
    P = P0.reshape(bshape) * (1.0 + 1e-3 * noise)
    zero = np.zeros(shape)
    U = conservative(rho, [zero] * ndim, P)
    bg = conservative(rho0, [np.zeros(n[axis])] * ndim, P0)
    return cfg, U, {"bg": bg, "bg_axis": axis}


def strat2d_box(n, contrast, xi, rng, form="pvs"):
    """One 2D stratified box: polytrope along -y, walls in y, periodic in x."""
    cfg = base_cfg(2, [n, n], xi=xi, form=form, bc_lo=["periodic", "reflect"],
                   g=[0.0, -1.0])
    y = centres(cfg, 1)
    rho0, P0 = polytrope(y, contrast=contrast)
    noise = rng.uniform(-1.0, 1.0, size=(n, n))
    rho = np.broadcast_to(rho0[:, None], (n, n))
    P = P0[:, None] * (1.0 + 1e-3 * noise)
    zero = np.zeros((n, n))
    U = conservative(rho, [zero, zero], P)
    bg = conservative(rho0, [np.zeros(n)] * 2, P0)
    return cfg, U, {"bg": bg, "bg_axis": 1}


def batch2d(nbox=512, nmin=64, nmax=256, form="pvs"):
    """Boxes with N ~ U{nmin..nmax}, contrast ~ logU[3,100], xi ~ logU[1,50],
    drawn in that order for all boxes, then each box's pressure noise."""
    rng = np.random.default_rng(seed(4))
    ns = rng.integers(nmin, nmax + 1, size=nbox)
    contrast = np.exp(rng.uniform(math.log(3.0), math.log(100.0), size=nbox))
    xis = np.exp(rng.uniform(0.0, math.log(50.0), size=nbox))
    boxes = []
    for b in range(nbox):
        boxes.append(strat2d_box(int(ns[b]), float(contrast[b]), float(xis[b]), rng, form))
    return boxes


# --------------------------------------------------------------- adjoint

def adjoint2d(n=256, xi=10.0, form="pvs", ndir=32):
    """Bubble as bubble2d with xi = 10 plus density noise rho <- rho (1 + 1e-5 U)
    (breaks exact limiter ties of flat regions), and ndir smooth unit-max
    directions for the initial density (Fourier modes |k| <= 4, N(0,1))."""
    rng = np.random.default_rng(seed(5))
    cfg, rho, vx, vy, P, v0 = _bubble_prims(n, xi, rng)
    cfg["form"] = form
    rho_clean = rho.copy()
    rho = rho * (1.0 + 1e-5 * rng.uniform(-1.0, 1.0, size=rho.shape))
    x = centres(cfg, 0)[None, :]
    y = centres(cfg, 1)[:, None]
    dirs = np.zeros((ndir, n, n))
    for q in range(ndir):
        f = np.zeros((n, n))
        for kx in range(-4, 5):
            for ky in range(-4, 5):
                a, b = rng.standard_normal(2)
                ph = 2 * math.pi * (kx * x + ky * y)
                f += a * np.cos(ph) + b * np.sin(ph)
        dirs[q] = f / np.abs(f).max()
    U = conservative(rho, [vx, vy], P)
    U_clean = conservative(rho_clean, [vx, vy], P)
    return cfg, U, {"rho": rho, "vx": vx, "vy": vy, "P": P, "dirs": dirs,
                    "U_clean": U_clean}


# --------------------------------------------------------------- Sec. 4.2

def wave2d_oblique(n, form="pvs", xi=5.0, theta_deg=30.0, eps=1e-5, P0=1000.0):
    """Linear entropy + shear wave travelling at theta to x (Sec. 4.2): domain
    [0, 1/cos] x [0, 1/sin] (one wavelength along the wave vector fits both
    periods), rho = 1 + eps sin(2 pi x_par), V_par = 1,
    V_perp = eps sin(2 pi x_par), P = P0; after t = 1 the exact solution is
    the initial state again."""
    th = math.radians(theta_deg)
    Lx, Ly = 1 / math.cos(th), 1 / math.sin(th)
    cfg = base_cfg(2, [n, n], xi=xi, form=form, length=[Lx, Ly])
    x = centres(cfg, 0)[None, :]
    y = centres(cfg, 1)[:, None]
    xp = x * math.cos(th) + y * math.sin(th)
    rho = 1 + eps * np.sin(2 * math.pi * xp)
    vperp = eps * np.sin(2 * math.pi * xp)
    vx = math.cos(th) - vperp * math.sin(th)
    vy = math.sin(th) + vperp * math.cos(th)
    P = np.full_like(rho, P0)
    return cfg, conservative(rho, [vx, vy], P), {"theta": th, "t_end": 1.0}


# --------------------------------------------------------------- Sec. 4.4

def _logcosh2(a):
    """ln(e^a + e^-a), overflow-free."""
    a = np.abs(a)
    return a + np.log1p(np.exp(-2.0 * a))


def rt_column_mass(y, rho1=1.0, rho2=10.0, L=0.025):
    """Background column mass from height y to the top (y = 1) of the
    unperturbed tanh profile, in the closed form of Sec. 4.4."""
    return (0.5 * (rho1 + rho2) * (1.0 - y)
            + 0.5 * L * (rho2 - rho1) * (_logcosh2(0.5 / L) - _logcosh2((y - 0.5) / L)))


def rt2d(n, form="pvs", xi=6.3, rho1=1.0, rho2=10.0, L=0.025, amp=0.01, Pc=1000.0, gy=-1.0,
         strip=False):
    """Rayleigh-Taylor problem of Sec. 4.4 on [0,1]^2: heavy fluid (rho2) on
    top of light (rho1) across a tanh layer of width L, density perturbed by
    (1 + amp sin 4 pi x), hydrostatic P = Pc - m_c g_y with the unperturbed
    column mass, V = 0, periodic x, closed free-slip walls in y.

    strip=True: the same n x n problem on the cells of x in [1/8, 3/8] only
    (n/4 x n cells), with mirror walls at both x ends.  sin 4 pi x is even
    about x = 1/8 and x = 3/8, the equations and the scheme are invariant
    under the mirror x -> 2a - x (m_x negated), and the periodic domain is a
    union of mirror copies of this strip, so the strip's solution is the
    periodic run's restricted to it (to rounding): a finer grid than the
    1024-cell rows of the 2D kernels, at a quarter of the cost."""
    if strip:
        if n % 8:
            raise ValueError("strip needs n divisible by 8 (x = 1/8 on a cell face)")
        nx, x0, lx, bcx = n // 4, 0.125, 0.25, "reflect"
    else:
        nx, x0, lx, bcx = n, 0.0, 1.0, "periodic"
    cfg = base_cfg(2, [nx, n], xi=xi, form=form, bc_lo=[bcx, "reflect"], g=[0.0, gy],
                   length=[lx, 1.0])
    x = x0 + centres(cfg, 0)[None, :]
    y = centres(cfg, 1)[:, None]
    eps = amp * np.sin(4.0 * math.pi * x)
    rho = (rho1 + 0.5 * (rho2 - rho1) * (1.0 + np.tanh((y - 0.5) / L))) * (1.0 + eps)
    P = np.broadcast_to(Pc - rt_column_mass(y, rho1, rho2, L) * gy, (n, nx)).copy()
    zero = np.zeros((n, nx))
    return cfg, conservative(rho, [zero, zero], P), {"t_end": 2.5, "x0": x0}


# --------------------------------------------------------------- random

def random_state(ndim, n, *, seed_k=100, xi=3.0, form="pvs", bc_lo=None, bc_hi=None,
                 g=None, mach=0.3, drho=0.5, dP=0.3, white=0.02, length=None, gas=None):
    """Smooth random admissible state plus small white noise (exercises every
    limiter branch).  rho in about [1-drho, 1+drho], P about 1 +- dP, |V|
    about mach * a.  gas: None (ideal) or a van der Waals gas."""
    rng = np.random.default_rng(seed(seed_k))
    cfg = with_gas(base_cfg(ndim, n, xi=xi, form=form, bc_lo=bc_lo, bc_hi=bc_hi, g=g, length=length),
                   gas)
    shape = tuple(reversed(list(n)))
    grids = np.meshgrid(*[centres(cfg, d) / (cfg["dx"][d] * cfg["n"][d])
                          for d in reversed(range(ndim))], indexing="ij")
    # grids[q] varies along axis ndim-1-q

    def smooth():
        f = np.zeros(shape)
        for _ in range(4):
            ph = rng.uniform(0, 2 * math.pi)
            arg = ph
            for q in range(ndim):
                arg = arg + 2 * math.pi * rng.integers(1, 4) * grids[q]
            f += rng.uniform(0.5, 1.0) * np.sin(arg)
        f /= 4.0
        return f + white * rng.uniform(-1, 1, size=shape)

    rho = 1.0 + drho * smooth()
    P = 1.0 + dP * smooth()
    a = np.sqrt(GAMMA * P / rho)
    vel = [mach * a * smooth() for _ in range(ndim)]
    return cfg, conservative(rho, vel, P, gas=gas)
