"""Seeded synthetic inputs for the free-surface LBM step.

This module produces initial *macroscopic* fields only -- cell classes, density,
velocity and fill level -- plus the model parameters.  It contains none of the
lattice Boltzmann arithmetic: the GPU library and the oracle each build their
own populations from these fields.  Both the tests and the benchmark use it.

Geometry conventions: cell (i, j, k) has linear index i + nx*(j + ny*k), its
centre sits at y = j + 1/2, and a wall at a non-periodic face lies half a cell
beyond the outermost cells (bounce-back, first node at distance 1/2; the
steady film experiment of section 4.3 uses that placement).  A liquid column of
height eta fills cell j with min(max(eta - j, 0), 1).  Fill 1 is liquid, fill 0
is gas, anything in between is interface; a liquid cell touching gas on any
D3Q19 link is turned into an interface cell with fill 1, so that a layer of
interface cells always separates liquid from gas (section 2.3).

Initial density: rho_gas plus the hydrostatic head 3|g_y| (eta - y) of the
liquid above the cell centre (c_s^2 = 1/3, incompressible form); velocity 0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAS, INTERFACE, LIQUID, SOLID = 0, 1, 2, 3

# Link order of the population buffers and wall tables at the library boundary:
# rest, the six axis links, then the twelve diagonals; odd q has its opposite
# at q + 1.
LINKS = np.array([(0, 0, 0),
                  (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                  (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
                  (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
                  (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=np.int64)

# offsets of the 18 nearest neighbours on the cubic lattice (|d|^2 = 1 or 2)
_NEIGHBOURS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
               if 1 <= dx * dx + dy * dy + dz * dz <= 2]


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    nz: int
    periodic: tuple = (0, 0, 0)
    tau: float = 0.8
    Lambda: float = 3.0 / 16.0
    incompressible: int = 1
    stokes: int = 0
    g: tuple = (0.0, 0.0, 0.0)
    rho_gas: float = 1.0
    eps: float = 1e-3
    wall_u: tuple = ((0.0, 0.0, 0.0),) * 6   # wall face velocities: x-, x+, y-, y+, z-, z+
    shear_b: tuple = (0.0,) * 6               # prescribed S^b [xx, yy, zz, xy, xz, yz]
    sigma: float = 0.0                        # surface tension coefficient
    plic: int = 0                             # FSL link distance from the PLIC plane
    hold: int = 0                             # fill levels and interface masses held (with frozen classes)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Workload:
    name: str
    params: Params
    flags: np.ndarray            # uint8[N]
    rho: np.ndarray              # float64[N]
    u: np.ndarray | None         # float64[3, N] or None (= at rest)
    fill: np.ndarray             # float64[N]
    meta: dict = dataclasses.field(default_factory=dict)
    # solid walls: {"cells": int32[n] ascending non-solid cells next to a solid
    # cell, "delta": float64[19, n] wall point x + delta c_p on link p,
    # "uw": float64[3, 19, n] wall velocity}; None without solid cells
    walls: dict | None = None
    # a prescribed surface (with params.hold): {"normal": float64[3, N] unit
    # normal towards the gas, "offset": float64[N] signed distance of the plane
    # from the node along it}, read at interface cells; None otherwise
    surface: dict | None = None

    def velocity(self) -> np.ndarray:
        if self.u is None:
            return np.zeros((3, self.params.n_cells))
        return self.u

    def counts(self) -> dict:
        b = np.bincount(self.flags, minlength=3)
        return {"gas": int(b[GAS]), "interface": int(b[INTERFACE]), "liquid": int(b[LIQUID])}


def _shift_any(mask3: np.ndarray, periodic) -> np.ndarray:
    """True where any of the 18 neighbours (walls excluded) is set in mask3."""
    out = np.zeros_like(mask3)
    nz, ny, nx = mask3.shape
    for dx, dy, dz in _NEIGHBOURS:
        src = mask3
        for axis, d, per in ((2, dx, periodic[0]), (1, dy, periodic[1]), (0, dz, periodic[2])):
            if d == 0:
                continue
            if per:
                src = np.roll(src, -d, axis=axis)
            else:
                # neighbour at +d; cells whose neighbour is beyond the wall get False
                sl_dst = [slice(None)] * 3
                sl_src = [slice(None)] * 3
                n = src.shape[axis]
                if d > 0:
                    sl_dst[axis] = slice(0, n - d)
                    sl_src[axis] = slice(d, n)
                else:
                    sl_dst[axis] = slice(-d, n)
                    sl_src[axis] = slice(0, n + d)
                tmp = np.zeros_like(src)
                tmp[tuple(sl_dst)] = src[tuple(sl_src)]
                src = tmp
        out |= src
    return out


def _from_height(params: Params, eta: np.ndarray, name: str, meta: dict) -> Workload:
    """Liquid below a surface height eta(x) (uniform in z) or eta(z, x)."""
    nx, ny, nz = params.nx, params.ny, params.nz
    eta3 = np.broadcast_to(np.asarray(eta, dtype=np.float64).reshape(-1, nx), (nz, nx))  # [nz, nx]
    j = np.arange(ny, dtype=np.float64)
    fill3 = np.clip(eta3[:, None, :] - j[None, :, None], 0.0, 1.0)  # [nz, ny, nx]
    types3 = np.where(fill3 >= 1.0, LIQUID, np.where(fill3 <= 0.0, GAS, INTERFACE)).astype(np.uint8)
    gas_near = _shift_any(types3 == GAS, params.periodic)
    promote = (types3 == LIQUID) & gas_near
    types3[promote] = INTERFACE
    fill3[promote] = 1.0
    yc = j + 0.5
    if params.g[1] == 0.0:
        rho3 = np.full((nz, ny, nx), params.rho_gas)
    else:
        rho3 = params.rho_gas + 3.0 * abs(params.g[1]) * (eta3[:, None, :] - yc[None, :, None])
    rho3[types3 == GAS] = params.rho_gas
    flags = types3.reshape(-1)
    return Workload(name=name, params=params, flags=flags, rho=rho3.reshape(-1), u=None,
                    fill=fill3.reshape(-1), meta=meta)


def channel(h: float = 32.5, nx: int = 8, ny: int = 48, nz: int = 8, gx: float = 1e-6,
            tau: float = 0.8, Lambda: float = 3.0 / 16.0, stokes: int = 0) -> Workload:
    """Gravity-driven open-channel film: x, z periodic, wall at y = 0 (and at
    the top, which only ever borders gas), flat surface at height h."""
    p = Params(nx=nx, ny=ny, nz=nz, periodic=(1, 0, 1), tau=tau, Lambda=Lambda,
               g=(gx, 0.0, 0.0), stokes=stokes)
    eta = np.full(nx, float(h))
    return _from_height(p, eta, "channel", {"h": h, "gx": gx})


def channel_sweep(h: int, tau: float = 0.8, Lambda: float = 3.0 / 16.0, frac: float = 0.5,
                  stokes: int = 0, nx: int = 4, nz: int = 4) -> Workload:
    """Convergence-sweep member: film of height h + frac on a 4 x (h+16) x 4
    grid, g_x = 1e-6 (32/h)^3 (diffusive scaling at fixed Reynolds number)."""
    gx = 1e-6 * (32.0 / h) ** 3
    w = channel(h=h + frac, nx=nx, ny=h + 16, nz=nz, gx=gx, tau=tau, Lambda=Lambda, stokes=stokes)
    w.name = f"sweep_h{h}"
    w.meta.update({"h_cells": h, "frac": frac})
    return w


def sloshing(nx: int = 256, ny: int = 160, nz: int = 256, depth: float = 96.0, amp: float = 6.0,
             seed: int = 0, gy: float = -2e-5, tau: float = 0.55, Lambda: float = 3.0 / 16.0,
             wavelength: float | None = None, periodic=(0, 0, 0), amp_z: float = 0.0) -> Workload:
    """Closed tank (walls on all faces) with a cosine surface
    eta(i, k) = depth + amp cos(2 pi (i + 1/2)/wavelength + theta)
                      + amp_z cos(2 pi (k + 1/2)/nz + theta_z),
    theta and theta_z drawn from the seed (in that order), liquid initially at
    hydrostatic rest.  amp_z = 0 gives a surface uniform in z."""
    rng = np.random.default_rng(seed)
    theta = 2.0 * math.pi * float(rng.random())
    theta_z = 2.0 * math.pi * float(rng.random())
    lam = float(nx if wavelength is None else wavelength)
    i = np.arange(nx, dtype=np.float64)
    k = np.arange(nz, dtype=np.float64)
    eta = depth + amp * np.cos(2.0 * math.pi * (i + 0.5) / lam + theta)
    if amp_z != 0.0:
        eta = eta[None, :] + amp_z * np.cos(2.0 * math.pi * (k[:, None] + 0.5) / nz + theta_z)
    p = Params(nx=nx, ny=ny, nz=nz, periodic=tuple(periodic), tau=tau, Lambda=Lambda, g=(0.0, gy, 0.0))
    return _from_height(p, eta, "sloshing",
                        {"depth": depth, "amp": amp, "amp_z": amp_z, "seed": seed, "theta": theta,
                         "theta_z": theta_z, "wavelength": lam})


def pool(nx: int = 32, ny: int = 64, nz: int = 32, level: float = 40.5, gy: float = -1e-5,
         tau: float = 0.8, Lambda: float = 3.0 / 16.0) -> Workload:
    """Flat pool at hydrostatic rest in a closed tank."""
    p = Params(nx=nx, ny=ny, nz=nz, periodic=(0, 0, 0), tau=tau, Lambda=Lambda, g=(0.0, gy, 0.0))
    return _from_height(p, np.full(nx, float(level)), "pool", {"level": level})


def droplet(n: int = 32, radius: float = 8.0, sigma: float = 1e-3, tau: float = 0.8,
            Lambda: float = 3.0 / 16.0, offset=(0.1, 0.23, 0.37), sub: int = 6) -> Workload:
    """Spherical liquid droplet at rest in a periodic box of gas, no gravity.
    Fill = volume fraction of the sphere in each cell (sub^3 sample points);
    density rho_b + 6 sigma / R inside (the Laplace pressure P_b + 2 sigma / R)."""
    p = Params(nx=n, ny=n, nz=n, periodic=(1, 1, 1), tau=tau, Lambda=Lambda, sigma=sigma)
    c = np.array([n / 2 + offset[0], n / 2 + offset[1], n / 2 + offset[2]])
    k = (np.arange(sub) + 0.5) / sub
    idx = np.indices((n, n, n)).astype(np.float64)  # [3 (z, y, x), n, n, n]
    fill3 = np.zeros((n, n, n))
    for a in k:
        for b in k:
            for cc in k:
                r2 = (idx[2] + a - c[0]) ** 2 + (idx[1] + b - c[1]) ** 2 + (idx[0] + cc - c[2]) ** 2
                fill3 += r2 <= radius * radius
    fill3 /= sub ** 3
    types3 = np.where(fill3 >= 1.0, LIQUID, np.where(fill3 <= 0.0, GAS, INTERFACE)).astype(np.uint8)
    gas_near = _shift_any(types3 == GAS, p.periodic)
    promote = (types3 == LIQUID) & gas_near
    types3[promote] = INTERFACE
    fill3[promote] = 1.0
    rho3 = np.where(types3 == GAS, p.rho_gas, p.rho_gas + 6.0 * sigma / radius)
    return Workload(name="droplet", params=p, flags=types3.reshape(-1), rho=rho3.reshape(-1), u=None,
                    fill=fill3.reshape(-1), meta={"radius": radius, "sigma": sigma})


def _skew_zeta(nx: int, nz: int, slope: float):
    """Vertical offset zeta = z - slope x of the cell centres, in [0, nz)
    ([nz, nx] array; the strips below are bands of zeta)."""
    xc = np.arange(nx) + 0.5
    zc = np.arange(nz) + 0.5
    return np.mod(zc[:, None] - slope * xc[None, :], float(nz))


def skew_strips(nx: int, ny: int, nz: int, slope: float, bands, p: Params):
    """Bands of zeta = z - slope x (x, y, z periodic; slope * nx a multiple of
    nz so that the bands close on themselves).  bands: consecutive
    (upper edge, kind, tangential velocity) from zeta = 0 to nz, kind "solid"
    or "fluid"; a solid band moves with its velocity along the tangent
    t = (1, 0, slope)/|.|.  Returns the class field [nz, ny, nx] (fluid cells
    LIQUID) and the wall table: for each fluid cell next to a solid cell and
    each link p into a solid cell, the exact distance delta of the crossing of
    the band edge along c_p and the wall's velocity."""
    if abs(slope * nx / nz - round(slope * nx / nz)) > 1e-12:
        raise ValueError("slope * nx must be a multiple of nz")
    zeta = _skew_zeta(nx, nz, slope)
    edges = [0.0] + [float(b[0]) for b in bands]
    kind = np.empty((nz, nx), dtype=np.uint8)
    band = np.empty((nz, nx), dtype=np.int64)
    for i, (hi, k, _) in enumerate(bands):
        sel = (zeta >= edges[i]) & (zeta < hi)
        kind[sel] = SOLID if k == "solid" else LIQUID
        band[sel] = i
    types3 = np.broadcast_to(kind[:, None, :], (nz, ny, nx)).copy()
    tang = np.array([1.0, 0.0, slope]) / np.hypot(1.0, slope)
    flags = types3.reshape(-1)
    N = nx * ny * nz
    idx = np.arange(N)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    solid = flags == SOLID
    near = np.zeros(N, dtype=bool)
    for q in range(1, 19):
        c = LINKS[q]
        s_ = ((x + c[0]) % nx) + nx * (((y + c[1]) % ny) + ny * ((z + c[2]) % nz))
        near |= solid[s_]
    cells = np.nonzero(near & ~solid)[0].astype(np.int32)
    n = cells.size
    delta = np.full((19, n), 0.5)
    uw = np.zeros((3, 19, n))
    cx, cy, cz = x[cells], y[cells], z[cells]
    zc = zeta[cz, cx]
    bc = band[cz, cx]
    for q in range(1, 19):
        c = LINKS[q]
        s_ = ((cx + c[0]) % nx) + nx * (((cy + c[1]) % ny) + ny * ((cz + c[2]) % nz))
        hit = solid[s_]
        if not hit.any():
            continue
        d = c[2] - slope * c[0]          # change of zeta along the link
        up = d > 0
        lo = np.array(edges)[bc]
        hi_ = np.array(edges)[bc + 1]
        dl = np.where(up, (hi_ - zc) / np.where(d != 0, d, 1.0), (lo - zc) / np.where(d != 0, d, 1.0))
        nb = np.where(up, (bc + 1) % len(bands), (bc - 1) % len(bands))
        vel = np.array([b[2] for b in bands])[nb]
        delta[q, hit] = dl[hit]
        for a in range(3):
            uw[a, q, hit] = vel[hit] * tang[a]
    return types3, {"cells": cells, "delta": delta, "uw": uw}, zeta


def skew_couette(nz: int = 16, slope: float = 0.25, U: float = 1e-3, ny: int = 1, tau: float = 0.8,
                 Lambda: float = 3.0 / 16.0, stokes: int = 1, bands=None) -> Workload:
    """Plane Couette flow in a channel rotated by atan(slope) against the
    lattice (section 4.2: CLI walls recover it exactly with the linear
    equilibrium): two solid bands, the lower one moving with U along the
    channel, the upper one at rest, two liquid layers between them; x, y, z
    periodic, nx = nz / slope; at rest at t = 0.  meta["profile"](zeta) is the
    steady tangential velocity."""
    nx = int(round(nz / slope))
    if bands is None:
        bands = ((3.3, "solid", U), (8.6, "fluid", 0.0), (11.2, "solid", 0.0), (float(nz), "fluid", 0.0))
    p = Params(nx=nx, ny=ny, nz=nz, periodic=(1, 1, 1), tau=tau, Lambda=Lambda, stokes=stokes)
    types3, walls, zeta = skew_strips(nx, ny, nz, slope, bands, p)
    edges = [0.0] + [float(b[0]) for b in bands]

    def profile(zz):
        out = np.full(np.shape(zz), np.nan)
        for i, (hi, k, _) in enumerate(bands):
            if k != "fluid":
                continue
            lo = edges[i]
            ulo = bands[(i - 1) % len(bands)][2]
            uhi = bands[(i + 1) % len(bands)][2]
            sel = (zz >= lo) & (zz < hi)
            out = np.where(sel, ulo + (uhi - ulo) * (zz - lo) / (hi - lo), out)
        return out

    N = p.n_cells
    return Workload(name="skew_couette", params=p, flags=types3.reshape(-1), rho=np.ones(N), u=None,
                    fill=np.where(types3.reshape(-1) == SOLID, 0.0, 1.0),
                    meta={"slope": slope, "U": U, "zeta": np.broadcast_to(zeta[:, None, :], (nz, ny, nx)).reshape(-1),
                          "tangent": np.array([1.0, 0.0, slope]) / np.hypot(1.0, slope), "profile": profile},
                    walls=walls)


def add_plane_obstacle(w: Workload, normal, offset: float, velocity=(0.0, 0.0, 0.0), name=None) -> Workload:
    """Make every cell whose centre x_c has normal . x_c < offset solid (a
    half-space obstacle, e.g. an inclined ramp), and build the wall table with
    the exact distance of each link's crossing of the plane and the obstacle's
    velocity.  Cells next to the obstacle keep their class; their fill and
    density are unchanged."""
    p = w.params
    nx, ny, nz = p.nx, p.ny, p.nz
    nrm = np.asarray(normal, dtype=np.float64)
    N = p.n_cells
    idx = np.arange(N)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    xc = np.stack([x + 0.5, y + 0.5, z + 0.5]).astype(np.float64)
    side = nrm @ xc - offset                     # < 0 inside the obstacle
    flags = w.flags.copy()
    flags[side < 0.0] = SOLID
    solid = flags == SOLID
    dims = (nx, ny, nz)

    def nb(c):
        cc = [x + c[0], y + c[1], z + c[2]]
        ok = np.ones(N, dtype=bool)
        for a in range(3):
            if p.periodic[a]:
                cc[a] = cc[a] % dims[a]
            else:
                ok &= (cc[a] >= 0) & (cc[a] < dims[a])
                cc[a] = np.clip(cc[a], 0, dims[a] - 1)
        return cc[0] + nx * (cc[1] + ny * cc[2]), ok

    near = np.zeros(N, dtype=bool)
    for q in range(1, 19):
        s_, ok = nb(LINKS[q])
        near |= ok & solid[s_]
    cells = np.nonzero(near & ~solid)[0].astype(np.int32)
    n = cells.size
    delta = np.full((19, n), 0.5)
    uw = np.zeros((3, 19, n))
    for q in range(1, 19):
        s_, ok = nb(LINKS[q])
        hit = (ok & solid[s_])[cells]
        if not hit.any():
            continue
        f0 = side[cells]
        f1 = f0 + nrm @ LINKS[q].astype(np.float64)
        delta[q, hit] = (f0 / (f0 - f1))[hit]
        for a in range(3):
            uw[a, q, hit] = velocity[a]
    rho = np.where(solid, 1.0, w.rho)
    fill = np.where(solid, 0.0, w.fill)
    u = None if w.u is None else np.where(solid[None, :], 0.0, w.u)
    return Workload(name=name or (w.name + "_obstacle"), params=p, flags=flags, rho=rho, u=u, fill=fill,
                    meta=dict(w.meta), walls={"cells": cells, "delta": delta, "uw": uw})


def _area_below_line(slope: float, c: float, i: int, k: int) -> float:
    """Exact area of the unit square [i, i+1] x [k, k+1] below z = slope x + c
    (the clipped height is piecewise linear in x: trapezoids between kinks)."""
    def h(x):
        return min(max(slope * x + c - k, 0.0), 1.0)
    pts = [float(i), float(i + 1)]
    if slope != 0.0:
        pts += [xb for xb in ((k - c) / slope, (k + 1 - c) / slope) if i < xb < i + 1]
    pts.sort()
    return sum(0.5 * (h(a) + h(b)) * (b - a) for a, b in zip(pts[:-1], pts[1:]))


def skew_film(H: float = 8.0, slope: float = 0.25, tau: float = 2.0, g0: float = 1e-4, H0: float = 4.0,
              Lambda: float = 0.25, plic: int = 0, wall: float = 3.3, surface: bool = False) -> Workload:
    """Gravity-driven film on a wall rotated by atan(slope) against the lattice
    (the rotated planar film flow of section 4.3): a solid band below
    zeta = z - slope x = wall, a liquid film of normal thickness H above it,
    gas beyond; x, y, z periodic (nx = nz / slope, ny = 1); gravity
    g0 (H0/H)^3 along the wall (constant Reynolds number).  Exact fills of the
    plane surface; uniform density.  meta["profile"](n) is the steady
    half-Poiseuille velocity along the wall at normal distance n.

    surface=True: the surface held at its exact plane (params.hold) and given
    to the step (Workload.surface).  Cells are classed by where their node
    lies: a node below the plane is fluid, and a fluid node with a D3Q19
    neighbour beyond the plane is an interface (boundary) node -- the
    boundary node of section 2.2, whose boundary links meet the plane at
    0 <= delta <= 1."""
    ca = 1.0 / np.hypot(1.0, slope)
    hz = H / ca
    nz = int(np.ceil(wall + hz + max(6.0, hz))) + 1
    nx = int(round(nz / slope))
    g = g0 * (H0 / H) ** 3
    t = np.array([1.0, 0.0, slope]) * ca
    p = Params(nx=nx, ny=1, nz=nz, periodic=(1, 1, 1), tau=tau, Lambda=Lambda, g=tuple(g * t), plic=plic)
    types3, walls, zeta = skew_strips(nx, 1, nz, slope, ((wall, "solid", 0.0), (float(nz), "fluid", 0.0)), p)
    solid = types3[:, 0, :] == SOLID
    fill = np.zeros((nz, nx))
    for k in range(nz):
        for i in range(nx):
            if solid[k, i] or zeta[k, i] < wall:
                continue
            base = (k + 0.5 - slope * (i + 0.5)) - zeta[k, i]      # the periodic image of the bands
            fill[k, i] = _area_below_line(slope, wall + hz + base, i, k)
    if surface:
        p = dataclasses.replace(p, hold=1)
        below = (zeta < wall + hz) & ~solid            # node below the plane
        cls = np.where(below, LIQUID, GAS).astype(np.uint8)
        cls[solid] = SOLID
        fill = np.where(below, np.maximum(fill, 0.5), 0.0)
    else:
        cls = np.where(fill >= 1.0, LIQUID, np.where(fill <= 0.0, GAS, INTERFACE)).astype(np.uint8)
        cls[solid] = SOLID
    t3 = cls[:, None, :].copy()
    promote = (t3 == LIQUID) & _shift_any(t3 == GAS, p.periodic)
    t3[promote] = INTERFACE
    if surface:
        fill[(t3[:, 0, :] == LIQUID)] = 1.0
    N = p.n_cells
    surf = None
    if surface:
        nrm = np.array([-slope, 0.0, 1.0]) * ca
        off = (wall + hz - zeta) * ca                   # plane above the node: positive
        surf = {"normal": np.repeat(nrm[:, None], N, axis=1),
                "offset": np.broadcast_to(off[:, None, :], (nz, 1, nx)).reshape(-1).copy()}
    nu = (tau - 0.5) / 3.0
    zflat = np.broadcast_to(zeta[:, None, :], (nz, 1, nx)).reshape(-1)
    return Workload(name="skew_film", params=p, flags=t3.reshape(-1), rho=np.full(N, p.rho_gas), u=None,
                    fill=fill[:, None, :].reshape(-1), walls=walls, surface=surf,
                    meta={"H": H, "slope": slope, "g": g, "nu": nu, "tangent": t,
                          "normal_dist": (zflat - wall) * ca,
                          "profile": lambda n, Hr=H: g / nu * (Hr * n - n * n / 2.0)})


# Named configurations (sizes of the measured workloads).
def config(name: str, seed: int = 0) -> Workload:
    if name == "channel":
        return channel()
    if name.startswith("sweep"):
        return channel_sweep(int(name[len("sweep"):]))
    if name == "slosh256":
        return sloshing(256, 160, 256, depth=96.0, amp=6.0, seed=seed)
    if name == "slosh512":
        return sloshing(512, 320, 512, depth=192.0, amp=12.0, seed=seed)
    if name == "slosh128":
        return sloshing(128, 96, 128, depth=48.0, amp=3.0, seed=seed)
    raise KeyError(name)
