"""Pins of the oracle's solid walls with the linear-interpolation closure (CLI)
for the rotated channels of section 4.2.

The closure for a wall link at distance delta follows from the fitting
conditions of section 3.3 (Eq. fitting, cl1) with no pressure term and the
wall momentum matched to first order; it is exact for linear velocity
profiles.  Pins: plane Couette flow between walls at arbitrary distances
(aligned: from rest; rotated by atan(1/4): the exact state is a fixed point,
halfway bounce-back is not), a solid row at delta = 1/2 equal bit for bit to
the domain-face wall it replaces (free surface and moving wall included), rest
states, and the wall-table checks.
"""
import dataclasses

import numpy as np
import pytest

from paper_1409_5645_amd import workloads as W

WQ = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
C = W.LINKS.astype(np.float64)


def _aligned(bands, nz=16, nx=4):
    p = W.Params(nx=nx, ny=1, nz=nz, periodic=(1, 1, 1), tau=0.8, stokes=1)
    types3, walls, zeta = W.skew_strips(nx, 1, nz, 0.0, bands, p)
    fl = types3.reshape(-1)
    w = W.Workload("aligned", p, fl, np.ones(p.n_cells), None, np.where(fl == W.SOLID, 0.0, 1.0), walls=walls)
    return w, np.broadcast_to(zeta[:, None, :], (nz, 1, nx)).reshape(-1)


def _linear_profile(bands, zz):
    edges = [0.0] + [b[0] for b in bands]
    out = np.full(zz.shape, np.nan)
    for i, (hi, kind, _) in enumerate(bands):
        if kind == "fluid":
            lo = edges[i]
            ulo, uhi = bands[i - 1][2], bands[(i + 1) % len(bands)][2]
            out = np.where((zz >= lo) & (zz < hi), ulo + (uhi - ulo) * (zz - lo) / (hi - lo), out)
    return out


@pytest.mark.parametrize("bands", [
    ((3.0, "solid", 1e-3), (9.0, "fluid", 0.0), (11.0, "solid", 0.0), (16.0, "fluid", 0.0)),   # delta = 1/2
    ((3.3, "solid", 1e-3), (8.6, "fluid", 0.0), (11.2, "solid", 0.0), (16.0, "fluid", 0.0)),   # 0.2 / 0.8 / 0.3 / 0.7
    ((2.05, "solid", -2e-3), (9.95, "fluid", 0.0), (12.45, "solid", 1e-3), (16.0, "fluid", 0.0)),
])
def test_aligned_couette_exact_from_rest(oracle_mod, bands):
    """Between walls at any distance from the nodes, plane Couette flow with
    the linear equilibrium converges from rest to the exact linear profile."""
    w, zz = _aligned(bands)
    o = oracle_mod.Oracle.from_workload(w)
    o.step(3000, 1)
    rho, u = o.macro()
    fl = w.flags == W.LIQUID
    prof = _linear_profile(bands, zz)
    assert np.abs(u[0, fl] - prof[fl]).max() < 1e-12
    assert np.abs(u[1:, fl]).max() < 1e-14
    assert np.abs(rho[fl] - 1.0).max() < 1e-13


def _exact_state(w):
    """Post-collision populations of the exact rotated Couette flow: linear
    equilibrium plus (1 + lambda_+) n+ with n+_q = (w_q/c_s^2) c_q c_q : grad j
    / lambda_+ (Eq. nqp; exact for a linear velocity field)."""
    p = w.params
    t, s = w.meta["tangent"], w.meta["slope"]
    nvec = np.array([-s, 0.0, 1.0]) / np.hypot(1.0, s)
    zeta = w.meta["zeta"]
    u = w.meta["profile"](zeta)[None, :] * t[:, None]
    h = 1e-6
    dudn = (w.meta["profile"](zeta + h) - w.meta["profile"](zeta - h)) / (2 * h) * np.hypot(1.0, s)
    grad = nvec[:, None, None] * t[None, :, None] * dudn[None, None, :]
    lp = -1.0 / p.tau
    e = WQ[:, None] * (1.0 + 3.0 * (C @ np.nan_to_num(u)))
    npl = 3.0 * WQ[:, None] * np.einsum("qa,qb,abn->qn", C, C, np.nan_to_num(grad)) / lp
    ft = e + (1.0 + lp) * npl
    ft[:, w.flags == W.SOLID] = 0.0
    return {"flags": w.flags, "f": ft, "mass": np.zeros(p.n_cells), "phi": np.zeros(p.n_cells)}, u


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_rotated_couette_exact_state_is_kept(oracle_mod, tau):
    """Couette flow in a channel rotated by atan(1/4) (section 4.2): with the
    exact wall distances the exact state stays exact over 2000 steps; halfway
    bounce-back (delta = 1/2 on every wall link) drifts away by percent."""
    w = W.skew_couette(tau=tau)
    st, u = _exact_state(w)
    fl = w.flags == W.LIQUID
    o = oracle_mod.Oracle(w.params, state=st)
    o.set_walls(w.walls["cells"], w.walls["delta"], w.walls["uw"])
    o.step(2000, 1)
    rho, ug = o.macro()
    assert np.abs(ug[:, fl] - u[:, fl]).max() < 1e-12 * 1e3 * w.meta["U"]
    assert np.abs(rho[fl] - 1.0).max() < 1e-13
    bb = oracle_mod.Oracle(w.params, state=st)
    bb.set_walls(w.walls["cells"], None, w.walls["uw"])
    bb.step(2000, 1)
    _, ub = bb.macro()
    assert np.abs(ub[:, fl] - u[:, fl]).max() > 1e-2 * w.meta["U"]


def _with_solid_floor(w, u_floor):
    """The same film with its bottom wall face replaced by a row of solid
    cells (wall half a cell below the first fluid row, as before)."""
    p = w.params
    nx, ny, nz = p.nx, p.ny, p.nz
    p2 = dataclasses.replace(p, ny=ny + 1, wall_u=((0.0, 0.0, 0.0),) * 6)
    def lift(a, fillv):
        a3 = a.reshape(nz, ny, nx)
        out = np.full((nz, ny + 1, nx), fillv, dtype=a.dtype)
        out[:, 1:, :] = a3
        return out.reshape(-1)
    flags = lift(w.flags, W.SOLID)
    N2 = p2.n_cells
    idx = np.arange(N2)
    x, y, z = idx % nx, (idx // nx) % (ny + 1), idx // (nx * (ny + 1))
    cells = []
    for c in idx[flags != W.SOLID]:
        if y[c] == 1:
            cells.append(c)
    cells = np.array(cells, dtype=np.int32)
    uw = np.zeros((3, 19, cells.size))
    for q in range(1, 19):
        if W.LINKS[q][1] == -1:
            uw[:, q, :] = np.asarray(u_floor)[:, None]
    walls = {"cells": cells, "delta": np.full((19, cells.size), 0.5), "uw": uw}
    return W.Workload("solid_floor", p2, flags, lift(w.rho, 1.0), None, lift(w.fill, 0.0), walls=walls)


@pytest.mark.parametrize("rule", [1, 0, 3])
def test_solid_row_at_half_equals_wall_face(oracle_mod, rule):
    """A film dragged by its bottom wall, once with the wall face of the box and
    once with a row of solid cells moving at the same speed: populations, mass,
    fill and classes agree bit for bit over 120 steps (free surface above)."""
    uf = (1e-3, 0.0, 2e-4)
    w = W.channel(h=9.4, nx=6, ny=14, nz=5, gx=2e-6)
    w = dataclasses.replace(w, params=dataclasses.replace(
        w.params, wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), uf, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))))
    ws = _with_solid_floor(w, uf)
    a = oracle_mod.Oracle.from_workload(w)
    b = oracle_mod.Oracle.from_workload(ws)
    a.step(120, rule)
    b.step(120, rule)
    p = w.params
    keep = (np.arange(ws.params.n_cells) // p.nx) % (p.ny + 1) != 0
    assert np.array_equal(b.flags()[keep], a.flags())
    assert np.array_equal(b.populations()[:, keep], a.populations())
    assert np.array_equal(b.mass()[keep], a.mass())
    assert b.total_mass() == a.total_mass()


def test_rest_state_with_solids_is_kept(oracle_mod):
    """Resting walls and fluid at rest with uniform density: nothing moves."""
    w = W.skew_couette(U=0.0)
    o = oracle_mod.Oracle.from_workload(w)
    f0 = o.populations()
    o.step(50, 1)
    fl = w.flags == W.LIQUID
    assert np.abs(o.populations()[:, fl] - f0[:, fl]).max() < 1e-16


def test_wall_table_checks(oracle_mod):
    w = W.skew_couette()
    o = oracle_mod.Oracle(w.params, w.flags, w.rho, w.u, w.fill)
    with pytest.raises(RuntimeError, match="no wall table"):
        o.step(1, 1)
    c = w.walls["cells"]
    with pytest.raises(RuntimeError, match="exactly"):
        o.set_walls(c[1:], w.walls["delta"][:, 1:], w.walls["uw"][:, :, 1:])
    bad = w.walls["delta"].copy()
    q = int(np.argmin(np.where(bad == 0.5, 9.0, bad).min(axis=1)))
    bad[q, :] = np.where(bad[q, :] != 0.5, 1.5, bad[q, :])
    with pytest.raises(RuntimeError, match="outside"):
        o.set_walls(c, bad, w.walls["uw"])


def test_ramp_tank_mass(oracle_mod):
    """A converting tank over an inclined solid ramp: with halfway bounce-back
    on every wall link (delta = 1/2) mass is conserved to rounding; the
    interpolated closure is not mass-conserving (its drift is bounded here)."""
    w = W.sloshing(37, 24, 10, depth=11.0, amp=3.0, seed=11, gy=-4e-4, tau=0.6)
    w = W.add_plane_obstacle(w, (-0.3, 1.0, 0.12), 3.1)
    half = dataclasses.replace(w, walls={"cells": w.walls["cells"]})
    for wk, tol in ((half, 1e-13), (w, 1e-3)):
        o = oracle_mod.Oracle.from_workload(wk)
        M0 = o.total_mass() + o.reservoir()
        o.step(60, 1)
        assert abs((o.total_mass() + o.reservoir()) / M0 - 1.0) < tol
        assert (o.flags() == W.SOLID).sum() == (w.flags == W.SOLID).sum()


def _film_error(oracle_mod, H, rule, plic):
    w = W.skew_film(H=H, plic=plic)
    o = oracle_mod.Oracle.from_workload(w)
    o.step(int(8 * H * H / w.meta["nu"]) + 200, rule)
    _, u = o.macro()
    liq = o.flags() == W.LIQUID
    ut = (u * w.meta["tangent"][:, None]).sum(0)
    ue = w.meta["profile"](w.meta["normal_dist"])
    return np.sqrt(((ut[liq] - ue[liq]) ** 2).sum() / (ue[liq] ** 2).sum())


def test_rotated_film_fsl_beats_fsk(oracle_mod):
    """Rotated film flow (slope 1/4, section 4.3) at film thicknesses 4 and 8:
    FSL (with the PLIC plane and height-function normals) is several times more
    accurate than FSK and both errors fall with resolution.  With the
    interface tracking of the method the steady surface is not exactly plane
    (the paper's conclusion), so neither reaches second order here."""
    e = {(H, r): _film_error(oracle_mod, H, r, 2 if r == 1 else 0) for H in (4.0, 8.0) for r in (0, 1)}
    for H in (4.0, 8.0):
        assert e[(H, 1)] < 0.5 * e[(H, 0)]
    assert e[(8.0, 0)] < 0.6 * e[(4.0, 0)]
    assert e[(8.0, 1)] < 0.6 * e[(4.0, 1)]


def _held_film_error(oracle_mod, H, rule):
    w = W.skew_film(H=H, surface=True)
    o = oracle_mod.Oracle.from_workload(w)
    o.step(int(8 * H * H / w.meta["nu"]) + 200, rule)
    _, u = o.macro()
    liq = o.flags() == W.LIQUID
    it = w.flags == W.INTERFACE
    assert (o.flags() == w.flags).all() and np.array_equal(o.phi()[it], w.fill[it])   # held
    ut = (u * w.meta["tangent"][:, None]).sum(0)
    ue = w.meta["profile"](w.meta["normal_dist"])
    return np.sqrt(((ut[liq] - ue[liq]) ** 2).sum() / (ue[liq] ** 2).sum())


def test_rotated_film_second_order_with_the_surface_held(oracle_mod):
    """The rotated film of section 4.3 (slope 1/4, CLI wall, Lambda = 1/4,
    tau = 2, g proportional to H^-3 at constant Reynolds number) with the
    surface held at its exact plane: boundary nodes are the fluid nodes with a
    link to a node beyond the plane (section 2.2), their link distances come
    from the plane and the fills stay put.  Then FSL converges at second order
    (fitted over H = 4, 6, 8, 12, 16; measured 2.10) and FSK clearly below it
    (measured 0.58: FSK puts the surface half a link from the node whatever
    the plane, so its error depends on how the staircase falls)."""
    Hs = [4.0, 6.0, 8.0, 12.0, 16.0]
    order = {}
    err = {}
    for rule in (0, 1):
        e = [_held_film_error(oracle_mod, H, rule) for H in Hs]
        err[rule] = e
        order[rule] = -np.polyfit(np.log(Hs), np.log(e), 1)[0]
    assert 1.75 <= order[1] <= 2.25, order
    assert order[0] < 1.5, order
    assert err[1][-1] < 0.1 * err[0][-1]
    assert err[1][-1] < 3e-4
