"""Pins of the serial FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it relies on.  None of them re-types the oracle's
formulas: they check moments, matching conditions, exact steady states,
convergence orders, conservation, symmetry and hand-computed conversions.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1409_5645_amd import workloads as W
from tests.d3q19 import C, opposite, index_of

HERE = os.path.dirname(os.path.abspath(__file__))


def _oracle(mod, w):
    return mod.Oracle.from_workload(w)


def _tiny(mod, g=(0.0, 0.0, 0.0), tau=0.8, Lambda=3.0 / 16.0, incompressible=1):
    p = W.Params(nx=2, ny=2, nz=2, periodic=(1, 1, 1), tau=tau, Lambda=Lambda, g=g,
                 incompressible=incompressible)
    N = 8
    return mod.Oracle(p, np.full(N, 2, np.uint8), np.ones(N), None, np.ones(N))


# ---------------------------------------------------------------- lattice / equilibrium
@pytest.mark.parametrize("incompressible", [1, 0])
def test_equilibrium_moments(oracle_mod, incompressible):
    """Eq. (eqEven), (eqOdd), (density), (momentum): sum e = rho, sum c e =
    rho_0 u, sum c c e+ = (rho/3) I + rho_0 u u  (w_q of Qian et al., c_s^2 = 1/3)."""
    o = _tiny(oracle_mod, incompressible=incompressible)
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        e = o.equilibrium_post(rho, u)  # g = 0: a plain equilibrium
        rho0 = 1.0 if incompressible else rho
        assert abs(e.sum() - rho) < 1e-14
        np.testing.assert_allclose(C.T @ e, rho0 * u, atol=1e-15)
        Pi = np.einsum("qa,qb,q->ab", C, C, e)
        np.testing.assert_allclose(Pi, rho / 3.0 * np.eye(3) + rho0 * np.outer(u, u), atol=1e-14)
        # even/odd structure
        ep = 0.5 * (e + e[[opposite(q) for q in range(19)]])
        np.testing.assert_allclose(ep.sum(), rho, atol=1e-14)


def test_rest_equilibrium_weights(oracle_mod):
    """At u = 0 the equilibrium is w_q rho with w = 1/3, 1/18, 1/36 (section 2.1)."""
    o = _tiny(oracle_mod)
    e = o.equilibrium_post(1.3, np.zeros(3))
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    np.testing.assert_allclose(e, 1.3 * w, rtol=1e-15)


def test_collision_relaxation_rates(oracle_mod):
    """Eq. (lbe2): a pure even non-equilibrium relaxes by (1+lambda_+), a pure odd
    one by (1+lambda_-), with lambda_+ = -1/tau and Lambda_+ Lambda_- = Lambda
    (section 3.1).  Non-equilibria chosen in the kernel of the conserved moments."""
    tau, Lam = 0.7, 0.25
    o = _tiny(oracle_mod, tau=tau, Lambda=Lam)
    lp = -1.0 / tau
    Lp = -(0.5 + 1.0 / lp)
    Lm = Lam / Lp
    lm = -1.0 / (Lm + 0.5)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    n_even = w * (C[:, 0] ** 2 - 1.0 / 3.0)                  # traceless, symmetric
    n_odd = w * C[:, 0] * (C[:, 1] ** 2 - 1.0 / 3.0)         # zero first moment
    assert abs(n_even.sum()) < 1e-16 and np.abs(C.T @ n_odd).max() < 1e-16
    rho, u = 1.02, np.array([0.01, -0.02, 0.005])
    e = o.equilibrium_post(rho, u)
    for n, rate in ((n_even, 1 + lp), (n_odd, 1 + lm)):
        f = e + 1e-3 * n
        out, r, uu = o.collide(f)
        np.testing.assert_allclose(out - e, rate * 1e-3 * n, atol=2e-16)
        assert abs(r - rho) < 1e-15
        np.testing.assert_allclose(uu, u, atol=1e-16)


@pytest.mark.parametrize("incompressible", [1, 0])
def test_collision_mass_and_force(oracle_mod, incompressible):
    """The collision conserves mass and adds F = rho_0 g to the momentum
    (u_eq = U - F/lambda_-, section 2.1)."""
    g = (1e-4, -2e-4, 3e-5)
    o = _tiny(oracle_mod, g=g, incompressible=incompressible)
    rng = np.random.default_rng(2)
    for _ in range(20):
        f = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12) * (1 + 0.05 * rng.standard_normal(19))
        out, rho, u = o.collide(f)
        rho0 = 1.0 if incompressible else rho
        assert abs(out.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ out - C.T @ f, rho0 * np.array(g), atol=1e-16)
        # u = U + g/2 with rho_0 U = sum c f (Eq. momentum)
        np.testing.assert_allclose(u, (C.T @ f) / rho0 + 0.5 * np.array(g), atol=1e-16)


# ------------------------------------------------------------ closure coefficients
def test_table1_golden(oracle_mod):
    """Table 1 rows and Eq. (fsli1)-(fsli4) at the printed points."""
    gold = json.load(open(os.path.join(HERE, "golden", "table1.json")))
    o = _tiny(oracle_mod)
    k = o.coeffs(0)
    np.testing.assert_array_equal(k, [gold["FSK"][n] for n in ("a0", "a0bar", "a1", "alpha_p", "C")])
    for pt in gold["FSL_points"]:
        tau = -1.0 / pt["lambda_p"]
        oo = _tiny(oracle_mod, tau=tau)
        k = oo.coeffs(1, 1.0, pt["delta"])
        np.testing.assert_allclose(k, [pt[n] for n in ("a0", "a0bar", "a1", "alpha_p", "C")], atol=1e-15)


def test_fsli_matching_conditions(oracle_mod):
    """Eq. (cl1)-(cl4): alpha_- = 0, beta_- = alpha_+ delta lambda_-, beta_+ =
    -alpha_+ Lambda_+ lambda_+, alpha_+ = 1 - a0 - a0bar - a1, for any delta and
    relaxation rates; the FSK row meets them at delta = 1/2 and equals Eq.
    (fsli) at alpha_+ = 2, delta = 1/2."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        tau = 0.51 + 2.0 * rng.random()
        Lam = 0.05 + rng.random()
        delta = rng.random()
        alpha = 0.5 + 1.5 * rng.random()
        o = _tiny(oracle_mod, tau=tau, Lambda=Lam)
        c = o.constants()
        lp, lm = c["lambda_p"], c["lambda_m"]
        Lp = -(0.5 + 1.0 / lp)
        for rule, al, de in ((1, alpha, delta), (0, 2.0, 0.5)):
            a0, a0b, a1, ap, Cc = o.coeffs(rule, al, de)
            assert abs(ap - (1 - a0 - a0b - a1)) < 1e-14                  # cl1
            assert abs(a0b - a0 - a1 - 1) < 1e-14                         # alpha_- = 0 (cl2)
            beta_m = (1 + lm) * a0b - (1 + lm) * a0 - a1 - 1
            assert abs(beta_m - ap * de * lm) < 1e-13                     # cl3
            beta_p = 1 - (1 + lp) * (a0 + a0b) - a1 - Cc
            assert abs(beta_p + ap * Lp * lp) < 1e-13                     # cl4
        np.testing.assert_allclose(o.coeffs(1, 2.0, 0.5), o.coeffs(0), atol=1e-15)


# -------------------------------------------------------------- exact steady states
def _film(oracle_mod, h, rule, frac=0.5, Lambda=3 / 16, tau=0.8, stokes=0, efolds=34):
    w = W.channel(h=h + frac, nx=1, ny=h + 4, nz=1, gx=1e-6 * (32.0 / h) ** 3, tau=tau,
                  Lambda=Lambda, stokes=stokes)
    o = _oracle(oracle_mod, w)
    nu = (tau - 0.5) / 3.0
    H = h + frac
    o.step(int(efolds * 4 * H * H / (math.pi ** 2 * nu)), rule)
    _, u = o.macro()
    y = np.arange(h + 4) + 0.5
    act = w.flags != W.GAS
    return w, o, u[0], y, act, nu


def _l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


@pytest.mark.parametrize("h,frac", [(8, 0.5), (16, 0.5), (8, 0.83), (16, 0.83)])
def test_fsl_steady_film_exact(oracle_mod, h, frac):
    """Section 4.3: FSL with S^b = 0 over a bounce-back bottom at the magic
    parametrisation Lambda = 3/16 reproduces the half-Poiseuille film
    u = (g/nu)(H y - y^2/2) without numerical error, for any film height."""
    w, o, ux, y, act, nu = _film(oracle_mod, h, oracle_mod.FSL, frac=frac)
    H = h + frac
    ua = w.params.g[0] / nu * (H * y - y * y / 2)
    assert _l2(ux[act], ua[act]) < 1e-11


@pytest.mark.parametrize("stokes", [1, 0])
def test_fsk_steady_film_is_shifted(oracle_mod, stokes):
    """Eq. (fsfit): FSK imposes the surface half a link beyond the boundary node
    (delta = 1/2), so its steady film is exact for the height h + 1 (the node of
    the interface row plus 1/2) and first order for the true height h + 1/2."""
    h = 8
    w, o, ux, y, act, nu = _film(oracle_mod, h, oracle_mod.FSK, stokes=stokes)
    g = w.params.g[0]
    assert _l2(ux[act], g / nu * ((h + 1) * y - y * y / 2)[act]) < 1e-11
    assert _l2(ux[act], g / nu * ((h + 0.5) * y - y * y / 2)[act]) > 1e-2


def test_convergence_orders(oracle_mod):
    """Sections 3.2, 3.3, 4.3: FSK converges at first order; FSL at second order
    once the bounce-back wall is not exact (Lambda = 1/4), in diffusive scaling
    g ~ h^-3."""
    errs = {}
    for rule, Lam in ((oracle_mod.FSK, 3 / 16), (oracle_mod.FSL, 1 / 4)):
        e = []
        for h in (8, 16):
            w, o, ux, y, act, nu = _film(oracle_mod, h, rule, Lambda=Lam, efolds=30)
            H = h + 0.5
            e.append(_l2(ux[act], (w.params.g[0] / nu * (H * y - y * y / 2))[act]))
        errs[rule] = math.log2(e[0] / e[1])
    assert 0.85 < errs[oracle_mod.FSK] < 1.15
    assert 1.75 < errs[oracle_mod.FSL] < 2.25


def _startup_series(y, t, g, nu, H, K=400):
    """Start-up of a film at rest: u(0) = 0, u_y(H) = 0 (separation of
    variables; the same family as Eq. (freeUniform))."""
    us = g / nu * (H * y - y * y / 2)
    for k in range(K):
        m = 2 * k + 1
        us = us - 16 * g * H * H / (nu * math.pi ** 3 * m ** 3) * np.sin(m * math.pi * y / (2 * H)) \
            * np.exp(-nu * m * m * math.pi ** 2 * t / (4 * H * H))
    return us


def test_channel_startup_at_3000_steps(oracle_mod):
    """Gravity-driven channel (8 x 48 x 8, g_x = 1e-6, tau = 0.8, film at 32.5)
    after 3000 steps against the start-up series: FSL tracks the true height,
    FSK the height shifted by half a cell."""
    w = W.channel()
    res = {}
    for rule in (oracle_mod.FSL, oracle_mod.FSK):
        o = _oracle(oracle_mod, w)
        o.step(3000, rule)
        _, u = o.macro()
        ux = u[0].reshape(8, 48, 8)
        assert np.ptp(ux[:, :33, :], axis=(0, 2)).max() < 1e-18   # uniform in x, z
        res[rule] = ux[0, :, 0]
    y = np.arange(48) + 0.5
    act = w.flags.reshape(8, 48, 8)[0, :, 0] != W.GAS
    sl = _startup_series(y, 3000, 1e-6, 0.1, 32.5)
    assert _l2(res[oracle_mod.FSL][act], sl[act]) < 5e-5
    assert _l2(res[oracle_mod.FSK][act], sl[act]) > 2e-3
    assert _l2(res[oracle_mod.FSK][act], _startup_series(y, 3000, 1e-6, 0.1, 33.0)[act]) < 5e-5


@pytest.mark.parametrize("level", [30.5, 30.83])
def test_hydrostatic_pool_stays_at_rest(oracle_mod, level):
    """A flat pool with a hydrostatic density profile is a steady state: FSL
    (linear interpolation of the pressure to the surface at delta = fill - 1/2,
    where the gas pressure P_b = rho_gas/3 holds) keeps it at rest to round-off;
    no cell changes class; mass is conserved."""
    w = W.pool(nx=12, ny=40, nz=12, level=level)
    o = _oracle(oracle_mod, w)
    M0 = o.total_mass()
    o.step(300, oracle_mod.FSL)
    _, u = o.macro()
    act = w.flags != W.GAS
    assert np.abs(u[:, act]).max() < 1e-13
    np.testing.assert_array_equal(o.flags(), w.flags)
    assert abs(o.total_mass() - M0) / M0 < 1e-13


def test_rest_state_any_geometry(oracle_mod):
    """Uniform rho = rho_b at rest with g = 0 is a fixed point of both rules for
    any surface shape: the closure coefficients sum to one (Eq. cl1 with
    alpha_+ e+ carrying the rest)."""
    w = W.sloshing(24, 20, 6, depth=10.0, amp=3.0, seed=4, gy=0.0, tau=0.7)
    for rule in (oracle_mod.FSK, oracle_mod.FSL):
        o = _oracle(oracle_mod, w)
        f0 = o.populations()
        o.step(20, rule)
        act = w.flags != W.GAS
        np.testing.assert_allclose(o.populations()[:, act], f0[:, act], atol=1e-15)
        np.testing.assert_array_equal(o.flags(), w.flags)


# ------------------------------------------------------- mass exchange / conversions
def _layer_invariant(flags3):
    """No liquid cell has a gas neighbour on the 18 links (walls excluded)."""
    nz, ny, nx = flags3.shape
    L = flags3 == W.LIQUID
    G = flags3 == W.GAS
    for c in C[1:]:
        dx, dy, dz = c
        a = L[max(0, -dz):nz - max(0, dz), max(0, -dy):ny - max(0, dy), max(0, -dx):nx - max(0, dx)]
        b = G[max(0, dz):nz - max(0, -dz) or None, max(0, dy):ny - max(0, -dy) or None,
              max(0, dx):nx - max(0, -dx) or None]
        if (a & b).any():
            return False
    return True


def test_sloshing_mass_conservation_and_invariants(oracle_mod):
    """Mass exchange is antisymmetric per link and conversions move excess mass
    exactly, so M = sum_L sum_q f + sum_I m + reservoir is constant to round-off;
    after every step no liquid cell touches gas and the conversion lists obey
    E' = E minus N(F), NI within N(F) and gas, NL within N(E') and liquid."""
    w = W.sloshing(40, 32, 6, depth=16.0, amp=3.0, seed=5, gy=-3e-4, tau=0.6)
    o = _oracle(oracle_mod, w)
    M0 = o.total_mass()
    shape = (6, 32, 40)
    seen = {k: 0 for k in ("F", "E", "E'", "NI", "NL")}
    prev = w.flags.copy()
    for it in range(200):
        o.step(1, oracle_mod.FSL)
        fl = o.flags()
        L = o.lists()
        for k in seen:
            seen[k] += len(L[k])
        assert set(L["E'"]) <= set(L["E"])
        assert np.all(prev[L["NI"]] == W.GAS) and np.all(fl[L["NI"]] == W.INTERFACE)
        assert np.all(prev[L["NL"]] == W.LIQUID) and np.all(fl[L["NL"]] == W.INTERFACE)
        assert np.all(fl[L["F"]] == W.LIQUID) and np.all(fl[L["E'"]] == W.GAS)
        if it % 20 == 0:
            assert _layer_invariant(fl.reshape(shape))
        prev = fl
    assert seen["F"] > 0 and seen["E'"] > 0 and seen["NI"] > 0 and seen["NL"] > 0
    assert abs(o.total_mass() - M0) / M0 < 1e-13


def _flat_film_state(oracle_mod, n=6, level=3.5):
    """Flat film at rest with g = 0, uniform density: every mass exchange term is
    exactly zero, so conversions can be computed by hand."""
    p = W.Params(nx=n, ny=n, nz=n, periodic=(1, 0, 1), tau=0.8, g=(0.0, 0.0, 0.0))
    w = W.pool(nx=n, ny=n, nz=n, level=level, gy=0.0)
    w.params = p
    o = _oracle(oracle_mod, w)
    return w, p, {"flags": w.flags.copy(), "f": o.populations(), "mass": o.mass(), "phi": o.phi()}


def _idx(x, y, z, n=6):
    return x + n * (y + n * z)


def test_hand_filled_cell(oracle_mod):
    """One interface cell pushed above (1+eps) rho: it becomes liquid, its five
    gas neighbours across the surface join the interface with the equilibrium of
    their interface neighbours, and its excess m - rho is split equally over its
    13 interface neighbours after conversion (8 in the surface row + 5 new)."""
    w, p, st = _flat_film_state(oracle_mod)
    c = _idx(2, 3, 2)
    st["mass"][c] = 1.5
    o = oracle_mod.Oracle(p, state=st)
    o.step(1, oracle_mod.FSL)
    L = o.lists()
    assert list(L["F"]) == [c] and len(L["E"]) == 0
    ni = sorted(_idx(2 + dx, 4, 2 + dz) for dx, dz in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)))
    assert list(L["NI"]) == ni and len(L["NL"]) == 0
    m = o.mass()
    fl = o.flags()
    assert fl[c] == W.LIQUID and all(fl[k] == W.INTERFACE for k in ni)
    share = 0.5 / 13
    for k in ni:
        assert m[k] == pytest.approx(share, abs=1e-16)
    for dx, dz in ((1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)):
        assert m[_idx(2 + dx, 3, 2 + dz)] == pytest.approx(0.5 + share, abs=1e-15)
    assert m[_idx(4, 3, 4)] == 0.5          # not a neighbour
    f = o.populations()
    w19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    for k in ni:
        np.testing.assert_allclose(f[:, k], w19, atol=1e-16)
    assert o.reservoir() == 0.0


def test_hand_emptied_cell_and_conflict(oracle_mod):
    """An interface cell below -eps rho empties: five liquid cells beneath join
    the interface with m = rho, and its (negative) mass is split over 13
    neighbours.  An emptied cell next to a filled one stays interface."""
    w, p, st = _flat_film_state(oracle_mod)
    e = _idx(2, 3, 2)
    st["mass"][e] = -0.5
    o = oracle_mod.Oracle(p, state=st)
    o.step(1, oracle_mod.FSL)
    L = o.lists()
    assert list(L["E"]) == [e] and list(L["E'"]) == [e]
    nl = sorted(_idx(2 + dx, 2, 2 + dz) for dx, dz in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)))
    assert list(L["NL"]) == nl
    m = o.mass()
    for k in nl:
        assert m[k] == pytest.approx(1.0 - 0.5 / 13, abs=1e-15)
    assert o.flags()[e] == W.GAS
    # conflict: filled neighbour protects the emptied cell
    w, p, st = _flat_film_state(oracle_mod)
    st["mass"][_idx(2, 3, 2)] = -0.5
    st["mass"][_idx(3, 3, 2)] = 1.5
    o = oracle_mod.Oracle(p, state=st)
    o.step(1, oracle_mod.FSL)
    L = o.lists()
    assert list(L["E"]) == [_idx(2, 3, 2)] and len(L["E'"]) == 0 and list(L["F"]) == [_idx(3, 3, 2)]
    assert o.flags()[_idx(2, 3, 2)] == W.INTERFACE


def test_orphan_excess_goes_to_reservoir(oracle_mod):
    """A filled cell with no interface neighbour after conversion hands its
    excess to the reservoir, keeping the mass total."""
    n = 5
    p = W.Params(nx=n, ny=n, nz=n, periodic=(1, 1, 1), tau=0.8)
    flags = np.full(n ** 3, W.LIQUID, np.uint8)
    c = _idx(2, 2, 2, n)
    flags[c] = W.INTERFACE
    fill = np.ones(n ** 3)
    fill[c] = 1.25
    o = oracle_mod.Oracle(p, flags, np.ones(n ** 3), None, fill)
    M0 = o.total_mass()
    o.step(1, oracle_mod.FSL)
    assert list(o.lists()["F"]) == [c]
    assert o.reservoir() == pytest.approx(0.25, abs=1e-15)
    assert o.total_mass() == pytest.approx(M0, abs=1e-13)
    assert (o.flags() == W.LIQUID).all()


# ------------------------------------------------------------------ symmetry
def test_axis_permutation_symmetry(oracle_mod):
    """The scheme is invariant under the lattice symmetry (x, y, z) -> (y, z, x):
    running a rotated tank gives the rotated result (catches wrong links, wrong
    normals and index slips in any one direction)."""
    w = W.sloshing(20, 16, 8, depth=8.0, amp=2.5, seed=6, gy=-3e-4, tau=0.6)
    nz, ny, nx = 8, 16, 20
    o1 = _oracle(oracle_mod, w)
    # rotated copy: new (x', y', z') = (y, z, x); arrays [z][y][x] -> [x][z][y]
    rot = lambda a: np.ascontiguousarray(a.reshape(nz, ny, nx).transpose(2, 0, 1)).reshape(-1)
    g = w.params.g
    p2 = W.Params(nx=ny, ny=nz, nz=nx, periodic=(0, 0, 0), tau=0.6, Lambda=w.params.Lambda,
                  g=(g[1], g[2], g[0]))
    o2 = oracle_mod.Oracle(p2, rot(w.flags), rot(w.rho), None, rot(w.fill))
    qmap = [index_of((c[1], c[2], c[0])) for c in C]
    for _ in range(3):
        o1.step(40, oracle_mod.FSL)
        o2.step(40, oracle_mod.FSL)
        f1, f2 = o1.populations(), o2.populations()
        fl1 = o1.flags()
        np.testing.assert_array_equal(rot(fl1), o2.flags())
        act = rot(fl1) != W.GAS
        for q in range(19):
            np.testing.assert_allclose(rot(f1[q])[act], f2[qmap[q]][act], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(rot(o1.mass())[rot(fl1) == 1], o2.mass()[rot(fl1) == 1], atol=1e-12)


def test_translation_symmetry_periodic(oracle_mod):
    """On a periodic box, shifting the input shifts the output bit for bit."""
    w = W.sloshing(16, 16, 6, depth=8.0, amp=2.5, seed=7, gy=-3e-4, tau=0.6, periodic=(1, 0, 1))
    p = w.params
    sh = lambda a: np.roll(a.reshape(6, 16, 16), (2, 5), axis=(0, 2)).reshape(-1)
    o1 = oracle_mod.Oracle(p, w.flags, w.rho, None, w.fill)
    o2 = oracle_mod.Oracle(p, sh(w.flags), sh(w.rho), None, sh(w.fill))
    o1.step(60, oracle_mod.FSL)
    o2.step(60, oracle_mod.FSL)
    np.testing.assert_array_equal(sh(o1.flags()), o2.flags())
    f1, f2 = o1.populations(), o2.populations()
    act = o2.flags() != W.GAS
    for q in range(19):
        np.testing.assert_array_equal(sh(f1[q])[act], f2[q][act])


def test_rejects_invalid_layer(oracle_mod):
    """A liquid cell adjacent to gas violates the interface layer: rejected."""
    p = W.Params(nx=4, ny=4, nz=4, periodic=(1, 1, 1))
    flags = np.full(64, W.LIQUID, np.uint8)
    flags[5] = W.GAS
    with pytest.raises(ValueError):
        oracle_mod.Oracle(p, flags, np.ones(64), None, np.ones(64))
