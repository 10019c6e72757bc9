"""Pins of the oracle's shear-rate boundary term (rules with D != 0).

Section 3.4 builds the boundary value of Eq. (bterm), D c_a c_b S^b_ab, from a
shear rate S extrapolated from the bulk and projected with the surface normal
(Eq. proj1, proj2, Table 1 column D).  The pieces are pinned against what the
mathematics fixes; the whole rule against states whose boundary shear is zero
(a pool at rest, the half-Poiseuille film), where it must agree with D = 0.
"""
import math

import numpy as np
import pytest

from paper_1409_5645_amd import workloads as W
from tests.d3q19 import C

W_Q = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def _full(S6):
    S = np.empty((3, 3))
    for i, (a, b) in enumerate(PAIRS):
        S[a, b] = S[b, a] = S6[i]
    return S


def _tiny(mod, tau, incompressible, g):
    p = W.Params(nx=2, ny=2, nz=2, periodic=(1, 1, 1), tau=tau, Lambda=3.0 / 16.0, g=tuple(g),
                 incompressible=incompressible)
    return mod.Oracle(p, np.full(8, 2, np.uint8), np.ones(8), None, np.ones(8))


@pytest.mark.parametrize("incompressible", [1, 0])
def test_shear_recovered_from_chapman_enskog_populations(oracle_mod, incompressible):
    """Eq. (nqp) at leading order: n+_q = (1/lambda_+)(w_q/c_s^2) c_q c_q : S.
    Populations built as e+(rho, u) + e-(rho_0, u + g/2) + (1 + lambda_+) n+
    (the rest population keeping the mass) must give back S, for any symmetric
    S, density, velocity, force and relaxation time."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        tau = 0.52 + 1.5 * rng.random()
        g = rng.normal(0, 1e-4, 3)
        o = _tiny(oracle_mod, tau, incompressible, g)
        lp = -1.0 / tau
        rho = 1.0 + 0.1 * rng.normal()
        rho0 = 1.0 if incompressible else rho
        u = rng.normal(0, 0.03, 3)           # velocity the oracle recovers: (j/rho0 - g) + g/2
        ue = u + 0.5 * g                      # momentum carried by e-
        S = _full(rng.normal(0, 1e-3, 6))
        cu = C @ u
        ep = W_Q * (rho + rho0 * (4.5 * cu ** 2 - 1.5 * (u @ u)))
        em = 3 * W_Q * rho0 * (C @ ue)
        nplus = (1 / lp) * 3 * W_Q * np.einsum("qa,ab,qb->q", C, S, C)
        nplus[0] -= nplus.sum()               # the rest link carries no shear; mass unchanged
        own = ep + em + (1 + lp) * nplus
        got = _full(o.shear(own))
        assert np.abs(got - S).max() <= 1e-10 * np.abs(S).max()


def test_boundary_shear_projection(oracle_mod):
    """Section 3.4: in a basis {t1, t2, n}, S^b keeps the tangential block of S,
    has zero tangential-normal entries (Eq. proj2) and the given normal entry;
    the result does not depend on the choice of t1, t2."""
    rng = np.random.default_rng(9)
    for _ in range(50):
        S6 = rng.normal(size=6)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        snn = rng.normal()
        Sb = _full(oracle_mod.boundary_shear(S6, n, snn))
        S = _full(S6)
        t1 = np.cross(n, rng.normal(size=3))
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(n, t1)
        assert abs(n @ Sb @ n - snn) < 1e-13
        for t in (t1, t2):
            assert abs(t @ Sb @ n) < 1e-13
            for s in (t1, t2):
                assert abs(t @ Sb @ s - t @ S @ s) < 1e-13
        assert np.abs(Sb - Sb.T).max() == 0.0
    # axis-aligned normal: the entries can be read off
    S6 = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    np.testing.assert_allclose(oracle_mod.boundary_shear(S6, [0.0, 1.0, 0.0], 7.0), [1, 7, 3, 0, 5, 0], atol=1e-15)


@pytest.mark.parametrize("level", [30.5, 30.83])
def test_stress_rule_keeps_pool_at_rest(oracle_mod, level):
    """A hydrostatic pool has no shear, so the boundary shear vanishes and the
    rule with D != 0 keeps the pool at rest to round-off, like D = 0."""
    w = W.pool(nx=12, ny=40, nz=12, level=level)
    o = oracle_mod.Oracle.from_workload(w)
    M0 = o.total_mass()
    o.step(300, oracle_mod.FSL_STRESS)
    _, u = o.macro()
    act = w.flags != W.GAS
    assert np.abs(u[:, act]).max() < 1e-13
    np.testing.assert_array_equal(o.flags(), w.flags)
    assert abs(o.total_mass() - M0) / M0 < 1e-13


def _film(mod, h, frac, rule, stokes):
    tau, Lam = 0.8, 3 / 16
    w = W.channel(h=h + frac, nx=1, ny=h + 4, nz=1, gx=1e-6 * (32.0 / h) ** 3, tau=tau, Lambda=Lam,
                  stokes=stokes)
    o = mod.Oracle.from_workload(w)
    nu = (tau - 0.5) / 3.0
    H = h + frac
    o.step(int(34 * 4 * H * H / (math.pi ** 2 * nu)), rule)
    _, u = o.macro()
    y = np.arange(h + 4) + 0.5
    act = w.flags != W.GAS
    return u[0][act], y[act], w.params.g[0] / nu


def _l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


@pytest.mark.parametrize("frac", [0.5, 0.83])
def test_stress_rule_keeps_film_exact(oracle_mod, frac):
    """The half-Poiseuille film has zero shear at its flat surface except the
    tangential-normal entry, which Eq. (proj2) sets to zero: the boundary shear
    vanishes.  With the linear (Stokes) equilibrium the bulk non-equilibrium is
    exactly Eq. (nqp) and FSL with D != 0 reproduces the film as exactly as FSL;
    FSK with D != 0 keeps FSK's film of height h + 1 (Eq. fsfit)."""
    h = 8
    ux, y, gn = _film(oracle_mod, h, frac, oracle_mod.FSL_STRESS, 1)
    assert _l2(ux, gn * ((h + frac) * y - y * y / 2)) < 1e-11
    ux, y, gn = _film(oracle_mod, h, 0.5, oracle_mod.FSK_STRESS, 1)
    assert _l2(ux, gn * ((h + 1) * y - y * y / 2)) < 1e-11


@pytest.mark.parametrize("frac", [0.5, 0.83])
def test_stress_rule_film_with_quadratic_equilibrium(oracle_mod, frac):
    """With the quadratic equilibrium Eq. (nqp) misses the Lambda_- d_q^2 Pi_q
    term of Eq. (ce), so the bulk estimate of S carries small spurious normal
    entries: the film stays within 2e-6 of the exact profile (FSK: 1e-2)."""
    h = 8
    ux, y, gn = _film(oracle_mod, h, frac, oracle_mod.FSL_STRESS, 0)
    assert _l2(ux, gn * ((h + frac) * y - y * y / 2)) < 2e-6


def test_stress_term_changes_a_sheared_surface(oracle_mod):
    """Where the surface is sheared along its tangent plane, the D term is not
    zero: a sloshing tank departs from D = 0 (mass conserved either way)."""
    w = W.sloshing(16, 14, 10, depth=7.0, amp=1.5, amp_z=1.0, seed=3, gy=-2e-4, tau=0.7)
    a = oracle_mod.Oracle.from_workload(w)
    b = oracle_mod.Oracle.from_workload(w)
    M0 = a.total_mass() + a.reservoir()
    a.step(60, oracle_mod.FSL)
    b.step(60, oracle_mod.FSL_STRESS)
    fa, fb = a.populations(), b.populations()
    assert np.abs(fa - fb).max() > 1e-9
    assert abs(b.total_mass() + b.reservoir() - M0) / M0 < 1e-13
