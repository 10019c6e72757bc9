"""The oracle on dual numbers: exact directional derivatives of a frozen-class
window, the reference for the adjoint.

Pins (nothing here uses the GPU library):
- the value part of a dual run is the plain FP64 oracle run, bit for bit
  (frozen classes, same T steps);
- the derivative part matches central finite differences of the FP64 oracle
  along the same direction, for initial populations, mass, fill, the gas
  density and each component of g, with FSK and FSL.  Steps are small enough
  that every run takes the same branches (delta clamps, FSK fallbacks): the
  finite difference is then accurate to O(h^2).
- a direction of zero gives a derivative of zero; the derivative is linear in
  the direction.
"""
import dataclasses

import numpy as np
import pytest

from paper_1409_5645_amd import workloads as W


@pytest.fixture(scope="module")
def case(oracle_mod):
    # 3-D surface (normals with all three components), driven out of rest
    w = W.sloshing(16, 14, 10, depth=7.0, amp=1.5, amp_z=1.0, seed=3, gy=-2e-4, tau=0.7)
    o = oracle_mod.Oracle.from_workload(w)
    o.step(40, oracle_mod.FSL)
    st = {"f": o.populations(), "mass": o.mass(), "phi": o.phi(), "flags": o.flags()}
    N = w.params.n_cells
    rng = np.random.default_rng(0)
    ut = rng.normal(0.0, 1e-3, (3, N))
    pt = rng.uniform(0.0, 1.0, N)
    return w.params, st, ut, pt


T = 20

# The random directions of the tests below: slot k holds the shapes ("f": the
# population array, "n": one value per cell) that test k draws.  Each test
# replays the draws of seed 0 up to its own, so its directions do not depend on
# which other tests ran before it in the same process.
_DRAWS = [("f",), ("f",), ("n", "n"), ("n", "n"), ("f", "f"), ("f", "f"), ("f", "f")]


def _rng(st, slot):
    N = st["flags"].size
    shape = {"f": st["f"].shape, "n": (N,)}
    rng = np.random.default_rng(0)
    rng.normal(0.0, 1e-3, (3, N))
    rng.uniform(0.0, 1.0, N)
    for k in range(slot):
        for d in _DRAWS[k]:
            rng.normal(0.0, 1.0, shape[d])
    return rng


def _L(oracle_mod, p, st, ut, pt, rule, f=None, m=None, phi=None):
    L, _ = oracle_mod.window_dual(p, st["flags"], st["f"] if f is None else f, st["mass"] if m is None else m,
                                  st["phi"] if phi is None else phi, ut, pt, T, rule)
    return L


@pytest.mark.parametrize("rule", [0, 1])
def test_value_part_is_the_fp64_oracle(oracle_mod, case, rule):
    p, st, ut, pt = case
    _, _, fin = oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, pt, T, rule,
                                       drho_b=1.0, dg=[0.3, -1.0, 0.2], want_state=True)
    o = oracle_mod.Oracle(p, state=dict(st, reservoir=0.0))
    o.set_freeze(True)
    o.step(T, rule)
    act = st["flags"] != W.GAS
    np.testing.assert_array_equal(fin["f"][:, act], o.populations()[:, act])
    it = st["flags"] == W.INTERFACE
    np.testing.assert_array_equal(fin["mass"][it], o.mass()[it])
    np.testing.assert_array_equal(fin["phi"][it], o.phi()[it])


@pytest.mark.parametrize("rule", [0, 1])
def test_populations_direction_vs_central_difference(oracle_mod, case, rule):
    p, st, ut, pt = case
    rng = _rng(st, rule)
    d = rng.normal(0.0, 1.0, st["f"].shape) * (st["flags"] != W.GAS)
    _, dL = oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, pt, T, rule, df0=d)
    h = 1e-6
    fd = (_L(oracle_mod, p, st, ut, pt, rule, f=st["f"] + h * d) -
          _L(oracle_mod, p, st, ut, pt, rule, f=st["f"] - h * d)) / (2 * h)
    assert abs(fd - dL) <= 1e-6 * abs(dL), (fd, dL)


@pytest.mark.parametrize("rule", [0, 1])
def test_mass_and_fill_direction_vs_central_difference(oracle_mod, case, rule):
    p, st, ut, pt = case
    rng = _rng(st, 2 + rule)
    it = st["flags"] == W.INTERFACE
    dphi = rng.normal(0.0, 1.0, it.size) * it
    dm = rng.normal(0.0, 1.0, it.size) * it
    _, dL = oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, pt, T, rule,
                                   dm0=dm, dphi0=dphi)
    h = 1e-6
    fd = (_L(oracle_mod, p, st, ut, pt, rule, m=st["mass"] + h * dm, phi=st["phi"] + h * dphi) -
          _L(oracle_mod, p, st, ut, pt, rule, m=st["mass"] - h * dm, phi=st["phi"] - h * dphi)) / (2 * h)
    assert abs(fd - dL) <= 1e-6 * abs(dL), (fd, dL)


@pytest.mark.parametrize("rule", [0, 1])
def test_gas_density_vs_central_difference(oracle_mod, case, rule):
    p, st, ut, pt = case
    _, dL = oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, pt, T, rule, drho_b=1.0)
    h = 1e-5 * p.rho_gas
    Lp = oracle_mod.window_dual(dataclasses.replace(p, rho_gas=p.rho_gas + h), st["flags"], st["f"], st["mass"],
                                st["phi"], ut, pt, T, rule)[0]
    Lm = oracle_mod.window_dual(dataclasses.replace(p, rho_gas=p.rho_gas - h), st["flags"], st["f"], st["mass"],
                                st["phi"], ut, pt, T, rule)[0]
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - dL) <= 1e-5 * abs(dL), (fd, dL)


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_body_force_vs_central_difference(oracle_mod, case, rule, axis):
    p, st, ut, pt = case
    dg = np.zeros(3)
    dg[axis] = 1.0
    _, dL = oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, pt, T, rule, dg=dg)
    h = 1e-7  # |g| = 2e-4; the loss is O(50), so a smaller step is rounding-limited
    gp, gm = list(p.g), list(p.g)
    gp[axis] += h
    gm[axis] -= h
    Lp = oracle_mod.window_dual(dataclasses.replace(p, g=tuple(gp)), st["flags"], st["f"], st["mass"], st["phi"],
                                ut, pt, T, rule)[0]
    Lm = oracle_mod.window_dual(dataclasses.replace(p, g=tuple(gm)), st["flags"], st["f"], st["mass"], st["phi"],
                                ut, pt, T, rule)[0]
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - dL) <= 1e-5 * abs(dL), (fd, dL)


def test_derivative_is_linear_in_the_direction(oracle_mod, case):
    p, st, ut, pt = case
    rng = _rng(st, 4)
    act = st["flags"] != W.GAS
    d1 = rng.normal(0.0, 1.0, st["f"].shape) * act
    d2 = rng.normal(0.0, 1.0, st["f"].shape) * act
    run = lambda **kw: oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, pt, T, 1,  # noqa
                                               **kw)[1]
    a, b = run(df0=d1, drho_b=0.5), run(df0=d2, dg=[0.0, 2.0, 0.0])
    c = run(df0=d1 + d2, drho_b=0.5, dg=[0.0, 2.0, 0.0])
    assert abs(c - (a + b)) <= 1e-9 * (abs(a) + abs(b))
    assert run() == 0.0


def test_linear_population_term_vs_central_difference(oracle_mod, case):
    p, st, ut, pt = case
    rng = _rng(st, 5)
    act = st["flags"] != W.GAS
    a = rng.normal(0.0, 1.0, st["f"].shape) * act
    d = rng.normal(0.0, 1.0, st["f"].shape) * act
    run = lambda f, **kw: oracle_mod.window_dual(p, st["flags"], f, st["mass"], st["phi"], ut, pt, T, 1,  # noqa
                                                  f_weight=a, **kw)
    L0, dL = run(st["f"], df0=d)
    L1 = oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, pt, T, 1)[0]
    assert L0 != L1
    h = 1e-6
    fd = (run(st["f"] + h * d)[0] - run(st["f"] - h * d)[0]) / (2 * h)
    assert abs(fd - dL) <= 1e-6 * abs(dL), (fd, dL)


def test_linear_term_alone(oracle_mod, case):
    """Without targets the loss is the linear functional alone: its derivative
    along d equals that of the full loss minus that of the interface term."""
    p, st, ut, pt = case
    rng = _rng(st, 6)
    act = st["flags"] != W.GAS
    a = rng.normal(0.0, 1.0, st["f"].shape) * act
    d = rng.normal(0.0, 1.0, st["f"].shape) * act
    run = lambda u, ph, fw: oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], u, ph,  # noqa
                                                    T, 1, df0=d, f_weight=fw)[1]
    lin, full, inter = run(None, None, a), run(ut, pt, a), run(ut, pt, None)
    assert abs(lin - (full - inter)) <= 1e-9 * (abs(full) + abs(inter))


def test_dual_window_refuses_what_it_does_not_differentiate(oracle_mod, case):
    """The exact derivative covers rules 0 and 1 without PLIC, surface tension
    or solid cells (as the GPU window does); anything else is refused."""
    import dataclasses
    p, st, ut, pt = case
    args = (st["flags"], st["f"], st["mass"], st["phi"], ut, pt, 2)
    for rule in (2, 3, 4, 5):
        with pytest.raises(ValueError, match="rules 0 and 1"):
            oracle_mod.window_dual(p, *args, rule)
    with pytest.raises(ValueError, match="PLIC"):
        oracle_mod.window_dual(dataclasses.replace(p, plic=1), *args, 1)
    with pytest.raises(ValueError, match="surface tension"):
        oracle_mod.window_dual(dataclasses.replace(p, sigma=1e-3), *args, 1)
    fl = st["flags"].copy()
    fl[0] = W.SOLID
    with pytest.raises(ValueError, match="solid"):
        oracle_mod.window_dual(p, fl, *args[1:], 1)
