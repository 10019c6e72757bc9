"""Health checks of the C-ABI (fslbm_stats, and fslbm_step with check_every):
failures are forced from the host through caller-owned data -- a NaN or a fast
cell in the initial state, a liquid cell written next to the gas into the
caller's flag buffer -- and each must come back as its status.  No kernel sees
an out-of-range index: the checks only read the state."""
import numpy as np
import pytest

from paper_1409_5645_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    from paper_1409_5645_amd import fslbm
    return fslbm


def _say(*a):
    print(*a, flush=True)


def _case(odd=False):
    # odd: N = 25 * 17 * 5 is odd, so the statistics take their one-cell-per-lane
    # kernel in every form (else the one with 16 bytes of each plane per lane)
    if odd:
        return W.sloshing(25, 17, 5, depth=8.0, amp=2.5, seed=2, gy=-4e-4, tau=0.6)
    return W.sloshing(24, 18, 6, depth=8.0, amp=2.5, seed=2, gy=-4e-4, tau=0.6)


def _first(flags, cls):
    return int(np.nonzero(flags == cls)[0][len(np.nonzero(flags == cls)[0]) // 2])


@pytest.mark.parametrize("odd", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_nan_population_is_unstable(fs, oracle_mod, precision, odd):
    w = _case(odd)
    _say(f"case nan {precision} odd={odd}")
    o = oracle_mod.Oracle.from_workload(w)
    f = o.populations().copy()
    c = _first(w.flags, W.LIQUID)
    f[3, c] = np.nan
    s = fs.Sim(w.params, w.flags, precision=precision)
    s.set_state(f, o.mass(), o.phi())
    with pytest.raises(fs.FslbmError, match="UNSTABLE") as e:
        s.stats()
    assert e.value.status == 4 and "1 cells with NaN" in str(e.value)
    s.close()
    # the same state under a check every 3 steps: the step call stops at step 3
    s = fs.Sim(w.params, w.flags, precision=precision, check_every=3)
    s.set_state(f, o.mass(), o.phi())
    with pytest.raises(fs.FslbmError, match="UNSTABLE") as e:
        s.step(10, fs.FSL)
    assert "after 3 steps" in str(e.value)
    s.close()


def test_fast_cell_is_unstable(fs):
    w = _case()
    _say("case fast cell")
    u = w.velocity().copy()
    c = _first(w.flags, W.LIQUID)
    u[0, c] = 0.45
    s = fs.Sim(w.params, w.flags)
    s.set_equilibrium(w.rho, u, w.fill)
    with pytest.raises(fs.FslbmError, match="UNSTABLE") as e:
        s.stats()
    assert "1 cells with |u| above 0.4" in str(e.value)
    s.close()
    s = fs.Sim(w.params, w.flags, u_max=0.5)
    s.set_equilibrium(w.rho, u, w.fill)
    st = s.stats()
    assert st["liquid"] == int((w.flags == W.LIQUID).sum())
    s.close()


@pytest.mark.parametrize("odd", [False, True])
def test_liquid_next_to_gas_breaks_the_layer_rule(fs, odd):
    w = _case(odd)
    _say("case layer rule")
    s = fs.Sim.from_workload(w)
    s.stats()
    nx, ny = w.params.nx, w.params.ny
    # an interface cell with a gas cell straight above it becomes liquid
    it = np.nonzero(w.flags == W.INTERFACE)[0]
    c = next(int(i) for i in it if w.flags[i + nx] == W.GAS)
    s.flags_t[c] = W.LIQUID
    with pytest.raises(fs.FslbmError, match="INVARIANT") as e:
        s.stats()
    assert e.value.status == 5 and "1 cells break the cell-class rule" in str(e.value)
    # an unknown class
    s.flags_t[c] = W.INTERFACE
    s.flags_t[_first(w.flags, W.GAS)] = 7
    with pytest.raises(fs.FslbmError, match="INVARIANT"):
        s.stats()
    s.close()


def test_checked_steps_equal_unchecked(fs):
    """A check after every step reads the state only: the populations after
    40 steps are bit-identical to a run without checks, and a healthy run
    passes every check."""
    w = _case()
    _say("case checked run")
    a = fs.Sim.from_workload(w)
    b = fs.Sim.from_workload(w, check_every=1)
    a.step(40, fs.FSL)
    b.step(40, fs.FSL)
    fa, fb = a.fields(("f", "flags")), b.fields(("f", "flags"))
    assert (fa["flags"] == fb["flags"]).all()
    assert np.array_equal(fa["f"], fb["f"])
    assert b.stats()["steps"] == 40
    a.close()
    b.close()


@pytest.mark.parametrize("nx,periodic", [(37, (0, 0, 0)), (37, (1, 0, 1)), (64, (0, 0, 0)), (64, (1, 1, 1))])
def test_layer_rule_count_matches_the_definition(fs, nx, periodic):
    """The count of liquid cells with a gas cell among their 18 neighbours
    (D3Q19 links; periodic faces wrap, walls give no neighbour), on a random
    class field written into the caller's flag buffer, equals the count taken
    straight from the definition with numpy: rows of 37 cells (chunks that
    end inside a row, unaligned rows) and of 64 (16-byte loads)."""
    w = W.sloshing(nx, 18, 6, depth=8.0, amp=2.5, seed=2, gy=-4e-4, tau=0.6, periodic=periodic)
    _say(f"case layer count nx={nx} periodic={periodic}")
    s = fs.Sim.from_workload(w)
    rng = np.random.default_rng(5)
    fl = rng.choice(np.array([W.GAS, W.INTERFACE, W.LIQUID], dtype=np.uint8), size=w.params.n_cells, p=[0.1, 0.3, 0.6])
    f3 = fl.reshape(w.params.nz, w.params.ny, nx)
    bad = np.zeros_like(f3, dtype=bool)
    for q in range(1, 19):
        cx, cy, cz = (int(v) for v in W.LINKS[q])
        nb = f3
        ok = np.ones_like(f3, dtype=bool)
        for ax, (c, per) in enumerate(((cz, periodic[2]), (cy, periodic[1]), (cx, periodic[0]))):
            if c == 0:
                continue
            nb = np.roll(nb, -c, axis=ax)
            if not per:
                idx = [slice(None)] * 3
                idx[ax] = slice(-1, None) if c > 0 else slice(0, 1)
                ok[tuple(idx)] = False
        bad |= ok & (nb == W.GAS)
    expect = int((bad & (f3 == W.LIQUID)).sum())
    assert expect > 0
    import torch
    # every cell liquid at rest first, so that the populations are sound
    # wherever the random field puts a fluid cell
    N = w.params.n_cells
    s.flags_t.fill_(W.LIQUID)
    s.set_equilibrium(np.ones(N), np.zeros((3, N)), np.ones(N))
    assert s.stats()["liquid"] == N
    s.flags_t.copy_(torch.from_numpy(fl).to(s.flags_t.device))
    with pytest.raises(fs.FslbmError, match="INVARIANT") as e:
        s.stats()
    assert f"{expect} cells break the cell-class rule" in str(e.value), (expect, str(e.value))
    s.close()


@pytest.mark.parametrize("odd", [False, True])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-6), ("fp16s", 1e-4)])
def test_total_mass_of_both_statistics_kernels(fs, oracle_mod, precision, tol, odd):
    """Total mass and class counts from fslbm_stats against the oracle at the
    initial state, through the kernel with 16 bytes of each plane per lane
    (N a multiple of 16 / s) and through the one-cell-per-lane kernel (odd N).
    The reduced forms recompute the liquid density from their stored
    populations, so they differ by the storage rounding."""
    w = _case(odd)
    _say(f"case stats mass {precision} odd={odd}")
    o = oracle_mod.Oracle.from_workload(w)
    s = fs.Sim.from_workload(w, precision=precision)
    st = s.stats()
    m0 = o.total_mass()
    err = abs(st["total_mass"] - m0) / m0
    _say(f"  total mass rel err {err:.2e}")
    assert err <= tol
    assert st["liquid"] == int((w.flags == W.LIQUID).sum())
    assert st["interface"] == int((w.flags == W.INTERFACE).sum())
    s.close()
