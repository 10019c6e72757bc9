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


def _case():
    return W.sloshing(24, 18, 6, depth=8.0, amp=2.5, seed=2, gy=-4e-4, tau=0.6)


def _first(flags, cls):
    return int(np.nonzero(flags == cls)[0][len(np.nonzero(flags == cls)[0]) // 2])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_nan_population_is_unstable(fs, oracle_mod, precision):
    w = _case()
    _say(f"case nan {precision}")
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


def test_liquid_next_to_gas_breaks_the_layer_rule(fs):
    w = _case()
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
