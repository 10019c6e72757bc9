"""fslbm_init_static (the context workspace in the library's static device
array, no device allocation) against fslbm_init (the caller's workspace):
identical results on two contexts in a row, the second on a smaller lattice
(the array keeps the first context's contents); the size limit and the
one-context-per-device rule are refused with their statuses."""
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


def _same(a, b, tag):
    fa = a.fields(("f", "flags", "mass", "phi"))
    fb = b.fields(("f", "flags", "mass", "phi"))
    assert (fa["flags"] == fb["flags"]).all(), tag
    for k in ("f", "mass", "phi"):
        assert np.array_equal(fa[k], fb[k]), f"{tag}: {k} differs"
    ca, cb = a.conversions(), b.conversions()
    for k in ca:
        np.testing.assert_array_equal(ca[k], cb[k], err_msg=f"{tag}: list {k}")
    sa, sb = a.stats(), b.stats()
    # the FP64 mass total is summed by atomics across blocks (the order of the
    # additions varies run to run): equal to rounding, the rest exactly
    ma, mb = sa.pop("total_mass"), sb.pop("total_mass")
    assert abs(ma - mb) <= 1e-13 * abs(ma), tag
    assert sa == sb, tag


@pytest.mark.parametrize("precision", ["fp64", "fp16s"])
def test_static_workspace_matches_caller_workspace(fs, precision):
    cases = [W.sloshing(48, 32, 16, depth=14.0, amp=4.0, amp_z=1.5, seed=1, gy=-4e-4, tau=0.6),
             W.sloshing(24, 18, 6, depth=8.0, amp=2.5, seed=2, gy=-4e-4, tau=0.6)]
    for w in cases:
        p = w.params
        _say(f"case static workspace {precision} {p.nx}x{p.ny}x{p.nz}")
        a = fs.Sim.from_workload(w, precision=precision)
        b = fs.Sim.from_workload(w, precision=precision, static_workspace=True)
        assert b.ws is None
        conv = 0
        for _ in range(6):
            a.step(10, fs.FSL)
            b.step(10, fs.FSL)
            conv += sum(v.size for v in a.conversions().values())
            _same(a, b, f"{p.nx}x{p.ny}x{p.nz}")
        assert conv > 0  # the conversion lists and epochs in the array were exercised
        b.close()
        a.close()


def test_static_workspace_limits(fs):
    w = W.sloshing(24, 18, 6, depth=8.0, amp=2.5, seed=2, gy=-4e-4, tau=0.6)
    b = fs.Sim.from_workload(w, static_workspace=True)
    with pytest.raises(fs.FslbmError, match="held by another context") as e:
        fs.Sim(w.params, w.flags, static_workspace=True)
    assert e.value.status == 1
    b.close()
    c = fs.Sim.from_workload(w, static_workspace=True)   # released by destroy
    c.step(5, fs.FSL)
    c.close()
    big = W.Params(nx=128, ny=96, nz=128)               # 1.57 M cells: about 120 MB of workspace
    with pytest.raises(fs.FslbmError, match="static workspace") as e:
        fs.Sim(big, np.zeros(big.n_cells, np.uint8), static_workspace=True)
    assert e.value.status == 6
