"""Pins of the seeded input generators shared by the oracle and the GPU
tests (host logic, no arithmetic of the method): reproducible from the seed,
the liquid volume equal to the integral of the surface height, and no liquid
cell next to gas in the initial classes."""
import math

import numpy as np

from paper_1409_5645_amd import workloads as W


def _liquid_next_to_gas(flags, shape, periodic):
    fl = flags.reshape(shape)
    L = fl == W.LIQUID
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if not 1 <= dx * dx + dy * dy + dz * dz <= 2:
                    continue
                g = fl == W.GAS
                for ax, d, per in ((2, dx, periodic[0]), (1, dy, periodic[1]), (0, dz, periodic[2])):
                    if d == 0:
                        continue
                    g = np.roll(g, -d, axis=ax)
                    if not per:
                        idx = [slice(None)] * 3
                        idx[ax] = -1 if d > 0 else 0
                        g[tuple(idx)] = False
                if np.any(L & g):
                    return True
    return False


def test_sloshing_is_reproducible_from_its_seed():
    a, b, c = W.config("slosh128", seed=3), W.config("slosh128", seed=3), W.config("slosh128", seed=4)
    assert np.array_equal(a.flags, b.flags) and np.array_equal(a.fill, b.fill) and np.array_equal(a.rho, b.rho)
    assert a.meta["theta"] == b.meta["theta"] != c.meta["theta"]
    assert not np.array_equal(a.fill, c.fill)


def test_sloshing_volume_is_the_integral_of_the_surface_height():
    """Each column holds exactly eta(i) of liquid (full cells below the
    surface, the cut cell's fraction at it), so the fills sum to nz sum eta."""
    w = W.sloshing(40, 32, 6, depth=16.0, amp=3.0, seed=5)
    m = w.meta
    i = np.arange(40) + 0.5
    eta = m["depth"] + m["amp"] * np.cos(2.0 * math.pi * i / m["wavelength"] + m["theta"])
    fill = np.where(w.flags == W.GAS, 0.0, w.fill)
    assert abs(fill.sum() - 6 * eta.sum()) < 1e-9 * fill.sum()
    col = fill.reshape(6, 32, 40).sum(axis=1)
    assert np.abs(col - eta[None, :]).max() < 1e-12


def test_initial_classes_have_no_liquid_next_to_gas():
    for w in (W.config("slosh128", seed=0), W.channel(), W.droplet(n=20, radius=6.0),
              W.sloshing(16, 16, 6, depth=8.0, amp=2.5, seed=7, periodic=(1, 0, 1))):
        p = w.params
        assert w.flags.size == p.n_cells
        assert set(np.unique(w.flags)) <= {W.GAS, W.INTERFACE, W.LIQUID, W.SOLID}
        assert not _liquid_next_to_gas(w.flags, (p.nz, p.ny, p.nx), p.periodic), w.name
