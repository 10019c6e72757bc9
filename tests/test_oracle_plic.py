"""Pins of the oracle's second-order interface position (section 5: the link
distance delta needs the interface plane to second order; PLIC is one such
reconstruction).

With the option on, an FSL interface cell places its surface on the plane
n.(x - x_node) = d whose cut of the unit cell holds the fill fraction phi, and
a link c_o meets it at delta = d / (c_o . n).  The cut volume is pinned against
closed forms and numerical quadrature, the plane offset against planes of known
offset, and the step against the plain phi - 1/2 reading where the two must
agree.
"""
import dataclasses

import numpy as np
import pytest
from scipy import integrate

from paper_1409_5645_amd import workloads as W


def _quad_volume(m, a):
    """Volume of {x in [0,1]^3 : m.x <= a} as the integral of the clipped
    column height over the axis with the largest component: the inner
    integral is exact (the height is piecewise linear in y), the outer one is
    adaptive quadrature over the pieces between its kinks."""
    m = np.asarray(m, dtype=float)
    k = int(np.argmax(m))
    o = [i for i in range(3) if i != k]
    mk, mx, my = m[k], m[o[0]], m[o[1]]

    def height(c, y):
        return min(max((c - my * y) / mk, 0.0), 1.0)

    def inner(x):
        c = a - mx * x
        pts = [0.0, 1.0]
        if my > 0.0:
            pts += [y for y in (c / my, (c - mk) / my) if 0.0 < y < 1.0]
        pts.sort()
        return sum(0.5 * (height(c, y0) + height(c, y1)) * (y1 - y0) for y0, y1 in zip(pts[:-1], pts[1:]))

    kinks = [0.0, 1.0]
    if mx > 0.0:
        kinks += [x for y in (0.0, 1.0) for h in (0.0, mk) for x in [(a - my * y - h) / mx] if 0.0 < x < 1.0]
    kinks.sort()
    return sum(integrate.quad(inner, x0, x1, epsabs=1e-14, epsrel=1e-14, limit=200)[0]
               for x0, x1 in zip(kinks[:-1], kinks[1:]))


@pytest.mark.parametrize("m,a,v", [
    ((1, 1, 1), 1.0, 1.0 / 6.0),       # corner tetrahedron
    ((1, 1, 1), 1.5, 0.5),             # through the centre
    ((1, 1, 1), 2.0, 5.0 / 6.0),       # complement of the opposite tetrahedron
    ((1, 1, 1), 3.0, 1.0),
    ((1, 2, 3), 1.0, 1.0 / 36.0),      # tetrahedron a^3 / (6 m0 m1 m2)
    ((1, 1, 0), 1.0, 0.5),             # prism over a half square
    ((1, 1, 0), 0.5, 0.125),
    ((0, 0, 1), 0.3, 0.3),             # slab
    ((0, 2, 0), 0.5, 0.25),
    ((1, 1, 1), 0.0, 0.0),
])
def test_cut_volume_closed_forms(oracle_mod, m, a, v):
    assert oracle_mod.cut_volume(m, a) == pytest.approx(v, abs=1e-15)


def test_cut_volume_against_quadrature_and_symmetry(oracle_mod):
    """Random planes, with and without zero components: the cut equals the
    integral of the clipped column height, and the point symmetry of the cube
    gives V(a) + V(|m|_1 - a) = 1."""
    rng = np.random.default_rng(5)
    for t in range(40):
        m = rng.random(3) + 0.05
        if t % 4 == 1:
            m[rng.integers(3)] = 0.0
        s = m.sum()
        a = rng.random() * s
        v = oracle_mod.cut_volume(m, a)
        assert v == pytest.approx(_quad_volume(m, a), abs=1e-12)
        assert v + oracle_mod.cut_volume(m, s - a) == pytest.approx(1.0, abs=1e-14)


def test_cut_volume_near_degenerate_normals(oracle_mod):
    """Components of 1e-13 .. 1e-4 beside O(1) ones (nearly grid-aligned
    surfaces, the common case of a central-difference normal): the volume
    stays within 1e-13 of the quadrature value, and shrinking a component to
    zero meets the lower-dimensional cut continuously."""
    rng = np.random.default_rng(11)
    for tiny in (1e-4, 1e-7, 1e-10, 1e-13):
        for _ in range(12):
            m = rng.random(3) + 0.05
            m[rng.integers(3)] = tiny * rng.random()
            if rng.random() < 0.3:
                j = int(np.argmax(m))
                m[(j + 1) % 3] = tiny * rng.random()
            a = rng.random() * m.sum()
            v = oracle_mod.cut_volume(m, a)
            assert v == pytest.approx(_quad_volume(m, a), abs=1e-13)
            m0 = np.where(m < 1e-3, 0.0, m)
            assert abs(v - oracle_mod.cut_volume(m0, a)) < 4.0 * tiny


def test_plic_offset_axis_aligned_and_diagonal(oracle_mod):
    """Axis-aligned normals give the plane phi - 1/2 from the node (the plain
    reading); along the body diagonal a half-full cell's plane passes through
    the node."""
    for phi in (0.0, 0.1, 0.37, 0.5, 0.9, 1.0):
        for n in ([0, 0, -1], [1, 0, 0], [0, -1, 0]):
            assert oracle_mod.plic_offset(phi, n) == pytest.approx(phi - 0.5, abs=1e-15)
    d = np.ones(3) / np.sqrt(3.0)
    assert oracle_mod.plic_offset(0.5, d) == pytest.approx(0.0, abs=1e-15)
    assert oracle_mod.plic_offset(0.5, -d) == pytest.approx(0.0, abs=1e-15)


def test_plic_offset_recovers_known_planes(oracle_mod):
    """A plane n.(x - x_node) = d of random unit normal and offset cuts the cell
    with a fill fraction computed by quadrature; the offset recovered from that
    fraction is d.  Flipping signs of n (reflections of the cell) leaves it
    unchanged."""
    rng = np.random.default_rng(9)
    for _ in range(30):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        m = np.abs(n)
        d = (rng.random() - 0.5) * 0.9 * m.sum()
        phi = _quad_volume(m, d + 0.5 * m.sum())
        assert oracle_mod.plic_offset(phi, n) == pytest.approx(d, abs=1e-11)
        flip = n * np.where(rng.random(3) < 0.5, -1.0, 1.0)
        assert oracle_mod.plic_offset(phi, flip) == oracle_mod.plic_offset(phi, n)


def _run(oracle_mod, w, rule, steps):
    o = oracle_mod.Oracle.from_workload(w)
    o.step(steps, rule)
    return o


def _with(w, **kw):
    return dataclasses.replace(w, params=dataclasses.replace(w.params, **kw))


def test_plic_leaves_fsk_and_flat_films_unchanged(oracle_mod):
    """The option moves only FSL link distances: FSK (no distance) is identical
    bit for bit on a curved surface, and a film with a grid-aligned surface
    (phi - 1/2 is already the plane) agrees with the plain reading to rounding."""
    w = W.sloshing(nx=24, ny=20, nz=16, depth=11.0, amp=2.0, seed=3)
    a = _run(oracle_mod, w, 0, 6)
    b = _run(oracle_mod, _with(w, plic=1), 0, 6)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.flags(), b.flags())
    f = W.channel(h=12.3, nx=4, ny=20, nz=4)
    a = _run(oracle_mod, f, 1, 30)
    b = _run(oracle_mod, _with(f, plic=1), 1, 30)
    assert np.array_equal(a.flags(), b.flags())
    assert np.abs(a.populations() - b.populations()).max() < 1e-13


def test_plic_changes_fsl_on_curved_surfaces_and_conserves_mass(oracle_mod):
    """On a sloshing surface the plane differs from phi - 1/2 and the FSL step
    changes; mass (cells plus the conversion reservoir) stays conserved."""
    w = _with(W.sloshing(nx=24, ny=20, nz=16, depth=11.0, amp=2.0, seed=3), plic=1)
    o = oracle_mod.Oracle.from_workload(w)
    M0 = o.total_mass() + o.reservoir()
    o.step(20, 1)
    assert abs((o.total_mass() + o.reservoir()) / M0 - 1.0) < 1e-13
    ref = _run(oracle_mod, _with(w, plic=0), 1, 20)
    assert np.abs(o.populations() - ref.populations()).max() > 1e-8
