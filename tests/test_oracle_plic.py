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


def _plane_box(n_true, c, nx=9, ny=9, nz=13, plic=2):
    """Walled box cut by the plane n.x = c (n towards the gas, x the position
    in cell units from the box corner): exact fill fractions by quadrature,
    classes from the fills (liquid next to gas promoted to interface)."""
    p = W.Params(nx=nx, ny=ny, nz=nz, plic=plic)
    N = p.n_cells
    m = np.abs(n_true)
    fill = np.zeros(N)
    idx = np.arange(N)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    for cell in range(N):
        # liquid where n.(corner + u) < c; reflect axes with n_a < 0 so that m >= 0
        corner = np.array([x[cell], y[cell], z[cell]], dtype=float)
        a = c - n_true @ corner - np.minimum(n_true, 0.0).sum()
        fill[cell] = 0.0 if a <= 0 else (1.0 if a >= m.sum() else _quad_volume(m, a))
    types3 = np.where(fill >= 1.0, W.LIQUID, np.where(fill <= 0.0, W.GAS, W.INTERFACE)).astype(np.uint8)
    t3 = types3.reshape(nz, ny, nx)
    prom = (t3 == W.LIQUID) & W._shift_any(t3 == W.GAS, p.periodic)
    t3[prom] = W.INTERFACE
    return W.Workload("plane", p, t3.reshape(-1), np.ones(N), None, fill), (x, y, z)


def test_height_function_normal_exact_for_planes(oracle_mod):
    """Inclined planes (slopes up to 0.9 against the dominant axis, any
    orientation): wherever the height function applies (all 3 x 3 columns of
    7 cells complete inside the box; elsewhere the normal stays the
    central-difference one, bit for bit) it equals the plane's normal to
    1e-12, and the PLIC offset from it puts the plane where it is; the
    central-difference normal is off by degrees."""
    rng = np.random.default_rng(21)
    exact_total = 0
    for trial in range(4):
        axis = trial % 3
        v = rng.uniform(-0.9, 0.9, size=3)
        v[axis] = 1.0 if rng.random() < 0.5 else -1.0
        n_true = v / np.linalg.norm(v)
        centre = np.array([4.5, 4.5, 6.5])
        centre[axis] = [4.5, 4.5, 6.5][axis] + rng.uniform(-0.5, 0.5)
        c = n_true @ centre
        w, (x, y, z) = _plane_box(n_true, c)
        o = oracle_mod.Oracle.from_workload(w)
        o1 = oracle_mod.Oracle.from_workload(dataclasses.replace(w, params=dataclasses.replace(w.params, plic=1)))
        worst_cd = 0.0
        for cell in np.nonzero(w.flags == W.INTERFACE)[0]:
            if not (0.0 < w.fill[cell] < 1.0):
                continue
            nh = o.interface_normal(int(cell), 1)
            ncd = o1.interface_normal(int(cell), 1)
            if nh is None or np.array_equal(nh, ncd):
                continue
            pos = np.array([x[cell], y[cell], z[cell]])
            assert np.abs(nh - n_true).max() < 1e-12, (trial, cell, nh, n_true)
            d = oracle_mod.plic_offset(w.fill[cell], nh)
            assert d == pytest.approx(c - n_true @ (pos + 0.5), abs=1e-11)
            worst_cd = max(worst_cd, np.degrees(np.arccos(min(1.0, ncd @ n_true))))
            exact_total += 1
        assert worst_cd > 1.0
    assert exact_total >= 60


def test_height_function_falls_back_and_leaves_fsk(oracle_mod):
    """FSK and plic = 1 keep the central-difference normal; a cell whose
    columns leave the box keeps it too."""
    n_true = np.array([0.3, -0.2, 1.0])
    n_true /= np.linalg.norm(n_true)
    w, (x, y, z) = _plane_box(n_true, n_true @ np.array([4.5, 4.5, 6.2]))
    o2 = oracle_mod.Oracle.from_workload(w)
    o1 = oracle_mod.Oracle.from_workload(dataclasses.replace(w, params=dataclasses.replace(w.params, plic=1)))
    for cell in np.nonzero(w.flags == W.INTERFACE)[0][:40]:
        a, b = o2.interface_normal(int(cell), 0), o1.interface_normal(int(cell), 1)
        assert np.array_equal(a, b)
    edge = [c for c in np.nonzero((w.flags == W.INTERFACE) & (x == 0))[0]]
    assert edge
    for cell in edge:
        assert np.array_equal(o2.interface_normal(int(cell), 1), o1.interface_normal(int(cell), 1))
