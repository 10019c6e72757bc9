"""Serial FP64 oracle of the free-surface LBM step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It wraps ``liboracle.so`` (built from ``fslbm_oracle.cpp`` by
``build()`` below) through ctypes and shares nothing with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["fslbm_oracle.cpp", "fslbm_oracle.hpp", "dual.hpp"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp, os.path.join(_HERE, "fslbm_oracle.cpp")]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _RefParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("px", ctypes.c_int), ("py", ctypes.c_int), ("pz", ctypes.c_int),
                ("tau", ctypes.c_double), ("Lambda", ctypes.c_double),
                ("incompressible", ctypes.c_int), ("stokes", ctypes.c_int),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double),
                ("rho_gas", ctypes.c_double), ("eps", ctypes.c_double),
                ("wall_u", ctypes.c_double * 18), ("shear_b", ctypes.c_double * 6),
                ("sigma", ctypes.c_double), ("plic", ctypes.c_int), ("hold", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.ref_create.restype = vp
        L.ref_create.argtypes = [ctypes.POINTER(_RefParams), u8p, dp, dp, dp]
        L.ref_create_state.restype = vp
        L.ref_create_state.argtypes = [ctypes.POINTER(_RefParams), u8p, dp, dp, dp, ctypes.c_double]
        L.ref_create_error.restype = ctypes.c_char_p
        L.ref_destroy.argtypes = [vp]
        L.ref_error.restype = ctypes.c_char_p
        L.ref_error.argtypes = [vp]
        L.ref_set_freeze.argtypes = [vp, ctypes.c_int]
        L.ref_step.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.ref_step.restype = ctypes.c_int
        for name in ("ref_get_populations", "ref_get_mass", "ref_get_phi"):
            getattr(L, name).argtypes = [vp, dp]
        L.ref_get_flags.argtypes = [vp, u8p]
        L.ref_get_collision_moments.argtypes = [vp, dp, dp]
        L.ref_get_macro.argtypes = [vp, dp, dp]
        L.ref_total_mass.restype = ctypes.c_double
        L.ref_total_mass.argtypes = [vp]
        L.ref_reservoir.restype = ctypes.c_double
        L.ref_reservoir.argtypes = [vp]
        L.ref_branch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.ref_list.restype = ctypes.c_int
        L.ref_list.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int]
        L.ref_constants.argtypes = [vp, dp]
        L.ref_equilibrium_post.argtypes = [vp, ctypes.c_double, dp, dp]
        L.ref_collide.argtypes = [vp, dp, dp, dp, dp]
        L.ref_coeffs.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        L.ref_shear.argtypes = [vp, dp, dp]
        L.ref_boundary_shear.argtypes = [dp, dp, ctypes.c_double, dp]
        L.ref_curvature.restype = ctypes.c_double
        L.ref_curvature.argtypes = [dp]
        L.ref_interface_curvature.restype = ctypes.c_double
        L.ref_interface_curvature.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ref_interface_normal.restype = ctypes.c_int
        L.ref_interface_normal.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp]
        L.ref_set_walls.restype = ctypes.c_int
        L.ref_set_surface.argtypes = [ctypes.c_void_p, dp, dp]
        L.ref_set_walls.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp, dp]
        L.ref_cut_volume.restype = ctypes.c_double
        L.ref_cut_volume.argtypes = [dp, ctypes.c_double]
        L.ref_plic_offset.restype = ctypes.c_double
        L.ref_plic_offset.argtypes = [ctypes.c_double, dp]
        L.ref_window_dual.restype = ctypes.c_int
        L.ref_window_dual.argtypes = [ctypes.POINTER(_RefParams), u8p, dp, dp, dp, dp, dp, dp, ctypes.c_double,
                                      dp, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(p) -> _RefParams:
    wall = getattr(p, "wall_u", ((0.0, 0.0, 0.0),) * 6)
    shear = getattr(p, "shear_b", (0.0,) * 6)
    return _RefParams(p.nx, p.ny, p.nz, int(p.periodic[0]), int(p.periodic[1]), int(p.periodic[2]),
                      float(p.tau), float(p.Lambda), int(p.incompressible), int(p.stokes),
                      float(p.g[0]), float(p.g[1]), float(p.g[2]), float(p.rho_gas), float(p.eps),
                      (ctypes.c_double * 18)(*[float(v) for face in wall for v in face]),
                      (ctypes.c_double * 6)(*[float(v) for v in shear]),
                      float(getattr(p, "sigma", 0.0)), int(getattr(p, "plic", 0)), int(getattr(p, "hold", 0)))


FSK, FSL = 0, 1
FSK_STRESS, FSL_STRESS = 2, 3  # with the shear-rate boundary term (Table 1, column D) from the bulk
FSK_SHEAR, FSL_SHEAR = 4, 5    # the same term with the prescribed S^b (params.shear_b)
LISTS = {"F": 0, "E": 1, "E'": 2, "NI": 3, "NL": 4}


class Oracle:
    """One oracle simulation (FP64, serial)."""

    def __init__(self, params, flags=None, rho=None, u=None, fill=None, state=None):
        self.params = params
        self.N = params.nx * params.ny * params.nz
        L = lib()
        self._p = _params(params)
        N = self.N
        if state is not None:
            fl = np.ascontiguousarray(state["flags"], dtype=np.uint8)
            ft = np.ascontiguousarray(state["f"], dtype=np.float64).reshape(-1)
            m = np.ascontiguousarray(state["mass"], dtype=np.float64)
            ph = np.ascontiguousarray(state["phi"], dtype=np.float64)
            assert ft.size == 19 * N and fl.size == N and m.size == N and ph.size == N
            h = L.ref_create_state(ctypes.byref(self._p), fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   _dptr(ft), _dptr(m), _dptr(ph), float(state.get("reservoir", 0.0)))
        else:
            fl = np.ascontiguousarray(flags, dtype=np.uint8)
            r = np.ascontiguousarray(rho, dtype=np.float64)
            uu = np.zeros((3, N)) if u is None else np.ascontiguousarray(u, dtype=np.float64)
            fi = np.ascontiguousarray(fill, dtype=np.float64)
            assert fl.size == N and r.size == N and uu.size == 3 * N and fi.size == N
            h = L.ref_create(ctypes.byref(self._p), fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                             _dptr(r), _dptr(uu), _dptr(fi))
        if not h:
            raise ValueError("oracle rejected input: " + L.ref_create_error().decode())
        self._h = ctypes.c_void_p(h)

    @classmethod
    def from_workload(cls, w):
        o = cls(w.params, w.flags, w.rho, w.u, w.fill)
        walls = getattr(w, "walls", None)
        if walls is not None:
            o.set_walls(walls["cells"], walls.get("delta"), walls.get("uw"))
        surf = getattr(w, "surface", None)
        if surf is not None:
            o.set_surface(surf["normal"], surf["offset"])
        return o

    def interface_curvature(self, cell: int) -> float:
        """Curvature kappa = -div n the step uses at an interface cell."""
        return float(lib().ref_interface_curvature(self._h, int(cell)))

    def interface_normal(self, cell: int, rule: int = FSL):
        """Normal (towards the gas) the step uses at an interface cell, or None."""
        out = np.zeros(3)
        ok = lib().ref_interface_normal(self._h, int(cell), int(rule), _dptr(out))
        return out if ok else None

    def set_walls(self, cells, delta=None, uw=None):
        """Wall table of the solid cells: ascending non-solid cells next to a
        solid cell, delta[19, n] (wall point x + delta c_p), uw[3, 19, n]."""
        c = np.ascontiguousarray(cells, dtype=np.int32)
        n = c.size
        d = None if delta is None else np.ascontiguousarray(delta, dtype=np.float64).reshape(-1)
        v = None if uw is None else np.ascontiguousarray(uw, dtype=np.float64).reshape(-1)
        assert d is None or d.size == 19 * n
        assert v is None or v.size == 3 * 19 * n
        rc = lib().ref_set_walls(self._h, n, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 None if d is None else _dptr(d), None if v is None else _dptr(v))
        if rc != 0:
            raise RuntimeError("oracle wall table rejected: " + lib().ref_error(self._h).decode())

    def set_surface(self, normal, offset):
        """Prescribed surface plane of every interface cell: normal[3, N] (unit,
        towards the gas) and offset[N] (signed distance of the plane from the
        node along the normal); FSL link distances delta = offset / (n . c)."""
        nn = np.ascontiguousarray(normal, dtype=np.float64).reshape(-1)
        dd = np.ascontiguousarray(offset, dtype=np.float64).reshape(-1)
        assert nn.size == 3 * self.N and dd.size == self.N
        self._surf = (nn, dd)
        lib().ref_set_surface(self._h, _dptr(nn), _dptr(dd))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ref_destroy(h)
            self._h = None

    def set_freeze(self, on: bool):
        lib().ref_set_freeze(self._h, int(bool(on)))

    def step(self, n: int = 1, rule: int = FSL):
        if lib().ref_step(self._h, int(n), int(rule)) != 0:
            raise RuntimeError("oracle step failed: " + lib().ref_error(self._h).decode())

    def populations(self) -> np.ndarray:
        out = np.empty(19 * self.N)
        lib().ref_get_populations(self._h, _dptr(out))
        return out.reshape(19, self.N)

    def flags(self) -> np.ndarray:
        out = np.empty(self.N, dtype=np.uint8)
        lib().ref_get_flags(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return out

    def mass(self) -> np.ndarray:
        out = np.empty(self.N)
        lib().ref_get_mass(self._h, _dptr(out))
        return out

    def phi(self) -> np.ndarray:
        out = np.empty(self.N)
        lib().ref_get_phi(self._h, _dptr(out))
        return out

    def collision_moments(self):
        rho = np.empty(self.N)
        u = np.empty(3 * self.N)
        lib().ref_get_collision_moments(self._h, _dptr(rho), _dptr(u))
        return rho, u.reshape(3, self.N)

    def macro(self):
        rho = np.empty(self.N)
        u = np.empty(3 * self.N)
        lib().ref_get_macro(self._h, _dptr(rho), _dptr(u))
        return rho, u.reshape(3, self.N)

    def branch_stats(self) -> dict:
        """Branches the FSL closure took so far: link distances clamped at 0
        and at 1, FSK fallbacks, and an order-independent signature of (step,
        cell, link, branch); equal for two runs that took the same branches."""
        out = (ctypes.c_uint64 * 4)()
        lib().ref_branch_stats(self._h, out)
        return {"clamp0": int(out[0]), "clamp1": int(out[1]), "fallback": int(out[2]), "signature": int(out[3])}

    def total_mass(self) -> float:
        return lib().ref_total_mass(self._h)

    def reservoir(self) -> float:
        return lib().ref_reservoir(self._h)

    def lists(self) -> dict:
        out = {}
        for name, which in LISTS.items():
            n = lib().ref_list(self._h, which, None, 0)
            buf = np.empty(max(n, 1), dtype=np.int32)
            lib().ref_list(self._h, which, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), n)
            out[name] = buf[:n].copy()
        return out

    def constants(self) -> dict:
        out = np.empty(4)
        lib().ref_constants(self._h, _dptr(out))
        return {"lambda_p": out[0], "lambda_m": out[1], "inv_1p_lambda_p": out[2], "thr_hi": out[3]}

    def equilibrium_post(self, rho: float, u) -> np.ndarray:
        uu = np.ascontiguousarray(u, dtype=np.float64)
        out = np.empty(19)
        lib().ref_equilibrium_post(self._h, float(rho), _dptr(uu), _dptr(out))
        return out

    def collide(self, f):
        ff = np.ascontiguousarray(f, dtype=np.float64)
        out = np.empty(19)
        rho = ctypes.c_double()
        u = np.empty(3)
        lib().ref_collide(self._h, _dptr(ff), _dptr(out), ctypes.byref(rho), _dptr(u))
        return out, rho.value, u

    def shear(self, own) -> np.ndarray:
        """Shear rate [xx, yy, zz, xy, xz, yz] from 19 post-collision populations
        (section 3.4; Eq. nqp at leading order)."""
        ff = np.ascontiguousarray(own, dtype=np.float64)
        out = np.empty(6)
        lib().ref_shear(self._h, _dptr(ff), _dptr(out))
        return out

    def coeffs(self, rule: int, alpha_p: float = 1.0, delta: float = 0.0) -> np.ndarray:
        out = np.empty(5)
        lib().ref_coeffs(self._h, int(rule), float(alpha_p), float(delta), _dptr(out))
        return out


def boundary_shear(S, n, s_nn: float) -> np.ndarray:
    """S^b = P S P + s_nn n n^T (section 3.4) for S = [xx, yy, zz, xy, xz, yz]."""
    SS = np.ascontiguousarray(S, dtype=np.float64)
    nn = np.ascontiguousarray(n, dtype=np.float64)
    out = np.empty(6)
    lib().ref_boundary_shear(_dptr(SS), _dptr(nn), float(s_nn), _dptr(out))
    return out


def curvature(block) -> float:
    """Curvature kappa = -div n of a fill field given on the 3x3x3 block around a
    cell, block[dx+1, dy+1, dz+1] (corners unused)."""
    b = np.ascontiguousarray(np.asarray(block, dtype=np.float64).transpose(2, 1, 0)).reshape(-1)
    return float(lib().ref_curvature(_dptr(b)))


def cut_volume(m, a: float) -> float:
    """Volume of the unit cube below the plane m.x = a (m_i >= 0)."""
    mm = np.ascontiguousarray(m, dtype=np.float64)
    return float(lib().ref_cut_volume(_dptr(mm), float(a)))


def plic_offset(phi: float, n) -> float:
    """Offset d of the plane n.(x - x_node) = d cutting the fill fraction phi."""
    nn = np.ascontiguousarray(n, dtype=np.float64)
    return float(lib().ref_plic_offset(float(phi), _dptr(nn)))


def window_dual(params, flags, f0, m0, phi0, u_target, phi_target, T: int, rule: int = FSL,
                df0=None, dm0=None, dphi0=None, drho_b: float = 0.0, dg=None, want_state: bool = False,
                f_weight=None):
    """Frozen-topology window of T steps and the loss
    L = sum over interface cells of |u_T - u*|^2 + (phi_T - phi*)^2  (left out
        when u_target and phi_target are None)
        [+ sum over non-gas cells and q of f_weight[q, cell] ft_q(T)],
    with its exact directional derivative along (df0, dm0, dphi0, drho_b, dg)
    from a dual-number run of the oracle.  Returns (L, dL) or, with want_state,
    (L, dL, {"f", "mass", "phi"}) of time T."""
    N = params.nx * params.ny * params.nz

    def arr(a, n):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)

    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    f0, m0, phi0 = arr(f0, 19 * N), arr(m0, N), arr(phi0, N)
    ut, pt = arr(u_target, 3 * N), arr(phi_target, N)  # both None: no interface term
    d = [arr(df0, 19 * N), arr(dm0, N), arr(dphi0, N), arr(dg, 3)]
    fw = arr(f_weight, 19 * N)
    assert f0.size == 19 * N and m0.size == N and phi0.size == N
    assert (ut is None) == (pt is None) and (ut is None or (ut.size == 3 * N and pt.size == N))
    out2 = np.zeros(2)
    fT = np.empty(19 * N) if want_state else None
    mT = np.empty(N) if want_state else None
    pT = np.empty(N) if want_state else None
    opt = lambda a: None if a is None else _dptr(a)  # noqa: E731
    p = _params(params)
    rc = lib().ref_window_dual(ctypes.byref(p), fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                               _dptr(f0), _dptr(m0), _dptr(phi0), opt(d[0]), opt(d[1]), opt(d[2]),
                               float(drho_b), opt(d[3]), int(T), int(rule), opt(ut), opt(pt), opt(fw), _dptr(out2),
                               opt(fT), opt(mT), opt(pT))
    if rc != 0:
        raise ValueError("oracle window failed: " + lib().ref_create_error().decode())
    if want_state:
        return out2[0], out2[1], {"f": fT.reshape(19, N), "mass": mT, "phi": pT}
    return out2[0], out2[1]
