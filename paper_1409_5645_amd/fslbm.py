"""ctypes binding of libfslbm.so (the C interface of include/fslbm.h).

Argument marshalling only: torch allocates the device buffers and supplies the
stream; every step of the method runs in the library's HIP kernels.  There is
no CPU fallback: if the library is missing or no GPU is present, construction
fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfslbm.so")

FSK, FSL = 0, 1
FSK_STRESS, FSL_STRESS = 2, 3  # with the shear-rate boundary term (Table 1, column D) from the bulk
FSK_SHEAR, FSL_SHEAR = 4, 5    # the same term with the prescribed S^b (params.shear_b)
FP64, FP32, FP16S = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16s": FP16S}
GAS, INTERFACE, LIQUID = 0, 1, 2
STATUS = {0: "OK", 1: "INVALID", 2: "UNSUPPORTED", 3: "DEVICE", 4: "UNSTABLE", 5: "INVARIANT", 6: "CAPACITY"}
FIELDS = ("rho", "u", "phi", "flags", "f", "mass", "rho_c", "u_c")
ABI_VERSION = 5


class FslbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fslbm {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("periodic", ctypes.c_int32 * 3), ("precision", ctypes.c_int32),
                ("tau", ctypes.c_double), ("magic", ctypes.c_double), ("incompressible", ctypes.c_int32),
                ("stokes", ctypes.c_int32), ("g", ctypes.c_double * 3), ("rho_gas", ctypes.c_double),
                ("conv_eps", ctypes.c_double), ("fp16_scale_log2", ctypes.c_int32), ("freeze", ctypes.c_int32),
                ("wall_u", (ctypes.c_double * 3) * 6), ("shear_b", ctypes.c_double * 6),
                ("sigma", ctypes.c_double), ("plic", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("u_max", ctypes.c_double), ("hold_fill", ctypes.c_int32)]


class Buffers(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p * 2), ("flags", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("phi", ctypes.c_void_p * 2), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p)]


EXPORTS = ("fslbm_workspace_size", "fslbm_init", "fslbm_init_static", "fslbm_set_equilibrium", "fslbm_set_state", "fslbm_step",
           "fslbm_fields", "fslbm_stats", "fslbm_conversions", "fslbm_timing", "fslbm_set_forcing", "fslbm_set_walls",
           "fslbm_set_surface",
           "fslbm_window_workspace_size", "fslbm_window_forward", "fslbm_window_backward", "fslbm_window_info",
           "fslbm_window_destroy", "fslbm_destroy", "fslbm_last_error")

_lib = None


def lib():
    """Load libfslbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1409_5645_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        dp = ctypes.POINTER(ctypes.c_double)
        L.fslbm_workspace_size.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]
        L.fslbm_init.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Buffers), ctypes.POINTER(vp)]
        L.fslbm_init_static.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Buffers), ctypes.POINTER(vp)]
        L.fslbm_set_equilibrium.argtypes = [vp, vp, vp, vp]
        L.fslbm_set_state.argtypes = [vp, vp, vp, vp, ctypes.c_double]
        L.fslbm_step.argtypes = [vp, i32, i32]
        L.fslbm_fields.argtypes = [vp, u32, ctypes.POINTER(vp)]
        L.fslbm_stats.argtypes = [vp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.fslbm_conversions.argtypes = [vp, ctypes.POINTER(ctypes.POINTER(i32)), i32, ctypes.POINTER(i32)]
        L.fslbm_timing.argtypes = [vp, i32, dp, ctypes.POINTER(ctypes.c_int64)]
        L.fslbm_set_forcing.argtypes = [vp, dp, ctypes.c_double]
        L.fslbm_set_walls.argtypes = [vp, i32, vp, vp, vp]
        L.fslbm_set_surface.argtypes = [vp, vp, vp]
        L.fslbm_window_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.fslbm_window_forward.argtypes = [vp, i32, i32, i32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.fslbm_window_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, dp]
        L.fslbm_window_info.argtypes = [vp, ctypes.POINTER(i32)]
        L.fslbm_window_destroy.argtypes = [vp]
        L.fslbm_destroy.argtypes = [vp]
        L.fslbm_last_error.argtypes = [vp]
        L.fslbm_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "fslbm_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def make_params(p, precision=FP64, freeze=False, fp16_scale_log2=13, check_every=0, u_max=0.0) -> Params:
    """C parameter block from a workloads.Params (check_every, u_max: the
    health check of fslbm_step; 0 = none / the default bound)."""
    return Params(ABI_VERSION, p.nx, p.ny, p.nz, (ctypes.c_int32 * 3)(*[int(v) for v in p.periodic]),
                  int(precision), float(p.tau), float(p.Lambda), int(p.incompressible), int(p.stokes),
                  (ctypes.c_double * 3)(*[float(v) for v in p.g]), float(p.rho_gas), float(p.eps),
                  int(fp16_scale_log2), int(bool(freeze)),
                  ((ctypes.c_double * 3) * 6)(*[(ctypes.c_double * 3)(*[float(v) for v in face])
                                                 for face in getattr(p, "wall_u", ((0.0, 0.0, 0.0),) * 6)]),
                  (ctypes.c_double * 6)(*[float(v) for v in getattr(p, "shear_b", (0.0,) * 6)]),
                  float(getattr(p, "sigma", 0.0)), int(getattr(p, "plic", 0)), int(check_every), float(u_max),
                  int(getattr(p, "hold", 0)))


class Sim:
    """One simulation on a GPU.  Buffers are torch tensors on `device`."""

    def __init__(self, params, flags, precision="fp64", device="cuda:0", stream=None, freeze=None,
                 fp16_scale_log2=13, check_every=0, u_max=0.0, static_workspace=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("fslbm needs a GPU (torch.cuda.is_available() is False)")
        L = lib()
        self.torch = torch
        self.device = torch.device(device)
        self.params = params
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.N = N = params.nx * params.ny * params.nz
        if freeze is None:  # a held surface implies frozen classes
            freeze = bool(getattr(params, "hold", 0))
        self.cp = make_params(params, self.precision, freeze, fp16_scale_log2, check_every, u_max)
        ws = ctypes.c_size_t()
        self._check(L.fslbm_workspace_size(ctypes.byref(self.cp), ctypes.byref(ws)), None)
        dt = {FP64: torch.float64, FP32: torch.float32, FP16S: torch.float16}[self.precision]
        with torch.cuda.device(self.device):
            self.stream = stream or torch.cuda.current_stream(self.device)
            self.f = [torch.empty(19 * N, dtype=dt, device=self.device) for _ in range(2)]
            self.flags_t = torch.as_tensor(np.ascontiguousarray(flags, dtype=np.uint8)).to(self.device)
            self.mass_t = torch.zeros(N, dtype=torch.float64, device=self.device)
            self.phi_t = [torch.zeros(N, dtype=torch.float64, device=self.device) for _ in range(2)]
            # static_workspace: the library's own array (fslbm_init_static), no workspace buffer
            self.ws = None if static_workspace else torch.empty(ws.value, dtype=torch.uint8, device=self.device)
        assert self.ws is None or self.ws.data_ptr() % 256 == 0
        b = Buffers((ctypes.c_void_p * 2)(self.f[0].data_ptr(), self.f[1].data_ptr()), self.flags_t.data_ptr(),
                    self.mass_t.data_ptr(), (ctypes.c_void_p * 2)(self.phi_t[0].data_ptr(), self.phi_t[1].data_ptr()),
                    None if self.ws is None else self.ws.data_ptr(), 0 if self.ws is None else ws.value,
                    self.stream.cuda_stream)
        torch.cuda.synchronize(self.device)
        h = ctypes.c_void_p()
        init = L.fslbm_init_static if static_workspace else L.fslbm_init
        with torch.cuda.device(self.device):
            self._check(init(ctypes.byref(self.cp), ctypes.byref(b), ctypes.byref(h)), None)
        self.ctx = h

    # ------------------------------------------------------------- helpers
    def _check(self, st, ctx):
        if st != 0:
            msg = lib().fslbm_last_error(ctx).decode()
            raise FslbmError(st, msg)

    def _as_dev64(self, a):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            return a.detach().to(device=self.device, dtype=torch.float64).contiguous()
        return self._dev(a)

    def _dev(self, a, dtype=None):
        t = self.torch.as_tensor(np.ascontiguousarray(a, dtype=dtype or np.float64))
        return t.to(self.device)

    @classmethod
    def from_workload(cls, w, precision="fp64", **kw):
        s = cls(w.params, w.flags, precision=precision, **kw)
        s.set_equilibrium(w.rho, w.velocity(), w.fill)
        walls = getattr(w, "walls", None)
        if walls is not None:
            s.set_walls(walls["cells"], walls.get("delta"), walls.get("uw"))
        surf = getattr(w, "surface", None)
        if surf is not None:
            s.set_surface(surf["normal"], surf["offset"])
        return s

    def set_surface(self, normal, offset):
        """Prescribed surface plane of the interface cells: normal[3, N]
        (unit, towards the gas) and offset[N] (plane offset from the node);
        needs params.hold.  The device copies are kept by this object."""
        self._surface = (self._dev(normal), self._dev(offset))
        self.torch.cuda.synchronize(self.device)
        self._check(lib().fslbm_set_surface(self.ctx, self._surface[0].data_ptr(), self._surface[1].data_ptr()),
                    self.ctx)

    def set_walls(self, cells, delta=None, uw=None):
        """Wall table of the solid cells (class 3): ascending non-solid cells
        next to a solid cell, delta[19, n] (default 1/2) and uw[3, 19, n]
        (default 0).  The device copies are kept by this object."""
        torch = self.torch
        c = np.ascontiguousarray(cells, dtype=np.int32)
        n = c.size
        d = np.full((19, n), 0.5) if delta is None else np.asarray(delta, dtype=np.float64).reshape(19, n)
        v = np.zeros((3, 19, n)) if uw is None else np.asarray(uw, dtype=np.float64).reshape(3, 19, n)
        self._walls = (torch.as_tensor(c).to(self.device), self._dev(d), self._dev(v))
        torch.cuda.synchronize(self.device)
        ct, dt, vt = self._walls
        self._check(lib().fslbm_set_walls(self.ctx, n, ct.data_ptr() if n else None, dt.data_ptr() if n else None,
                                          vt.data_ptr() if n else None), self.ctx)

    # ---------------------------------------------------------------- API
    def set_equilibrium(self, rho, u, fill):
        r, uu, fi = self._dev(rho), self._dev(u), self._dev(fill)
        self.torch.cuda.synchronize(self.device)
        self._check(lib().fslbm_set_equilibrium(self.ctx, r.data_ptr(), uu.data_ptr(), fi.data_ptr()), self.ctx)

    def set_state(self, f, mass, fill, reservoir=0.0):
        """Post-collision populations f[19, N] (unshifted), mass[N], fill[N]:
        numpy arrays or float64 device tensors."""
        ff, m, fi = (self._as_dev64(a) for a in (f, mass, fill))
        self.torch.cuda.synchronize(self.device)
        self._check(lib().fslbm_set_state(self.ctx, ff.data_ptr(), m.data_ptr(), fi.data_ptr(), float(reservoir)),
                    self.ctx)

    def step(self, n=1, rule=FSL):
        self._check(lib().fslbm_step(self.ctx, int(n), int(rule)), self.ctx)

    def fields(self, names=FIELDS, device=False) -> dict:
        """Requested fields as numpy arrays, or torch device tensors when
        device=True (synchronises)."""
        torch = self.torch
        N = self.N
        shapes = {"rho": (N,), "u": (3, N), "phi": (N,), "flags": (N,), "f": (19, N), "mass": (N,),
                  "rho_c": (N,), "u_c": (3, N)}
        out = {}
        ptrs = (ctypes.c_void_p * 8)()
        mask = 0
        for name in names:
            i = FIELDS.index(name)
            dt = torch.uint8 if name == "flags" else torch.float64
            out[name] = torch.empty(shapes[name], dtype=dt, device=self.device)
            ptrs[i] = out[name].data_ptr()
            mask |= 1 << i
        self._check(lib().fslbm_fields(self.ctx, mask, ptrs), self.ctx)
        if device:
            return out
        return {k: v.cpu().numpy() for k, v in out.items()}

    def stats(self) -> dict:
        M, R = ctypes.c_double(), ctypes.c_double()
        c = (ctypes.c_int64 * 8)()
        self._check(lib().fslbm_stats(self.ctx, ctypes.byref(M), ctypes.byref(R), c), self.ctx)
        keys = ("filled", "emptied", "emptied_converted", "new_from_gas", "new_from_liquid", "interface",
                "liquid", "steps")
        d = {k: int(v) for k, v in zip(keys, c)}
        d.update(total_mass=M.value, reservoir=R.value)
        return d

    def conversions(self, cap=None) -> dict:
        """Lists of the last step, ascending: F, E, E', NI, NL."""
        cap = self.N if cap is None else cap
        bufs = [np.empty(max(cap, 1), dtype=np.int32) for _ in range(5)]
        arr = (ctypes.POINTER(ctypes.c_int32) * 5)(*[b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for b in bufs])
        n = (ctypes.c_int32 * 5)()
        self._check(lib().fslbm_conversions(self.ctx, arr, int(cap), n), self.ctx)
        return {k: bufs[i][:n[i]].copy() for i, k in enumerate(("F", "E", "E'", "NI", "NL"))}

    def timing(self, enable: bool):
        """Start (True) or stop (False) sweep-kernel event timing; returns the
        summed sweep milliseconds and the number of sweeps recorded."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(lib().fslbm_timing(self.ctx, int(bool(enable)), ctypes.byref(ms), ctypes.byref(n)), self.ctx)
        return ms.value, n.value

    def set_forcing(self, g, rho_gas):
        """Body acceleration g (3 values) and gas density rho_b = 3 P_b for the
        steps enqueued from now on."""
        gg = (ctypes.c_double * 3)(*[float(v) for v in g])
        self._check(lib().fslbm_set_forcing(self.ctx, gg, float(rho_gas)), self.ctx)

    def window(self, T, rule=FSL, K=0):
        """Forward pass of an adjoint window of T frozen-class steps from the
        current state, with checkpoint spacing K (0 = the library's default:
        every step's record when it fits in half the free device memory, else
        ceil(sqrt T)).  Returns a Window whose backward() gives the gradients."""
        w = Window(self, int(T), int(rule), int(K))
        self.last_window_K = w.K
        return w

    def close(self):
        if getattr(self, "ctx", None):
            lib().fslbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Window:
    """Adjoint window on a Sim: the forward pass runs at construction."""

    def __init__(self, sim: Sim, T: int, rule: int, K: int = 0):
        torch = sim.torch
        L = lib()
        self.sim = sim
        nb = ctypes.c_size_t()
        sim._check(L.fslbm_window_workspace_size(sim.ctx, T, K, ctypes.byref(nb)), sim.ctx)
        with torch.cuda.device(sim.device):
            self.ws = torch.empty(nb.value, dtype=torch.uint8, device=sim.device)
        assert self.ws.data_ptr() % 256 == 0
        h = ctypes.c_void_p()
        sim._check(L.fslbm_window_forward(sim.ctx, T, K, int(rule), self.ws.data_ptr(), nb.value, ctypes.byref(h)),
                   sim.ctx)
        self.h = h
        info = (ctypes.c_int32 * 4)()
        L.fslbm_window_info(h, info)
        self.T, self.K, self.checkpoints, self.n_interface = (int(v) for v in info)
        self.workspace_bytes = nb.value

    def backward(self, dL_df=None, dL_dm=None, dL_dphi=None) -> dict:
        """Gradients of the state of time 0 and of (rho_b, g) from the loss
        gradients of time T (float64 device tensors or None)."""
        sim = self.sim
        torch = sim.torch
        N = sim.N

        def ptr(t, n):
            if t is None:
                return None, None
            t = t.detach().to(device=sim.device, dtype=torch.float64).contiguous().reshape(-1)
            assert t.numel() == n
            return t, t.data_ptr()

        keep = [ptr(dL_df, 19 * N), ptr(dL_dm, N), ptr(dL_dphi, N)]
        out = {"f": torch.empty((19, N), dtype=torch.float64, device=sim.device),
               "mass": torch.empty(N, dtype=torch.float64, device=sim.device),
               "phi": torch.empty(N, dtype=torch.float64, device=sim.device)}
        g4 = (ctypes.c_double * 4)()
        sim.torch.cuda.synchronize(sim.device)
        sim._check(lib().fslbm_window_backward(self.h, keep[0][1], keep[1][1], keep[2][1], out["f"].data_ptr(),
                                                 out["mass"].data_ptr(), out["phi"].data_ptr(), g4), sim.ctx)
        out["rho_b"] = g4[0]
        out["P_b"] = 3.0 * g4[0]
        out["g"] = np.array([g4[1], g4[2], g4[3]])
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().fslbm_window_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _window_function():
    import torch

    class FslbmWindow(torch.autograd.Function):
        """(f0, m0, phi0, P_b, g) -> (f_T, m_T, phi_T) over T steps with frozen
        cell classes on `sim` (whose state it overwrites), differentiable by the
        library's hand-written adjoint with sqrt(T) checkpointing.  f is
        [19, N] post-collision populations (unshifted), m and phi [N]; outputs
        at gas cells (f) or outside interface cells (m, phi) are constants."""

        @staticmethod
        def forward(ctx, sim, T, rule, K, f0, m0, phi0, P_b, g):
            sim.set_state(f0, m0, phi0)
            sim.set_forcing([float(v) for v in g.detach().cpu()], 3.0 * float(P_b))
            win = sim.window(T, rule, K)
            ctx.win = win
            out = sim.fields(("f", "mass", "phi"), device=True)
            return out["f"], out["mass"], out["phi"]

        @staticmethod
        def backward(ctx, df, dm, dphi):
            gr = ctx.win.backward(df, dm, dphi)
            dev = gr["f"].device
            return (None, None, None, None, gr["f"], gr["mass"], gr["phi"],
                    torch.tensor(gr["P_b"], dtype=torch.float64, device=dev),
                    torch.tensor(gr["g"], dtype=torch.float64, device=dev))

    return FslbmWindow


_FW = None


def window_apply(sim, T, rule, f0, m0, phi0, P_b, g, K=0):
    """FslbmWindow.apply with the window options first (see FslbmWindow)."""
    global _FW
    if _FW is None:
        _FW = _window_function()
    return _FW.apply(sim, int(T), int(rule), int(K), f0, m0, phi0, P_b, g)
