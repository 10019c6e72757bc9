"""Adjoint window on the GPU (C-ABI and the torch.autograd.Function) against
the oracle's exact directional derivatives (dual numbers) and central finite
differences of the GPU's own FP64 forward pass.

Loss: L = sum over interface cells at time T of |u_T - u*|^2 + (phi_T - phi*)^2
(+ a random linear functional of all populations of time T, which reaches every
element the adjoint pushes).  u_T is recovered from the post-collision
populations, u = (j - g) + g/2, in torch.

Bars: FP64 directional derivatives within 1e-6 relative of the oracle's dual
numbers (the two compute the same derivative in different orders, so agreement
is expected near 1e-12), at the adjoint's own configuration (128 x 96 x 128,
T = 400) against golden values written by an oracle-only script; within 1e-6
of FP64 central differences whose steps the oracle's branch record shows on
one branch (h^2 truncation and rounding of the loss lie far below); the
checkpoint spacing does not change the result (bit for bit).  FP32: error
against the FP64 gradient stated.
"""
import dataclasses
import math
import time

import numpy as np
import pytest

from paper_1409_5645_amd import workloads as W

pytestmark = pytest.mark.gpu

from d3q19 import C as CV  # noqa: E402


@pytest.fixture(scope="module")
def fs():
    from paper_1409_5645_amd import fslbm
    return fslbm


def _say(*a):
    print(*a, flush=True)


T = 20


@pytest.fixture(scope="module")
def case(oracle_mod):
    w = W.sloshing(16, 14, 10, depth=7.0, amp=1.5, amp_z=1.0, seed=3, gy=-2e-4, tau=0.7)
    o = oracle_mod.Oracle.from_workload(w)
    o.step(40, oracle_mod.FSL)
    st = {"f": o.populations(), "mass": o.mass(), "phi": o.phi(), "flags": o.flags()}
    N = w.params.n_cells
    rng = np.random.default_rng(0)
    tg = {"u": rng.normal(0.0, 1e-3, (3, N)), "phi": rng.uniform(0.0, 1.0, N),
          "a": rng.normal(0.0, 1.0, (19, N)) * (st["flags"] != W.GAS)}
    dirs = {"f": rng.normal(0.0, 1.0, (19, N)) * (st["flags"] != W.GAS),
            "m": rng.normal(0.0, 1.0, N) * (st["flags"] == W.INTERFACE),
            "phi": rng.normal(0.0, 1.0, N) * (st["flags"] == W.INTERFACE)}
    return w.params, st, tg, dirs


def _loss(torch, fT, phiT, g, iface, tg, with_linear=True):
    C = torch.as_tensor(CV, dtype=torch.float64, device=fT.device)
    u = (C.T @ fT - g[:, None]) + 0.5 * g[:, None]
    ut = torch.as_tensor(tg["u"], device=fT.device)
    pt = torch.as_tensor(tg["phi"], device=fT.device)
    m = torch.as_tensor(iface, device=fT.device)
    L = ((u - ut) ** 2).sum(0)[m].sum() + ((phiT - pt) ** 2)[m].sum()
    if with_linear:
        L = L + (torch.as_tensor(tg["a"], device=fT.device) * fT).sum()
    return L


def _gpu_grad(fs, case, rule, precision="fp64", K=0, with_linear=True):
    import torch
    p, st, tg, _ = case
    sim = fs.Sim(p, st["flags"], precision=precision)
    dev = sim.device
    leaf = lambda a: torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True)  # noqa: E731
    f0, m0, phi0 = leaf(st["f"]), leaf(st["mass"]), leaf(st["phi"])
    P_b = leaf(p.rho_gas / 3.0)
    g = leaf(np.array(p.g, dtype=np.float64))
    fT, mT, phiT = fs.window_apply(sim, T, rule, f0, m0, phi0, P_b, g, K=K)
    L = _loss(torch, fT, phiT, g, st["flags"] == W.INTERFACE, tg, with_linear)
    L.backward()
    out = {"L": float(L.detach()), "f": f0.grad.cpu().numpy(), "m": m0.grad.cpu().numpy(), "phi": phi0.grad.cpu().numpy(),
           "P_b": float(P_b.grad), "g": g.grad.cpu().numpy()}
    sim.close()
    return out


def _dual(oracle_mod, case, rule, with_linear=True, **kw):
    p, st, tg, _ = case
    return oracle_mod.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], tg["u"], tg["phi"], T, rule,
                                  f_weight=tg["a"] if with_linear else None, **kw)


@pytest.mark.parametrize("rule", [0, 1])
def test_adjoint_matches_oracle_dual_fp64(fs, oracle_mod, case, rule):
    _say(f"case adjoint fp64 rule={rule}: 16x14x10 T={T} vs oracle dual numbers")
    gr = _gpu_grad(fs, case, rule)
    _, st, _, dirs = case
    L0, _ = _dual(oracle_mod, case, rule)
    _say("loss gpu", gr["L"], "oracle", L0)
    assert abs(gr["L"] - L0) <= 1e-12 * abs(L0)
    checks = [
        ("f0", dict(df0=dirs["f"]), float((gr["f"] * dirs["f"]).sum())),
        ("m0", dict(dm0=dirs["m"]), float((gr["m"] * dirs["m"]).sum())),
        ("phi0", dict(dphi0=dirs["phi"]), float((gr["phi"] * dirs["phi"]).sum())),
        ("rho_b", dict(drho_b=1.0), gr["P_b"] / 3.0),
    ] + [(f"g{a}", dict(dg=np.eye(3)[a]), float(gr["g"][a])) for a in range(3)]
    worst = 0.0
    for name, kw, gpu in checks:
        _, ref = _dual(oracle_mod, case, rule, **kw)
        rel = abs(gpu - ref) / max(abs(ref), 1e-300)
        worst = max(worst, rel) if math.isfinite(rel) else math.inf
        _say(f"  {name:6s} adjoint {gpu:+.15e} dual {ref:+.15e} rel {rel:.2e}")
    assert worst <= 1e-6


@pytest.mark.parametrize("rule", [0, 1])
def test_adjoint_with_moving_walls_matches_oracle_dual(fs, oracle_mod, case, rule):
    """Moving wall faces add a constant to the bounced-back populations, so the
    adjoint is that of resting walls on the moving trajectory: FP64 directional
    derivatives against the oracle's dual numbers with three faces moving."""
    p, st, tg, dirs = case
    pw = dataclasses.replace(p, wall_u=((0.0, 0.0, 2e-3), (0.0, 0.0, 0.0), (1e-3, 0.0, -5e-4), (0.0, 0.0, 0.0),
                                        (0.0, 0.0, 0.0), (3e-3, 0.0, 0.0)))
    c2 = (pw, st, tg, dirs)
    _say(f"case adjoint fp64 moving walls rule={rule}")
    gr = _gpu_grad(fs, c2, rule)
    L0, _ = _dual(oracle_mod, c2, rule)
    assert abs(gr["L"] - L0) <= 1e-12 * abs(L0)
    for name, kw, gpu in (("f0", dict(df0=dirs["f"]), float((gr["f"] * dirs["f"]).sum())),
                          ("rho_b", dict(drho_b=1.0), gr["P_b"] / 3.0),
                          ("g0", dict(dg=np.eye(3)[0]), float(gr["g"][0]))):
        _, ref = _dual(oracle_mod, c2, rule, **kw)
        rel = abs(gpu - ref) / abs(ref)
        _say(f"  {name:6s} rel {rel:.2e}")
        assert math.isfinite(rel) and rel <= 1e-6


def test_adjoint_only_interface_loss(fs, oracle_mod, case):
    """Without the linear term the gradient reaches the state only through the
    interface cells' velocity and fill."""
    _say("case adjoint fp64 FSL, interface-only loss")
    gr = _gpu_grad(fs, case, 1, with_linear=False)
    _, st, _, dirs = case
    for name, kw, gpu in (("f0", dict(df0=dirs["f"]), float((gr["f"] * dirs["f"]).sum())),
                          ("phi0", dict(dphi0=dirs["phi"]), float((gr["phi"] * dirs["phi"]).sum())),
                          ("rho_b", dict(drho_b=1.0), gr["P_b"] / 3.0)):
        _, ref = _dual(oracle_mod, case, 1, with_linear=False, **kw)
        rel = abs(gpu - ref) / abs(ref)
        _say(f"  {name:6s} rel {rel:.2e}")
        assert math.isfinite(rel) and rel <= 1e-6


def _branches(oracle_mod, p, st, f0, rho_b):
    q = dataclasses.replace(p, rho_gas=rho_b)
    o = oracle_mod.Oracle(q, state={"flags": st["flags"], "f": f0, "mass": st["mass"], "phi": st["phi"]})
    o.set_freeze(True)
    o.step(T, 1)
    return o.branch_stats()


def test_adjoint_vs_central_difference_fp64(fs, oracle_mod, case):
    """Central differences of the GPU's own FP64 forward window, with steps
    for which the oracle's branch record shows the +-h runs taking the base
    run's branch at every link-distance clamp and FSK fallback: then the
    difference is the derivative of one smooth branch and must agree to 1e-6."""
    import torch
    _say("case adjoint fp64 FSL vs GPU central differences")
    p, st, tg, dirs = case
    gr = _gpu_grad(fs, case, 1)
    iface = st["flags"] == W.INTERFACE

    def loss_at(f0, rho_b):
        sim = fs.Sim(p, st["flags"], precision="fp64")
        sim.set_state(f0, st["mass"], st["phi"])
        sim.set_forcing(p.g, rho_b)
        sim.window(T, 1)
        out = sim.fields(("f", "phi"), device=True)
        g = torch.tensor(p.g, dtype=torch.float64, device=sim.device)
        L = float(_loss(torch, out["f"], out["phi"], g, iface, tg))
        sim.close()
        return L

    base = _branches(oracle_mod, p, st, st["f"], p.rho_gas)
    h = 1e-6
    for sgn in (1, -1):
        assert _branches(oracle_mod, p, st, st["f"] + sgn * h * dirs["f"], p.rho_gas) == base
    fd = (loss_at(st["f"] + h * dirs["f"], p.rho_gas) - loss_at(st["f"] - h * dirs["f"], p.rho_gas)) / (2 * h)
    ad = float((gr["f"] * dirs["f"]).sum())
    _say("  f0    adjoint", ad, "fd", fd, "rel", abs(ad - fd) / abs(fd))
    assert math.isfinite(ad) and abs(ad - fd) <= 1e-6 * abs(fd)
    hr = 1e-5 * p.rho_gas
    for sgn in (1, -1):
        assert _branches(oracle_mod, p, st, st["f"], p.rho_gas + sgn * hr) == base
    fd = (loss_at(st["f"], p.rho_gas + hr) - loss_at(st["f"], p.rho_gas - hr)) / (2 * hr)
    ad = gr["P_b"] / 3.0
    _say("  rho_b adjoint", ad, "fd", fd, "rel", abs(ad - fd) / abs(fd))
    assert math.isfinite(ad) and abs(ad - fd) <= 1e-6 * abs(fd)


def test_checkpoint_spacing_does_not_change_the_gradient(fs, case):
    _say("case adjoint fp64 FSL: checkpoint spacings 1, 3, 20 and the default")
    ref = _gpu_grad(fs, case, 1)
    for K in (1, 3, 5, T):
        gr = _gpu_grad(fs, case, 1, K=K)
        for k in ("f", "m", "phi", "g"):
            np.testing.assert_array_equal(gr[k], ref[k], err_msg=f"K={K} {k}")
        assert gr["P_b"] == ref["P_b"]
    # the default keeps every step's record when that fits in memory (here it does)
    p, st, _, _ = case
    sim = fs.Sim(p, st["flags"])
    sim.set_state(st["f"], st["mass"], st["phi"])
    win = sim.window(T, 1)
    assert win.K == T and win.checkpoints == 1
    win.close()
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("rule", [0, 1])
def test_window_interface_kernels_agree(fs, case, monkeypatch, precision, rule):
    """The window's forward steps record their interface cells with the
    four-lanes-per-cell kernel (the default) or with the one-lane kernel
    (FSLBM_IFACE_QUAD=0).  FP64: the same gradient bit for bit (the two
    kernels compute the same bits, and the recorded value pulled from a gas
    source, which only the one-lane kernel loads, is never read by the
    reverse step).  FP32: the two kernels sum in different orders, so the
    gradients agree to the FP32 rounding, well inside 1e-3."""
    _say(f"case adjoint window interface kernels {precision} rule {rule}")
    monkeypatch.setenv("FSLBM_IFACE_QUAD", "0")
    g1 = _gpu_grad(fs, case, rule, precision=precision)
    monkeypatch.delenv("FSLBM_IFACE_QUAD")
    g4 = _gpu_grad(fs, case, rule, precision=precision)
    for k in ("f", "m", "phi", "g"):
        if precision == "fp64":
            np.testing.assert_array_equal(g4[k], g1[k], err_msg=k)
        else:
            rel = np.linalg.norm(g4[k] - g1[k]) / np.linalg.norm(g1[k])
            _say(f"  {k} relative difference {rel:.2e}")
            assert rel <= 1e-3, k
    if precision == "fp64":
        assert g4["P_b"] == g1["P_b"] and g4["L"] == g1["L"]
    else:
        assert abs(g4["P_b"] - g1["P_b"]) <= 1e-3 * abs(g1["P_b"])


def test_fp32_gradient_error_stated(fs, case):
    _say("case adjoint fp32 vs fp64 gradient")
    g64 = _gpu_grad(fs, case, 1)
    g32 = _gpu_grad(fs, case, 1, precision="fp32")
    errs = {}
    for k in ("f", "m", "phi", "g"):
        errs[k] = float(np.linalg.norm(g32[k] - g64[k]) / np.linalg.norm(g64[k]))
    errs["P_b"] = abs(g32["P_b"] - g64["P_b"]) / abs(g64["P_b"])
    _say("  fp32 relative gradient error", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(math.isfinite(v) for v in errs.values()) and max(errs.values()) < 1e-2


def test_no_interface_cells(fs, oracle_mod):
    """A liquid-only periodic box: the adjoint is the liquid sweep alone."""
    import torch
    _say("case adjoint fp64, 12x10x8 periodic liquid box")
    p = W.Params(nx=12, ny=10, nz=8, periodic=(1, 1, 1), tau=0.6, g=(1e-5, -2e-5, 3e-6))
    N = p.n_cells
    rng = np.random.default_rng(5)
    flags = np.full(N, W.LIQUID, dtype=np.uint8)
    rho = 1.0 + 1e-3 * rng.normal(size=N)
    u = 1e-3 * rng.normal(size=(3, N))
    o = oracle_mod.Oracle(p, flags, rho, u, np.ones(N))
    st = {"f": o.populations(), "mass": np.zeros(N), "phi": np.zeros(N), "flags": flags}
    a = rng.normal(size=(19, N))
    d = rng.normal(size=(19, N))
    sim = fs.Sim(p, flags, precision="fp64")
    dev = sim.device
    leaf = lambda v: torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True)  # noqa: E731
    f0, m0, phi0, P_b, g = leaf(st["f"]), leaf(st["mass"]), leaf(st["phi"]), leaf(1.0 / 3.0), leaf(np.array(p.g))
    fT, _, _ = fs.window_apply(sim, 15, 1, f0, m0, phi0, P_b, g, K=4)
    L = (torch.as_tensor(a, device=dev) * fT).sum()
    L.backward()
    zero_u, zero_p = np.zeros((3, N)), np.zeros(N)
    for name, kw, gpu in (("f0", dict(df0=d), float((f0.grad.cpu().numpy() * d).sum())),
                          ("gx", dict(dg=[1.0, 0, 0]), float(g.grad[0])), ("gz", dict(dg=[0, 0, 1.0]), float(g.grad[2]))):
        _, ref = oracle_mod.window_dual(p, flags, st["f"], st["mass"], st["phi"], zero_u, zero_p, 15, 1,
                                        f_weight=a, **kw)
        rel = abs(gpu - ref) / abs(ref)
        _say(f"  {name} rel {rel:.2e}")
        assert math.isfinite(rel) and rel <= 1e-6
    assert float(P_b.grad) == 0.0
    sim.close()


def test_window_errors(fs, case):
    p, st, _, _ = case
    s16 = fs.Sim(p, st["flags"], precision="fp16s")
    with pytest.raises(fs.FslbmError, match="UNSUPPORTED"):
        s16.window(5, 1)
    s16.close()
    s = fs.Sim(p, st["flags"], precision="fp64")
    s.set_state(st["f"], st["mass"], st["phi"])
    with pytest.raises(fs.FslbmError, match="INVALID"):
        s.window(0, 1)
    with pytest.raises(fs.FslbmError, match="INVALID"):
        s.window(5, 7)  # unknown rule
    for rule in (fs.FSK_STRESS, fs.FSL_STRESS, fs.FSK_SHEAR, fs.FSL_SHEAR):  # no adjoint of the D term
        with pytest.raises(fs.FslbmError, match="UNSUPPORTED"):
            s.window(5, rule)
    s.close()
    import dataclasses
    st_ = fs.Sim(dataclasses.replace(p, sigma=1e-3), st["flags"], precision="fp64")
    st_.set_state(st["f"], st["mass"], st["phi"])
    with pytest.raises(fs.FslbmError, match="UNSUPPORTED"):  # no adjoint of the curvature
        st_.window(5, 1)
    st_.close()
    sp = fs.Sim(dataclasses.replace(p, plic=1), st["flags"], precision="fp64")
    sp.set_state(st["f"], st["mass"], st["phi"])
    with pytest.raises(fs.FslbmError, match="UNSUPPORTED"):  # no adjoint of the plane offset
        sp.window(5, 1)
    sp.close()


def test_full_size_against_oracle_golden(fs, oracle_mod):
    """Configuration of the adjoint at its own size: 128 x 96 x 128 sloshing
    tank, T = 400 frozen FSL steps, loss against a seed-generated target run
    (tests/golden/make_adjoint_slosh128.py, which calls only the oracle).

    - The target run is repeated on the GPU in FP64 from the same seeded
      inputs; its interface-cell velocities and fills must hash to the oracle's
      (the GPU's FP64 window forward is the oracle's bit for bit).
    - FP64 adjoint: L, dL/drho_b, dL/dg and the derivative along a seeded
      direction of f0 within 1e-6 of the oracle's dual numbers (the same
      derivative computed in a different order; measured near 1e-12).
    - Central differences: along g_y a relative step of 1e-6 keeps every
      link-distance clamp and FSK fallback on the base run's branch (the
      oracle's branch record in the golden file), so the difference must agree
      to 1e-6.  Along rho_b no step does: the record shows the +-h runs crossing
      about 10^2..10^4 clamp decisions at h = 1e-7..1e-5 (the loss has kinks
      everywhere along rho_b), so that difference is reported, not asserted.
    - FP32 gradient error against FP64 stated; forward and backward timed."""
    import hashlib
    import json
    import os
    import torch
    sys_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    gold = json.load(open(os.path.join(sys_path, "adjoint_slosh128.json")))
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_adjoint_slosh128",
                                                  os.path.join(sys_path, "make_adjoint_slosh128.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    TT = gold["T"]
    p, st = mk.base_case()                      # oracle initial state (no steps)
    N = p.n_cells
    it = st["flags"] == W.INTERFACE
    _say(f"case adjoint full size {p.nx}x{p.ny}x{p.nz} T={TT} ({int(it.sum())} interface cells)")
    pt, f_t = mk.target_inputs(p, st)
    tgt = fs.Sim(p, st["flags"])
    tgt.set_state(f_t, st["mass"], st["phi"])
    tgt.set_forcing(pt.g, pt.rho_gas)
    tgt.window(TT, 1)
    out = tgt.fields(("f", "phi"))
    tgt.close()
    tg_u, tg_phi = mk.velocity(out["f"][:, it], pt.g), out["phi"][it]
    tb = np.concatenate([tg_u.ravel(), tg_phi])
    np.testing.assert_allclose(tg_u.sum(axis=1), gold["target"]["sum_u"], rtol=1e-12, atol=1e-15)
    assert abs(float((tb ** 2).sum()) - gold["target"]["sumsq"]) <= 1e-12 * gold["target"]["sumsq"]
    same_bits = hashlib.sha256(tb.tobytes()).hexdigest() == gold["target"]["sha256_u_phi"]
    _say(f"  target run: same bits as the oracle's: {same_bits}")
    assert same_bits
    tg = {"u": np.zeros((3, N)), "phi": np.zeros(N)}
    tg["u"][:, it] = tg_u
    tg["phi"][it] = tg_phi
    dvec = mk.f0_direction(p, st)

    def grad(precision):
        sim = fs.Sim(p, st["flags"], precision=precision)
        dev = sim.device
        leaf = lambda a: torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True)  # noqa: E731
        f0, m0, phi0 = leaf(st["f"]), leaf(st["mass"]), leaf(st["phi"])
        P_b = leaf(p.rho_gas / 3.0)
        g = leaf(np.array(p.g, dtype=np.float64))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fT, mT, phiT = fs.window_apply(sim, TT, 1, f0, m0, phi0, P_b, g)
        L = _loss(torch, fT, phiT, g, it, tg, with_linear=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = {"L": float(L.detach()), "P_b": float(P_b.grad), "g": g.grad.cpu().numpy(),
               "df": float((f0.grad.cpu().numpy() * dvec).sum()), "f": f0.grad.detach().clone(),
               "t_fwd": t1 - t0, "t_bwd": t2 - t1}
        sim.close()
        return out

    g64 = grad("fp64")
    _say(f"  fp64 L {g64['L']:.10e} dL/dP_b {g64['P_b']:.10e} dL/dg {g64['g']}  "
         f"fwd {g64['t_fwd']*1e3:.1f} ms bwd {g64['t_bwd']*1e3:.1f} ms")
    checks = [("L", g64["L"], gold["L"]), ("dL/drho_b", g64["P_b"] / 3.0, gold["dL_drho_b"]),
              ("dL/df0.d", g64["df"], gold["dL_df0_along_direction"])]
    checks += [(f"dL/dg_{a}", float(g64["g"][i]), gold["dL_dg"][i]) for i, a in enumerate("xyz")]
    for name, got, want in checks:
        rel = abs(got - want) / abs(want)
        _say(f"  {name:10s} gpu {got:.12e} oracle {want:.12e} rel {rel:.2e}")
        assert math.isfinite(rel) and rel <= 1e-6, name

    def loss_at(rho_b, gv):
        sim = fs.Sim(p, st["flags"], precision="fp64")
        sim.set_state(st["f"], st["mass"], st["phi"])
        sim.set_forcing(gv, rho_b)
        sim.window(TT, 1)
        out = sim.fields(("f", "phi"), device=True)
        L = float(_loss(torch, out["f"], out["phi"], torch.tensor(gv, dtype=torch.float64, device=sim.device),
                        it, tg, with_linear=False))
        sim.close()
        return L

    row = next(r for r in gold["fd"]["g_y"] if r["h_rel"] == 1e-6)
    assert row["same_branches_as_base"]
    hg = 1e-6 * abs(p.g[1])
    gp, gm = list(p.g), list(p.g)
    gp[1] += hg
    gm[1] -= hg
    fd = (loss_at(p.rho_gas, gp) - loss_at(p.rho_gas, gm)) / (2 * hg)
    ad = float(g64["g"][1])
    _say(f"  g_y   adjoint {ad:.10e} fd {fd:.10e} rel {abs(ad - fd) / abs(fd):.2e} (one branch)")
    assert abs(ad - fd) <= 1e-6 * abs(fd)
    hr = 1e-6 * p.rho_gas
    fd = (loss_at(p.rho_gas + hr, p.g) - loss_at(p.rho_gas - hr, p.g)) / (2 * hr)
    ad = g64["P_b"] / 3.0
    row = next(r for r in gold["fd"]["rho_b"] if r["h_rel"] == 1e-6)
    _say(f"  rho_b adjoint {ad:.10e} fd {fd:.10e} rel {abs(ad - fd) / abs(fd):.2e} (crosses "
         f"{row['branches_plus']['clamp0'] - gold['base_branches']['clamp0']:+d} / "
         f"{row['branches_minus']['clamp0'] - gold['base_branches']['clamp0']:+d} clamps; oracle fd rel "
         f"{row['rel_err_vs_dual']:.2e})")

    g32 = grad("fp32")
    ef = float(torch.linalg.norm(g32["f"] - g64["f"]) / torch.linalg.norm(g64["f"]))
    eP = abs(g32["P_b"] - g64["P_b"]) / abs(g64["P_b"])
    eg = float(np.linalg.norm(g32["g"] - g64["g"]) / np.linalg.norm(g64["g"]))
    _say(f"  fp32 gradient error: f0 {ef:.2e}  P_b {eP:.2e}  g {eg:.2e}")
    _say(f"  fp32 fwd {g32['t_fwd']*1e3:.1f} ms bwd {g32['t_bwd']*1e3:.1f} ms")
    assert math.isfinite(ef) and ef < 0.1


@pytest.mark.gpu
def test_many_interface_cells_fd_and_spacing(fs):
    """512 x 48 x 512 tank with ~286 K interface cells: more than one grid of
    the four-lanes-per-cell interface kernel (16 K blocks x 16 cells), so some
    wavefronts take a second pass of its loop.  FP64, T = 4: adjoint against
    central differences for rho_b and a random direction of f0, and the same
    gradient bit for bit with two checkpoint spacings."""
    import torch
    w = W.sloshing(512, 48, 512, depth=24.0, amp=10.0, amp_z=8.0, seed=0)
    p = w.params
    n_if = int((w.flags == W.INTERFACE).sum())
    assert n_if > 16384 * 16
    TT = 4
    _say(f"case adjoint many interface cells {p.nx}x{p.ny}x{p.nz} ({n_if} interface) T={TT}")
    ref = fs.Sim.from_workload(w)
    base = ref.fields(("f", "mass", "phi", "flags"), device=True)
    ref.close()
    dev = base["f"].device
    gen = torch.Generator(device=dev).manual_seed(11)
    act = (base["flags"] != W.GAS).to(torch.float64)
    a = torch.randn(base["f"].shape, dtype=torch.float64, device=dev, generator=gen) * act
    d = torch.randn(base["f"].shape, dtype=torch.float64, device=dev, generator=gen) * act
    b = torch.randn(base["phi"].shape, dtype=torch.float64, device=dev, generator=gen) * (base["flags"] == W.INTERFACE)

    def loss(fT, phiT):
        return (a * fT).sum() + (b * phiT).sum()

    def grad(K):
        sim = fs.Sim(p, w.flags)
        f0 = base["f"].clone().requires_grad_(True)
        P_b = torch.tensor(p.rho_gas / 3.0, dtype=torch.float64, device=sim.device, requires_grad=True)
        g = torch.tensor(p.g, dtype=torch.float64, device=sim.device, requires_grad=True)
        fT, _, phiT = fs.window_apply(sim, TT, 1, f0, base["mass"], base["phi"], P_b, g, K=K)
        loss(fT, phiT).backward()
        out = {"df": float((f0.grad * d).sum()), "P_b": float(P_b.grad), "f": f0.grad.detach().clone()}
        sim.close()
        return out

    def loss_at(f0, rho_b):
        sim = fs.Sim(p, w.flags)
        sim.set_state(f0, base["mass"], base["phi"])
        sim.set_forcing(p.g, rho_b)
        sim.window(TT, 1)
        out = sim.fields(("f", "phi"), device=True)
        L = float(loss(out["f"], out["phi"]))
        sim.close()
        return L

    g2 = grad(0)  # K = ceil(sqrt(4)) = 2: two segments, one recomputed
    g4 = grad(TT)  # every step's record kept
    assert torch.equal(g2["f"], g4["f"]) and g2["P_b"] == g4["P_b"]
    hr = 1e-7 * p.rho_gas
    fd = (loss_at(base["f"], p.rho_gas + hr) - loss_at(base["f"], p.rho_gas - hr)) / (2 * hr)
    ad = g2["P_b"] / 3.0
    _say(f"  rho_b adjoint {ad:.10e} fd {fd:.10e} rel {abs(ad - fd) / abs(fd):.2e}")
    assert abs(ad - fd) <= 1e-5 * abs(fd)
    # over T = 4 steps a step of 1e-7 along f0 moves few link distances (measured agreement 7e-12)
    h = 1e-7
    fd = (loss_at(base["f"] + h * d, p.rho_gas) - loss_at(base["f"] - h * d, p.rho_gas)) / (2 * h)
    ad = g2["df"]
    _say(f"  f0 dir adjoint {ad:.10e} fd {fd:.10e} rel {abs(ad - fd) / abs(fd):.2e}")
    assert abs(ad - fd) <= 1e-5 * abs(fd)
