"""Writes adjoint_slosh128.json: the oracle's exact gradients of the adjoint
window on the 128 x 96 x 128 sloshing tank (T = 400 frozen FSL steps), and a
finite-difference study of the same loss.  Calls only the oracle and the seeded
input generator; nothing here runs the GPU library.

Loss (interface cells of time T): L = sum |u_T - u*|^2 + (phi_T - phi*)^2 with
u = (j - g) + g/2 from the post-collision populations.  The target (u*, phi*)
is a seed-generated run: numpy.random.default_rng(7) draws xi1, xi2 and
xi[19, N]; the target starts from f0 + 1e-4 w_q xi (active cells) with
rho_b (1 + 0.01 xi1) and g (1 + 0.01 xi2).  The direction for the initial
populations is default_rng(8).normal(size=(19, N)) on the active cells.

Gradients are the oracle's dual numbers (the exact derivative of the branch
the FP64 run takes).  The finite-difference study runs the plain FP64 oracle
at rho_b (1 +- h) and g_y (1 +- h) and records, next to each central
difference, whether both runs took the base run's branch at every link of
every step (link-distance clamps and FSK fallbacks, Oracle.branch_stats).

Run from the repository root:  python tests/golden/make_adjoint_slosh128.py
(about half an hour on 8 cores).
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1409_5645_amd import workloads as W  # noqa: E402

T = 400
RULE = oracle.FSL
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_slosh128.json")
W_Q = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
C = W.LINKS
STEPS_FD = (1e-5, 1e-6, 1e-7)


def base_case():
    w = W.config("slosh128", seed=0)
    o = oracle.Oracle.from_workload(w)
    st = {"f": o.populations(), "mass": o.mass(), "phi": o.phi(), "flags": o.flags()}
    return w.params, st


def target_inputs(p, st):
    N = p.n_cells
    act = st["flags"] != W.GAS
    rng = np.random.default_rng(7)
    xi1, xi2 = rng.normal(size=2)
    xi = rng.normal(size=(19, N))
    f_t = st["f"] + 1e-4 * W_Q[:, None] * xi * act
    pt = dataclasses.replace(p, rho_gas=p.rho_gas * (1 + 0.01 * xi1), g=tuple(v * (1 + 0.01 * xi2) for v in p.g))
    return pt, f_t


def f0_direction(p, st):
    act = st["flags"] != W.GAS
    return np.random.default_rng(8).normal(size=(19, p.n_cells)) * act


def velocity(f, g):
    """u = (j - g) + g/2 (rho_0 = 1) of post-collision populations f[19, n],
    j summed over ascending q with elementwise operations only, so that the
    same populations give the same bits on any machine."""
    j = np.zeros((3, f.shape[1]))
    for a in range(3):
        for q in range(19):
            if C[q, a] > 0:
                j[a] = j[a] + f[q]
            elif C[q, a] < 0:
                j[a] = j[a] - f[q]
    g = np.asarray(g, dtype=np.float64)[:, None]
    return (j - g) + 0.5 * g


def run_plain(p, st, f0):
    """T frozen FSL steps; interface-cell velocity and fill of time T and the
    branch record."""
    o = oracle.Oracle(p, state={"flags": st["flags"], "f": f0, "mass": st["mass"], "phi": st["phi"]})
    o.set_freeze(True)
    o.step(T, RULE)
    it = st["flags"] == W.INTERFACE
    return {"u": velocity(o.populations()[:, it], p.g), "phi": o.phi()[it], "branches": o.branch_stats()}


def loss(res, tgt):
    return float(((res["u"] - tgt["u"]) ** 2).sum() + ((res["phi"] - tgt["phi"]) ** 2).sum())


def _job(job):
    t0 = time.time()
    kind = job[0]
    p, st = base_case()
    if kind == "target":
        pt, f_t = target_inputs(p, st)
        out = run_plain(pt, st, f_t)
    elif kind == "plain":
        _, which, h = job
        q = p
        if which == "rho_b":
            q = dataclasses.replace(p, rho_gas=p.rho_gas * (1 + h))
        elif which == "g_y":
            q = dataclasses.replace(p, g=(p.g[0], p.g[1] * (1 + h), p.g[2]))
        out = run_plain(q, st, st["f"])
    else:  # dual
        _, which, tgt = job
        N = p.n_cells
        ut = np.zeros((3, N))
        ph = np.zeros(N)
        it = st["flags"] == W.INTERFACE
        ut[:, it] = tgt["u"]
        ph[it] = tgt["phi"]
        kw = {}
        if which == "rho_b":
            kw["drho_b"] = 1.0
        elif which.startswith("g"):
            dg = np.zeros(3)
            dg["xyz".index(which[1])] = 1.0
            kw["dg"] = dg
        else:
            kw["df0"] = f0_direction(p, st)
        L, dL = oracle.window_dual(p, st["flags"], st["f"], st["mass"], st["phi"], ut, ph, T, RULE, **kw)
        out = {"L": L, "dL": dL}
    print(f"  {job[:2] if kind != 'plain' else job} done in {time.time() - t0:.0f} s", flush=True)
    return out


def main():
    t0 = time.time()
    p, st = base_case()
    it = st["flags"] == W.INTERFACE
    jobs = [("target",), ("plain", "base", 0.0)]
    for which in ("rho_b", "g_y"):
        for h in STEPS_FD:
            jobs += [("plain", which, h), ("plain", which, -h)]
    nproc = int(os.environ.get("GOLDEN_PROCS", "8"))
    with mp.get_context("fork").Pool(nproc) as pool:
        res = pool.map(_job, jobs, chunksize=1)
        tgt = res[0]
        plain = {(j[1], j[2]): r for j, r in zip(jobs[1:], res[1:])}
        duals = pool.map(_job, [("dual", w, tgt) for w in ("rho_b", "gx", "gy", "gz", "f0")], chunksize=1)
    dual = dict(zip(("rho_b", "gx", "gy", "gz", "f0"), duals))
    L = dual["rho_b"]["L"]
    for d in dual.values():
        assert d["L"] == L
    base = plain[("base", 0.0)]
    assert abs(loss(base, tgt) - L) <= 1e-12 * L
    tb = np.concatenate([tgt["u"].ravel(), tgt["phi"]])
    fd = {}
    for which, scale, exact in (("rho_b", p.rho_gas, dual["rho_b"]["dL"]), ("g_y", p.g[1], dual["gy"]["dL"])):
        rows = []
        for h in STEPS_FD:
            a, b = plain[(which, h)], plain[(which, -h)]
            d = (loss(a, tgt) - loss(b, tgt)) / (2 * h * scale)
            same = a["branches"] == base["branches"] and b["branches"] == base["branches"]
            rows.append({"h_rel": h, "fd": d, "rel_err_vs_dual": abs(d - exact) / abs(exact),
                         "same_branches_as_base": same, "branches_plus": a["branches"],
                         "branches_minus": b["branches"]})
        fd[which] = rows
    out = {
        "workload": "sloshing tank 128x96x128 (depth 48, amplitude 3, seed 0), FSL, tau 0.55, g_y -2e-5",
        "T": T, "rule": "FSL", "n_interface": int(it.sum()),
        "target": {"seed": 7, "sha256_u_phi": hashlib.sha256(tb.tobytes()).hexdigest(),
                   "sum_u": [float(v) for v in tgt["u"].sum(axis=1)], "sum_phi": float(tgt["phi"].sum()),
                   "sumsq": float((tb ** 2).sum())},
        "f0_direction_seed": 8,
        "L": L, "dL_drho_b": dual["rho_b"]["dL"], "dL_dPb": 3.0 * dual["rho_b"]["dL"],
        "dL_dg": [dual["gx"]["dL"], dual["gy"]["dL"], dual["gz"]["dL"]],
        "dL_df0_along_direction": dual["f0"]["dL"],
        "base_branches": base["branches"], "fd": fd,
        "seconds": round(time.time() - t0),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: out[k] for k in ("L", "dL_drho_b", "dL_dg", "dL_df0_along_direction")}), flush=True)


if __name__ == "__main__":
    main()
