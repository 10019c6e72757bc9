"""The C-ABI library loads and exports every symbol include/fslbm.h declares
(no compute: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fslbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fslbm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1409_5645_amd import build, fslbm
    if not os.path.exists(fslbm.LIB_PATH):
        build.build()
    return fslbm.LIB_PATH


def test_header_declares_entry_points():
    names = _declared()
    for n in ("fslbm_init", "fslbm_step", "fslbm_fields", "fslbm_stats", "fslbm_conversions",
              "fslbm_set_equilibrium", "fslbm_set_state", "fslbm_destroy", "fslbm_last_error",
              "fslbm_workspace_size"):
        assert n in names


def test_library_exports_all_declared(libpath):
    lib = ctypes.CDLL(libpath)
    for n in _declared():
        assert hasattr(lib, n), n


def test_workspace_size_and_param_validation(libpath):
    from paper_1409_5645_amd import fslbm, workloads as W
    L = fslbm.lib()
    p = W.Params(nx=10, ny=12, nz=14)
    cp = fslbm.make_params(p)
    ws = ctypes.c_size_t()
    assert L.fslbm_workspace_size(ctypes.byref(cp), ctypes.byref(ws)) == 0
    assert ws.value >= 76 * 10 * 12 * 14
    for field, bad in (("tau", 0.5), ("magic", 0.0), ("precision", 7), ("nx", 0), ("abi_version", 99),
                       ("fp16_scale_log2", 40), ("rho_gas", -1.0), ("plic", 3), ("sigma", -1.0),
                       ("check_every", -1), ("u_max", -1.0), ("u_max", float("inf"))):
        cp2 = fslbm.make_params(p)
        setattr(cp2, field, bad)
        assert L.fslbm_workspace_size(ctypes.byref(cp2), ctypes.byref(ws)) == 1, field
        assert L.fslbm_last_error(None)
    # init with NULL buffers is rejected before any device work
    b = fslbm.Buffers()
    h = ctypes.c_void_p()
    assert L.fslbm_init(ctypes.byref(cp), ctypes.byref(b), ctypes.byref(h)) == 1
    assert b"NULL" in L.fslbm_last_error(None)


def test_workspace_grows_for_curvature_arrays(libpath):
    """The workspace holds one 8-byte value per cell (256-byte aligned) for the
    surface-tension correction when sigma != 0, and one more for the
    height-function curvature when plic = 2 as well, as the header states."""
    from paper_1409_5645_amd import fslbm, workloads as W
    L = fslbm.lib()
    N = 10 * 12 * 14
    pad = (8 * N + 255) // 256 * 256

    def size(**kw):
        cp = fslbm.make_params(W.Params(nx=10, ny=12, nz=14, **kw))
        ws = ctypes.c_size_t()
        assert L.fslbm_workspace_size(ctypes.byref(cp), ctypes.byref(ws)) == 0
        return ws.value

    base = size()
    assert size(plic=2) == base
    assert size(sigma=1e-3) == base + pad
    assert size(sigma=1e-3, plic=1) == base + pad
    assert size(sigma=1e-3, plic=2) == base + 2 * pad

def test_size_limit(libpath):
    """Population offsets are 32-bit: 19 N must stay below 2^32 (N up to
    226,050,910 cells); a larger lattice is rejected before any device work."""
    from paper_1409_5645_amd import fslbm, workloads as W
    L = fslbm.lib()
    ws = ctypes.c_size_t()
    ok = fslbm.make_params(W.Params(nx=1024, ny=1024, nz=215))     # 225,443,840 cells
    assert L.fslbm_workspace_size(ctypes.byref(ok), ctypes.byref(ws)) == 0
    assert ws.value > 0
    big = fslbm.make_params(W.Params(nx=1024, ny=1024, nz=216))    # 226,492,416 cells
    assert L.fslbm_workspace_size(ctypes.byref(big), ctypes.byref(ws)) == 1
    assert b"2^32" in L.fslbm_last_error(None)


def test_binding_fails_loudly_without_gpu(libpath):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1409_5645_amd import fslbm, workloads as W
    w = W.channel(nx=2, nz=2)
    with pytest.raises(RuntimeError):
        fslbm.Sim.from_workload(w)


def test_parameter_block_layout_matches_header(tmp_path):
    """The ctypes mirrors of fslbm_params and fslbm_buffers have the size and
    field offsets the C compiler gives the header's structs."""
    import subprocess
    from paper_1409_5645_amd import fslbm
    fields = [f for f, _ in fslbm.Params._fields_]
    bfields = [f for f, _ in fslbm.Buffers._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "fslbm.h"', "int main(void) {",
            'printf("%zu\\n", sizeof(fslbm_params));']
    prog += [f'printf("%zu\\n", offsetof(fslbm_params, {f}));' for f in fields]
    prog += ['printf("%zu\\n", sizeof(fslbm_buffers));']
    prog += [f'printf("%zu\\n", offsetof(fslbm_buffers, {f}));' for f in bfields]
    prog += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(fslbm.Params)] + [getattr(fslbm.Params, f).offset for f in fields]
    want += [ctypes.sizeof(fslbm.Buffers)] + [getattr(fslbm.Buffers, f).offset for f in bfields]
    assert got == want
