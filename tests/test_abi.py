"""The C-ABI library loads and exports every entry point include/gks.h declares; host-only
paths (workspace sizing, configuration validation, the flop count) work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from inputs import cases as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "gks.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gks_[a-z_0-9]+)\s*\(", txt)))


def test_header_and_binding_agree():
    import paper_1302_2132_amd as P
    assert sorted(P.EXPORTED) == declared()


def test_library_exports_every_declared_symbol():
    import paper_1302_2132_amd as P
    L = ctypes.CDLL(P.lib_path)
    for name in declared():
        assert hasattr(L, name), name


def test_workspace_bytes_and_validation():
    import paper_1302_2132_amd as P
    c = C.mixing_layer(64)
    nb = P.gks_workspace_bytes(P.config_from_case(c))
    # two FP64 state buffers + k, omega, strain at least (2D fluxes never leave LDS)
    assert 8 * 64 * 64 * (4 * 2 + 3) <= nb < 8 * 64 * 64 * (4 * 2 + 3) + 8 * 4 * 2 * 65 * 64
    bad = c.copy()
    bad.bc = [["periodic", "outflow"], ["periodic", "periodic"]]
    with pytest.raises(P.GksError) as e:
        P.gks_workspace_bytes(P.config_from_case(bad))
    assert e.value.status == P.GKS_ERR_ARG
    bad = c.copy()
    bad.xf = [c.xf[0][::-1].copy(), c.xf[1]]
    with pytest.raises(P.GksError):
        P.gks_workspace_bytes(P.config_from_case(bad))
    bad = c.copy()
    bad.gamma = 2.5          # fewer than D total degrees of freedom
    with pytest.raises(P.GksError):
        P.gks_workspace_bytes(P.config_from_case(bad))
    c3 = C.isotropic_box(16, precision="fp64")
    nb3 = P.gks_workspace_bytes(P.config_from_case(c3))
    # 3D, fused step: two state buffers + k, omega, strain; no face fluxes in HBM
    assert 8 * 16 ** 3 * (5 * 2 + 3) <= nb3 < 8 * 16 ** 3 * (5 * 2 + 3) + 8 * 5 * 3 * 17 * 16 * 16
    # a transported 3D solve also steps in the fused kernel: two 7-component states, k, omega,
    # strain, rho k/omega and the two sources, no face fluxes
    kw3 = c3.copy()
    kw3.kw_transport = True
    nkw = P.gks_workspace_bytes(P.config_from_case(kw3))
    assert 8 * 16 ** 3 * (7 * 2 + 6) <= nkw < 8 * 16 ** 3 * (7 * 2 + 6) + 8 * 5 * 3 * 17 * 16 * 16
    # WENO5 keeps the face-kernel path: x/y/z face fluxes (FP64) in HBM
    w3 = c3.copy()
    w3.recon = "weno5"
    assert P.gks_workspace_bytes(P.config_from_case(w3)) >= 8 * 16 ** 3 * (5 * 2 + 3) + 8 * 5 * 3 * 17 * 16 * 16
    fp32 = c3.copy()
    fp32.precision = "fp32_flux"
    assert P.gks_workspace_bytes(P.config_from_case(fp32)) == nb3    # face fluxes FP64 in both forms
    bad = c.copy()
    bad.res_tol = -1.0
    with pytest.raises(P.GksError) as e:
        P.gks_workspace_bytes(P.config_from_case(bad))
    assert e.value.status == P.GKS_ERR_ARG


def test_option_combinations_validated():
    """WENO5 needs three cells per axis; the multi-dimensional expansion takes second-order
    face values; every reconstruction and the expansion combine with transport and tau_hat."""
    import paper_1302_2132_amd as P

    def cfg(**kw):
        c = C.uniform_flow(dim=2, n=kw.pop("n", (8, 6, 1)), bc=[["periodic", "periodic"]] * 2)
        for k, v in kw.items():
            setattr(c, k, v)
        return P.config_from_case(c)

    for bad in (dict(recon="weno5", n=(2, 6, 1)), dict(recon="weno5", n=(8, 2, 1)),
                dict(multi_d=True, recon="muscl3"), dict(multi_d=True, recon="weno5")):
        with pytest.raises(P.GksError) as e:
            P.gks_workspace_bytes(cfg(**bad))
        assert e.value.status == P.GKS_ERR_ARG, bad
    for good in (dict(recon="weno5", n=(3, 3, 1)), dict(recon="weno5", kw_transport=True, eps_mode="tauhat"),
                 dict(recon="muscl3", kw_transport=True), dict(multi_d=True, kw_transport=True, eps_mode="tauhat")):
        assert P.gks_workspace_bytes(cfg(**good)) > 0, good


def test_missing_library_fails_loudly():
    """Without a built libgks.so the binding raises; nothing runs on the CPU instead."""
    import subprocess
    import sys
    code = ("import paper_1302_2132_amd.gks as G\n"
            "G.lib_path = '/nonexistent/libgks.so'\n"
            "from inputs import cases as C\n"
            "try:\n"
            "    G.Solver(C.mixing_layer(16))\n"
            "except RuntimeError as e:\n"
            "    print('raised', 'not found' in str(e))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.stdout.strip() == "raised True", (r.stdout, r.stderr[-2000:])


def test_init_validation_before_any_device_call():
    import paper_1302_2132_amd as P
    c = C.mixing_layer(16)
    cfg = P.config_from_case(c)
    with pytest.raises(P.GksError) as e:     # workspace too small
        P.gks_init(cfg, 256, 16, 0, c.W, c.k, c.omega)
    assert e.value.status == P.GKS_ERR_NOMEM
    with pytest.raises(P.GksError) as e:     # misaligned workspace
        P.gks_init(cfg, 257, 1 << 30, 0, c.W, c.k, c.omega)
    assert e.value.status == P.GKS_ERR_ARG
    # non-finite or out-of-range fields are refused on the host, before the workspace (a
    # bogus pointer here) is touched: NaN in k or omega is an argument error, NaN in the
    # flow state a non-physical one
    for field, idx, val, want in [("k", (0, 3, 5), np.nan, P.GKS_ERR_ARG), ("k", (0, 0, 0), -1e-9, P.GKS_ERR_ARG),
                                  ("k", (0, 7, 1), np.inf, P.GKS_ERR_ARG),
                                  ("omega", (0, 2, 2), np.nan, P.GKS_ERR_ARG), ("omega", (0, 1, 9), 0.0, P.GKS_ERR_ARG),
                                  ("W", (0, 0, 4, 4), np.nan, P.GKS_ERR_NONPHYSICAL),
                                  ("W", (3, 0, 1, 1), np.nan, P.GKS_ERR_NONPHYSICAL)]:
        arrs = {"W": c.W.copy(), "k": c.k.copy(), "omega": c.omega.copy()}
        arrs[field][idx] = val
        with pytest.raises(P.GksError) as e:
            P.gks_init(cfg, 256, 1 << 30, 0, arrs["W"], arrs["k"], arrs["omega"])
        assert e.value.status == want, (field, idx, val)
    with pytest.raises(P.GksError) as e:     # resume without a handle
        P.gks_resume(None, None, None, 0.0, 0.0, 0)
    assert e.value.status == P.GKS_ERR_ARG


def test_face_flop_count():
    import paper_1302_2132_amd as P
    f2, f3 = P.gks_face_flops(2), P.gks_face_flops(3)
    assert 500 < f2 < f3 < 5000
    # rho k / rho omega fluxes: face eddy viscosity 0.5 (nl + nr) (2 operations), then per
    # field frho * k_up, sigma * nut, mu + ., dt * ., (kr - kl), two products and the
    # difference (8 each)
    assert P.gks_kw_face_flops() == 18.0
    # the multi-dimensional expansion adds the tangential slopes' solves and moments
    assert f2 < P.gks_face_flops_multid(2) < P.gks_face_flops_multid(3)
    assert P.gks_face_flops_multid(3) - f3 > P.gks_face_flops_multid(2) - f2
    # reconstructions: MUSCL2 is the default count; a WENO5 value takes 70 operations (three
    # candidates 16, smoothness indicators 18 + 3 + 18, weights and mean 15) and replaces
    # the 2 of a MUSCL face value, twice per component
    for d, f in ((2, f2), (3, f3)):
        assert P.gks_face_flops_recon(d, "muscl2") == f
        assert P.gks_face_flops_recon(d, "muscl3") > f
        assert P.gks_face_flops_recon(d, "weno5") - f == (d + 2) * 2 * (70 - 2)


def test_binding_loads_torch_runtime_first():
    """After lib() and a later `import torch` the process maps one HIP runtime (loading
    libgks.so before torch used to map two, and the device was then invisible to one)."""
    import subprocess
    import sys
    code = ("import paper_1302_2132_amd as P; P.lib(); import torch; "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-1000:]
    paths = eval(r.stdout.strip().splitlines()[-1])
    assert len(paths) == 1, paths


def test_failed_init_frees_its_context():
    """A gks_init that fails after creating its context (here: the first device copy, on
    a host without a device or with a bogus workspace pointer) frees it: repeating the
    failure does not grow the process (each context holds ~1.5 KB)."""
    import subprocess
    import sys
    code = ("import ctypes\n"
            "import paper_1302_2132_amd as P\n"
            "from inputs import cases as C\n"
            "P.lib()\n"
            "n = ctypes.c_int(-1)\n"
            "ctypes.CDLL('libamdhip64.so.7').hipGetDeviceCount(ctypes.byref(n))\n"
            "assert n.value <= 0, 'a device is visible: the bogus workspace must never reach one'\n"
            "c = C.mixing_layer(4); cfg = P.config_from_case(c)\n"
            "def rss(): return int(open('/proc/self/statm').read().split()[1]) * 4096\n"
            "def fail(n):\n"
            "    for _ in range(n):\n"
            "        try: P.gks_init(cfg, 256, 1 << 30, 0, c.W, c.k, c.omega)\n"
            "        except P.GksError as e: assert e.status == P.GKS_ERR_DEVICE, e\n"
            "fail(500); r0 = rss(); fail(20000)\n"
            "print('growth', (rss() - r0) / 1e6)\n")
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    growth = float(r.stdout.split()[-1])
    assert growth < 5.0, growth          # 20000 leaked contexts would be ~30 MB


def test_entry_points_carry_marker_ranges():
    """The stepping, set-up and read-back entry points push named roctx ranges (shown by a
    profiler's marker trace, profiles/gks_step_marker_trace_sbli_1024x512.md): the library
    imports the range calls."""
    import subprocess
    from paper_1302_2132_amd.gks import lib_path
    syms = subprocess.run(["nm", "-D", lib_path], capture_output=True, text=True, check=True).stdout
    assert "roctxRangePushA" in syms and "roctxRangePop" in syms


def test_mesh_size_limits():
    """The kernels index cells and faces with 32-bit integers, so the host refuses meshes
    they cannot address before any device call: more than 2^29 cells, or an axis longer
    than 2^24 cells; it also refuses an axis of fewer than two cells, and WENO5 on an axis
    of fewer than three (its three ghost layers).  The largest accepted mesh gets a
    workspace size (two state buffers, k, omega, strain: 13 doubles a cell in 3D)."""
    import numpy as np

    import paper_1302_2132_amd as P
    base = C.isotropic_box(4, precision="fp64")          # periodic on every axis: no boundary data

    def cfg_with(n, recon="muscl2"):
        b = base.copy()
        b.recon = recon
        cfg = P.config_from_case(b)
        for d in range(3):
            xf = np.linspace(0.0, 1.0, n[d] + 1)
            cfg.keep.append(xf)
            cfg.c.n[d] = n[d]
            cfg.c.xf[d] = xf.ctypes.data
        return cfg

    def refused(cfg, why):
        with pytest.raises(P.GksError) as e:
            P.gks_workspace_bytes(cfg)
        assert e.value.status == P.GKS_ERR_ARG and why in str(e.value), str(e.value)

    nb = P.gks_workspace_bytes(cfg_with((1024, 1024, 512)))             # 2^29 cells
    assert nb >= 8 * 2 ** 29 * 13
    refused(cfg_with((1024, 1024, 513)), "too many cells")
    refused(cfg_with(((1 << 24) + 1, 2, 2)), "axis too long")
    assert P.gks_workspace_bytes(cfg_with((1 << 24, 2, 2))) > 0          # the longest axis
    refused(cfg_with((8, 1, 8)), "at least 2 cells")
    refused(cfg_with((8, 2, 8), recon="weno5"), "WENO5 needs at least 3 cells")
    assert P.gks_workspace_bytes(cfg_with((8, 3, 8), recon="weno5")) > 0
