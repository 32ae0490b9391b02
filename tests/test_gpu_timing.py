"""Per-kernel timing (gks_set_timing / gks_kernel_times): every launch kind a step makes
gets a positive duration (2D steps and fused 3D steps, frozen or transported, have no
separate update launch: the tile kernels update; a WENO5 3D solve keeps it), and stamping
launches with events changes no result."""
import numpy as np
import pytest

from gpu_util import banner
from inputs import cases as C

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["2d", "3d_fused", "3d_transported", "3d_weno5"])
def test_timed_steps_match_untimed_bitwise(kind):
    import paper_1302_2132_amd as P
    case = C.mixing_layer(64, seed=5) if kind == "2d" else C.isotropic_box(16, precision="fp64")
    case.kw_transport = kind == "3d_transported"
    if kind == "3d_weno5":
        case.recon = "weno5"
    banner(f"timing: {case.name}, 2 x 15 steps")
    a = P.Solver(case)
    a.step(30)
    Wa = a.fields("cons")
    a.close()
    b = P.Solver(case)
    b.step(15)
    P.gks_set_timing(b.h, True)
    b.step(15)
    kt = P.gks_kernel_times(b.h)
    P.gks_set_timing(b.h, False)
    Wb = b.fields("cons")
    b.close()
    print(f"  kernel ms over 15 steps: {kt}", flush=True)
    assert kt["steps"] == 15
    for k in ("strain_ms", "face_ms", "finish_ms"):
        assert kt[k] > 0.0, kt
    assert (kt["update_ms"] > 0.0) == (kind == "3d_weno5"), kt
    assert np.array_equal(Wa, Wb)
