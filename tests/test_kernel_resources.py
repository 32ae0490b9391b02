"""Register budget of the gfx950 kernels, from the compiler's resource remarks.

The face kernels must stay spill-free at the occupancy they were designed for (2D FP64
at three waves per SIMD, 3D FP64 at two, every FP32-flux variant at four): a spill means
the flux path stopped being inlined or grew, and costs scratch traffic on every face."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def remarks(tmp_path_factory):
    from paper_1302_2132_amd import build as B
    out = tmp_path_factory.mktemp("res") / "libgks_res.so"
    cmd = [B.HIPCC] + B.FLAGS + ["-Rpass-analysis=kernel-resource-usage", "-o", str(out),
                                 os.path.join(B.CSRC, "gks_lib.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    res, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            res[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]+\])?: (\d+)", line)
        if m and name:
            res[name][m.group(1).strip()] = int(m.group(2))
    return res


def _face(res, r, d):
    return {k: v for k, v in res.items() if re.match(rf"_ZN3gks6k_faceI{r}Li{d}ELi\d+EEEvPKvii", k)}


@pytest.mark.parametrize("d,waves", [(2, 3), (3, 2)])
def test_fp64_face_kernels_fit_without_spill(remarks, d, waves):
    ks = _face(remarks, "d", d)
    assert len(ks) == 3
    for k, v in ks.items():
        assert v["ScratchSize"] == 0, (k, v)
        assert v["Occupancy"] >= waves, (k, v)


@pytest.mark.parametrize("d", [2, 3])
def test_fp32_face_kernels_fit_four_waves_without_spill(remarks, d):
    ks = _face(remarks, "f", d)
    assert len(ks) == 3
    for k, v in ks.items():
        assert v["ScratchSize"] == 0, (k, v)
        assert v["Occupancy"] >= 4, (k, v)


def test_cell_kernels_do_not_spill(remarks):
    for k, v in remarks.items():
        if any(s in k for s in ("k_strain", "k_update", "k_finish", "k_rate")):
            assert v["ScratchSize"] == 0, (k, v)
