"""Register budget of the gfx950 kernels, from the compiler's resource remarks.

The flux kernels must stay spill-free at the occupancy they were designed for.  The fused
2D tile kernel runs at three waves per SIMD in FP64; in the FP32-flux form (whose FP64
share -- the interface state, the Euler and collisionless parts of the flux -- lifts its
registers) at four for the plain scheme and three for its variants (the transported ones
are held to three by their LDS).  The 3D face kernel runs at two waves (FP64) and three
(FP32), the FP32 third-order, WENO5 and multi-dimensional forms at two.  Exceptions with a
bounded spill of a few doubles per face: the third-order and WENO5 2D FP64 tiles at three
waves (two would cost more), the multi-dimensional 3D FP64 kernel at two, and the plain
FP32-flux 2D tile at four, which holds the tile's staging loads in registers (all issued
before the first LDS store) and reloads one dword per face pass (measured faster than the
spill-free form, whose staging waited on memory once per loop pass); the
multi-dimensional expansion, with its tangential gradients, runs one wave lower in 2D.  A
spill means the flux path stopped being inlined or grew (or values derived from the thread
index were kept live across the tile loop), and costs scratch traffic to HBM on every
face."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def remarks(tmp_path_factory):
    import concurrent.futures as cf

    from paper_1302_2132_amd import build as B
    out = tmp_path_factory.mktemp("res")
    units = B.units()
    with cf.ThreadPoolExecutor(max_workers=min(len(units), os.cpu_count() or 1)) as ex:
        runs = list(ex.map(lambda u: B.compile_unit(u[0], u[1], str(out / u[2]),
                                                     ["-Rpass-analysis=kernel-resource-usage"]), units))
    for r in runs:
        assert r.returncode == 0, r.stderr[-2000:]
    res, name = {}, None
    for line in "\n".join(r.stderr for r in runs).splitlines():
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
    return {k: v for k, v in res.items() if re.match(rf"_ZN3gks6k_faceI{r}Li{d}ELi\d+ELi\d+EEEvPKvii", k)}


def _tile2(res, r):
    return {k: v for k, v in res.items() if re.match(rf"_ZN3gks7k_tile2I{r}Li\d+ELi\d+EEEvPKvii", k)}


def _variant(name):
    """Variant bits: 1 transport, 2 tau_hat, 4 third-order MUSCL, 8 multi-dimensional, 16 WENO5."""
    m = re.search(r"k_tile2I[df]Li(\d+)ELi\d+E", name)
    return int(m.group(1) if m else re.search(r"Li(\d+)EEEvPKvii$", name).group(1))


def test_fused_2d_kernels_occupancy(remarks):
    k64, k32 = _tile2(remarks, "d"), _tile2(remarks, "f")
    # transport x tau_hat x (MUSCL2, MUSCL3, WENO5, multi-d), plus the plain scheme in the
    # 32 x 7 and 8 x 28 tile shapes
    assert len(k64) == 18 and len(k32) == 18
    for k, v in k64.items():
        md = bool(_variant(k) & 8)
        # the cells' states are reread from LDS late in the flux: at most 20 bytes remain
        # (third-order without tau_hat, and the transported WENO5 forms)
        assert v["ScratchSize"] <= (24 if _variant(k) & (4 | 16) else 0), (k, v)
        assert v["Occupancy"] >= (2 if md else 3), (k, v)
    for k, v in k32.items():
        assert v["ScratchSize"] <= (8 if _variant(k) == 0 else 0), (k, v)
        want = 4 if _variant(k) == 0 else (2 if _variant(k) & 8 else 3)
        assert v["Occupancy"] >= want, (k, v)


def _tile3(res, r):
    return {k: v for k, v in res.items() if re.match(rf"_ZN3gks7k_tile3I{r}Li\d+EEEvPKvii", k)}


def test_fused_3d_kernels_fit_without_spill(remarks):
    """The fused 3D step (one flux evaluation serving its three axes) at two waves per SIMD,
    and its LDS (a four-plane ring, halo arms, k/omega/S and the fluxes of a plane) within
    half a CU's 160 KiB, so two workgroups share a CU.  No spill, except a few doubles in the
    FP64 transported forms, whose update also forms the k-omega fluxes of the cell's six
    faces (the update phase, once per cell and plane, not the flux)."""
    for r in ("d", "f"):
        ks = _tile3(remarks, r)
        # plain, tau_hat, MUSCL3, both; each frozen and transported
        assert sorted(_variant(k) for k in ks) == [0, 1, 2, 3, 4, 5, 6, 7]
        for k, v in ks.items():
            kw = bool(_variant(k) & 1)
            assert v["ScratchSize"] <= (24 if kw and r == "d" else 0), (k, v)
            assert v["Occupancy"] >= 2, (k, v)
            assert v["LDS Size"] <= 80 * 1024, (k, v)


def test_3d_face_kernels_fit_without_spill(remarks):
    for r, waves in (("d", 2), ("f", 3)):
        ks = _face(remarks, r, 3)
        assert len(ks) == 8                         # multi-d, WENO5, each alone, with transport, tau_hat
        for k, v in ks.items():
            md = bool(_variant(k) & 8)
            assert v["ScratchSize"] <= (48 if md and r == "d" else 0), (k, v)
            drop = (1 if _variant(k) & (4 | 8 | 16) else 0) if r == "f" else 0
            assert v["Occupancy"] >= waves - drop, (k, v)


def test_cell_kernels_do_not_spill(remarks):
    for k, v in remarks.items():
        if any(s in k for s in ("k_strain", "k_update", "k_finish", "k_rate", "k_eps")):
            assert v["ScratchSize"] == 0, (k, v)
