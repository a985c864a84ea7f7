"""Host-side tests of the C ABI: the library loads, exports every symbol of
include/dmet.h, and validates arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_08596_amd import dmet
    if not os.path.exists(dmet.LIB_PATH):
        pytest.skip("libdmet.so not built")
    return dmet.load()


def test_exports_match_header(lib):
    from paper_1909_08596_amd import dmet
    hdr = open(os.path.join(ROOT, "include", "dmet.h")).read()
    declared = set(re.findall(r"\b(dmet_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(dmet.EXPORTS)
    for name in declared:
        assert hasattr(lib, name)


def test_version(lib):
    assert lib.dmet_version() >= 100


def _lat(kmesh=(2, 2, 1), nao=8, naux=40, nspin=1):
    from paper_1909_08596_amd import dmet
    return dmet.lattice(kmesh, nao, naux, nspin)


def test_eri_argument_validation(lib):
    nb = ctypes.c_size_t()
    assert lib.dmet_transform_eri_workspace(ctypes.byref(_lat()), 16, 0, 0, ctypes.byref(nb)) == 0
    assert nb.value > 0
    assert lib.dmet_transform_eri_workspace(ctypes.byref(_lat()), 0, 0, 0, ctypes.byref(nb)) == 1
    assert b"neo" in lib.dmet_last_error()
    assert lib.dmet_transform_eri_workspace(ctypes.byref(_lat()), 16, 9, 0, ctypes.byref(nb)) == 1
    assert lib.dmet_transform_eri_workspace(ctypes.byref(_lat(kmesh=(0, 1, 1))), 16, 0, 0, ctypes.byref(nb)) == 1
    assert lib.dmet_transform_eri_workspace(ctypes.byref(_lat(nspin=3)), 16, 0, 0, ctypes.byref(nb)) == 1
    # null pointers and spin-block consistency are rejected before any launch
    assert lib.dmet_transform_eri(ctypes.byref(_lat()), 16, None, 0, None, 0, None, None, None, None, 0, None) == 1
    fake = ctypes.c_void_p(0x1000)
    st = lib.dmet_transform_eri(ctypes.byref(_lat()), 16, fake, 0, fake, 0, fake, fake, None, fake, 1 << 30, None)
    assert st == 1 and b"nspin == 1" in lib.dmet_last_error()
    st = lib.dmet_transform_eri(ctypes.byref(_lat(nspin=2)), 16, fake, 0, fake, 0, fake, None, None, fake, 1 << 30,
                                None)
    assert st == 1 and b"eri_bb" in lib.dmet_last_error()
    st = lib.dmet_transform_eri(ctypes.byref(_lat()), 16, fake, 0, fake, 0, fake, None, None, None, 0, None)
    assert st == 6


def test_bath_argument_validation(lib):
    nb = ctypes.c_size_t()
    assert lib.dmet_build_bath_workspace(ctypes.byref(_lat()), 8, 8, ctypes.byref(nb)) == 0
    assert lib.dmet_build_bath_workspace(ctypes.byref(_lat()), 8, 9, ctypes.byref(nb)) == 1
    fake = ctypes.c_void_p(0x1000)
    neo = (ctypes.c_int * 1)()
    # imp_idx == NULL needs nimp == nao
    st = lib.dmet_build_bath(ctypes.byref(_lat()), fake, 5, None, 5, None, 0.0, None, fake, fake, neo, None, fake, 1 << 20,
                             None)
    assert st == 1
    # negative tolerance
    st = lib.dmet_build_bath(ctypes.byref(_lat()), fake, 8, None, 8, None, -1.0, None, fake, fake, neo, None, fake, 1 << 20,
                             None)
    assert st == 1
    # out-of-range impurity index is caught on the host
    imp = (ctypes.c_int * 8)(*range(0, 7), 99)
    st = lib.dmet_build_bath(ctypes.byref(_lat()), fake, 8, imp, 8, None, 0.0, None, fake, fake, neo, None, fake, 1 << 20,
                             None)
    assert st == 1 and b"imp_idx" in lib.dmet_last_error()
    # repeated impurity orbital
    imp = (ctypes.c_int * 8)(0, 1, 2, 3, 4, 5, 6, 6)
    st = lib.dmet_build_bath(ctypes.byref(_lat()), fake, 8, imp, 8, None, 0.0, None, fake, fake, neo, None, fake, 1 << 20,
                             None)
    assert st == 1 and b"repeated" in lib.dmet_last_error()


def test_onebody_argument_validation(lib):
    assert lib.dmet_transform_1e(ctypes.byref(_lat()), 0, None, None, None, None, None) == 1
    assert lib.dmet_energy_1e(3, 4, None, None, None, None) == 1


def test_batched_kpoint_limit(lib):
    """The split-bf16 batched transform keeps at most 256 k-points per fragment
    (its slot tables); larger meshes are refused on the host."""
    from paper_1909_08596_amd import dmet
    fake = ctypes.c_void_p(0x1000)
    fr = (dmet.Fragment * 1)()
    fr[0].lat = _lat(kmesh=(8, 8, 8), nao=4, naux=4)
    fr[0].neo, fr[0].lmunu, fr[0].dtype, fr[0].c_k, fr[0].eri = 4, fake, 0, fake, fake
    nb = ctypes.c_size_t()
    assert lib.dmet_transform_eri_batched_workspace(1, fr, dmet.DMET_BF16X6_3M, ctypes.byref(nb)) == 7
    assert b"256 k-points" in lib.dmet_last_error()
    # FP32 batches too (checked before any branch is forked); FP64 has no such limit
    assert lib.dmet_transform_eri_batched_workspace(1, fr, dmet.DMET_FP32_3M, ctypes.byref(nb)) == 7
    assert lib.dmet_transform_eri_batched_workspace(1, fr, dmet.DMET_FP64, ctypes.byref(nb)) == 0
    fr[0].lat = _lat(kmesh=(4, 4, 4), nao=4, naux=4)
    assert lib.dmet_transform_eri_batched_workspace(1, fr, dmet.DMET_BF16X6_3M, ctypes.byref(nb)) == 0


def test_energy_mf_argument_validation(lib):
    fake = ctypes.c_void_p(16)
    assert lib.dmet_energy_mf(3, 4, fake, fake, fake, fake, None) == 1
    assert lib.dmet_energy_mf(1, 0, fake, fake, fake, fake, None) == 1
    assert lib.dmet_energy_mf(2, 4, fake, None, fake, fake, None) == 1
    assert b"null" in lib.dmet_last_error()


def test_fftdf_argument_validation(lib):
    """The plane-wave entry points check the grid against naux and the cell on
    the host (no GPU call)."""
    from paper_1909_08596_amd import dmet
    E_ARG = 1   # DMET_E_ARG
    nb = ctypes.c_size_t()
    lat = _lat(naux=216)
    good = dmet.pw_grid((6, 6, 6), (3.0, 3.0, 3.0))
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(good), 16, 0, 0,
                                                  ctypes.byref(nb)) == 0
    assert nb.value > 0
    bad_n = dmet.pw_grid((6, 6, 5), (3.0, 3.0, 3.0))          # 180 points != naux
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(bad_n), 16, 0, 0,
                                                  ctypes.byref(nb)) == E_ARG
    bad_c = dmet.pw_grid((6, 6, 6), (3.0, 0.0, 3.0))
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(bad_c), 16, 0, 0,
                                                  ctypes.byref(nb)) == E_ARG
    # a general (hexagonal) cell is accepted; linearly dependent or non-finite vectors are not
    hexa = dmet.pw_grid((6, 6, 6), ((2.6, 0, 0), (1.3, 2.25, 0), (0, 0, 3.2)))
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(hexa), 16, 0, 0,
                                                  ctypes.byref(nb)) == 0
    flat = dmet.pw_grid((6, 6, 6), ((2.6, 0, 0), (1.3, 2.25, 0), (3.9, 2.25, 0)))   # a_3 = a_1 + a_2
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(flat), 16, 0, 0,
                                                  ctypes.byref(nb)) == E_ARG
    assert b"linearly independent" in lib.dmet_last_error()
    nan = dmet.pw_grid((6, 6, 6), ((2.6, 0, 0), (1.3, float("nan"), 0), (0, 0, 3.2)))
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(nan), 16, 0, 0,
                                                  ctypes.byref(nb)) == E_ARG
    # edge lengths are the diagonal cell
    g = dmet.pw_grid((2, 3, 4), (3.0, 4.0, 5.0))
    assert [[g.cell[a][b] for b in range(3)] for a in range(3)] == [[3, 0, 0], [0, 4, 0], [0, 0, 5]]
    with pytest.raises(ValueError):
        dmet.pw_grid((2, 3, 4), ((1.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)))
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), None, 16, 0, 0, ctypes.byref(nb)) == E_ARG
    # null arrays are rejected before any launch
    assert lib.dmet_transform_eri_fftdf(ctypes.byref(lat), ctypes.byref(good), 16, None, 0, 0, None, None, None,
                                        None, None, 0, None) == E_ARG
    # precision forms: the split-bf16 ones are accepted (larger workspace than FP64), FP32 and the int8
    # contraction are not offered on the plane-wave route
    nb64 = ctypes.c_size_t()
    assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(good), 16, 0, dmet.DMET_FP64,
                                                  ctypes.byref(nb64)) == 0
    for prec in (dmet.DMET_BF16X6_3M, dmet.DMET_BF16X3_3M):
        assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(good), 16, 0, prec,
                                                      ctypes.byref(nb)) == 0
        assert nb.value > 0
    for prec in (dmet.DMET_FP32_3M, dmet.DMET_BF16X6_I8):
        assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(good), 16, 0, prec,
                                                      ctypes.byref(nb)) == 7   # DMET_E_UNSUPPORTED


def test_fftdf_row_split_workspace(lib, monkeypatch):
    """A few-tile plane-wave block has its split-bf16 contraction split over the
    rows into partial outputs kept in the workspace (added in row order
    afterwards).  At the benchmark's plane-wave shape (2x2x2 mesh, 16^3 grid,
    52 EOs: 36 output tiles of 128 x 256 for 65536 rows, so 256 // 36 = 7 splits)
    the workspace holds exactly seven packed outputs more than with the split
    turned off (DMET_ROW_SPLIT=0), up to the 256-byte alignment of its regions;
    the FP64 form is not affected."""
    from paper_1909_08596_amd import dmet
    lat = _lat(kmesh=(2, 2, 2), nao=26, naux=16 ** 3)
    grid = dmet.pw_grid((16, 16, 16), (5.1, 5.1, 5.1))

    def ws(prec):
        nb = ctypes.c_size_t()
        assert lib.dmet_transform_eri_fftdf_workspace(ctypes.byref(lat), ctypes.byref(grid), 52, 0, prec,
                                                      ctypes.byref(nb)) == 0
        return nb.value

    forms = (dmet.DMET_BF16X6_3M, dmet.DMET_BF16X3_3M)
    split = [ws(p) for p in forms]
    f64 = ws(dmet.DMET_FP64)
    monkeypatch.setenv("DMET_ROW_SPLIT", "0")
    one = [ws(p) for p in forms]
    assert ws(dmet.DMET_FP64) == f64
    npair = 52 * 53 // 2
    slices = 7 * (npair * (npair + 1) // 2) * 8
    for a, b in zip(split, one):
        assert 0 <= (a - b) - slices < 256, (a - b, slices)


def test_binding_rejects_mismatched_shapes():
    """The ctypes binding checks every tensor's extent against kmesh, nao,
    naux and neo before calling the library (a wrong shape would otherwise
    make the kernels read or write past the tensor).  CPU tensors suffice:
    the shape check comes before the device check."""
    import torch

    from paper_1909_08596_amd import dmet
    if not os.path.exists(dmet.LIB_PATH):
        pytest.skip("libdmet.so not built")
    c128, f64 = torch.complex128, torch.float64
    km = (2, 2, 1)
    with pytest.raises(ValueError, match="dm_k must have shape"):
        dmet.dmet_build_bath(km, 8, torch.zeros((1, 3, 8, 8), dtype=c128))
    with pytest.raises(ValueError, match="c_ao_lo must have shape"):
        dmet.dmet_build_bath(km, 8, torch.zeros((1, 4, 8, 8), dtype=c128), c_ao_lo=torch.zeros((4, 8, 7), dtype=c128))
    with pytest.raises(ValueError, match="device tensor"):
        dmet.dmet_build_bath(km, 8, torch.zeros((1, 4, 8, 8), dtype=c128))
    with pytest.raises(ValueError, match="op_k must have shape"):
        dmet.dmet_transform_1e(km, 8, torch.zeros((1, 4, 8, 16), dtype=c128), torch.zeros((1, 4, 8, 9), dtype=c128))
    with pytest.raises(ValueError, match="c_k must have shape"):
        dmet.dmet_transform_1e(km, 8, torch.zeros((1, 4, 9, 16), dtype=c128), torch.zeros((1, 4, 8, 8), dtype=c128))
    with pytest.raises(ValueError, match="dm_eo must have shape"):
        dmet.dmet_energy_1e(torch.zeros((1, 16, 16), dtype=f64), torch.zeros((1, 16, 15), dtype=f64))
    ck = torch.zeros((1, 4, 8, 16), dtype=c128)
    with pytest.raises(ValueError, match="lmunu must have shape"):
        dmet.dmet_transform_eri(km, 8, 40, torch.zeros((4, 4, 39, 8, 8), dtype=c128), ck)
    with pytest.raises(ValueError, match="lmunu must have shape"):
        dmet.dmet_transform_eri_df(km, 8, 40, torch.zeros((4, 3, 40, 8, 8), dtype=c128), ck)
    with pytest.raises(ValueError, match="c_k must have shape"):
        dmet.dmet_transform_eri(km, 8, 40, torch.zeros((4, 4, 40, 8, 8), dtype=c128), torch.zeros((1, 4, 9, 16), dtype=c128))
    with pytest.raises(ValueError, match="rho must have shape"):
        dmet.dmet_transform_eri_fftdf(km, 8, (6, 6, 6), (3.0, 3.0, 3.0), torch.zeros((4, 4, 215, 8, 8), dtype=c128), ck)
    with pytest.raises(ValueError, match="z must have shape"):
        dmet.dmet_fock_dc(torch.zeros((1, 160, 135), dtype=f64), torch.zeros((1, 16, 16), dtype=f64),
                          torch.zeros((1, 16, 16), dtype=f64))
    with pytest.raises(ValueError, match="f_tilde must have shape"):
        dmet.dmet_energy_mf(torch.zeros((2, 16, 16), dtype=f64), torch.zeros((1, 16, 16), dtype=f64),
                            torch.zeros((1, 16, 16), dtype=f64))
    frag = {"kmesh": km, "nao": 8, "naux": 40, "lmunu": torch.zeros((4, 4, 40, 8, 8), dtype=c128),
            "c_k": torch.zeros((4, 8, 16), dtype=c128), "eri": torch.zeros(100, dtype=f64)}
    with pytest.raises(ValueError, match="eri must hold"):
        dmet.dmet_transform_eri_batched([frag])
    frag["c_k"] = torch.zeros((4, 7, 16), dtype=c128)
    with pytest.raises(ValueError, match="c_k must have shape"):
        dmet.dmet_transform_eri_batched([frag])


def test_binding_rejects_bad_output_blocks():
    import torch

    from paper_1909_08596_amd import dmet
    with pytest.raises(ValueError, match="must hold"):
        dmet._eri_outputs({"aa": torch.zeros(10, dtype=torch.float64)}, 1, 136)
    with pytest.raises(ValueError, match="one spin"):
        dmet._eri_outputs({"aa": torch.zeros(136 * 137 // 2), "bb": torch.zeros(136 * 137 // 2)}, 1, 136)
    with pytest.raises(ValueError, match="'bb'"):
        dmet._eri_outputs({"aa": torch.zeros(136 * 137 // 2, dtype=torch.float64)}, 2, 136)


def test_int8_contraction_row_limit(lib):
    """The int8 contraction keeps exact int32 sums for at most 44032 rows
    (3 * K * 127^2 < 2^31).  A single call with more rows runs them in chunks
    (its workspace query accepts them); the batched pipeline, one contraction
    launch over all fragments, refuses a fragment above the limit on the host."""
    from paper_1909_08596_amd import dmet
    nb = ctypes.c_size_t()
    lat = _lat(kmesh=(4, 4, 4), nao=4, naux=700)           # 44800 rows
    assert lib.dmet_transform_eri_workspace(ctypes.byref(lat), 4, dmet.DMET_BF16X6_I8, 0, ctypes.byref(nb)) == 0
    assert nb.value > 0
    fake = ctypes.c_void_p(0x1000)
    fr = (dmet.Fragment * 1)()
    fr[0].lat = _lat(kmesh=(4, 4, 4), nao=4, naux=700)
    fr[0].neo, fr[0].lmunu, fr[0].dtype, fr[0].c_k, fr[0].eri = 4, fake, 0, fake, fake
    assert lib.dmet_transform_eri_batched_workspace(1, fr, dmet.DMET_BF16X6_I8, ctypes.byref(nb)) == 7
    assert b"44032" in lib.dmet_last_error()
    fr[0].lat = _lat(kmesh=(4, 4, 4), nao=4, naux=688)     # 44032 rows: accepted
    assert lib.dmet_transform_eri_batched_workspace(1, fr, dmet.DMET_BF16X6_I8, ctypes.byref(nb)) == 0