"""GPU parity on degenerate and ragged shapes, every precision form.

* one embedding orbital (npair = 1) with a single fitting function;
* two orbitals (npair = 3) on an odd 1x1x3 mesh with nao = 9 (padded to 16)
  and a non-self-conjugate q pair;
* UHF with unequal random alpha / beta orbitals on a 2x1x1 mesh.

The embedding coefficients are random real C^R Fourier transformed by the
oracle's convention (C^k = sum_R exp(-i k.R) C^R), so the ERIs are real.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kspace as ok
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": None, "fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 1e-5, "bf16x6_i8": 1e-6}

SHAPES = {
    # name: (kmesh, nao, naux, neo, nspin, seed)
    "one_orbital": ((2, 1, 1), 3, 1, 1, 1, 31),
    "odd_mesh": ((1, 1, 3), 9, 3, 2, 1, 32),
    "uhf_small": ((2, 1, 1), 5, 4, 3, 2, 33),
}


@pytest.fixture(scope="module")
def dmet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_08596_amd import dmet as d
    d.load()
    return d


def _inputs(name):
    kmesh, nao, naux, neo, nspin, seed = SHAPES[name]
    wl = synth.Workload(name, kmesh, nao, naux, nao, nao, 1, 1.5, seed)
    lm = synth.three_index(wl)
    rng = np.random.default_rng(seed)
    nk = int(np.prod(kmesh))
    c_k = np.stack([ok.emb_coeffs_k(rng.standard_normal((nk, nao, neo)) / np.sqrt(nk * nao), kmesh)
                    for _ in range(nspin)])
    return kmesh, nao, naux, neo, lm, c_k


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3", "bf16x6_i8"])
@pytest.mark.parametrize("name", list(SHAPES))
def test_degenerate_shapes(dmet, name, prec):
    kmesh, nao, naux, neo, lm, c_k = _inputs(name)
    out = dmet.dmet_transform_eri(kmesh, nao, naux, to_dev(lm), to_dev(c_k), prec)
    torch.cuda.synchronize()
    blocks = {"aa": (0, None)} if c_k.shape[0] == 1 else {"aa": (0, None), "bb": (1, None), "ab": (0, 1)}
    for key, (a, b) in blocks.items():
        ref, im = ok.alg1_eri(lm, c_k[a], kmesh, None if b is None else c_k[b])
        assert im < 1e-12 * max(1.0, np.abs(ref).max())
        ref = ok.pack_s8(ref) if b is None else ok.pack_s4(ref)
        got = out[key].cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref).max()
        tol = TOL[prec] if TOL[prec] is not None else 1e-10 * np.abs(ref).max()
        print(f"{name} {prec} {key} npair {neo * (neo + 1) // 2} max abs err {err:.3e}")
        assert err < tol, (key, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3", "bf16x6_i8"])
def test_nonfinite_input_gives_nan_output(dmet, prec):
    """The ERI entry points are asynchronous and report no input check: a NaN
    in a block of the 3-index tensor that the transform reads must come out as
    NaN ERIs (never as finite numbers), in every form; clean input stays finite."""
    kmesh, nao, naux, neo, lm, c_k = _inputs("odd_mesh")
    lm = lm.copy()
    lm[0, 0, 0, 0, 0] = np.nan                  # (q = 0, k = 0) is read by every form
    out = dmet.dmet_transform_eri(kmesh, nao, naux, to_dev(lm), to_dev(c_k), prec)
    torch.cuda.synchronize()
    assert bool(torch.isnan(out["aa"]).any()), prec
    clean = dmet.dmet_transform_eri(kmesh, nao, naux, to_dev(_inputs("odd_mesh")[4]), to_dev(c_k), prec)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(clean["aa"]).all()), prec


def test_int8_contraction_in_chunks(dmet, monkeypatch):
    """Z longer than one int8 launch: forced 64-row chunks (3 on 160 rows) agree
    with the oracle and, to FP64 rounding, with one chunk; and a 4x4x4 mesh with
    700 fitting functions (44800 rows, above the 44032 of one launch) runs in two
    chunks and agrees with the oracle."""
    wl = synth.Workload("chunks", (2, 2, 1), 6, 40, 6, 6, 1, 1.5, 41)
    lm = synth.three_index(wl)
    rng = np.random.default_rng(41)
    ck = np.stack([ok.emb_coeffs_k(rng.standard_normal((wl.nk, wl.nao, 5)) / np.sqrt(wl.nk * wl.nao), wl.kmesh)])
    whole = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(ck), "bf16x6_i8")["aa"].cpu().numpy()
    monkeypatch.setenv("DMET_I8_CHUNK_ROWS", "64")
    parts = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(ck), "bf16x6_i8")["aa"].cpu().numpy()
    monkeypatch.delenv("DMET_I8_CHUNK_ROWS")
    ref, _ = ok.alg1_eri(lm, ck[0], wl.kmesh)
    refp = ok.pack_s8(ref)
    assert np.abs(parts - whole).max() < 1e-13 * np.abs(refp).max()
    assert np.abs(parts - refp).max() < 1e-6 * max(1.0, np.abs(refp).max())
    wl = synth.Workload("k64", (4, 4, 4), 2, 700, 2, 2, 1, 1.5, 42)
    lm = synth.three_index(wl)
    rng = np.random.default_rng(42)
    ck = np.stack([ok.emb_coeffs_k(rng.standard_normal((wl.nk, wl.nao, 2)) / np.sqrt(wl.nk * wl.nao), wl.kmesh)])
    got = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(ck), "bf16x6_i8")["aa"].cpu().numpy()
    ref, _ = ok.alg1_eri(lm, ck[0], wl.kmesh)
    refp = ok.pack_s8(ref)
    err = np.abs(got - refp).max()
    print(f"44800 rows, int8 contraction in two chunks: max err {err:.3e} (max {np.abs(refp).max():.3f})")
    assert err < 1e-6 * max(1.0, np.abs(refp).max())
