"""GPU parity at a single k-point: the molecular limit of the method.

With N_k = 1 there is one q and one k, and Alg. 1 reduces to plain
density-fitted ao2mo: (ij|kl) = sum_L (C^T B_L C)_ij (C^T B_L C)_kl for any
real orthonormal C, with B_L the real 3-index tensor of the cell.  An impurity
that is the whole cell leaves no environment, so the bath is empty and C is
the identity on the impurity (the oracle's build_bath gives the same).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kspace as ok
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

LP_TOL = 1e-6
WL = synth.Workload("gamma", (1, 1, 1), 10, 30, 10, 10, 2, 1.5, 91)


@pytest.fixture(scope="module")
def dmet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_08596_amd import dmet as d
    d.load()
    return d


@pytest.fixture(scope="module")
def inputs():
    lat = synth.make_lattice(WL)
    lm, b = synth.three_index(WL, real_space=True)
    return lat, lm, b.reshape(WL.naux, WL.nao, WL.nao)


def test_gamma_bath_is_the_impurity(dmet, inputs):
    lat, lm, bl = inputs
    ck, sv, neo = dmet.dmet_build_bath(WL.kmesh, WL.nao, to_dev(lat.dm_k))
    torch.cuda.synchronize()
    ref = ok.build_bath(lat.dm_k, WL.kmesh, WL.nao)
    assert neo == list(ref["neo"]) == [WL.nao] * WL.nspin
    ck = ck.cpu().numpy()
    eye = np.broadcast_to(np.eye(WL.nao), ck[..., : WL.nao].shape)
    assert np.array_equal(ck[..., : WL.nao], eye)
    assert np.array_equal(ck[..., : WL.nao], ref["c_k"])
    assert not ck[..., WL.nao:].any()
    assert not sv.cpu().numpy().any()
    # with C = 1 the embedding one-body operators are the cell's own
    c = to_dev(ck[..., : WL.nao])
    h, mi = dmet.dmet_transform_1e(WL.kmesh, WL.nao, c, to_dev(lat.h_k), want_imag=True)
    g, _ = dmet.dmet_transform_1e(WL.kmesh, WL.nao, c, to_dev(lat.dm_k))
    assert np.abs(h.cpu().numpy() - lat.h_k[:, 0].real).max() < 1e-14
    e1 = float(dmet.dmet_energy_1e(h, g).cpu())
    rh, _ = ok.transform_1e(ref["c_k"], lat.h_k)
    rg, _ = ok.transform_1e(ref["c_k"], lat.dm_k)
    assert abs(e1 - ok.energy_1e(rh, rg)) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x6_i8"])
def test_gamma_eri_is_molecular_df(dmet, inputs, prec):
    lat, lm, bl = inputs
    rng = np.random.default_rng(7)
    ca = synth.random_orthonormal(rng, WL.nao, 7)
    cb = synth.random_orthonormal(rng, WL.nao, 7)
    ck = np.stack([ca, cb])[:, None].astype(np.complex128)    # [spin][k][nao][neo]
    out = dmet.dmet_transform_eri(WL.kmesh, WL.nao, WL.naux, to_dev(lm), to_dev(ck), prec)
    torch.cuda.synchronize()
    ta = np.einsum("Lmn,mi,nj->Lij", bl, ca, ca)
    tb = np.einsum("Lmn,mi,nj->Lij", bl, cb, cb)
    refs = {"aa": ok.pack_s8(np.einsum("Lij,Lkl->ijkl", ta, ta)),
            "bb": ok.pack_s8(np.einsum("Lij,Lkl->ijkl", tb, tb)),
            "ab": ok.pack_s4(np.einsum("Lij,Lkl->ijkl", ta, tb))}
    for key, ref in refs.items():
        got = out[key].cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref).max()
        tol = 1e-10 * np.abs(ref).max() if prec == "fp64" else LP_TOL
        print(f"gamma {prec} {key} max abs err {err:.3e}")
        assert err < tol, (key, err)
