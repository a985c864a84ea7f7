"""GPU bath construction (Eqs. bath R SVD, C loemb R / k) against the oracle at
the shapes that select each form of the Jacobi SVD:

* one column block (3 SVD columns, the partner block missing);
* the NiO-like shape (1050 x 150 per spin, two spins), the block form with
  8-column blocks at the size the benchmark runs;
* the Si-like shape (1352 x 52), too many rows for 8-column blocks in LDS,
  which takes 4-column blocks;
* more environment rows than the block form stages in LDS (2520 x 40 on a
  4x4x4 mesh), which takes the per-pair form.

Gauge-free comparisons as in the parity tests: singular values, the EO
projector C^k C^k^H per k, orthonormality, the identity impurity block; and a
second call must give the same bits.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kspace as ok
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

SHAPES = {
    # name: (kmesh, nao, nspin, seed)
    "one_block": ((2, 1, 1), 3, 1, 41),
    "nio": ((2, 2, 2), 150, 2, 1003),
    "si": ((3, 3, 3), 52, 1, 1002),
    "many_rows": ((4, 4, 4), 40, 1, 77),
}


@pytest.fixture(scope="module")
def dmet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_08596_amd import dmet as d
    d.load()
    return d


@pytest.mark.parametrize("name", list(SHAPES))
def test_bath_forms(dmet, name):
    kmesh, nao, nspin, seed = SHAPES[name]
    wl = synth.Workload(name, kmesh, nao, 4, nao, nao, nspin, 1.5, seed)
    lat = synth.make_lattice(wl)
    ref = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    nk = int(np.prod(kmesh))
    print(f"bath {name}: {(nk - 1) * nao} rows x {nao} columns, nspin {nspin}", flush=True)
    dm = to_dev(lat.dm_k)
    ck, sv, neo = dmet.dmet_build_bath(wl.kmesh, wl.nao, dm)
    ck2, sv2, _ = dmet.dmet_build_bath(wl.kmesh, wl.nao, dm)
    torch.cuda.synchronize()
    assert neo == list(ref["neo"]) == [2 * nao] * nspin
    assert torch.equal(ck, ck2) and torch.equal(sv, sv2)
    sv = sv.cpu().numpy()
    assert np.abs(sv - ref["sigma"]).max() < 1e-12
    ck = ck.cpu().numpy()
    eye = np.broadcast_to(np.eye(nao), ck[..., :nao].shape)
    assert np.abs(ck[..., :nao] - eye).max() < 1e-14
    p_gpu = np.einsum("skmi,skni->skmn", ck, ck.conj())
    p_ref = np.einsum("skmi,skni->skmn", ref["c_k"], ref["c_k"].conj())
    assert np.abs(p_gpu - p_ref).max() < 1e-10
    s = np.einsum("skmi,skmj->sij", ck.conj(), ck) / nk
    assert np.abs(s - np.eye(2 * nao)).max() < 1e-12
