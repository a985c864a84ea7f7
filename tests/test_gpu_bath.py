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
    # the one-block lattice has a rank-deficient M (a singular value at the
    # rounding level), whose undetermined vector is dropped by both sides
    assert neo == list(ref["neo"])
    assert neo == ([2 * nao - 1] if name == "one_block" else [2 * nao] * nspin)
    assert torch.equal(ck, ck2) and torch.equal(sv, sv2)
    sv = sv.cpu().numpy()
    assert np.abs(sv - ref["sigma"]).max() < 1e-12
    ck = ck.cpu().numpy()
    eye = np.broadcast_to(np.eye(nao), ck[..., :nao].shape)
    assert np.abs(ck[..., :nao] - eye).max() < 1e-14
    n = neo[0]
    assert np.abs(ck[..., n:]).max(initial=0.0) == 0.0
    ck = ck[..., :n]
    p_gpu = np.einsum("skmi,skni->skmn", ck, ck.conj())
    p_ref = np.einsum("skmi,skni->skmn", ref["c_k"], ref["c_k"].conj())
    assert np.abs(p_gpu - p_ref).max() < 1e-10
    s = np.einsum("skmi,skmj->sij", ck.conj(), ck) / nk
    assert np.abs(s - np.eye(n)).max() < 1e-12


def _bath_columns_r(ck, nk, kmesh):
    """C^R = 1/N_k sum_k exp(+i k.R) C^k (inverse of Eq. C loemb k), real part."""
    ph = ok.phase_matrix(kmesh)                       # [k][R] = exp(i k.R)
    cr = np.einsum("kR,kmi->Rmi", ph, ck) / nk
    return cr.real, float(np.abs(cr.imag).max())


def _compare_bath(ck, sv, neo, mi, ref, kmesh, nao, imp, tol_vec=1e-9):
    """Gauge-fixed comparison with the oracle: sigma, kept count, EO
    projectors per k, identity entries on the impurity, orthonormality, the
    bath vectors themselves (sign gauge) where sigma is well separated, and
    max |Im gamma^{R,0}|."""
    nk = int(np.prod(kmesh))
    nimp = len(imp)
    sv = sv.cpu().numpy()
    assert neo == list(ref["neo"])
    assert np.abs(sv - ref["sigma"]).max() < 1e-12
    assert abs(mi - ref["max_imag_dm"]) < 1e-14 and mi < 1e-12
    ck = ck.cpu().numpy()
    for s in range(ck.shape[0]):
        n = neo[s]
        c, r = ck[s], ref["c_k"][s]
        assert np.abs(c[..., n:]).max(initial=0.0) == 0.0          # dropped columns are zero
        c = c[..., :n]
        p_gpu = np.einsum("kmi,kni->kmn", c, c.conj())
        p_ref = np.einsum("kmi,kni->kmn", r, r.conj())
        assert np.abs(p_gpu - p_ref).max() < 1e-10
        so = np.einsum("kmi,kmj->ij", c.conj(), c) / nk
        assert np.abs(so - np.eye(n)).max() < 1e-12
        cr, cri = _bath_columns_r(c, nk, kmesh)
        assert cri < 1e-12
        cr = cr.reshape(nk * nao, n)
        assert np.abs(cr[np.asarray(imp), np.arange(nimp)] - 1.0).max() < 1e-13
        rr = ref["c_r"][s].reshape(nk * nao, n)
        sig = ref["sigma"][s]
        for b in range(n - nimp):
            gaps = [abs(sig[b] - sig[x]) for x in (b - 1, b + 1) if 0 <= x < len(sig)]
            if min(gaps) > 1e-6 * sig[0]:
                col = cr[:, nimp + b]
                i = int(np.argmax(np.abs(col)))
                assert col[i] > 0                                 # sign gauge
                assert np.abs(col - rr[:, nimp + b]).max() < tol_vec


FRAGMENTS = {
    # name: (lattice workload, neo, nspin); impurity = the first ceil(neo/2)
    # orbitals in supercell order, bath = the first SVD columns
    "b222_neo150": (synth.BATCH_LATTICES["b222"], 150),
    "b333_neo200": (synth.BATCH_LATTICES["b333"], 200),
    "b333_neo37": (synth.BATCH_LATTICES["b333"], 37),
}


@pytest.mark.parametrize("name", list(FRAGMENTS))
def test_bath_supercell_fragment(dmet, name):
    """Batched-form fragments: impurity LOs spanning several cells, valence
    subset of the columns, the shapes the batched benchmark runs."""
    wl, neo = FRAGMENTS[name]
    lat = synth.make_lattice(wl)
    nimp = (neo + 1) // 2
    imp = synth.supercell_order(wl.kmesh, wl.nao)[:nimp]
    val = list(range(neo - nimp))
    print(f"bath fragment {name}: nimp {nimp}, nval {len(val)}", flush=True)
    ref = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, imp_idx=imp, val_idx=val)
    ck, sv, got, mi = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k), imp_idx=imp, val_idx=val,
                                           return_imag=True)
    _compare_bath(ck, sv, got, mi, ref, wl.kmesh, wl.nao, imp)


def test_bath_bn33(dmet):
    """The paper's BN 3x3 impurity on the 6x6x1 mesh (234 impurity LOs, 72
    valence SVD columns, 702 environment rows): the bath the bn33 benchmark
    step builds."""
    wl = synth.BN33
    lat = synth.make_lattice(wl)
    imp, val = synth.bn33_impurity()
    print("bath bn33", flush=True)
    ref = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, imp_idx=imp, val_idx=val)
    ck, sv, got, mi = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k), imp_idx=imp, val_idx=val,
                                           return_imag=True)
    assert got == [306]
    _compare_bath(ck, sv, got, mi, ref, wl.kmesh, wl.nao, imp)


def test_bath_sv_tol(dmet):
    """sv_tol between two singular values keeps exactly the larger ones; the
    dropped columns of C^k are zero and every sigma is still returned."""
    wl = synth.Workload("tol", (3, 2, 1), 10, 4, 10, 10, 2, 1.5, 71)
    lat = synth.make_lattice(wl)
    full = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    sig = full["sigma"]
    tol = 0.5 * (max(sig[0][6], sig[1][6]) + min(sig[0][5], sig[1][5]))
    assert all(sig[s][6] < tol < sig[s][5] for s in range(2))
    ref = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, sv_tol=tol)
    ck, sv, got, mi = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k), sv_tol=tol, return_imag=True)
    assert got == [wl.nao + 6] * 2
    _compare_bath(ck, sv, got, mi, ref, wl.kmesh, wl.nao, list(range(wl.nao)))


def test_bath_ao_lo(dmet):
    """C^{k,AO,EO} = C^{k,AO,LO} C^{k,LO,EO} with a k-dependent unitary
    C^{k,AO,LO} (Eq. C loemb k): the GPU composition equals the oracle's."""
    wl = synth.Workload("aolo", (3, 2, 1), 10, 4, 10, 10, 1, 1.5, 59)
    lat = synth.make_lattice(wl)
    u = synth.random_lattice_unitary(wl.kmesh, wl.nao, 9)
    ref = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, c_ao_lo=u)
    lo = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    ck, sv, got = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k), c_ao_lo=to_dev(u))
    ck_lo, sv_lo, got_lo, mi = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k), return_imag=True)
    _compare_bath(ck_lo, sv_lo, got_lo, mi, lo, wl.kmesh, wl.nao, list(range(wl.nao)))
    ck, ck_lo = ck.cpu().numpy(), ck_lo.cpu().numpy()
    assert got == ref["neo"]
    assert torch.equal(sv, sv_lo)
    assert np.abs(ck - u[None] @ ck_lo).max() < 1e-13
    p_gpu = np.einsum("skmi,skni->skmn", ck, ck.conj())
    p_ref = np.einsum("skmi,skni->skmn", ref["c_k"], ref["c_k"].conj())
    assert np.abs(p_gpu - p_ref).max() < 1e-10
    assert np.abs(ck - ck_lo).max() > 1e-2
    # the sign-gauged vectors, rotated by U, are the oracle's
    assert np.abs(ck - ref["c_k"]).max() < 1e-9


def test_bath_decoupled_orbital(dmet):
    """An impurity LO with no coherence to the environment has sigma = 0 and
    no determined bath vector: it is dropped at sv_tol = 0, as in the oracle
    (instead of a zero bath column and a failed orthonormality check)."""
    wl = synth.Workload("dec", (3, 2, 1), 10, 4, 10, 10, 1, 1.5, 63)
    lat = synth.make_lattice(wl)
    dm = synth.decouple_orbital(lat.dm_k, 3)
    ref = ok.build_bath(dm, wl.kmesh, wl.nao)
    ck, sv, got, mi = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(dm), return_imag=True)
    assert got == [2 * wl.nao - 1]
    _compare_bath(ck, sv, got, mi, ref, wl.kmesh, wl.nao, list(range(wl.nao)))


def test_bath_error_status(dmet):
    """Failure paths come back as status codes (no fault, no hang): NaN in
    dm_k is DMET_E_NONFINITE, found before the SVD sweeps; sv_tol above every
    singular value leaves no bath, DMET_E_RANK.  The library stays usable."""
    wl = synth.Workload("err", (2, 2, 1), 8, 4, 8, 8, 1, 1.5, 64)
    lat = synth.make_lattice(wl)
    dm = lat.dm_k.copy()
    dm[0, 1, 2, 3] = np.nan
    with pytest.raises(dmet.DmetError) as e:
        dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(dm))
    assert e.value.status == 5 and "non-finite" in str(e.value)
    dm = lat.dm_k.copy()
    dm[0, 0, 0, 0] = np.inf
    with pytest.raises(dmet.DmetError) as e:
        dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(dm))
    assert e.value.status == 5
    with pytest.raises(dmet.DmetError) as e:
        dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k), sv_tol=10.0)
    assert e.value.status == 4
    ck, sv, got = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k))
    assert got == [16]


def test_bath_noconv_status(dmet, monkeypatch):
    """A sweep cap below what the SVD needs returns DMET_E_NOCONV (forced from
    the host through the library's sweep limit; every kernel exits normally),
    and the next call with the default cap succeeds."""
    wl = synth.Workload("nc", (2, 2, 2), 20, 4, 20, 20, 1, 1.5, 65)
    lat = synth.make_lattice(wl)
    dm = to_dev(lat.dm_k)
    monkeypatch.setenv("DMET_SVD_MAX_SWEEPS", "1")
    with pytest.raises(dmet.DmetError) as e:
        dmet.dmet_build_bath(wl.kmesh, wl.nao, dm)
    assert e.value.status == 3 and "1 sweeps" in str(e.value)
    monkeypatch.delenv("DMET_SVD_MAX_SWEEPS")
    ck, sv, neo = dmet.dmet_build_bath(wl.kmesh, wl.nao, dm)
    assert neo == [2 * wl.nao]
