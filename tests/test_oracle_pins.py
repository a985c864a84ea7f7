"""Pins of the FP64 oracle against things other than itself.

* the real-space supercell brute force (Alg. 1 is exact on the BvK torus);
* closed forms: sigma_i = sqrt(lambda_i (1 - lambda_i)) for an idempotent
  mean-field DM, gamma^EO idempotent with trace n_imp;
* the N_k = 1 molecular limit of Eq. ``density fitting`` (plain DF ao2mo);
* invariants: 8-fold symmetry, vanishing imaginary part, positive
  semidefiniteness, rank, invariance of gauge-free scalars under EO rotations;
* the paper's worked example count (BN 3x3x1 in a 6x6x1 mesh: 936 crystal AOs
  -> 306 embedding orbitals, Sec. 2.1 after Alg. 1);
* planted mistakes (in the oracle, on the CPU) that these pins must catch.
"""
import dataclasses
import json
import os

import numpy as np
import pytest

import synth
from oracle import kspace as ok
from oracle import supercell as sc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(name):
    wl = synth.CONFIGS[name]
    lat = synth.make_lattice(wl)
    lm, b = synth.three_index(wl, real_space=True)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    return wl, lat, lm, b, bath


@pytest.fixture(scope="module")
def tiny():
    return _setup("tiny")


@pytest.fixture(scope="module")
def hbn():
    return _setup("hbn")


@pytest.fixture(scope="module")
def odd():
    """3x2x1 mesh: k != -k on the first axis, so sign and k-q errors show."""
    wl = synth.Workload("odd", (3, 2, 1), 4, 12, 4, 4, 1, 1.5, 77)
    lat = synth.make_lattice(wl)
    lm, b = synth.three_index(wl, real_space=True)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    return wl, lat, lm, b, bath


# ---------------------------------------------------------------- supercell
@pytest.mark.parametrize("name", ["tiny", "odd", "hbn"])
def test_kspace_equals_supercell(name, request):
    wl, lat, lm, b, bath = request.getfixturevalue(name)
    ck = bath["c_k"][0]
    # gamma^{R,0} vs the supercell projector's (R, 0) block
    gsup, gim = sc.supercell_dm(lat.dm_k[0], wl.kmesh)
    assert gim < 1e-13
    g = gsup.reshape(wl.nk, wl.nao, wl.nk, wl.nao)[:, :, 0, :]
    assert np.abs(g - bath["dm_r"][0]).max() < 1e-13
    assert bath["max_imag_dm"] < 1e-13
    # gamma_sup is the mean-field projector of the real-space Fock matrix
    fsup = sc.supercell_operator(lat.t_f[0], wl.kmesh)
    assert np.abs(gsup @ gsup - gsup).max() < 1e-12
    assert np.abs(fsup @ gsup - gsup @ fsup).max() < 1e-12
    assert abs(np.trace(gsup) - wl.nk * wl.nao // 2) < 1e-10
    # bath: singular values, and the EO space (projector, gauge-free)
    csup, s = sc.embedding_orbitals(gsup, np.arange(wl.nao))
    assert np.abs(s - bath["sigma"][0]).max() < 1e-13
    cr = bath["c_r"][0].reshape(wl.nk * wl.nao, wl.neo)
    assert np.abs(cr @ cr.T - csup @ csup.T).max() < 1e-11
    # one-body transform (Eq. fock transform) vs C^T h_sup C
    h1, him = ok.transform_1e(bath["c_k"], lat.h_k)
    hsup = sc.supercell_operator(lat.t_h, wl.kmesh)
    assert him < 1e-13
    assert np.abs(h1[0] - cr.T @ hsup @ cr).max() < 1e-12
    # ERIs: Alg. 1 in k-space vs Z.Z in real space, on the same EOs
    eri_k, im = ok.alg1_eri(lm, ck, wl.kmesh)
    eri_s = sc.eri(b, cr, wl.kmesh)
    assert im < 1e-12 * np.abs(eri_k).max()
    assert np.abs(eri_k - eri_s).max() < 1e-12 * np.abs(eri_s).max()


def test_supercell_bloch_convention(tiny):
    """The generator's h(k) is the Bloch block of the real-space operator."""
    wl, lat, *_ = tiny
    u = sc.bloch_unitary(wl.kmesh, wl.nao)
    hsup = sc.supercell_operator(lat.t_h, wl.kmesh)
    blk = u.conj().T @ hsup @ u
    for k in range(wl.nk):
        s = slice(k * wl.nao, (k + 1) * wl.nao)
        assert np.abs(blk[s, s] - lat.h_k[0, k]).max() < 1e-13
    off = blk.copy()
    for k in range(wl.nk):
        s = slice(k * wl.nao, (k + 1) * wl.nao)
        off[s, s] = 0
    assert np.abs(off).max() < 1e-13


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("name", ["tiny", "hbn"])
def test_sigma_closed_form(name, request):
    """For an idempotent gamma, M^T M = g00 - g00^2, so sigma = sqrt(l(1-l))."""
    wl, lat, lm, b, bath = request.getfixturevalue(name)
    lam = np.linalg.eigvalsh(bath["dm_r"][0][0])
    sig = np.sort(np.sqrt(np.clip(lam * (1 - lam), 0, None)))[::-1]
    assert np.abs(sig - bath["sigma"][0]).max() < 1e-13


@pytest.mark.parametrize("name", ["tiny", "odd", "hbn"])
def test_embedding_structure(name, request):
    wl, lat, lm, b, bath = request.getfixturevalue(name)
    cr, ck = bath["c_r"][0], bath["c_k"][0]
    # identity block on the impurity (Eq. C loemb R), zero bath weight there
    assert np.abs(cr[0][:, : wl.nimp] - np.eye(wl.nao)).max() < 1e-14
    assert np.abs(cr[0][:, wl.nimp:]).max() < 1e-14
    # orthonormal EOs: 1/N_k sum_k C^k^H C^k = I
    s = np.einsum("kmi,kmj->ij", ck.conj(), ck) / wl.nk
    assert np.abs(s - np.eye(wl.neo)).max() < 1e-13
    # time reversal: C^{-k} = conj(C^k)
    neg = synth.neg_index(wl.kmesh)
    assert np.abs(ck[neg] - ck.conj()).max() < 1e-14
    # gamma^EO idempotent, trace n_imp (all sigma > 0)
    g, gi = ok.transform_1e(bath["c_k"], lat.dm_k)
    assert gi < 1e-13
    assert np.abs(g[0] @ g[0] - g[0]).max() < 1e-12
    assert abs(np.trace(g[0]) - wl.nimp) < 1e-11


# ------------------------------------------------------- N_k = 1 molecular
def test_nk1_molecular_limit():
    """At one k-point Alg. 1 is plain density-fitted ao2mo with any real
    orthonormal C: (ij|kl) = sum_L (C^T B_L C)_ij (C^T B_L C)_kl."""
    wl = dataclasses.replace(synth.CONFIGS["tiny"], name="mol", kmesh=(1, 1, 1), nao=10, naux=30)
    lm, b = synth.three_index(wl, real_space=True)
    c = synth.random_orthonormal(np.random.default_rng(7), wl.nao, 7)
    bl = b.reshape(wl.naux, wl.nao, wl.nao)
    ref = np.einsum("Lmn,mi,nj,Lpr,pk,rl->ijkl", bl, c, c, bl, c, c, optimize=True)
    got, im = ok.alg1_eri(lm, c[None].astype(np.complex128), wl.kmesh)
    assert im == 0.0 or im < 1e-15
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


# --------------------------------------------------------------- invariants
def test_eri_invariants(hbn):
    wl, lat, lm, b, bath = hbn
    eri, im = ok.alg1_eri(lm, bath["c_k"][0], wl.kmesh)
    mx = np.abs(eri).max()
    assert im < 1e-12 * mx
    assert np.abs(eri - eri.transpose(1, 0, 2, 3)).max() < 1e-13 * mx
    assert np.abs(eri - eri.transpose(0, 1, 3, 2)).max() < 1e-13 * mx
    assert np.abs(eri - eri.transpose(2, 3, 0, 1)).max() < 1e-13 * mx
    n = wl.neo
    tri = np.tril_indices(n)
    mat = eri[tri[0], tri[1]][:, tri[0], tri[1]]
    w = np.linalg.eigvalsh(mat)
    assert w.min() > -1e-12 * w.max()
    rank = int(np.count_nonzero(w > 1e-10 * w.max()))
    assert rank == min(mat.shape[0], wl.nk * wl.naux)
    # packing round trip
    assert np.array_equal(ok.unpack_s8(ok.pack_s8(eri), n), eri) or \
        np.abs(ok.unpack_s8(ok.pack_s8(eri), n) - eri).max() < 1e-13 * mx


def test_gauge_invariance(tiny):
    """Frobenius norm, E_J and E_K do not depend on the choice of real EO basis."""
    wl, lat, lm, b, bath = tiny
    ck = bath["c_k"]
    o = synth.random_orthonormal(np.random.default_rng(3), wl.neo, wl.neo)
    ck2 = ck @ o
    vals = []
    for c in (ck, ck2):
        eri, _ = ok.alg1_eri(lm, c[0], wl.kmesh)
        g, _ = ok.transform_1e(c, lat.dm_k)
        g = g[0]
        ej = 0.5 * np.einsum("ijkl,ji,lk->", eri, g, g)
        ek = 0.5 * np.einsum("ijkl,jk,li->", eri, g, g)
        vals.append((np.linalg.norm(eri), ej, ek))
    assert np.allclose(vals[0], vals[1], rtol=1e-12, atol=0)


# ---------------------------------------------------- paper worked example
def test_bn_worked_example_orbital_count():
    """BN 3x3x1 impurity in a 6x6x1 lattice, valence-only bath: n_EO = 306."""
    g = json.load(open(os.path.join(GOLDEN, "bn_3x3_counts.json")))
    kmesh = tuple(g["kmesh"])
    nao, nvpc = g["nao_per_cell"], g["nval_per_cell"]
    wl = synth.Workload("bn66", kmesh, nao, 1, 0, 0, 1, 2.0, 4242)
    lat = synth.make_lattice(wl)
    pts = synth.cells(kmesh)
    ic = g["impurity_cells"]
    imp_cells = [i for i, p in enumerate(pts) if p[0] < ic[0] and p[1] < ic[1] and p[2] < ic[2]]
    imp = np.array([c * nao + m for c in imp_cells for m in range(nao)])
    # valence = 2s2p of each of the two atoms (first 4 AOs of each 13-AO block)
    val = np.array([ci * nao + a * 13 + m for ci in range(len(imp_cells))
                    for a in range(2) for m in range(4)])
    assert len(val) == len(imp_cells) * nvpc
    out = ok.build_bath(lat.dm_k, kmesh, nao, imp_idx=imp, val_idx=val)
    assert wl.nk * nao == g["n_crystal_ao"]
    assert out["neo"][0] == g["n_embedding_orbitals"]
    ck = out["c_k"][0]
    s = np.einsum("kmi,kmj->ij", ck.conj(), ck) / wl.nk
    assert np.abs(s - np.eye(306)).max() < 1e-12


# ----------------------------------------------------------- planted bugs
def _planted_eri(lm, ck, kmesh, kind):
    nk = lm.shape[0]
    pts = ok.mesh_points(kmesh)
    eri = 0
    for q in range(nk):
        x = 0
        for k in range(nk):
            kmq = ok.mesh_index(kmesh, pts[k] - pts[q])
            if kind == "plus_q":
                kmq = ok.mesh_index(kmesh, pts[k] + pts[q])
            a = lm[q, k]
            if kind == "transposed":
                a = a.transpose(0, 2, 1)
            left = ck[k] if kind == "no_conj" else ck[k].conj()
            x = x + left.T @ (a @ ck[kmq]) / nk
        xl = x if kind == "no_conj_contract" else x.conj()
        n = x.shape[1]
        eri = eri + xl.reshape(x.shape[0], -1).T @ x.reshape(x.shape[0], -1) / nk
    n = ck.shape[2]
    return eri.reshape(n, n, n, n).real


@pytest.mark.parametrize("kind", ["plus_q", "transposed", "no_conj", "no_conj_contract"])
def test_planted_mistakes_are_caught(odd, kind):
    wl, lat, lm, b, bath = odd
    cr = bath["c_r"][0].reshape(wl.nk * wl.nao, wl.neo)
    ref = sc.eri(b, cr, wl.kmesh)
    bad = _planted_eri(lm, bath["c_k"][0], wl.kmesh, kind)
    assert np.abs(bad - ref).max() > 1e-6 * np.abs(ref).max()


def test_planted_phase_sign_is_caught(odd):
    """C^k built with exp(+ikR) instead of exp(-ikR) breaks supercell parity."""
    wl, lat, lm, b, bath = odd
    p = ok.phase_matrix(wl.kmesh)
    ck_bad = np.einsum("kR,Rmi->kmi", p, bath["c_r"][0].astype(complex))
    cr = bath["c_r"][0].reshape(wl.nk * wl.nao, wl.neo)
    ref = sc.eri(b, cr, wl.kmesh)
    bad, _ = ok.alg1_eri(lm, ck_bad, wl.kmesh)
    assert np.abs(bad - ref).max() > 1e-6 * np.abs(ref).max()


# ------------------------------------------------------------- spin blocks
def test_uhf_blocks_equal_supercell():
    """alpha-alpha, beta-beta and alpha-beta blocks of the spin-unrestricted
    case (separate alpha/beta bath, Sec. 3.3) against the supercell."""
    wl = synth.Workload("uodd", (3, 2, 1), 6, 16, 6, 6, 2, 1.5, 91)
    lat = synth.make_lattice(wl)
    lm, b = synth.three_index(wl, real_space=True)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    cs = []
    for s in range(2):
        gsup, _ = sc.supercell_dm(lat.dm_k[s], wl.kmesh)
        c, sig = sc.embedding_orbitals(gsup, np.arange(wl.nao))
        assert np.abs(sig - bath["sigma"][s]).max() < 1e-13
        cs.append(bath["c_r"][s].reshape(-1, wl.neo))
    assert np.abs(bath["c_r"][0] - bath["c_r"][1]).max() > 1e-3   # spins really differ
    for sa, sb in ((0, 0), (1, 1), (0, 1)):
        got, im = ok.alg1_eri(lm, bath["c_k"][sa], wl.kmesh,
                              None if sa == sb else bath["c_k"][sb])
        ref = sc.eri(b, cs[sa], wl.kmesh, None if sa == sb else cs[sb])
        assert im < 1e-12 * np.abs(ref).max()
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # sampled-column form agrees with the full contraction
    pairs = [(0, 0), (3, 1), (11, 5), (7, 7)]
    cols, _ = ok.alg1_eri_columns(lm, bath["c_k"][0], wl.kmesh, pairs, bath["c_k"][1], pairs[::-1])
    full, _ = ok.alg1_eri(lm, bath["c_k"][0], wl.kmesh, bath["c_k"][1])
    ref = np.array([[full[i, j, k, l] for (k, l) in pairs[::-1]] for (i, j) in pairs])
    assert np.abs(cols - ref).max() < 1e-13 * np.abs(full).max()


def test_valence_subset_and_truncation(odd):
    """Valence-only SVD columns (n_EO = n_imp + n_val) and sv_tol truncation
    agree with the supercell SVD restricted to the same columns."""
    wl, lat, lm, b, bath = odd
    val = np.array([0, 2, 3])
    out = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, val_idx=val)
    assert out["neo"][0] == wl.nimp + len(val)
    gsup, _ = sc.supercell_dm(lat.dm_k[0], wl.kmesh)
    c, s = sc.embedding_orbitals(gsup, np.arange(wl.nao), val)
    cr = out["c_r"][0].reshape(-1, out["neo"][0])
    assert np.abs(cr @ cr.T - c @ c.T).max() < 1e-12
    tol = 0.5 * (out["sigma"][0][1] + out["sigma"][0][2])
    out2 = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, val_idx=val, sv_tol=tol)
    assert out2["neo"][0] == wl.nimp + 2


def test_impurity_columns_give_impurity_block():
    """Cutting C^k to its impurity columns gives exactly the impurity block of
    the full embedding ERIs (the non-interacting-bath ERIs, Sec. 2.1), and the
    real-space brute force with C_sup = the cell-0 unit vectors agrees."""
    wl = synth.Workload("imp", (3, 2, 1), 6, 17, 6, 6, 1, 1.5, 23)
    lat = synth.make_lattice(wl)
    lm, b_real = synth.three_index(wl, real_space=True)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    ck = bath["c_k"][0]
    full, _ = ok.alg1_eri(lm, ck, wl.kmesh)
    imp, _ = ok.alg1_eri(lm, np.ascontiguousarray(ck[:, :, :wl.nimp]), wl.kmesh)
    n = wl.nimp
    assert np.abs(imp - full[:n, :n, :n, :n]).max() < 1e-14 * np.abs(full).max()
    csup = np.zeros((wl.nk * wl.nao, n))
    csup[np.arange(n), np.arange(n)] = 1.0
    ref = sc.eri(b_real, csup, wl.kmesh)
    assert np.abs(imp - ref).max() < 1e-12 * np.abs(ref).max()


# ------------------------------------------------ supercell impurity, gauge
def _bath_vs_supercell(dm_k, kmesh, nao, imp, val):
    """Oracle bath (translation-invariant blocks of gamma^{R,0}) against the
    SVD of the explicit supercell projector gamma_sup = U blockdiag U^H for an
    impurity anywhere in the supercell: singular values, the EO projector
    C C^T, and the identity entries on the impurity rows."""
    out = ok.build_bath(dm_k, kmesh, nao, imp_idx=imp, val_idx=val)
    gsup, gim = sc.supercell_dm(dm_k[0], kmesh)
    assert gim < 1e-12
    c_sc, s_sc = sc.embedding_orbitals(gsup, np.asarray(imp), np.asarray(val))
    assert np.abs(out["sigma"][0] - s_sc).max() < 1e-12
    neo = out["neo"][0]
    cr = out["c_r"][0].reshape(-1, neo)
    assert neo == len(imp) + len(val)
    assert np.abs(cr @ cr.T - c_sc @ c_sc.T).max() < 1e-11
    assert np.abs(cr[np.asarray(imp), np.arange(len(imp))] - 1.0).max() < 1e-14
    return out, cr, c_sc


def test_supercell_impurity_bath_bn33():
    """The paper's BN 3x3 impurity (9 cells, 8 valence LOs per cell) on the
    6x6x1 mesh: the bath of the k-space oracle equals the supercell SVD, which
    fixes every cell offset of gamma_sup[env, imp[val]] (cells != 0 included)."""
    wl = synth.BN33
    lat = synth.make_lattice(wl)
    imp, val = synth.bn33_impurity()
    _bath_vs_supercell(lat.dm_k, wl.kmesh, wl.nao, imp, val)


@pytest.mark.parametrize("lattice,neo", [("b222", 150), ("b333", 57)])
def test_supercell_impurity_bath_fragment(lattice, neo):
    """A batched-form fragment: ceil(neo/2) LOs in supercell order (nearest
    cells first, so it straddles cells), bath from the first SVD columns."""
    base = synth.BATCH_LATTICES[lattice]
    wl = dataclasses.replace(base, nao=12, naux=4) if lattice == "b333" else base
    lat = synth.make_lattice(wl)
    nimp = (neo + 1) // 2
    imp = synth.supercell_order(wl.kmesh, wl.nao)[:nimp]
    _bath_vs_supercell(lat.dm_k, wl.kmesh, wl.nao, imp, list(range(neo - nimp)))


def test_planted_cell_offset_is_caught():
    """gamma^{R'-R} in place of gamma^{R-R'} for the supercell block (a wrong
    cell offset) breaks agreement with the supercell SVD for an impurity that
    spans several cells."""
    wl = synth.Workload("offs", (3, 2, 1), 6, 4, 6, 6, 1, 1.5, 31)
    lat = synth.make_lattice(wl)
    imp = synth.supercell_order(wl.kmesh, wl.nao)[:9]
    dm_r, _ = ok.real_space_dm(lat.dm_k, wl.kmesh)
    env = [r for r in range(wl.nk * wl.nao) if r not in set(imp)]
    good = ok.supercell_block(dm_r[0], wl.kmesh, wl.nao, env, imp)
    gsup, _ = sc.supercell_dm(lat.dm_k[0], wl.kmesh)
    assert np.abs(good - gsup[np.ix_(env, imp)]).max() < 1e-13
    pts = ok.mesh_points(wl.kmesh)
    bad = np.empty_like(good)
    for a, r in enumerate(env):
        cr, mu = divmod(r, wl.nao)
        for b, c in enumerate(imp):
            cc, nu = divmod(c, wl.nao)
            bad[a, b] = dm_r[0][ok.mesh_index(wl.kmesh, pts[cc] - pts[cr]), mu, nu]
    assert np.abs(bad - gsup[np.ix_(env, imp)]).max() > 1e-3


def test_ao_lo_composition():
    """Eq. ``C loemb k``, second form: with a k-dependent unitary AO->LO map U(k)
    (orthonormal AOs), C^{k,AO,EO} = U(k) C^{k,LO,EO}, so any operator given in
    the AO basis, X_AO(k) = U X_LO U^H, transforms to the same embedding matrix
    as X_LO; and the composed C^k keeps the time-reversal symmetry of U."""
    wl = synth.Workload("aolo", (3, 2, 1), 6, 4, 6, 6, 1, 1.5, 57)
    lat = synth.make_lattice(wl)
    u = synth.random_lattice_unitary(wl.kmesh, wl.nao, 5)
    assert np.abs(np.einsum("kmi,kmj->kij", u.conj(), u) - np.eye(wl.nao)).max() < 1e-13
    lo = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    ao = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, c_ao_lo=u)
    assert np.abs(ao["c_r"] - lo["c_r"]).max() == 0.0
    neg = synth.neg_index(wl.kmesh)
    assert np.abs(ao["c_k"][0][neg] - ao["c_k"][0].conj()).max() < 1e-13
    for x_lo in (lat.h_k, lat.f_k, lat.dm_k):
        x_ao = u[None] @ x_lo @ u.conj().transpose(0, 2, 1)[None]
        a, aim = ok.transform_1e(ao["c_k"], x_ao)
        b, _ = ok.transform_1e(lo["c_k"], x_lo)
        assert aim < 1e-13
        assert np.abs(a - b).max() < 1e-13
    # the composition is not the identity: the AO-basis C^k differs
    assert np.abs(ao["c_k"] - lo["c_k"]).max() > 1e-2


@pytest.mark.parametrize("name", ["tiny", "odd", "hbn"])
def test_bath_sign_gauge(name, request):
    """Every bath column of the oracle has its entry of largest modulus
    positive (the gauge dmet_build_bath promises); columns come in descending
    singular value."""
    wl, lat, lm, b, bath = request.getfixturevalue(name)
    cr = bath["c_r"][0].reshape(wl.nk * wl.nao, wl.neo)[:, wl.nimp:]
    for j in range(cr.shape[1]):
        i = int(np.argmax(np.abs(cr[:, j])))
        assert cr[i, j] > 0
    assert np.all(np.diff(bath["sigma"][0]) <= 0)


def test_sign_fix_tie_rule():
    """Ties within 1e-12 of the largest modulus: the lowest index decides."""
    u = np.array([[-0.5, 0.6], [0.5, -0.6 * (1 - 1e-14)], [0.1, 0.1]])
    v = ok.sign_fix(u)
    assert v[0, 0] == 0.5 and v[1, 0] == -0.5       # flipped: index 0 was negative
    assert v[0, 1] == 0.6                           # kept: index 0 positive


def test_decoupled_orbital_has_no_bath():
    """An impurity LO with no coherence to the environment (a core-like,
    fully occupied orbital) gives a zero column of M and a zero singular
    value; its bath vector is undetermined, so it is dropped even at
    sv_tol = 0 (neo = nimp + nval - 1), and the rest of the bath is the
    supercell SVD's."""
    wl = synth.Workload("dec", (3, 2, 1), 6, 4, 6, 6, 1, 1.5, 63)
    lat = synth.make_lattice(wl)
    dm = synth.decouple_orbital(lat.dm_k, 2)
    out = ok.build_bath(dm, wl.kmesh, wl.nao)
    assert out["neo"][0] == 2 * wl.nao - 1
    assert out["sigma"][0][-1] < 1e-15
    gsup, _ = sc.supercell_dm(dm[0], wl.kmesh)
    c_sc, s_sc = sc.embedding_orbitals(gsup, np.arange(wl.nao), nbath=wl.nao - 1)
    assert np.abs(out["sigma"][0] - s_sc).max() < 1e-13
    cr = out["c_r"][0].reshape(-1, out["neo"][0])
    assert np.abs(cr @ cr.T - c_sc @ c_sc.T).max() < 1e-11


def test_eri_block_and_diag_forms():
    """The restricted forms of the contraction (listed rows / columns, the
    diagonal) reproduce the corresponding entries of the full alg1_eri tensor,
    for a same-spin and a mixed-spin block."""
    wl = synth.Workload("blk", (3, 2, 1), 6, 16, 6, 6, 2, 1.5, 93)
    lat = synth.make_lattice(wl)
    lm = synth.three_index(wl)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    ck = bath["c_k"]
    xa = ok.alg1_embedded_all(lm, ck[0], wl.kmesh)
    xb = ok.alg1_embedded_all(lm, ck[1], wl.kmesh)
    tri = list(zip(*np.tril_indices(wl.neo)))
    rng = np.random.default_rng(1)
    rows = [tri[int(x)] for x in rng.choice(len(tri), 9, replace=False)]
    for b, full_args in ((None, (lm, ck[0], wl.kmesh)), (xb, (lm, ck[0], wl.kmesh, ck[1]))):
        full, _ = ok.alg1_eri(*full_args)
        got, im = ok.alg1_eri_block(xa, rows, tri, b)
        ref = np.array([[full[i, j, k, l] for (k, l) in tri] for (i, j) in rows])
        assert im < 1e-12
        assert np.abs(got - ref).max() < 1e-13 * np.abs(full).max()
    full, _ = ok.alg1_eri(lm, ck[0], wl.kmesh)
    d = ok.alg1_eri_diag(xa, tri)
    assert np.abs(d - np.array([full[i, j, i, j] for (i, j) in tri])).max() < 1e-13 * np.abs(full).max()


def test_energy_1e_against_supercell(odd):
    """E1 (Eq. emb Ham) from the k-space transforms equals the trace of the
    supercell operators projected on the embedding orbitals, and does not
    change under a rotation of the embedding orbitals."""
    wl, lat, lm, b, bath = odd
    h1, _ = ok.transform_1e(bath["c_k"], lat.h_k)
    g1, _ = ok.transform_1e(bath["c_k"], lat.dm_k)
    cr = bath["c_r"][0].reshape(wl.nk * wl.nao, wl.neo)
    hsup = sc.supercell_operator(lat.t_h, wl.kmesh)
    gsup, _ = sc.supercell_dm(lat.dm_k[0], wl.kmesh)
    e_sup = float(np.trace((cr.T @ hsup @ cr) @ (cr.T @ gsup @ cr)))
    assert abs(ok.energy_1e(h1, g1) - e_sup) < 1e-12 * max(1.0, abs(e_sup))
    q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((wl.neo, wl.neo)))
    rot = lambda x: np.einsum("ai,sab,bj->sij", q, x, q)
    assert abs(ok.energy_1e(rot(h1), rot(g1)) - e_sup) < 1e-12 * max(1.0, abs(e_sup))


def test_pair_packing_brute_force():
    """pair_index enumerates i >= j row by row; pack_s4 holds [ij][kl] over those
    pairs (both spins have the same neo) and pack_s8 the lower triangle
    IJ >= KL, element by element, on tensors without any symmetry."""
    n = m = 4
    pairs_n = [(i, j) for i in range(n) for j in range(i + 1)]
    pairs_m = [(k, l) for k in range(m) for l in range(k + 1)]
    assert [ok.pair_index(i, j) for i, j in pairs_n] == list(range(len(pairs_n)))
    assert all(ok.pair_index(j, i) == ok.pair_index(i, j) for i, j in pairs_n)
    rng = np.random.default_rng(9)
    e4 = rng.standard_normal((n, n, m, m))
    p4 = ok.pack_s4(e4)
    assert p4.shape == (len(pairs_n), len(pairs_m))
    for a, (i, j) in enumerate(pairs_n):
        for c, (k, l) in enumerate(pairs_m):
            assert p4[a, c] == e4[i, j, k, l]
    e8 = rng.standard_normal((n, n, n, n))
    p8 = ok.pack_s8(e8)
    pos = 0
    for a, (i, j) in enumerate(pairs_n):
        for c, (k, l) in enumerate(pairs_n[: a + 1]):
            assert p8[pos] == e8[i, j, k, l]
            pos += 1
    assert pos == p8.size
