"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 GPU path within 1e-10 of max|ERI| (element-wise), one-body
matrices within 1e-12 Ha, E1 within 1e-10 Ha.  The ERI tests feed the oracle's
C^k to the GPU so that the bath gauge cannot leak into the comparison; the
end-to-end test compares gauge-free scalars only.
"""
import numpy as np
import pytest
import torch

from oracle import kspace as ok
from tests.gpu_common import case, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dmet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_08596_amd import dmet as d
    d.load()
    return d


CASES = {
    "tiny": dict(name="tiny"),
    "odd": dict(name="odd", kmesh=(3, 2, 1), nao=5, naux=13, nspin=1, seed=11),
    "hbn": dict(name="hbn"),
}


@pytest.mark.parametrize("key", ["tiny", "odd", "hbn"])
def test_bath_parity(dmet, key):
    wl, lat, lm, bath = case(**CASES[key])
    ck, sv, neo = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k))
    torch.cuda.synchronize()
    assert neo == [wl.neo] * wl.nspin
    sv = sv.cpu().numpy()
    assert np.abs(sv - bath["sigma"]).max() < 1e-12
    ck = ck.cpu().numpy()
    ref = bath["c_k"]
    # impurity block is the identity at every k (Eq. C loemb R at R = 0)
    eye = np.broadcast_to(np.eye(wl.nao), ck[:, :, :, : wl.nimp].shape)
    assert np.abs(ck[:, :, :, : wl.nimp] - eye).max() < 1e-14
    # EO space per k (gauge-free): C^k C^k^H
    p_gpu = np.einsum("skmi,skni->skmn", ck, ck.conj())
    p_ref = np.einsum("skmi,skni->skmn", ref, ref.conj())
    assert np.abs(p_gpu - p_ref).max() < 1e-10
    # orthonormality
    s = np.einsum("skmi,skmj->sij", ck.conj(), ck) / wl.nk
    assert np.abs(s - np.eye(wl.neo)).max() < 1e-12


@pytest.mark.parametrize("key", ["tiny", "odd", "hbn"])
def test_onebody_parity(dmet, key):
    wl, lat, lm, bath = case(**CASES[key])
    ck = to_dev(bath["c_k"])
    outs = {}
    for nm, op in (("h", lat.h_k), ("f", lat.f_k), ("g", lat.dm_k)):
        x, mi = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck, to_dev(op), want_imag=True)
        ref, rim = ok.transform_1e(bath["c_k"], op)
        assert np.abs(x.cpu().numpy() - ref).max() < 1e-12
        assert mi < 1e-12
        outs[nm] = (x, ref)
    e1 = dmet.dmet_energy_1e(outs["h"][0], outs["g"][0])
    ref_e1 = ok.energy_1e(outs["h"][1], outs["g"][1])
    assert abs(float(e1.cpu()) - ref_e1) < 1e-10


@pytest.mark.parametrize("key", ["tiny", "odd", "hbn"])
def test_eri_fp64_parity(dmet, key):
    wl, lat, lm, bath = case(**CASES[key])
    out = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(bath["c_k"]), "fp64")
    torch.cuda.synchronize()
    ref, im = ok.alg1_eri(lm, bath["c_k"][0], wl.kmesh)
    ref8 = ok.pack_s8(ref)
    got = out["aa"].cpu().numpy()
    mx = np.abs(ref8).max()
    assert np.abs(got - ref8).max() < 1e-10 * mx


def test_eri_fp64_uhf_blocks(dmet):
    wl, lat, lm, bath = case("uodd", kmesh=(3, 2, 1), nao=6, naux=17, nspin=2, seed=19)
    ck = bath["c_k"]
    out = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(ck), "fp64")
    torch.cuda.synchronize()
    for key, (a, b) in {"aa": (0, None), "bb": (1, None), "ab": (0, 1)}.items():
        ref, _ = ok.alg1_eri(lm, ck[a], wl.kmesh, None if b is None else ck[b])
        ref = ok.pack_s8(ref) if b is None else ok.pack_s4(ref)
        got = out[key].cpu().numpy().reshape(ref.shape)
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max(), key


def test_eri_c64_input(dmet):
    """complex64 3-index input promoted to FP64 in the kernels."""
    wl, lat, lm, bath = case(**CASES["odd"])
    lm32 = lm.astype(np.complex64)
    out = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm32), to_dev(bath["c_k"]), "fp64")
    ref, _ = ok.alg1_eri(lm32.astype(np.complex128), bath["c_k"][0], wl.kmesh)
    got = out["aa"].cpu().numpy()
    assert np.abs(got - ok.pack_s8(ref)).max() < 1e-10 * np.abs(ref).max()


def test_end_to_end_gauge_free(dmet):
    """GPU bath -> GPU 1e -> GPU ERI against the oracle chain, gauge-free scalars."""
    wl, lat, lm, bath = case(**CASES["hbn"])
    ck, sv, neo = dmet.dmet_build_bath(wl.kmesh, wl.nao, to_dev(lat.dm_k))
    h, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck, to_dev(lat.h_k))
    g, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck, to_dev(lat.dm_k))
    e1 = float(dmet.dmet_energy_1e(h, g).cpu())
    eri = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), ck, "fp64")["aa"].cpu().numpy()
    full = ok.unpack_s8(eri, wl.neo)
    gg = g[0].cpu().numpy()
    ej = 0.5 * np.einsum("ijkl,ji,lk->", full, gg, gg)
    ek = 0.5 * np.einsum("ijkl,jk,li->", full, gg, gg)
    ref, _ = ok.alg1_eri(lm, bath["c_k"][0], wl.kmesh)
    rh, _ = ok.transform_1e(bath["c_k"], lat.h_k)
    rg, _ = ok.transform_1e(bath["c_k"], lat.dm_k)
    assert abs(e1 - ok.energy_1e(rh, rg)) < 1e-10
    assert abs(np.linalg.norm(full) - np.linalg.norm(ref)) < 1e-10 * np.linalg.norm(ref)
    assert abs(ej - 0.5 * np.einsum("ijkl,ji,lk->", ref, rg[0], rg[0])) < 1e-9
    assert abs(ek - 0.5 * np.einsum("ijkl,jk,li->", ref, rg[0], rg[0])) < 1e-9


# ------------------------------------------------------------ precision forms
# Bound from the target accuracy of the reduced-precision forms: 1e-6 Ha
# max-abs on every ERI element (synthetic ERIs are scaled so that on-site
# (mu0 mu0|mu0 mu0) ~ 1 Ha).
LP_TOL = 1e-6


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x6_i8"])
@pytest.mark.parametrize("key", ["tiny", "odd", "hbn"])
def test_eri_reduced_precision(dmet, key, prec):
    wl, lat, lm, bath = case(**CASES[key])
    out = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(bath["c_k"]), prec)
    torch.cuda.synchronize()
    ref, _ = ok.alg1_eri(lm, bath["c_k"][0], wl.kmesh)
    err = np.abs(out["aa"].cpu().numpy() - ok.pack_s8(ref)).max()
    print(f"{key} {prec} max abs err {err:.3e}")
    assert err < LP_TOL


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x6_i8"])
def test_eri_reduced_precision_uhf(dmet, prec):
    wl, lat, lm, bath = case("uodd", kmesh=(3, 2, 1), nao=6, naux=17, nspin=2, seed=19)
    ck = bath["c_k"]
    out = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(ck), prec)
    torch.cuda.synchronize()
    for key, (a, b) in {"aa": (0, None), "bb": (1, None), "ab": (0, 1)}.items():
        ref, _ = ok.alg1_eri(lm, ck[a], wl.kmesh, None if b is None else ck[b])
        ref = ok.pack_s8(ref) if b is None else ok.pack_s4(ref)
        err = np.abs(out[key].cpu().numpy().reshape(ref.shape) - ref).max()
        assert err < LP_TOL, (key, err)


@pytest.mark.parametrize("key", ["tiny", "hbn"])
def test_eri_bf16x3_error_as_derived(dmet, key):
    """The two-way bf16 split keeps ~2^-17 relative per operand: its error
    stays below 1e-5 Ha but is not held to the 1e-6 bound (the error
    analysis and measured values are in the design notes)."""
    wl, lat, lm, bath = case(**CASES[key])
    out = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(bath["c_k"]), "bf16x3")
    torch.cuda.synchronize()
    ref, _ = ok.alg1_eri(lm, bath["c_k"][0], wl.kmesh)
    err = np.abs(out["aa"].cpu().numpy() - ok.pack_s8(ref)).max()
    print(f"{key} bf16x3 max abs err {err:.3e}")
    assert err < 1e-5


# ------------------------------------------------------------ batched form
def _small_batch():
    """Fragments of uneven size on two small lattices, supercell impurities."""
    import synth
    lats = {"a": synth.Workload("ba", (2, 2, 1), 8, 24, 8, 8, 1, 1.5, 2101),
            "b": synth.Workload("bb", (3, 1, 1), 8, 20, 8, 8, 1, 1.5, 2102)}
    data = {}
    for key, wl in lats.items():
        lat = synth.make_lattice(wl)
        lm = synth.three_index(wl)
        data[key] = (wl, lat, lm)
    rng = np.random.default_rng(5)
    frags = []
    for f in range(9):
        key = "ab"[f % 2]
        wl, lat, lm = data[key]
        neo = int(rng.integers(4, 17))
        nimp = (neo + 1) // 2
        order = synth.supercell_order(wl.kmesh, wl.nao)
        bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, imp_idx=order[:nimp], val_idx=list(range(neo - nimp)))
        frags.append((wl, lm, bath["c_k"][0][:, :, :neo]))
    return frags


@pytest.mark.parametrize("prec", ["bf16x6", "bf16x3", "fp32", "bf16x6_i8", "fp64"])
def test_batched_matches_single_and_oracle(dmet, prec):
    frags = _small_batch()
    dev_lm = {}
    specs = []
    for wl, lm, ck in frags:
        if id(lm) not in dev_lm:
            dev_lm[id(lm)] = to_dev(lm.astype(np.complex64))
        specs.append({"kmesh": wl.kmesh, "nao": wl.nao, "naux": wl.naux, "lmunu": dev_lm[id(lm)],
                      "c_k": to_dev(np.ascontiguousarray(ck))})
    outs = [o.clone() for o in dmet.dmet_transform_eri_batched(specs, prec)]
    torch.cuda.synchronize()
    for (wl, lm, ck), spec, got in zip(frags, specs, outs):
        single = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, spec["lmunu"], spec["c_k"][None], prec)["aa"]
        assert torch.equal(single, got)   # same kernels' arithmetic, same order
        ref, _ = ok.alg1_eri(lm.astype(np.complex64).astype(np.complex128), ck, wl.kmesh)
        err = np.abs(got.cpu().numpy() - ok.pack_s8(ref)).max()
        tol = 1e-10 * max(1.0, np.abs(ref).max()) if prec == "fp64" else (1e-5 if prec == "bf16x3" else LP_TOL)
        assert err < tol, err


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_fp_branches_graph_replay(dmet, prec):
    """FP32 / FP64 batches run the per-fragment kernels on concurrent branches
    (9 fragments over 4 branches, each with its own workspace slice); eager,
    graph-captured replays and single calls give the same bits, with other
    work and synchronisations between the replays."""
    frags = _small_batch()
    dev_lm = {}
    specs = []
    for wl, lm, ck in frags:
        if id(lm) not in dev_lm:
            dev_lm[id(lm)] = to_dev(lm.astype(np.complex64))
        specs.append({"kmesh": wl.kmesh, "nao": wl.nao, "naux": wl.naux, "lmunu": dev_lm[id(lm)],
                      "c_k": to_dev(np.ascontiguousarray(ck))})
    eager = [o.clone() for o in dmet.dmet_transform_eri_batched(specs, prec)]
    torch.cuda.synchronize()
    singles = [dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, sp["lmunu"], sp["c_k"][None], prec)["aa"]
               for (wl, _, _), sp in zip(frags, specs)]
    for a, b in zip(eager, singles):
        assert torch.equal(a, b)
    ws = torch.empty(dmet.dmet_transform_eri_batched_workspace(specs, prec), dtype=torch.uint8, device="cuda:0")
    for rep in range(3):
        for sp in specs:
            sp["eri"].zero_()
        junk = torch.randn(1 << 20, device="cuda:0").sum()   # eager work between replays
        torch.cuda.synchronize()
        outs = dmet.dmet_transform_eri_batched(specs, prec, graph=True, workspace=ws)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(eager, outs):
            assert torch.equal(a, b), rep


def test_batched_graph_replay_and_autotune(dmet, tmp_path, monkeypatch):
    monkeypatch.setenv("DMET_TUNE_CACHE", str(tmp_path / "tune.txt"))
    frags = _small_batch()
    dev_lm = {}
    specs = []
    for wl, lm, ck in frags:
        if id(lm) not in dev_lm:
            dev_lm[id(lm)] = to_dev(lm.astype(np.complex64))
        specs.append({"kmesh": wl.kmesh, "nao": wl.nao, "naux": wl.naux, "lmunu": dev_lm[id(lm)],
                      "c_k": to_dev(np.ascontiguousarray(ck))})
    eager = [o.clone() for o in dmet.dmet_transform_eri_batched(specs, "bf16x6")]
    ws = torch.empty(dmet.dmet_transform_eri_batched_workspace(specs, "bf16x6"), dtype=torch.uint8,
                     device="cuda:0")
    for rep in range(3):
        for s in specs:
            s["eri"].zero_()
        torch.cuda.synchronize()
        outs = dmet.dmet_transform_eri_batched(specs, "bf16x6", graph=True, autotune=True, workspace=ws)
        torch.cuda.synchronize()
        for a, b in zip(eager, outs):
            assert torch.equal(a, b), rep


# ------------------------------------------------- DF output and double counting
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_df_factors_reproduce_eri(dmet, prec):
    """z^T z equals the oracle's ERI (the contraction skipped, Sec. 2.1)."""
    wl, lat, lm, bath = case("uodd", kmesh=(3, 2, 1), nao=6, naux=17, nspin=2, seed=19)
    ck = bath["c_k"]
    z = dmet.dmet_transform_eri_df(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(ck), prec).cpu().numpy()
    assert z.shape == (2, wl.nk * wl.naux, wl.npair)
    tol = 1e-10 if prec == "fp64" else LP_TOL
    for a, b in ((0, 0), (1, 1), (0, 1)):
        ref, _ = ok.alg1_eri(lm, ck[a], wl.kmesh, None if a == b else ck[b])
        got = z[a].T @ z[b]
        refp = ok.pack_s4(ref)
        err = np.abs(got - refp).max()
        assert err < tol * (np.abs(refp).max() if prec == "fp64" else 1.0), (a, b, err)


@pytest.mark.parametrize("nspin", [1, 2])
def test_fock_dc_parity(dmet, nspin):
    from tests.test_fock_dc_pins import _hf_lattice
    import synth
    wl = synth.Workload("dcg", (3, 2, 1), 5, 14, 5, 5, nspin, 1.5, 311 + nspin)
    lat, lm, b, hsup, gs, fk = _hf_lattice(wl)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    ck = bath["c_k"]
    f_eo, _ = ok.transform_1e(ck, fk)
    g_eo, _ = ok.transform_1e(ck, lat.dm_k)
    if nspin == 1:
        eri = ok.alg1_eri(lm, ck[0], wl.kmesh)[0]
    else:
        eri = tuple(ok.alg1_eri(lm, ck[a], wl.kmesh, None if c is None else ck[c])[0]
                    for a, c in ((0, None), (1, None), (0, 1)))
    ref = ok.fock_double_counting(f_eo, g_eo, eri)
    ck_d = to_dev(ck)
    fe, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck_d, to_dev(fk))
    ge, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck_d, to_dev(lat.dm_k))
    e_ref = ok.energy_mf(ref, g_eo, eri)
    for prec, tol in (("fp64", 1e-10), ("bf16x6", 1e-6), ("bf16x6_i8", 1e-6)):
        z = dmet.dmet_transform_eri_df(wl.kmesh, wl.nao, wl.naux, to_dev(lm), ck_d, prec)
        ft_d = dmet.dmet_fock_dc(z, fe, ge)
        ft = ft_d.cpu().numpy()
        err = np.abs(ft - ref).max()
        # mean-field energy of the embedding Hamiltonian from the GPU F~ and F^EO
        e = float(dmet.dmet_energy_mf(ft_d, fe, ge).cpu())
        print(f"fock_dc nspin={nspin} {prec}: {err:.3e}; E_mf {e:.12f} vs {e_ref:.12f}")
        assert err < tol, (prec, err)
        assert abs(e - e_ref) < tol * max(1.0, abs(e_ref)), (prec, e, e_ref)


def test_fock_dc_chunked_against_torch(dmet):
    """Large neo (several 64-wide tiles plus a ragged one) and enough rows P
    that W is built in two chunks with a ragged last split; reference is the
    plain definition J = Z^T (Z g_vec), K = sum_P Z_P g Z_P in float64 torch."""
    neo, nrows, nspin = 200, 4003, 2
    npair = neo * (neo + 1) // 2
    gen = torch.Generator().manual_seed(71)
    z = torch.randn(nspin, nrows, npair, generator=gen, dtype=torch.float64) * 1e-2
    a = torch.randn(nspin, neo, neo, generator=gen, dtype=torch.float64)
    g = (a + a.transpose(1, 2)) * 0.05
    b = torch.randn(nspin, neo, neo, generator=gen, dtype=torch.float64)
    f = b + b.transpose(1, 2)
    zd, gd, fd = z.cuda(), g.cuda().contiguous(), f.cuda().contiguous()
    got = dmet.dmet_fock_dc(zd, fd, gd)
    torch.cuda.synchronize()
    ii, jj = (torch.as_tensor(x, device="cuda") for x in np.tril_indices(neo))
    idx = ii * (ii + 1) // 2 + jj
    full = torch.zeros(nspin, nrows, neo, neo, dtype=torch.float64, device="cuda")
    full[:, :, ii, jj] = zd[:, :, idx]
    full[:, :, jj, ii] = zd[:, :, idx]
    ref = torch.empty_like(fd)
    vtot = sum(torch.einsum("pkl,kl->p", full[t], gd[t]) for t in range(nspin))
    for s in range(nspin):
        jm = torch.einsum("pij,p->ij", full[s], vtot)
        km = torch.zeros(neo, neo, dtype=torch.float64, device="cuda")
        for p0 in range(0, nrows, 512):
            zp = full[s, p0:p0 + 512]
            km += torch.matmul(torch.matmul(zp, gd[s]), zp).sum(0)
        ref[s] = fd[s] - (jm - km)
    err = (got - ref).abs().max().item()
    scale = ref.abs().max().item()
    print(f"fock_dc chunked: max err {err:.3e} (scale {scale:.2e})")
    assert err < 1e-11 * scale


@pytest.mark.parametrize("prec", ["fp64", "bf16x6", "bf16x6_i8"])
def test_non_interacting_bath_impurity_eri(dmet, prec):
    """Impurity-only ERIs (non-interacting bath, Sec. 2.1) equal the impurity
    block of the oracle's full embedding ERIs, for both spins and the ab block."""
    wl, lat, lm, bath = case("uodd", kmesh=(3, 2, 1), nao=6, naux=17, nspin=2, seed=19)
    ck = bath["c_k"]
    nimp = wl.nimp
    out = dmet.dmet_transform_eri_impurity(wl.kmesh, wl.nao, wl.naux, to_dev(lm), to_dev(ck), nimp, prec)
    torch.cuda.synchronize()
    tol = 1e-10 if prec == "fp64" else LP_TOL
    for key, (a, b) in {"aa": (0, None), "bb": (1, None), "ab": (0, 1)}.items():
        full, _ = ok.alg1_eri(lm, ck[a], wl.kmesh, None if b is None else ck[b])
        ref = full[:nimp, :nimp, :nimp, :nimp]
        ref = ok.pack_s8(ref) if b is None else ok.pack_s4(ref)
        err = np.abs(out[key].cpu().numpy().reshape(ref.shape) - ref).max()
        assert err < tol * (np.abs(ref).max() if prec == "fp64" else 1.0), (key, err)


def _unread_blocks(kmesh):
    """(q, k) blocks of lmunu outside the k <-> q-k paired transform: q with
    -q < q (its partner -q is transformed instead) or k > q - k (its partner
    q - k carries the transposed term)."""
    pts = synth_cells(kmesh)
    km = np.asarray(kmesh)

    def idx(v):
        v = np.asarray(v) % km
        return int((v[0] * km[1] + v[1]) * km[2] + v[2])
    nk = len(pts)
    out = []
    for q in range(nk):
        for k in range(nk):
            if idx(-pts[q]) < q or k > idx(pts[q] - pts[k]):
                out.append((q, k))
    return out


def synth_cells(kmesh):
    import synth
    return synth.cells(kmesh)


@pytest.mark.parametrize("prec", ["bf16x6", "fp32"])
@pytest.mark.parametrize("key", ["odd", "hbn"])
def test_paired_transform_reads_half_the_input(dmet, key, prec):
    """The split-bf16 and FP32-3M transforms pair k with q - k (time reversal
    and the Hermiticity of the 3-index tensor): the blocks they do not read may
    hold anything.  Filled with NaN, the ERIs come out bit for bit the same, for
    the single call and for the batched form."""
    wl, lat, lm, bath = case(**CASES[key])
    ck = to_dev(bath["c_k"])
    unread = _unread_blocks(wl.kmesh)
    assert 0.45 * wl.nk ** 2 < len(unread) < 0.8 * wl.nk ** 2
    ref = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, to_dev(lm), ck, prec)["aa"].clone()
    lm_nan = lm.copy()
    for q, k in unread:
        lm_nan[q, k] = np.nan
    lm_d = to_dev(lm_nan)
    got = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, lm_d, ck, prec)["aa"]
    torch.cuda.synchronize()
    assert torch.equal(ref, got)
    spec = [{"kmesh": wl.kmesh, "nao": wl.nao, "naux": wl.naux, "lmunu": lm_d, "c_k": ck[0].contiguous()}]
    bat = dmet.dmet_transform_eri_batched(spec, prec)[0]
    torch.cuda.synchronize()
    assert torch.equal(ref, bat)


@pytest.mark.parametrize("prec", ["bf16x6", "bf16x3"])
def test_batched_64x64_stage2_tiles(dmet, prec, monkeypatch):
    """DMET_XF2_SMALL_NEO=0 sends every fragment through the 64 x 64 one-L
    stage-2 tiles (k_xf2_batched, the path of fragments above 256 orbitals):
    same bits as the single-fragment call and within the bound of the oracle."""
    monkeypatch.setenv("DMET_XF2_SMALL_NEO", "0")
    frags = _small_batch()
    dev_lm = {}
    specs = []
    for wl, lm, ck in frags:
        if id(lm) not in dev_lm:
            dev_lm[id(lm)] = to_dev(lm.astype(np.complex64))
        specs.append({"kmesh": wl.kmesh, "nao": wl.nao, "naux": wl.naux, "lmunu": dev_lm[id(lm)],
                      "c_k": to_dev(np.ascontiguousarray(ck))})
    outs = [o.clone() for o in dmet.dmet_transform_eri_batched(specs, prec)]
    torch.cuda.synchronize()
    for (wl, lm, ck), spec, got in zip(frags, specs, outs):
        single = dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, spec["lmunu"], spec["c_k"][None], prec)["aa"]
        assert torch.equal(single, got)
        ref, _ = ok.alg1_eri(lm.astype(np.complex64).astype(np.complex128), ck, wl.kmesh)
        err = np.abs(got.cpu().numpy() - ok.pack_s8(ref)).max()
        tol = 1e-10 * max(1.0, np.abs(ref).max()) if prec == "fp64" else (1e-5 if prec == "bf16x3" else LP_TOL)
        assert err < tol, err


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_fp_branches_graph_replay(dmet, prec):
    """FP32 / FP64 batches run the per-fragment kernels on concurrent branches
    (9 fragments over 4 branches, each with its own workspace slice); eager,
    graph-captured replays and single calls give the same bits, with other
    work and synchronisations between the replays."""
    frags = _small_batch()
    dev_lm = {}
    specs = []
    for wl, lm, ck in frags:
        if id(lm) not in dev_lm:
            dev_lm[id(lm)] = to_dev(lm.astype(np.complex64))
        specs.append({"kmesh": wl.kmesh, "nao": wl.nao, "naux": wl.naux, "lmunu": dev_lm[id(lm)],
                      "c_k": to_dev(np.ascontiguousarray(ck))})
    eager = [o.clone() for o in dmet.dmet_transform_eri_batched(specs, prec)]
    torch.cuda.synchronize()
    singles = [dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, sp["lmunu"], sp["c_k"][None], prec)["aa"]
               for (wl, _, _), sp in zip(frags, specs)]
    for a, b in zip(eager, singles):
        assert torch.equal(a, b)
    ws = torch.empty(dmet.dmet_transform_eri_batched_workspace(specs, prec), dtype=torch.uint8, device="cuda:0")
    for rep in range(3):
        for sp in specs:
            sp["eri"].zero_()
        junk = torch.randn(1 << 20, device="cuda:0").sum()   # eager work between replays
        torch.cuda.synchronize()
        outs = dmet.dmet_transform_eri_batched(specs, prec, graph=True, workspace=ws)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(eager, outs):
            assert torch.equal(a, b), rep
