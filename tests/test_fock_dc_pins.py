"""Pins of the double-counting correction (Eq. ``fock double counting``).

With the lattice Fock matrix defined from the same density-fitted ERIs,
F = h + J[g] - K[g]/2 (restricted, g the spin-summed density; per-spin
F_s = h + J[g_a + g_b] - K[g_s] unrestricted), linearity of J and K gives the
supercell identity

    F~ = C^T (h + J[g_core] - K[g_core]/2) C,   g_core = g - C C^T g C C^T,

for any orthonormal embedding orbitals C: the correction removes exactly the
mean-field interaction of the embedded density.  Both sides are computed
independently (the left side by the k-space oracle with embedding ERIs from
Alg. 1, the right side by supercell J/K).
"""
import numpy as np
import pytest

import synth
from oracle import kspace as ok
from oracle import supercell as sc


def _hf_lattice(wl):
    """Lattice whose F(k) is the HF Fock matrix of its own density."""
    lat = synth.make_lattice(wl)
    lm, b = synth.three_index(wl, real_space=True)
    hsup = sc.supercell_operator(lat.t_h, wl.kmesh)
    gs = [sc.supercell_dm(lat.dm_k[s], wl.kmesh)[0] for s in range(wl.nspin)]
    if wl.nspin == 1:
        j, k = sc.coulomb_exchange(b, wl.kmesh, 2 * gs[0])
        fsup = [hsup + j - 0.5 * k]
    else:
        j, _ = sc.coulomb_exchange(b, wl.kmesh, gs[0] + gs[1])
        fsup = [hsup + j - sc.coulomb_exchange(b, wl.kmesh, gs[s])[1] for s in range(2)]
    u = sc.bloch_unitary(wl.kmesh, wl.nao)
    fk = np.empty((wl.nspin, wl.nk, wl.nao, wl.nao), dtype=np.complex128)
    for s in range(wl.nspin):
        blk = u.conj().T @ fsup[s] @ u
        for q in range(wl.nk):
            fk[s, q] = blk[q * wl.nao:(q + 1) * wl.nao, q * wl.nao:(q + 1) * wl.nao]
    return lat, lm, b, hsup, gs, fk


def _dc_case(wl):
    lat, lm, b, hsup, gs, fk = _hf_lattice(wl)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    ck = bath["c_k"]
    f_eo, _ = ok.transform_1e(ck, fk)
    g_eo, _ = ok.transform_1e(ck, lat.dm_k)
    if wl.nspin == 1:
        eri = ok.alg1_eri(lm, ck[0], wl.kmesh)[0]
    else:
        eri = tuple(ok.alg1_eri(lm, ck[a], wl.kmesh, None if c is None else ck[c])[0]
                    for a, c in ((0, None), (1, None), (0, 1)))
    ft = ok.fock_double_counting(f_eo, g_eo, eri)
    # supercell right side
    cs = [bath["c_r"][s].reshape(-1, bath["neo"][s]) for s in range(wl.nspin)]
    core = [gs[s] - cs[s] @ cs[s].T @ gs[s] @ cs[s] @ cs[s].T for s in range(wl.nspin)]
    if wl.nspin == 1:
        j, k = sc.coulomb_exchange(b, wl.kmesh, 2 * core[0])
        ref = [cs[0].T @ (hsup + j - 0.5 * k) @ cs[0]]
    else:
        j, _ = sc.coulomb_exchange(b, wl.kmesh, core[0] + core[1])
        ref = [cs[s].T @ (hsup + j - sc.coulomb_exchange(b, wl.kmesh, core[s])[1]) @ cs[s] for s in range(2)]
    return ft, np.array(ref), (f_eo, g_eo, eri)


@pytest.mark.parametrize("nspin", [1, 2])
def test_double_counting_supercell_identity(nspin):
    wl = synth.Workload("dc", (3, 2, 1), 5, 14, 5, 5, nspin, 1.5, 301 + nspin)
    ft, ref, _ = _dc_case(wl)
    assert np.abs(ft - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


def test_double_counting_planted_mistakes():
    """Dropping the 1/2, or using (ij|kl) for exchange, breaks the identity."""
    wl = synth.Workload("dc1", (3, 2, 1), 5, 14, 5, 5, 1, 1.5, 302)
    ft, ref, (f_eo, g_eo, eri) = _dc_case(wl)
    g = 2 * g_eo[0]
    j = np.einsum("ijkl,lk->ij", eri, g)
    k_ok = np.einsum("iklj,kl->ij", eri, g)
    bad1 = f_eo[0] - (j - k_ok)
    bad2 = f_eo[0] - (j - 0.5 * np.einsum("ijkl,kl->ij", eri, g))
    for bad in (bad1, bad2):
        assert np.abs(bad - ref[0]).max() > 1e-4


def _hf_energy(hsup, b, kmesh, dens):
    """Hartree-Fock energy of the BvK supercell at per-spin densities `dens`
    (restricted: one per-spin density, spin-summed 2 g)."""
    if len(dens) == 1:
        g = 2.0 * dens[0]
        j, k = sc.coulomb_exchange(b, kmesh, g)
        return float(np.sum(hsup * g) + 0.5 * np.sum((j - 0.5 * k) * g))
    j, _ = sc.coulomb_exchange(b, kmesh, dens[0] + dens[1])
    e = 0.0
    for g in dens:
        k = sc.coulomb_exchange(b, kmesh, g)[1]
        e += float(np.sum(hsup * g) + 0.5 * np.sum((j - k) * g))
    return e


@pytest.mark.parametrize("nspin", [1, 2])
def test_mean_field_energy_splits_the_lattice_energy(nspin):
    """Mean-field energy of the embedding Hamiltonian (F~ plus embedding ERIs,
    Hartree-Fock expression) plus the Hartree-Fock energy of the core density
    equals the Hartree-Fock energy of the whole supercell: the core-embedding
    interaction sits in F~, the embedding-embedding one in the ERIs."""
    wl = synth.Workload("emf", (3, 2, 1), 5, 14, 5, 5, nspin, 1.5, 321 + nspin)
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
    ft = ok.fock_double_counting(f_eo, g_eo, eri)
    e_emb = ok.energy_mf(ft, g_eo, eri)
    cs = [bath["c_r"][s].reshape(-1, bath["neo"][s]) for s in range(nspin)]
    core = [gs[s] - cs[s] @ cs[s].T @ gs[s] @ cs[s] @ cs[s].T for s in range(nspin)]
    e_tot = _hf_energy(hsup, b, wl.kmesh, gs)
    e_core = _hf_energy(hsup, b, wl.kmesh, core)
    assert abs(e_emb + e_core - e_tot) < 1e-10 * max(1.0, abs(e_tot))
    # a dropped 1/2 on exchange, or F^EO in place of F~, breaks the split
    if nspin == 1:
        g = 2.0 * g_eo[0]
        wrong = e_emb - 0.25 * np.einsum("ijkl,jk,li->", eri, g, g)
        assert abs(wrong + e_core - e_tot) > 1e-6
    assert abs(ok.energy_mf(f_eo, g_eo, eri) + e_core - e_tot) > 1e-6
