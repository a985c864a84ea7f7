"""Pins of the plane-wave (FFTDF) oracle, App. B / Alg. 2 (NEXT-4).

Alg. 2 on k-space inputs (oracle.kspace.alg2_eri) is checked against an
independent brute force on the Born-von Karman supercell grid
(oracle.supercell.fftdf_eri: EO orbitals on the full grid, one supercell FFT of
their pair densities): the k-blocking of the grid is exact, so the two agree to
rounding.  Planted mistakes in the k-space steps (the e^{iq.r} phase, the
kernel's q shift, the side of the conjugation) break that agreement, and the
result has the symmetry, realness and positive semidefiniteness of a Coulomb
ERI.
"""
import numpy as np
import pytest

import synth
from oracle import kspace as ok
from oracle import supercell as sc


@pytest.fixture(scope="module", params=["fft_tiny", "fft_odd"])
def fcase(request):
    wl, g = synth.FFT_CONFIGS[request.param]
    lat = synth.make_lattice(wl)
    rho = synth.fftdf_pair_density(wl, g)
    chi = synth.fftdf_ao_supercell(wl, g)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    return wl, g, rho, chi, bath


def test_alg2_equals_supercell_fft(fcase):
    wl, g, rho, chi, bath = fcase
    ck = bath["c_k"][0]
    cr = bath["c_r"][0].reshape(wl.nk * wl.nao, wl.neo)
    ek, im = ok.alg2_eri(rho, ck, wl.kmesh, g.n, g.cell)
    es = sc.fftdf_eri(chi, cr, wl.kmesh, g.n, g.cell)
    scale = np.abs(es).max()
    assert 0.1 < scale < 10.0
    assert im < 1e-12 * scale
    assert np.abs(ek - es).max() < 1e-12 * scale


def test_alg2_invariants(fcase):
    wl, g, rho, chi, bath = fcase
    e, _ = ok.alg2_eri(rho, bath["c_k"][0], wl.kmesh, g.n, g.cell)
    assert np.abs(e - e.transpose(1, 0, 2, 3)).max() < 1e-13
    assert np.abs(e - e.transpose(2, 3, 0, 1)).max() < 1e-13
    n = e.shape[0]
    ev = np.linalg.eigvalsh(e.reshape(n * n, n * n))
    assert ev.min() > -1e-12 * ev.max()          # 4 pi / |q+G|^2 >= 0


def test_frequencies_partition_the_supercell_grid():
    """Every supercell frequency appears for exactly one (q, G)."""
    kmesh, n = (3, 2, 1), (6, 5, 8)
    seen = set()
    nk = int(np.prod(kmesh))
    for q in range(nk):
        for j in map(tuple, ok.fftdf_frequencies(kmesh, n, q)):
            assert j not in seen
            seen.add(j)
    full = set()
    f = [np.fft.fftfreq(a * b, 1.0 / (a * b)).astype(int) for a, b in zip(kmesh, n)]
    for x in f[0]:
        for y in f[1]:
            for z in f[2]:
                full.add((x, y, z))
    assert seen == full


def _alg2_planted(rho, c_k, kmesh, grid_n, cell, mistake):
    """Alg. 2 with one planted mistake (oracle side only)."""
    nk = rho.shape[0]
    nr = int(np.prod(grid_n))
    dv = float(np.prod(cell)) / nr
    idx = np.indices(grid_n).reshape(3, -1).T
    eri = 0
    for q in range(nk):
        m = ok.mesh_points(kmesh)[q]
        ph = np.exp(2j * np.pi * (idx * (m / (np.asarray(kmesh) * np.asarray(grid_n)))[None, :]).sum(axis=1))
        if mistake == "no_phase":
            ph = np.ones_like(ph)
        kern = ok.coulomb_kernel(kmesh, grid_n, cell, 0 if mistake == "no_q_in_kernel" else q)
        x = ok.alg1_embedded_3index(rho, c_k, kmesh, q)
        n = x.shape[1]
        w = np.fft.ifftn((ph[:, None, None] * x).reshape(*grid_n, n, n), axes=(0, 1, 2)).reshape(nr, n, n) * nr
        v = np.fft.fftn((w * kern[:, None, None]).reshape(*grid_n, n, n), axes=(0, 1, 2)).reshape(nr, n, n) / nr
        v = v * ph.conj()[:, None, None]
        lhs = x if mistake == "conj_right" else x.conj()
        eri = eri + dv / nk * (lhs.reshape(nr, n * n).T @ v.reshape(nr, n * n))
    return eri.real.reshape(n, n, n, n)


@pytest.mark.parametrize("mistake", ["no_phase", "no_q_in_kernel", "conj_right"])
def test_planted_mistakes_break_parity(mistake):
    wl, g = synth.FFT_CONFIGS["fft_odd"]
    lat = synth.make_lattice(wl)
    rho = synth.fftdf_pair_density(wl, g)
    chi = synth.fftdf_ao_supercell(wl, g)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    cr = bath["c_r"][0].reshape(wl.nk * wl.nao, wl.neo)
    es = sc.fftdf_eri(chi, cr, wl.kmesh, g.n, g.cell)
    bad = _alg2_planted(rho, bath["c_k"][0], wl.kmesh, g.n, g.cell, mistake)
    assert np.abs(bad - es).max() > 1e-4 * np.abs(es).max()
