"""Pins of the plane-wave (FFTDF) oracle, App. B / Alg. 2 (NEXT-4).

Alg. 2 on k-space inputs (oracle.kspace.alg2_eri) is checked against an
independent brute force on the Born-von Karman supercell grid
(oracle.supercell.fftdf_eri: EO orbitals on the full grid, one supercell FFT of
their pair densities): the k-blocking of the grid is exact, so the two agree to
rounding.  Planted mistakes in the k-space steps (the e^{iq.r} phase, the
kernel's q shift, the side of the conjugation) break that agreement, and the
result has the symmetry, realness and positive semidefiniteness of a Coulomb
ERI.  Non-orthogonal cells: the reciprocal vectors satisfy a_i . b_j = 2 pi
delta_ij and have the closed form of the hexagonal lattice, and the ERIs do not
change when the whole cell is rotated (which a transposed reciprocal metric
would break).
"""
import numpy as np
import pytest

import synth
from oracle import kspace as ok
from oracle import supercell as sc


@pytest.fixture(scope="module", params=["fft_tiny", "fft_odd", "fft_hex"])
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


def test_reciprocal_vectors():
    rng = np.random.default_rng(5)
    a = np.eye(3) * 3.0 + rng.uniform(-0.8, 0.8, (3, 3))
    b = ok.reciprocal_vectors(a)
    assert np.abs(a @ b.T - 2 * np.pi * np.eye(3)).max() < 1e-12
    # hexagonal lattice, a_1 = (a, 0, 0), a_2 = (a/2, a sqrt3/2, 0), a_3 = (0, 0, c):
    # |b_1| = |b_2| = 4 pi / (a sqrt 3) and b_1 . b_2 = -|b_1|^2 / 2 (120 degrees)
    h = np.asarray(synth.HEX_CELL)
    alen, c = h[0, 0], h[2, 2]
    bh = ok.reciprocal_vectors(h)
    gm = bh @ bh.T
    b2 = (4 * np.pi / (alen * np.sqrt(3))) ** 2
    assert np.allclose(np.diag(gm), [b2, b2, (2 * np.pi / c) ** 2], rtol=1e-13)
    assert abs(gm[0, 1] + 0.5 * b2) < 1e-12 * b2 and abs(gm[0, 2]) < 1e-12 and abs(gm[1, 2]) < 1e-12
    # three lengths are the orthorhombic cell
    assert np.array_equal(ok.cell_vectors((2.0, 3.0, 4.0)), np.diag([2.0, 3.0, 4.0]))


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    return q if np.linalg.det(q) > 0 else -q


def test_alg2_rotation_invariant():
    """Rotating every lattice vector (and with them the AO centres, which are
    fractional) leaves the pair densities on the grid and the ERIs unchanged."""
    wl, g = synth.FFT_CONFIGS["fft_hex"]
    rot = _rotation(11)
    g_rot = synth.FftGrid(g.n, tuple(map(tuple, g.lattice @ rot.T)))
    lat = synth.make_lattice(wl)
    ck = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)["c_k"][0]
    rho = synth.fftdf_pair_density(wl, g)
    rho_rot = synth.fftdf_pair_density(wl, g_rot)
    assert np.abs(rho - rho_rot).max() < 1e-12 * np.abs(rho).max()
    e, _ = ok.alg2_eri(rho, ck, wl.kmesh, g.n, g.cell)
    e_rot, _ = ok.alg2_eri(rho_rot, ck, wl.kmesh, g_rot.n, g_rot.cell)
    assert np.abs(e - e_rot).max() < 1e-12 * np.abs(e).max()
    # the same check fails for a kernel built on the transposed metric b^T b
    bt = ok.reciprocal_vectors(g.lattice)
    brt = ok.reciprocal_vectors(g_rot.lattice)
    assert np.abs(bt.T @ bt - brt.T @ brt).max() > 1e-3 * np.abs(bt).max() ** 2
    assert np.abs(bt @ bt.T - brt @ brt.T).max() < 1e-12 * np.abs(bt).max() ** 2
