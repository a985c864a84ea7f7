"""Seeded synthetic inputs for the periodic DMET embedding transform.

This module is shared by the FP64 CPU oracle (``oracle/``), the tests and the
benchmark.  It holds none of the embedding method's arithmetic (no bath, no
embedding-orbital construction, no integral transformation): it only draws
random real-space lattice quantities and hands them over in the k-space form
that the embedding transform consumes.

Stand-ins.  The paper computes its inputs with PySCF (Gaussian density fitting
of GTH-DZVP crystal AOs, Sec. 2.2).  None of that is available here, so every
workload is synthetic, with the paper's shapes: a Gamma-centred k-mesh
(Sec. 2.2), nao crystal AOs per cell, an auxiliary basis about ten times the AO
count (Sec. 2.2) and up to ~300 embedding orbitals (the BN example after
Alg. 1).

Conventions (the paper fixes only the sign of the LO->EO Fourier transform,
Eq. ``C loemb k``; the rest is this project's reading, chosen so that
Alg. 1 reproduces the real-space supercell transform exactly):

* k-mesh: Gamma-centred, N_k = N1*N2*N3 points, k index (n1*N2 + n2)*N3 + n3;
  cells R indexed the same way over the Born-von Karman (BvK) supercell;
  exp(i k.R) = exp(2 pi i sum_d n_d m_d / N_d).
* one-body: t_{mu nu}(R) = <mu,0|h|nu,R> (real, t(-R) = t(R)^T) and
  h(k) = sum_R exp(+i k.R) t(R).
* 3-index: (L|mu k1, nu k2) = sum_{R1,R2} exp(-i k1.R1) exp(+i k2.R2)
  B_L(mu R1, nu R2), with the fitting function L in cell 0, B real and
  symmetric under (mu R1) <-> (nu R2), so that the lattice 4-index integral is
  sum_{L,R_L} B_L(..-R_L) B_L(..-R_L) (Eq. ``density fitting``).  It is stored
  as lmunu[q][k][L][mu][nu] = (L| mu k, nu k-q), the momentum transfer of the
  fitting function being q = k_mu - k_nu (Sec. 2.1, text before Alg. 1).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "CONFIGS", "cells", "min_image_length", "kq_index",
    "make_lattice", "three_index", "three_index_block", "Lattice",
    "FftGrid", "FFT_CONFIGS", "fftdf_pair_density", "fftdf_ao_supercell",
    "random_lattice_unitary", "decouple_orbital",
]


@dataclass(frozen=True)
class Workload:
    """Shape of one synthetic workload (all sizes per unit cell)."""
    name: str
    kmesh: tuple
    nao: int
    naux: int
    nimp: int
    nval: int
    nspin: int
    xi: float            # decay length of hopping and 3-index, in cells
    seed: int
    dtype: str = "c128"  # storage type of the 3-index tensor

    @property
    def nk(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def neo(self) -> int:
        return self.nimp + self.nval

    @property
    def npair(self) -> int:
        return self.neo * (self.neo + 1) // 2


# Shapes of the paper's three solids (Sec. 2.2 / Sec. 3): a 2D h-BN monolayer
# with 26 AOs per cell (GTH-DZVP, B and N), a Si crystal with 2x26 AOs and an
# AFM NiO rhombohedral cell with two formula units, spin unrestricted.  The
# auxiliary size is about 8-10x nao (Sec. 2.2).  Impurity = all LOs of cell 0,
# bath = one SVD column per impurity LO, so neo = 2 nao.
CONFIGS = {
    "tiny": Workload("tiny", (2, 2, 1), 8, 40, 8, 8, 1, 1.5, 1000),
    "hbn": Workload("hbn", (4, 4, 1), 26, 200, 26, 26, 1, 2.0, 1001),
    "si": Workload("si", (3, 3, 3), 52, 400, 52, 52, 1, 2.0, 1002),
    "nio": Workload("nio", (2, 2, 2), 150, 1200, 150, 150, 2, 2.0, 1003),
}


# The paper's own timed example (Sec. 2.1, after Alg. 1): a BN 3x3x1 cluster
# in a 6x6x1 mean-field mesh, 26 AOs per cell (GTH-DZVP), an auxiliary basis
# of ~10 x nao, and a valence-only bath of 8 orbitals per impurity cell
# (GTH-SZV minimal basis): 936 crystal AOs -> 234 + 72 = 306 embedding orbitals.
BN33 = Workload("bn33", (6, 6, 1), 26, 260, 234, 72, 1, 2.0, 1006)


def bn33_impurity():
    """(imp_idx, val_idx) of the BN 3x3x1 example: the 9 cells (a, b) with
    a, b < 3, all 26 LOs each; valence = the first 4 AOs (2s2p) of each of the
    two 13-AO atom blocks of every impurity cell (positions in imp_idx)."""
    pts = cells(BN33.kmesh)
    imp_cells = [i for i, p in enumerate(pts) if p[0] < 3 and p[1] < 3]
    imp = [c * BN33.nao + m for c in imp_cells for m in range(BN33.nao)]
    val = [ci * BN33.nao + a * 13 + m for ci in range(len(imp_cells)) for a in range(2) for m in range(4)]
    return imp, val


def cells(kmesh) -> np.ndarray:
    """Integer coordinates (row-major) of the N_k cells / k-points, [N_k][3]."""
    n1, n2, n3 = kmesh
    g = np.indices((n1, n2, n3)).reshape(3, -1).T
    return g.astype(np.int64)


def min_image_length(kmesh) -> np.ndarray:
    """Minimum-image length |R| (cell units, orthonormal axes) on the BvK torus."""
    c = cells(kmesh).astype(np.float64)
    n = np.asarray(kmesh, dtype=np.float64)
    c = np.minimum(c, n - c)
    return np.sqrt((c * c).sum(axis=1))


def kq_index(kmesh) -> np.ndarray:
    """kmq[q][k] = index of k - q, wrapped per axis modulo N_d."""
    c = cells(kmesh)
    n = np.asarray(kmesh)
    nk = len(c)
    out = np.empty((nk, nk), dtype=np.int64)
    for iq in range(nk):
        d = (c - c[iq]) % n
        out[iq] = (d[:, 0] * n[1] + d[:, 1]) * n[2] + d[:, 2]
    return out


def neg_index(kmesh) -> np.ndarray:
    """Index of -k (wrapped)."""
    c = cells(kmesh)
    n = np.asarray(kmesh)
    d = (-c) % n
    return (d[:, 0] * n[1] + d[:, 1]) * n[2] + d[:, 2]


def _phase_kR(kmesh) -> np.ndarray:
    """exp(+i k.R) as a [N_k(k)][N_k(R)] matrix (generator use only)."""
    c = cells(kmesh)
    n = np.asarray(kmesh)
    nk = len(c)
    num = np.zeros((nk, nk), dtype=np.int64)
    for d in range(3):
        num += np.outer(c[:, d], c[:, d]) * (nk // n[d])
    num %= nk
    return np.exp(2j * np.pi * num / nk)


def _hopping(rng, kmesh, nao, xi, scale) -> np.ndarray:
    """Real t(R) [N_k][nao][nao] with t(-R) = t(R)^T and an exp(-|R|/xi) envelope."""
    nk = int(np.prod(kmesh))
    env = np.exp(-min_image_length(kmesh) / xi)
    g = rng.standard_normal((nk, nao, nao)) * scale * env[:, None, None]
    neg = neg_index(kmesh)
    return 0.5 * (g + g[neg].transpose(0, 2, 1))


@dataclass
class Lattice:
    """One-body inputs of a workload (all FP64/complex128)."""
    wl: Workload
    t_h: np.ndarray          # [N_k R][nao][nao] real hopping of h
    t_f: np.ndarray          # [nspin][N_k R][nao][nao] real Fock in real space
    h_k: np.ndarray          # [nspin][N_k][nao][nao] complex128 (same for both spins)
    f_k: np.ndarray          # [nspin][N_k][nao][nao] complex128
    dm_k: np.ndarray         # [nspin][N_k][nao][nao] complex128, per-spin projector
    mo_energy: np.ndarray    # [nspin][N_k][nao]
    attempts: int = 1
    extra: dict = field(default_factory=dict)


def make_lattice(wl: Workload, spin_split: float = 0.2, v_scale: float = 0.05,
                 hop_scale: float = 0.1, min_gap: float = 1e-4) -> Lattice:
    """Random insulating mean-field on the k-mesh.

    h(k) from a decaying random hopping t(R) (std ``hop_scale`` Ha), a Fock
    matrix F_s(k) = h(k) + v(k) + s*Delta*diag(m) with v an independent draw
    (std ``v_scale``) and, for nspin = 2, an antiferromagnetic staggered field
    m = +1 on AOs [0, nao/4), -1 on [nao/4, nao/2), 0 elsewhere (the two Ni
    sublattices of AFM NiO).  The per-spin density matrix gamma_s(k) is the
    projector onto the lowest nao/2 bands of F_s(k); a draw whose per-k gap
    is below ``min_gap`` is rejected and redrawn with seed + 1000*attempt.
    """
    nk, nao = wl.nk, wl.nao
    ph = _phase_kR(wl.kmesh)
    nocc = nao // 2
    for attempt in range(20):
        seed = wl.seed + 1000 * attempt
        t_h = _hopping(np.random.default_rng([seed, 0]), wl.kmesh, nao, wl.xi, hop_scale)
        t_v = _hopping(np.random.default_rng([seed, 1]), wl.kmesh, nao, wl.xi, v_scale)
        m = np.zeros(nao)
        m[: nao // 4] = 1.0
        m[nao // 4: nao // 2] = -1.0
        t_f = np.empty((wl.nspin, nk, nao, nao))
        for s in range(wl.nspin):
            sign = 1.0 if s == 0 else -1.0
            t_f[s] = t_h + t_v
            if wl.nspin == 2:
                t_f[s, 0] += sign * spin_split * np.diag(m)
        h_k1 = np.einsum("kR,Rij->kij", ph, t_h)
        h_k = np.broadcast_to(h_k1, (wl.nspin, nk, nao, nao)).copy()
        f_k = np.einsum("kR,sRij->skij", ph, t_f)
        f_k = 0.5 * (f_k + f_k.conj().transpose(0, 1, 3, 2))
        h_k = 0.5 * (h_k + h_k.conj().transpose(0, 1, 3, 2))
        dm_k = np.empty_like(f_k)
        mo_e = np.empty((wl.nspin, nk, nao))
        ok = True
        for s in range(wl.nspin):
            for k in range(nk):
                e, v = np.linalg.eigh(f_k[s, k])
                mo_e[s, k] = e
                if e[nocc] - e[nocc - 1] < min_gap:
                    ok = False
                occ = v[:, :nocc]
                dm_k[s, k] = occ @ occ.conj().T
        if ok:
            return Lattice(wl, t_h, t_f, h_k, f_k, dm_k, mo_e, attempts=attempt + 1)
    raise RuntimeError("could not draw a gapped mean-field")


def _three_index_scale(wl: Workload) -> float:
    """s_B such that the expected on-site (mu0 mu0|mu0 mu0) = sum_{L,R} B_L(muR,muR)^2 is 1 Ha."""
    e4 = np.exp(-4.0 * min_image_length(wl.kmesh) / wl.xi).sum()
    return 1.0 / math.sqrt(2.0 * wl.naux * e4)


def three_index_block(wl: Workload, l0: int, l1: int, real_space: bool = False):
    """3-index quantities for auxiliary functions L in [l0, l1).

    Returns ``(kspace, B)`` where kspace has shape [L][N_k k1][nao][N_k k2][nao]
    (complex128, (L|mu k1, nu k2)) and B (only if ``real_space``) has shape
    [L][N_k R1][nao][N_k R2][nao] (real).  Each L draws from its own stream
    default_rng([seed, 100, L]), so any block can be produced independently.
    """
    n1, n2, n3 = wl.kmesh
    nk, nao = wl.nk, wl.nao
    env = np.exp(-min_image_length(wl.kmesh) / wl.xi).reshape(n1, n2, n3)
    sb = _three_index_scale(wl)
    envb = (env[:, :, :, None, None, None, None, None]
            * env[None, None, None, None, :, :, :, None])
    nl = l1 - l0
    ks = np.empty((nl, nk, nao, nk, nao), dtype=np.complex128)
    bs = np.empty((nl, nk, nao, nk, nao)) if real_space else None
    for i, L in enumerate(range(l0, l1)):
        g = np.random.default_rng([wl.seed, 100, L]).standard_normal(
            (n1, n2, n3, nao, n1, n2, n3, nao))
        b = (g + g.transpose(4, 5, 6, 7, 0, 1, 2, 3)) * (sb / math.sqrt(2.0))
        b *= envb
        if real_space:
            bs[i] = b.reshape(nk, nao, nk, nao)
        # sum_R1 exp(-i k1.R1): forward DFT; sum_R2 exp(+i k2.R2): N_k * inverse DFT
        a = np.fft.fftn(b, axes=(0, 1, 2))
        a = np.fft.ifftn(a, axes=(4, 5, 6)) * nk
        ks[i] = a.reshape(nk, nao, nk, nao)
    return ks, bs


def three_index(wl: Workload, real_space: bool = False, dtype=np.complex128,
                threads: Optional[int] = None, out: Optional[np.ndarray] = None):
    """Full lmunu[q][k][L][mu][nu] = (L|mu k, nu k-q) tensor (and optionally B).

    Built in auxiliary blocks on a thread pool; ``out`` may be a preallocated
    (e.g. pinned) array of the right shape and dtype.
    """
    nk, nao, naux = wl.nk, wl.nao, wl.naux
    kmq = kq_index(wl.kmesh)
    if out is None:
        out = np.empty((nk, nk, naux, nao, nao), dtype=dtype)
    bfull = np.empty((naux, nk, nao, nk, nao)) if real_space else None
    blk = max(1, min(32, naux // 8))
    starts = list(range(0, naux, blk))

    def work(l0):
        l1 = min(naux, l0 + blk)
        ks, bs = three_index_block(wl, l0, l1, real_space)
        for q in range(nk):
            for k in range(nk):
                out[q, k, l0:l1] = ks[:, k, :, kmq[q, k], :]
        if real_space:
            bfull[l0:l1] = bs

    nthr = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(nthr) as ex:
        list(ex.map(work, starts))
    return (out, bfull) if real_space else out


def random_lattice_unitary(kmesh, nao, seed, scale=0.3) -> np.ndarray:
    """A k-dependent unitary U(k) [N_k][nao][nao] complex128 that stands in for
    a crystal-AO -> LO rotation C^{k,AO,LO} (orthonormal AOs assumed):
    U(k) = expm(S(k)), S(k) = sum_R exp(+i k.R) A(R) with real A(-R) = -A(R)^T,
    so S(k) is anti-Hermitian (U unitary) and U(-k) = conj(U(k)) (a real
    rotation in the supercell, time-reversal symmetric)."""
    from scipy.linalg import expm
    nk = int(np.prod(kmesh))
    rng = np.random.default_rng([seed, 500])
    env = np.exp(-min_image_length(kmesh))
    g = rng.standard_normal((nk, nao, nao)) * scale * env[:, None, None]
    a = 0.5 * (g - g[neg_index(kmesh)].transpose(0, 2, 1))
    sk = np.einsum("kR,Rij->kij", _phase_kR(kmesh), a)
    return np.array([expm(x) for x in sk])


def decouple_orbital(dm_k, mu) -> np.ndarray:
    """A copy of the per-spin density matrices in which orbital mu of every cell
    is fully occupied and has no coherence with any other orbital (a core-like
    orbital): gamma(k)[mu, :] = gamma(k)[:, mu] = e_mu for every k.  Its column
    of the impurity-environment block vanishes, so it couples to no bath."""
    out = np.array(dm_k, copy=True)
    out[..., mu, :] = 0.0
    out[..., :, mu] = 0.0
    out[..., mu, mu] = 1.0
    return out


def random_orthonormal(rng, n, m) -> np.ndarray:
    """n x m real matrix with orthonormal columns (QR of a Gaussian draw)."""
    q, r = np.linalg.qr(rng.standard_normal((n, m)))
    return q * np.sign(np.diag(r))[None, :]


# Batched workload: many fragments of uneven size on two lattices (an
# h-BN/Si-sized cell, nao 52, naux 400, on 2x2x2 and 3x3x3 meshes); each
# fragment is a supercell impurity of ceil(neo/2) LOs taken from the cells
# nearest the origin (by minimum-image |R|, then mu) and a bath of
# neo - n_imp orbitals from the first SVD columns (Sec. 2.1: the impurity
# may be a cell or a supercell).
BATCH_LATTICES = {
    "b222": Workload("b222", (2, 2, 2), 52, 400, 52, 52, 1, 2.0, 1004, "c64"),
    "b333": Workload("b333", (3, 3, 3), 52, 400, 52, 52, 1, 2.0, 1005, "c64"),
}


def supercell_order(kmesh, nao):
    """Supercell orbitals (cell*nao + mu) ordered by |R| (min image), then cell, then mu."""
    d = min_image_length(kmesh)
    cells_sorted = sorted(range(len(d)), key=lambda c: (round(float(d[c]), 12), c))
    return [c * nao + m for c in cells_sorted for m in range(nao)]


def batched_fragments(nfrag=64, seed=1004, neo_range=(20, 200), lattices=("b222", "b333")):
    """Fragment specs: list of dicts (lattice name, neo, imp_idx, val_idx)."""
    rng = np.random.default_rng([seed, 7])
    out = []
    for f in range(nfrag):
        neo = int(rng.integers(neo_range[0], neo_range[1] + 1))
        lat = lattices[int(rng.integers(0, len(lattices)))]
        wl = BATCH_LATTICES.get(lat)
        nimp = (neo + 1) // 2
        nval = neo - nimp
        order = supercell_order(wl.kmesh, wl.nao) if wl is not None else None
        out.append({"lattice": lat, "neo": neo, "nimp": nimp, "nval": nval,
                    "imp_idx": None if order is None else order[:nimp], "val_idx": list(range(nval))})
    return out


# --------------------------------------------------------------------------
# Plane-wave (FFTDF) workloads: Gaussian AOs sampled on a real-space grid of a
# cell (orthorhombic, or any lattice given by its three vectors).  The "fitting
# functions" are the grid points r of the reference cell; the 3-index input is
# the AO pair density
#   rho[q][k][r][mu][nu] = sum_{R1,R2} e^{-i k.R1} e^{+i (k-q).R2} chi_mu(r - R1) chi_nu(r - R2)
#                        = A_mu(k, r) conj(A_nu(k-q, r)),  A_mu(k, r) = sum_R e^{-i k.R} chi_mu(r - R),
# with chi_mu periodic on the Born-von Karman supercell (each displacement wrapped to the nearest image in supercell fractional coordinates).
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class FftGrid:
    n: tuple             # grid points per cell axis
    cell: tuple          # orthorhombic edge lengths, or the lattice vectors as rows (bohr)

    @property
    def nr(self) -> int:
        return int(np.prod(self.n))

    @property
    def lattice(self) -> np.ndarray:
        a = np.asarray(self.cell, float)
        return np.diag(a) if a.shape == (3,) else a.reshape(3, 3)

    @property
    def volume(self) -> float:
        return abs(float(np.linalg.det(self.lattice)))


# hexagonal reference cell (the shape of the paper's hBN layer cell): a_1 = (a, 0, 0),
# a_2 = (a/2, a sqrt(3)/2, 0), a_3 = (0, 0, c)
HEX_CELL = ((2.6, 0.0, 0.0), (1.3, 1.3 * 3 ** 0.5, 0.0), (0.0, 0.0, 3.2))


# (workload, grid): naux of the workload is the number of grid points
FFT_CONFIGS = {
    "fft_tiny": (Workload("fft_tiny", (2, 2, 1), 4, 216, 4, 4, 1, 1.5, 1010), FftGrid((6, 6, 6), (3.0, 3.0, 3.0))),
    "fft_odd": (Workload("fft_odd", (3, 2, 1), 5, 240, 5, 5, 1, 1.5, 1011), FftGrid((6, 5, 8), (3.0, 2.6, 3.4))),
    "fft_si": (Workload("fft_si", (2, 2, 2), 26, 4096, 26, 26, 1, 2.0, 1012), FftGrid((16, 16, 16), (5.1, 5.1, 5.1))),
    # odd N_d n_d on every axis: with a non-orthogonal cell the Nyquist plane of an even
    # axis has no -G partner of the same |q+G|^2
    "fft_hex": (Workload("fft_hex", (3, 3, 1), 5, 175, 5, 5, 1, 1.5, 1015), FftGrid((5, 5, 7), HEX_CELL)),
}


def _fft_gaussians(wl: Workload, grid: FftGrid):
    """Centres (fractional), exponents (bohr^-2) and norms of the cell's AOs."""
    rng = np.random.default_rng([wl.seed, 300])
    centres = rng.random((wl.nao, 3))
    alpha = rng.uniform(0.8, 2.0, wl.nao)
    norm = (2.0 * alpha / np.pi) ** 0.75
    return centres, alpha, norm


def _chi_on_points(wl: Workload, grid: FftGrid, pts_cart, shift_cells):
    """chi_mu(x - R) for cartesian points x [np][3] and cell shifts R [nR][3]
    (integer cell coordinates): [nR][nao][np], the image nearest in supercell fractional coordinates."""
    centres, alpha, norm = _fft_gaussians(wl, grid)
    a = grid.lattice
    a_sup = np.asarray(wl.kmesh, float)[:, None] * a
    inv_sup = np.linalg.inv(a_sup)
    out = np.empty((len(shift_cells), wl.nao, len(pts_cart)))
    for ir, rc in enumerate(shift_cells):
        for mu in range(wl.nao):
            c = (np.asarray(rc) + centres[mu]) @ a
            f = (pts_cart - c[None, :]) @ inv_sup      # supercell fractional displacement
            f -= np.round(f)                            # periodic image nearest in fractional terms
            d = f @ a_sup
            out[ir, mu] = norm[mu] * np.exp(-alpha[mu] * (d * d).sum(axis=1))
    return out


def _cell_grid(grid: FftGrid):
    idx = np.indices(grid.n).reshape(3, -1).T
    return (idx / np.asarray(grid.n, float)[None, :]) @ grid.lattice


def fftdf_pair_density(wl: Workload, grid: FftGrid, dtype=np.complex128) -> np.ndarray:
    """rho[q][k][r][mu][nu] = (r | mu k, nu k-q) on the reference-cell grid."""
    assert wl.naux == grid.nr
    nk = wl.nk
    chi = _chi_on_points(wl, grid, _cell_grid(grid), cells(wl.kmesh))   # [R][mu][r]
    a = np.fft.fftn(chi.reshape(*wl.kmesh, wl.nao, grid.nr), axes=(0, 1, 2)).reshape(nk, wl.nao, grid.nr)
    a = a.transpose(0, 2, 1)                                             # A[k][r][mu]
    kmq = kq_index(wl.kmesh)
    out = np.empty((nk, nk, grid.nr, wl.nao, wl.nao), dtype=dtype)
    for q in range(nk):
        for k in range(nk):
            out[q, k] = a[k][:, :, None] * a[kmq[q, k]].conj()[:, None, :]
    return out


def fftdf_ao_supercell(wl: Workload, grid: FftGrid) -> np.ndarray:
    """chi_mu(X - R') on the supercell grid X (row-major over (N_d n_d) per
    axis): [N_k R'][nao][N_k nr] real."""
    n = np.asarray(grid.n) * np.asarray(wl.kmesh)
    idx = np.indices(tuple(n)).reshape(3, -1).T
    pts = (idx / np.asarray(grid.n, float)[None, :]) @ grid.lattice
    return _chi_on_points(wl, grid, pts, cells(wl.kmesh))
