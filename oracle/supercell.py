"""Brute-force real-space supercell transform: the independent check of the
k-space oracle.

TEST INFRASTRUCTURE ONLY (tests / smoke / CPU baseline).  Shares no code with
``oracle.kspace`` or with the HIP library.

On the Born-von Karman torus of N_k cells the lattice problem is a finite
molecule of N_k*nao real orbitals, and every quantity of Sec. 2.1 has a plain
real-space definition that needs no Fourier transform of the method's own:

* the mean-field density matrix gamma_sup, a real projector;
* the bath: SVD of the environment x impurity block of gamma_sup
  (Eq. ``bath R SVD`` read in the supercell);
* the embedding orbitals C_sup = [impurity unit vectors | bath] (Eq. ``C loemb R``);
* one-body matrices: C_sup^T X_sup C_sup (Eq. ``fock transform`` in real space);
* ERIs: with B_L(mu R1, nu R2) the density-fitted 3-index tensor of a fitting
  function in cell 0 (Eq. ``density fitting``), translation invariance gives
  (ij|kl) = sum_{L,R_L} Z_{(L,R_L),ij} Z_{(L,R_L),kl},
  Z_{(L,R_L),ij} = sum C_sup[(R1,mu),i] B_L(mu R1-R_L, nu R2-R_L) C_sup[(R2,nu),j].

Alg. 1 is exact on the torus (k-blocking loses nothing), so the k-space
oracle must reproduce these numbers to rounding.
"""
from __future__ import annotations

import numpy as np


def _cells(kmesh):
    n1, n2, n3 = kmesh
    return np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)])


def _index(kmesh, n):
    n = np.asarray(n) % np.asarray(kmesh)
    return (n[..., 0] * kmesh[1] + n[..., 1]) * kmesh[2] + n[..., 2]


def translation(kmesh, shift):
    """perm[R] = index of cell R + shift (on the torus)."""
    return _index(kmesh, _cells(kmesh) + np.asarray(shift))


def supercell_operator(t_r, kmesh):
    """X_sup[(R,mu),(R',nu)] = <mu R|X|nu R'> = t(R'-R)_{mu nu} (t real)."""
    nk, nao = t_r.shape[0], t_r.shape[1]
    c = _cells(kmesh)
    x = np.empty((nk, nao, nk, nao))
    for a in range(nk):
        for b in range(nk):
            x[a, :, b, :] = t_r[_index(kmesh, c[b] - c[a])]
    return x.reshape(nk * nao, nk * nao)


def bloch_unitary(kmesh, nao):
    """U[(R,mu),(k,nu)] = delta_{mu nu} exp(i k.R)/sqrt(N_k): the map from
    Bloch-block to cell-local orbitals used by the generator's h(k)."""
    c = _cells(kmesh)
    nk = len(c)
    ang = 2.0 * np.pi * (c[:, None, :] * c[None, :, :] / np.asarray(kmesh)).sum(-1)
    ph = np.exp(1j * ang) / np.sqrt(nk)                    # [R][k]
    u = np.zeros((nk, nao, nk, nao), dtype=np.complex128)
    for mu in range(nao):
        u[:, mu, :, mu] = ph
    return u.reshape(nk * nao, nk * nao)


def supercell_dm(dm_k, kmesh):
    """gamma_sup = U blockdiag(gamma(k)) U^dagger (real up to rounding)."""
    nk, nao = dm_k.shape[0], dm_k.shape[1]
    u = bloch_unitary(kmesh, nao)
    blk = np.zeros((nk * nao, nk * nao), dtype=np.complex128)
    for k in range(nk):
        blk[k * nao:(k + 1) * nao, k * nao:(k + 1) * nao] = dm_k[k]
    g = u @ blk @ u.conj().T
    return g.real.copy(), float(np.abs(g.imag).max())


def embedding_orbitals(gamma_sup, imp, val=None, nbath=None):
    """C_sup [N_k*nao][neo] from the SVD of gamma_sup[env, imp[val]].

    Bath columns are ordered by descending singular value, each with its
    largest-modulus entry positive (ties: lowest index)."""
    nsup = gamma_sup.shape[0]
    imp = np.asarray(imp)
    val = np.arange(len(imp)) if val is None else np.asarray(val)
    mask = np.ones(nsup, dtype=bool)
    mask[imp] = False
    env = np.nonzero(mask)[0]
    u, s, _ = np.linalg.svd(gamma_sup[np.ix_(env, imp[val])], full_matrices=False)
    nb = len(s) if nbath is None else nbath
    u = u[:, :nb].copy()
    for j in range(nb):
        a = np.abs(u[:, j])
        i = int(np.nonzero(a >= a.max() * (1 - 1e-12))[0][0])
        if u[i, j] < 0:
            u[:, j] *= -1
    c = np.zeros((nsup, len(imp) + nb))
    c[imp, np.arange(len(imp))] = 1.0
    c[env, len(imp):] = u
    return c, s


def one_body(c_sup, x_sup):
    return c_sup.T @ x_sup @ c_sup


def eri(b_real, c_sup_a, kmesh, c_sup_b=None):
    """(ij|kl) = sum_{L,R_L} Z^a_{(L,R_L),ij} Z^b_{(L,R_L),kl}, all real.

    b_real: [naux][N_k R1][nao][N_k R2][nao] with the fitting function in cell 0.
    Shifting the fitting function to R_L is a relabelling of cells, so
    Z_{(L,R_L)} = C_s^T B_L C_s with C_s[(R,mu)] = C_sup[(R+R_L, mu)]."""
    naux, nk, nao = b_real.shape[0], b_real.shape[1], b_real.shape[2]
    c_sup_b = c_sup_a if c_sup_b is None else c_sup_b
    na, nb = c_sup_a.shape[1], c_sup_b.shape[1]
    out = np.zeros((na * na, nb * nb))
    cells = _cells(kmesh)
    for rl in range(nk):
        perm = translation(kmesh, cells[rl])
        ca = c_sup_a.reshape(nk, nao, na)[perm].reshape(nk * nao, na)
        cb = c_sup_b.reshape(nk, nao, nb)[perm].reshape(nk * nao, nb)
        bl = b_real.reshape(naux, nk * nao, nk * nao)
        za = np.einsum("pi,Lpr,rj->Lij", ca, bl, ca, optimize=True).reshape(naux, na * na)
        zb = za if c_sup_b is c_sup_a else np.einsum(
            "pi,Lpr,rj->Lij", cb, bl, cb, optimize=True).reshape(naux, nb * nb)
        out += za.T @ zb
    return out.reshape(na, na, nb, nb)


def coulomb_exchange(b_real, kmesh, gamma_sup):
    """J[g] and K[g] of the lattice (density-fitted ERIs of Eq. ``density
    fitting`` in real space) for a real supercell density g:
        (pq|rs) = sum_{L,R_L} B_L(p - R_L, q - R_L) B_L(r - R_L, s - R_L)
        J_pq = sum_rs (pq|rs) g_sr,   K_pq = sum_rs (pr|sq) g_rs."""
    naux, nk, nao = b_real.shape[0], b_real.shape[1], b_real.shape[2]
    n = nk * nao
    cells = _cells(kmesh)
    bl = b_real.reshape(naux, nk, nao, nk, nao)
    j = np.zeros((n, n))
    k = np.zeros((n, n))
    for rl in range(nk):
        perm = translation(kmesh, cells[rl])      # cell R -> R + R_L
        inv = np.argsort(perm)                    # cell R -> R - R_L
        bs = bl[:, inv][:, :, :, inv].reshape(naux, n, n)   # B_L(p - R_L, q - R_L)
        j += np.einsum("Lpq,L->pq", bs, np.einsum("Lrs,sr->L", bs, gamma_sup))
        k += np.einsum("Lpr,rs,Lsq->pq", bs, gamma_sup, bs, optimize=True)
    return j, k


def fftdf_eri(chi_sup, c_sup_a, kmesh, grid_n, cell, c_sup_b=None):
    """Plane-wave embedding ERIs by brute force on the supercell grid: the EO
    orbitals phi_i(X) = sum_{R,mu} C_sup[(R,mu),i] chi_mu(X - R) are formed on
    the whole Born-von Karman grid, their pair densities are Fourier
    transformed with one supercell FFT, and

        (ij|kl) = dV^2 / Omega_sup sum_{Gs != 0} 4 pi/|Gs|^2 conj(P_ij(Gs)) P_kl(Gs),

    the Coulomb integral of the pair densities under the periodic Coulomb
    operator of the supercell.  chi_sup: [N_k R][nao][X]."""
    nk, nao, nx = chi_sup.shape
    shape = tuple(int(a) * int(b) for a, b in zip(kmesh, grid_n))
    assert nx == int(np.prod(shape))
    cell = np.asarray(cell, float)
    a_cell = np.diag(cell) if cell.shape == (3,) else cell.reshape(3, 3)   # rows: lattice vectors
    a_sup = np.asarray(kmesh, float)[:, None] * a_cell                      # supercell lattice vectors
    omega_sup = abs(float(np.linalg.det(a_sup)))
    dv = omega_sup / nx
    # plane waves of the supercell: G = sum_d f_d b_d, b_d the supercell's reciprocal vectors
    b_sup = 2.0 * np.pi * np.linalg.inv(a_sup).T
    freqs = np.stack(np.meshgrid(*[np.fft.fftfreq(shape[d], 1.0 / shape[d]) for d in range(3)], indexing="ij"),
                     axis=-1).reshape(-1, 3)
    gvec = freqs @ b_sup
    g2 = (gvec * gvec).sum(axis=1).reshape(shape)
    kern = np.zeros_like(g2)
    kern[g2 > 0] = 4.0 * np.pi / g2[g2 > 0]

    def pair_hat(c_sup):
        n = c_sup.shape[1]
        phi = np.einsum("rmx,rmi->ix", chi_sup, c_sup.reshape(nk, nao, n))
        pair = (phi[:, None, :] * phi[None, :, :]).reshape(n * n, *shape)
        return np.fft.fftn(pair, axes=(1, 2, 3)).reshape(n * n, -1), n

    pa, na = pair_hat(c_sup_a)
    pb, nb = (pa, na) if c_sup_b is None else pair_hat(c_sup_b)
    eri = (pa.conj() * kern.ravel()[None, :]) @ pb.T * (dv * dv / omega_sup)
    assert np.abs(eri.imag).max() <= 1e-10 * max(1.0, np.abs(eri.real).max())
    return eri.real.reshape(na, na, nb, nb)
