"""FP64 CPU oracle of the periodic DMET lattice-to-embedding transformation.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP
library: it is a plain, slow, literal numpy transcription of the paper's
equations, in the paper's order and notation (Cui, Zhu & Chan, "Efficient
implementation of ab initio quantum embedding in periodic systems: density
matrix embedding theory", Sec. 2.1):

* Eq. ``bath R SVD``   : gamma^{R!=0,0} = B^{R!=0} Lambda V^{0 dagger}
* Eq. ``C loemb R``    : C^{R,LO,EO} = [[1, 0], [0, B^{R!=0}]]
* Eq. ``C loemb k``    : C^{k,LO,EO} = sum_R exp(-i k.R) C^{R,LO,EO};
                         C^{k,AO,EO} = C^{k,AO,LO} C^{k,LO,EO}
* Eq. ``fock transform``: F^{0,EO} = 1/N_k sum_k C^{k dagger} F^k C^k
* Eq. ``density fitting`` with the embedding orbitals substituted (what Alg. 1
  computes): the fitted 3-index of an EO pair in the reference cell,
  X_L(q)_ij = 1/N_k sum_k [C^{k dagger} (L|k, k-q) C^{k-q}]_ij, and the ERI
  (ij|kl) = 1/N_k sum_q sum_L conj(X_L(q)_ij) X_L(q)_kl.
* App. B, Eq. ``FFTDF`` (what Alg. 2 computes): the Coulomb energy of the EO
  pair densities, written as a sum over the plane waves q + G of the
  Born-von Karman supercell with the kernel 4 pi / |q + G|^2.

Readings of points the paper leaves open (k ordering, Fourier sign of gamma,
normalisation of the 3-index tensor, which index of (0i0j|L) is conjugated,
the bath sign gauge) are the ones listed in the design notes; they are the
unique choices for which Alg. 1 equals the real-space supercell transform of
``oracle.supercell``, which pins them.

Array conventions: complex arrays are numpy complex128, row-major; k and R
are flattened row-major over the mesh; lmunu[q][k][L][mu][nu] = (L|mu k, nu k-q).
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# k-mesh bookkeeping (Gamma-centred mesh, Sec. 2.2)
# --------------------------------------------------------------------------
def mesh_points(kmesh):
    """Integer coordinates (n1, n2, n3) of the mesh points, row-major."""
    pts = []
    for a in range(kmesh[0]):
        for b in range(kmesh[1]):
            for c in range(kmesh[2]):
                pts.append((a, b, c))
    return np.array(pts, dtype=np.int64)


def mesh_index(kmesh, n):
    """Row-major index of integer point n, wrapped per axis."""
    a, b, c = (int(n[0]) % kmesh[0], int(n[1]) % kmesh[1], int(n[2]) % kmesh[2])
    return (a * kmesh[1] + b) * kmesh[2] + c


def phase_matrix(kmesh):
    """P[k, R] = exp(i k.R) = exp(2 pi i sum_d n_d m_d / N_d)."""
    pts = mesh_points(kmesh)
    nk = len(pts)
    p = np.empty((nk, nk), dtype=np.complex128)
    for ik in range(nk):
        for ir in range(nk):
            x = sum(pts[ik][d] * pts[ir][d] / kmesh[d] for d in range(3))
            p[ik, ir] = np.exp(2j * np.pi * x)
    return p


# --------------------------------------------------------------------------
# Step a1: real-space density matrix gamma^{R,0} (Eq. bath R SVD, left side)
# --------------------------------------------------------------------------
def real_space_dm(dm_k, kmesh):
    """gamma^{R,0} = 1/N_k sum_k exp(+i k.R) gamma(k)   (per spin).

    dm_k: [nspin][N_k][nao][nao] complex.  Returns (real [nspin][N_k R][nao][nao],
    max |Im|).  The imaginary part vanishes for time-reversal-symmetric input.
    """
    nk = dm_k.shape[1]
    p = phase_matrix(kmesh)
    g = np.einsum("kR,skij->sRij", p, dm_k) / nk
    return g.real.copy(), float(np.abs(g.imag).max())


def supercell_block(dm_r, kmesh, nao, rows, cols):
    """gamma_sup[(R,mu),(R',nu)] = gamma^{R-R',0}_{mu nu} for the listed
    supercell orbitals (index = cell*nao + mu), by translation invariance."""
    pts = mesh_points(kmesh)
    out = np.empty((len(rows), len(cols)))
    for a, r in enumerate(rows):
        cr, mu = divmod(int(r), nao)
        for b, c in enumerate(cols):
            cc, nu = divmod(int(c), nao)
            d = mesh_index(kmesh, pts[cr] - pts[cc])
            out[a, b] = dm_r[d, mu, nu]
    return out


# --------------------------------------------------------------------------
# Step a2: bath orbitals from the SVD of the impurity-environment block
# --------------------------------------------------------------------------
def sign_fix(u):
    """Gauge of each singular vector: the entry of largest modulus is made
    positive (ties within 1e-12 of the maximum: lowest index wins)."""
    u = u.copy()
    for j in range(u.shape[1]):
        a = np.abs(u[:, j])
        m = a.max()
        i = int(np.nonzero(a >= m - 1e-12 * m)[0][0])
        if u[i, j] < 0:
            u[:, j] = -u[:, j]
    return u


def bath_orbitals(dm_r, kmesh, nao, imp_idx=None, val_idx=None, sv_tol=0.0):
    """Eq. ``bath R SVD`` for one spin.

    Rows of M are every supercell orbital outside the impurity, in supercell
    order (for a cell-0 impurity: R != 0, then mu); columns are the impurity
    valence LOs ``imp_idx[val_idx]`` (valence-only SVD, Sec. 2.1 "DMET bath and
    truncation").  Returns (env_rows, B [n_env][n_bath], sigma [n_val]).
    Singular values are sorted descending.  Bath orbitals with vanishing
    singular values carry no entanglement with the impurity and are dropped
    (Sec. 2.1, bath truncation): a vector is kept when sigma > max(sv_tol,
    sigma_max * max(n_env, n_val) * eps), the second term being the rounding
    level below which M does not determine the singular vector (the usual
    numerical-rank tolerance).  sv_tol = 0 thus keeps every determined vector.
    """
    nk = int(np.prod(kmesh))
    nsup = nk * nao
    imp = np.arange(nao) if imp_idx is None else np.asarray(imp_idx)
    val = np.arange(len(imp)) if val_idx is None else np.asarray(val_idx)
    imp_set = set(int(i) for i in imp)
    env = np.array([r for r in range(nsup) if r not in imp_set], dtype=np.int64)
    m = supercell_block(dm_r, kmesh, nao, env, imp[val])
    u, s, _vt = np.linalg.svd(m, full_matrices=False)
    order = np.argsort(-s, kind="stable")
    s = s[order]
    u = u[:, order]
    thr = max(float(sv_tol), float(s.max(initial=0.0)) * max(m.shape) * np.finfo(np.float64).eps)
    nb = int(np.count_nonzero(s > thr))
    b = sign_fix(u[:, :nb])
    return env, b, s


# --------------------------------------------------------------------------
# Step a3: embedding coefficients (Eqs. C loemb R, C loemb k)
# --------------------------------------------------------------------------
def emb_coeffs_real(env, b, kmesh, nao, imp_idx=None):
    """C^{R,LO,EO} [N_k R][nao][neo]: impurity columns are unit vectors on the
    impurity LOs (the identity block), bath columns carry B on the
    environment rows (Eq. ``C loemb R``)."""
    nk = int(np.prod(kmesh))
    imp = np.arange(nao) if imp_idx is None else np.asarray(imp_idx)
    nimp, nb = len(imp), b.shape[1]
    c = np.zeros((nk * nao, nimp + nb))
    for i, r in enumerate(imp):
        c[int(r), i] = 1.0
    c[env, nimp:] = b
    return c.reshape(nk, nao, nimp + nb)


def lowdin(c_r):
    """Loewdin orthonormalisation C <- C S^{-1/2}, S = sum_R C^{R T} C^R."""
    s = np.einsum("Rmi,Rmj->ij", c_r, c_r)
    w, v = np.linalg.eigh(s)
    return np.einsum("Rmi,ij->Rmj", c_r, (v / np.sqrt(w)) @ v.T)


def emb_coeffs_k(c_r, kmesh, c_ao_lo=None):
    """C^k = sum_R exp(-i k.R) C^R, then C^{k,AO,EO} = C^{k,AO,LO} C^{k,LO,EO}."""
    p = phase_matrix(kmesh)
    ck = np.einsum("kR,Rmi->kmi", p.conj(), c_r.astype(np.complex128))
    if c_ao_lo is not None:
        ck = np.einsum("kmn,kni->kmi", c_ao_lo, ck)
    return ck


def build_bath(dm_k, kmesh, nao, imp_idx=None, val_idx=None, sv_tol=0.0, c_ao_lo=None):
    """Steps a1-a3 for every spin.  Returns dict with c_k [nspin][N_k][nao][neo],
    c_r, sigma [nspin][n_val], dm_r, neo list and the max |Im gamma^{R,0}|."""
    dm_r, im = real_space_dm(dm_k, kmesh)
    out = {"c_k": [], "c_r": [], "sigma": [], "neo": [], "dm_r": dm_r, "max_imag_dm": im}
    for s in range(dm_k.shape[0]):
        env, b, sig = bath_orbitals(dm_r[s], kmesh, nao, imp_idx, val_idx, sv_tol)
        c_r = lowdin(emb_coeffs_real(env, b, kmesh, nao, imp_idx))
        out["c_r"].append(c_r)
        out["c_k"].append(emb_coeffs_k(c_r, kmesh, c_ao_lo))
        out["sigma"].append(sig)
        out["neo"].append(c_r.shape[2])
    if len(set(out["neo"])) == 1:
        out["c_k"] = np.array(out["c_k"])
        out["c_r"] = np.array(out["c_r"])
    out["sigma"] = np.array(out["sigma"])
    return out


# --------------------------------------------------------------------------
# Step a4: one-body transform (Eq. fock transform) and E1
# --------------------------------------------------------------------------
def transform_1e(c_k, op_k):
    """X^{0,EO} = 1/N_k sum_k C^{k dagger} X^k C^k, per spin.

    Returns (real [nspin][neo][neo], max |Im|)."""
    nk = c_k.shape[1]
    x = 0
    for k in range(nk):
        x = x + c_k[:, k].conj().transpose(0, 2, 1) @ op_k[:, k] @ c_k[:, k]
    x = x / nk
    return x.real.copy(), float(np.abs(x.imag).max())


def energy_1e(h_eo, dm_eo):
    """E1 = sum_spin sum_ij h_ij gamma_ji (per-spin density matrices)."""
    return float(np.einsum("sij,sji->", h_eo, dm_eo))


# --------------------------------------------------------------------------
# Steps a5-a7: Alg. 1, embedding ERIs from the k-point GDF 3-index tensor
# --------------------------------------------------------------------------
def alg1_embedded_3index(lmunu, c_k, kmesh, q):
    """The fitted 3-index of the embedding-orbital pairs for one fitting
    momentum q (Eq. ``density fitting`` in the EO basis, as used by Alg. 1):

        X_L(q)_ij = 1/N_k sum_k sum_{mu nu} conj(C^k_{mu i}) (L|mu k, nu k-q) C^{k-q}_{nu j}

    The pair (i, j) lives in the reference cell, so every k contributes with
    weight 1/N_k.  Returns X [L][neo][neo] complex."""
    nk = lmunu.shape[0]
    pts = mesh_points(kmesh)
    x = 0
    for k in range(nk):
        kmq = mesh_index(kmesh, pts[k] - pts[q])
        x = x + (c_k[k].conj().T @ lmunu[q, k] @ c_k[kmq]) / nk
    return x


def alg1_eri(lmunu, c_k_a, kmesh, c_k_b=None):
    """Embedding ERI as Alg. 1 defines it:

        (ij|kl) = 1/N_k sum_q sum_L conj(X_L(q)_ij) X_L(q)_kl,

    the fitted Coulomb integral of the reference-cell EO pairs (the bra side
    of Eq. ``density fitting`` is the complex conjugate of the ket side).
    With a second spin's C^k the mixed (alpha alpha|beta beta) block is
    returned.  Returns (real [n][n][n][n], max |Im|)."""
    nk = lmunu.shape[0]
    n = c_k_a.shape[2]
    m = n if c_k_b is None else c_k_b.shape[2]
    eri = np.zeros((n * n, m * m), dtype=np.complex128)
    for q in range(nk):
        xa = alg1_embedded_3index(lmunu, c_k_a, kmesh, q)
        xb = xa if c_k_b is None else alg1_embedded_3index(lmunu, c_k_b, kmesh, q)
        naux = xa.shape[0]
        eri += (xa.reshape(naux, n * n).conj().T @ xb.reshape(naux, m * m)) / nk
    eri = eri.reshape(n, n, m, m)
    return eri.real.copy(), float(np.abs(eri.imag).max())


def alg1_embedded_all(lmunu, c_k, kmesh):
    """X_L(q) of ``alg1_embedded_3index`` for every q (a list over q)."""
    return [alg1_embedded_3index(lmunu, c_k, kmesh, q) for q in range(lmunu.shape[0])]


def alg1_eri_block(xa, rows, cols, xb=None):
    """Entries of the Alg. 1 contraction for listed output pairs only:
    E[p, r] = (i_p j_p | k_r l_r) = 1/N_k sum_q sum_L conj(X_L(q)_{i_p j_p}) X_L(q)_{k_r l_r},
    from the embedded 3-index tensors of every q (``alg1_embedded_all``; xb
    those of the second spin for the mixed block).  Returns (real [len(rows)]
    [len(cols)], max |Im|).  The same sum as ``alg1_eri``, restricted to the
    requested entries so that it runs where the full tensor does not fit."""
    xb = xa if xb is None else xb
    nk = len(xa)
    ra = (np.array([p[0] for p in rows]), np.array([p[1] for p in rows]))
    cb = (np.array([p[0] for p in cols]), np.array([p[1] for p in cols]))
    out = np.zeros((len(rows), len(cols)), dtype=np.complex128)
    for q in range(nk):
        out += xa[q][:, ra[0], ra[1]].conj().T @ xb[q][:, cb[0], cb[1]] / nk
    return out.real.copy(), float(np.abs(out.imag).max(initial=0.0))


def alg1_eri_diag(xa, pairs):
    """The diagonal (ij|ij) of the Alg. 1 contraction for the listed pairs:
    1/N_k sum_q sum_L |X_L(q)_ij|^2 (real by construction)."""
    nk = len(xa)
    i, j = np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])
    out = np.zeros(len(pairs))
    for q in range(nk):
        out += (np.abs(xa[q][:, i, j]) ** 2).sum(axis=0) / nk
    return out


def alg1_eri_columns(lmunu, c_k_a, kmesh, pairs_a, c_k_b=None, pairs_b=None):
    """The same contraction restricted to listed pairs: returns
    E[p, r] = (i_p j_p | k_r l_r) for p in pairs_a, r in pairs_b.

    Needed at sizes where the full 4-index tensor does not fit; the embedded
    3-index is only formed for the pair columns that are asked for."""
    nk = lmunu.shape[0]
    pts = mesh_points(kmesh)
    c_k_b = c_k_a if c_k_b is None else c_k_b
    pairs_b = pairs_a if pairs_b is None else pairs_b
    ia, ja = np.array([p[0] for p in pairs_a]), np.array([p[1] for p in pairs_a])
    ib, jb = np.array([p[0] for p in pairs_b]), np.array([p[1] for p in pairs_b])
    out = 0
    for q in range(nk):
        xa = 0
        xb = 0
        for k in range(nk):
            kmq = mesh_index(kmesh, pts[k] - pts[q])
            a = lmunu[q, k]
            ta = a @ c_k_a[kmq][:, ja]                                   # [L][m][p]
            xa = xa + (c_k_a[k][:, ia].conj()[None] * ta).sum(axis=1) / nk
            tb = a @ c_k_b[kmq][:, jb]
            xb = xb + (c_k_b[k][:, ib].conj()[None] * tb).sum(axis=1) / nk
        out = out + (xa.conj().T @ xb) / nk
    return out.real.copy(), float(np.abs(out.imag).max())


# --------------------------------------------------------------------------
# NEXT-4: Alg. 2, embedding ERIs with plane-wave density fitting (App. B)
# --------------------------------------------------------------------------
def fftdf_frequencies(kmesh, grid_n, q):
    """Integer supercell frequency j' (one axis per column) of every (q, G):
    j = N_d g_d + m_d with q = m and G = g on the cell grid, taken in
    (-(N_d n_d)/2, (N_d n_d)/2] the way a length-N_d n_d FFT orders them.
    Returns [nr][3] (G row-major over the cell grid)."""
    m = mesh_points(kmesh)[q]
    out = []
    for d in range(3):
        L = kmesh[d] * grid_n[d]
        j = kmesh[d] * np.arange(grid_n[d]) + m[d]
        out.append(np.where(j <= (L - 1) // 2, j, j - L))
    jx, jy, jz = np.meshgrid(out[0], out[1], out[2], indexing="ij")
    return np.stack([jx.ravel(), jy.ravel(), jz.ravel()], axis=1)


def cell_vectors(cell):
    """Lattice vectors of the reference cell as the rows a_1, a_2, a_3 (bohr);
    three numbers are the edge lengths of an orthorhombic cell."""
    a = np.asarray(cell, float)
    return np.diag(a) if a.shape == (3,) else a.reshape(3, 3)


def reciprocal_vectors(cell):
    """Rows b_1, b_2, b_3 of the reciprocal lattice, a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(cell_vectors(cell)).T


def coulomb_kernel(kmesh, grid_n, cell, q):
    """4 pi / |q + G|^2 on the cell grid of G; the q + G = 0 term is dropped
    (neutralising background).  A supercell frequency j (per axis, as
    fftdf_frequencies orders them) is the vector q + G = sum_d (j_d / N_d) b_d."""
    j = fftdf_frequencies(kmesh, grid_n, q).astype(float)
    kvec = (j / np.asarray(kmesh, float)[None, :]) @ reciprocal_vectors(cell)
    k2 = (kvec * kvec).sum(axis=1)
    out = np.zeros_like(k2)
    nz = k2 > 0
    out[nz] = 4.0 * np.pi / k2[nz]
    return out


def alg2_eri(rho, c_k_a, kmesh, grid_n, cell, c_k_b=None):
    """Plane-wave embedding ERI (App. B, Eq. ``FFTDF``; the quantity Alg. 2
    evaluates).  The EO pair density of the reference cell with momentum q,
    X_ij(q)[r] = 1/N_k sum_k [C^{k dagger} (r|k, k-q) C^{k-q}]_ij, has the
    plane-wave coefficients W_ij(q)[G] = sum_r exp(+i (q+G).r) X_ij(q)[r] on the
    cell grid; the ERI is the Coulomb energy of the pair densities on the
    Born-von Karman supercell,

        (ij|kl) = dV^2 / (N_k Omega) sum_q sum_G 4 pi/|q+G|^2 conj(W_ij(q)[G]) W_kl(q)[G],

    dV = Omega / n_r, with the q + G = 0 term left out (neutralising
    background).  rho[q][k][r][mu][nu] = (r|mu k, nu k-q).
    Returns (real [n][n][m][m], max |Im|)."""
    nk = rho.shape[0]
    grid_n = tuple(grid_n)
    nr = int(np.prod(grid_n))
    omega = abs(float(np.linalg.det(cell_vectors(cell))))
    dv = omega / nr
    idx = np.indices(grid_n).reshape(3, -1).T
    eri = 0
    for q in range(nk):
        m = mesh_points(kmesh)[q]
        ph = np.exp(2j * np.pi * (idx * (m / (np.asarray(kmesh) * np.asarray(grid_n)))[None, :]).sum(axis=1))
        kern = coulomb_kernel(kmesh, grid_n, cell, q)
        w = []
        for c in ((c_k_a,) if c_k_b is None else (c_k_a, c_k_b)):
            x = alg1_embedded_3index(rho, c, kmesh, q)                     # [r][i][j]
            n = x.shape[1]
            # sum_r exp(+i G.r) f(r) over the cell grid is n_r times numpy's inverse DFT
            wq = np.fft.ifftn((ph[:, None, None] * x).reshape(*grid_n, n, n), axes=(0, 1, 2)) * nr
            w.append(wq.reshape(nr, n * n))
        wa, wb = w[0], w[-1]
        eri = eri + dv * dv / (nk * omega) * ((wa.conj() * kern[:, None]).T @ wb)
    n = c_k_a.shape[2]
    m = n if c_k_b is None else c_k_b.shape[2]
    eri = eri.reshape(n, n, m, m)
    return eri.real.copy(), float(np.abs(eri.imag).max())


# --------------------------------------------------------------------------
# Output packing (8-fold / 4-fold symmetric storage)
# --------------------------------------------------------------------------
def pair_index(i, j):
    """Packed pair index of (i, j), i >= j: i(i+1)/2 + j."""
    if i < j:
        i, j = j, i
    return i * (i + 1) // 2 + j


def pack_s8(eri):
    """Packed lower triangle over pairs: eri8[IJ(IJ+1)/2 + KL], IJ >= KL."""
    n = eri.shape[0]
    npair = n * (n + 1) // 2
    tri = np.tril_indices(n)
    mat = eri[tri[0], tri[1]][:, tri[0], tri[1]]          # [npair][npair]
    assert mat.shape == (npair, npair)
    r, c = np.tril_indices(npair)
    return mat[r, c].copy()


def pack_s4(eri):
    """[ij][kl] over pairs i >= j, k >= l (mixed-spin block)."""
    n = eri.shape[0]
    tri = np.tril_indices(n)
    return eri[tri[0], tri[1]][:, tri[0], tri[1]].copy()


def unpack_s8(eri8, n):
    """Full [n][n][n][n] tensor from the packed s8 vector."""
    npair = n * (n + 1) // 2
    mat = np.zeros((npair, npair))
    r, c = np.tril_indices(npair)
    mat[r, c] = eri8
    mat[c, r] = eri8
    tri = np.tril_indices(n)
    pidx = np.zeros((n, n), dtype=np.int64)
    pidx[tri[0], tri[1]] = np.arange(npair)
    pidx[tri[1], tri[0]] = np.arange(npair)
    return mat[pidx][:, :, pidx]


# --------------------------------------------------------------------------
# Double counting (Eq. fock double counting): F~ = F^EO - [J(gamma) - 1/2 K(gamma)]
# --------------------------------------------------------------------------
def fock_double_counting(f_eo, dm_eo, eri):
    """Eq. ``fock double counting`` written out with a spin-summed density.

    Restricted (nspin = 1): gamma = 2 * dm_eo[0] (dm_eo is per spin), eri the
    [n][n][n][n] ERI tensor:
        F~_ij = F_ij - [sum_kl (ij|kl) gamma_lk - 1/2 sum_kl (ik|lj) gamma_kl].
    Unrestricted (nspin = 2, eri = (aa, bb, ab) tensors): the same Coulomb
    term with the total density and the exchange term of the spin's own
    density (per-spin density, so no factor 1/2):
        F~_s = F_s - [J_ss(g_s) + J_st(g_t) - K_ss(g_s)].
    """
    f_eo = np.asarray(f_eo)
    if f_eo.shape[0] == 1:
        g = 2.0 * dm_eo[0]
        j = np.einsum("ijkl,lk->ij", eri, g)
        k = np.einsum("ikl j,kl->ij".replace(" ", ""), eri, g)
        return (f_eo[0] - (j - 0.5 * k))[None]
    aa, bb, ab = eri
    ga, gb = dm_eo[0], dm_eo[1]
    ja = np.einsum("ijkl,lk->ij", aa, ga) + np.einsum("ijkl,lk->ij", ab, gb)
    jb = np.einsum("ijkl,lk->ij", bb, gb) + np.einsum("klij,lk->ij", ab, ga)
    ka = np.einsum("iklj,kl->ij", aa, ga)
    kb = np.einsum("iklj,kl->ij", bb, gb)
    return np.stack([f_eo[0] - (ja - ka), f_eo[1] - (jb - kb)])


def energy_mf(f_tilde, dm_eo, eri):
    """Mean-field energy of the embedding Hamiltonian (one-body part F~ of Eq.
    ``fock double counting``, two-body part the embedding ERIs), evaluated
    with the Hartree-Fock expression at the embedding density (Sec. 2.2: DMET
    energies use the Hartree-Fock form of the mean-field energy).

    Restricted: gamma = 2 dm_eo[0] (spin-summed),
        E = sum_ij F~_ij gamma_ji + 1/2 sum_ijkl (ij|kl) [gamma_ji gamma_lk - 1/2 gamma_jk gamma_li].
    Unrestricted (eri = (aa, bb, ab)), per-spin densities g_a, g_b:
        E = sum_s sum_ij F~_s,ij g_s,ji
          + 1/2 sum_{s,t} sum (ij|kl)_st g_s,ji g_t,lk - 1/2 sum_s sum (ij|kl)_ss g_s,jk g_s,li.
    """
    f_tilde = np.asarray(f_tilde)
    if f_tilde.shape[0] == 1:
        g = 2.0 * dm_eo[0]
        one = np.einsum("ij,ji->", f_tilde[0], g)
        coul = np.einsum("ijkl,ji,lk->", eri, g, g)
        exch = np.einsum("ijkl,jk,li->", eri, g, g)
        return float(one + 0.5 * coul - 0.25 * exch)
    aa, bb, ab = eri
    ga, gb = dm_eo[0], dm_eo[1]
    one = np.einsum("ij,ji->", f_tilde[0], ga) + np.einsum("ij,ji->", f_tilde[1], gb)
    coul = (np.einsum("ijkl,ji,lk->", aa, ga, ga) + np.einsum("ijkl,ji,lk->", bb, gb, gb)
            + 2.0 * np.einsum("ijkl,ji,lk->", ab, ga, gb))
    exch = np.einsum("ijkl,jk,li->", aa, ga, ga) + np.einsum("ijkl,jk,li->", bb, gb, gb)
    return float(one + 0.5 * coul - 0.5 * exch)
