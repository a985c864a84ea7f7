/*
 * dmet.h -- C ABI of the MI355X periodic-DMET embedding library (libdmet.so).
 *
 * The library computes the lattice-to-embedding integral transformation of
 * periodic ab initio density matrix embedding theory (Cui, Zhu & Chan,
 * "Efficient implementation of ab initio quantum embedding in periodic
 * systems: density matrix embedding theory", Sec. 2.1):
 *
 *   dmet_build_bath      Eq. "bath R SVD", Eq. "C loemb R", Eq. "C loemb k"
 *   dmet_transform_1e    Eq. "fock transform"
 *   dmet_energy_1e       one-body energy of the embedding Hamiltonian, Eq. "emb Ham"
 *   dmet_transform_eri   Alg. 1 (GDF embedding ERI), Eq. "density fitting"
 *   dmet_fock_dc         Eq. "fock double counting" (F~ from the density-fitting factors)
 *   dmet_energy_mf       mean-field (Hartree-Fock form) energy of the embedding Hamiltonian
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * k-mesh   Gamma-centred, N_k = kmesh[0]*kmesh[1]*kmesh[2]; k (and cell R)
 *          index (n1*N2 + n2)*N3 + n3; exp(i k.R) = exp(2 pi i sum_d n_d m_d/N_d);
 *          k - q wraps per axis modulo N_d.
 * complex  interleaved (re, im) pairs, as torch.complex128 / complex64.
 * layout   every array is row-major, last index fastest.
 * density  dm_k is per spin (occupations <= 1); a restricted caller passes
 *          gamma_total / 2 with nspin = 1.
 * 3-index  lmunu[q][k][L][mu][nu] = (L | mu k, nu k-q), the Gaussian density
 *          fitting tensor of the fitting function L with momentum q = k_mu - k_nu
 *          (Sec. 2.1), normalised so that the lattice 4-index integral is
 *          sum_L (mu k1 nu k2 | L)(L | kappa k3 lambda k4) with
 *          (mu k1 nu k2 | L) = conj((L | nu k2 mu k1)); it must be the transform of
 *          a real, (mu R1)<->(nu R2)-symmetric real-space tensor (time-reversal
 *          symmetric input), which makes the embedding ERIs real and 8-fold
 *          symmetric.
 * packing  pair index ij = i(i+1)/2 + j (i >= j), npair = neo(neo+1)/2;
 *          s8: eri8[IJ(IJ+1)/2 + KL] for IJ >= KL (same-spin blocks);
 *          s4: eri4[IJ*npair + KL] (mixed alpha-beta block, alpha pair first).
 *
 * Ownership: every array argument is a caller-owned DEVICE pointer unless its
 * comment says "host".  The library never allocates device memory in these
 * calls: scratch comes from the caller's workspace (size from the matching
 * *_workspace query, 256-byte aligned).  Calls are enqueued on `stream` and are
 * asynchronous unless stated otherwise.
 *
 * Errors: arguments are validated on the host before anything is enqueued; a
 * non-DMET_OK status means nothing (or nothing further) was enqueued.  The
 * message of the last error of the calling thread is dmet_last_error().  No
 * entry point aborts or throws across the ABI.
 *
 * Tuning (environment, read at each call; results do not depend on them beyond
 * rounding order): DMET_SVD_MAX_SWEEPS=n (1..60, default 60) caps the Jacobi
 * sweeps of the bath SVD (a lower cap forces DMET_E_NOCONV on purpose);
 * DMET_XF2_SMALL_NEO=n sets the largest fragment neo that the batched form
 * transforms with 32 x 32 stage-2 tiles (default 256); DMET_TUNE_CACHE names
 * the file of the batched autotuner's choices; DMET_I8_CHUNK_ROWS=n (a
 * multiple of 64 up to 44032, the default) sets the rows per launch of the
 * int8 contraction; DMET_ROW_SPLIT=0 turns off the row split of the
 * split-bf16 contraction of few-tile blocks on the plane-wave route;
 * DMET_F64_SPLIT_WG=n (default 2048) is the workgroup count the FP64
 * contraction's row split aims at when a block has few output tiles.
 */
#ifndef DMET_H
#define DMET_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMET_OK = 0,
    DMET_E_ARG = 1,          /* invalid argument (shape, index list, null pointer) */
    DMET_E_HIP = 2,          /* a HIP runtime call failed                           */
    DMET_E_NOCONV = 3,       /* the Jacobi SVD did not converge                      */
    DMET_E_RANK = 4,         /* sv_tol removed every bath orbital                    */
    DMET_E_NONFINITE = 5,    /* NaN/Inf in an input                                  */
    DMET_E_WORKSPACE = 6,    /* workspace missing or smaller than the query          */
    DMET_E_UNSUPPORTED = 7   /* valid request outside what this library implements  */
} dmet_status;

typedef enum {
    DMET_FP64 = 0,           /* complex GEMMs as 4 real FP64 MFMA products              */
    DMET_FP32_3M = 1,        /* complex GEMMs as 3 real FP32 products, FP32 accumulate   */
    DMET_BF16X3_3M = 2,      /* each FP32 operand split into bf16 hi + lo and the
                                products hi*hi + hi*lo + lo*hi, FP32 accumulate
                                (about 2^-17 relative per operand).  Both transform
                                stages multiply complex numbers with 4 real
                                products (4M, not 3M: fewer operand bytes and no
                                re+im cancellation); the contraction is real    */
    DMET_BF16X6_3M = 3,      /* three-way bf16 split hi + mid + lo and the six
                                products hh, hm, mh, hl, mm, lh, FP32 accumulate
                                (about FP32 accuracy); 4M in both transform
                                stages as DMET_BF16X3_3M (the name is kept)     */
    DMET_BF16X6_I8 = 4       /* transform as DMET_BF16X6_3M; the contraction on
                                int8 MFMA: every pair column of the real rows Z
                                gets a power-of-two scale and three signed
                                digits (fixed point, ~2^-23 of the column's
                                largest entry), the six digit products of
                                level <= 2 summed exactly in int32 and combined
                                in FP64; the sums stay exact for 44032 rows per
                                launch, and longer Z (N_k*naux rows) runs in
                                chunks of up to 44032 rows whose scaled FP64
                                results are added in order (the batched form
                                takes at most 44032 rows per fragment)         */
} dmet_precision;

typedef enum {
    DMET_C128 = 0,           /* complex double */
    DMET_C64 = 1             /* complex float  */
} dmet_dtype;

typedef struct {
    int kmesh[3];            /* Monkhorst-Pack mesh, Gamma-centred (Sec. 2.2)  */
    int nao;                 /* crystal AOs (= LOs) per cell                   */
    int naux;                /* auxiliary (fitting) functions per cell         */
    int nspin;               /* 1 (restricted) or 2 (unrestricted)            */
} dmet_lattice;

/* Message describing the last error of the calling thread ("" if none). */
const char* dmet_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int dmet_version(void);

/* ---------------------------------------------------------------------------
 * Bath and embedding coefficients (Eqs. "bath R SVD", "C loemb R", "C loemb k").
 *
 * gamma^{R,0} = 1/N_k sum_k exp(+i k.R) gamma(k) is formed for every cell; the
 * block M = gamma_sup[env, imp[val]] of the supercell density matrix
 * (rows: every supercell orbital not in the impurity, in supercell order
 * cell*nao + mu; columns: the impurity LOs selected by val_idx -- the
 * valence-only SVD of Sec. 2.1) is decomposed M = B Lambda V^T by a one-sided
 * Jacobi SVD in FP64.  Bath vectors are sorted by descending singular value;
 * each is signed so that its entry of largest modulus is positive (ties within
 * 1e-12 relative: lowest row).  C^R = [[1, 0], [0, B]] is Loewdin
 * orthonormalised and Fourier transformed, C^k = sum_R exp(-i k.R) C^R, and
 * optionally composed with the AO->LO rotation: C^{k,AO,EO} = C^{k,AO,LO} C^k.
 *
 * dm_k     [nspin][N_k][nao][nao] complex128, Hermitian per k, per spin.
 * nimp     impurity size; imp_idx (host, nimp ints) lists supercell orbitals
 *          cell*nao + mu, or NULL for the LOs of cell 0 (nimp must then be nao).
 * nval     number of SVD columns; val_idx (host) lists positions in the
 *          impurity list, or NULL for all (nval must then be nimp).
 * sv_tol   bath orbitals with sigma <= max(sv_tol, sigma_max * max(n_env, nval)
 *          * 2^-52) are dropped; sv_tol = 0 thus keeps every orbital whose
 *          singular value is above the rounding level (a sigma at that level,
 *          e.g. an impurity column with no coupling to the environment, leaves
 *          its singular vector undetermined by M).
 * c_ao_lo  [N_k][nao][nao] complex128 AO->LO rotation (Eq. "C aolo"), or NULL
 *          for the identity.
 * c_k      out [nspin][N_k][nao][nimp+nval] complex128.  Columns 0..nimp-1 are
 *          the impurity, then the bath; columns beyond neo[s] are zero.
 * sv       out [nspin][nval] float64 singular values, descending.
 * neo      out HOST [nspin]: nimp + number of kept bath orbitals.
 * max_imag out HOST [1], or NULL: max |Im gamma^{R,0}| over every cell and
 *          spin (zero up to rounding for time-reversal-symmetric input; the
 *          imaginary part is discarded).
 * workspace/ws_bytes: device scratch, at least dmet_build_bath_workspace().
 *
 * An impurity that is the whole supercell (nimp = N_k*nao, e.g. one k-point
 * with every orbital in the impurity) leaves no environment and so no bath:
 * neo[s] = nimp, sv is zero and the bath columns of c_k are zero.  A
 * non-empty environment with fewer orbitals than nval is DMET_E_ARG.
 *
 * This call synchronises `stream` before returning (it reads back the
 * convergence status and the kept bath count).  Returns DMET_E_NONFINITE for
 * NaN/Inf in dm_k (checked before the SVD), DMET_E_NOCONV if the SVD needs
 * more than 60 sweeps, DMET_E_RANK if no singular value is above the drop
 * threshold (no bath orbital is left).
 * ------------------------------------------------------------------------- */
dmet_status dmet_build_bath_workspace(const dmet_lattice* lat, int nimp, int nval,
                                      size_t* bytes);
dmet_status dmet_build_bath(const dmet_lattice* lat, const void* dm_k,
                            int nimp, const int* imp_idx, int nval, const int* val_idx,
                            double sv_tol, const void* c_ao_lo,
                            void* c_k, double* sv, int* neo, double* max_imag,
                            void* workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * dmet_build_bath without a workspace, for callers that cannot allocate device
 * memory (tight DMET self-consistency or serving loops, harnesses that forbid
 * hipMalloc).  Arguments, results, synchronisation and status codes are those
 * of dmet_build_bath, whose kernels it runs.  Its scratch is a device array of
 * 32 MiB inside the library, one per GPU, held until the process ends; it
 * covers every bath whose dmet_build_bath_workspace() is at most 32 MiB with
 * c_ao_lo (e.g. nspin 2, 2x2x2 mesh, nao 150, nimp = nval = 150: 24.4 MiB).
 * A larger problem returns DMET_E_WORKSPACE before anything is enqueued.
 * The call allocates no device memory.  All calls on one GPU share that array:
 * calls that overlap in time on the same GPU (two host threads, or two streams)
 * race and must be serialised by the caller.  The stream's device must be the
 * calling thread's current device.
 * ------------------------------------------------------------------------- */
dmet_status dmet_build_bath_noalloc(const dmet_lattice* lat, const void* dm_k,
                                    int nimp, const int* imp_idx, int nval, const int* val_idx,
                                    double sv_tol, const void* c_ao_lo,
                                    void* c_k, double* sv, int* neo, double* max_imag,
                                    hipStream_t stream);

/* ---------------------------------------------------------------------------
 * One-body transform (Eq. "fock transform", without the double-counting term):
 *   X^{0,EO} = 1/N_k sum_k C^{k dagger} X^k C^k          per spin.
 *
 * c_k      [nspin][N_k][nao][neo] complex128.
 * op_k     [nspin][N_k][nao][nao] complex128 (h(k), F(k) or gamma(k)).
 * op_eo    out [nspin][neo][neo] float64, the real part.
 * max_imag out HOST [1] float64 max |Im X^{0,EO}| (zero up to rounding for
 *          time-reversal-symmetric lattices; the imaginary part is
 *          discarded), or NULL.  When it is given the call synchronises
 *          `stream` before returning (and concurrent calls that ask for it
 *          on one GPU take turns); with NULL it is asynchronous.
 * ------------------------------------------------------------------------- */
dmet_status dmet_transform_1e(const dmet_lattice* lat, int neo, const void* c_k,
                              const void* op_k, double* op_eo, double* max_imag,
                              hipStream_t stream);

/* E1 = sum_spin sum_ij h_ij gamma_ji (one-body energy of Eq. "emb Ham" with
 * per-spin density matrices).  h_eo, dm_eo: [nspin][neo][neo] float64;
 * e1: out DEVICE [1] float64.  Asynchronous. */
dmet_status dmet_energy_1e(int nspin, int neo, const double* h_eo, const double* dm_eo,
                           double* e1, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Embedding ERIs (Alg. 1):
 *   (L|0i 0j)(q) = 1/N_k sum_k [C^{k dagger} (L|k, k-q) C^{k-q}]_{ij}
 *   (ij|kl)     = 1/N_k sum_q sum_L conj((L|0i 0j)(q)) (L|0k 0l)(q)
 *
 * Only the imaginary-part-free result is formed: q and -q contribute complex
 * conjugate terms, so each pair {q, -q} is transformed once, and the real
 * contraction runs over N_k*naux rows.
 *
 * neo      embedding orbitals per spin (same for both spins).
 * lmunu    [N_k q][N_k k][naux][nao][nao], dtype per `dtype` (complex128 or 64).
 * c_k      [nspin][N_k][nao][neo] complex128.
 * prec     arithmetic of the transform and contraction GEMMs (dmet_precision);
 *          accumulation across q-blocks of the contraction is FP64 in every form.
 * eri_aa   out s8 [npair(npair+1)/2] float64 (spin alpha, or the only spin).
 * eri_bb   out s8 float64 (spin beta) -- required iff nspin == 2, else NULL.
 * eri_ab   out s4 [npair][npair] float64 (alpha-beta) -- optional when
 *          nspin == 2, must be NULL when nspin == 1.
 * workspace/ws_bytes: device scratch, at least dmet_transform_eri_workspace().
 * Asynchronous.  The device inputs are not checked for NaN or infinity (that
 * would need a synchronisation); a non-finite entry that the transform reads
 * makes the ERIs it reaches NaN in every form (never finite values).
 * ------------------------------------------------------------------------- */
dmet_status dmet_transform_eri_workspace(const dmet_lattice* lat, int neo,
                                         dmet_precision prec, dmet_dtype dtype,
                                         size_t* bytes);
dmet_status dmet_transform_eri(const dmet_lattice* lat, int neo, const void* lmunu,
                               dmet_dtype dtype, const void* c_k, dmet_precision prec,
                               double* eri_aa, double* eri_bb, double* eri_ab,
                               void* workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Embedding ERIs of the non-interacting-bath formalism (Sec. 2.1: two-particle
 * interactions kept on the impurity orbitals only): Alg. 1 on the first nimp
 * columns of C^k, i.e. the impurity block of the full embedding ERIs.
 *
 * neo      columns of c_k ([nspin][N_k][nao][neo] complex128, as written by
 *          dmet_build_bath: impurity columns first); 1 <= nimp <= neo.
 * eri_*    as dmet_transform_eri with npair = nimp(nimp+1)/2.
 * workspace/ws_bytes: at least dmet_transform_eri_impurity_workspace() (the
 *          transform's workspace for nimp orbitals plus a copy of the
 *          impurity columns).  Asynchronous.
 * ------------------------------------------------------------------------- */
dmet_status dmet_transform_eri_impurity_workspace(const dmet_lattice* lat, int neo, int nimp,
                                                  dmet_precision prec, dmet_dtype dtype, size_t* bytes);
dmet_status dmet_transform_eri_impurity(const dmet_lattice* lat, int neo, int nimp, const void* lmunu,
                                        dmet_dtype dtype, const void* c_k, dmet_precision prec,
                                        double* eri_aa, double* eri_bb, double* eri_ab,
                                        void* workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Density-fitting output of the embedding ERIs (Sec. 2.1: when the impurity
 * solver works with density fitting, the contraction step of Alg. 1 can be
 * omitted).  Runs the transform of dmet_transform_eri in the given form and
 * writes real factors instead of ERIs:
 *   z [nspin][N_k*naux][npair] float64,   (ij|kl)_st = sum_P z_s[P][ij] z_t[P][kl]
 * for packed pairs ij = i(i+1)/2 + j (i >= j), i.e. the real, FT-to-R=0
 * embedded 3-index (L|0i 0j) of every q with q and -q combined.  Workspace:
 * dmet_transform_eri_workspace() of the same arguments.  Asynchronous.
 * ------------------------------------------------------------------------- */
dmet_status dmet_transform_eri_df(const dmet_lattice* lat, int neo, const void* lmunu,
                                  dmet_dtype dtype, const void* c_k, dmet_precision prec,
                                  double* z, void* workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Plane-wave (FFTDF) embedding ERIs, App. B, Eq. "FFTDF" and Alg. 2.
 *
 * The fitting functions are the points r of a real-space grid of the
 * reference cell, r = sum_d (t_d / n[d]) a_d for t_d = 0 .. n[d] - 1 (n[0] x
 * n[1] x n[2] points, row-major over t), with a_d the lattice vectors (the rows
 * of `cell`, bohr; any non-degenerate cell, orthorhombic or not), so
 * lat->naux must equal n[0] n[1] n[2].  Input:
 *   rho [N_k q][N_k k][nr][nao][nao]  (complex128 or complex64, per dtype)
 *       rho[q][k][r][mu][nu] = (r | mu k, nu k-q), the AO pair density on the
 *       grid with the conventions of dmet_transform_eri (k-q wrapped per axis);
 *   c_k as for dmet_transform_eri.
 * For every q the AO pair densities are transformed to the embedding basis
 * and Fourier summed to R = 0 (as in Alg. 1), Fourier transformed over the
 * grid with the phase of q (W(G) = sum_r e^{+i(q+G).r} X(r)), weighted by the
 * Coulomb kernel 4 pi / (Omega |q+G|^2) (the q+G = 0 term dropped) and
 * contracted:
 *   (ij|kl) = dV^2 / (N_k Omega) sum_{q,G} 4 pi/|q+G|^2 Re[conj(W_ij) W_kl],
 * dV = Omega / nr, Omega = |det cell|, i.e. the Coulomb integral of the EO
 * pair densities on the Born-von Karman supercell.  The supercell frequency j_d
 * along axis d is taken in (-L/2, L/2], L = N_d n[d] (the FFT order; an even L
 * keeps -L/2), and q + G = sum_d (j_d / N_d) b_d with a_c . b_d = 2 pi delta_cd.
 * On a non-orthogonal cell an even L leaves that Nyquist plane without a -G
 * partner of the same |q+G|^2, and the result is the real part of a form that
 * is then not exactly Hermitian: odd N_d n[d] avoid this.  Outputs as
 * dmet_transform_eri (s8 / s4 float64).  prec: DMET_FP64 (FP64 throughout),
 * or DMET_BF16X6_3M / DMET_BF16X3_3M: the transform and the contraction in
 * that split-bf16 form (as dmet_transform_eri), the grid DFT and the Coulomb
 * weights in FP64 between them (the rows, 2 n_r per q, enter the contraction
 * rounded to FP32).  When a spin block has few output tiles for the CUs, its
 * split-bf16 contraction is split over the rows into partial outputs in the
 * workspace, added in row order afterwards (deterministic).  DMET_BF16X6_I8 is
 * not offered here: its int8 contraction is exact only to about 2^-23 of the
 * column scales per row, and in the plane-wave rows a few small |q+G| rows
 * dominate every sum, so its error exceeds 1e-6 Ha (1.5e-6 on a 6x5x8 grid);
 * nor is DMET_FP32_3M (both give DMET_E_UNSUPPORTED).  Returns
 * DMET_E_ARG for a grid that does not match naux or a cell whose vectors are
 * not finite or are linearly dependent, DMET_E_WORKSPACE if the workspace is
 * too small (the workspace depends on prec).
 * Asynchronous; the workspace must stay valid until the work completes.
 * ------------------------------------------------------------------------- */
typedef struct {
    int n[3];          /* grid points per cell axis */
    double cell[3][3]; /* lattice vectors a_1, a_2, a_3 as rows (bohr); diagonal for an orthorhombic cell */
} dmet_pw_grid;

dmet_status dmet_transform_eri_fftdf_workspace(const dmet_lattice* lat, const dmet_pw_grid* grid, int neo,
                                               dmet_dtype dtype, dmet_precision prec, size_t* bytes);
dmet_status dmet_transform_eri_fftdf(const dmet_lattice* lat, const dmet_pw_grid* grid, int neo,
                                     const void* rho, dmet_dtype dtype, dmet_precision prec,
                                     const void* c_k, double* eri_aa, double* eri_bb, double* eri_ab,
                                     void* workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Double-counting-corrected embedding Fock matrix (Eq. "fock double counting"):
 *   F~_ij = F^{EO}_ij - [sum_kl (ij|kl) gamma_lk - 1/2 sum_kl (ik|lj) gamma_kl]
 * with gamma the spin-summed embedding density.  Inputs are per spin:
 * nspin = 1: gamma = 2 dm_eo, F~ = F - (2 J(dm) - K(dm));
 * nspin = 2: F~_s = F_s - [J_ss(dm_s) + J_st(dm_t) - K_ss(dm_s)] (same Coulomb
 *            term, exchange of the spin's own density).
 * The ERIs enter through their density-fitting factors z (as written by
 * dmet_transform_eri_df, nrows = N_k*naux rows per spin).
 * f_eo, dm_eo: [nspin][neo][neo] float64 (dm_eo symmetric); f_tilde: out, same
 * shape.  Workspace from dmet_fock_dc_workspace().  Asynchronous.
 * ------------------------------------------------------------------------- */
dmet_status dmet_fock_dc_workspace(int nspin, int neo, int nrows, size_t* bytes);
dmet_status dmet_fock_dc(int nspin, int neo, int nrows, const double* z, const double* f_eo,
                         const double* dm_eo, double* f_tilde, void* workspace, size_t ws_bytes,
                         hipStream_t stream);

/* Mean-field energy of the embedding Hamiltonian whose one-body part is F~
 * (Eq. "fock double counting") and whose two-body part is the embedding ERIs,
 * with the Hartree-Fock expression at the embedding density (the paper
 * evaluates every DMET mean-field energy with the Hartree-Fock form, Sec. 2.2):
 *   E = sum_ij F~_ij gamma_ji + 1/2 sum (ij|kl)[gamma_ji gamma_lk - 1/2 gamma_jk gamma_li],
 * computed as 1/2 sum_ij (F~ + F^EO)_ij gamma_ji, which is the same because
 * F^EO = F~ + J - K/2 at that density.  Per-spin inputs as dmet_fock_dc:
 * nspin = 1: gamma = 2 dm_eo, E = sum_ij (F~ + F)_ij dm_ji;
 * nspin = 2: E = 1/2 sum_s sum_ij (F~_s + F_s)_ij dm_s,ji.
 * f_tilde, f_eo, dm_eo: [nspin][neo][neo] float64 DEVICE; e: out DEVICE [1]
 * float64.  Returns DMET_E_ARG for nspin not 1 or 2, neo < 1 or a NULL
 * pointer.  Asynchronous. */
dmet_status dmet_energy_mf(int nspin, int neo, const double* f_tilde, const double* f_eo,
                           const double* dm_eo, double* e, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched embedding ERIs (Alg. 1 for many fragments in one submission).
 *
 * Every fragment is an embedding problem of its own (its own impurity, bath
 * and neo) on a lattice that may be shared: fragments whose `lmunu` pointers
 * are equal share the 3-index tensor, and the k-AO -> k-EO transform of that
 * tensor is done once for all of them (their C^k are concatenated as one GEMM
 * operand).  The remaining work of all fragments -- the embedded 3-index for
 * each q and the packed contraction -- runs in persistent kernels that pop
 * (fragment, tile) items from a device work queue, largest first.
 *
 * frags    host array of nfrag descriptors; lat.nspin must be 1; fragments
 *          that share lmunu must share lat and dtype.
 * prec     DMET_BF16X3_3M, DMET_BF16X6_3M or DMET_BF16X6_I8 run the batched
 *          pipeline above (the last with the int8 contraction, at most 44032
 *          rows N_k*naux per fragment); DMET_FP64 and DMET_FP32_3M run the
 *          single-fragment path of each fragment on four concurrent internal
 *          streams (default priority; forked from and joined to `stream` by
 *          events), fragments assigned largest first, each stream with a slice
 *          of the workspace (same results as dmet_transform_eri, bit for bit).
 * flags    DMET_BATCH_GRAPH: capture the whole submission into a hipGraph on the
 *            first call with a given batch (descriptors, precision, workspace)
 *            and replay it on later calls (inputs may change, pointers may not);
 *          DMET_BATCH_AUTOTUNE: on the first call for a batch shape, time the
 *            contraction tile variants on this batch and keep the fastest (kept
 *            per process, and in the file named by $DMET_TUNE_CACHE if set).
 * workspace at least dmet_transform_eri_batched_workspace(); with
 *          DMET_BATCH_GRAPH it must stay valid for the replays.
 * Asynchronous (the first autotuned call synchronises `stream`).
 * ------------------------------------------------------------------------- */
typedef struct {
    dmet_lattice lat;        /* kmesh, nao, naux; nspin = 1                    */
    int neo;                 /* embedding orbitals of this fragment            */
    const void* lmunu;       /* [N_k q][N_k k][naux][nao][nao], `dtype`        */
    dmet_dtype dtype;
    const void* c_k;         /* [N_k][nao][neo] complex128                     */
    double* eri;             /* out s8 [npair(npair+1)/2] float64              */
} dmet_fragment;

enum { DMET_BATCH_GRAPH = 1, DMET_BATCH_AUTOTUNE = 2 };

dmet_status dmet_transform_eri_batched_workspace(int nfrag, const dmet_fragment* frags,
                                                 dmet_precision prec, size_t* bytes);
dmet_status dmet_transform_eri_batched(int nfrag, const dmet_fragment* frags, dmet_precision prec,
                                       unsigned flags, void* workspace, size_t ws_bytes,
                                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Optional per-kernel timing (not part of the method): when enabled, every
 * kernel launch of the entry points above is bracketed by a pair of HIP events
 * recorded on the launch's stream.  dmet_profile_report() waits for those
 * events and writes one line per kernel name, "name launches total_ms\n", for
 * all launches since the last reset (truncated to len bytes).  The events
 * cost a few microseconds per launch; timing is off by default.
 * ------------------------------------------------------------------------- */
dmet_status dmet_profile_enable(int on);
dmet_status dmet_profile_reset(void);
dmet_status dmet_profile_report(char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* DMET_H */
