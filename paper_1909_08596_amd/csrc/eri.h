// Internal plan of the embedding-ERI transformation (Alg. 1).
#pragma once

#include <vector>

#include "common.h"

namespace dmet {

// One fitting momentum q that is transformed: either q = -q (self-conjugate,
// real embedded 3-index, one Z row per L) or the representative of the pair
// {q, -q} (two rows per L: real and imaginary part, weight sqrt(2)).
struct QBlock {
    int q;
    int self_conj;
    size_t zrow0;     // first Z row of this block
    double weight;    // 1/(N_k sqrt(N_k)) or sqrt(2)/(N_k sqrt(N_k))
};

struct EriPlan {
    Mesh mesh;
    int nao, naux, neo, nspin;
    int npair;
    int zrows;        // N_k * naux
    dmet_dtype dtype;
    dmet_precision prec;
    std::vector<QBlock> qblocks;
};

EriPlan make_eri_plan(const dmet_lattice* lat, int neo, dmet_precision prec, dmet_dtype dtype);

// k <-> q-k pairing of the k-sum of Alg. 1.  Time reversal of the real basis
// and the Hermiticity of the 3-index tensor give (L|mu (q-k), nu (-k)) =
// (L|nu k, mu (k-q)), so the k-sum term at q-k is the plain transpose (in the
// EO pair ij) of the term at k.  The sum runs over the kept k (k <= q-k as mesh
// indices): slots [0, npaired) hold the k < q-k in increasing order (their term
// enters as M + M^T), slots [npaired, npaired + nself) the k = q-k (M is
// symmetric and enters once).
__host__ __device__ inline void kpair_counts(const Mesh& m, int q, int& npaired, int& nself) {
    npaired = nself = 0;
    for (int k = 0; k < m.nk; ++k) {
        const int kp = mesh_sub(m, q, k);
        if (k < kp) ++npaired;
        else if (k == kp) ++nself;
    }
}

__host__ __device__ inline int kpair_slot_k(const Mesh& m, int q, int slot) {
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < m.nk; ++k) {
            const int kp = mesh_sub(m, q, k);
            if ((pass == 0 && k < kp) || (pass == 1 && k == kp)) {
                if (slot == 0) return k;
                --slot;
            }
        }
    return -1;
}

// Kept k of one q for the paired transform (slot order of kpair_slot_k),
// passed to kernels by value.
constexpr int KP_MAX = 256;
struct KSlots {
    int npaired, nself;
    short k[KP_MAX];
};

inline KSlots kpair_slots(const Mesh& m, int q) {
    KSlots ks;
    kpair_counts(m, q, ks.npaired, ks.nself);
    for (int sl = 0; sl < ks.npaired + ks.nself; ++sl) ks.k[sl] = (short)kpair_slot_k(m, q, sl);
    return ks;
}

// the (q, k) blocks of lmunu that the paired transform reads
__host__ __device__ inline bool kpair_needed(const Mesh& m, int q, int k) {
    return mesh_neg(m, q) >= q && k <= mesh_sub(m, q, k);
}

// df_out != NULL: write the FP64 DF factors Z [nspin][zrows][npair] there and
// skip the contraction (eri pointers unused).
size_t eri_f64_workspace(const EriPlan& p);
dmet_status eri_f64_prepare();
dmet_status eri_f32_prepare();
// split-bf16 pieces used by the plane-wave route
size_t lp_transform_workspace(const EriPlan& p);
dmet_status lp_transform(const EriPlan& p, const void* lmunu, const double* ck, float* z, void* ws, size_t ws_bytes,
                         hipStream_t st);
size_t lp_rows_contract_workspace(dmet_precision prec, int nspin, int npair, int krows);
dmet_status lp_rows_contract(dmet_precision prec, int nspin, int npair, int krows, const double* z, size_t zsp,
                             size_t ldz, double* eri_aa, double* eri_bb, double* eri_ab, void* ws, size_t ws_bytes,
                             hipStream_t st);
dmet_status eri_f64(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa, double* eri_bb,
                    double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st, double* df_out = nullptr);

size_t eri_lp_workspace(const EriPlan& p);
dmet_status eri_lp(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa, double* eri_bb,
                   double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st, double* df_out = nullptr);

// (ij|kl) = sum_rows z_s[row][ij] z_t[row][kl] in FP64 for z [nspin][krows_p][ldz]
// (ldz even, krows_p a multiple of 16 with zero rows past the data); `part`
// holds contract_f64_workspace() doubles for the split-K partials.
size_t contract_f64_workspace(int nspin, int npair, int krows_p);
dmet_status contract_f64(int nspin, int npair, int ldz, int krows_p, const double* z, double* eri_aa,
                         double* eri_bb, double* eri_ab, double* part, hipStream_t st);

size_t eri_f32_workspace(const EriPlan& p);
dmet_status eri_f32(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa, double* eri_bb,
                    double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st, double* df_out = nullptr);

size_t fftdf_workspace(const EriPlan& p);
dmet_status fftdf_eri(const EriPlan& p, const dmet_pw_grid* grid, const void* rho, const double* ck, double* eri_aa,
                      double* eri_bb, double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st);

size_t fock_dc_workspace(int nspin, int neo, int nrows);
dmet_status fock_dc(int nspin, int neo, int nrows, const double* z, const double* f_eo, const double* dm_eo,
                    double* f_tilde, void* ws, size_t ws_bytes, hipStream_t st);

size_t batch_workspace(int nfrag, const dmet_fragment* frags, dmet_precision prec);
dmet_status eri_batched(int nfrag, const dmet_fragment* frags, dmet_precision prec, unsigned flags, void* ws,
                        size_t ws_bytes, hipStream_t st);

// bath / one-body (bath.hip, onebody.hip)
size_t bath_workspace_bytes(const dmet_lattice* lat, int nimp, int nval);
// size of the file-scope device scratch of build_bath_noalloc (one per GPU)
constexpr size_t BATH_SCRATCH_MAX = (size_t)32 << 20;
dmet_status build_bath_noalloc(const dmet_lattice* lat, const double2* dm_k, int nimp, const int* imp_idx,
                               int nval, const int* val_idx, double sv_tol, const double2* c_ao_lo,
                               double2* c_k, double* sv, int* neo, double* max_imag, hipStream_t st);
dmet_status build_bath(const dmet_lattice* lat, const double2* dm_k, int nimp, const int* imp_idx,
                       int nval, const int* val_idx, double sv_tol, const double2* c_ao_lo,
                       double2* c_k, double* sv, int* neo, double* max_imag, void* ws, size_t ws_bytes,
                       hipStream_t st);
dmet_status transform_1e(const dmet_lattice* lat, int neo, const double2* ck, const double2* op,
                         double* out, double* max_imag, hipStream_t st);
dmet_status energy_1e(int nspin, int neo, const double* h, const double* g, double* e1, hipStream_t st);
dmet_status energy_mf(int nspin, int neo, const double* f_tilde, const double* f_eo, const double* dm_eo,
                      double* e, hipStream_t st);

}  // namespace dmet
