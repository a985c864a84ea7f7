// extern "C" entry points of libdmet: argument validation, planning and
// dispatch.  Every compute step runs in the kernels of bath.hip, onebody.hip
// and eri_*.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "eri.h"

namespace dmet {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

dmet_status fail(dmet_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

dmet_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return DMET_E_HIP;
}

__global__ void k_fill_zero(unsigned int* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

void fill_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    const unsigned blocks = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    k_fill_zero<<<blocks ? blocks : 1, 256, 0, s>>>(static_cast<unsigned int*>(p), n);
}

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRecord {
    std::string name;
    hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;
}  // namespace

static bool g_prof_suspended = false;

bool prof_suspend(bool on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    const bool was = g_prof_suspended;
    g_prof_suspended = on;
    return was;
}

ProfScope::ProfScope(const char* name, hipStream_t s) : slot(-1), st(s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || g_prof_suspended) return;
    ProfRecord r;
    r.name = name;
    if (hipEventCreate(&r.start) != hipSuccess) return;
    if (hipEventCreate(&r.stop) != hipSuccess) {
        (void)hipEventDestroy(r.start);
        return;
    }
    (void)hipEventRecord(r.start, s);
    g_prof.push_back(r);
    slot = (int)g_prof.size() - 1;
}

void ProfScope::stop() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (slot >= 0 && slot < (int)g_prof.size()) (void)hipEventRecord(g_prof[slot].stop, st);
    slot = -1;
}

static void prof_clear() {
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof.clear();
}

static dmet_status check_lattice(const dmet_lattice* lat) {
    if (!lat) return fail(DMET_E_ARG, "lattice is NULL");
    for (int d = 0; d < 3; ++d)
        if (lat->kmesh[d] < 1 || lat->kmesh[d] > 64) return fail(DMET_E_ARG, "kmesh entries must be in [1, 64]");
    const long nk = (long)lat->kmesh[0] * lat->kmesh[1] * lat->kmesh[2];
    if (nk > 4096) return fail(DMET_E_ARG, "more than 4096 k-points");
    if (lat->nao < 1 || lat->nao > 4096) return fail(DMET_E_ARG, "nao must be in [1, 4096]");
    if (lat->nspin != 1 && lat->nspin != 2) return fail(DMET_E_ARG, "nspin must be 1 or 2");
    return DMET_OK;
}

EriPlan make_eri_plan(const dmet_lattice* lat, int neo, dmet_precision prec, dmet_dtype dtype) {
    EriPlan p;
    p.mesh = make_mesh(lat->kmesh);
    p.nao = lat->nao;
    p.naux = lat->naux;
    p.neo = neo;
    p.nspin = lat->nspin;
    p.npair = neo * (neo + 1) / 2;
    p.zrows = p.mesh.nk * lat->naux;
    p.dtype = dtype;
    p.prec = prec;
    const double nk = (double)p.mesh.nk;
    size_t row = 0;
    for (int q = 0; q < p.mesh.nk; ++q) {
        const int nq = mesh_neg(p.mesh, q);
        if (nq < q) continue;
        QBlock b;
        b.q = q;
        b.self_conj = nq == q;
        b.zrow0 = row;
        b.weight = (b.self_conj ? 1.0 : sqrt(2.0)) / (nk * sqrt(nk));
        row += (size_t)(b.self_conj ? 1 : 2) * lat->naux;
        p.qblocks.push_back(b);
    }
    return p;
}

static dmet_status check_eri_args(const dmet_lattice* lat, int neo, dmet_precision prec, dmet_dtype dtype) {
    dmet_status s = check_lattice(lat);
    if (s != DMET_OK) return s;
    if (lat->naux < 1) return fail(DMET_E_ARG, "naux must be positive");
    if (neo < 1 || neo > 2048) return fail(DMET_E_ARG, "neo must be in [1, 2048]");
    if (prec != DMET_FP64 && prec != DMET_FP32_3M && prec != DMET_BF16X3_3M && prec != DMET_BF16X6_3M &&
        prec != DMET_BF16X6_I8)
        return fail(DMET_E_ARG, "unknown precision");
    if (dtype != DMET_C128 && dtype != DMET_C64) return fail(DMET_E_ARG, "unknown dtype");
    const double zbytes = (double)lat->kmesh[0] * lat->kmesh[1] * lat->kmesh[2] * lat->naux *
                          (double)neo * (neo + 1) / 2 * 8.0;
    if (zbytes > 1.0e12) return fail(DMET_E_ARG, "problem too large for one device");
    return DMET_OK;
}

// c_imp[s][k][mu][i] = c_k[s][k][mu][i] for i < nimp (the impurity columns)
__global__ void k_impurity_columns(size_t rows, int neo, int nimp, const double2* __restrict__ c_k,
                                   double2* __restrict__ c_imp) {
    const size_t n = rows * (size_t)nimp;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        c_imp[e] = c_k[(e / nimp) * neo + e % nimp];
}

}  // namespace dmet

using namespace dmet;

extern "C" {

const char* dmet_last_error(void) { return g_last_error.c_str(); }

int dmet_version(void) { return 300; }   // 0.3.0: dmet_build_bath reports max |Im gamma^{R,0}|

dmet_status dmet_build_bath_workspace(const dmet_lattice* lat, int nimp, int nval, size_t* bytes) {
    dmet_status s = check_lattice(lat);
    if (s != DMET_OK) return s;
    if (!bytes) return fail(DMET_E_ARG, "bytes is NULL");
    if (nimp < 1 || nval < 1 || nval > nimp) return fail(DMET_E_ARG, "need 1 <= nval <= nimp");
    *bytes = bath_workspace_bytes(lat, nimp, nval);
    return DMET_OK;
}

static dmet_status check_bath_args(const dmet_lattice* lat, const void* dm_k, int nimp, const int* imp_idx,
                                   int nval, const int* val_idx, double sv_tol, const void* c_k, const double* sv,
                                   const int* neo) {
    dmet_status s = check_lattice(lat);
    if (s != DMET_OK) return s;
    const int nsup = lat->kmesh[0] * lat->kmesh[1] * lat->kmesh[2] * lat->nao;
    if (!dm_k || !c_k || !sv || !neo) return fail(DMET_E_ARG, "null array argument");
    if (nimp < 1 || nimp > nsup) return fail(DMET_E_ARG, "nimp must be in [1, N_k*nao]");
    if (!imp_idx && nimp != lat->nao) return fail(DMET_E_ARG, "imp_idx == NULL requires nimp == nao");
    if (nval < 1 || nval > nimp) return fail(DMET_E_ARG, "nval must be in [1, nimp]");
    if (!val_idx && nval != nimp) return fail(DMET_E_ARG, "val_idx == NULL requires nval == nimp");
    if (!(sv_tol >= 0.0)) return fail(DMET_E_ARG, "sv_tol must be >= 0");
    if (nval > 1024) return fail(DMET_E_UNSUPPORTED, "more than 1024 SVD columns");
    return DMET_OK;
}

dmet_status dmet_build_bath_noalloc(const dmet_lattice* lat, const void* dm_k, int nimp, const int* imp_idx,
                                    int nval, const int* val_idx, double sv_tol, const void* c_ao_lo, void* c_k,
                                    double* sv, int* neo, double* max_imag, hipStream_t stream) {
    g_last_error.clear();
    dmet_status s = check_bath_args(lat, dm_k, nimp, imp_idx, nval, val_idx, sv_tol, c_k, sv, neo);
    if (s != DMET_OK) return s;
    return build_bath_noalloc(lat, static_cast<const double2*>(dm_k), nimp, imp_idx, nval, val_idx, sv_tol,
                              static_cast<const double2*>(c_ao_lo), static_cast<double2*>(c_k), sv, neo, max_imag,
                              stream);
}

dmet_status dmet_build_bath(const dmet_lattice* lat, const void* dm_k, int nimp, const int* imp_idx, int nval,
                            const int* val_idx, double sv_tol, const void* c_ao_lo, void* c_k, double* sv,
                            int* neo, double* max_imag, void* workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    dmet_status s = check_lattice(lat);
    if (s != DMET_OK) return s;
    s = check_bath_args(lat, dm_k, nimp, imp_idx, nval, val_idx, sv_tol, c_k, sv, neo);
    if (s != DMET_OK) return s;
    if (!workspace) return fail(DMET_E_WORKSPACE, "workspace is NULL");
    return build_bath(lat, static_cast<const double2*>(dm_k), nimp, imp_idx, nval, val_idx, sv_tol,
                      static_cast<const double2*>(c_ao_lo), static_cast<double2*>(c_k), sv, neo, max_imag,
                      workspace, ws_bytes, stream);
}

dmet_status dmet_transform_1e(const dmet_lattice* lat, int neo, const void* c_k, const void* op_k, double* op_eo,
                              double* max_imag, hipStream_t stream) {
    g_last_error.clear();
    dmet_status s = check_lattice(lat);
    if (s != DMET_OK) return s;
    if (neo < 1 || neo > 4096) return fail(DMET_E_ARG, "neo must be in [1, 4096]");
    if (!c_k || !op_k || !op_eo) return fail(DMET_E_ARG, "null array argument");
    return transform_1e(lat, neo, static_cast<const double2*>(c_k), static_cast<const double2*>(op_k), op_eo,
                        max_imag, stream);
}

dmet_status dmet_energy_1e(int nspin, int neo, const double* h_eo, const double* dm_eo, double* e1,
                           hipStream_t stream) {
    g_last_error.clear();
    if (nspin != 1 && nspin != 2) return fail(DMET_E_ARG, "nspin must be 1 or 2");
    if (neo < 1) return fail(DMET_E_ARG, "neo must be positive");
    if (!h_eo || !dm_eo || !e1) return fail(DMET_E_ARG, "null array argument");
    return energy_1e(nspin, neo, h_eo, dm_eo, e1, stream);
}

// FP64 and FP32-3M have kernels of their own; the split-BF16 forms share one
dmet_status dmet_energy_mf(int nspin, int neo, const double* f_tilde, const double* f_eo, const double* dm_eo,
                           double* e, hipStream_t stream) {
    g_last_error.clear();
    if (nspin != 1 && nspin != 2) return fail(DMET_E_ARG, "nspin must be 1 or 2");
    if (neo < 1) return fail(DMET_E_ARG, "neo must be positive");
    if (!f_tilde || !f_eo || !dm_eo || !e) return fail(DMET_E_ARG, "null array argument");
    return energy_mf(nspin, neo, f_tilde, f_eo, dm_eo, e, stream);
}

static size_t eri_workspace(const EriPlan& p) {
    if (p.prec == DMET_FP64) return eri_f64_workspace(p);
    if (p.prec == DMET_FP32_3M) return eri_f32_workspace(p);
    return eri_lp_workspace(p);
}

dmet_status dmet_transform_eri_workspace(const dmet_lattice* lat, int neo, dmet_precision prec, dmet_dtype dtype,
                                         size_t* bytes) {
    dmet_status s = check_eri_args(lat, neo, prec, dtype);
    if (s != DMET_OK) return s;
    if (!bytes) return fail(DMET_E_ARG, "bytes is NULL");
    EriPlan p = make_eri_plan(lat, neo, prec, dtype);
    *bytes = eri_workspace(p);
    return DMET_OK;
}

dmet_status dmet_transform_eri(const dmet_lattice* lat, int neo, const void* lmunu, dmet_dtype dtype,
                               const void* c_k, dmet_precision prec, double* eri_aa, double* eri_bb,
                               double* eri_ab, void* workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    dmet_status s = check_eri_args(lat, neo, prec, dtype);
    if (s != DMET_OK) return s;
    if (!lmunu || !c_k || !eri_aa) return fail(DMET_E_ARG, "null array argument");
    if (lat->nspin == 2 && !eri_bb) return fail(DMET_E_ARG, "nspin == 2 requires eri_bb");
    if (lat->nspin == 1 && (eri_bb || eri_ab)) return fail(DMET_E_ARG, "nspin == 1 takes no eri_bb / eri_ab");
    if (!workspace) return fail(DMET_E_WORKSPACE, "workspace is NULL");
    EriPlan p = make_eri_plan(lat, neo, prec, dtype);
    if (prec == DMET_FP64)
        return eri_f64(p, lmunu, static_cast<const double*>(c_k), eri_aa, eri_bb, eri_ab, workspace, ws_bytes,
                       stream);
    if (prec == DMET_FP32_3M)
        return eri_f32(p, lmunu, static_cast<const double*>(c_k), eri_aa, eri_bb, eri_ab, workspace, ws_bytes,
                       stream);
    return eri_lp(p, lmunu, static_cast<const double*>(c_k), eri_aa, eri_bb, eri_ab, workspace, ws_bytes, stream);
}

dmet_status dmet_transform_eri_impurity_workspace(const dmet_lattice* lat, int neo, int nimp, dmet_precision prec,
                                                  dmet_dtype dtype, size_t* bytes) {
    dmet_status s = check_eri_args(lat, nimp, prec, dtype);
    if (s != DMET_OK) return s;
    if (nimp > neo) return fail(DMET_E_ARG, "need 1 <= nimp <= neo");
    if (!bytes) return fail(DMET_E_ARG, "bytes is NULL");
    EriPlan p = make_eri_plan(lat, nimp, prec, dtype);
    Carve cv(nullptr, 0);
    cv.take<char>(eri_workspace(p));
    cv.take<double2>((size_t)lat->nspin * p.mesh.nk * lat->nao * nimp);
    *bytes = cv.bytes();
    return DMET_OK;
}

dmet_status dmet_transform_eri_impurity(const dmet_lattice* lat, int neo, int nimp, const void* lmunu,
                                        dmet_dtype dtype, const void* c_k, dmet_precision prec, double* eri_aa,
                                        double* eri_bb, double* eri_ab, void* workspace, size_t ws_bytes,
                                        hipStream_t stream) {
    g_last_error.clear();
    size_t need = 0;
    dmet_status s = dmet_transform_eri_impurity_workspace(lat, neo, nimp, prec, dtype, &need);
    if (s != DMET_OK) return s;
    if (!lmunu || !c_k || !eri_aa) return fail(DMET_E_ARG, "null array argument");
    if (lat->nspin == 2 && !eri_bb) return fail(DMET_E_ARG, "nspin == 2 requires eri_bb");
    if (lat->nspin == 1 && (eri_bb || eri_ab)) return fail(DMET_E_ARG, "nspin == 1 takes no eri_bb / eri_ab");
    if (!workspace || ws_bytes < need) return fail(DMET_E_WORKSPACE, "transform_eri_impurity workspace too small");
    EriPlan p = make_eri_plan(lat, nimp, prec, dtype);
    Carve cv(workspace, ws_bytes);
    const size_t ews = eri_workspace(p);
    void* eri_ws = cv.take<char>(ews);
    const size_t rows = (size_t)lat->nspin * p.mesh.nk * lat->nao;
    double2* c_imp = cv.take<double2>(rows * nimp);
    k_impurity_columns<<<1024, 256, 0, stream>>>(rows, neo, nimp, static_cast<const double2*>(c_k), c_imp);
    DMET_LAUNCH_CHECK("k_impurity_columns");
    const double* ci = reinterpret_cast<const double*>(c_imp);
    if (prec == DMET_FP64) return eri_f64(p, lmunu, ci, eri_aa, eri_bb, eri_ab, eri_ws, ews, stream);
    if (prec == DMET_FP32_3M) return eri_f32(p, lmunu, ci, eri_aa, eri_bb, eri_ab, eri_ws, ews, stream);
    return eri_lp(p, lmunu, ci, eri_aa, eri_bb, eri_ab, eri_ws, ews, stream);
}

dmet_status dmet_transform_eri_df(const dmet_lattice* lat, int neo, const void* lmunu, dmet_dtype dtype,
                                  const void* c_k, dmet_precision prec, double* z, void* workspace, size_t ws_bytes,
                                  hipStream_t stream) {
    g_last_error.clear();
    dmet_status s = check_eri_args(lat, neo, prec, dtype);
    if (s != DMET_OK) return s;
    if (!lmunu || !c_k || !z) return fail(DMET_E_ARG, "null array argument");
    if (!workspace) return fail(DMET_E_WORKSPACE, "workspace is NULL");
    EriPlan p = make_eri_plan(lat, neo, prec, dtype);
    if (eri_workspace(p) > ws_bytes) return fail(DMET_E_WORKSPACE, "transform_eri workspace too small");
    if (prec == DMET_FP64)
        return eri_f64(p, lmunu, static_cast<const double*>(c_k), nullptr, nullptr, nullptr, workspace, ws_bytes,
                       stream, z);
    if (prec == DMET_FP32_3M)
        return eri_f32(p, lmunu, static_cast<const double*>(c_k), nullptr, nullptr, nullptr, workspace, ws_bytes,
                       stream, z);
    return eri_lp(p, lmunu, static_cast<const double*>(c_k), nullptr, nullptr, nullptr, workspace, ws_bytes, stream,
                  z);
}

static dmet_status check_pw(const dmet_lattice* lat, const dmet_pw_grid* grid) {
    if (!grid) return fail(DMET_E_ARG, "grid is NULL");
    long nr = 1;
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 1) return fail(DMET_E_ARG, "grid points per axis must be >= 1");
        nr *= grid->n[a];
    }
    if (nr != lat->naux) return fail(DMET_E_ARG, "naux must equal the number of grid points");
    // volume against the product of the vector lengths: a flat or degenerate cell is refused
    const double(*c)[3] = grid->cell;
    double len = 1.0;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            if (!std::isfinite(c[a][b])) return fail(DMET_E_ARG, "cell vectors must be finite");
        len *= sqrt(c[a][0] * c[a][0] + c[a][1] * c[a][1] + c[a][2] * c[a][2]);
    }
    const double det = c[0][0] * (c[1][1] * c[2][2] - c[1][2] * c[2][1]) -
                       c[0][1] * (c[1][0] * c[2][2] - c[1][2] * c[2][0]) +
                       c[0][2] * (c[1][0] * c[2][1] - c[1][1] * c[2][0]);
    if (!(len > 0.0) || !(fabs(det) > 1e-10 * len))
        return fail(DMET_E_ARG, "cell vectors must be linearly independent");
    return DMET_OK;
}

static dmet_status check_pw_prec(dmet_precision prec) {
    if (prec == DMET_FP64 || prec == DMET_BF16X6_3M || prec == DMET_BF16X3_3M) return DMET_OK;
    if (prec == DMET_FP32_3M || prec == DMET_BF16X6_I8)
        return fail(DMET_E_UNSUPPORTED, "fftdf: precision forms FP64, BF16X6_3M and BF16X3_3M");
    return fail(DMET_E_ARG, "unknown precision");
}

dmet_status dmet_transform_eri_fftdf_workspace(const dmet_lattice* lat, const dmet_pw_grid* grid, int neo,
                                               dmet_dtype dtype, dmet_precision prec, size_t* bytes) {
    dmet_status s = check_pw_prec(prec);
    if (s != DMET_OK) return s;
    s = check_eri_args(lat, neo, prec, dtype);
    if (s != DMET_OK) return s;
    s = check_pw(lat, grid);
    if (s != DMET_OK) return s;
    if (!bytes) return fail(DMET_E_ARG, "bytes is NULL");
    *bytes = fftdf_workspace(make_eri_plan(lat, neo, prec, dtype));
    return DMET_OK;
}

dmet_status dmet_transform_eri_fftdf(const dmet_lattice* lat, const dmet_pw_grid* grid, int neo, const void* rho,
                                     dmet_dtype dtype, dmet_precision prec, const void* c_k, double* eri_aa,
                                     double* eri_bb, double* eri_ab, void* workspace, size_t ws_bytes,
                                     hipStream_t stream) {
    g_last_error.clear();
    dmet_status s = check_pw_prec(prec);
    if (s != DMET_OK) return s;
    s = check_eri_args(lat, neo, prec, dtype);
    if (s != DMET_OK) return s;
    s = check_pw(lat, grid);
    if (s != DMET_OK) return s;
    if (!rho || !c_k || !eri_aa) return fail(DMET_E_ARG, "null array argument");
    if (lat->nspin == 2 && !eri_bb) return fail(DMET_E_ARG, "nspin == 2 requires eri_bb");
    if (lat->nspin == 1 && (eri_bb || eri_ab)) return fail(DMET_E_ARG, "nspin == 1 takes no eri_bb / eri_ab");
    if (!workspace) return fail(DMET_E_WORKSPACE, "workspace is NULL");
    EriPlan p = make_eri_plan(lat, neo, prec, dtype);
    if (fftdf_workspace(p) > ws_bytes) return fail(DMET_E_WORKSPACE, "fftdf workspace too small");
    return fftdf_eri(p, grid, rho, static_cast<const double*>(c_k), eri_aa, eri_bb, eri_ab, workspace, ws_bytes,
                     stream);
}

dmet_status dmet_fock_dc_workspace(int nspin, int neo, int nrows, size_t* bytes) {
    if (nspin != 1 && nspin != 2) return fail(DMET_E_ARG, "nspin must be 1 or 2");
    if (neo < 1 || neo > 512) return fail(DMET_E_ARG, "neo must be in [1, 512]");
    if (nrows < 1) return fail(DMET_E_ARG, "nrows must be positive");
    if (!bytes) return fail(DMET_E_ARG, "bytes is NULL");
    *bytes = fock_dc_workspace(nspin, neo, nrows);
    return DMET_OK;
}

dmet_status dmet_fock_dc(int nspin, int neo, int nrows, const double* z, const double* f_eo, const double* dm_eo,
                         double* f_tilde, void* workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    size_t need = 0;
    dmet_status s = dmet_fock_dc_workspace(nspin, neo, nrows, &need);
    if (s != DMET_OK) return s;
    if (!z || !f_eo || !dm_eo || !f_tilde) return fail(DMET_E_ARG, "null array argument");
    if (!workspace || ws_bytes < need) return fail(DMET_E_WORKSPACE, "fock_dc workspace too small");
    return fock_dc(nspin, neo, nrows, z, f_eo, dm_eo, f_tilde, workspace, ws_bytes, stream);
}

static dmet_status check_batch(int nfrag, const dmet_fragment* frags, dmet_precision prec) {
    if (nfrag < 1 || nfrag > 65535 || !frags) return fail(DMET_E_ARG, "need 1 <= nfrag <= 65535 fragments");
    for (int f = 0; f < nfrag; ++f) {
        const dmet_fragment& d = frags[f];
        dmet_status s = check_eri_args(&d.lat, d.neo, prec, d.dtype);
        if (s != DMET_OK) return fail(s, "fragment " + std::to_string(f) + ": " + dmet_last_error());
        const long nk = (long)d.lat.kmesh[0] * d.lat.kmesh[1] * d.lat.kmesh[2];
        const bool slots = prec == DMET_BF16X3_3M || prec == DMET_BF16X6_3M || prec == DMET_BF16X6_I8 ||
                           prec == DMET_FP32_3M;
        if (slots && nk > KP_MAX)
            return fail(DMET_E_UNSUPPORTED, "fragment " + std::to_string(f) +
                                                ": the split-bf16 and FP32 transforms support at most 256 k-points");
        if (d.lat.nspin != 1) return fail(DMET_E_ARG, "fragment " + std::to_string(f) + ": nspin must be 1");
        if (prec == DMET_BF16X6_I8 && nk * (long)d.lat.naux > 44032)
            return fail(DMET_E_UNSUPPORTED, "fragment " + std::to_string(f) +
                                                ": the int8 contraction holds exact sums for at most 44032 rows");
        if (!d.lmunu || !d.c_k || !d.eri) return fail(DMET_E_ARG, "fragment " + std::to_string(f) + ": null pointer");
        for (int g = 0; g < f; ++g)
            if (frags[g].lmunu == d.lmunu &&
                (frags[g].dtype != d.dtype || frags[g].lat.nao != d.lat.nao || frags[g].lat.naux != d.lat.naux ||
                 frags[g].lat.kmesh[0] != d.lat.kmesh[0] || frags[g].lat.kmesh[1] != d.lat.kmesh[1] ||
                 frags[g].lat.kmesh[2] != d.lat.kmesh[2]))
                return fail(DMET_E_ARG, "fragments sharing lmunu must share the lattice and dtype");
    }
    return DMET_OK;
}

dmet_status dmet_transform_eri_batched_workspace(int nfrag, const dmet_fragment* frags, dmet_precision prec,
                                                 size_t* bytes) {
    dmet_status s = check_batch(nfrag, frags, prec);
    if (s != DMET_OK) return s;
    if (!bytes) return fail(DMET_E_ARG, "bytes is NULL");
    *bytes = batch_workspace(nfrag, frags, prec);
    return DMET_OK;
}

dmet_status dmet_transform_eri_batched(int nfrag, const dmet_fragment* frags, dmet_precision prec, unsigned flags,
                                       void* workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    dmet_status s = check_batch(nfrag, frags, prec);
    if (s != DMET_OK) return s;
    if (flags & ~(unsigned)(DMET_BATCH_GRAPH | DMET_BATCH_AUTOTUNE)) return fail(DMET_E_ARG, "unknown flag bits");
    if (!workspace) return fail(DMET_E_WORKSPACE, "workspace is NULL");
    if (batch_workspace(nfrag, frags, prec) > ws_bytes) return fail(DMET_E_WORKSPACE, "batched workspace too small");
    return eri_batched(nfrag, frags, prec, flags, workspace, ws_bytes, stream);
}

dmet_status dmet_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return DMET_OK;
}

dmet_status dmet_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear();
    return DMET_OK;
}

dmet_status dmet_profile_report(char* buf, size_t len) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!buf || len == 0) return fail(DMET_E_ARG, "empty report buffer");
    std::map<std::string, std::pair<int, double>> agg;
    std::vector<std::string> order;
    for (auto& r : g_prof) {
        hipError_t e = hipEventSynchronize(r.stop);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        if (!agg.count(r.name)) order.push_back(r.name);
        agg[r.name].first += 1;
        agg[r.name].second += ms;
    }
    std::string out;
    for (auto& n : order) {
        char line[512];
        snprintf(line, sizeof(line), "%s %d %.6f\n", n.c_str(), agg[n].first, agg[n].second);
        out += line;
    }
    size_t n = out.size() < len - 1 ? out.size() : len - 1;
    memcpy(buf, out.data(), n);
    buf[n] = 0;
    return DMET_OK;
}

}  // extern "C"
