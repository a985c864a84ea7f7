// Embedding ERIs by Alg. 1, FP64 form: every complex product is carried out as
// a real FP64 MFMA GEMM (v_mfma_f64_16x16x4f64) on the 2x2 real embedding of
// complex numbers (4 real products per complex MAC).
//
// For each q in {q : q <= -q} (q and -q give complex-conjugate terms):
//   stage 1 (batched over k):  T_k[(L,mu)][j]  = sum_nu (L|mu k, nu k-q) C^{k-q}_{nu j}
//   stage 2 (sum over k, mu):  X[i][(L,j)]     = sum_{k,mu} conj(C^k_{mu i}) T_k[(L,mu)][j]
//                              i.e. (L|0i 0j)(q) = X / N_k, kept for i >= j only
//   rows of Z:                 Z[(q,L,re/im)][ij] = w_q Re/Im X,
//                              w_q = 1/(N_k sqrt N_k) (q = -q) or sqrt(2)/(N_k sqrt N_k)
// then the contraction (ij|kl) = sum_rows Z[r][ij] Z[r][kl] as a packed SYRK
// (same spin) or GEMM (alpha-beta).
#include <vector>

#include "common.h"
#include "eri.h"
#include "mfma_f64.h"

namespace dmet {

template <class T>
__device__ inline double ld(const T* p, size_t i);
template <>
__device__ inline double ld<double>(const double* p, size_t i) { return p[i]; }
template <>
__device__ inline double ld<float>(const float* p, size_t i) { return (double)p[i]; }

// ---------------------------------------------------------------- stage 1
// A: lmunu[q][k] rows (L,mu), K = (nu, re/im) contiguous; B: real embedding
// of C^{k-q}: B[(nu,c')][(j,c)] = [[Cr, Ci], [-Ci, Cr]][c'][c].
// Output T[k][mu][L][(j,c)] (interleaved complex, row length 2 neo).
template <int BM, int BN, int BK, class TIn>
__global__ void __launch_bounds__(256) k_xform1_f64(Mesh mesh, int q, int nao, int naux, int neo,
                                                    const TIn* __restrict__ lmunu,
                                                    const double* __restrict__ ck,
                                                    double* __restrict__ tout) {
    using T = F64Tile<BM, BN, BK>;
    __shared__ double As[BK * T::LDA];
    __shared__ double Bs[BK * T::LDB];
    const int k = blockIdx.z;
    const int kmq = mesh_sub(mesh, k, q);
    const int M = naux * nao, K = 2 * nao, N = 2 * neo;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const TIn* a_base = lmunu + ((size_t)q * mesh.nk + k) * (size_t)M * K;
    const double* c_base = ck + (size_t)kmq * nao * neo * 2;
    d4 acc[BM / 32][BN / 32];
    zero_acc<BM, BN>(acc);
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < K; k0 += BK) {
        for (int e = tid; e < BM * BK; e += 256) {
            const int kk = e % BK, mm = e / BK;
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk * T::LDA + mm] = (gm < M && gk < K) ? ld(a_base, (size_t)gm * K + gk) : 0.0;
        }
        for (int e = tid; e < BK * BN; e += 256) {
            const int nn = e % BN, kk = e / BN;
            const int gn = n0 + nn, gk = k0 + kk;
            double v = 0.0;
            if (gn < N && gk < K) {
                const int nu = gk >> 1, cp = gk & 1, j = gn >> 1, c = gn & 1;
                const double cr = c_base[((size_t)nu * neo + j) * 2], ci = c_base[((size_t)nu * neo + j) * 2 + 1];
                v = cp == 0 ? (c == 0 ? cr : ci) : (c == 0 ? -ci : cr);
            }
            Bs[kk * T::LDB + nn] = v;
        }
        __syncthreads();
        f64_mma<BM, BN, BK>(As, Bs, acc);
        __syncthreads();
    }
    f64_visit<BM, BN, BK>(acc, [&](int r, int c, double v) {
        const int gm = m0 + r, gn = n0 + c;
        if (gm < M && gn < N) {
            const int L = gm / nao, mu = gm % nao;
            tout[(((size_t)k * nao + mu) * naux + L) * N + gn] = v;
        }
    });
}

// ---------------------------------------------------------------- stage 2
// A[(k,mu,c')][i] = (Cr, Ci)[c'] of C^k_{mu i}; B[(k,mu,c')][(j,c)] from T:
// row c'=0 is (Tr, Ti), row c'=1 is (Ti, -Tr).  Grid: (i tiles, L * j tiles).
// Writes Z rows for i >= j.
template <int BM, int BN, int BK>
__global__ void __launch_bounds__(256) k_xform2_f64(Mesh mesh, int nao, int naux, int neo, int self_conj,
                                                    size_t zrow0, double wq, const double* __restrict__ ck,
                                                    const double* __restrict__ tin, double* __restrict__ z,
                                                    size_t ldz) {
    using T = F64Tile<BM, BN, BK>;
    __shared__ double As[BK * T::LDA];
    __shared__ double Bs[BK * T::LDB];
    const int N2 = 2 * neo;
    const int njt = (N2 + BN - 1) / BN;
    const int L = blockIdx.y / njt, jt = blockIdx.y % njt;
    const int m0 = blockIdx.x * BM, n0 = jt * BN;     // n within this L: (j, c)
    const int j_first = n0 >> 1;
    if (m0 + BM - 1 < j_first) return;                  // tile entirely above the diagonal
    const int K = 2 * mesh.nk * nao;
    d4 acc[BM / 32][BN / 32];
    zero_acc<BM, BN>(acc);
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < K; k0 += BK) {
        for (int e = tid; e < BK * BM; e += 256) {
            const int mm = e % BM, kk = e / BM;
            const int gm = m0 + mm, gk = k0 + kk;
            double v = 0.0;
            if (gm < neo && gk < K) {
                const int kmu = gk >> 1, cp = gk & 1;
                v = ck[((size_t)kmu * neo + gm) * 2 + cp];
            }
            As[kk * T::LDA + mm] = v;
        }
        for (int e = tid; e < BK * BN; e += 256) {
            const int nn = e % BN, kk = e / BN;
            const int gn = n0 + nn, gk = k0 + kk;
            double v = 0.0;
            if (gn < N2 && gk < K) {
                const int kmu = gk >> 1, cp = gk & 1, j = gn >> 1, c = gn & 1;
                const double* row = tin + ((size_t)kmu * naux + L) * N2 + 2 * j;
                v = cp == 0 ? row[c] : (c == 0 ? row[1] : -row[0]);
            }
            Bs[kk * T::LDB + nn] = v;
        }
        __syncthreads();
        f64_mma<BM, BN, BK>(As, Bs, acc);
        __syncthreads();
    }
    f64_visit<BM, BN, BK>(acc, [&](int r, int c, double v) {
        const int i = m0 + r, gn = n0 + c;
        if (i >= neo || gn >= N2) return;
        const int j = gn >> 1, part = gn & 1;
        if (j > i) return;
        if (self_conj && part == 1) return;
        const size_t row = zrow0 + (self_conj ? (size_t)L : (size_t)2 * L + part);
        z[row * ldz + (size_t)i * (i + 1) / 2 + j] = wq * v;
    });
}

// ---------------------------------------------------------------- contraction
// out = Za^T Zb over rows, Za/Zb [K][ldz].  mode 0: packed s8 (IJ >= KL, lower
// triangle of tiles only, Za == Zb); mode 1: full s4 [IJ][KL].
template <int BM, int BN, int BK, int mode>
__global__ void __launch_bounds__(256) k_contract_f64(int npair, int krows, const double* __restrict__ za,
                                                      const double* __restrict__ zb, size_t ldz,
                                                      double* __restrict__ out) {
    using T = F64Tile<BM, BN, BK>;
    __shared__ double As[BK * T::LDA];
    __shared__ double Bs[BK * T::LDB];
    int mt, nt;
    if constexpr (mode == 0) {
        // linear block id -> (mt, nt) with mt >= nt
        const long b = blockIdx.x;
        mt = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((long)mt * (mt + 1) / 2 > b) --mt;
        while ((long)(mt + 1) * (mt + 2) / 2 <= b) ++mt;
        nt = (int)(b - (long)mt * (mt + 1) / 2);
    } else {
        mt = blockIdx.x;
        nt = blockIdx.y;
    }
    const int m0 = mt * BM, n0 = nt * BN;
    d4 acc[BM / 32][BN / 32];
    zero_acc<BM, BN>(acc);
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < krows; k0 += BK) {
        for (int e = tid; e < BK * BM; e += 256) {
            const int mm = e % BM, kk = e / BM;
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk * T::LDA + mm] = (gm < npair && gk < krows) ? za[(size_t)gk * ldz + gm] : 0.0;
        }
        for (int e = tid; e < BK * BN; e += 256) {
            const int nn = e % BN, kk = e / BN;
            const int gn = n0 + nn, gk = k0 + kk;
            Bs[kk * T::LDB + nn] = (gn < npair && gk < krows) ? zb[(size_t)gk * ldz + gn] : 0.0;
        }
        __syncthreads();
        f64_mma<BM, BN, BK>(As, Bs, acc);
        __syncthreads();
    }
    f64_visit<BM, BN, BK>(acc, [&](int r, int c, double v) {
        const int IJ = m0 + r, KL = n0 + c;
        if (IJ >= npair || KL >= npair) return;
        if (mode == 0) {
            if (KL <= IJ) out[(size_t)IJ * (IJ + 1) / 2 + KL] = v;
        } else {
            out[(size_t)IJ * npair + KL] = v;
        }
    });
}

// ---------------------------------------------------------------- driver
constexpr int X1_BM = 64, X1_BN = 64, X1_BK = 16;
constexpr int X2_BM = 64, X2_BN = 64, X2_BK = 16;
constexpr int C_BM = 64, C_BN = 64, C_BK = 16;

size_t eri_f64_workspace(const EriPlan& p) {
    Carve cv(nullptr, 0);
    cv.take<double>((size_t)p.mesh.nk * p.nao * p.naux * 2 * p.neo);     // T
    cv.take<double>((size_t)p.nspin * p.zrows * p.npair);                 // Z per spin
    return cv.bytes();
}

dmet_status eri_f64(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa, double* eri_bb,
                    double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st, double* df_out) {
    Carve cv(ws, ws_bytes);
    double* t = cv.take<double>((size_t)p.mesh.nk * p.nao * p.naux * 2 * p.neo);
    double* z = cv.take<double>((size_t)p.nspin * p.zrows * p.npair);
    if (df_out) z = df_out;
    if (cv.bytes() > ws_bytes) return fail(DMET_E_WORKSPACE, "transform_eri workspace too small");
    const size_t ldz = (size_t)p.npair;
    const int M1 = p.naux * p.nao, N1 = 2 * p.neo;
    for (int s = 0; s < p.nspin; ++s) {
        const double* cks = ck + (size_t)s * p.mesh.nk * p.nao * p.neo * 2;
        double* zs = z + (size_t)s * p.zrows * ldz;
        for (const QBlock& qb : p.qblocks) {
            dim3 g1((M1 + X1_BM - 1) / X1_BM, (N1 + X1_BN - 1) / X1_BN, p.mesh.nk);
            ProfScope ps1("xform1_f64", st);
            if (p.dtype == DMET_C128)
                k_xform1_f64<X1_BM, X1_BN, X1_BK, double><<<g1, 256, 0, st>>>(
                    p.mesh, qb.q, p.nao, p.naux, p.neo, static_cast<const double*>(lmunu), cks, t);
            else
                k_xform1_f64<X1_BM, X1_BN, X1_BK, float><<<g1, 256, 0, st>>>(
                    p.mesh, qb.q, p.nao, p.naux, p.neo, static_cast<const float*>(lmunu), cks, t);
            ps1.stop();
            DMET_LAUNCH_CHECK("k_xform1_f64");
            const int njt = (N1 + X2_BN - 1) / X2_BN;
            dim3 g2((p.neo + X2_BM - 1) / X2_BM, p.naux * njt);
            ProfScope ps2("xform2_f64", st);
            k_xform2_f64<X2_BM, X2_BN, X2_BK><<<g2, 256, 0, st>>>(p.mesh, p.nao, p.naux, p.neo, qb.self_conj,
                                                                  qb.zrow0, qb.weight, cks, t, zs, ldz);
            ps2.stop();
            DMET_LAUNCH_CHECK("k_xform2_f64");
        }
    }
    if (df_out) return DMET_OK;
    return contract_f64(p.nspin, p.npair, p.zrows, z, eri_aa, eri_bb, eri_ab, st);
}

dmet_status contract_f64(int nspin, int npair, int krows, const double* z, double* eri_aa, double* eri_bb,
                         double* eri_ab, hipStream_t st) {
    const size_t ldz = (size_t)npair;
    const int nt = (npair + C_BM - 1) / C_BM;
    for (int s = 0; s < nspin; ++s) {
        const double* zs = z + (size_t)s * krows * ldz;
        double* out = s == 0 ? eri_aa : eri_bb;
        ProfScope ps("contract_s8_f64", st);
        k_contract_f64<C_BM, C_BN, C_BK, 0><<<dim3((unsigned)((long)nt * (nt + 1) / 2)), 256, 0, st>>>(
            npair, krows, zs, zs, ldz, out);
        ps.stop();
        DMET_LAUNCH_CHECK("k_contract_f64 s8");
    }
    if (nspin == 2 && eri_ab) {
        ProfScope ps("contract_s4_f64", st);
        k_contract_f64<C_BM, C_BN, C_BK, 1><<<dim3(nt, nt), 256, 0, st>>>(npair, krows, z, z + (size_t)krows * ldz,
                                                                        ldz, eri_ab);
        ps.stop();
        DMET_LAUNCH_CHECK("k_contract_f64 s4");
    }
    return DMET_OK;
}

}  // namespace dmet
