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
#include <algorithm>
#include <mutex>
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
// Both stages gather the next BK-deep slice of A and B into registers while
// the MFMAs run on the current one, then store it into the other half of a
// double-buffered LDS tile (one barrier per slice).  The gathers load from
// clamped, always valid addresses with no condition, so that no load is waited
// for before the MFMAs; the real embedding of the complex values and the zero
// padding are applied when the slice is stored.
template <int BM, int BN, int BK, class TIn>
__global__ void __launch_bounds__(256) k_xform1_f64(Mesh mesh, int q, int nao, int naux, int neo,
                                                    const TIn* __restrict__ lmunu,
                                                    const double* __restrict__ ck,
                                                    double* __restrict__ tout) {
    using T = F64Tile<BM, BN, BK>;
    constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
    static_assert(NA * 256 == BM * BK && NB * 256 == BK * BN, "slice per thread");
    __shared__ double As[2][BK * T::LDA];
    __shared__ double Bs[2][BK * T::LDB];
    const int k = blockIdx.z;
    const int kmq = mesh_sub(mesh, k, q);
    const int M = naux * nao, K = 2 * nao, N = 2 * neo;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const TIn* a_base = lmunu + ((size_t)q * mesh.nk + k) * (size_t)M * K;
    const double* c_base = ck + (size_t)kmq * nao * neo * 2;
    d4 acc[BM / 32][BN / 32];
    zero_acc<BM, BN>(acc);
    const int tid = threadIdx.x;
    const double2* c2 = reinterpret_cast<const double2*>(c_base);
    double ra[NA];
    double2 rb[NB];
    auto gather = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * 256, kk = e % BK, mm = e / BK;
            const int gm = min(m0 + mm, M - 1), gk = min(k0 + kk, K - 1);
            ra[u] = ld(a_base, (size_t)gm * K + gk);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + u * 256, nn = e % BN, kk = e / BN;
            const int nu = min(k0 + kk, K - 1) >> 1, j = min(n0 + nn, N - 1) >> 1;
            rb[u] = c2[(size_t)nu * neo + j];
        }
    };
    auto stash = [&](int k0, int b) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * 256, kk = e % BK, mm = e / BK;
            const bool ok = m0 + mm < M && k0 + kk < K;
            As[b][kk * T::LDA + mm] = ok ? ra[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + u * 256, nn = e % BN, kk = e / BN;
            const int gn = n0 + nn, gk = k0 + kk;
            const int cp = gk & 1, c = gn & 1;
            const double cr = rb[u].x, ci = rb[u].y;
            const double v = cp == 0 ? (c == 0 ? cr : ci) : (c == 0 ? -ci : cr);
            Bs[b][kk * T::LDB + nn] = (gn < N && gk < K) ? v : 0.0;
        }
    };
    const int nkt = (K + BK - 1) / BK;
    gather(0);
    stash(0, 0);
    __syncthreads();
    for (int it = 0; it < nkt; ++it) {
        if (it + 1 < nkt) gather((it + 1) * BK);
        f64_mma<BM, BN, BK>(As[it & 1], Bs[it & 1], acc);
        if (it + 1 < nkt) stash((it + 1) * BK, (it + 1) & 1);
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
    constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
    static_assert(NA * 256 == BM * BK && NB * 256 == BK * BN, "slice per thread");
    __shared__ double As[2][BK * T::LDA];
    __shared__ double Bs[2][BK * T::LDB];
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
    const double2* t2 = reinterpret_cast<const double2*>(tin);
    double ra[NA];
    double2 rb[NB];
    auto gather = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * 256, mm = e % BM, kk = e / BM;
            const int gm = min(m0 + mm, neo - 1), gk = min(k0 + kk, K - 1);
            ra[u] = ck[((size_t)(gk >> 1) * neo + gm) * 2 + (gk & 1)];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + u * 256, nn = e % BN, kk = e / BN;
            const int kmu = min(k0 + kk, K - 1) >> 1, j = min(n0 + nn, N2 - 1) >> 1;
            rb[u] = t2[((size_t)kmu * naux + L) * neo + j];
        }
    };
    auto stash = [&](int k0, int b) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * 256, mm = e % BM, kk = e / BM;
            As[b][kk * T::LDA + mm] = (m0 + mm < neo && k0 + kk < K) ? ra[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + u * 256, nn = e % BN, kk = e / BN;
            const int gn = n0 + nn, gk = k0 + kk;
            const int cp = gk & 1, c = gn & 1;
            const double tr = rb[u].x, ti = rb[u].y;
            const double v = cp == 0 ? (c == 0 ? tr : ti) : (c == 0 ? ti : -tr);
            Bs[b][kk * T::LDB + nn] = (gn < N2 && gk < K) ? v : 0.0;
        }
    };
    const int nkt = (K + BK - 1) / BK;
    gather(0);
    stash(0, 0);
    __syncthreads();
    for (int it = 0; it < nkt; ++it) {
        if (it + 1 < nkt) gather((it + 1) * BK);
        f64_mma<BM, BN, BK>(As[it & 1], Bs[it & 1], acc);
        if (it + 1 < nkt) stash((it + 1) * BK, (it + 1) & 1);
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
// Contraction with 128 x 128 output tiles (4 waves of 64 x 64, 16 FP64 MFMA
// tiles each) and a double ring of 16-row stages moved by direct
// global->LDS loads: one wave instruction moves one 1 KB row of a tile
// (64 lanes x 2 doubles).  LDS rows are padded to 144 doubles so that the four
// rows read by one MFMA fragment fall on different bank halves.  z rows hold
// ldz (even) doubles and krows_p (multiple of 16) rows, the rows past krows
// being zero.  Optional split of the row range (split-K) for few tiles: split
// s of nsplit sums rows [s kchunk, (s+1) kchunk) into part[s][tile][128][128],
// reduced afterwards in a fixed order.
#define F64_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))
constexpr int R_BM = 128, R_BK = 16, R_LD = 144, R_SB = 8, R_NXCD = 8;

__device__ inline long r_xcd(long b, long n) {
    const long per = (n + R_NXCD - 1) / R_NXCD;
    return (b % R_NXCD) * per + b / R_NXCD;
}

template <int MODE>
__device__ inline bool r_tile(long t, int ntile, int& mt, int& nt) {
    const long sb = t / (R_SB * R_SB);
    const int within = (int)(t % (R_SB * R_SB));
    const int nsb = (ntile + R_SB - 1) / R_SB;
    long I, J;
    if constexpr (MODE == 0) {
        I = (long)((sqrt(8.0 * (double)sb + 1.0) - 1.0) * 0.5);
        while (I * (I + 1) / 2 > sb) --I;
        while ((I + 1) * (I + 2) / 2 <= sb) ++I;
        J = sb - I * (I + 1) / 2;
    } else {
        I = sb / nsb;
        J = sb % nsb;
    }
    if (I >= nsb) return false;
    mt = (int)(I * R_SB + within / R_SB);
    nt = (int)(J * R_SB + within % R_SB);
    if (mt >= ntile || nt >= ntile) return false;
    if (MODE == 0 && nt > mt) return false;
    return true;
}

template <int MODE>
inline long r_tiles_per_split(int ntile) {
    const long nsb = (ntile + R_SB - 1) / R_SB;
    return (MODE == 0 ? nsb * (nsb + 1) / 2 : nsb * nsb) * R_SB * R_SB;
}

template <int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_contract_f64r(int npair, int ldz, int krows_p, const double* __restrict__ za, const double* __restrict__ zb,
                long per_split, int kchunk, long nblocks, double* __restrict__ out, double* __restrict__ part) {
    constexpr int SA = R_BK * R_LD, STG = 2 * SA;
    extern __shared__ __align__(16) double rring[];
    const long logical = r_xcd(blockIdx.x, nblocks);
    const long split = logical / per_split;
    int mt, nt;
    const int ntile = (npair + R_BM - 1) / R_BM;
    if (!r_tile<MODE>(logical % per_split, ntile, mt, nt)) return;
    const int k0 = (int)split * kchunk;
    if (k0 >= krows_p) return;
    const int nst = (min(krows_p, k0 + kchunk) - k0) / R_BK;
    const int m0 = mt * R_BM, n0 = nt * R_BM;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
    // chunk of this lane in a 128-wide row, clamped to the row (columns past
    // npair only feed outputs that are not stored)
    const int xa = min(m0 + 2 * lane, ldz - 2), xb = min(n0 + 2 * lane, ldz - 2);
    auto issue = [&](int st) {
        double* dst = rring + (size_t)(st & 1) * STG;
        const size_t row0 = (size_t)k0 + (size_t)st * R_BK;
#pragma unroll
        for (int r = wave; r < R_BK; r += 4) {
            __builtin_amdgcn_global_load_lds((const void*)(za + (row0 + r) * ldz + xa), F64_LDS_PTR(dst + r * R_LD),
                                             16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)(zb + (row0 + r) * ldz + xb),
                                             F64_LDS_PTR(dst + SA + r * R_LD), 16, 0, 0);
        }
    };
    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    issue(0);
    for (int st = 0; st < nst; ++st) {
        const double* cur = rring + (size_t)(st & 1) * STG;
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // own loads of stage st landed
        __builtin_amdgcn_s_barrier();         // everyone's landed; stage st-1 fully read
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) issue(st + 1);
#pragma unroll
        for (int kk = 0; kk < R_BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = cur[kr * R_LD + wm0 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = cur[SA + kr * R_LD + wn0 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // result layout of v_mfma_f64_16x16x4f64: register r of lane l holds D[4 r + l / 16][l % 16]
    if (part) {
        const long tix = MODE == 0 ? (long)mt * (mt + 1) / 2 + nt : (long)mt * ntile + nt;
        const long ntiles = MODE == 0 ? (long)ntile * (ntile + 1) / 2 : (long)ntile * ntile;
        double* o = part + ((size_t)split * ntiles + tix) * (R_BM * R_BM);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    o[(wm0 + i * 16 + 4 * r + (lane >> 4)) * R_BM + wn0 + j * 16 + (lane & 15)] = acc[i][j][r];
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int IJ = m0 + wm0 + i * 16 + 4 * r + (lane >> 4);
                const int KL = n0 + wn0 + j * 16 + (lane & 15);
                if (IJ >= npair || KL >= npair) continue;
                if constexpr (MODE == 0) {
                    if (KL <= IJ) out[(size_t)IJ * (IJ + 1) / 2 + KL] = acc[i][j][r];
                } else {
                    out[(size_t)IJ * npair + KL] = acc[i][j][r];
                }
            }
}

// out[IJ, KL] = sum_s part[s][tile(IJ, KL)][IJ % 128][KL % 128], s in order
template <int MODE>
__global__ void k_contract_f64_reduce(int npair, int nsplit, const double* __restrict__ part,
                                      double* __restrict__ out) {
    const int ntile = (npair + R_BM - 1) / R_BM;
    const long ntiles = MODE == 0 ? (long)ntile * (ntile + 1) / 2 : (long)ntile * ntile;
    const long n = MODE == 0 ? (long)npair * (npair + 1) / 2 : (long)npair * npair;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        long IJ, KL;
        if constexpr (MODE == 0) {
            IJ = (long)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
            while (IJ * (IJ + 1) / 2 > e) --IJ;
            while ((IJ + 1) * (IJ + 2) / 2 <= e) ++IJ;
            KL = e - IJ * (IJ + 1) / 2;
        } else {
            IJ = e / npair;
            KL = e % npair;
        }
        const long mt = IJ / R_BM, nt = KL / R_BM;
        const long tix = MODE == 0 ? mt * (mt + 1) / 2 + nt : mt * ntile + nt;
        const size_t off = (size_t)tix * (R_BM * R_BM) + (IJ % R_BM) * R_BM + (KL % R_BM);
        double v = 0.0;
        for (int s = 0; s < nsplit; ++s) v += part[(size_t)s * ntiles * (R_BM * R_BM) + off];
        out[e] = v;
    }
}

// ---------------------------------------------------------------- driver
// stage 1: 128 x 128 tiles; stage 2: 64 x 64 (its i >= j triangle of neo x neo pairs per L pads
// less, and the complex gather of T keeps registers high enough that larger tiles drop to one
// wave per SIMD)
constexpr int X1_BM = 128, X1_BN = 128, X1_BK = 8;
constexpr int X2_BM = 64, X2_BN = 64, X2_BK = 16;

// padded Z of the contraction: even row length, rows a multiple of 16
static inline int f64_ldz(int npair) { return (npair + 1) / 2 * 2; }
static inline int f64_krows_p(int krows) { return (krows + R_BK - 1) / R_BK * R_BK; }

// split of the row range for the tile counts of s8 and s4: at least about
// DMET_F64_SPLIT_WG workgroups (default 2048, four rounds of the two per CU;
// on 66 tiles over 65536 rows 512 / 1024 / 2048 / 4096 took 3.79 / 2.97 /
// 2.82 / 2.84 ms), at least 32 stages per split
static void f64_split(int npair, int krows_p, int mode, int& nsplit, int& kchunk) {
    const long ntile = (npair + R_BM - 1) / R_BM;
    const long tiles = mode == 0 ? ntile * (ntile + 1) / 2 : ntile * ntile;
    const int stages = krows_p / R_BK;
    const char* e = getenv("DMET_F64_SPLIT_WG");
    const long target = e ? std::max(1, atoi(e)) : 2048;
    long s = (target + tiles - 1) / tiles;
    s = std::min<long>(s, std::max(1, stages / 32));
    nsplit = (int)std::max<long>(1, s);
    kchunk = (stages + nsplit - 1) / nsplit * R_BK;
    nsplit = (krows_p + kchunk - 1) / kchunk;
}

size_t contract_f64_workspace(int nspin, int npair, int krows_p) {
    size_t mx = 0;
    const long ntile = (npair + R_BM - 1) / R_BM;
    for (int mode = 0; mode < (nspin == 2 ? 2 : 1); ++mode) {
        int ns, kc;
        f64_split(npair, krows_p, mode, ns, kc);
        if (ns > 1) {
            const long tiles = mode == 0 ? ntile * (ntile + 1) / 2 : ntile * ntile;
            mx = std::max(mx, (size_t)ns * tiles * R_BM * R_BM);
        }
    }
    return mx;
}

size_t eri_f64_workspace(const EriPlan& p) {
    Carve cv(nullptr, 0);
    cv.take<double>((size_t)p.mesh.nk * p.nao * p.naux * 2 * p.neo);                       // T
    cv.take<double>((size_t)p.nspin * f64_krows_p(p.zrows) * f64_ldz(p.npair));            // Z per spin
    cv.take<double>(contract_f64_workspace(p.nspin, p.npair, f64_krows_p(p.zrows)));      // split partials
    return cv.bytes();
}

dmet_status eri_f64(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa, double* eri_bb,
                    double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st, double* df_out) {
    Carve cv(ws, ws_bytes);
    const int krows_p = f64_krows_p(p.zrows);
    double* t = cv.take<double>((size_t)p.mesh.nk * p.nao * p.naux * 2 * p.neo);
    double* z = cv.take<double>((size_t)p.nspin * krows_p * f64_ldz(p.npair));
    double* part = cv.take<double>(contract_f64_workspace(p.nspin, p.npair, krows_p));
    if (cv.bytes() > ws_bytes) return fail(DMET_E_WORKSPACE, "transform_eri workspace too small");
    // DF output goes to the caller's [nspin][zrows][npair]; the contraction's
    // own Z is padded (even rows, zero rows up to a multiple of 16)
    const size_t ldz = df_out ? (size_t)p.npair : (size_t)f64_ldz(p.npair);
    const size_t zsp = df_out ? (size_t)p.zrows * ldz : (size_t)krows_p * ldz;
    if (df_out) {
        z = df_out;
    } else if (krows_p > p.zrows) {
        for (int s = 0; s < p.nspin; ++s)
            fill_zero(z + s * zsp + (size_t)p.zrows * ldz, (size_t)(krows_p - p.zrows) * ldz * sizeof(double), st);
    }
    const int M1 = p.naux * p.nao, N1 = 2 * p.neo;
    for (int s = 0; s < p.nspin; ++s) {
        const double* cks = ck + (size_t)s * p.mesh.nk * p.nao * p.neo * 2;
        double* zs = z + (size_t)s * zsp;
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
    return contract_f64(p.nspin, p.npair, (int)ldz, krows_p, z, eri_aa, eri_bb, eri_ab, part, st);
}

// Dynamic LDS limit of the FP64 contraction, set once per device (a host call,
// kept out of graph captures: the batched driver calls this before capturing).
dmet_status eri_f64_prepare() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    DMET_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= 0 && dev < 64 && done[dev]) return DMET_OK;
    const size_t lds = (size_t)2 * 2 * R_BK * R_LD * sizeof(double);
    DMET_HIP(hipFuncSetAttribute((const void*)k_contract_f64r<0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    DMET_HIP(hipFuncSetAttribute((const void*)k_contract_f64r<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    if (dev >= 0 && dev < 64) done[dev] = true;
    return DMET_OK;
}

dmet_status contract_f64(int nspin, int npair, int ldz, int krows_p, const double* z, double* eri_aa,
                         double* eri_bb, double* eri_ab, double* part, hipStream_t st) {
    {
        dmet_status sp = eri_f64_prepare();
        if (sp != DMET_OK) return sp;
    }
    const size_t zsp = (size_t)krows_p * ldz;
    const size_t lds = (size_t)2 * 2 * R_BK * R_LD * sizeof(double);
    const int ntile = (npair + R_BM - 1) / R_BM;
    for (int mode = 0; mode < 2; ++mode) {
        if (mode == 1 && !(nspin == 2 && eri_ab)) break;
        int ns, kc;
        f64_split(npair, krows_p, mode, ns, kc);
        const long per = mode == 0 ? r_tiles_per_split<0>(ntile) : r_tiles_per_split<1>(ntile);
        const long nb = (per * ns + R_NXCD - 1) / R_NXCD * R_NXCD;
        auto kern = mode == 0 ? k_contract_f64r<0> : k_contract_f64r<1>;
        for (int s = 0; s < (mode == 0 ? nspin : 1); ++s) {
            const double* za = z + (mode == 0 ? s * zsp : 0);
            const double* zb = z + (mode == 0 ? s * zsp : zsp);
            double* out = mode == 1 ? eri_ab : (s == 0 ? eri_aa : eri_bb);
            ProfScope ps(mode == 0 ? "contract_s8_f64" : "contract_s4_f64", st);
            kern<<<dim3((unsigned)nb), 256, lds, st>>>(npair, ldz, krows_p, za, zb, per, kc, nb, out,
                                                       ns > 1 ? part : nullptr);
            if (ns > 1) {
                const long n = mode == 0 ? (long)npair * (npair + 1) / 2 : (long)npair * npair;
                const unsigned nbr = (unsigned)std::min<long>((n + 255) / 256, 65536L);
                if (mode == 0)
                    k_contract_f64_reduce<0><<<nbr, 256, 0, st>>>(npair, ns, part, out);
                else
                    k_contract_f64_reduce<1><<<nbr, 256, 0, st>>>(npair, ns, part, out);
            }
            ps.stop();
            DMET_LAUNCH_CHECK(mode == 0 ? "contract_s8_f64" : "contract_s4_f64");
        }
    }
    return DMET_OK;
}

}  // namespace dmet
