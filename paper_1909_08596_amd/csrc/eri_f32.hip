// FP32-3M form of the embedding-ERI transformation on packed K-outer operands.
//
// Every complex GEMM runs as three real FP32 GEMMs (P1 = Ar Br, P2 = Ai Bi,
// P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2, Im = P3 - P1 - P2) on
// v_mfma_f32_32x32x2f32.  Operands are kept K-outer, [plane][k][x] with x
// contiguous and every row padded to a multiple of 4 floats, so a lane's MFMA
// fragment (one float of row l%32 at k + l/32) is a conflict-free LDS read and
// operand tiles move by 16-byte direct global->LDS loads into a double ring.
// The contraction reads the FP32 rows Z[k][pair] as they are and flushes FP32
// partials into FP64 every 256 rows.
#include <stdio.h>

#include <mutex>
#include <vector>

#include "common.h"
#include "eri.h"

namespace dmet {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
#define F32_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

constexpr int NXCD = 8;
constexpr int FLUSH = 256;

__device__ inline long xcd_map(long b, long n) {
    const long per = (n + NXCD - 1) / NXCD;
    return (b % NXCD) * per + b / NXCD;
}

inline int pad4(int n) { return (n + 3) / 4 * 4; }

// ------------------------------------------------------------------ packing
// lmunu[qk][L][mu][nu] -> PL[qk][plane][nu (nao_p)][L*nao_p + mu]; 32 rows x 32 nu
// per workgroup through LDS: each thread reads 4 consecutive nu of one row (16-byte
// complex loads, all issued before the LDS stores) and writes 4 consecutive rows
// of one nu and plane as one 16-byte store.  Blocks (q, k) that the k <-> q-k
// paired transform does not read are skipped.
template <class TIn>
__global__ void __launch_bounds__(256) k_f32_pack_lmunu(const TIn* __restrict__ lm, int nao, int nao_p, int naux,
                                                        float* __restrict__ out, Mesh mesh) {
    __shared__ float sh[3][32][33];
    const int M1 = naux * nao_p;
    const int row0 = blockIdx.x * 32, nu0 = blockIdx.y * 32, qk = blockIdx.z;
    if (!kpair_needed(mesh, qk / mesh.nk, qk % mesh.nk)) return;
    const int t = threadIdx.x;
    {
        const int r = t / 8, v0 = (t % 8) * 4, row = row0 + r;
        const int L = min(row, M1 - 1) / nao_p, mu = min(row, M1 - 1) % nao_p;
        const bool rok = row < M1 && mu < nao;
        const TIn* src = lm + (((size_t)qk * naux + L) * nao + min(mu, nao - 1)) * (size_t)nao * 2;
        float re[4], im[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int nu = min(nu0 + v0 + u, nao - 1);
            re[u] = (float)src[2 * nu];
            im[u] = (float)src[2 * nu + 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = rok && nu0 + v0 + u < nao;
            const float a = ok ? re[u] : 0.f, b = ok ? im[u] : 0.f;
            sh[0][v0 + u][r] = a;
            sh[1][v0 + u][r] = b;
            sh[2][v0 + u][r] = a + b;
        }
    }
    __syncthreads();
    const int v = t / 8, r0 = (t % 8) * 4, nu = nu0 + v, row = row0 + r0;
    if (row < M1 && nu < nao_p) {
        const size_t plane = (size_t)nao_p * M1;
        float* o = out + (size_t)qk * 3 * plane + (size_t)nu * M1 + row;
#pragma unroll
        for (int pl = 0; pl < 3; ++pl)
            *reinterpret_cast<float4*>(o + pl * plane) =
                make_float4(sh[pl][v][r0], sh[pl][v][r0 + 1], sh[pl][v][r0 + 2], sh[pl][v][r0 + 3]);
    }
}

// C^k[s][k][nu][j] -> PC1[k][plane][nu][s*neo_p + j] (Cr, Ci, Cr + Ci)
__global__ void k_f32_pack_c1(const double* __restrict__ ck, int nk, int nspin, int nao, int nao_p, int neo,
                              int neo_p, float* __restrict__ out) {
    const int nbp = nspin * neo_p;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int nu = blockIdx.y, k = blockIdx.z;
    if (col >= nbp) return;
    const int s = col / neo_p, j = col % neo_p;
    float re = 0.f, im = 0.f;
    if (nu < nao && j < neo) {
        const double* c = ck + ((((size_t)s * nk + k) * nao + nu) * neo + j) * 2;
        re = (float)c[0];
        im = (float)c[1];
    }
    const size_t plane = (size_t)nao_p * nbp;
    float* o = out + (size_t)k * 3 * plane + (size_t)nu * nbp + col;
    o[0] = re;
    o[plane] = im;
    o[2 * plane] = re + im;
}

// conj(C^k)[s][(k,mu)][i] -> PC2[s][plane][k*nao_p + mu][i] (Cr, -Ci, Cr - Ci)
__global__ void k_f32_pack_c2(const double* __restrict__ ck, int nk, int nao, int nao_p, int neo, int neo_p,
                              float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = blockIdx.y, s = blockIdx.z;
    if (i >= neo_p) return;
    const int k = kk / nao_p, mu = kk % nao_p;
    float re = 0.f, im = 0.f;
    if (mu < nao && i < neo) {
        const double* c = ck + ((((size_t)s * nk + k) * nao + mu) * neo + i) * 2;
        re = (float)c[0];
        im = (float)c[1];
    }
    const size_t plane = (size_t)nk * nao_p * neo_p;
    float* o = out + (size_t)s * 3 * plane + (size_t)kk * neo_p + i;
    o[0] = re;
    o[plane] = -im;
    o[2 * plane] = re - im;
}

// ------------------------------------------------------------------ ring pieces
// Stage of NPL planes x BK k-rows x ROWS floats of a K-outer operand
// (row length X floats, a multiple of 4; plane stride pst floats) moved to
// LDS [plane][k][ROWS]; chunk columns past the row end are clamped.
template <int NPL, int BK, int ROWS>
__device__ inline void f32_issue(const float* base, size_t pst, int X, int x0, int k0, float* dst) {
    constexpr int CPR = ROWS / 4;                 // 16-byte chunks per k-row
    constexpr int CH = NPL * BK * CPR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int first = wave * 64; first < CH; first += 256) {
        const int c = first + lane;
        const int p = c / (BK * CPR), rem = c % (BK * CPR), k = rem / CPR, xq = rem % CPR;
        const int x = min(x0 + 4 * xq, X - 4);
        const float* src = base + (size_t)p * pst + (size_t)(k0 + k) * X + x;
        __builtin_amdgcn_global_load_lds((const void*)src, F32_LDS_PTR(dst + 4 * first), 16, 0, 0);
    }
}

template <int NPL, int BK, int BM, int BN, int TM, int TN>
__device__ inline void f32_mma(const float* sA, const float* sB, int wm0, int wn0, f16v (&acc)[NPL][TM][TN]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
        const int kr = kk + (lane >> 5);
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            float a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = sA[(p * BK + kr) * BM + wm0 + i * 32 + (lane & 31)];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = sB[(p * BK + kr) * BN + wn0 + j * 32 + (lane & 31)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[p][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[p][i][j], 0, 0, 0);
        }
    }
}

// K loop with a double ring; `nst` stages of BK rows each.
template <int NPL, int BK, int BM, int BN, int TM, int TN>
__device__ inline void f32_loop(const float* pa, size_t pa_st, int XA, int m0, const float* pb, size_t pb_st, int XB,
                                int n0, int nst, float* ring, int wm0, int wn0, f16v (&acc)[NPL][TM][TN]) {
    constexpr int SA = NPL * BK * BM, SB = NPL * BK * BN;
    f32_issue<NPL, BK, BM>(pa, pa_st, XA, m0, 0, ring);
    f32_issue<NPL, BK, BN>(pb, pb_st, XB, n0, 0, ring + SA);
    for (int st = 0; st < nst; ++st) {
        float* cur = ring + (size_t)(st & 1) * (SA + SB);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) {
            float* nxt = ring + (size_t)((st + 1) & 1) * (SA + SB);
            f32_issue<NPL, BK, BM>(pa, pa_st, XA, m0, BK * (st + 1), nxt);
            f32_issue<NPL, BK, BN>(pb, pb_st, XB, n0, BK * (st + 1), nxt + SA);
        }
        f32_mma<NPL, BK, BM, BN, TM, TN>(cur, cur + SA, wm0, wn0, acc);
    }
}

// ------------------------------------------------------------------ stage 1
// T[(L,mu)][(s,j)] for one (q, k), both spins; planes (Tr, Ti, Tr + Ti) written
// to T[s][plane][k*nao_p + mu][L*neo_p + j].
constexpr int S1_BM = 128, S1_BN = 128, S1_BK = 8;

// Only the kept k of the k <-> q-k pairing; T rows slot*nao_p + mu hold k = ks.k[slot].
__global__ void __launch_bounds__(256) k_f32_xf1(Mesh mesh, int q, int naux, int nao_p, int neo, int neo_p, int nspin,
                                                 KSlots ks, const float* __restrict__ plm,
                                                 const float* __restrict__ pc1, float* __restrict__ t) {
    constexpr int BM = S1_BM, BN = S1_BN, BK = S1_BK, TM = 2, TN = 2;
    extern __shared__ __align__(16) float ring[];
    const int nk = mesh.nk, M1 = naux * nao_p, NBp = nspin * neo_p;
    const int nmt = (M1 + BM - 1) / BM, nnt = (NBp + BN - 1) / BN;
    const long logical = xcd_map(blockIdx.x, gridDim.x);
    if (logical >= (long)(ks.npaired + ks.nself) * nmt * nnt) return;
    const int slot = (int)(logical / ((long)nmt * nnt));
    const int k = ks.k[slot];
    const int rem = (int)(logical % ((long)nmt * nnt));
    const int m0 = (rem / nnt) * BM, n0 = (rem % nnt) * BN;
    const int kmq = mesh_sub(mesh, k, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
    f16v acc[3][TM][TN];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[p][i][j][r] = 0.f;
    const float* pa = plm + ((size_t)q * nk + k) * 3 * (size_t)nao_p * M1;
    const float* pb = pc1 + (size_t)kmq * 3 * (size_t)nao_p * NBp;
    f32_loop<3, BK, BM, BN, TM, TN>(pa, (size_t)nao_p * M1, M1, m0, pb, (size_t)nao_p * NBp, NBp, n0, nao_p / BK, ring,
                                    wm0, wn0, acc);
    const size_t N2p = (size_t)naux * neo_p, K2 = (size_t)nk * nao_p;
    const size_t plane = K2 * N2p;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int col = n0 + wn0 + j * 32 + (lane & 31);
                if (row >= M1 || col >= NBp) continue;
                const int s = col / neo_p, jj = col % neo_p;
                if (jj >= neo) continue;
                const int L = row / nao_p, mu = row % nao_p;
                const float p1 = acc[0][i][j][r], p2 = acc[1][i][j][r], p3 = acc[2][i][j][r];
                const float tr = p1 - p2, ti = p3 - p1 - p2;
                float* o = t + (size_t)s * 3 * plane + ((size_t)slot * nao_p + mu) * N2p + (size_t)L * neo_p + jj;
                o[0] = tr;
                o[plane] = ti;
                o[2 * plane] = tr + ti;
            }
}

// ------------------------------------------------------------------ stage 2
constexpr int S2_BM = 64, S2_BN = 64, S2_BK = 8;

// Stage 2 under the k <-> q-k pairing: pass 1 over the rows (k, mu) of all
// kept k (A = conj C rows i, B = T columns (L, j)), pass 2 over the paired k
// with the operands swapped (A = T columns (L, i), B = conj C rows j), which
// adds the partners' transposed terms.  T rows are compact by slot.
__global__ void __launch_bounds__(256) k_f32_xf2(int naux, int neo, int neo_p, int nao_p, int K2, KSlots ks,
                                                 int self_conj, size_t zrow0, float wq, const float* __restrict__ pc2,
                                                 const float* __restrict__ t, float* __restrict__ z, size_t ldz) {
    constexpr int BM = S2_BM, BN = S2_BN, BK = S2_BK, TM = 1, TN = 1;
    constexpr int SA = 3 * BK * BM, SB = 3 * BK * BN;
    extern __shared__ __align__(16) float ring[];
    const int njt = (neo + BN - 1) / BN, nit = (neo + BM - 1) / BM;
    const long id = xcd_map(blockIdx.x, gridDim.x);
    const int per_l = njt * nit;
    const int L = (int)(id / per_l), rem = (int)(id % per_l);
    const int jt = rem / nit, it = rem % nit;
    if (L >= naux) return;
    const int m0 = it * BM, j0 = jt * BN;
    if (m0 + BM - 1 < j0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
    const size_t N2p = (size_t)naux * neo_p;
    f16v acc[3][TM][TN];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[p][0][0][r] = 0.f;
    const int spk = nao_p / BK;                               // stages per k slot
    const int s1 = (ks.npaired + ks.nself) * spk, nst = s1 + ks.npaired * spk;
    __shared__ short ksh[KP_MAX];   // the slot -> k table in LDS (no memory round trip per stage)
    for (int t = threadIdx.x; t < ks.npaired + ks.nself; t += blockDim.x) ksh[t] = ks.k[t];
    __syncthreads();
    const size_t cst = (size_t)K2 * neo_p, tst = (size_t)K2 * N2p;
    // running position: pass, stage within the pass, its slot and row offset
    int pass = 0, sp = 0, slot = 0, roff = 0;
    auto issue = [&](float* dst) {
        if (pass == 0 && sp == s1) {
            pass = 1;
            sp = slot = roff = 0;
        }
        const int kc = ksh[slot] * nao_p + roff, kt_ = sp * BK;   // rows of conj C and of T
        // B columns past L's own neo_p would belong to L+1 (or are clamped at
        // the end of T): they only reach outputs that are dropped
        if (!pass) {
            f32_issue<3, BK, BM>(pc2, cst, neo_p, m0, kc, dst);
            f32_issue<3, BK, BN>(t, tst, (int)N2p, L * neo_p + j0, kt_, dst + SA);
        } else {
            f32_issue<3, BK, BM>(t, tst, (int)N2p, L * neo_p + m0, kt_, dst);
            f32_issue<3, BK, BN>(pc2, cst, neo_p, j0, kc, dst + SA);
        }
        ++sp;
        roff += BK;
        if (roff == nao_p) {
            roff = 0;
            ++slot;
        }
    };
    issue(ring);
    for (int st = 0; st < nst; ++st) {
        float* cur = ring + (size_t)(st & 1) * (SA + SB);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) issue(ring + (size_t)((st + 1) & 1) * (SA + SB));
        f32_mma<3, BK, BM, BN, TM, TN>(cur, cur + SA, wm0, wn0, acc);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = m0 + wm0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = j0 + wn0 + (lane & 31);
        if (i >= neo || j >= neo || j > i) continue;
        const size_t pair = (size_t)i * (i + 1) / 2 + j;
        const float p1 = acc[0][0][0][r], p2 = acc[1][0][0][r], p3 = acc[2][0][0][r];
        const float xr = p1 - p2, xi = p3 - p1 - p2;
        if (self_conj) {
            z[(zrow0 + L) * ldz + pair] = wq * xr;
        } else {
            z[(zrow0 + 2 * (size_t)L) * ldz + pair] = wq * xr;
            z[(zrow0 + 2 * (size_t)L + 1) * ldz + pair] = wq * xi;
        }
    }
}

// ------------------------------------------------------------------ contraction
template <int MODE>
__device__ inline bool f32_tile(long logical, int ntile, int& mt, int& nt) {
    constexpr int SB = 8;
    const long sb = logical / (SB * SB);
    const int within = (int)(logical % (SB * SB));
    const int nsb = (ntile + SB - 1) / SB;
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
    mt = (int)(I * SB + within / SB);
    nt = (int)(J * SB + within % SB);
    if (mt >= ntile || nt >= ntile) return false;
    if (MODE == 0 && nt > mt) return false;
    return true;
}

template <int MODE>
long f32_grid(int ntile) {
    const long nsb = (ntile + 7) / 8;
    const long n = (MODE == 0 ? nsb * (nsb + 1) / 2 : nsb * nsb) * 64;
    return (n + NXCD - 1) / NXCD * NXCD;
}

constexpr int C_BK = 16, C_NBUF = 3;

template <int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_f32_contract(int npair, int krows, const float* __restrict__ za, const float* __restrict__ zb, size_t ldz,
               long nblocks, double* __restrict__ out) {
    constexpr int BM = 128, BN = 128, BK = C_BK, TM = 2, TN = 2, NBUF = C_NBUF;
    constexpr int SA = BK * BM, SB = BK * BN;
    constexpr int LOADS = (BK * (BM + BN) / 4) / 256;
    extern __shared__ __align__(16) float ring[];
    int mt, nt;
    const long logical = xcd_map(blockIdx.x, nblocks);
    const int ntile = (npair + BM - 1) / BM;
    if (!f32_tile<MODE>(logical, ntile, mt, nt)) return;
    const int m0 = mt * BM, n0 = nt * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
    const int X = (int)ldz;
    f16v acc[1][TM][TN];
    double acc64[TM][TN][16];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[0][i][j][r] = 0.f;
                acc64[i][j][r] = 0.0;
            }
    const int nst = (krows + BK - 1) / BK;
    auto issue = [&](int st) {
        float* d = ring + (size_t)(st % NBUF) * (SA + SB);
        f32_issue<1, BK, BM>(za, 0, X, m0, st * BK, d);
        f32_issue<1, BK, BN>(zb, 0, X, n0, st * BK, d + SA);
    };
    for (int s = 0; s < NBUF - 1; ++s)
        if (s < nst) issue(s);
    int since = 0;
    for (int st = 0; st < nst; ++st) {
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) __builtin_amdgcn_s_waitcnt(0x0F70 | (LOADS & 15) | ((LOADS >> 4) << 14));
        else __builtin_amdgcn_s_waitcnt(0x0F70);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (st + NBUF - 1 < nst) issue(st + NBUF - 1);
        const float* cur = ring + (size_t)(st % NBUF) * (SA + SB);
        f32_mma<1, BK, BM, BN, TM, TN>(cur, cur + SA, wm0, wn0, acc);
        since += BK;
        if (since >= FLUSH || st + 1 == nst) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        acc64[i][j][r] += (double)acc[0][i][j][r];
                        acc[0][i][j][r] = 0.f;
                    }
            since = 0;
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int IJ = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int KL = n0 + wn0 + j * 32 + (lane & 31);
                if (IJ >= npair || KL >= npair) continue;
                if constexpr (MODE == 0) {
                    if (KL <= IJ) out[(size_t)IJ * (IJ + 1) / 2 + KL] = acc64[i][j][r];
                } else {
                    out[(size_t)IJ * npair + KL] = acc64[i][j][r];
                }
            }
}

// zero the padding of Z [nspin][rows_p][ldz]: rows [rows, rows_p) enter every
// contraction sum; columns [npair, ldz) only reach dropped outputs but are
// cleared as well so no stale value is ever read
__global__ void k_f32_zero_pad(float* __restrict__ z, int nspin, int rows, int rows_p, int npair, int ldz) {
    const int padc = ldz - npair;
    const long ncol = (long)nspin * rows * padc;
    const long nrow = (long)nspin * (rows_p - rows) * ldz;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < ncol + nrow; e += (long)gridDim.x * blockDim.x) {
        long s, r, c;
        if (e < ncol) {
            s = e / ((long)rows * padc);
            const long rem = e % ((long)rows * padc);
            r = rem / padc;
            c = npair + rem % padc;
        } else {
            const long f = e - ncol;
            s = f / ((long)(rows_p - rows) * ldz);
            const long rem = f % ((long)(rows_p - rows) * ldz);
            r = rows + rem / ldz;
            c = rem % ldz;
        }
        z[(s * rows_p + r) * ldz + c] = 0.f;
    }
}

struct F32Dims {
    int nao_p, neo_p, M1, NBp, K2, ldz, rows_p;
    size_t N2p;
    size_t lm, c1, c2, t, z;
};

F32Dims f32_dims(const EriPlan& p) {
    F32Dims d;
    d.nao_p = (p.nao + 7) / 8 * 8;
    d.neo_p = pad4(p.neo);
    d.M1 = p.naux * d.nao_p;
    d.NBp = p.nspin * d.neo_p;
    d.K2 = p.mesh.nk * d.nao_p;
    d.N2p = (size_t)p.naux * d.neo_p;
    d.ldz = pad4(p.npair);
    d.rows_p = (p.zrows + C_BK - 1) / C_BK * C_BK;
    d.lm = (size_t)p.mesh.nk * p.mesh.nk * 3 * d.nao_p * d.M1;
    d.c1 = (size_t)p.mesh.nk * 3 * d.nao_p * d.NBp;
    d.c2 = (size_t)p.nspin * 3 * d.K2 * d.neo_p;
    d.t = (size_t)p.nspin * 3 * d.K2 * d.N2p;
    d.z = (size_t)p.nspin * d.rows_p * d.ldz;
    return d;
}

}  // namespace

// Dynamic LDS limits of the FP32 kernels, set once per device (a host call,
// kept out of graph captures: the batched driver calls this before capturing).
dmet_status eri_f32_prepare() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    DMET_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= 0 && dev < 64 && done[dev]) return DMET_OK;
    constexpr size_t lds1 = (size_t)2 * 3 * S1_BK * (S1_BM + S1_BN) * 4;
    constexpr size_t lds2 = (size_t)2 * 3 * S2_BK * (S2_BM + S2_BN) * 4;
    constexpr size_t lds3 = (size_t)C_NBUF * C_BK * 256 * 4;
    DMET_HIP(hipFuncSetAttribute((const void*)k_f32_xf1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1));
    DMET_HIP(hipFuncSetAttribute((const void*)k_f32_xf2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
    DMET_HIP(hipFuncSetAttribute((const void*)k_f32_contract<0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds3));
    DMET_HIP(hipFuncSetAttribute((const void*)k_f32_contract<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds3));
    if (dev >= 0 && dev < 64) done[dev] = true;
    return DMET_OK;
}

size_t eri_f32_workspace(const EriPlan& p) {
    F32Dims d = f32_dims(p);
    Carve cv(nullptr, 0);
    cv.take<float>(d.lm);
    cv.take<float>(d.c1);
    cv.take<float>(d.c2);
    cv.take<float>(d.t);
    cv.take<float>(d.z);
    return cv.bytes();
}

__global__ void k_f32_z_to_f64(const float* __restrict__ z, int rows, int rows_p, int npair, int ldz, int nspin,
                               double* __restrict__ out) {
    const long n = (long)nspin * rows * npair;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const long s = e / ((long)rows * npair), rem = e % ((long)rows * npair);
        const long r = rem / npair, c = rem % npair;
        out[e] = (double)z[(s * rows_p + r) * ldz + c];
    }
}

dmet_status eri_f32(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa, double* eri_bb,
                    double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st, double* df_out) {
    F32Dims d = f32_dims(p);
    Carve cv(ws, ws_bytes);
    float* plm = cv.take<float>(d.lm);
    float* pc1 = cv.take<float>(d.c1);
    float* pc2 = cv.take<float>(d.c2);
    float* t = cv.take<float>(d.t);
    float* z = cv.take<float>(d.z);
    if (cv.bytes() > ws_bytes) return fail(DMET_E_WORKSPACE, "transform_eri workspace too small");
    const int nk = p.mesh.nk;
    if (nk > KP_MAX) return fail(DMET_E_UNSUPPORTED, "FP32-3M transform supports at most 256 k-points");
    {
        ProfScope ps("pack_in_f32", st);
        if (p.dtype == DMET_C128)
            k_f32_pack_lmunu<double><<<dim3((d.M1 + 31) / 32, (d.nao_p + 31) / 32, nk * nk), 256, 0, st>>>(
                static_cast<const double*>(lmunu), p.nao, d.nao_p, p.naux, plm, p.mesh);
        else
            k_f32_pack_lmunu<float><<<dim3((d.M1 + 31) / 32, (d.nao_p + 31) / 32, nk * nk), 256, 0, st>>>(
                static_cast<const float*>(lmunu), p.nao, d.nao_p, p.naux, plm, p.mesh);
        k_f32_pack_c1<<<dim3((d.NBp + 255) / 256, d.nao_p, nk), 256, 0, st>>>(ck, nk, p.nspin, p.nao, d.nao_p, p.neo,
                                                                            d.neo_p, pc1);
        k_f32_pack_c2<<<dim3((d.neo_p + 255) / 256, d.K2, p.nspin), 256, 0, st>>>(ck, nk, p.nao, d.nao_p, p.neo,
                                                                                  d.neo_p, pc2);
        k_f32_zero_pad<<<1024, 256, 0, st>>>(z, p.nspin, p.zrows, d.rows_p, p.npair, d.ldz);
        ps.stop();
    }
    DMET_LAUNCH_CHECK("f32 pack");
    constexpr size_t lds1 = (size_t)2 * 3 * S1_BK * (S1_BM + S1_BN) * 4;
    constexpr size_t lds2 = (size_t)2 * 3 * S2_BK * (S2_BM + S2_BN) * 4;
    constexpr size_t lds3 = (size_t)C_NBUF * C_BK * 256 * 4;
    {
        dmet_status sp = eri_f32_prepare();
        if (sp != DMET_OK) return sp;
    }
    const size_t tsp = (size_t)3 * d.K2 * d.N2p, c2sp = (size_t)3 * d.K2 * d.neo_p;
    const size_t zsp = (size_t)d.rows_p * d.ldz;
    const int njt = (p.neo + S2_BN - 1) / S2_BN, nit = (p.neo + S2_BM - 1) / S2_BM;
    for (const QBlock& qb : p.qblocks) {
        const KSlots ks = kpair_slots(p.mesh, qb.q);
        const long nb1 = ((long)(ks.npaired + ks.nself) * ((d.M1 + S1_BM - 1) / S1_BM) *
                              ((d.NBp + S1_BN - 1) / S1_BN) + NXCD - 1) / NXCD * NXCD;
        ProfScope ps1("xform1_f32", st);
        k_f32_xf1<<<dim3((unsigned)nb1), 256, lds1, st>>>(p.mesh, qb.q, p.naux, d.nao_p, p.neo, d.neo_p, p.nspin, ks,
                                                          plm, pc1, t);
        ps1.stop();
        DMET_LAUNCH_CHECK("xform1_f32");
        for (int s = 0; s < p.nspin; ++s) {
            const long nb2 = ((long)p.naux * njt * nit + NXCD - 1) / NXCD * NXCD;
            ProfScope ps2("xform2_f32", st);
            k_f32_xf2<<<dim3((unsigned)nb2), 256, lds2, st>>>(p.naux, p.neo, d.neo_p, d.nao_p, d.K2, ks, qb.self_conj,
                                                              qb.zrow0, (float)qb.weight, pc2 + s * c2sp,
                                                              t + s * tsp, z + s * zsp, (size_t)d.ldz);
            ps2.stop();
            DMET_LAUNCH_CHECK("xform2_f32");
        }
    }
    if (df_out) {
        k_f32_z_to_f64<<<1024, 256, 0, st>>>(z, p.zrows, d.rows_p, p.npair, d.ldz, p.nspin, df_out);
        DMET_LAUNCH_CHECK("k_f32_z_to_f64");
        return DMET_OK;
    }
    auto kc0 = k_f32_contract<0>;
    auto kc1 = k_f32_contract<1>;
    const int ntile = (p.npair + 127) / 128;
    for (int s = 0; s < p.nspin; ++s) {
        const long nb = f32_grid<0>(ntile);
        ProfScope ps("contract_s8_f32", st);
        kc0<<<dim3((unsigned)nb), 256, lds3, st>>>(p.npair, d.rows_p, z + s * zsp, z + s * zsp, (size_t)d.ldz, nb,
                                                   s == 0 ? eri_aa : eri_bb);
        ps.stop();
        DMET_LAUNCH_CHECK("contract_s8_f32");
    }
    if (p.nspin == 2 && eri_ab) {
        const long nb = f32_grid<1>(ntile);
        ProfScope ps("contract_s4_f32", st);
        kc1<<<dim3((unsigned)nb), 256, lds3, st>>>(p.npair, d.rows_p, z, z + zsp, (size_t)d.ldz, nb, eri_ab);
        ps.stop();
        DMET_LAUNCH_CHECK("contract_s4_f32");
    }
    return DMET_OK;
}

}  // namespace dmet
