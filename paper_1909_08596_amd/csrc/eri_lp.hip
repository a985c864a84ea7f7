// Split-BF16 forms of the embedding-ERI transformation (Alg. 1).
//
// Every complex GEMM of the transform runs as 4 real GEMMs (4M) on (re, im)
// planes, Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br (against 3M on three planes
// it moves a third fewer operand bytes, which bound these kernels, and has no
// (re + im) cancellation), with each FP32 operand split into bf16 parts for
// v_mfma_f32_32x32x16_bf16 (the precision names keep their 3M suffix):
//   DMET_BF16X3_3M : x = hi + lo (hi = bf16(x), lo = bf16(x - hi)); each real
//                    product formed as hi*hi + hi*lo + lo*hi with FP32
//                    accumulation.  On the diagonal tiles of the contraction
//                    (which hold (ij|ij), where the dropped lo*lo terms are
//                    squares and do not average out) lo*lo is added as well.
//                    The split leaves ~2^-17 relative per operand.
//   DMET_BF16X6_3M : three-way split x = hi + mid + lo and the six products
//                    whose order is at most 2^-16 (hh, hm, mh, hl, mm, lh):
//                    ~2^-24 relative, FP32-level accuracy on the bf16 pipes.
//
// Intermediates are FP32: T (stage-1 output, two planes Tr, Ti) and
// Z (real rows of the contraction), both stored as packed bf16 parts
// [plane][part][k/8][x][8] so that one MFMA operand fragment (8 consecutive k
// of one row) is one aligned 16-byte chunk moved straight from global memory
// into LDS.  The contraction accumulates FP32 MFMA partials over chunks of
// FLUSH_K rows and adds them into FP64 registers.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

#include <vector>

#include "common.h"
#include "eri.h"

namespace dmet {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int NS>
__device__ inline void split_bf16(float x, __bf16 (&part)[NS]) {
    float r = x;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        part[s] = (__bf16)r;
        r = r - (float)part[s];
    }
}

// ------------------------------------------------------------------ packed split operands
// P[t][g][x][v] (bf16) = part t of Z[8 g + v][x]: the k-index in groups of 8 so
// that one MFMA operand fragment (8 consecutive k of one row) is one aligned
// 16-byte chunk.  Rows beyond krows are zero.  FP64 rows are rounded to FP32
// first (the three parts carry FP32's 24 bits).  Groups g = blockIdx.y +
// j gridDim.y (the grid's y extent is capped at 65535).
template <int NS, class T = float>
__global__ void k_pack_parts(const T* __restrict__ z, size_t ldz, int krows, int ncol, int kgroups,
                             __bf16* __restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ncol) return;
    const size_t plane = (size_t)kgroups * ncol;
    for (int g = blockIdx.y; g < kgroups; g += gridDim.y) {
        bf8 part[NS];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int k = 8 * g + v;
            const float val = k < krows ? (float)z[(size_t)k * ldz + x] : 0.f;
            __bf16 sp[NS];
            split_bf16<NS>(val, sp);
#pragma unroll
            for (int t = 0; t < NS; ++t) part[t][v] = sp[t];
        }
#pragma unroll
        for (int t = 0; t < NS; ++t)
            *reinterpret_cast<bf8*>(out + ((size_t)t * plane + (size_t)g * ncol + x) * 8) = part[t];
    }
}

// grid y extent for a kernel that loops over row groups
inline unsigned group_grid(int groups) { return (unsigned)std::min(groups, 65535); }

// Tile order: super-blocks of SB x SB output tiles, visited (for s8) in
// lower-triangular order; logical ids are assigned so that each XCD (the
// hardware hands workgroup b to XCD b % 8) receives a contiguous run of
// super-blocks and the tiles it runs together share A/B panels in its L2.
constexpr int SB = 8;
constexpr int NXCD = 8;

__device__ inline long xcd_logical(long b, long nblocks) {
    const long per = (nblocks + NXCD - 1) / NXCD;
    return (b % NXCD) * per + b / NXCD;
}

template <int MODE, int SB = SB>
__device__ inline bool tile_of(long logical, int ntile, int& mt, int& nt) {
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

template <int MODE, int SB = SB>
inline long tile_grid(int ntile) {
    const long nsb = (ntile + SB - 1) / SB;
    const long nsbt = MODE == 0 ? nsb * (nsb + 1) / 2 : nsb * nsb;
    const long n = nsbt * SB * SB;
    return (n + NXCD - 1) / NXCD * NXCD;
}

// Contraction on packed bf16 parts.  Operand tiles move by direct
// global->LDS loads (lane l of a wave writes its 16 bytes at the wave's LDS
// base + 16 l; FLAT global_load_lds_dwordx4 or, where exact LDS waits matter,
// buffer_load_dwordx4 ... lds) into a ring of stages, so that the tiles of the
// next stages are in flight while one is multiplied.  Rows past the matrix
// edge are clamped to the last row: they only feed output rows / columns that
// are not stored.
#define DMET_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))
// Word 3 of a raw buffer resource (32-bit dwords, no swizzle, range-checked)
#define DMET_RSRC_WORD3 0x00020000

// A pointer that is the same in every lane, moved to scalar registers.
__device__ inline const void* wave_uniform(const void* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (const void*)(((unsigned long long)hi << 32) | lo);
}

// Direct load of this lane's 16 bytes at byte offset off of a row (the same
// in every lane, nbytes long) into LDS at dst + 16 * lane.  The buffer form
// bounds the load by the row and keeps the compiler's LDS waits exact.
__device__ inline void lds_dma16(const void* row, unsigned nbytes, unsigned off, void* dst) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(wave_uniform(row)), (short)0, (int)nbytes, DMET_RSRC_WORD3),
        DMET_LDS_PTR(dst), 16, (int)off, 0, 0, 0);
}

// One scheduling section: nr LDS reads issued first, then nm MFMAs; nothing is
// moved across its end
#define DMET_SECTION(nr, nm)                                 \
    __builtin_amdgcn_sched_group_barrier(0x100, nr, 0);      \
    __builtin_amdgcn_sched_group_barrier(0x008, nm, 0);      \
    __builtin_amdgcn_sched_barrier(0)

// Tile order of k_contract_w8 (128 x 256 tiles): super-blocks of 8 x 4 tiles
// (1024 x 1024 outputs), lower-triangular order of super-blocks for s8.  A
// tile is kept for s8 if it holds any KL <= IJ.
template <int MODE>
__device__ inline bool w8_tile_of(long logical, int ntm, int ntn, int& mt, int& nt) {
    const long sb = logical / 32;
    const int within = (int)(logical % 32);
    const int nsb = (ntm + 7) / 8;
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
    mt = (int)(I * 8 + within / 4);
    nt = (int)(J * 4 + within % 4);
    if (mt >= ntm || nt >= ntn) return false;
    if (MODE == 0 && nt * 256 > mt * 128 + 127) return false;
    return true;
}

inline long w8_grid(int mode, int npair) {
    const long nsb = ((npair + 127) / 128 + 7) / 8;
    const long n = (mode == 0 ? nsb * (nsb + 1) / 2 : nsb * nsb) * 32;
    return (n + NXCD - 1) / NXCD * NXCD;
}

// 128 x 256 output tiles: 8 waves as 2 x 4, wave tile 64 x 64 (FP32 MFMA
// partials flushed into FP64 registers every flush_k rows), one workgroup per
// CU and a ring of G-group stages in LDS (three-way split: two 72 KB stages of
// 32 rows; two-way: three 48 KB stages).  Against two 128 x 128 workgroups per
// CU it moves 25% fewer operand bytes per flop, and the two column halves that
// share the A panel run in step by construction.  Operands are staged with buffer
// loads straight into LDS: each buffer resource spans one row group of one
// part, so the hardware range check bounds every load, and (unlike the FLAT
// form) the compiler keeps exact lgkmcnt waits for the LDS reads behind them.
// Row split: the workgroups of blockIdx.y = y sum the row groups
// [y ksplit, min((y + 1) ksplit, kgroups)) (parts kplane groups apart) into
// out + y out_split; one split (ksplit = kgroups, out_split 0) is the plain sum.
template <int NS, int MODE, int G, int NBUF>
__global__ void __launch_bounds__(512) k_contract_w8(int npair, int kgroups, const __bf16* __restrict__ pa,
                                                     const __bf16* __restrict__ pb, int flush_k, long nblocks,
                                                     double* __restrict__ out, int kplane, int ksplit,
                                                     size_t out_split) {
    constexpr int BM = 128, BN = 256;
    constexpr int TM = 2, TN = 2;
    constexpr int PA = G * BM, PB = G * BN;      // 16-byte chunks of one part of A / B per stage
    constexpr int STAGE = NS * (PA + PB);
    // every wave stages PA / 8 chunks of each part of A (with that many lanes)
    // and PB / 8 of B, so all waves wait on the same load count
    constexpr int CA = PA / 8, NLB = PB / 512;
    static_assert(CA == 32 || CA == 64, "A chunks per wave");
    static_assert(PB % 512 == 0, "B chunks per wave");
    constexpr int LOADS = NS * (1 + NLB);        // load instructions per thread per stage
    extern __shared__ __align__(16) bf8 ring[];
    int mt, nt;
    const long logical = xcd_logical(blockIdx.x, nblocks);
    const int ntm = (npair + BM - 1) / BM, ntn = (npair + BN - 1) / BN;
    if (!w8_tile_of<MODE>(logical, ntm, ntn, mt, nt)) return;
    const int m0 = mt * BM, n0 = nt * BN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar registers
    const int wm0 = (wave >> 2) * 64, wn0 = (wave & 3) * 64;
    const int kbeg = blockIdx.y * ksplit;
    pa += (size_t)kbeg * npair * 8;
    pb += (size_t)kbeg * npair * 8;
    out += blockIdx.y * out_split;
    const size_t plane = (size_t)kplane * npair;
    const int nkt = min(ksplit, kgroups - kbeg) / G;
    // this lane's byte offset within its rows (fixed over stages) and the
    // wave-uniform row pointers of the next stage to issue
    const int fa = wave * CA;
    const unsigned offa = (unsigned)min(m0 + fa % BM + (lane & (CA - 1)), npair - 1) * 16u;
    unsigned offb[NLB];
    const char* rowa[NS];
    const char* rowb[NS][NLB];
#pragma unroll
    for (int h = 0; h < NLB; ++h) offb[h] = (unsigned)min(n0 + (h * 512 + wave * 64) % BN + lane, npair - 1) * 16u;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        rowa[t] = (const char*)pa + (t * plane + (size_t)(fa / BM) * npair) * 16;
#pragma unroll
        for (int h = 0; h < NLB; ++h)
            rowb[t][h] = (const char*)pb + (t * plane + (size_t)((h * 512 + wave * 64) / BN) * npair) * 16;
    }
    const size_t stage_bytes = (size_t)G * npair * 16;
    auto issue = [&](int kt) {   // stages are issued in increasing order
        bf8* st = ring + (size_t)(kt % NBUF) * STAGE;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (CA == 64 || lane < CA)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    __builtin_amdgcn_make_buffer_rsrc((void*)rowa[t], (short)0, npair * 16, DMET_RSRC_WORD3),
                    DMET_LDS_PTR(st + t * PA + fa), 16, (int)offa, 0, 0, 0);
            rowa[t] += stage_bytes;
#pragma unroll
            for (int h = 0; h < NLB; ++h) {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    __builtin_amdgcn_make_buffer_rsrc((void*)rowb[t][h], (short)0, npair * 16, DMET_RSRC_WORD3),
                    DMET_LDS_PTR(st + NS * PA + t * PB + h * 512 + wave * 64), 16, (int)offb[h], 0, 0, 0);
                rowb[t][h] += stage_bytes;
            }
        }
    };

    f16v acc[TM][TN];
    double acc64[TM][TN][16];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[i][j][r] = 0.f;
                acc64[i][j][r] = 0.0;
            }
#pragma unroll
    for (int s2 = 0; s2 < NBUF - 1; ++s2)
        if (s2 < nkt) issue(s2);
    int since = 0;
    // one stage: wait (vmcnt immediate YOUNGER * LOADS: the loads of the
    // younger stages in flight may stay outstanding), barrier, issue, multiply
    auto stage = [&](int kt, auto younger_c) {
        constexpr int YOUNGER = decltype(younger_c)::value;
        constexpr int VM = YOUNGER * LOADS;
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0F70 | (VM & 15) | ((VM >> 4) << 14));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (kt + NBUF - 1 < nkt) issue(kt + NBUF - 1);
        const bf8* sA = ring + (size_t)(kt % NBUF) * STAGE;
        const bf8* sB = sA + NS * PA;
        if constexpr (NS == 3 && G == 4) {
            // two k-steps, software-pipelined: every LDS read is issued four to
            // twelve MFMAs ahead of its first use and at most ten fragments are
            // live; the products of each step keep the order of the generic
            // loop below (smallest first), so the sums are the same bits
            const int g0 = lane >> 5, g1 = 2 + (lane >> 5);
            auto rdA = [&](bf8 (&r)[2], int t, int g) {
                r[0] = sA[t * PA + g * BM + wm0 + (lane & 31)];
                r[1] = sA[t * PA + g * BM + wm0 + 32 + (lane & 31)];
            };
            auto rdB = [&](bf8 (&r)[2], int t, int g) {
                r[0] = sB[t * PB + g * BN + wn0 + (lane & 31)];
                r[1] = sB[t * PB + g * BN + wn0 + 32 + (lane & 31)];
            };
            auto mm = [&](const bf8 (&a)[2], const bf8 (&b)[2]) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            };
            auto flush = [&](bool last) {
                since += 16;
                if (since >= flush_k || last) {
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                acc64[i][j][r] += (double)acc[i][j][r];
                                acc[i][j][r] = 0.f;
                            }
                    since = 0;
                }
            };
            // parts of the first step (a, b) and of the second (c, d)
            bf8 a2[2], a1[2], a0[2], b0[2], b1[2], b2[2];
            bf8 c2[2], c1[2], c0[2], d0[2], d1[2], d2[2];
            rdA(a2, 2, g0); rdB(b0, 0, g0);
            DMET_SECTION(4, 0);
            rdA(a1, 1, g0); rdB(b1, 1, g0);
            DMET_SECTION(4, 0);
            mm(a2, b0);
            DMET_SECTION(0, 4);
            rdA(a0, 0, g0); rdB(b2, 2, g0);
            mm(a1, b1);
            mm(a1, b0);
            DMET_SECTION(4, 8);
            rdA(c2, 2, g1);
            mm(a0, b2);
            DMET_SECTION(2, 4);
            rdB(d0, 0, g1);
            mm(a0, b1);
            DMET_SECTION(2, 4);
            rdA(c1, 1, g1);
            mm(a0, b0);
            DMET_SECTION(2, 4);
            rdB(d1, 1, g1); rdA(c0, 0, g1);
            DMET_SECTION(4, 0);
            flush(false);
            __builtin_amdgcn_sched_barrier(0);
            mm(c2, d0);
            DMET_SECTION(0, 4);
            rdB(d2, 2, g1);
            mm(c1, d1);
            mm(c1, d0);
            DMET_SECTION(2, 8);
            mm(c0, d2);
            mm(c0, d1);
            mm(c0, d0);
            DMET_SECTION(0, 12);
            flush(kt + 1 == nkt);
        } else {
#pragma unroll
        for (int ks = 0; ks < G; ks += 2) {
            const int g = ks + (lane >> 5);
            bf8 b[NS][TN];
#pragma unroll
            for (int t = 0; t < NS; ++t)
#pragma unroll
                for (int j = 0; j < TN; ++j) b[t][j] = sB[t * PB + g * BN + wn0 + j * 32 + (lane & 31)];
            // parts of A outermost and both row tiles per part, so that four
            // independent accumulators separate two MFMAs on the same one (the
            // order of the products per output element is unchanged)
#pragma unroll
            for (int ta = NS - 1; ta >= 0; --ta) {
                bf8 a[TM];
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = sA[ta * PA + g * BM + wm0 + i * 32 + (lane & 31)];
#pragma unroll
                for (int tb = NS - 1 - ta; tb >= 0; --tb)
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[tb][j], acc[i][j], 0, 0, 0);
                if constexpr (NS == 2) {
                    // lo*lo where the 128 x 128 tile of these outputs is a
                    // diagonal one (the same elements as in the other kernels)
                    if (ta == 1 && (n0 + wn0) / 128 == mt)
#pragma unroll
                        for (int i = 0; i < TM; ++i)
#pragma unroll
                            for (int j = 0; j < TN; ++j)
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[1][j], acc[i][j], 0, 0, 0);
                }
            }
            since += 16;
            if (since >= flush_k || (kt + 1 == nkt && ks + 2 >= G)) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            acc64[i][j][r] += (double)acc[i][j][r];
                            acc[i][j][r] = 0.f;
                        }
                since = 0;
            }
        }
        }
    };
    // a kernel-argument load still in flight would make the first LDS wait of
    // every stage a full one
    __builtin_amdgcn_s_waitcnt(0xC07F);
    // steady state with NBUF - 2 younger stages in flight, then the tail
    int kt = 0;
    for (; kt + NBUF - 2 < nkt; ++kt) stage(kt, std::integral_constant<int, NBUF - 2>{});
    if constexpr (NBUF >= 4) {
        if (kt + 1 < nkt) {
            stage(kt, std::integral_constant<int, 1>{});
            ++kt;
        }
    }
    for (; kt < nkt; ++kt) stage(kt, std::integral_constant<int, 0>{});
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

template <int NS, int G, int NBUF>
constexpr size_t w8_lds() { return (size_t)NBUF * NS * G * (128 + 256) * 16; }



// ------------------------------------------------------------------ int8 fixed-point contraction
// DMET_BF16X6_I8: the contraction (ij|kl) = sum_r Z[r][ij] Z[r][kl] on the int8
// matrix cores.  Each column x of Z (one EO pair) gets a power-of-two scale
// 2^e_x >= max_r |Z[r][x]| and its entries y = Z / 2^e_x in [-1, 1] are written
// exactly in three signed digits (a fixed-point split in the manner of the
// Ozaki scheme):
//   y = d0 / 127 + d1 / (127 * 254) + d2 / (127 * 254^2) + rho,
//   |d_t| <= 127,  |rho| <= 1 / (2 * 127 * 254^2)  (about 2^-23),
// d0 = rint(127 y) and d_{t+1} = rint(254 * residual): a residual of at most
// one half times 254 stays within [-127, 127], so every digit fits int8 (with
// base 256 a residual of +1/2 would need +128).  The products of digit pairs
// are exact in int32, summed per level l = t + u in its own accumulator:
//   L0 = d0.d0,  L1 = d0.d1 + d1.d0,  L2 = d0.d2 + d1.d1 + d2.d0,
// and (ij|kl) = 2^(e_ij + e_kl) / 127^2 * (L0 + (L1 + L2 / 254) / 254) in FP64.
// Level 3 and 4 products are dropped: at most 2 / 254^3 (about 2^-23) of
// 2^(e_ij + e_kl) per row, so the error is relative to the column scales, not
// to each element: small while the rows are of one magnitude (density-fitting
// rows), too large where a few rows dominate every sum.  The int32
// sums are exact while 3 * K * 127^2 < 2^31, i.e. for K <= I8_KMAX rows.  The
// operands move as the bf16 ones do: 16-byte chunks = 16 consecutive rows of
// one column of one digit plane, one MFMA fragment of v_mfma_i32_32x32x32_i8.
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));
constexpr int I8_KMAX = 44032;
constexpr int I8_EBAD = 1 << 20;   // exponent marking a column with a non-finite entry

// cmax[x] = max_r |Z[r][x]| as float bits (non-negative floats order as
// unsigned integers); a NaN or infinity raises it to at least 0x7f800000.
__global__ void k_colmax(const float* __restrict__ z, size_t ldz, int krows, int ncol, int rows_per,
                         unsigned* __restrict__ cmax) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ncol) return;
    const int r0 = blockIdx.y * rows_per, r1 = min(krows, r0 + rows_per);
    unsigned m = 0u;
    for (int r = r0; r < r1; ++r) {
        const float v = z[(size_t)r * ldz + x];
        const unsigned b = __float_as_uint(fabsf(v));
        m = max(m, isfinite(v) ? b : 0x7fc00000u);
    }
    atomicMax(cmax + x, m);
}

// Digit planes P[t][g][x][16] (int8) of Z[16 g + v][x] / 2^e_x, and ex[x] = e_x
// (I8_EBAD for a non-finite column).  Rows at or past krows are zero.
__global__ void k_pack_i8(const float* __restrict__ z, size_t ldz, int krows, int ncol, int kg16,
                          const unsigned* __restrict__ cmax, int* __restrict__ ex, i4v* __restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ncol) return;
    const unsigned cb = cmax[x];
    int e = 0;
    if (cb >= 0x7f800000u) e = I8_EBAD;
    else if (cb != 0u) frexpf(__uint_as_float(cb), &e);   // cmax = m 2^e, m in [0.5, 1): cmax < 2^e
    if (blockIdx.y == 0) ex[x] = e;
    const double sc = e == I8_EBAD ? 0.0 : ldexp(127.0, -e);
    const size_t plane = (size_t)kg16 * ncol;
    for (int g = blockIdx.y; g < kg16; g += gridDim.y) {   // the grid's y extent is capped at 65535
        union {
            signed char c[16];
            i4v v;
        } d[3];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int k = 16 * g + v;
            double r = k < krows ? (double)z[(size_t)k * ldz + x] * sc : 0.0;   // |r| < 127, exact
            const double d0 = rint(r);
            r = (r - d0) * 254.0;
            const double d1 = rint(r);
            r = (r - d1) * 254.0;
            const double d2 = rint(r);
            d[0].c[v] = (signed char)(int)d0;
            d[1].c[v] = (signed char)(int)d1;
            d[2].c[v] = (signed char)(int)d2;
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) out[(size_t)t * plane + (size_t)g * ncol + x] = d[t].v;
    }
}

// 128 x 256 output tiles, 8 waves as 2 x 4, wave tile 64 x 64 (2 x 2 blocks of
// 32 x 32), a 2-deep ring of 64-row stages (4 chunk groups of 16 rows; 72 KB
// per stage for three digit planes) moved by buffer loads straight into LDS,
// as in k_contract_w8; per 32-row k-step 24 MFMAs into three int32
// accumulator sets (levels 0, 1, 2).  No partial flush: the sums are exact.
// A launch sums the kgroups 16-row groups it is given (a chunk of at most
// I8_KMAX rows of planes holding kplane groups each); with accumulate the
// scaled chunk result is added to out (ACC), so longer Z runs chunk by chunk.
template <int MODE, bool ACC>
__global__ void __launch_bounds__(512) k_contract_i8(int npair, int kgroups, const i4v* __restrict__ pa,
                                                     const i4v* __restrict__ pb, const int* __restrict__ exa,
                                                     const int* __restrict__ exb, long nblocks,
                                                     double* __restrict__ out, int kplane) {
    constexpr int NS = 3, G = 4, NBUF = 2;
    constexpr int BM = 128, BN = 256;
    constexpr int TM = 2, TN = 2;
    constexpr int PA = G * BM, PB = G * BN;      // 16-byte chunks of one plane of A / B per stage
    constexpr int STAGE = NS * (PA + PB);
    constexpr int CA = PA / 8, NLB = PB / 512;
    constexpr int LOADS = NS * (1 + NLB);
    extern __shared__ __align__(16) i4v ring_i8[];
    int mt, nt;
    const long logical = xcd_logical(blockIdx.x, nblocks);
    const int ntm = (npair + BM - 1) / BM, ntn = (npair + BN - 1) / BN;
    if (!w8_tile_of<MODE>(logical, ntm, ntn, mt, nt)) return;
    const int m0 = mt * BM, n0 = nt * BN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm0 = (wave >> 2) * 64, wn0 = (wave & 3) * 64;
    const size_t plane = (size_t)kplane * npair;
    const int nkt = kgroups / G;
    const int fa = wave * CA;
    const unsigned offa = (unsigned)min(m0 + fa % BM + (lane & (CA - 1)), npair - 1) * 16u;
    unsigned offb[NLB];
    const char* rowa[NS];
    const char* rowb[NS][NLB];
#pragma unroll
    for (int h = 0; h < NLB; ++h) offb[h] = (unsigned)min(n0 + (h * 512 + wave * 64) % BN + lane, npair - 1) * 16u;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        rowa[t] = (const char*)pa + (t * plane + (size_t)(fa / BM) * npair) * 16;
#pragma unroll
        for (int h = 0; h < NLB; ++h)
            rowb[t][h] = (const char*)pb + (t * plane + (size_t)((h * 512 + wave * 64) / BN) * npair) * 16;
    }
    const size_t stage_bytes = (size_t)G * npair * 16;
    auto issue = [&](int kt) {
        i4v* st = ring_i8 + (size_t)(kt % NBUF) * STAGE;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (CA == 64 || lane < CA)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    __builtin_amdgcn_make_buffer_rsrc((void*)rowa[t], (short)0, npair * 16, DMET_RSRC_WORD3),
                    DMET_LDS_PTR(st + t * PA + fa), 16, (int)offa, 0, 0, 0);
            rowa[t] += stage_bytes;
#pragma unroll
            for (int h = 0; h < NLB; ++h) {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    __builtin_amdgcn_make_buffer_rsrc((void*)rowb[t][h], (short)0, npair * 16, DMET_RSRC_WORD3),
                    DMET_LDS_PTR(st + NS * PA + t * PB + h * 512 + wave * 64), 16, (int)offb[h], 0, 0, 0);
                rowb[t][h] += stage_bytes;
            }
        }
    };

    i16v acc0[TM][TN], acc1[TM][TN], acc2[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc0[i][j][r] = 0;
                acc1[i][j][r] = 0;
                acc2[i][j][r] = 0;
            }
    if (nkt > 0) issue(0);
    auto stage = [&](int kt, auto younger_c) {
        constexpr int YOUNGER = decltype(younger_c)::value;
        constexpr int VM = YOUNGER * LOADS;
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0F70 | (VM & 15) | ((VM >> 4) << 14));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (kt + NBUF - 1 < nkt) issue(kt + NBUF - 1);
        const i4v* sA = ring_i8 + (size_t)(kt % NBUF) * STAGE;
        const i4v* sB = sA + NS * PA;
        // two k-steps of 32 rows, software-pipelined as in k_contract_w8
        const int g0 = lane >> 5, g1 = 2 + (lane >> 5);
        auto rdA = [&](i4v (&r)[2], int t, int g) {
            r[0] = sA[t * PA + g * BM + wm0 + (lane & 31)];
            r[1] = sA[t * PA + g * BM + wm0 + 32 + (lane & 31)];
        };
        auto rdB = [&](i4v (&r)[2], int t, int g) {
            r[0] = sB[t * PB + g * BN + wn0 + (lane & 31)];
            r[1] = sB[t * PB + g * BN + wn0 + 32 + (lane & 31)];
        };
        auto mm = [&](i16v (&acc)[TM][TN], const i4v (&a)[2], const i4v (&b)[2]) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        };
        i4v a2[2], a1[2], a0[2], b0[2], b1[2], b2[2];
        i4v c2[2], c1[2], c0[2], d0[2], d1[2], d2[2];
        rdA(a2, 2, g0); rdB(b0, 0, g0);
        DMET_SECTION(4, 0);
        rdA(a1, 1, g0); rdB(b1, 1, g0);
        DMET_SECTION(4, 0);
        mm(acc2, a2, b0);
        DMET_SECTION(0, 4);
        rdA(a0, 0, g0); rdB(b2, 2, g0);
        mm(acc2, a1, b1);
        mm(acc1, a1, b0);
        DMET_SECTION(4, 8);
        rdA(c2, 2, g1);
        mm(acc2, a0, b2);
        DMET_SECTION(2, 4);
        rdB(d0, 0, g1);
        mm(acc1, a0, b1);
        DMET_SECTION(2, 4);
        rdA(c1, 1, g1);
        mm(acc0, a0, b0);
        DMET_SECTION(2, 4);
        rdB(d1, 1, g1); rdA(c0, 0, g1);
        DMET_SECTION(4, 0);
        mm(acc2, c2, d0);
        DMET_SECTION(0, 4);
        rdB(d2, 2, g1);
        mm(acc2, c1, d1);
        mm(acc1, c1, d0);
        DMET_SECTION(2, 8);
        mm(acc2, c0, d2);
        mm(acc1, c0, d1);
        mm(acc0, c0, d0);
        DMET_SECTION(0, 12);
    };
    __builtin_amdgcn_s_waitcnt(0xC07F);
    int kt = 0;
    for (; kt + NBUF - 2 < nkt; ++kt) stage(kt, std::integral_constant<int, NBUF - 2>{});
    for (; kt < nkt; ++kt) stage(kt, std::integral_constant<int, 0>{});
    constexpr double inv_b = 1.0 / 254.0, inv_b0sq = 1.0 / (127.0 * 127.0);
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int KL = n0 + wn0 + j * 32 + (lane & 31);
        const int eb = exb[min(KL, npair - 1)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int IJ = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (IJ >= npair || KL >= npair) continue;
                if (MODE == 0 && KL > IJ) continue;
                const int ea = exa[IJ];
                double v = (double)acc0[i][j][r] + ((double)acc1[i][j][r] + (double)acc2[i][j][r] * inv_b) * inv_b;
                v = (ea == I8_EBAD || eb == I8_EBAD) ? __builtin_nan("") : ldexp(v * inv_b0sq, ea + eb);
                double& o = MODE == 0 ? out[(size_t)IJ * (IJ + 1) / 2 + KL] : out[(size_t)IJ * npair + KL];
                if constexpr (ACC) o += v;
                else o = v;
            }
    }
}

constexpr size_t i8_lds() { return (size_t)2 * 3 * 4 * (128 + 256) * 16; }

// ------------------------------------------------------------------ packed transform (bf16 forms)
// Operand packing for the transform.  Every packed operand has the layout
//   [plane][part][group][x][8]   (bf16; group = 8 consecutive contraction indices)
// with planes (re, im) for the 4M products.  nao is padded to
// nao_p = 8 * ceil(nao / 8) (zero rows / columns) and the group count of each
// contraction index is padded to an even number (a zero group) so that a
// stage always holds two groups (16 contraction indices).

inline size_t pack_lds_bytes(int mb, int ngv) { return (size_t)mb * (8 * ngv + 1) * sizeof(float2); }

// Both transform stages multiply complex operands with four real products
// (4M) on two planes (re, im) per operand: every packed transform operand has
// P2 planes.
constexpr int P2 = 2;

// lmunu[q][k][L][mu][nu] -> P1[q][k][plane][part][nu/8][L*nao_p + mu][8]
// With only_needed, blocks (q, k) that the k <-> q-k paired transform never
// reads are skipped (their input is not touched).  One workgroup takes `mb`
// rows mu of one (q, k, L): the rows are one contiguous run of the input, read
// with consecutive lanes on consecutive elements, and staged as float pairs in
// LDS (8 ngv columns, row stride 8 ngv + 1); each thread then packs one
// 8-column chunk of one row.  Padding rows (up to nao_p) and columns (up to
// 8 ngv) are written as zeros.
inline int pack_rows_per_block(int ngv) {
    int mb = 32;
    while (mb > 1 && pack_lds_bytes(mb, ngv) > 48 * 1024) mb /= 2;
    return mb;
}

template <int NS, class TIn>
__global__ void __launch_bounds__(256) k_pack_lmunu(const TIn* __restrict__ lm, int nao, int nao_p, int naux,
                                                    int ngv, int mb, __bf16* __restrict__ out, Mesh mesh,
                                                    int only_needed) {
    extern __shared__ float2 tile[];   // [mb][8 ngv + 1]
    const int W = 8 * ngv, ld = W + 1;
    const int nmb = (nao_p + mb - 1) / mb;
    const long b = blockIdx.x;
    const int blk = (int)(b % nmb), L = (int)((b / nmb) % naux), qk = (int)(b / ((long)nmb * naux));
    if (only_needed && !kpair_needed(mesh, qk / mesh.nk, qk % mesh.nk)) return;
    const int mu0 = blk * mb;
    const int rows = min(mb, nao_p - mu0);          // rows of this block (padding rows included)
    const int live = max(0, min(rows, nao - mu0));  // rows that exist in the input
    const TIn* src = lm + (((size_t)qk * naux + L) * nao + mu0) * (size_t)nao * 2;
    // rows mu0 .. mu0+live-1 are contiguous in the input: live * nao complex
    // PU elements per thread are loaded (clamped, unconditional) before any is
    // stored, so that several loads per thread are in flight
    constexpr int PU = 8;
    const int nel = live * nao;
    for (int e0 = threadIdx.x; e0 < nel; e0 += PU * blockDim.x) {
        float2 v[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int e = min(e0 + u * (int)blockDim.x, nel - 1);
            if constexpr (sizeof(TIn) == 8) {
                const double2 d = reinterpret_cast<const double2*>(src)[e];
                v[u] = make_float2((float)d.x, (float)d.y);
            } else {
                v[u] = reinterpret_cast<const float2*>(src)[e];
            }
        }
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int e = e0 + u * (int)blockDim.x;
            if (e < nel) tile[(e / nao) * ld + e % nao] = v[u];
        }
    }
    // zero padding columns of every row, and the padding rows
    for (int e = threadIdx.x; e < rows * (W - nao); e += blockDim.x) {
        const int r = e / (W - nao), c = nao + e % (W - nao);
        tile[r * ld + c] = make_float2(0.f, 0.f);
    }
    for (int e = threadIdx.x; e < (rows - live) * nao; e += blockDim.x) {
        const int r = live + e / nao, c = e % nao;
        tile[r * ld + c] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int M1 = naux * nao_p;
    const size_t pt_stride = (size_t)ngv * M1;
    __bf16* o = out + (size_t)qk * P2 * NS * pt_stride * 8;
    for (int item = threadIdx.x; item < rows * ngv; item += blockDim.x) {
        const int r = item % rows, g = item / rows;   // consecutive threads: consecutive rows
        bf8 part[P2][NS];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const float2 x = tile[r * ld + 8 * g + v];
            const float pl[P2] = {x.x, x.y};
#pragma unroll
            for (int p = 0; p < P2; ++p) {
                __bf16 sp[NS];
                split_bf16<NS>(pl[p], sp);
#pragma unroll
                for (int t = 0; t < NS; ++t) part[p][t][v] = sp[t];
            }
        }
        const size_t row = (size_t)L * nao_p + mu0 + r;
#pragma unroll
        for (int p = 0; p < P2; ++p)
#pragma unroll
            for (int t = 0; t < NS; ++t)
                *reinterpret_cast<bf8*>(o + (((size_t)(p * NS + t) * ngv + g) * M1 + row) * 8) = part[p][t];
    }
}

// C^k[s][k][nu][j] -> P1c[k][plane][part][nu/8][s*neo + j][8]   (planes Cr, Ci)
template <int NS>
__global__ void k_pack_c1(const double* __restrict__ ck, int nk, int nspin, int nao, int neo, int ngv,
                          __bf16* __restrict__ out, int col0, int nb_total) {
    const int nb = nspin * neo;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y, k = blockIdx.z;
    if (col >= nb) return;
    const int s = col / neo, j = col % neo;
    bf8 part[P2][NS];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int nu = 8 * g + v;
        float re = 0.f, im = 0.f;
        if (nu < nao) {
            const double* c = ck + ((((size_t)s * nk + k) * nao + nu) * neo + j) * 2;
            re = (float)c[0];
            im = (float)c[1];
        }
        const float pl[P2] = {re, im};
#pragma unroll
        for (int p = 0; p < P2; ++p) {
            __bf16 sp[NS];
            split_bf16<NS>(pl[p], sp);
#pragma unroll
            for (int t = 0; t < NS; ++t) part[p][t][v] = sp[t];
        }
    }
    const size_t per_k = (size_t)P2 * NS * ngv * nb_total;
#pragma unroll
    for (int p = 0; p < P2; ++p)
#pragma unroll
        for (int t = 0; t < NS; ++t)
            *reinterpret_cast<bf8*>(
                out + ((size_t)k * per_k + ((size_t)(p * NS + t) * ngv + g) * nb_total + col0 + col) * 8) = part[p][t];
}

// conj(C^k)[s][(k,mu)][i] -> P2c[s][plane][part][(k*nao_p + mu)/8][i][8]  (planes Cr, -Ci)
template <int NS>
__global__ void k_pack_c2(const double* __restrict__ ck, int nk, int nao, int nao_p, int neo, int ng2,
                          __bf16* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y, s = blockIdx.z;
    if (i >= neo) return;
    bf8 part[P2][NS];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int kk = 8 * g + v, k = kk / nao_p, mu = kk % nao_p;
        float re = 0.f, im = 0.f;
        if (k < nk && mu < nao) {
            const double* c = ck + ((((size_t)s * nk + k) * nao + mu) * neo + i) * 2;
            re = (float)c[0];
            im = (float)c[1];
        }
        const float pl[P2] = {re, -im};
#pragma unroll
        for (int p = 0; p < P2; ++p) {
            __bf16 sp[NS];
            split_bf16<NS>(pl[p], sp);
#pragma unroll
            for (int t = 0; t < NS; ++t) part[p][t][v] = sp[t];
        }
    }
    const size_t per_s = (size_t)P2 * NS * ng2 * neo;
#pragma unroll
    for (int p = 0; p < P2; ++p)
#pragma unroll
        for (int t = 0; t < NS; ++t)
            *reinterpret_cast<bf8*>(out + ((size_t)s * per_s + ((size_t)(p * NS + t) * ng2 + g) * neo + i) * 8) =
                part[p][t];
}

// One stage of a stage-2 operand (P2 planes x NS parts x 2 groups x ROWS rows)
// from two explicit groups g0, g1 (a zero group pads an odd count).
template <int NS, int ROWS>
__device__ inline void pk_issue_g(const __bf16* base, size_t pt_stride, int X, int x0, int g0, int g1, bf8* dst) {
    constexpr int CH = P2 * NS * 2 * ROWS;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int first = wave * 64; first < CH; first += 256) {
        const int pt = first / (2 * ROWS), g = (first / ROWS) % 2, row0 = first % ROWS;
        const int x = min(x0 + row0 + lane, X - 1);
        const __bf16* src = base + ((size_t)pt * pt_stride + (size_t)(g ? g1 : g0) * X + x) * 8;
        __builtin_amdgcn_global_load_lds((const void*)src, DMET_LDS_PTR(dst + first), 16, 0, 0);
    }
}

// One stage of a packed operand (P2 planes x NS parts x 2 groups x ROWS rows)
// moved to LDS [plane*NS + part][group][row] by direct loads of NW waves; rows
// clamped.
template <int NS, int ROWS, int NW = 4>
__device__ inline void pk_issue(const __bf16* base, size_t pt_stride /*chunks per part*/, int X, int x0, int g0,
                                bf8* dst) {
    constexpr int CH = P2 * NS * 2 * ROWS;  // chunks in the stage
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int first = wave * 64; first < CH; first += 64 * NW) {
        const int pt = first / (2 * ROWS), g = (first / ROWS) % 2, row0 = first % ROWS;
        const int x = min(x0 + row0 + lane, X - 1);
        const __bf16* src = base + ((size_t)pt * pt_stride + (size_t)(g0 + g) * X + x) * 8;
        __builtin_amdgcn_global_load_lds((const void*)src, DMET_LDS_PTR(dst + first), 16, 0, 0);
    }
}

// Negated bf16 fragment: the sign bit of each of the eight values flipped (exact).
__device__ inline bf8 neg_bf8(bf8 x) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 u = __builtin_bit_cast(u4, x);
    u ^= 0x80008000u;
    return __builtin_bit_cast(bf8, u);
}

// 4M x NS-split products of one 16-deep stage on (re, im) planes, two
// accumulators per output: acc[0] += Ar Br + (-Ai) Bi (the real part),
// acc[1] += Ar Bi + Ai Br (the imaginary part), the negation applied to the
// staged Ai fragment.  Each real product's split products run smallest first:
// lo*hi terms, then mid*mid and hi*lo, ..., hi*hi; the four real products in
// the order Ar Br, Ai Bi, Ar Bi, Ai Br.
// The operand fragments of one 16-deep stage for a wave's TM x TN blocks.
template <int NS, int TM, int TN>
struct PkFrags {
    bf8 a[P2][TM][NS], b[P2][TN][NS];
};

template <int NS, int BM, int BN, int TM, int TN>
__device__ inline void pk_read(const bf8* sA, const bf8* sB, int wm0, int wn0, PkFrags<NS, TM, TN>& f) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 5;
#pragma unroll
    for (int p = 0; p < P2; ++p)
#pragma unroll
        for (int t = 0; t < NS; ++t) {
#pragma unroll
            for (int i = 0; i < TM; ++i) f.a[p][i][t] = sA[((p * NS + t) * 2 + g) * BM + wm0 + i * 32 + (lane & 31)];
#pragma unroll
            for (int j = 0; j < TN; ++j) f.b[p][j][t] = sB[((p * NS + t) * 2 + g) * BN + wn0 + j * 32 + (lane & 31)];
        }
}

template <int NS, int TM, int TN>
__device__ inline void pk_mma_f(const PkFrags<NS, TM, TN>& f, f16v (&acc)[2][TM][TN]) {
    if constexpr (TM == 1 && TN == 1) {
        // every LDS read of the stage first, then the MFMAs
        __builtin_amdgcn_sched_group_barrier(0x100, P2 * NS * (TM + TN), 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * TM * TN * (NS == 3 ? 6 : 3), 0);
    }
    constexpr int PA[4] = {0, 1, 0, 1}, PB[4] = {0, 1, 1, 0}, DST[4] = {0, 0, 1, 1};
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                bf8 x[NS];
#pragma unroll
                for (int t = 0; t < NS; ++t) x[t] = c == 1 ? neg_bf8(f.a[1][i][t]) : f.a[PA[c]][i][t];
                const bf8* y = f.b[PB[c]][j];
                f16v d = acc[DST[c]][i][j];
                if constexpr (NS == 2) {
                    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[0], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[1], d, 0, 0, 0);
                } else {
                    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[2], y[0], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[1], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[2], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[0], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[1], d, 0, 0, 0);
                }
                d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[0], d, 0, 0, 0);
                acc[DST[c]][i][j] = d;
            }
}

template <int NS, int BM, int BN, int TM, int TN>
__device__ inline void pk_mma4(const bf8* sA, const bf8* sB, int wm0, int wn0, f16v (&acc)[2][TM][TN]) {
    PkFrags<NS, TM, TN> f;
    pk_read<NS, BM, BN, TM, TN>(sA, sB, wm0, wn0, f);
    pk_mma_f<NS, TM, TN>(f, acc);
}

// Double-buffered K loop over `nst` stages of two groups each (NW waves).
template <int NS, int BM, int BN, int TM, int TN, int NW = 4>
__device__ inline void pk_loop3(const __bf16* pa, size_t pa_pt, int XA, int m0, const __bf16* pb, size_t pb_pt,
                                int XB, int n0, int nst, bf8* ring, int wm0, int wn0, f16v (&acc)[2][TM][TN]) {
    constexpr int SA = P2 * NS * 2 * BM, SB = P2 * NS * 2 * BN;
    pk_issue<NS, BM, NW>(pa, pa_pt, XA, m0, 0, ring);
    pk_issue<NS, BN, NW>(pb, pb_pt, XB, n0, 0, ring + SA);
    for (int st = 0; st < nst; ++st) {
        bf8* cur = ring + (size_t)(st & 1) * (SA + SB);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // own loads of stage st landed
        __builtin_amdgcn_s_barrier();         // everyone's loads landed; stage st-1 fully read
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) {
            bf8* nxt = ring + (size_t)((st + 1) & 1) * (SA + SB);
            pk_issue<NS, BM, NW>(pa, pa_pt, XA, m0, 2 * (st + 1), nxt);
            pk_issue<NS, BN, NW>(pb, pb_pt, XB, n0, 2 * (st + 1), nxt + SA);
        }
        pk_mma4<NS, BM, BN, TM, TN>(cur, cur + SA, wm0, wn0, acc);
    }
}

// Stage order of stage 2's two sums over the k groups: pass 0 walks the n1
// groups of every kept slot, pass 1 the n2 groups of the paired slots (the
// first n2 of pass 0's), two groups per stage, a zero group zg padding an odd
// count.  Stages alternate between the passes while pass 1 has stages left, so
// the workgroups of one fitting function read T for their i and for their j
// columns at nearly the same time and T comes from HBM once per launch, not
// once per pass.  Every stage-2 kernel walks this one order, so they give the
// same bits for the same element.
struct PairedWalk {
    struct Cur {
        int j, slot, gl;
    };
    int n1, n2, gpk, zg, s2, ist;
    Cur c0, c1;
    __device__ PairedWalk(int n1_, int n2_, int gpk_, int zg_)
        : n1(n1_), n2(n2_), gpk(gpk_), zg(zg_), s2((n2_ + 1) / 2), ist(0), c0{0, 0, 0}, c1{0, 0, 0} {}
    __device__ int stages() const { return (n1 + 1) / 2 + s2; }
    __device__ int pass_of(int st) const { return st < 2 * s2 ? (st & 1) : 0; }
    template <class KOf>
    __device__ void take(Cur& c, int n, KOf kof, int& gc, int& gt) {
        if (c.j < n) {
            gc = kof(c.slot) * gpk + c.gl;
            gt = c.j;
            ++c.j;
            if (++c.gl == gpk) {
                c.gl = 0;
                ++c.slot;
            }
        } else {
            gc = gt = zg;
        }
    }
    // the next stage in order: its pass, and its two groups of conj C and of T
    template <class KOf>
    __device__ int next(KOf kof, int& gc0, int& gt0, int& gc1, int& gt1) {
        const int p = pass_of(ist++);
        if (p) {
            take(c1, n2, kof, gc0, gt0);
            take(c1, n2, kof, gc1, gt1);
        } else {
            take(c0, n1, kof, gc0, gt0);
            take(c0, n1, kof, gc1, gt1);
        }
        return p;
    }
};

// K loop of stage 2 under the k <-> q-k pairing: pass 0 over the groups of
// all kept k (A = conj C, rows i; B = T, columns (L, j)), pass 1 over the
// paired k with the operands swapped (A = T columns (L, i), B = conj C rows j),
// which adds the transposed terms of the partners; stages in PairedWalk order.
// The 4M products on the (re, im) planes give the plain complex product of the
// two operands in both passes.  Double-buffered stages of two groups.
template <int NS, int BM, int BN, int TM, int TN, class KOf>
__device__ inline void pk_loop_paired(const __bf16* pc2, size_t cst, int neo, const __bf16* ptt, size_t tst, int N2,
                                      int L, int m0, int j0, int gpk, int zg, int npaired, int nself, KOf kof,
                                      bf8* ring, int wm0, int wn0, f16v (&acc)[2][TM][TN]) {
    constexpr int SA = P2 * NS * 2 * BM, SB = P2 * NS * 2 * BN;
    PairedWalk walk((npaired + nself) * gpk, npaired * gpk, gpk, zg);
    const int nst = walk.stages();
    auto issue = [&](bf8* dst) {
        int gc0, gt0, gc1, gt1;
        const int pass = walk.next(kof, gc0, gt0, gc1, gt1);
        if (!pass) {
            pk_issue_g<NS, BM>(pc2, cst, neo, m0, gc0, gc1, dst);
            pk_issue_g<NS, BN>(ptt, tst, N2, L * neo + j0, gt0, gt1, dst + SA);
        } else {
            pk_issue_g<NS, BM>(ptt, tst, N2, L * neo + m0, gt0, gt1, dst);
            pk_issue_g<NS, BN>(pc2, cst, neo, j0, gc0, gc1, dst + SA);
        }
    };
    issue(ring);
    for (int st = 0; st < nst; ++st) {
        bf8* cur = ring + (size_t)(st & 1) * (SA + SB);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // own loads of stage st landed
        __builtin_amdgcn_s_barrier();         // everyone's loads landed; stage st-1 fully read
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) issue(ring + (size_t)((st + 1) & 1) * (SA + SB));
        pk_mma4<NS, BM, BN, TM, TN>(cur, cur + SA, wm0, wn0, acc);
    }
}

// Stage 1 (both spins at once): T[(L,mu)][(s,j)] for one (q, k) from packed
// lmunu and packed C^{k-q}; 4M products combined into (re, im) and split into
// bf16 parts in the epilogue, written as stage 2's packed B operand
//   PT[s][plane][part][(k*nao_p + mu)/8][L*neo + j][8].
// Lanes l and l+32 hold rows 0-3 and 4-7 of each 8-row group of a 32x32
// result tile; one exchange gives each lane a full 8-row column chunk.
// Only the kept k of the k <-> q-k pairing are formed; T slot `slot` (groups
// slot * nao_p / 8 ...) holds k = ks.k[slot].  NW = 8 runs the 128 x 128
// tile as eight 64 x 32 waves (two per SIMD) instead of four 64 x 64.
template <int NS, int NW>
__global__ void __launch_bounds__(64 * NW) k_xf1_pk(Mesh mesh, int q, int naux, int nao_p, int neo, int nspin,
                                                    int ngv, int ng2, KSlots ks,
                                                    const __bf16* __restrict__ plm, const __bf16* __restrict__ pc1,
                                                    __bf16* __restrict__ pt) {
    static_assert(NW == 4 || NW == 8, "four waves of 64 x 64 or eight of 64 x 32");
    constexpr int BM = 128, BN = 128, TM = 2, TN = NW == 4 ? 2 : 1;
    extern __shared__ __align__(16) bf8 ring[];
    const int nk = mesh.nk;
    const int M1 = naux * nao_p, NB = nspin * neo;
    // workgroup -> (slot, m tile, n tile), n fastest, each XCD a contiguous run:
    // the n tiles of one m tile share the lmunu panel in that XCD's L2
    const int nmt = (M1 + BM - 1) / BM, nnt = (NB + BN - 1) / BN;
    const long logical = xcd_logical(blockIdx.x, gridDim.x);
    const long nt_all = (long)(ks.npaired + ks.nself) * nmt * nnt;
    if (logical >= nt_all) return;
    const int slot = (int)(logical / ((long)nmt * nnt));
    const int k = ks.k[slot];
    const int rem = (int)(logical % ((long)nmt * nnt));
    const int m0 = (rem / nnt) * BM, n0 = (rem % nnt) * BN;
    const int kmq = mesh_sub(mesh, k, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = NW == 4 ? (wave >> 1) * 64 : (wave >> 2) * 64;
    const int wn0 = NW == 4 ? (wave & 1) * 64 : (wave & 3) * 32;
    const __bf16* pa = plm + ((size_t)q * nk + k) * P2 * NS * (size_t)ngv * M1 * 8;
    const __bf16* pb = pc1 + (size_t)kmq * P2 * NS * (size_t)ngv * NB * 8;
    f16v acc[2][TM][TN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[p][i][j][r] = 0.f;
    pk_loop3<NS, BM, BN, TM, TN, NW>(pa, (size_t)ngv * M1, M1, m0, pb, (size_t)ngv * NB, NB, n0, ngv / 2, ring, wm0,
                                 wn0, acc);
    const int h = lane >> 5;
    const size_t N2 = (size_t)naux * neo;
    const size_t per_part = (size_t)ng2 * N2;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int col = n0 + wn0 + j * 32 + (lane & 31);
            const int s = col / neo, jj = col % neo;
#pragma unroll
            for (int qq = 0; qq < 4; qq += 2) {
                // rows of register groups qq (this lane: h == 0) and qq + 1 (h == 1)
                float pl[P2][8];
#pragma unroll
                for (int p3 = 0; p3 < P2; ++p3) {
                    float mine[4], send[4], recv[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        // 4M: re = Ar Br - Ai Bi, im = Ar Bi + Ai Br
                        const int ra = 4 * qq + r, rb = 4 * (qq + 1) + r;
                        const float va = acc[p3][i][j][ra];
                        const float vb = acc[p3][i][j][rb];
                        mine[r] = h == 0 ? va : vb;
                        send[r] = h == 0 ? vb : va;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) recv[r] = __shfl_xor(send[r], 32, 64);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        pl[p3][h == 0 ? r : 4 + r] = mine[r];
                        pl[p3][h == 0 ? 4 + r : r] = recv[r];
                    }
                }
                const int grp_row = m0 + wm0 + i * 32 + 8 * (qq + h);   // first row of this lane's 8-row group
                if (col < NB && grp_row < M1) {
                    const int L = grp_row / nao_p, mu0 = grp_row % nao_p;
                    const size_t g2 = ((size_t)slot * nao_p + mu0) / 8;
                    const size_t x = (size_t)L * neo + jj;
                    __bf16* base = pt + (size_t)s * P2 * NS * per_part * 8;
#pragma unroll
                    for (int p3 = 0; p3 < P2; ++p3) {
                        bf8 part[NS];
#pragma unroll
                        for (int v = 0; v < 8; ++v) {
                            __bf16 sp[NS];
                            split_bf16<NS>(pl[p3][v], sp);
#pragma unroll
                            for (int t = 0; t < NS; ++t) part[t][v] = sp[t];
                        }
#pragma unroll
                        for (int t = 0; t < NS; ++t)
                            *reinterpret_cast<bf8*>(base + (((size_t)(p3 * NS + t) * ng2 + g2) * N2 + x) * 8) = part[t];
                    }
                }
            }
        }
}

// Stage 2 for one q and spin, i >= j only; 4M products; Z rows (FP32):
//   X[i][(L,j)] = sum_{kept k, mu} conj(C^k_{mu i}) T_k[mu][(L,j)]
//               + sum_{paired k, mu} T_k[mu][(L,i)] conj(C^k_{mu j}),
// the second sum being the transposed terms of the partners q-k (a symmetric
// rank-2k update).  Tiles of 64 x 64 per L; tiles with every i < every j are
// skipped.  Group zg is a zero group of both operands (pads odd counts).

// One stage of a stage-2 operand region of ROWS rows made of ROWS / 64
// segments of 64 rows starting at x00 and x01 (rows clamped to X - 1),
// laid out [plane*NS + part][group][ROWS] as pk_mma4 reads it; NW waves share
// the loads.
template <int NS, int ROWS, int NW>
__device__ inline void pk_issue_seg(const __bf16* base, size_t pt_stride, int X, int x00, int x01, int g0, int g1,
                                    bf8* dst) {
    static_assert(ROWS == 64 || ROWS == 128, "one or two segments");
    constexpr int CH = P2 * NS * 2 * ROWS;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int first = wave * 64; first < CH; first += 64 * NW) {
        const int pt = first / (2 * ROWS), g = (first / ROWS) % 2, row0 = first % ROWS;
        const int x = min((row0 >= 64 ? x01 : x00) + (row0 & 63) + lane, X - 1);
        const __bf16* src = base + ((size_t)pt * pt_stride + (size_t)(g ? g1 : g0) * X + x) * 8;
        __builtin_amdgcn_global_load_lds((const void*)src, DMET_LDS_PTR(dst + first), 16, 0, 0);
    }
}

// Stage 2 for one q and spin on two fitting functions per workgroup: the 64 x 64
// tile (i, j) of X_L for L = L0 and L0 + 1, eight waves with a 32 x 32 sub-tile
// each (wave w: L0 + w / 4, rows 32 ((w / 2) % 2), columns 32 (w % 2)).  The conj C
// rows of a stage serve both fitting functions, so a stage stages 192 rows for
// 192 MFMAs (128 rows for 96 with one fitting function), and two workgroups fit
// a CU (four waves per SIMD).  Stages in PairedWalk order with the products of
// pk_mma4 per element: the same bits as the batched kernel k_xf2_batched.
template <int NS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4))) k_xf2_pk2(int naux, int neo, int ng2, int gpk, int zg, KSlots ks,
                                                 int self_conj, size_t zrow0, float wq,
                                                 const __bf16* __restrict__ pc2, const __bf16* __restrict__ ptt,
                                                 float* __restrict__ z, size_t ldz) {
    constexpr int RC = 64, RT = 128;                  // conj C rows and T columns (two L) per stage
    constexpr int SC = P2 * NS * 2 * RC, ST = P2 * NS * 2 * RT;
    extern __shared__ __align__(16) bf8 ring[];
    const int nt = (neo + 63) / 64;
    const long tid_ = xcd_logical(blockIdx.x, gridDim.x);
    const int per_l = nt * nt;
    const int LP = (int)(tid_ / per_l), rem = (int)(tid_ % per_l);
    const int jt = rem / nt, it = rem % nt;
    const int L0 = 2 * LP;
    if (L0 >= naux) return;
    const int m0 = it * 64, j0 = jt * 64;
    if (m0 + 63 < j0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lw = wave >> 2, si = (wave >> 1) & 1, sj = wave & 1;
    const int L1 = min(L0 + 1, naux - 1);              // odd naux: the second half is computed, not stored
    const int N2 = naux * neo;
    __shared__ short ksh[KP_MAX];
    for (int t = threadIdx.x; t < ks.npaired + ks.nself; t += blockDim.x) ksh[t] = ks.k[t];
    __syncthreads();
    f16v acc[2][1][1];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[p][0][0][r] = 0.f;
    const size_t cst = (size_t)ng2 * neo, tst = (size_t)ng2 * N2;
    PairedWalk walk((ks.npaired + ks.nself) * gpk, ks.npaired * gpk, gpk, zg);
    const int nst = walk.stages();
    auto kof = [&](int sl) { return (int)ksh[sl]; };
    auto issue = [&](bf8* dst) {
        int gc0, gt0, gc1, gt1;
        if (!walk.next(kof, gc0, gt0, gc1, gt1)) {   // A = conj C rows i, B = T columns (L, j)
            pk_issue_seg<NS, RC, 8>(pc2, cst, neo, m0, m0, gc0, gc1, dst);
            pk_issue_seg<NS, RT, 8>(ptt, tst, N2, L0 * neo + j0, L1 * neo + j0, gt0, gt1, dst + SC);
        } else {                                      // A = T columns (L, i), B = conj C rows j
            pk_issue_seg<NS, RT, 8>(ptt, tst, N2, L0 * neo + m0, L1 * neo + m0, gt0, gt1, dst);
            pk_issue_seg<NS, RC, 8>(pc2, cst, neo, j0, j0, gc0, gc1, dst + ST);
        }
    };
    issue(ring);
    for (int st = 0; st < nst; ++st) {
        bf8* cur = ring + (size_t)(st & 1) * (SC + ST);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // own loads of stage st landed
        __builtin_amdgcn_s_barrier();         // everyone's loads landed; stage st-1 fully read
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) issue(ring + (size_t)((st + 1) & 1) * (SC + ST));
        if (!walk.pass_of(st)) pk_mma4<NS, RC, RT, 1, 1>(cur, cur + SC, 32 * si, 64 * lw + 32 * sj, acc);
        else pk_mma4<NS, RT, RC, 1, 1>(cur, cur + ST, 64 * lw + 32 * si, 32 * sj, acc);
    }
    const int L = L0 + lw;
    if (L >= naux) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = m0 + 32 * si + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = j0 + 32 * sj + (lane & 31);
        if (i >= neo || j >= neo || j > i) continue;
        const size_t pair = (size_t)i * (i + 1) / 2 + j;
        const float xr = acc[0][0][0][r], xi = acc[1][0][0][r];
        if (self_conj) {
            z[(zrow0 + L) * ldz + pair] = wq * xr;
        } else {
            z[(zrow0 + 2 * (size_t)L) * ldz + pair] = wq * xr;
            z[(zrow0 + 2 * (size_t)L + 1) * ldz + pair] = wq * xi;
        }
    }
}

template <int NS>
constexpr size_t xf2_pk2_lds() { return (size_t)2 * P2 * NS * 2 * (64 + 128) * 16; }

// ------------------------------------------------------------------ batched pipeline
// Per-fragment data read by the batched kernels.
struct BFrag {
    const __bf16* pc2;   // packed conj(C) [plane][part][ng2][neo][8]
    __bf16* ptt;         // packed T of the current q [plane][part][ng2][naux*neo][8]
    float* z;            // Z rows [zrows][npair]
    const __bf16* zp;    // packed parts of Z [part][kgroups][npair][8]
    double* eri;         // s8 output
    int neo, naux, ng2, npair, zrows, kgroups;
    const i4v* zp8;      // int8 digit planes of Z [digit][kg16][npair] (int8 contraction)
    unsigned* cmax;      // column max of Z (float bits)
    int* ex;             // column exponents
    int kg16;            // 16-row groups of the digit planes
};

// Per (round, fragment) q-block of the stage-2 items, with the kept k of the
// k <-> q-k pairing (k[slot]) and the group layout of T.
struct BQ {
    int self_conj;
    int npaired, nself, gpk, zg;
    size_t zrow0;
    float wq;
    short k[KP_MAX];
};

// Stage-2 work item: fragment slot, fitting function, j tile, i tile.
struct BItem2 {
    int slot, L, jt, it;
};

// Contraction work item: fragment slot and output tile (mt >= nt).
struct BItemC {
    int slot, mt, nt, pad;
};

// Stage 1 of a group of fragments sharing one 3-index tensor: columns of the
// concatenated C^{k-q} are routed to their fragment by `colmap` (slot, j).
template <int NS, int NW>
__global__ void __launch_bounds__(64 * NW) k_xf1_batched(Mesh mesh, int q, int naux, int nao_p, int nbtot, int ngv,
                                                     KSlots ks, const int2* __restrict__ colmap,
                                                     const BFrag* __restrict__ frags,
                                                     const __bf16* __restrict__ plm, const __bf16* __restrict__ pc1) {
    constexpr int BM = 128, BN = 128, TM = 2, TN = NW == 4 ? 2 : 1;
    extern __shared__ __align__(16) bf8 ring[];
    const int nk = mesh.nk;
    const int M1 = naux * nao_p, NB = nbtot;
    const int nmt = (M1 + BM - 1) / BM, nnt = (NB + BN - 1) / BN;
    const long logical = xcd_logical(blockIdx.x, gridDim.x);
    if (logical >= (long)(ks.npaired + ks.nself) * nmt * nnt) return;
    const int slot = (int)(logical / ((long)nmt * nnt));
    const int k = ks.k[slot];
    const int rem = (int)(logical % ((long)nmt * nnt));
    const int m0 = (rem / nnt) * BM, n0 = (rem % nnt) * BN;
    const int kmq = mesh_sub(mesh, k, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = NW == 4 ? (wave >> 1) * 64 : (wave >> 2) * 64;
    const int wn0 = NW == 4 ? (wave & 1) * 64 : (wave & 3) * 32;
    const __bf16* pa = plm + ((size_t)q * nk + k) * P2 * NS * (size_t)ngv * M1 * 8;
    const __bf16* pb = pc1 + (size_t)kmq * P2 * NS * (size_t)ngv * NB * 8;
    f16v acc[2][TM][TN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[p][i][j][r] = 0.f;
    pk_loop3<NS, BM, BN, TM, TN, NW>(pa, (size_t)ngv * M1, M1, m0, pb, (size_t)ngv * NB, NB, n0, ngv / 2, ring, wm0,
                                 wn0, acc);
    const int h = lane >> 5;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int col = n0 + wn0 + j * 32 + (lane & 31);
            int2 cm = make_int2(-1, 0);
            if (col < NB) cm = colmap[col];
#pragma unroll
            for (int qq = 0; qq < 4; qq += 2) {
                float pl[P2][8];
#pragma unroll
                for (int p3 = 0; p3 < P2; ++p3) {
                    float mine[4], send[4], recv[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        // 4M: re = Ar Br - Ai Bi, im = Ar Bi + Ai Br
                        const int ra = 4 * qq + r, rb = 4 * (qq + 1) + r;
                        const float va = acc[p3][i][j][ra];
                        const float vb = acc[p3][i][j][rb];
                        mine[r] = h == 0 ? va : vb;
                        send[r] = h == 0 ? vb : va;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) recv[r] = __shfl_xor(send[r], 32, 64);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        pl[p3][h == 0 ? r : 4 + r] = mine[r];
                        pl[p3][h == 0 ? 4 + r : r] = recv[r];
                    }
                }
                const int grp_row = m0 + wm0 + i * 32 + 8 * (qq + h);
                if (cm.x >= 0 && grp_row < M1) {
                    const BFrag fr = frags[cm.x];
                    const int L = grp_row / nao_p, mu0 = grp_row % nao_p;
                    const size_t N2 = (size_t)naux * fr.neo;
                    const size_t g2 = ((size_t)slot * nao_p + mu0) / 8;
                    const size_t x = (size_t)L * fr.neo + cm.y;
#pragma unroll
                    for (int p3 = 0; p3 < P2; ++p3) {
                        bf8 part[NS];
#pragma unroll
                        for (int v = 0; v < 8; ++v) {
                            __bf16 sp[NS];
                            split_bf16<NS>(pl[p3][v], sp);
#pragma unroll
                            for (int t = 0; t < NS; ++t) part[t][v] = sp[t];
                        }
#pragma unroll
                        for (int t = 0; t < NS; ++t)
                            *reinterpret_cast<bf8*>(fr.ptt + (((size_t)(p3 * NS + t) * fr.ng2 + g2) * N2 + x) * 8) =
                                part[t];
                    }
                }
            }
        }
}

// Stage 2 over the items of one round (all fragments).
template <int NS>
__global__ void __launch_bounds__(256) k_xf2_batched(int nitems, const BItem2* __restrict__ items,
                                                     const BFrag* __restrict__ frags, const BQ* __restrict__ qs) {
    constexpr int BM = 64, BN = 64, TM = 1, TN = 1;
    extern __shared__ __align__(16) bf8 ring[];
    const long it_id = xcd_logical(blockIdx.x, gridDim.x);
    if (it_id >= nitems) return;
    const BItem2 item = items[it_id];
    const BFrag fr = frags[item.slot];
    const BQ& qb = qs[item.slot];
    const int neo = fr.neo, naux = fr.naux, L = item.L;
    const int m0 = item.it * BM, j0 = item.jt * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
    const int N2 = naux * neo;
    f16v acc[2][TM][TN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[p][0][0][r] = 0.f;
    __shared__ short ksh[KP_MAX];   // the slot -> k table, staged once
    for (int t = threadIdx.x; t < qb.npaired + qb.nself; t += blockDim.x) ksh[t] = qb.k[t];
    __syncthreads();
    pk_loop_paired<NS, BM, BN, TM, TN>(fr.pc2, (size_t)fr.ng2 * neo, neo, fr.ptt, (size_t)fr.ng2 * N2, N2, L, m0, j0,
                                       qb.gpk, qb.zg, qb.npaired, qb.nself, [&](int sl) { return (int)ksh[sl]; },
                                       ring, wm0, wn0, acc);
    const size_t ldz = (size_t)fr.npair;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = m0 + wm0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = j0 + wn0 + (lane & 31);
        if (i >= neo || j >= neo || j > i) continue;
        const size_t pair = (size_t)i * (i + 1) / 2 + j;
        const float xr = acc[0][0][0][r], xi = acc[1][0][0][r];
        if (qb.self_conj) {
            fr.z[(qb.zrow0 + L) * ldz + pair] = qb.wq * xr;
        } else {
            fr.z[(qb.zrow0 + 2 * (size_t)L) * ldz + pair] = qb.wq * xr;
            fr.z[(qb.zrow0 + 2 * (size_t)L + 1) * ldz + pair] = qb.wq * xi;
        }
    }
}

// Stage 2 of small fragments with 32 x 32 tiles: the four waves of a
// workgroup take the same (i, j) tile of four consecutive fitting functions
// (item.L is the group of four), so the operand that does not depend on L
// (conj C) is staged once for the four.  Against 64 x 64 tiles of one L it
// pads a triangle of neo x neo pairs far less when neo is small.  The k <->
// q-k passes, group walk and 4M products are those of pk_loop_paired.
// LDS per stage: [conj C tile][T tile of L0] .. [T tile of L3], each
// P2 x NS x 2 groups x 32 rows.
constexpr int L4_ROWS = 32;

template <int NS>
constexpr size_t xf2_l4_lds() { return (size_t)2 * 5 * P2 * NS * 2 * L4_ROWS * 16; }

// one 32-row tile operand (P2 x NS parts x groups g0, g1 x 32 rows) of a
// stage, loaded by one wave: lanes 0-31 take group g0, lanes 32-63 group g1
template <int NS>
__device__ inline void l4_issue(const __bf16* base, size_t pt_stride, int X, int x0, int g0, int g1, bf8* dst) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 5, x = min(x0 + (lane & 31), X - 1);
#pragma unroll
    for (int pt = 0; pt < P2 * NS; ++pt) {
        const __bf16* src = base + ((size_t)pt * pt_stride + (size_t)(g ? g1 : g0) * X + x) * 8;
        __builtin_amdgcn_global_load_lds((const void*)src, DMET_LDS_PTR(dst + pt * 2 * L4_ROWS), 16, 0, 0);
    }
}

template <int NS>
__global__ void __launch_bounds__(256) k_xf2_batched_l4(int nitems, const BItem2* __restrict__ items,
                                                        const BFrag* __restrict__ frags, const BQ* __restrict__ qs) {
    constexpr int TCH = P2 * NS * 2 * L4_ROWS;      // chunks of one tile operand
    constexpr int STAGE = 5 * TCH;
    extern __shared__ __align__(16) bf8 ring[];
    const long it_id = xcd_logical(blockIdx.x, gridDim.x);
    if (it_id >= nitems) return;
    const BItem2 item = items[it_id];
    const BFrag fr = frags[item.slot];
    const BQ& qb = qs[item.slot];
    const int neo = fr.neo, naux = fr.naux;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int L = 4 * item.L + wave;
    const int Lc = min(L, naux - 1);                 // a wave past naux stages a valid block, stores nothing
    const int m0 = item.it * L4_ROWS, j0 = item.jt * L4_ROWS;
    const int N2 = naux * neo;
    const size_t cst = (size_t)fr.ng2 * neo, tst = (size_t)fr.ng2 * N2;
    __shared__ short ksh[KP_MAX];   // the slot -> k table, staged once
    for (int t = threadIdx.x; t < qb.npaired + qb.nself; t += blockDim.x) ksh[t] = qb.k[t];
    __syncthreads();
    f16v acc[2][1][1];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][0][0][r] = 0.f;
    PairedWalk walk((qb.npaired + qb.nself) * qb.gpk, qb.npaired * qb.gpk, qb.gpk, qb.zg);
    const int nst = walk.stages();
    auto kof = [&](int sl) { return (int)ksh[sl]; };
    // wave w stages the T tile of its own L; wave 0 also the conj C tile
    auto issue = [&](bf8* dst) {
        int gc0, gt0, gc1, gt1;
        const int pass = walk.next(kof, gc0, gt0, gc1, gt1);
        const int xc = pass ? j0 : m0;                        // conj C rows
        const int xt = Lc * neo + (pass ? m0 : j0);            // T columns of this wave's L
        if (wave == 0) l4_issue<NS>(fr.pc2, cst, neo, xc, gc0, gc1, dst);
        l4_issue<NS>(fr.ptt, tst, N2, xt, gt0, gt1, dst + (1 + wave) * TCH);
    };
    issue(ring);
    for (int st = 0; st < nst; ++st) {
        bf8* cur = ring + (size_t)(st & 1) * STAGE;
        __builtin_amdgcn_s_waitcnt(0x0F70);   // own loads of stage st landed
        __builtin_amdgcn_s_barrier();         // everyone's loads landed; stage st-1 fully read
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) issue(ring + (size_t)((st + 1) & 1) * STAGE);
        const bf8* sc = cur;                      // conj C tile
        const bf8* stt = cur + (1 + wave) * TCH;  // T tile of this wave's L
        if (!walk.pass_of(st)) pk_mma4<NS, L4_ROWS, L4_ROWS, 1, 1>(sc, stt, 0, 0, acc);
        else pk_mma4<NS, L4_ROWS, L4_ROWS, 1, 1>(stt, sc, 0, 0, acc);
    }
    if (L >= naux) return;
    const size_t ldz = (size_t)fr.npair;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int jj = j0 + (lane & 31);
        if (i >= neo || jj >= neo || jj > i) continue;
        const size_t pair = (size_t)i * (i + 1) / 2 + jj;
        const float xr = acc[0][0][0][r], xi = acc[1][0][0][r];
        if (qb.self_conj) {
            fr.z[(qb.zrow0 + L) * ldz + pair] = qb.wq * xr;
        } else {
            fr.z[(qb.zrow0 + 2 * (size_t)L) * ldz + pair] = qb.wq * xr;
            fr.z[(qb.zrow0 + 2 * (size_t)L + 1) * ldz + pair] = qb.wq * xi;
        }
    }
}

// Persistent packed contraction over the tiles of all fragments.  Workgroup b
// pops items from the queue of XCD b % 8 (items of one 8 x 8 super-block of one
// fragment are in one queue, so tiles sharing panels run on one XCD).
// BM = 128: two workgroups per CU, 3-stage ring; BM = 64: 2-stage ring.
template <int NS, int BM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_contract_persist(const int* __restrict__ qstart, const int* __restrict__ qlen, int* __restrict__ qctr,
                   const BItemC* __restrict__ items, const BFrag* __restrict__ frags, int flush_k) {
    constexpr int BN = BM, G = 2;
    constexpr int NBUF = BM == 128 ? 3 : 2;
    constexpr int TM = BM / 64, TN = BN / 64;
    constexpr int PART = G * BM;
    constexpr int STAGE = 2 * NS * PART;
    constexpr int WM = BM / 2, WN = BN / 2;
    extern __shared__ __align__(16) bf8 ring[];
    __shared__ int s_item;
    const int xcd = blockIdx.x % NXCD;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
    const int g = lane >> 5;
    static_assert(BM % 64 == 0, "a wave's 64 chunks lie in one row group");
    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(&qctr[xcd], 1);
        __syncthreads();
        const int idx = s_item;
        if (idx >= qlen[xcd]) break;
        const BItemC item = items[qstart[xcd] + idx];
        const BFrag fr = frags[item.slot];
        const int npair = fr.npair, nkt = fr.kgroups / G;
        const int m0 = item.mt * BM, n0 = item.nt * BN;
        const bool diag = item.mt == item.nt;
        const size_t plane = (size_t)fr.kgroups * npair;
        const __bf16* pa = fr.zp;

        auto issue = [&](int kt) {
            bf8* st = ring + (size_t)(kt % NBUF) * STAGE;
            for (int first = wave * 64; first < NS * PART; first += 256) {
                const int t = first / PART, w = first % PART, gg = w / BM, row0 = w % BM;
                const size_t grp = (size_t)kt * G + gg;
                const int xa = min(m0 + row0 + lane, npair - 1), xb = min(n0 + row0 + lane, npair - 1);
                const __bf16* row = pa + (t * plane + grp * npair) * 8;
                lds_dma16(row, (unsigned)npair * 16u, (unsigned)xa * 16u, st + first);
                lds_dma16(row, (unsigned)npair * 16u, (unsigned)xb * 16u, st + NS * PART + first);
            }
        };

        f16v acc[TM][TN];
        double acc64[TM][TN][16];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc[i][j][r] = 0.f;
                    acc64[i][j][r] = 0.0;
                }
        for (int s2 = 0; s2 < NBUF - 1; ++s2)
            if (s2 < nkt) issue(s2);
        __builtin_amdgcn_s_waitcnt(0xC07F);   // no scalar load in flight at the loop head
        int since = 0;
        for (int kt = 0; kt < nkt; ++kt) {
            // with NBUF = 3 the loads of one younger stage may stay in flight; every
            // wave issues the same number of loads per stage when BM = 128
            if constexpr (NBUF == 3) {
                constexpr int LOADS = 2 * NS * (PART / 256);
                if (kt + 1 < nkt) __builtin_amdgcn_s_waitcnt(0x0F70 | (LOADS & 15) | ((LOADS >> 4) << 14));
                else __builtin_amdgcn_s_waitcnt(0x0F70);
            } else {
                __builtin_amdgcn_s_waitcnt(0x0F70);
            }
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
            if (kt + NBUF - 1 < nkt) issue(kt + NBUF - 1);
            const bf8* sA = ring + (size_t)(kt % NBUF) * STAGE;
            const bf8* sB = sA + NS * PART;
            bf8 b[NS][TN];
#pragma unroll
            for (int t = 0; t < NS; ++t)
#pragma unroll
                for (int j = 0; j < TN; ++j) b[t][j] = sB[t * PART + g * BN + wn0 + j * 32 + (lane & 31)];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
#pragma unroll
                for (int ta = NS - 1; ta >= 0; --ta) {
                    const bf8 a = sA[ta * PART + g * BM + wm0 + i * 32 + (lane & 31)];
#pragma unroll
                    for (int tb = NS - 1 - ta; tb >= 0; --tb)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[tb][j], acc[i][j], 0, 0, 0);
                    if constexpr (NS == 2) {
                        if (ta == 1 && diag)
#pragma unroll
                            for (int j = 0; j < TN; ++j)
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[1][j], acc[i][j], 0, 0, 0);
                    }
                }
            }
            since += 8 * G;
            if (since >= flush_k || kt + 1 == nkt) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            acc64[i][j][r] += (double)acc[i][j][r];
                            acc[i][j][r] = 0.f;
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
                    if (IJ < npair && KL <= IJ) fr.eri[(size_t)IJ * (IJ + 1) / 2 + KL] = acc64[i][j][r];
                }
    }
}

template <int NS, int BM>
constexpr size_t persist_lds() { return (size_t)(BM == 128 ? 3 : 2) * 2 * NS * 2 * BM * 16; }

// Persistent int8 contraction over the tiles of all fragments (the int8 form of
// k_contract_persist): 128 x 128 tiles, four waves of 64 x 64, 32-row stages
// of three digit planes in a 3-deep ring (two workgroups per CU), three int32
// accumulator sets, the FP64 combination with the column exponents at the end.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_contract_persist_i8(const int* __restrict__ qstart, const int* __restrict__ qlen, int* __restrict__ qctr,
                      const BItemC* __restrict__ items, const BFrag* __restrict__ frags) {
    constexpr int NS = 3, BM = 128, BN = 128, G = 2, NBUF = 3;
    constexpr int TM = 2, TN = 2;
    constexpr int PART = G * BM;
    constexpr int STAGE = 2 * NS * PART;
    extern __shared__ __align__(16) i4v ring_p8[];
    __shared__ int s_item;
    const int xcd = blockIdx.x % NXCD;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
    const int g = lane >> 5;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(&qctr[xcd], 1);
        __syncthreads();
        const int idx = s_item;
        if (idx >= qlen[xcd]) break;
        const BItemC item = items[qstart[xcd] + idx];
        const BFrag fr = frags[item.slot];
        const int npair = fr.npair, nkt = fr.kg16 / G;
        const int m0 = item.mt * BM, n0 = item.nt * BN;
        const size_t plane = (size_t)fr.kg16 * npair;
        const i4v* pa = fr.zp8;

        auto issue = [&](int kt) {
            i4v* st = ring_p8 + (size_t)(kt % NBUF) * STAGE;
            for (int first = wave * 64; first < NS * PART; first += 256) {
                const int t = first / PART, w = first % PART, gg = w / BM, row0 = w % BM;
                const size_t grp = (size_t)kt * G + gg;
                const int xa = min(m0 + row0 + lane, npair - 1), xb = min(n0 + row0 + lane, npair - 1);
                const i4v* row = pa + t * plane + grp * npair;
                lds_dma16(row, (unsigned)npair * 16u, (unsigned)xa * 16u, st + first);
                lds_dma16(row, (unsigned)npair * 16u, (unsigned)xb * 16u, st + NS * PART + first);
            }
        };

        i16v acc[3][TM][TN];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[l][i][j][r] = 0;
        for (int s2 = 0; s2 < NBUF - 1; ++s2)
            if (s2 < nkt) issue(s2);
        __builtin_amdgcn_s_waitcnt(0xC07F);   // no scalar load in flight at the loop head
        for (int kt = 0; kt < nkt; ++kt) {
            // the loads of one younger stage may stay in flight; every wave issues
            // the same number of loads per stage
            constexpr int LOADS = 2 * NS * (PART / 256);
            if (kt + 1 < nkt) __builtin_amdgcn_s_waitcnt(0x0F70 | (LOADS & 15) | ((LOADS >> 4) << 14));
            else __builtin_amdgcn_s_waitcnt(0x0F70);
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
            if (kt + NBUF - 1 < nkt) issue(kt + NBUF - 1);
            const i4v* sA = ring_p8 + (size_t)(kt % NBUF) * STAGE;
            const i4v* sB = sA + NS * PART;
            i4v b[NS][TN];
#pragma unroll
            for (int t = 0; t < NS; ++t)
#pragma unroll
                for (int j = 0; j < TN; ++j) b[t][j] = sB[t * PART + g * BN + wn0 + j * 32 + (lane & 31)];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
#pragma unroll
                for (int ta = NS - 1; ta >= 0; --ta) {
                    const i4v a = sA[ta * PART + g * BM + wm0 + i * 32 + (lane & 31)];
#pragma unroll
                    for (int tb = NS - 1 - ta; tb >= 0; --tb)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            acc[ta + tb][i][j] =
                                __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b[tb][j], acc[ta + tb][i][j], 0, 0, 0);
                }
            }
        }
        constexpr double inv_b = 1.0 / 254.0, inv_b0sq = 1.0 / (127.0 * 127.0);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int KL = n0 + wn0 + j * 32 + (lane & 31);
            const int eb = fr.ex[min(KL, npair - 1)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int IJ = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    if (IJ >= npair || KL > IJ) continue;
                    const int ea = fr.ex[IJ];
                    double v = (double)acc[0][i][j][r] +
                               ((double)acc[1][i][j][r] + (double)acc[2][i][j][r] * inv_b) * inv_b;
                    v = (ea == I8_EBAD || eb == I8_EBAD) ? __builtin_nan("") : ldexp(v * inv_b0sq, ea + eb);
                    fr.eri[(size_t)IJ * (IJ + 1) / 2 + KL] = v;
                }
        }
    }
}

constexpr size_t persist_i8_lds() { return (size_t)3 * 2 * 3 * 2 * 128 * 16; }

template <int NS>
constexpr size_t xf1_lds() { return (size_t)2 * P2 * NS * 2 * (128 + 128) * 16; }
constexpr int XF1_NW = 8;   // waves per stage-1 workgroup
template <int NS>
constexpr size_t xf2_lds() { return (size_t)2 * P2 * NS * 2 * (64 + 64) * 16; }

// ------------------------------------------------------------------ driver
constexpr int FLUSH_K = 256;

static int kgroups_of(int krows) { return (krows + 31) / 32 * 4; }

static size_t packed_elems(const EriPlan& p) {
    const int ns = p.prec == DMET_BF16X6_3M ? 3 : (p.prec == DMET_BF16X3_3M ? 2 : 0);
    return (size_t)ns * kgroups_of(p.zrows) * 8 * p.npair;
}

// int8 digit planes: groups of 16 rows, a multiple of the 4 groups of a stage
static int kgroups16_of(int krows) { return (krows + 63) / 64 * 4; }

// Rows per int8 contraction launch: I8_KMAX, or DMET_I8_CHUNK_ROWS (a multiple
// of 64 in [64, I8_KMAX]) to run Z in smaller chunks.
static int i8_chunk_rows() {
    const char* e = getenv("DMET_I8_CHUNK_ROWS");
    const int v = e ? atoi(e) : I8_KMAX;
    return v >= 64 && v <= I8_KMAX && v % 64 == 0 ? v : I8_KMAX;
}
static size_t i8_chunks(const EriPlan& p) { return (size_t)3 * kgroups16_of(p.zrows) * p.npair; }

// padded sizes of the packed transform operands
struct PkDims {
    int ns, nao_p, ngv, ng2, M1, NB;
    size_t N2;
    size_t lm_elems, c1_elems, c2_elems, t_elems;
};

static PkDims pk_dims(const EriPlan& p) {
    PkDims d;
    d.ns = p.prec == DMET_BF16X3_3M ? 2 : 3;
    d.nao_p = (p.nao + 7) / 8 * 8;
    d.ngv = (d.nao_p / 8 + 1) / 2 * 2;
    // groups of (k, mu) plus at least one zero group (index nk * nao_p / 8), even
    d.ng2 = (p.mesh.nk * d.nao_p / 8 + 2) / 2 * 2;
    d.M1 = p.naux * d.nao_p;
    d.NB = p.nspin * p.neo;
    d.N2 = (size_t)p.naux * p.neo;
    const size_t pl2 = (size_t)P2 * d.ns * 8;
    d.lm_elems = (size_t)p.mesh.nk * p.mesh.nk * pl2 * d.ngv * d.M1;
    d.c1_elems = (size_t)p.mesh.nk * pl2 * d.ngv * d.NB;
    d.c2_elems = (size_t)p.nspin * pl2 * d.ng2 * p.neo;
    d.t_elems = (size_t)p.nspin * pl2 * d.ng2 * d.N2;
    return d;
}

size_t eri_lp_workspace(const EriPlan& p) {
    Carve cv(nullptr, 0);
    PkDims d = pk_dims(p);
    cv.take<__bf16>(d.lm_elems);
    cv.take<__bf16>(d.c1_elems);
    cv.take<__bf16>(d.c2_elems);
    cv.take<__bf16>(d.t_elems);
    cv.take<float>((size_t)p.nspin * p.zrows * p.npair);              // Z per spin
    if (p.prec == DMET_BF16X6_I8) {
        cv.take<i4v>((size_t)p.nspin * i8_chunks(p));                 // int8 digit planes of Z
        cv.take<unsigned>((size_t)p.nspin * p.npair);                 // column max
        cv.take<int>((size_t)p.nspin * p.npair);                      // column exponents
    } else {
        cv.take<__bf16>((size_t)p.nspin * packed_elems(p));           // split parts of Z
    }
    return cv.bytes();
}

// Transform of the bf16 forms on packed operands (replaces the generic
// staged kernels for these forms).
template <int NS>
static dmet_status xform_packed(const EriPlan& p, const void* lmunu, const double* ck, float* z, Carve& cv,
                                hipStream_t st) {
    PkDims d = pk_dims(p);
    __bf16* plm = cv.take<__bf16>(d.lm_elems);
    __bf16* pc1 = cv.take<__bf16>(d.c1_elems);
    __bf16* pc2 = cv.take<__bf16>(d.c2_elems);
    __bf16* ptt = cv.take<__bf16>(d.t_elems);
    const int nk = p.mesh.nk;
    if (nk > KP_MAX) return fail(DMET_E_UNSUPPORTED, "split-bf16 transform supports at most 256 k-points");
    const int gpk = d.nao_p / 8, zg = nk * gpk;   // groups per k; the zero group
    const char* nm = NS == 3 ? "pack_in_bf16x6" : "pack_in_bf16x3";
    {
        ProfScope ps(nm, st);
        const int mb = pack_rows_per_block(d.ngv);
        const long nblk = (long)nk * nk * p.naux * ((d.nao_p + mb - 1) / mb);
        const size_t lds = pack_lds_bytes(mb, d.ngv);
        if (p.dtype == DMET_C128)
            k_pack_lmunu<NS, double><<<dim3((unsigned)nblk), 256, lds, st>>>(
                static_cast<const double*>(lmunu), p.nao, d.nao_p, p.naux, d.ngv, mb, plm, p.mesh, 1);
        else
            k_pack_lmunu<NS, float><<<dim3((unsigned)nblk), 256, lds, st>>>(
                static_cast<const float*>(lmunu), p.nao, d.nao_p, p.naux, d.ngv, mb, plm, p.mesh, 1);
        k_pack_c1<NS><<<dim3((d.NB + 255) / 256, d.ngv, nk), 256, 0, st>>>(ck, nk, p.nspin, p.nao, p.neo, d.ngv, pc1,
                                                                          0, d.NB);
        k_pack_c2<NS><<<dim3((p.neo + 255) / 256, d.ng2, p.nspin), 256, 0, st>>>(ck, nk, p.nao, d.nao_p, p.neo,
                                                                                 d.ng2, pc2);
        // groups zg .. ng2-1 of T pad odd group counts in stage 2: make them zero
        // (stage 1 writes compact slots below zg only; conj C is zero there too)
        const size_t part = (size_t)d.ng2 * d.N2 * 8;
        for (int sp = 0; sp < p.nspin * P2 * NS; ++sp)
            fill_zero(ptt + (size_t)sp * part + (size_t)zg * d.N2 * 8, (size_t)(d.ng2 - zg) * d.N2 * 8 * sizeof(__bf16),
                      st);
        ps.stop();
    }
    DMET_LAUNCH_CHECK("pack inputs");
    auto k1 = k_xf1_pk<NS, XF1_NW>;
    auto k2 = k_xf2_pk2<NS>;
    DMET_HIP(hipFuncSetAttribute((const void*)k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)xf2_pk2_lds<NS>()));
    DMET_HIP(hipFuncSetAttribute((const void*)k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)xf1_lds<NS>()));

    const char* n1 = NS == 3 ? "xform1_bf16x6" : "xform1_bf16x3";
    const char* n2 = NS == 3 ? "xform2_bf16x6" : "xform2_bf16x3";
    const size_t ldz = (size_t)p.npair;
    const int njt = (p.neo + 63) / 64, nit = (p.neo + 63) / 64;
    const size_t t_spin = (size_t)P2 * NS * d.ng2 * d.N2 * 8;
    const size_t c2_spin = (size_t)P2 * NS * d.ng2 * p.neo * 8;
    for (const QBlock& qb : p.qblocks) {
        const KSlots ks = kpair_slots(p.mesh, qb.q);
        ProfScope ps1(n1, st);
        const long nb1 = ((long)(ks.npaired + ks.nself) * ((d.M1 + 127) / 128) * ((d.NB + 127) / 128) + NXCD - 1) /
                         NXCD * NXCD;
        k1<<<dim3((unsigned)nb1), 64 * XF1_NW, xf1_lds<NS>(), st>>>(p.mesh, qb.q, p.naux, d.nao_p, p.neo, p.nspin, d.ngv,
                                                            d.ng2, ks, plm, pc1, ptt);
        ps1.stop();
        DMET_LAUNCH_CHECK(n1);
        for (int s = 0; s < p.nspin; ++s) {
            ProfScope ps2(n2, st);
            const long nb2 = ((long)((p.naux + 1) / 2) * njt * nit + NXCD - 1) / NXCD * NXCD;
            k2<<<dim3((unsigned)nb2), 512, xf2_pk2_lds<NS>(), st>>>(p.naux, p.neo, d.ng2, gpk, zg, ks, qb.self_conj,
                                                                qb.zrow0, (float)qb.weight, pc2 + s * c2_spin,
                                                                ptt + s * t_spin, z + (size_t)s * p.zrows * ldz, ldz);
            ps2.stop();
            DMET_LAUNCH_CHECK(n2);
        }
    }
    return DMET_OK;
}

__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

template <int NS>
static dmet_status eri_lp_run(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa,
                              double* eri_bb, double* eri_ab, float* z, __bf16* zp, Carve& cv, hipStream_t st,
                              double* df_out) {
    const char* n3 = NS == 3 ? "contract_s8_bf16x6" : "contract_s8_bf16x3";
    const char* n4 = NS == 3 ? "contract_s4_bf16x6" : "contract_s4_bf16x3";
    const size_t ldz = (size_t)p.npair;
    dmet_status xs = xform_packed<NS>(p, lmunu, ck, z, cv, st);
    if (xs != DMET_OK) return xs;
    if (df_out) {
        const size_t n = (size_t)p.nspin * p.zrows * p.npair;
        k_f32_to_f64<<<1024, 256, 0, st>>>(z, df_out, n);
        DMET_LAUNCH_CHECK("k_f32_to_f64");
        return DMET_OK;
    }
    const int kg = kgroups_of(p.zrows);
    const size_t per_spin = (size_t)NS * kg * 8 * p.npair;
    for (int s = 0; s < p.nspin; ++s) {
        ProfScope ps(NS == 2 ? "pack_bf16x3" : "pack_bf16x6", st);
        k_pack_parts<NS><<<dim3((p.npair + 255) / 256, group_grid(kg)), 256, 0, st>>>(
            z + (size_t)s * p.zrows * ldz, ldz, p.zrows, p.npair, kg, zp + s * per_spin);
        ps.stop();
        DMET_LAUNCH_CHECK("k_pack_parts");
    }
    // 32-row stages; three-way split: 2-deep ring, two-way: 3-deep
    constexpr int G = 4, NB = NS == 3 ? 2 : 3;
    auto kw0 = k_contract_w8<NS, 0, G, NB>;
    auto kw1 = k_contract_w8<NS, 1, G, NB>;
    constexpr size_t lds = w8_lds<NS, G, NB>();
    static_assert(lds <= 160 * 1024, "LDS per workgroup");
    DMET_HIP(hipFuncSetAttribute((const void*)kw0, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    DMET_HIP(hipFuncSetAttribute((const void*)kw1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    for (int s = 0; s < p.nspin; ++s) {
        const long nb = w8_grid(0, p.npair);
        ProfScope ps(n3, st);
        kw0<<<dim3((unsigned)nb), 512, lds, st>>>(p.npair, kg, zp + s * per_spin, zp + s * per_spin, FLUSH_K, nb,
                                                  s == 0 ? eri_aa : eri_bb, kg, kg, 0);
        ps.stop();
        DMET_LAUNCH_CHECK(n3);
    }
    if (p.nspin == 2 && eri_ab) {
        const long nb = w8_grid(1, p.npair);
        ProfScope ps(n4, st);
        kw1<<<dim3((unsigned)nb), 512, lds, st>>>(p.npair, kg, zp, zp + per_spin, FLUSH_K, nb, eri_ab, kg, kg, 0);
        ps.stop();
        DMET_LAUNCH_CHECK(n4);
    }
    return DMET_OK;
}

// DMET_BF16X6_I8: the BF16X6 transform, then the int8 fixed-point contraction
static dmet_status eri_i8_run(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa,
                              double* eri_bb, double* eri_ab, float* z, i4v* zp, unsigned* cmax, int* ex, Carve& cv,
                              hipStream_t st, double* df_out) {
    const size_t ldz = (size_t)p.npair;
    dmet_status xs = xform_packed<3>(p, lmunu, ck, z, cv, st);
    if (xs != DMET_OK) return xs;
    if (df_out) {
        const size_t n = (size_t)p.nspin * p.zrows * p.npair;
        k_f32_to_f64<<<1024, 256, 0, st>>>(z, df_out, n);
        DMET_LAUNCH_CHECK("k_f32_to_f64");
        return DMET_OK;
    }
    const int kg = kgroups16_of(p.zrows);
    const size_t per_spin = (size_t)3 * kg * p.npair;
    fill_zero(cmax, (size_t)p.nspin * p.npair * sizeof(unsigned), st);
    const int rows_per = 256;
    for (int s = 0; s < p.nspin; ++s) {
        ProfScope ps("pack_i8", st);
        const float* zs = z + (size_t)s * p.zrows * ldz;
        k_colmax<<<dim3((p.npair + 255) / 256, (p.zrows + rows_per - 1) / rows_per), 256, 0, st>>>(
            zs, ldz, p.zrows, p.npair, rows_per, cmax + (size_t)s * p.npair);
        k_pack_i8<<<dim3((p.npair + 255) / 256, group_grid(kg)), 256, 0, st>>>(zs, ldz, p.zrows, p.npair, kg,
                                                                     cmax + (size_t)s * p.npair,
                                                                     ex + (size_t)s * p.npair, zp + s * per_spin);
        ps.stop();
        DMET_LAUNCH_CHECK("k_pack_i8");
    }
    constexpr size_t lds = i8_lds();
    static_assert(lds <= 160 * 1024, "LDS per workgroup");
    const void* kc[4] = {(const void*)k_contract_i8<0, false>, (const void*)k_contract_i8<0, true>,
                         (const void*)k_contract_i8<1, false>, (const void*)k_contract_i8<1, true>};
    for (const void* f : kc) DMET_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    // chunks of at most I8_KMAX rows (exact int32 sums each), added in FP64 in order
    const int kg_chunk = i8_chunk_rows() / 16;
    for (int s = 0; s < p.nspin; ++s) {
        const long nb = w8_grid(0, p.npair);
        ProfScope ps("contract_s8_i8", st);
        for (int g0 = 0; g0 < kg; g0 += kg_chunk) {
            const size_t off = (size_t)g0 * p.npair;
            const int kc = std::min(kg_chunk, kg - g0);
            auto k8 = g0 > 0 ? k_contract_i8<0, true> : k_contract_i8<0, false>;
            k8<<<dim3((unsigned)nb), 512, lds, st>>>(p.npair, kc, zp + s * per_spin + off, zp + s * per_spin + off,
                                                     ex + (size_t)s * p.npair, ex + (size_t)s * p.npair, nb,
                                                     s == 0 ? eri_aa : eri_bb, kg);
        }
        ps.stop();
        DMET_LAUNCH_CHECK("contract_s8_i8");
    }
    if (p.nspin == 2 && eri_ab) {
        const long nb = w8_grid(1, p.npair);
        ProfScope ps("contract_s4_i8", st);
        for (int g0 = 0; g0 < kg; g0 += kg_chunk) {
            const size_t off = (size_t)g0 * p.npair;
            const int kc = std::min(kg_chunk, kg - g0);
            auto k4 = g0 > 0 ? k_contract_i8<1, true> : k_contract_i8<1, false>;
            k4<<<dim3((unsigned)nb), 512, lds, st>>>(p.npair, kc, zp + off, zp + per_spin + off, ex, ex + p.npair, nb,
                                                     eri_ab, kg);
        }
        ps.stop();
        DMET_LAUNCH_CHECK("contract_s4_i8");
    }
    return DMET_OK;
}

dmet_status eri_lp(const EriPlan& p, const void* lmunu, const double* ck, double* eri_aa, double* eri_bb,
                   double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st, double* df_out) {
    if (p.prec != DMET_BF16X3_3M && p.prec != DMET_BF16X6_3M && p.prec != DMET_BF16X6_I8)
        return fail(DMET_E_ARG, "eri_lp: split-bf16 forms only");
    if (eri_lp_workspace(p) > ws_bytes) return fail(DMET_E_WORKSPACE, "transform_eri workspace too small");
    // layout: [packed transform operands] [Z] [split parts of Z]
    Carve cv(ws, ws_bytes);
    Carve pre(ws, ws_bytes);
    PkDims d = pk_dims(p);
    cv.take<__bf16>(d.lm_elems);
    cv.take<__bf16>(d.c1_elems);
    cv.take<__bf16>(d.c2_elems);
    cv.take<__bf16>(d.t_elems);
    float* z = cv.take<float>((size_t)p.nspin * p.zrows * p.npair);
    if (p.prec == DMET_BF16X6_I8) {
        i4v* zp8 = cv.take<i4v>((size_t)p.nspin * i8_chunks(p));
        unsigned* cmax = cv.take<unsigned>((size_t)p.nspin * p.npair);
        int* ex = cv.take<int>((size_t)p.nspin * p.npair);
        return eri_i8_run(p, lmunu, ck, eri_aa, eri_bb, eri_ab, z, zp8, cmax, ex, pre, st, df_out);
    }
    __bf16* zp = cv.take<__bf16>((size_t)p.nspin * packed_elems(p));
    if (p.prec == DMET_BF16X3_3M) return eri_lp_run<2>(p, lmunu, ck, eri_aa, eri_bb, eri_ab, z, zp, pre, st, df_out);
    return eri_lp_run<3>(p, lmunu, ck, eri_aa, eri_bb, eri_ab, z, zp, pre, st, df_out);
}

// The split-bf16 transform alone: FP32 rows z[nspin][zrows][npair] (the rows of
// eri_lp before its contraction).  Workspace: the packed transform operands.
size_t lp_transform_workspace(const EriPlan& p) {
    Carve cv(nullptr, 0);
    PkDims d = pk_dims(p);
    cv.take<__bf16>(d.lm_elems);
    cv.take<__bf16>(d.c1_elems);
    cv.take<__bf16>(d.c2_elems);
    cv.take<__bf16>(d.t_elems);
    return cv.bytes();
}

dmet_status lp_transform(const EriPlan& p, const void* lmunu, const double* ck, float* z, void* ws, size_t ws_bytes,
                         hipStream_t st) {
    if (lp_transform_workspace(p) > ws_bytes) return fail(DMET_E_WORKSPACE, "split-bf16 transform workspace");
    Carve cv(ws, ws_bytes);
    return p.prec == DMET_BF16X3_3M ? xform_packed<2>(p, lmunu, ck, z, cv, st) : xform_packed<3>(p, lmunu, ck, z, cv, st);
}

// The packed split-bf16 contraction (s8 per spin, s4 alpha-beta) of FP64 rows
// made elsewhere (the plane-wave route), z[s] krows x ldz (row-major, npair used
// columns).  Few output tiles over many rows (2 n_r rows per q there) would
// leave most CUs idle, so such launches split the rows (blockIdx.y) into slices
// of the output that k_sum_slices adds in row order (deterministic).

constexpr int NCU = 256;   // compute units of an MI355X: one contraction workgroup each

// Output tiles (128 x 256) of one contraction launch that hold outputs.
static long w8_tiles(int mode, int npair) {
    const int ntm = (npair + 127) / 128, ntn = (npair + 255) / 256;
    if (mode == 1) return (long)ntm * ntn;
    long n = 0;
    for (int mt = 0; mt < ntm; ++mt) n += std::min(ntn, (mt * 128 + 127) / 256 + 1);
    return n;
}

static size_t out_elems(int mode, int npair) {
    return mode == 0 ? (size_t)npair * (npair + 1) / 2 : (size_t)npair * npair;
}

struct RowSplit {
    int n = 1;        // row splits (slices of the output)
    int groups = 0;   // 8-row groups per split
};

// As many splits as tiles x splits workgroups fit on the CUs at once; a launch
// with half a tile per CU or more keeps one split.  Splits are whole FP32
// flush windows (FLUSH_K rows), so every split forms the FP32 partial sums of
// the unsplit launch and the results differ only in the order of FP64 adds.
static RowSplit row_split(int mode, int npair, int kg) {
    constexpr int W = FLUSH_K / 8;
    RowSplit r;
    r.groups = kg;
    const char* e = getenv("DMET_ROW_SPLIT");
    if (e && atoi(e) == 0) return r;
    const long tiles = w8_tiles(mode, npair);
    if (2 * tiles > NCU) return r;
    const int windows = (kg + W - 1) / W;
    const int n = std::min((int)(NCU / tiles), windows);
    if (n < 2) return r;
    r.groups = (windows + n - 1) / n * W;
    r.n = (kg + r.groups - 1) / r.groups;
    return r;
}

// out[i] = sum over the slices y of part[y n + i], in slice (row) order
__global__ void k_sum_slices(const double* __restrict__ part, size_t n, int nsl, double* __restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double v = part[i];
        for (int y = 1; y < nsl; ++y) v += part[(size_t)y * n + i];
        out[i] = v;
    }
}

struct RowsWs {
    __bf16* parts = nullptr;
    double* slices = nullptr;
};

// Workspace layout of the rows contraction (sizes only when ws is null).
static size_t rows_layout(dmet_precision prec, int nspin, int npair, int krows, void* ws, size_t ws_bytes,
                          RowsWs& w) {
    Carve cv(ws, ws_bytes);
    const int kg = kgroups_of(krows);
    const int ns = prec == DMET_BF16X3_3M ? 2 : 3;
    w.parts = cv.take<__bf16>((size_t)nspin * ns * kg * 8 * npair);
    size_t sl = 0;
    const RowSplit a = row_split(0, npair, kg);
    if (a.n > 1) sl = (size_t)a.n * out_elems(0, npair);
    if (nspin == 2) {
        const RowSplit b = row_split(1, npair, kg);
        if (b.n > 1) sl = std::max(sl, (size_t)b.n * out_elems(1, npair));
    }
    w.slices = cv.take<double>(sl);
    return cv.bytes();
}

size_t lp_rows_contract_workspace(dmet_precision prec, int nspin, int npair, int krows) {
    RowsWs w;
    return rows_layout(prec, nspin, npair, krows, nullptr, 0, w);
}

template <int NS>
static dmet_status rows_contract_bf16(int nspin, int npair, int krows, const double* z, size_t zsp, size_t ldz,
                                      double* eri_aa, double* eri_bb, double* eri_ab, const RowsWs& w,
                                      hipStream_t st) {
    const int kg = kgroups_of(krows);
    __bf16* zp = w.parts;
    const size_t per_spin = (size_t)NS * kg * 8 * npair;
    for (int s = 0; s < nspin; ++s) {
        ProfScope ps(NS == 2 ? "pack_bf16x3" : "pack_bf16x6", st);
        k_pack_parts<NS, double><<<dim3((npair + 255) / 256, group_grid(kg)), 256, 0, st>>>(
            z + s * zsp, ldz, krows, npair, kg, zp + s * per_spin);
        ps.stop();
        DMET_LAUNCH_CHECK("k_pack_parts");
    }
    constexpr int G = 4, NB = NS == 3 ? 2 : 3;
    auto kw0 = k_contract_w8<NS, 0, G, NB>;
    auto kw1 = k_contract_w8<NS, 1, G, NB>;
    constexpr size_t lds = w8_lds<NS, G, NB>();
    DMET_HIP(hipFuncSetAttribute((const void*)kw0, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    DMET_HIP(hipFuncSetAttribute((const void*)kw1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    auto block = [&](int mode, const __bf16* a, const __bf16* b, double* out) -> dmet_status {
        const RowSplit r = row_split(mode, npair, kg);
        const long nb = w8_grid(mode, npair);
        const size_t n = out_elems(mode, npair);
        ProfScope ps(mode == 0 ? (NS == 3 ? "contract_s8_bf16x6" : "contract_s8_bf16x3")
                               : (NS == 3 ? "contract_s4_bf16x6" : "contract_s4_bf16x3"),
                     st);
        auto kf = mode == 0 ? kw0 : kw1;
        kf<<<dim3((unsigned)nb, (unsigned)r.n), 512, lds, st>>>(npair, kg, a, b, FLUSH_K, nb, r.n > 1 ? w.slices : out,
                                                              kg, r.groups, r.n > 1 ? n : 0);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && r.n > 1) {
            k_sum_slices<<<(unsigned)std::min<size_t>((n + 255) / 256, 4096), 256, 0, st>>>(w.slices, n, r.n, out);
            e = hipGetLastError();
        }
        ps.stop();
        if (e != hipSuccess) return hip_fail(e, "contract rows");
        return DMET_OK;
    };
    for (int s = 0; s < nspin; ++s) {
        const dmet_status bs = block(0, zp + s * per_spin, zp + s * per_spin, s == 0 ? eri_aa : eri_bb);
        if (bs != DMET_OK) return bs;
    }
    if (nspin == 2 && eri_ab) return block(1, zp, zp + per_spin, eri_ab);
    return DMET_OK;
}

dmet_status lp_rows_contract(dmet_precision prec, int nspin, int npair, int krows, const double* z, size_t zsp,
                             size_t ldz, double* eri_aa, double* eri_bb, double* eri_ab, void* ws, size_t ws_bytes,
                             hipStream_t st) {
    if (prec != DMET_BF16X3_3M && prec != DMET_BF16X6_3M)
        return fail(DMET_E_ARG, "split-bf16 rows contraction: BF16X3_3M or BF16X6_3M");
    RowsWs w;
    if (rows_layout(prec, nspin, npair, krows, ws, ws_bytes, w) > ws_bytes)
        return fail(DMET_E_WORKSPACE, "split-bf16 rows contraction workspace");
    if (prec == DMET_BF16X3_3M)
        return rows_contract_bf16<2>(nspin, npair, krows, z, zsp, ldz, eri_aa, eri_bb, eri_ab, w, st);
    return rows_contract_bf16<3>(nspin, npair, krows, z, zsp, ldz, eri_aa, eri_bb, eri_ab, w, st);
}

}  // namespace dmet

// ====================================================================== batched driver
namespace dmet {

struct BatchGroup {
    const void* lm;
    dmet_dtype dt;
    Mesh mesh;
    int nao, naux, nao_p, ngv, ng2, M1, nbtot;
    std::vector<int> members;
    std::vector<QBlock> qbs;
    size_t off_plm, off_pc1, off_colmap;
};

struct BatchFrag {
    int group, neo, npair, zrows, kgroups, col0, kg16 = 0;
    size_t off_pc2, off_ptt, off_z, off_zp, off_ex = 0, cmax_idx = 0;
};

// Fragments with at most this many embedding orbitals take the 32 x 32
// four-L stage-2 tiles in the batched pipeline (DMET_XF2_SMALL_NEO overrides).
// On 64 fragments with neo 21-199 all-32 x 32 was fastest (495 ms against 511
// for all-64 x 64); a split at 128 was slower than either (532: two launches
// per round, each with fewer workgroups).
static int xf2_small_neo() {
    const char* e = getenv("DMET_XF2_SMALL_NEO");
    return e ? atoi(e) : 256;
}

struct BatchPlan {
    std::vector<dmet_fragment> frags;
    int prec = 0, ns = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<BatchGroup> groups;
    std::vector<BatchFrag> fs;
    int rounds = 0;
    size_t off_bfrag = 0, off_items2 = 0, off_bq = 0, off_itemsc = 0, off_q = 0, off_cmax = 0, ncmax = 0;
    std::vector<int> items2_off, items2_cnt;     // 64 x 64 stage-2 items per round
    std::vector<int> items2s_off, items2s_cnt;   // 32 x 32 four-L items (small fragments) per round
    std::vector<BFrag> h_bfrag;
    std::vector<int2> h_colmap;
    std::vector<BItem2> h_items2;
    std::vector<BQ> h_bq;
    std::vector<BItemC> h_itemsc[2];   // per contraction tile size (128, 64)
    std::vector<int> h_qstart[2], h_qlen[2];
    size_t bytes = 0;
    int variant = 128;
    bool uploaded = false;
    hipGraphExec_t exec = nullptr;
    std::string key;
};

static std::mutex g_batch_mu;
static std::map<std::string, BatchPlan*> g_batch_plans;
static std::map<std::string, int> g_tune;   // shape key -> chosen contraction tile

static std::string batch_key(int nfrag, const dmet_fragment* f, int prec, bool with_ptrs, void* ws, size_t wsb) {
    std::string k = std::to_string(prec) + ":" + std::to_string(nfrag);
    char buf[256];
    for (int i = 0; i < nfrag; ++i) {
        snprintf(buf, sizeof(buf), "|%d,%d,%d,%d,%d,%d,%d", f[i].lat.kmesh[0], f[i].lat.kmesh[1], f[i].lat.kmesh[2],
                 f[i].lat.nao, f[i].lat.naux, f[i].neo, (int)f[i].dtype);
        k += buf;
        if (with_ptrs) {
            snprintf(buf, sizeof(buf), "@%p,%p,%p", f[i].lmunu, f[i].c_k, (void*)f[i].eri);
            k += buf;
        }
    }
    if (with_ptrs) {
        snprintf(buf, sizeof(buf), "#%p,%zu", ws, wsb);
        k += buf;
    }
    // the stage-2 tile choice is part of a plan
    snprintf(buf, sizeof(buf), "~%d", xf2_small_neo());
    k += buf;
    return k;
}

// Build groups, per-fragment dims, workspace offsets and the work lists.
static void plan_batch(BatchPlan& bp) {
    const int nfrag = (int)bp.frags.size();
    bp.ns = bp.prec == DMET_BF16X3_3M ? 2 : 3;
    const bool i8 = bp.prec == DMET_BF16X6_I8;
    const int NS = bp.ns;
    // groups by lmunu pointer
    for (int f = 0; f < nfrag; ++f) {
        const dmet_fragment& d = bp.frags[f];
        int g = -1;
        for (size_t i = 0; i < bp.groups.size(); ++i)
            if (bp.groups[i].lm == d.lmunu) g = (int)i;
        if (g < 0) {
            BatchGroup G;
            G.lm = d.lmunu;
            G.dt = d.dtype;
            G.mesh = make_mesh(d.lat.kmesh);
            G.nao = d.lat.nao;
            G.naux = d.lat.naux;
            G.nao_p = (G.nao + 7) / 8 * 8;
            G.ngv = (G.nao_p / 8 + 1) / 2 * 2;
            G.ng2 = (G.mesh.nk * G.nao_p / 8 + 2) / 2 * 2;   // with at least one zero group
            G.M1 = G.naux * G.nao_p;
            G.nbtot = 0;
            dmet_lattice lat1 = d.lat;
            lat1.nspin = 1;
            G.qbs = make_eri_plan(&lat1, d.neo, (dmet_precision)bp.prec, d.dtype).qblocks;
            bp.groups.push_back(G);
            g = (int)bp.groups.size() - 1;
        }
        BatchGroup& G = bp.groups[g];
        BatchFrag F;
        F.group = g;
        F.neo = d.neo;
        F.npair = d.neo * (d.neo + 1) / 2;
        F.zrows = G.mesh.nk * G.naux;
        F.kgroups = (F.zrows + 31) / 32 * 4;
        F.kg16 = (F.zrows + 31) / 32 * 2;      // 32-row stages of two 16-row groups
        F.col0 = G.nbtot;
        G.nbtot += d.neo;
        G.members.push_back(f);
        bp.fs.push_back(F);
    }
    bp.rounds = 0;
    for (auto& G : bp.groups) bp.rounds = std::max(bp.rounds, (int)G.qbs.size());
    // work lists
    bp.h_bfrag.resize(nfrag);
    bp.h_bq.assign((size_t)bp.rounds * nfrag, BQ{});
    bp.items2_off.assign(bp.rounds, 0);
    bp.items2_cnt.assign(bp.rounds, 0);
    bp.items2s_off.assign(bp.rounds, 0);
    bp.items2s_cnt.assign(bp.rounds, 0);
    const int small_neo = xf2_small_neo();
    for (int r = 0; r < bp.rounds; ++r) {
        bp.items2_off[r] = (int)bp.h_items2.size();
        for (int f = 0; f < nfrag; ++f) {
            const BatchFrag& F = bp.fs[f];
            const BatchGroup& G = bp.groups[F.group];
            if (r >= (int)G.qbs.size()) continue;
            const QBlock& qb = G.qbs[r];
            BQ& b = bp.h_bq[(size_t)r * nfrag + f];
            b.self_conj = qb.self_conj;
            b.zrow0 = qb.zrow0;
            b.wq = (float)qb.weight;
            kpair_counts(G.mesh, qb.q, b.npaired, b.nself);
            for (int sl = 0; sl < b.npaired + b.nself; ++sl) b.k[sl] = (short)kpair_slot_k(G.mesh, qb.q, sl);
            b.gpk = G.nao_p / 8;
            b.zg = G.mesh.nk * b.gpk;
            if (F.neo <= small_neo) continue;
            const int nt = (F.neo + 63) / 64;
            for (int L = 0; L < G.naux; ++L)
                for (int jt = 0; jt < nt; ++jt)
                    for (int it = jt; it < nt; ++it) bp.h_items2.push_back(BItem2{f, L, jt, it});
        }
        bp.items2_cnt[r] = (int)bp.h_items2.size() - bp.items2_off[r];
        // small fragments: 32 x 32 tiles, four fitting functions per item
        bp.items2s_off[r] = (int)bp.h_items2.size();
        for (int f = 0; f < nfrag; ++f) {
            const BatchFrag& F = bp.fs[f];
            const BatchGroup& G = bp.groups[F.group];
            if (r >= (int)G.qbs.size() || F.neo > small_neo) continue;
            const int nt = (F.neo + L4_ROWS - 1) / L4_ROWS, nlg = (G.naux + 3) / 4;
            for (int lg = 0; lg < nlg; ++lg)
                for (int jt = 0; jt < nt; ++jt)
                    for (int it = jt; it < nt; ++it) bp.h_items2.push_back(BItem2{f, lg, jt, it});
        }
        bp.items2s_cnt[r] = (int)bp.h_items2.size() - bp.items2s_off[r];
    }
    for (int v = 0; v < 2; ++v) {
        const int BM = v == 0 ? 128 : 64;
        // chunks = 8x8 super-blocks of one fragment, largest contraction depth first
        struct Chunk {
            int f, I, J, k;
        };
        std::vector<Chunk> ch;
        for (int f = 0; f < nfrag; ++f) {
            const int nt = (bp.fs[f].npair + BM - 1) / BM, nsb = (nt + 7) / 8;
            for (int I = 0; I < nsb; ++I)
                for (int J = 0; J <= I; ++J) ch.push_back(Chunk{f, I, J, bp.fs[f].zrows});
        }
        std::stable_sort(ch.begin(), ch.end(), [](const Chunk& a, const Chunk& b) { return a.k > b.k; });
        std::vector<std::vector<BItemC>> q(NXCD);
        for (size_t c = 0; c < ch.size(); ++c) {
            const int nt = (bp.fs[ch[c].f].npair + BM - 1) / BM;
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b) {
                    const int mt = ch[c].I * 8 + a, ntt = ch[c].J * 8 + b;
                    if (mt < nt && ntt < nt && ntt <= mt) q[c % NXCD].push_back(BItemC{ch[c].f, mt, ntt, 0});
                }
        }
        bp.h_itemsc[v].clear();
        bp.h_qstart[v].assign(NXCD, 0);
        bp.h_qlen[v].assign(NXCD, 0);
        for (int x = 0; x < NXCD; ++x) {
            bp.h_qstart[v][x] = (int)bp.h_itemsc[v].size();
            bp.h_qlen[v][x] = (int)q[x].size();
            bp.h_itemsc[v].insert(bp.h_itemsc[v].end(), q[x].begin(), q[x].end());
        }
    }
    // column maps
    for (auto& G : bp.groups) {
        G.off_colmap = bp.h_colmap.size();
        for (int f : G.members)
            for (int j = 0; j < bp.fs[f].neo; ++j) bp.h_colmap.push_back(make_int2(f, j));
    }
    // workspace layout: tables, then per group, then per fragment (256-byte aligned)
    size_t cur = 0;
    auto off = [&](size_t bytes) {
        const size_t o = (cur + 255) & ~size_t(255);
        cur = o + bytes;
        return o;
    };
    bp.off_bfrag = off(sizeof(BFrag) * nfrag);
    const size_t colmap_off = off(sizeof(int2) * bp.h_colmap.size());
    for (auto& G : bp.groups) G.off_colmap = colmap_off + G.off_colmap * sizeof(int2);
    bp.off_items2 = off(sizeof(BItem2) * std::max<size_t>(1, bp.h_items2.size()));
    bp.off_bq = off(sizeof(BQ) * std::max<size_t>(1, bp.h_bq.size()));
    bp.off_itemsc = off(sizeof(BItemC) * std::max(bp.h_itemsc[0].size(), bp.h_itemsc[1].size()) + 16);
    bp.off_q = off(sizeof(int) * 3 * NXCD);
    const size_t pl2 = (size_t)P2 * NS * 8;
    for (auto& G : bp.groups) {
        G.off_plm = off(sizeof(__bf16) * (size_t)G.mesh.nk * G.mesh.nk * pl2 * G.ngv * G.M1);
        G.off_pc1 = off(sizeof(__bf16) * (size_t)G.mesh.nk * pl2 * G.ngv * G.nbtot);
    }
    for (auto& F : bp.fs) {
        const BatchGroup& G = bp.groups[F.group];
        F.off_pc2 = off(sizeof(__bf16) * pl2 * G.ng2 * F.neo);
        F.off_ptt = off(sizeof(__bf16) * pl2 * G.ng2 * (size_t)G.naux * F.neo);
        F.off_z = off(sizeof(float) * (size_t)F.zrows * F.npair);
        if (i8) {
            F.off_zp = off(sizeof(i4v) * (size_t)3 * F.kg16 * F.npair);
            F.off_ex = off(sizeof(int) * (size_t)F.npair);
        } else {
            F.off_zp = off(sizeof(__bf16) * (size_t)NS * F.kgroups * 8 * F.npair);
        }
    }
    if (i8) {   // column maxima of every fragment in one region (one fill per call)
        size_t n = 0;
        for (auto& F : bp.fs) {
            F.cmax_idx = n;
            n += F.npair;
        }
        bp.off_cmax = off(sizeof(unsigned) * std::max<size_t>(1, n));
        bp.ncmax = n;
    }
    bp.bytes = (cur + 255) & ~size_t(255);
}

template <class T>
static T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Enqueue the whole batched pipeline (bf16 forms) on `st`.  Tables must
// already be on the device.  When `prof` is false no events are recorded
// (graph capture).
// Kernel attributes and the CU count (host calls, kept out of graph capture).
static int g_ncu = 0;

template <int NS>
static dmet_status batch_prepare() {
    DMET_HIP(hipFuncSetAttribute((const void*)k_xf1_batched<NS, XF1_NW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)xf1_lds<NS>()));
    DMET_HIP(hipFuncSetAttribute((const void*)k_xf2_batched<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)xf2_lds<NS>()));
    DMET_HIP(hipFuncSetAttribute((const void*)k_xf2_batched_l4<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)xf2_l4_lds<NS>()));
    DMET_HIP(hipFuncSetAttribute((const void*)k_contract_persist<NS, 128>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)persist_lds<NS, 128>()));
    DMET_HIP(hipFuncSetAttribute((const void*)k_contract_persist<NS, 64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)persist_lds<NS, 64>()));
    DMET_HIP(hipFuncSetAttribute((const void*)k_contract_persist_i8, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)persist_i8_lds()));
    int dev = 0;
    DMET_HIP(hipGetDevice(&dev));
    DMET_HIP(hipDeviceGetAttribute(&g_ncu, hipDeviceAttributeMultiprocessorCount, dev));
    return DMET_OK;
}

template <int NS>
static dmet_status batch_enqueue(BatchPlan& bp, int variant, bool prof, hipStream_t st) {
    void* ws = bp.ws;
    const int nfrag = (int)bp.frags.size();
    BFrag* dfr = at<BFrag>(ws, bp.off_bfrag);
    auto k1 = k_xf1_batched<NS, XF1_NW>;
    auto k2 = k_xf2_batched<NS>;
    auto kc = variant == 128 ? k_contract_persist<NS, 128> : k_contract_persist<NS, 64>;
    const size_t lc = variant == 128 ? persist_lds<NS, 128>() : persist_lds<NS, 64>();
    auto scope = [&](const char* n) { return prof ? new ProfScope(n, st) : nullptr; };
    auto done = [&](ProfScope* p) {
        if (p) {
            p->stop();
            delete p;
        }
    };
    // 1. pack inputs
    ProfScope* ps = scope(NS == 3 ? "batch_pack_in_bf16x6" : "batch_pack_in_bf16x3");
    for (auto& G : bp.groups) {
        const int nk = G.mesh.nk;
        __bf16* plm = at<__bf16>(ws, G.off_plm);
        const int mb = pack_rows_per_block(G.ngv);
        const long nblk = (long)nk * nk * G.naux * ((G.nao_p + mb - 1) / mb);
        const size_t lds = pack_lds_bytes(mb, G.ngv);
        if (G.dt == DMET_C128)
            k_pack_lmunu<NS, double><<<dim3((unsigned)nblk), 256, lds, st>>>(
                static_cast<const double*>(G.lm), G.nao, G.nao_p, G.naux, G.ngv, mb, plm, G.mesh, 1);
        else
            k_pack_lmunu<NS, float><<<dim3((unsigned)nblk), 256, lds, st>>>(
                static_cast<const float*>(G.lm), G.nao, G.nao_p, G.naux, G.ngv, mb, plm, G.mesh, 1);
        for (int f : G.members) {
            const BatchFrag& F = bp.fs[f];
            k_pack_c1<NS><<<dim3((F.neo + 255) / 256, G.ngv, nk), 256, 0, st>>>(
                static_cast<const double*>(bp.frags[f].c_k), nk, 1, G.nao, F.neo, G.ngv, at<__bf16>(ws, G.off_pc1),
                F.col0, G.nbtot);
            k_pack_c2<NS><<<dim3((F.neo + 255) / 256, G.ng2, 1), 256, 0, st>>>(
                static_cast<const double*>(bp.frags[f].c_k), nk, G.nao, G.nao_p, F.neo, G.ng2,
                at<__bf16>(ws, F.off_pc2));
            {
                // groups zg .. ng2-1 of T pad odd group counts in stage 2: zero
                const int zg = nk * (G.nao_p / 8);
                const size_t n2 = (size_t)G.naux * F.neo, part = (size_t)G.ng2 * n2 * 8;
                __bf16* ptt = at<__bf16>(ws, F.off_ptt);
                for (int sp = 0; sp < P2 * NS; ++sp)
                    fill_zero(ptt + (size_t)sp * part + (size_t)zg * n2 * 8,
                              (size_t)(G.ng2 - zg) * n2 * 8 * sizeof(__bf16), st);
            }
        }
    }
    done(ps);
    DMET_LAUNCH_CHECK("batch pack");
    // 2. rounds of (stage 1 per group, stage 2 for all fragments)
    for (int r = 0; r < bp.rounds; ++r) {
        ps = scope(NS == 3 ? "batch_xform1_bf16x6" : "batch_xform1_bf16x3");
        for (auto& G : bp.groups) {
            if (r >= (int)G.qbs.size()) continue;
            const KSlots ks = kpair_slots(G.mesh, G.qbs[r].q);
            const long nb = ((long)(ks.npaired + ks.nself) * ((G.M1 + 127) / 128) * ((G.nbtot + 127) / 128) + NXCD - 1) /
                            NXCD * NXCD;
            k1<<<dim3((unsigned)nb), 64 * XF1_NW, xf1_lds<NS>(), st>>>(G.mesh, G.qbs[r].q, G.naux, G.nao_p, G.nbtot, G.ngv, ks,
                                                               at<int2>(ws, G.off_colmap), dfr,
                                                               at<__bf16>(ws, G.off_plm), at<__bf16>(ws, G.off_pc1));
        }
        done(ps);
        DMET_LAUNCH_CHECK("batch xform1");
        if (bp.items2_cnt[r] + bp.items2s_cnt[r] > 0) {
            ps = scope(NS == 3 ? "batch_xform2_bf16x6" : "batch_xform2_bf16x3");
            if (bp.items2_cnt[r] > 0) {
                const long nb = ((long)bp.items2_cnt[r] + NXCD - 1) / NXCD * NXCD;
                k2<<<dim3((unsigned)nb), 256, xf2_lds<NS>(), st>>>(bp.items2_cnt[r],
                                                                  at<BItem2>(ws, bp.off_items2) + bp.items2_off[r],
                                                                  dfr, at<BQ>(ws, bp.off_bq) + (size_t)r * nfrag);
                DMET_LAUNCH_CHECK("batch xform2");
            }
            if (bp.items2s_cnt[r] > 0) {
                const long nb = ((long)bp.items2s_cnt[r] + NXCD - 1) / NXCD * NXCD;
                k_xf2_batched_l4<NS><<<dim3((unsigned)nb), 256, xf2_l4_lds<NS>(), st>>>(
                    bp.items2s_cnt[r], at<BItem2>(ws, bp.off_items2) + bp.items2s_off[r], dfr,
                    at<BQ>(ws, bp.off_bq) + (size_t)r * nfrag);
                DMET_LAUNCH_CHECK("batch xform2 (32 x 32)");
            }
            done(ps);
        }
    }
    if (bp.prec == DMET_BF16X6_I8) {
        // 3. column scales and int8 digits of every fragment's Z, 4. persistent int8 contraction
        ps = scope("batch_pack_i8");
        fill_zero(at<unsigned>(ws, bp.off_cmax), bp.ncmax * sizeof(unsigned), st);
        for (int f = 0; f < nfrag; ++f) {
            const BatchFrag& F = bp.fs[f];
            const int rows_per = 256;
            unsigned* cm = at<unsigned>(ws, bp.off_cmax) + F.cmax_idx;
            k_colmax<<<dim3((F.npair + 255) / 256, (F.zrows + rows_per - 1) / rows_per), 256, 0, st>>>(
                at<float>(ws, F.off_z), (size_t)F.npair, F.zrows, F.npair, rows_per, cm);
            k_pack_i8<<<dim3((F.npair + 255) / 256, group_grid(F.kg16)), 256, 0, st>>>(
                at<float>(ws, F.off_z), (size_t)F.npair, F.zrows, F.npair, F.kg16, cm, at<int>(ws, F.off_ex),
                at<i4v>(ws, F.off_zp));
        }
        done(ps);
        DMET_LAUNCH_CHECK("batch pack i8");
        int* qd = at<int>(ws, bp.off_q);
        fill_zero(qd + 2 * NXCD, NXCD * sizeof(int), st);
        const int ncu = g_ncu > 0 ? g_ncu : 256;
        ps = scope("batch_contract_i8");
        k_contract_persist_i8<<<dim3((unsigned)(2 * ncu)), 256, persist_i8_lds(), st>>>(
            qd, qd + NXCD, qd + 2 * NXCD, at<BItemC>(ws, bp.off_itemsc), dfr);
        done(ps);
        DMET_LAUNCH_CHECK("batch contract i8");
        return DMET_OK;
    }
    // 3. split Z into bf16 parts
    ps = scope(NS == 3 ? "batch_pack_bf16x6" : "batch_pack_bf16x3");
    for (int f = 0; f < nfrag; ++f) {
        const BatchFrag& F = bp.fs[f];
        k_pack_parts<NS><<<dim3((F.npair + 255) / 256, group_grid(F.kgroups)), 256, 0, st>>>(
            at<float>(ws, F.off_z), (size_t)F.npair, F.zrows, F.npair, F.kgroups, at<__bf16>(ws, F.off_zp));
    }
    done(ps);
    DMET_LAUNCH_CHECK("batch pack parts");
    // 4. persistent contraction over every fragment's tiles
    int* qd = at<int>(ws, bp.off_q);   // [queue starts | queue lengths | counters], counters zeroed here
    fill_zero(qd + 2 * NXCD, NXCD * sizeof(int), st);
    const int ncu = g_ncu > 0 ? g_ncu : 256;
    ps = scope(NS == 3 ? "batch_contract_bf16x6" : "batch_contract_bf16x3");
    kc<<<dim3((unsigned)(2 * ncu)), 256, lc, st>>>(qd, qd + NXCD, qd + 2 * NXCD, at<BItemC>(ws, bp.off_itemsc), dfr,
                                                   FLUSH_K);
    done(ps);
    DMET_LAUNCH_CHECK("batch contract");
    return DMET_OK;
}

// Upload the tables of variant `variant` (synchronous).
static dmet_status batch_upload(BatchPlan& bp, int variant, hipStream_t st) {
    void* ws = bp.ws;
    const int nfrag = (int)bp.frags.size();
    for (int f = 0; f < nfrag; ++f) {
        const BatchFrag& F = bp.fs[f];
        const BatchGroup& G = bp.groups[F.group];
        BFrag b;
        b.pc2 = at<__bf16>(ws, F.off_pc2);
        b.ptt = at<__bf16>(ws, F.off_ptt);
        b.z = at<float>(ws, F.off_z);
        b.zp = at<__bf16>(ws, F.off_zp);
        b.eri = bp.frags[f].eri;
        b.neo = F.neo;
        b.naux = G.naux;
        b.ng2 = G.ng2;
        b.npair = F.npair;
        b.zrows = F.zrows;
        b.kgroups = F.kgroups;
        const bool i8 = bp.prec == DMET_BF16X6_I8;
        b.zp8 = i8 ? at<i4v>(ws, F.off_zp) : nullptr;
        b.cmax = i8 ? at<unsigned>(ws, bp.off_cmax) + F.cmax_idx : nullptr;
        b.ex = i8 ? at<int>(ws, F.off_ex) : nullptr;
        b.kg16 = F.kg16;
        bp.h_bfrag[f] = b;
    }
    const int v = variant == 128 ? 0 : 1;
    std::vector<int> q(2 * NXCD);
    for (int x = 0; x < NXCD; ++x) {
        q[x] = bp.h_qstart[v][x];
        q[NXCD + x] = bp.h_qlen[v][x];
    }
    DMET_HIP(hipMemcpyAsync(at<char>(ws, bp.off_bfrag), bp.h_bfrag.data(), sizeof(BFrag) * nfrag,
                            hipMemcpyHostToDevice, st));
    // the column maps of all groups are one contiguous region
    size_t cm0 = bp.groups[0].off_colmap;
    for (auto& G : bp.groups) cm0 = std::min(cm0, G.off_colmap);
    DMET_HIP(hipMemcpyAsync(at<char>(ws, cm0), bp.h_colmap.data(), sizeof(int2) * bp.h_colmap.size(),
                            hipMemcpyHostToDevice, st));
    if (!bp.h_items2.empty())
        DMET_HIP(hipMemcpyAsync(at<char>(ws, bp.off_items2), bp.h_items2.data(), sizeof(BItem2) * bp.h_items2.size(),
                                hipMemcpyHostToDevice, st));
    DMET_HIP(hipMemcpyAsync(at<char>(ws, bp.off_bq), bp.h_bq.data(), sizeof(BQ) * bp.h_bq.size(),
                            hipMemcpyHostToDevice, st));
    if (!bp.h_itemsc[v].empty())
        DMET_HIP(hipMemcpyAsync(at<char>(ws, bp.off_itemsc), bp.h_itemsc[v].data(),
                                sizeof(BItemC) * bp.h_itemsc[v].size(), hipMemcpyHostToDevice, st));
    DMET_HIP(hipMemcpyAsync(at<char>(ws, bp.off_q), q.data(), sizeof(int) * 2 * NXCD, hipMemcpyHostToDevice, st));
    DMET_HIP(hipStreamSynchronize(st));
    return DMET_OK;
}

// FP64 and FP32-3M batches run the per-fragment drivers on NBR concurrent
// branches (internal streams forked from and joined to the caller's stream by
// events): fragments go largest first to the branch with the least work so
// far, and each branch has a workspace slice of its own.  With
// DMET_BATCH_GRAPH the fork / join is captured once per plan and replayed.
constexpr int NBR = 4;

struct LoopPlan {
    std::vector<std::vector<int>> branch;   // fragment indices per branch, in run order
    std::vector<size_t> off;                // workspace offset per branch
    size_t bytes = 0;
    hipGraphExec_t exec = nullptr;
};

static EriPlan frag_plan(const dmet_fragment& f, dmet_precision prec) {
    dmet_lattice lat = f.lat;
    lat.nspin = 1;
    return make_eri_plan(&lat, f.neo, prec, f.dtype);
}

static void plan_loop(int nfrag, const dmet_fragment* frags, dmet_precision prec, LoopPlan& lp) {
    std::vector<double> cost(nfrag);
    std::vector<int> order(nfrag);
    for (int f = 0; f < nfrag; ++f) {
        const double nk = (double)frags[f].lat.kmesh[0] * frags[f].lat.kmesh[1] * frags[f].lat.kmesh[2];
        const double nao = frags[f].lat.nao, naux = frags[f].lat.naux, neo = frags[f].neo;
        const double npair = neo * (neo + 1) / 2;
        cost[f] = nk * nk * naux * nao * neo * (nao + neo) + nk * naux * npair * npair;   // transform + contraction
        order[f] = f;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    const int nb = std::min(NBR, std::max(1, nfrag));
    lp.branch.assign(nb, {});
    std::vector<double> load(nb, 0.0);
    std::vector<size_t> ws(nb, 256);
    for (int f : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lp.branch[b].push_back(f);
        load[b] += cost[f];
        const EriPlan p = frag_plan(frags[f], prec);
        ws[b] = std::max(ws[b], prec == DMET_FP64 ? eri_f64_workspace(p) : eri_f32_workspace(p));
    }
    lp.off.assign(nb, 0);
    size_t cur = 0;
    for (int b = 0; b < nb; ++b) {
        lp.off[b] = cur;
        cur += (ws[b] + 255) & ~size_t(255);
    }
    lp.bytes = cur;
}

static std::map<std::string, LoopPlan*> g_loop_plans;

// branch streams and events of the current device (created once, default priority)
struct Branches {
    hipStream_t st[NBR] = {};
    hipEvent_t fork = nullptr, join[NBR] = {};
};

static dmet_status branches_of_device(Branches*& out) {
    static Branches per_dev[64];
    static bool made[64] = {};
    int dev = 0;
    DMET_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(DMET_E_UNSUPPORTED, "device index above 63");
    Branches& b = per_dev[dev];
    if (!made[dev]) {
        for (int i = 0; i < NBR; ++i) {
            DMET_HIP(hipStreamCreateWithFlags(&b.st[i], hipStreamNonBlocking));
            DMET_HIP(hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming));
        }
        DMET_HIP(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
        made[dev] = true;
    }
    out = &b;
    return DMET_OK;
}

static dmet_status loop_enqueue(int nfrag, const dmet_fragment* frags, dmet_precision prec, const LoopPlan& lp,
                                void* ws, Branches& br, hipStream_t st) {
    (void)nfrag;
    DMET_HIP(hipEventRecord(br.fork, st));
    dmet_status s = DMET_OK;
    size_t forked = 0;
    for (size_t b = 0; b < lp.branch.size() && s == DMET_OK; ++b) {
        hipStream_t bs = br.st[b];
        DMET_HIP(hipStreamWaitEvent(bs, br.fork, 0));
        ++forked;
        void* slice = static_cast<char*>(ws) + lp.off[b];
        const size_t cap = (b + 1 < lp.branch.size() ? lp.off[b + 1] : lp.bytes) - lp.off[b];
        for (int f : lp.branch[b]) {
            const EriPlan p = frag_plan(frags[f], prec);
            const double* ckf = static_cast<const double*>(frags[f].c_k);
            s = prec == DMET_FP64 ? eri_f64(p, frags[f].lmunu, ckf, frags[f].eri, nullptr, nullptr, slice, cap, bs)
                                  : eri_f32(p, frags[f].lmunu, ckf, frags[f].eri, nullptr, nullptr, slice, cap, bs);
            if (s != DMET_OK) break;
        }
    }
    // every forked branch joins the caller's stream, also after an error, so
    // that later work on `stream` is ordered after whatever was enqueued
    for (size_t b = 0; b < forked; ++b) {
        DMET_HIP(hipEventRecord(br.join[b], br.st[b]));
        DMET_HIP(hipStreamWaitEvent(st, br.join[b], 0));
    }
    return s;
}

size_t batch_workspace(int nfrag, const dmet_fragment* frags, dmet_precision prec) {
    if (prec == DMET_FP64 || prec == DMET_FP32_3M) {
        LoopPlan lp;
        plan_loop(nfrag, frags, prec, lp);
        return lp.bytes;
    }
    BatchPlan bp;
    bp.frags.assign(frags, frags + nfrag);
    bp.prec = prec;
    plan_batch(bp);
    return bp.bytes;
}

static std::string tune_file() {
    const char* e = getenv("DMET_TUNE_CACHE");
    return e ? std::string(e) : std::string();
}

static void tune_load() {
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    std::string fn = tune_file();
    if (fn.empty()) return;
    FILE* fp = fopen(fn.c_str(), "r");
    if (!fp) return;
    char line[65536];
    while (fgets(line, sizeof(line), fp)) {
        char* sp = strrchr(line, ' ');
        if (!sp) continue;
        int v = atoi(sp + 1);
        *sp = 0;
        if (v == 64 || v == 128) g_tune[line] = v;
    }
    fclose(fp);
}

static void tune_store(const std::string& key, int v, float ms128, float ms64) {
    std::string fn = tune_file();
    if (fn.empty()) return;
    FILE* fp = fopen(fn.c_str(), "a");
    if (!fp) return;
    fprintf(fp, "%s %d\n", key.c_str(), v);
    fclose(fp);
    (void)ms128;
    (void)ms64;
}

dmet_status eri_batched(int nfrag, const dmet_fragment* frags, dmet_precision prec, unsigned flags, void* ws,
                        size_t ws_bytes, hipStream_t st) {
    if (prec == DMET_FP64 || prec == DMET_FP32_3M) {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        const std::string key = batch_key(nfrag, frags, prec, true, ws, ws_bytes);
        LoopPlan* lp = nullptr;
        auto it = g_loop_plans.find(key);
        if (it != g_loop_plans.end()) {
            lp = it->second;
        } else {
            lp = new LoopPlan();
            plan_loop(nfrag, frags, prec, *lp);
            if (lp->bytes > ws_bytes) {
                delete lp;
                return fail(DMET_E_WORKSPACE, "batched workspace too small");
            }
            if (g_loop_plans.size() >= 32) {   // bounded cache of plans / captured graphs
                for (auto& kv : g_loop_plans) {
                    if (kv.second->exec) (void)hipGraphExecDestroy(kv.second->exec);
                    delete kv.second;
                }
                g_loop_plans.clear();
            }
            g_loop_plans[key] = lp;
        }
        Branches* br = nullptr;
        {
            dmet_status s = branches_of_device(br);
            if (s != DMET_OK) return s;
            s = prec == DMET_FP64 ? eri_f64_prepare() : eri_f32_prepare();
            if (s != DMET_OK) return s;
        }
        if (!(flags & DMET_BATCH_GRAPH)) return loop_enqueue(nfrag, frags, prec, *lp, ws, *br, st);
        if (!lp->exec) {
            // capture on a private stream (the caller's may be the legacy null
            // stream, which cannot be captured); nothing executes during capture
            static hipStream_t cap = nullptr;
            if (!cap) DMET_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            const bool was = prof_suspend(true);
            DMET_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            dmet_status s = loop_enqueue(nfrag, frags, prec, *lp, ws, *br, cap);
            hipError_t e = hipStreamEndCapture(cap, &g);
            prof_suspend(was);
            if (s != DMET_OK) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&lp->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        }
        ProfScope ps("batch_graph", st);
        DMET_HIP(hipGraphLaunch(lp->exec, st));
        ps.stop();
        return DMET_OK;
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    const std::string key = batch_key(nfrag, frags, prec, true, ws, ws_bytes);
    BatchPlan* bp = nullptr;
    auto itp = g_batch_plans.find(key);
    if (itp != g_batch_plans.end()) {
        bp = itp->second;
    } else {
        bp = new BatchPlan();
        bp->frags.assign(frags, frags + nfrag);
        bp->prec = prec;
        bp->ws = ws;
        bp->ws_bytes = ws_bytes;
        bp->key = key;
        plan_batch(*bp);
        if (bp->bytes > ws_bytes) {
            delete bp;
            return fail(DMET_E_WORKSPACE, "batched workspace too small");
        }
        if (g_batch_plans.size() >= 32) {  // bounded cache of plans / captured graphs
            for (auto& kv : g_batch_plans) {
                if (kv.second->exec) (void)hipGraphExecDestroy(kv.second->exec);
                delete kv.second;
            }
            g_batch_plans.clear();
        }
        g_batch_plans[key] = bp;
    }
    const bool ns3 = prec != DMET_BF16X3_3M;
    {
        dmet_status s = ns3 ? batch_prepare<3>() : batch_prepare<2>();
        if (s != DMET_OK) return s;
    }
    auto enqueue = [&](int variant, bool prof) {
        return ns3 ? batch_enqueue<3>(*bp, variant, prof, st) : batch_enqueue<2>(*bp, variant, prof, st);
    };
    // contraction tile: cached choice, autotune, or default
    tune_load();
    const std::string shape = batch_key(nfrag, frags, prec, false, nullptr, 0);
    int variant = 128;
    auto itt = g_tune.find(shape);
    if (prec == DMET_BF16X6_I8) {
        // one contraction variant (128 x 128 tiles) in the int8 form: nothing to tune
    } else if (itt != g_tune.end()) {
        variant = itt->second;
    } else if (flags & DMET_BATCH_AUTOTUNE) {
        float best = 1e30f;
        float ms[2] = {0.f, 0.f};
        for (int v : {128, 64}) {
            dmet_status s = batch_upload(*bp, v, st);
            if (s != DMET_OK) return s;
            hipEvent_t e0, e1;
            DMET_HIP(hipEventCreate(&e0));
            DMET_HIP(hipEventCreate(&e1));
            DMET_HIP(hipEventRecord(e0, st));
            s = enqueue(v, false);
            if (s != DMET_OK) return s;
            DMET_HIP(hipEventRecord(e1, st));
            DMET_HIP(hipEventSynchronize(e1));
            float t = 0.f;
            DMET_HIP(hipEventElapsedTime(&t, e0, e1));
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            ms[v == 128 ? 0 : 1] = t;
            if (t < best) {
                best = t;
                variant = v;
            }
        }
        g_tune[shape] = variant;
        tune_store(shape, variant, ms[0], ms[1]);
    }
    // The work tables live in the caller's workspace, whose contents the caller
    // may reuse between calls: upload them on every call (a few MB, before any
    // kernel of this call), graph replays included.
    if (bp->variant != variant && bp->exec) {
        (void)hipGraphExecDestroy(bp->exec);
        bp->exec = nullptr;
    }
    bp->variant = variant;
    {
        dmet_status s = batch_upload(*bp, variant, st);
        if (s != DMET_OK) return s;
    }
    if (flags & DMET_BATCH_GRAPH) {
        if (!bp->exec) {
            // capture on a private stream (the caller's may be the legacy null
            // stream, which cannot be captured); nothing executes during capture
            static hipStream_t cap = nullptr;
            if (!cap) DMET_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            DMET_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            dmet_status s = ns3 ? batch_enqueue<3>(*bp, variant, false, cap) : batch_enqueue<2>(*bp, variant, false, cap);
            hipError_t e = hipStreamEndCapture(cap, &g);
            if (s != DMET_OK) return s;
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&bp->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        }
        ProfScope ps("batch_graph", st);
        DMET_HIP(hipGraphLaunch(bp->exec, st));
        ps.stop();
        return DMET_OK;
    }
    return enqueue(variant, true);
}

}  // namespace dmet
