// Double-counting-corrected embedding Fock matrix (Eq. "fock double counting")
// from the density-fitting factors of the embedding ERIs:
//   (ij|kl)_st = sum_P Z_s[P][ij] Z_t[P][kl]          (pairs packed, i >= j)
//   J_s[ij] = sum_t sum_kl (ij|kl)_st g_t,lk  = sum_P Z_s[P][ij] v[P],
//             v[P] = sum_t sum_{k>=l} Z_t[P][kl] g_t,kl (2 - delta_kl)
//   K_s[ij] = sum_kl (ik|lj)_ss g_s,kl = sum_P (Z_s[P] g_s Z_s[P])_ij
//   F~_s = F_s - (J_s - K_s)            (per-spin densities)
// For nspin = 1 the densities are per spin and the paper's spin-summed
// gamma = 2 g, so F~ = F - (J(gamma) - K(gamma)/2) = F - (2 J(g) - K(g)).
// FP64 throughout: vector arithmetic for J, FP64 MFMA GEMMs for K.
#include "common.h"
#include "eri.h"
#include "mfma_f64.h"

#include <algorithm>

namespace dmet {

__device__ inline size_t pidx(int i, int j) {
    return i >= j ? (size_t)i * (i + 1) / 2 + j : (size_t)j * (j + 1) / 2 + i;
}

// v[P] += scale * sum_{k>=l} Z[P][kl] g_kl (2 - delta_kl); one wave per row P
__global__ void k_dc_v(int nrows, int neo, int npair, const double* __restrict__ z, const double* __restrict__ g,
                       double scale, double* __restrict__ v) {
    const int lane = threadIdx.x & 63;
    const int P = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (P >= nrows) return;
    const double* zr = z + (size_t)P * npair;
    double acc = 0.0;
    for (int kl = lane; kl < npair; kl += 64) {
        int k = (int)((sqrt(8.0 * kl + 1.0) - 1.0) * 0.5);
        while ((size_t)k * (k + 1) / 2 > (size_t)kl) --k;
        while ((size_t)(k + 1) * (k + 2) / 2 <= (size_t)kl) ++k;
        const int l = kl - k * (k + 1) / 2;
        acc += zr[kl] * g[(size_t)k * neo + l] * (k == l ? 1.0 : 2.0);
    }
    acc = wave_sum(acc);
    if (lane == 0) v[P] += scale * acc;
}

// J[ij] = sum_P Z[P][ij] v[P] for pair columns (one thread per pair, loop over P
// in order; eight rows' loads in flight per thread)
__global__ void k_dc_j(int nrows, int npair, const double* __restrict__ z, const double* __restrict__ v,
                       double* __restrict__ jp) {
    const int kl = blockIdx.x * blockDim.x + threadIdx.x;
    if (kl >= npair) return;
    double acc = 0.0;
    int P = 0;
    for (; P + 8 <= nrows; P += 8) {
        double zv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) zv[u] = z[(size_t)(P + u) * npair + kl];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += zv[u] * v[P + u];
    }
    for (; P < nrows; ++P) acc += z[(size_t)P * npair + kl] * v[P];
    jp[kl] = acc;
}

// Exchange K_s = sum_P Z_P g Z_P (Z_P the symmetric neo x neo matrix of row P)
// as two FP64 MFMA GEMMs over chunks of rows P:
//   W[(P,i)][l] = sum_k Z_P[i][k] g[k][l]                       (k_dc_w)
//   K[i][j]    += sum_{P,l} W[(P,i)][l] Z_P[l][j]                (k_dc_k)
// K is symmetric, so k_dc_k forms only the 64 x 64 tiles with it >= jt.  Each
// workgroup of k_dc_k reduces DK_PCW rows P into a partial tile of its own;
// k_dc_final sums the partials in a fixed order (deterministic result).
// Both GEMMs gather the next DBK-deep slice of their operands into registers
// while the MFMAs run on the current one, into a double-buffered LDS tile.
// The gathers load from clamped, always valid indices with no condition (the
// zero padding is applied when the slice is stored), and the row-dependent
// parts of the addresses are computed once per workgroup.
constexpr int DT = 64, DBK = 16;
constexpr int DNE = DBK * DT / 256;              // slice elements per thread and operand
constexpr int DK_PCW = 16;                       // rows P per k_dc_k workgroup
constexpr size_t DW_CAP = size_t(1) << 30;       // bytes of W per chunk of rows P

__global__ void __launch_bounds__(256) k_dc_w(long p0, int np, int neo, int npair, const double* __restrict__ z,
                                               const double* __restrict__ g, double* __restrict__ w) {
    using T = F64Tile<DT, DT, DBK>;
    __shared__ double As[2][DBK * T::LDA];
    __shared__ double Bs[2][DBK * T::LDB];
    const long M = (long)np * neo;
    const int n0 = blockIdx.x * DT;          // x fastest: tiles sharing A run together
    const long m0 = (long)blockIdx.y * DT;
    d4 acc[DT / 32][DT / 32];
    zero_acc<DT, DT>(acc);
    const int tid = threadIdx.x;
    double ra[DNE], rb[DNE];
    const double* zrow[DNE];   // row P of Z for this thread's A rows m (clamped)
    int irow[DNE];             // i = m mod neo
#pragma unroll
    for (int u = 0; u < DNE; ++u) {
        const long m = std::min(m0 + (tid + u * 256) / DBK, M - 1);
        zrow[u] = z + (p0 + m / neo) * npair;
        irow[u] = (int)(m % neo);
    }
    auto gather = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < DNE; ++u) {
            const int kk = (tid + u * 256) % DBK;
            ra[u] = zrow[u][pidx(irow[u], min(k0 + kk, neo - 1))];
        }
#pragma unroll
        for (int u = 0; u < DNE; ++u) {
            const int e = tid + u * 256, nn = e % DT, kk = e / DT;
            rb[u] = g[(size_t)min(k0 + kk, neo - 1) * neo + min(n0 + nn, neo - 1)];
        }
    };
    auto stash = [&](int k0, int b) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < DNE; ++u) {
            const int e = tid + u * 256;
            const int ka = k0 + e % DBK, kb = k0 + e / DT;
            As[b][(e % DBK) * T::LDA + e / DBK] = (m0 + e / DBK < M && ka < neo) ? ra[u] : 0.0;
            Bs[b][(e / DT) * T::LDB + e % DT] = (kb < neo && n0 + e % DT < neo) ? rb[u] : 0.0;
        }
    };
    const int nkt = (neo + DBK - 1) / DBK;
    gather(0);
    stash(0, 0);
    __syncthreads();
    for (int it = 0; it < nkt; ++it) {
        if (it + 1 < nkt) gather((it + 1) * DBK);
        f64_mma<DT, DT, DBK>(As[it & 1], Bs[it & 1], acc);
        if (it + 1 < nkt) stash((it + 1) * DBK, (it + 1) & 1);
        __syncthreads();
    }
    f64_visit<DT, DT, DBK>(acc, [&](int r, int c, double v) {
        const long m = m0 + r;
        const int l = n0 + c;
        if (m < M && l < neo) w[m * neo + l] = v;
    });
}

// partial tile (split0 + blockIdx.y, tri) over rows P in
// [p0 + DK_PCW * blockIdx.y, min(p0 + np, ... + DK_PCW)); W rows are chunk-local
__global__ void __launch_bounds__(256) k_dc_k(long p0, int np, int neo, int npair, int ntri, long split0,
                                               const double* __restrict__ z, const double* __restrict__ w,
                                               double* __restrict__ part) {
    using T = F64Tile<DT, DT, DBK>;
    __shared__ double As[2][DBK * T::LDA];
    __shared__ double Bs[2][DBK * T::LDB];
    const int tri = blockIdx.x;
    int it = (int)((sqrt(8.0 * tri + 1.0) - 1.0) * 0.5);
    while (it * (it + 1) / 2 > tri) --it;
    while ((it + 1) * (it + 2) / 2 <= tri) ++it;
    const int jt = tri - it * (it + 1) / 2;
    const int i0 = it * DT, j0 = jt * DT;
    const int pl0 = blockIdx.y * DK_PCW;                       // chunk-local first row
    const int npl = min(DK_PCW, np - pl0);
    const int R = npl * neo;                                   // reduction length (P, l)
    d4 acc[DT / 32][DT / 32];
    zero_acc<DT, DT>(acc);
    const int tid = threadIdx.x;
    double ra[DNE], rb[DNE];
    const float rneo = 1.0f / (float)neo;
    // (r / neo, r mod neo) for 0 <= r < 2^24: float quotient, corrected by one step
    auto divmod = [&](int r, int& q, int& l) __attribute__((always_inline)) {
        q = (int)((float)r * rneo);
        l = r - q * neo;
        if (l < 0) {
            --q;
            l += neo;
        } else if (l >= neo) {
            ++q;
            l -= neo;
        }
    };
    const double* wrow = w + ((size_t)pl0 * neo) * neo;
    const double* zrow = z + (p0 + pl0) * npair;
    auto gather = [&](int r0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < DNE; ++u) {
            const int e = tid + u * 256, kk = e % DBK, mm = e / DBK;
            int pl, l;
            divmod(min(r0 + kk, R - 1), pl, l);
            ra[u] = wrow[((size_t)pl * neo + min(i0 + mm, neo - 1)) * neo + l];
        }
#pragma unroll
        for (int u = 0; u < DNE; ++u) {
            const int e = tid + u * 256, nn = e % DT, kk = e / DT;
            int pl, l;
            divmod(min(r0 + kk, R - 1), pl, l);
            rb[u] = zrow[(size_t)pl * npair + pidx(l, min(j0 + nn, neo - 1))];
        }
    };
    auto stash = [&](int r0, int b) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < DNE; ++u) {
            const int e = tid + u * 256;
            const int ra_r = r0 + e % DBK, rb_r = r0 + e / DT;
            As[b][(e % DBK) * T::LDA + e / DBK] = (ra_r < R && i0 + e / DBK < neo) ? ra[u] : 0.0;
            Bs[b][(e / DT) * T::LDB + e % DT] = (rb_r < R && j0 + e % DT < neo) ? rb[u] : 0.0;
        }
    };
    const int nkt = (R + DBK - 1) / DBK;
    gather(0);
    stash(0, 0);
    __syncthreads();
    for (int it = 0; it < nkt; ++it) {
        if (it + 1 < nkt) gather((it + 1) * DBK);
        f64_mma<DT, DT, DBK>(As[it & 1], Bs[it & 1], acc);
        if (it + 1 < nkt) stash((it + 1) * DBK, (it + 1) & 1);
        __syncthreads();
    }
    double* out = part + ((size_t)(split0 + blockIdx.y) * ntri + tri) * (DT * DT);
    f64_visit<DT, DT, DBK>(acc, [&](int r, int c, double v) { out[r * DT + c] = v; });
}

// F~[s][i][j] = F[s][i][j] - (cj * J_s[pair(i,j)] - K_s[i][j]); K_s[i][j] is the
// ordered sum of the partial tiles holding (max, min) of (i, j) by tile
__global__ void k_dc_final(int neo, int ntri, long nsplit, const double* __restrict__ f,
                           const double* __restrict__ jp, const double* __restrict__ part, double cj,
                           double* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= neo * neo) return;
    int i = e / neo, j = e % neo;
    const double jv = jp[pidx(i, j)];
    if (i / DT < j / DT) {
        const int t = i;
        i = j;
        j = t;
    }
    const int it = i / DT, jt = j / DT;
    const size_t off = (size_t)(it * (it + 1) / 2 + jt) * (DT * DT) + (i % DT) * DT + (j % DT);
    double k = 0.0;
    for (long s = 0; s < nsplit; ++s) k += part[(size_t)s * ntri * (DT * DT) + off];
    out[e] = f[e] - (cj * jv - k);
}

static int dc_rows_per_chunk(int neo, int nrows) {
    const size_t per = (size_t)neo * neo * sizeof(double);
    // W bytes per chunk within DW_CAP, and at most 65535 row tiles in grid y
    long rc = std::min<long>((long)(DW_CAP / per), 65535L * DT / neo) / DK_PCW * DK_PCW;
    if (rc < DK_PCW) rc = DK_PCW;
    return (int)std::min<long>(rc, nrows);
}

static long dc_nsplit(int neo, int nrows) {
    const int rc = dc_rows_per_chunk(neo, nrows);
    long n = 0;
    for (long p0 = 0; p0 < nrows; p0 += rc) n += (std::min<long>(rc, nrows - p0) + DK_PCW - 1) / DK_PCW;
    return n;
}

size_t fock_dc_workspace(int nspin, int neo, int nrows) {
    const size_t npair = (size_t)neo * (neo + 1) / 2;
    const int nt = (neo + DT - 1) / DT;
    const size_t ntri = (size_t)nt * (nt + 1) / 2;
    Carve cv(nullptr, 0);
    cv.take<double>(nrows);                                              // v
    cv.take<double>((size_t)nspin * npair);                              // J per spin
    cv.take<double>((size_t)dc_rows_per_chunk(neo, nrows) * neo * neo);  // W of one chunk
    cv.take<double>((size_t)dc_nsplit(neo, nrows) * ntri * DT * DT);     // partial K tiles
    return cv.bytes();
}

dmet_status fock_dc(int nspin, int neo, int nrows, const double* z, const double* f_eo, const double* dm_eo,
                    double* f_tilde, void* ws, size_t ws_bytes, hipStream_t st) {
    const int npair = neo * (neo + 1) / 2;
    const int nt = (neo + DT - 1) / DT, ntri = nt * (nt + 1) / 2;
    const int rc = dc_rows_per_chunk(neo, nrows);
    const long nsplit = dc_nsplit(neo, nrows);
    Carve cv(ws, ws_bytes);
    double* v = cv.take<double>(nrows);
    double* jp = cv.take<double>((size_t)nspin * npair);
    double* w = cv.take<double>((size_t)rc * neo * neo);
    double* part = cv.take<double>((size_t)nsplit * ntri * DT * DT);
    if (cv.bytes() > ws_bytes) return fail(DMET_E_WORKSPACE, "fock_dc workspace too small");
    const size_t zs = (size_t)nrows * npair, gs = (size_t)neo * neo;
    fill_zero(v, nrows * sizeof(double), st);
    ProfScope ps("fock_dc", st);
    // Coulomb: one density vector over all spins (the alpha-beta block is Z_a^T Z_b)
    for (int t = 0; t < nspin; ++t)
        k_dc_v<<<(nrows + 3) / 4, 256, 0, st>>>(nrows, neo, npair, z + t * zs, dm_eo + t * gs, 1.0, v);
    for (int s = 0; s < nspin; ++s)
        k_dc_j<<<(npair + 255) / 256, 256, 0, st>>>(nrows, npair, z + s * zs, v, jp + (size_t)s * npair);
    const double cj = nspin == 1 ? 2.0 : 1.0;
    for (int s = 0; s < nspin; ++s) {
        long split = 0;
        for (long p0 = 0; p0 < nrows; p0 += rc) {
            const int np = (int)std::min<long>(rc, nrows - p0);
            const long mt = ((long)np * neo + DT - 1) / DT;
            k_dc_w<<<dim3(nt, (unsigned)mt), 256, 0, st>>>(p0, np, neo, npair, z + s * zs, dm_eo + s * gs, w);
            const int nsp = (np + DK_PCW - 1) / DK_PCW;
            k_dc_k<<<dim3(ntri, nsp), 256, 0, st>>>(p0, np, neo, npair, ntri, split, z + s * zs, w, part);
            split += nsp;
        }
        k_dc_final<<<(neo * neo + 255) / 256, 256, 0, st>>>(neo, ntri, nsplit, f_eo + s * gs, jp + (size_t)s * npair,
                                                            part, cj, f_tilde + s * gs);
    }
    ps.stop();
    DMET_LAUNCH_CHECK("fock_dc");
    return DMET_OK;
}

// Mean-field energy of the embedding Hamiltonian with the Hartree-Fock
// expression: since F^EO = F~ + J - K/2 at the same density, the one- and
// two-body terms combine into E = 1/2 sum_s sum_ij (F~_s + F_s)_ij gamma_s,ji
// with the spin-summed gamma (restricted: gamma = 2 g, so E = sum (F~ + F) g;
// unrestricted: per-spin g and the factor 1/2).  One workgroup, fixed order.
__global__ void __launch_bounds__(1024) k_energy_mf(int nspin, int neo, const double* __restrict__ ft,
                                                    const double* __restrict__ f, const double* __restrict__ g,
                                                    double* __restrict__ e) {
    __shared__ double part[16];
    double acc = 0.0;
    const size_t per = (size_t)neo * neo;
    for (size_t x = threadIdx.x; x < (size_t)nspin * per; x += blockDim.x) {
        const size_t sp = x / per, ij = x % per, i = ij / neo, j = ij % neo;
        acc += (ft[x] + f[x]) * g[sp * per + j * neo + i];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        e[0] = (nspin == 1 ? 1.0 : 0.5) * t;
    }
}

dmet_status energy_mf(int nspin, int neo, const double* f_tilde, const double* f_eo, const double* dm_eo,
                      double* e, hipStream_t st) {
    k_energy_mf<<<1, 1024, 0, st>>>(nspin, neo, f_tilde, f_eo, dm_eo, e);
    DMET_LAUNCH_CHECK("k_energy_mf");
    return DMET_OK;
}

}  // namespace dmet
