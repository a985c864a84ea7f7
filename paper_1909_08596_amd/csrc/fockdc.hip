// Double-counting-corrected embedding Fock matrix (Eq. "fock double counting")
// from the density-fitting factors of the embedding ERIs:
//   (ij|kl)_st = sum_P Z_s[P][ij] Z_t[P][kl]          (pairs packed, i >= j)
//   J_s[ij] = sum_t sum_kl (ij|kl)_st g_t,lk  = sum_P Z_s[P][ij] v[P],
//             v[P] = sum_t sum_{k>=l} Z_t[P][kl] g_t,kl (2 - delta_kl)
//   K_s[ij] = sum_kl (ik|lj)_ss g_s,kl = sum_P (Z_s[P] g_s Z_s[P])_ij
//   F~_s = F_s - (J_s - K_s)            (per-spin densities)
// For nspin = 1 the densities are per spin and the paper's spin-summed
// gamma = 2 g, so F~ = F - (J(gamma) - K(gamma)/2) = F - (2 J(g) - K(g)).
// FP64 vector arithmetic throughout (a few percent of the ERI build).
#include "common.h"
#include "eri.h"

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

// J[ij] = sum_P Z[P][ij] v[P] for pair columns (one thread per pair, loop over P)
__global__ void k_dc_j(int nrows, int npair, const double* __restrict__ z, const double* __restrict__ v,
                       double* __restrict__ jp) {
    const int kl = blockIdx.x * blockDim.x + threadIdx.x;
    if (kl >= npair) return;
    double acc = 0.0;
    for (int P = 0; P < nrows; ++P) acc += z[(size_t)P * npair + kl] * v[P];
    jp[kl] = acc;
}

// K[i][j] += sum_{P in chunk} sum_l W_P[i][l] Z_P[l][j] with W_P = Z_P g.
// A workgroup owns DC_T rows i of K (all columns j) and a chunk of rows P:
// per P it stages Z_P(i, :) in LDS, forms W_P(i, :) in LDS once, then each
// thread accumulates its (i, j) entries in registers; the chunk's partial rows
// are added to K with FP64 atomics.
constexpr int DC_T = 16;
constexpr int DC_MAXJ = 32;   // columns per thread: neo <= 16 * DC_MAXJ

__global__ void __launch_bounds__(256) k_dc_k(int nrows, int neo, int npair, int pchunk,
                                               const double* __restrict__ z, const double* __restrict__ g,
                                               double* __restrict__ kmat) {
    extern __shared__ double sh[];
    double* zi = sh;                        // [DC_T][neo]  Z_P(i0 + r, k)
    double* wi = zi + DC_T * neo;           // [DC_T][neo]  W_P(i0 + r, l)
    const int i0 = blockIdx.x * DC_T;
    const int p0 = blockIdx.y * pchunk, p1 = min(nrows, p0 + pchunk);
    const int tid = threadIdx.x, r = tid / 16, jl = tid % 16;
    double acc[DC_MAXJ];
#pragma unroll
    for (int c = 0; c < DC_MAXJ; ++c) acc[c] = 0.0;
    for (int P = p0; P < p1; ++P) {
        const double* zr = z + (size_t)P * npair;
        __syncthreads();
        for (int e = tid; e < DC_T * neo; e += 256) {
            const int rr = e / neo, k = e % neo;
            zi[e] = (i0 + rr < neo) ? zr[pidx(i0 + rr, k)] : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < DC_T * neo; e += 256) {
            const int rr = e / neo, l = e % neo;
            double s = 0.0;
            for (int k = 0; k < neo; ++k) s += zi[rr * neo + k] * g[(size_t)k * neo + l];
            wi[e] = s;
        }
        __syncthreads();
        const double* w = wi + r * neo;
#pragma unroll
        for (int c = 0; c < DC_MAXJ; ++c) {
            const int j = jl + 16 * c;
            if (j < neo) {
                double s = 0.0;
                for (int l = 0; l < neo; ++l) s += w[l] * zr[pidx(l, j)];
                acc[c] += s;
            }
        }
    }
    if (i0 + r < neo) {
#pragma unroll
        for (int c = 0; c < DC_MAXJ; ++c) {
            const int j = jl + 16 * c;
            if (j < neo) atomicAdd(&kmat[(size_t)(i0 + r) * neo + j], acc[c]);
        }
    }
}

// F~[s][i][j] = F[s][i][j] - (cj * J_s[pair(i,j)] - ck * K_s[i][j])
__global__ void k_dc_final(int neo, const double* __restrict__ f, const double* __restrict__ jp,
                           const double* __restrict__ kmat, double cj, double ck, double* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= neo * neo) return;
    const int i = e / neo, j = e % neo;
    out[e] = f[e] - (cj * jp[pidx(i, j)] - ck * kmat[e]);
}

size_t fock_dc_workspace(int nspin, int neo, int nrows) {
    const size_t npair = (size_t)neo * (neo + 1) / 2;
    Carve cv(nullptr, 0);
    cv.take<double>(nrows);                       // v
    cv.take<double>((size_t)nspin * npair);       // J per spin
    cv.take<double>((size_t)nspin * neo * neo);   // K per spin
    return cv.bytes();
}

dmet_status fock_dc(int nspin, int neo, int nrows, const double* z, const double* f_eo, const double* dm_eo,
                    double* f_tilde, void* ws, size_t ws_bytes, hipStream_t st) {
    const int npair = neo * (neo + 1) / 2;
    Carve cv(ws, ws_bytes);
    double* v = cv.take<double>(nrows);
    double* jp = cv.take<double>((size_t)nspin * npair);
    double* km = cv.take<double>((size_t)nspin * neo * neo);
    if (cv.bytes() > ws_bytes) return fail(DMET_E_WORKSPACE, "fock_dc workspace too small");
    const size_t zs = (size_t)nrows * npair, gs = (size_t)neo * neo;
    fill_zero(v, nrows * sizeof(double), st);
    fill_zero(km, nspin * gs * sizeof(double), st);
    ProfScope ps("fock_dc", st);
    // Coulomb: one density vector over all spins (the alpha-beta block is Z_a^T Z_b)
    for (int t = 0; t < nspin; ++t)
        k_dc_v<<<(nrows + 3) / 4, 256, 0, st>>>(nrows, neo, npair, z + t * zs, dm_eo + t * gs, 1.0, v);
    for (int s = 0; s < nspin; ++s)
        k_dc_j<<<(npair + 255) / 256, 256, 0, st>>>(nrows, npair, z + s * zs, v, jp + (size_t)s * npair);
    const int pchunk = 32;
    const size_t shm = (size_t)2 * DC_T * neo * sizeof(double);
    if (neo > 16 * DC_MAXJ) return fail(DMET_E_UNSUPPORTED, "neo above 512 is not supported by fock_dc");
    DMET_HIP(hipFuncSetAttribute((const void*)k_dc_k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    const int nt = (neo + DC_T - 1) / DC_T;
    for (int s = 0; s < nspin; ++s)
        k_dc_k<<<dim3(nt, (nrows + pchunk - 1) / pchunk), 256, shm, st>>>(nrows, neo, npair, pchunk, z + s * zs,
                                                                          dm_eo + s * gs, km + s * gs);
    const double cj = nspin == 1 ? 2.0 : 1.0;
    for (int s = 0; s < nspin; ++s)
        k_dc_final<<<(neo * neo + 255) / 256, 256, 0, st>>>(neo, f_eo + s * gs, jp + (size_t)s * npair, km + s * gs,
                                                            cj, 1.0, f_tilde + s * gs);
    ps.stop();
    DMET_LAUNCH_CHECK("fock_dc");
    return DMET_OK;
}

}  // namespace dmet
