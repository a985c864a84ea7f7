// One-body transform to the embedding basis (Eq. "fock transform"):
//   X^{0,EO}_{ij} = 1/N_k sum_k sum_{mu nu} conj(C^k_{mu i}) X^k_{mu nu} C^k_{nu j}
// and the one-body energy E1 = sum_spin Tr(h^EO gamma^EO).  FP64 vector ALU:
// the work is N_k nao neo (nao + neo) complex MACs, a few GFLOP at most.
#include "common.h"

namespace dmet {

// Each workgroup owns a 64 x 32 tile (i, j) of one spin's output and walks k and mu chunks of 32:
//   T[mu][j] = sum_nu X^k[mu][nu] C^k[nu][j]   (nu in slices of 16 staged through LDS, the next
//                                              slice prefetched into registers during the current)
//   out[i][j] += sum_mu conj(C^k[mu][i]) T[mu][j]
constexpr int OB_TI = 64, OB_TJ = 32, OB_MC = 32, OB_NC = 16;

__global__ void __launch_bounds__(256) k_onebody(Mesh mesh, int nao, int neo, const double2* __restrict__ ck,
                                                 const double2* __restrict__ op, double* __restrict__ out,
                                                 double* __restrict__ max_imag) {
    const int s = blockIdx.z;
    const int i0 = blockIdx.y * OB_TI, j0 = blockIdx.x * OB_TJ;
    __shared__ double2 xs[2][OB_MC][OB_NC];   // X[mu][nu] slice
    __shared__ double2 cs[2][OB_NC][OB_TJ];   // C[nu][j] slice
    __shared__ double2 ts[OB_MC][OB_TJ];      // T[mu][j] of the current mu chunk
    const int tid = threadIdx.x;
    const int tj = tid % OB_TJ, tm = tid / OB_TJ;     // T: mu = tm + 8 m, m < 4
    const int oi = tid % OB_TI, og = tid / OB_TI;     // out: i = oi, j = 8 og + r, r < 8
    const int nmc = (nao + OB_MC - 1) / OB_MC, nnc = (nao + OB_NC - 1) / OB_NC;
    const int total = mesh.nk * nmc * nnc;
    double2 rx[2], rc[2];
    auto gather = [&](int it) {
        const int nc = it % nnc, mc = (it / nnc) % nmc, k = it / (nnc * nmc);
        const double2* x = op + ((size_t)s * mesh.nk + k) * nao * nao;
        const double2* c = ck + ((size_t)s * mesh.nk + k) * nao * neo;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = tid + 256 * u;
            const int xm = mc * OB_MC + e / OB_NC, xn = nc * OB_NC + e % OB_NC;
            rx[u] = (xm < nao && xn < nao) ? x[(size_t)xm * nao + xn] : make_double2(0.0, 0.0);
            const int cn = nc * OB_NC + e / OB_TJ, cj = j0 + e % OB_TJ;
            rc[u] = (cn < nao && cj < neo) ? c[(size_t)cn * neo + cj] : make_double2(0.0, 0.0);
        }
    };
    auto stash = [&](int b) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = tid + 256 * u;
            xs[b][e / OB_NC][e % OB_NC] = rx[u];
            cs[b][e / OB_TJ][e % OB_TJ] = rc[u];
        }
    };
    double2 tacc[4] = {};
    double re[8] = {}, im[8] = {};
    gather(0);
    stash(0);
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const int b = it & 1;
        if (it + 1 < total) gather(it + 1);
#pragma unroll
        for (int n = 0; n < OB_NC; ++n) {
            const double2 cv = cs[b][n][tj];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double2 xv = xs[b][tm + 8 * m][n];
                tacc[m].x += xv.x * cv.x - xv.y * cv.y;
                tacc[m].y += xv.x * cv.y + xv.y * cv.x;
            }
        }
        if (it % nnc == nnc - 1) {      // T of this mu chunk is complete
            const int mc = (it / nnc) % nmc, k = it / (nnc * nmc);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                ts[tm + 8 * m][tj] = tacc[m];
                tacc[m] = make_double2(0.0, 0.0);
            }
            __syncthreads();
            const double2* c = ck + ((size_t)s * mesh.nk + k) * nao * neo;
            const int mlen = min(OB_MC, nao - mc * OB_MC);
            const bool iok = i0 + oi < neo;
            for (int mm = 0; mm < mlen; ++mm) {
                const double2 a = iok ? c[(size_t)(mc * OB_MC + mm) * neo + i0 + oi] : make_double2(0.0, 0.0);
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const double2 t = ts[mm][8 * og + r];
                    re[r] += a.x * t.x + a.y * t.y;      // conj(a) * t
                    im[r] += a.x * t.y - a.y * t.x;
                }
            }
        }
        if (it + 1 < total) stash(b ^ 1);
        __syncthreads();
    }
    double mi = 0.0;
    const int i = i0 + oi;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int j = j0 + 8 * og + r;
        if (i < neo && j < neo) {
            out[((size_t)s * neo + i) * neo + j] = re[r] / mesh.nk;
            mi = fmax(mi, fabs(im[r] / mesh.nk));
        }
    }
    if (max_imag) {
        mi = wave_max(mi);
        if ((tid & 63) == 0) atomic_max_nonneg(max_imag, mi);
    }
}

__global__ void __launch_bounds__(1024) k_energy_1e(int nspin, int neo, const double* __restrict__ h,
                                                    const double* __restrict__ g, double* __restrict__ e1) {
    __shared__ double part[16];
    double acc = 0.0;
    const size_t per = (size_t)neo * neo;
    for (size_t e = threadIdx.x; e < (size_t)nspin * per; e += blockDim.x) {
        const size_t s = e / per, ij = e % per, i = ij / neo, j = ij % neo;
        acc += h[e] * g[s * per + j * neo + i];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        e1[0] = t;
    }
}

dmet_status transform_1e(const dmet_lattice* lat, int neo, const double2* ck, const double2* op,
                         double* out, double* max_imag, hipStream_t st) {
    Mesh mesh = make_mesh(lat->kmesh);
    if (max_imag) fill_zero(max_imag, sizeof(double), st);
    const int ntj = (neo + OB_TJ - 1) / OB_TJ, nti = (neo + OB_TI - 1) / OB_TI;
    k_onebody<<<dim3(ntj, nti, lat->nspin), 256, 0, st>>>(mesh, lat->nao, neo, ck, op, out, max_imag);
    DMET_LAUNCH_CHECK("k_onebody");
    return DMET_OK;
}

dmet_status energy_1e(int nspin, int neo, const double* h, const double* g, double* e1, hipStream_t st) {
    k_energy_1e<<<1, 1024, 0, st>>>(nspin, neo, h, g, e1);
    DMET_LAUNCH_CHECK("k_energy_1e");
    return DMET_OK;
}

}  // namespace dmet
