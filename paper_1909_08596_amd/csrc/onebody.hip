// One-body transform to the embedding basis (Eq. "fock transform"):
//   X^{0,EO}_{ij} = 1/N_k sum_k sum_{mu nu} conj(C^k_{mu i}) X^k_{mu nu} C^k_{nu j}
// and the one-body energy E1 = sum_spin Tr(h^EO gamma^EO).  FP64 vector ALU:
// the work is N_k nao neo (nao + neo) complex MACs, a few GFLOP at most.
#include "common.h"

namespace dmet {

constexpr int OB_T = 32;   // output tile (i, j)
constexpr int OB_C = 16;   // mu chunk staged in LDS

__global__ void __launch_bounds__(256) k_onebody(Mesh mesh, int nao, int neo, const double2* __restrict__ ck,
                                                 const double2* __restrict__ op, double* __restrict__ out,
                                                 double* __restrict__ max_imag) {
    const int s = blockIdx.z;
    const int i0 = blockIdx.y * OB_T, j0 = blockIdx.x * OB_T;
    __shared__ double2 t_sh[OB_C][OB_T];   // T[mu][j] = sum_nu X[mu][nu] C[nu][j]
    __shared__ double2 c_sh[OB_C][OB_T];   // C[mu][i]
    const int tid = threadIdx.x;
    const int ti = tid / 8, tj = tid % 8;  // each thread: i = i0+ti, j = j0+tj+8*r
    double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    for (int k = 0; k < mesh.nk; ++k) {
        const double2* c = ck + ((size_t)s * mesh.nk + k) * nao * neo;
        const double2* x = op + ((size_t)s * mesh.nk + k) * nao * nao;
        for (int m0 = 0; m0 < nao; m0 += OB_C) {
            __syncthreads();
            for (int e = tid; e < OB_C * OB_T; e += 256) {
                const int mu = m0 + e / OB_T, jj = e % OB_T;
                double2 tv = make_double2(0.0, 0.0), cv = make_double2(0.0, 0.0);
                if (mu < nao) {
                    if (j0 + jj < neo) {
                        for (int nu = 0; nu < nao; ++nu) {
                            const double2 a = x[(size_t)mu * nao + nu];
                            const double2 b = c[(size_t)nu * neo + j0 + jj];
                            tv.x += a.x * b.x - a.y * b.y;
                            tv.y += a.x * b.y + a.y * b.x;
                        }
                    }
                    if (i0 + jj < neo) cv = c[(size_t)mu * neo + i0 + jj];
                }
                t_sh[e / OB_T][jj] = tv;
                c_sh[e / OB_T][jj] = cv;
            }
            __syncthreads();
            for (int mm = 0; mm < OB_C; ++mm) {
                const double2 a = c_sh[mm][ti];          // conj taken below
                for (int r = 0; r < 4; ++r) {
                    const double2 b = t_sh[mm][tj + 8 * r];
                    re[r] += a.x * b.x + a.y * b.y;
                    im[r] += a.x * b.y - a.y * b.x;
                }
            }
        }
    }
    double mi = 0.0;
    const int i = i0 + ti;
    for (int r = 0; r < 4; ++r) {
        const int j = j0 + tj + 8 * r;
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
    const int nt = (neo + OB_T - 1) / OB_T;
    k_onebody<<<dim3(nt, nt, lat->nspin), 256, 0, st>>>(mesh, lat->nao, neo, ck, op, out, max_imag);
    DMET_LAUNCH_CHECK("k_onebody");
    return DMET_OK;
}

dmet_status energy_1e(int nspin, int neo, const double* h, const double* g, double* e1, hipStream_t st) {
    k_energy_1e<<<1, 1024, 0, st>>>(nspin, neo, h, g, e1);
    DMET_LAUNCH_CHECK("k_energy_1e");
    return DMET_OK;
}

}  // namespace dmet
