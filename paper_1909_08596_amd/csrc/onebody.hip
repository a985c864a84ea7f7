// One-body transform to the embedding basis (Eq. "fock transform"):
//   X^{0,EO}_{ij} = 1/N_k sum_k sum_{mu nu} conj(C^k_{mu i}) X^k_{mu nu} C^k_{nu j}
// and the one-body energy E1 = sum_spin Tr(h^EO gamma^EO).  FP64 vector ALU:
// the work is N_k nao neo (nao + neo) complex MACs, a few GFLOP at most.
#include <mutex>

#include "common.h"

namespace dmet {

// Each workgroup owns a 64 x 32 tile (i, j) of one spin's output and walks k and mu chunks of 64:
//   T[mu][j] = sum_nu X^k[mu][nu] C^k[nu][j]   (nu in slices of 32 staged through LDS, the next
//                                              slice prefetched into registers during the current)
//   out[i][j] += sum_mu conj(C^k[mu][i]) T[mu][j]
// Every thread computes a 4 x 2 block of T and a 2 x 4 block of the output, so that each value
// read from LDS feeds several multiply-adds.  The X slice is stored transposed ([nu][mu], rows
// padded by one element so that the transposing stores do not collide in the LDS banks).
constexpr int OB_TI = 64, OB_TJ = 32, OB_MC = 64, OB_NC = 32, OB_XLD = OB_MC + 1;

inline size_t onebody_lds() {
    return sizeof(double2) * (2 * OB_NC * OB_XLD + 2 * OB_NC * OB_TJ + OB_MC * OB_TJ);
}

__device__ inline void cmac(double2& acc, double2 a, double2 b) {   // acc += a b
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}

__global__ void __launch_bounds__(256) k_onebody(Mesh mesh, int nao, int neo, const double2* __restrict__ ck,
                                                 const double2* __restrict__ op, double* __restrict__ out,
                                                 double* __restrict__ max_imag) {
    extern __shared__ double2 ob_lds[];
    double2(*xt)[OB_NC][OB_XLD] = reinterpret_cast<double2(*)[OB_NC][OB_XLD]>(ob_lds);   // X^T slices
    double2(*cs)[OB_NC][OB_TJ] = reinterpret_cast<double2(*)[OB_NC][OB_TJ]>(ob_lds + 2 * OB_NC * OB_XLD);
    double2(*ts)[OB_TJ] = reinterpret_cast<double2(*)[OB_TJ]>(ob_lds + 2 * OB_NC * OB_XLD + 2 * OB_NC * OB_TJ);
    const int s = blockIdx.z;
    const int i0 = blockIdx.y * OB_TI, j0 = blockIdx.x * OB_TJ;
    const int tid = threadIdx.x;
    const int tjg = tid % 16, tmg = tid / 16;     // T: mu = 4 tmg + a (a < 4), j = 2 tjg + c (c < 2)
    const int oi = tid % 32, og = tid / 32;       // out: i = oi + 32 a (a < 2), j = 4 og + r (r < 4)
    const int nmc = (nao + OB_MC - 1) / OB_MC, nnc = (nao + OB_NC - 1) / OB_NC;
    const int total = mesh.nk * nmc * nnc;
    constexpr int UX = OB_MC * OB_NC / 256, UC = OB_NC * OB_TJ / 256;
    // loads use clamped (always valid) indices and are unconditional, so that
    // none of them is waited for before the slice is stored; out-of-range
    // elements are replaced by zero when stored
    double2 rx[UX], rc[UC];
    auto gather = [&](int it) __attribute__((always_inline)) {
        const int nc = it % nnc, mc = (it / nnc) % nmc, k = it / (nnc * nmc);
        const double2* x = op + ((size_t)s * mesh.nk + k) * nao * nao;
        const double2* c = ck + ((size_t)s * mesh.nk + k) * nao * neo;
#pragma unroll
        for (int u = 0; u < UX; ++u) {
            const int e = tid + 256 * u;
            const int xm = min(mc * OB_MC + e / OB_NC, nao - 1), xn = min(nc * OB_NC + e % OB_NC, nao - 1);
            rx[u] = x[(size_t)xm * nao + xn];
        }
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int e = tid + 256 * u;
            const int cn = min(nc * OB_NC + e / OB_TJ, nao - 1), cj = min(j0 + e % OB_TJ, neo - 1);
            rc[u] = c[(size_t)cn * neo + cj];
        }
    };
    auto stash = [&](int it, int b) __attribute__((always_inline)) {
        const int nc = it % nnc, mc = (it / nnc) % nmc;
#pragma unroll
        for (int u = 0; u < UX; ++u) {
            const int e = tid + 256 * u;
            const bool ok = mc * OB_MC + e / OB_NC < nao && nc * OB_NC + e % OB_NC < nao;
            xt[b][e % OB_NC][e / OB_NC] = make_double2(ok ? rx[u].x : 0.0, ok ? rx[u].y : 0.0);
        }
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int e = tid + 256 * u;
            const bool ok = nc * OB_NC + e / OB_TJ < nao && j0 + e % OB_TJ < neo;
            cs[b][e / OB_TJ][e % OB_TJ] = make_double2(ok ? rc[u].x : 0.0, ok ? rc[u].y : 0.0);
        }
    };
    double2 tacc[4][2] = {};
    double2 oacc[2][4] = {};
    gather(0);
    stash(0, 0);
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const int b = it & 1;
        if (it + 1 < total) gather(it + 1);
#pragma unroll 4
        for (int n = 0; n < OB_NC; ++n) {
            double2 xv[4], cv[2];
#pragma unroll
            for (int a = 0; a < 4; ++a) xv[a] = xt[b][n][4 * tmg + a];
#pragma unroll
            for (int c = 0; c < 2; ++c) cv[c] = cs[b][n][2 * tjg + c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) cmac(tacc[a][c], xv[a], cv[c]);
        }
        if (it % nnc == nnc - 1) {      // T of this mu chunk is complete
            const int mc = (it / nnc) % nmc, k = it / (nnc * nmc);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    ts[4 * tmg + a][2 * tjg + c] = tacc[a][c];
                    tacc[a][c] = make_double2(0.0, 0.0);
                }
            __syncthreads();
            const double2* cp = ck + ((size_t)s * mesh.nk + k) * nao * neo;
            const int ia = min(i0 + oi, neo - 1), ib = min(i0 + oi + 32, neo - 1);
            // C[mu][i] of 16 mu at a time, all loaded (clamped rows) before use; rows past nao
            // meet zero rows of T, and columns i past neo are never written
            for (int h = 0; h < OB_MC; h += 16) {
                double2 av[16][2];
#pragma unroll
                for (int mm = 0; mm < 16; ++mm) {
                    const size_t row = (size_t)min(mc * OB_MC + h + mm, nao - 1) * neo;
                    av[mm][0] = cp[row + ia];
                    av[mm][1] = cp[row + ib];
                }
#pragma unroll
                for (int mm = 0; mm < 16; ++mm) {
                    double2 tv[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) tv[r] = ts[h + mm][4 * og + r];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            cmac(oacc[a][r], make_double2(av[mm][a].x, -av[mm][a].y), tv[r]);   // conj(C) T
                }
            }
        }
        if (it + 1 < total) stash(it + 1, b ^ 1);
        __syncthreads();
    }
    double mi = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int i = i0 + oi + 32 * a;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = j0 + 4 * og + r;
            if (i < neo && j < neo) {
                out[((size_t)s * neo + i) * neo + j] = oacc[a][r].x / mesh.nk;
                mi = fmax(mi, fabs(oacc[a][r].y / mesh.nk));
            }
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

// max |Im X^{0,EO}| is gathered in a device word of the library (one per GPU,
// its address looked up once per device); a call that asks for it holds the
// mutex from the clearing of that word to the read-back, so concurrent calls
// on one GPU take turns and each reads its own value.
static __device__ double imag_slot;

namespace {
std::mutex g_imag_mu;
double* g_imag_ptr[64] = {};
}  // namespace

dmet_status transform_1e(const dmet_lattice* lat, int neo, const double2* ck, const double2* op,
                         double* out, double* max_imag, hipStream_t st) {
    Mesh mesh = make_mesh(lat->kmesh);
    const int ntj = (neo + OB_TJ - 1) / OB_TJ, nti = (neo + OB_TI - 1) / OB_TI;
    DMET_HIP(hipFuncSetAttribute((const void*)k_onebody, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)onebody_lds()));
    if (!max_imag) {
        k_onebody<<<dim3(ntj, nti, lat->nspin), 256, onebody_lds(), st>>>(mesh, lat->nao, neo, ck, op, out, nullptr);
        DMET_LAUNCH_CHECK("k_onebody");
        return DMET_OK;
    }
    int dev = 0;
    DMET_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(DMET_E_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_imag_mu);
    if (!g_imag_ptr[dev]) {
        void* a = nullptr;
        DMET_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(imag_slot)));
        if (!a) return fail(DMET_E_HIP, "hipGetSymbolAddress returned a null address");
        g_imag_ptr[dev] = static_cast<double*>(a);
    }
    double* slot = g_imag_ptr[dev];
    fill_zero(slot, sizeof(double), st);
    k_onebody<<<dim3(ntj, nti, lat->nspin), 256, onebody_lds(), st>>>(mesh, lat->nao, neo, ck, op, out, slot);
    DMET_LAUNCH_CHECK("k_onebody");
    DMET_HIP(hipMemcpyAsync(max_imag, slot, sizeof(double), hipMemcpyDeviceToHost, st));
    DMET_HIP(hipStreamSynchronize(st));
    return DMET_OK;
}

dmet_status energy_1e(int nspin, int neo, const double* h, const double* g, double* e1, hipStream_t st) {
    k_energy_1e<<<1, 1024, 0, st>>>(nspin, neo, h, g, e1);
    DMET_LAUNCH_CHECK("k_energy_1e");
    return DMET_OK;
}

}  // namespace dmet
