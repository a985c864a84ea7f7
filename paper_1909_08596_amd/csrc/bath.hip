// Bath construction and embedding coefficients on the GPU, FP64 throughout.
//
//   gamma^{R,0} = 1/N_k sum_k exp(+i k.R) gamma(k)            (left side of Eq. "bath R SVD")
//   M = gamma_sup[env, imp[val]] = B Lambda V^T               (Eq. "bath R SVD", valence columns)
//   C^R = [[1, 0], [0, B]]  -> Loewdin -> C^k = sum_R exp(-i k.R) C^R   (Eqs. "C loemb R/k")
//
// The SVD is a one-sided (Hestenes) Jacobi iteration on the columns of M,
// stored column-major so that every column is one contiguous vector; pairs are
// visited in round-robin order, so the n/2 rotations of a round touch
// disjoint columns and run on separate wavefronts of one workgroup.
#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "eri.h"

namespace dmet {

// ---------------------------------------------------------------- step a1
// dm_r[s][R][mu][nu] = Re(1/N_k sum_k exp(i k.R) dm_k[s][k][mu][nu]); also
// the largest |Im| and a non-finite flag.
__global__ void k_dm_real(Mesh mesh, int nao, const double2* __restrict__ dm_k,
                          double* __restrict__ dm_r, int* flags, double* max_imag) {
    const int s = blockIdx.z, r = blockIdx.y;
    const int nn = nao * nao;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double im_abs = 0.0;
    if (e < nn) {
        double re = 0.0, im = 0.0;
        bool finite = true;
        for (int k = 0; k < mesh.nk; ++k) {
            double2 g = dm_k[((size_t)s * mesh.nk + k) * nn + e];
            finite = finite && isfinite(g.x) && isfinite(g.y);
            double2 p = phase_kR(mesh, k, r);
            re += p.x * g.x - p.y * g.y;
            im += p.x * g.y + p.y * g.x;
        }
        if (!finite) atomicOr(flags, FLAG_NONFINITE);
        dm_r[((size_t)s * mesh.nk + r) * nn + e] = re / mesh.nk;
        im_abs = fabs(im / mesh.nk);
    }
    im_abs = wave_max(im_abs);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(max_imag, im_abs);
}

// ---------------------------------------------------------------- step a2
// Mt[s][c][r] = gamma^{R_r - R_c, 0}[mu_r][mu_c]  (column-major M)
__global__ void k_build_m(Mesh mesh, int nao, int nenv, int nval, const int* __restrict__ env,
                          const int* __restrict__ cols, const double* __restrict__ dm_r,
                          double* __restrict__ mt) {
    const int s = blockIdx.z, c = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nenv) return;
    const int er = env[r], ec = cols[c];
    const int cell = mesh_sub(mesh, er / nao, ec / nao);
    mt[((size_t)s * nval + c) * nenv + r] =
        dm_r[(((size_t)s * mesh.nk + cell) * nao + er % nao) * nao + ec % nao];
}

// Round-robin schedule: seat 0 holds player 0, seats 1..n-1 rotate.
__device__ inline int rr_player(int seat, int round, int n) {
    return seat == 0 ? 0 : 1 + (seat - 1 + round) % (n - 1);
}

// One round of the cyclic round-robin ordering of the one-sided Jacobi SVD:
// workgroup (p, s) orthogonalises column pair p of the round for spin s (the
// pairs of a round are disjoint, so a round is one launch).  The three dot
// products are reduced over the block in a fixed order; rot[s] counts the
// rotations applied (a sweep with none has converged: |a.b| <= tol |a||b|
// for every pair).  A sweep after one with no rotation for spin s (prev[s] ==
// 0; prev null in the first sweep) would apply none either and returns at
// once, and so does every sweep when the density was not finite: the host can
// enqueue several sweeps between its reads of the counts.
__global__ void __launch_bounds__(256) k_jacobi_round(int m, int n, int np, int round,
                                                      double* __restrict__ mt, double tol, int* rot,
                                                      const int* __restrict__ prev, const int* __restrict__ flags) {
    const int pr = blockIdx.x, s = blockIdx.y;
    if ((prev && prev[s] == 0) || (flags[0] & FLAG_NONFINITE)) return;
    const int ca = rr_player(pr, round, np), cb = rr_player(np - 1 - pr, round, np);
    if (ca >= n || cb >= n) return;   // the dummy column of an odd count (whole block)
    double* a = mt + ((size_t)s * n + ca) * m;
    double* b = mt + ((size_t)s * n + cb) * m;
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double x = a[i], y = b[i];
        al += x * x;
        be += y * y;
        ga += x * y;
    }
    __shared__ double red[3][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    al = wave_sum(al);
    be = wave_sum(be);
    ga = wave_sum(ga);
    if (lane == 0) {
        red[0][wave] = al;
        red[1][wave] = be;
        red[2][wave] = ga;
    }
    __syncthreads();
    al = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    be = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    ga = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
    if (al == 0.0 || be == 0.0 || fabs(ga) <= tol * sqrt(al) * sqrt(be)) return;   // same in every thread
    const double zeta = (be - al) / (2.0 * ga);
    double t;
    if (fabs(zeta) > 1e150) t = 0.5 / zeta;
    else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double x = a[i], y = b[i];
        a[i] = c * x - sn * y;
        b[i] = sn * x + c * y;
    }
    if (threadIdx.x == 0) atomicAdd(&rot[s], 1);
}

// Wave sum through DPP lane moves (row shifts, then row broadcasts into the
// last lane; the GCN cross-lane reduction sequence), read back from lane 63
// so every lane holds the same total.  A double moves as two 32-bit halves.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ inline double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, BANK_MASK, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, BANK_MASK, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_sum_dpp(double x) {
    double v = x + dpp_mov<0x111, 0xf, 0xf>(x);     // row_shr:1
    v += dpp_mov<0x112, 0xf, 0xf>(x);               // row_shr:2
    v += dpp_mov<0x113, 0xf, 0xf>(x);               // row_shr:3: lane i holds x[i-3..i] within its row
    v += dpp_mov<0x114, 0xf, 0xe>(v);               // row_shr:4 into banks 1-3
    v += dpp_mov<0x118, 0xf, 0xc>(v);               // row_shr:8 into banks 2-3: lane 15 of a row has the row sum
    v += dpp_mov<0x142, 0xa, 0xf>(v);               // row_bcast:15 into rows 1 and 3
    v += dpp_mov<0x143, 0xc, 0xf>(v);               // row_bcast:31 into rows 2 and 3: lane 63 has the total
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Block form of the same sweep: the columns are grouped in blocks of JB and
// a round-robin round pairs the blocks.  Workgroup (p, s) stages the 2 JB
// columns of its block pair in LDS and rotates every pair across the two
// blocks (one wave per pair, dot products reduced over the wave in a fixed
// order); pairs inside a block are rotated in the sweep's first round.  An
// outer sweep (nbp - 1 launches) therefore visits every column pair once, and
// a sweep with no rotation has converged exactly as in the per-pair form.
// Columns of a missing block (odd block count) or past n take no part.
// JB = 8 (eight waves) when 16 columns fit in LDS, else JB = 4.
constexpr int JB_LDS = 150 * 1024;
constexpr int jb_maxm(int jb) { return JB_LDS / (2 * jb * 8) / 2 * 2; }   // rows that fit: 2 JB mp doubles

template <int JB>
__global__ void __launch_bounds__(64 * JB) k_jacobi_block(int m, int n, int nbp, int round,
                                                          double* __restrict__ mt, double tol, int* rot,
                                                          const int* __restrict__ prev,
                                                          const int* __restrict__ flags) {
    extern __shared__ __align__(16) double colsh[];   // [2 JB][mp], rows m..mp-1 zero
    const int mp = m + (m & 1);                        // even stride: rows move in pairs
    const int pr = blockIdx.x, s = blockIdx.y;
    if ((prev && prev[s] == 0) || (flags[0] & FLAG_NONFINITE)) return;   // as in k_jacobi_round
    const int nb = (n + JB - 1) / JB;
    const int ba = rr_player(pr, round, nbp), bb = rr_player(nbp - 1 - pr, round, nbp);
    auto colof = [&](int e) {   // column of slot e, or n if it takes no part
        const int b = e < JB ? ba : bb;
        const int c = b * JB + (e % JB);
        return (b < nb && c < n) ? c : n;
    };
    // JB_RU rows of every column per thread are loaded before any is stored,
    // so that one memory latency covers the whole stage at m <= 64 JB JB_RU
    constexpr int JB_RU = JB == 4 ? 5 : 3;
    for (int i0 = threadIdx.x; i0 < mp; i0 += 64 * JB * JB_RU) {
        double v[JB_RU][2 * JB];
#pragma unroll
        for (int u = 0; u < JB_RU; ++u) {
            const int i = i0 + u * 64 * JB;
#pragma unroll
            for (int e = 0; e < 2 * JB; ++e) {
                const int c = colof(e);
                v[u][e] = (c < n && i < m) ? mt[((size_t)s * n + c) * m + i] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < JB_RU; ++u) {
            const int i = i0 + u * 64 * JB;
#pragma unroll
            for (int e = 0; e < 2 * JB; ++e)
                if (i < mp) colsh[(size_t)e * mp + i] = v[u][e];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int nrot = 0;
    // pairs across the two blocks: JB rounds of JB disjoint pairs (wave w takes
    // slot w of the first block and slot (w + r) mod JB of the second); pairs
    // inside a block only in the sweep's first round (every block plays in
    // every round), JB - 1 rounds with JB / 2 waves per block
    const int nintra = round == 0 ? JB - 1 : 0;
    for (int ir = 0; ir < nintra + JB; ++ir) {
        int ea, eb;
        if (ir < nintra) {
            const int base = wave < JB / 2 ? 0 : JB, w = wave % (JB / 2);
            ea = base + rr_player(w, ir, JB);
            eb = base + rr_player(JB - 1 - w, ir, JB);
        } else {
            ea = wave;
            eb = JB + (wave + ir - nintra) % JB;
        }
        if (colof(ea) < n && colof(eb) < n) {
            double2* a = reinterpret_cast<double2*>(colsh + (size_t)ea * mp);
            double2* b = reinterpret_cast<double2*>(colsh + (size_t)eb * mp);
            const int mh = mp / 2;
            double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll 4
            for (int i = lane; i < mh; i += 64) {
                const double2 x = a[i], y = b[i];
                al += x.x * x.x + x.y * x.y;
                be += y.x * y.x + y.y * y.y;
                ga += x.x * y.x + x.y * y.y;
            }
            al = wave_sum_dpp(al);
            be = wave_sum_dpp(be);
            ga = wave_sum_dpp(ga);
            if (!(al == 0.0 || be == 0.0 || fabs(ga) <= tol * sqrt(al) * sqrt(be))) {   // wave-uniform
                const double zeta = (be - al) / (2.0 * ga);
                double t;
                if (fabs(zeta) > 1e150) t = 0.5 / zeta;
                else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll 4
                for (int i = lane; i < mh; i += 64) {
                    const double2 x = a[i], y = b[i];
                    a[i] = make_double2(c * x.x - sn * y.x, c * x.y - sn * y.y);
                    b[i] = make_double2(sn * x.x + c * y.x, sn * x.y + c * y.y);
                }
                ++nrot;
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < m; i += 64 * JB) {
#pragma unroll
        for (int e = 0; e < 2 * JB; ++e) {
            const int c = colof(e);
            if (c < n) mt[((size_t)s * n + c) * m + i] = colsh[(size_t)e * mp + i];
        }
    }
    if (lane == 0 && nrot) atomicAdd(&rot[s], nrot);
}

// sigma, descending order, normalised and sign-fixed left vectors.
// One workgroup per spin.  ub[s][b][r] = u_b, sv[s][b] = sigma_b, and
// flags[4 + s] = number of kept bath vectors: sigma > max(sv_tol, rank_tol)
// with rank_tol = sigma_max * max(m, n) * 2^-52, the rounding level below
// which M does not determine a singular vector (such a column is exactly
// zero after the sweeps, so its bath vector would be zero).
__global__ void __launch_bounds__(1024) k_svd_finalize(int m, int n, const double* __restrict__ mt,
                                                       double* __restrict__ ub, double* __restrict__ sv,
                                                       double sv_tol, int* flags) {
    const int s = blockIdx.x;
    const double* a_base = mt + (size_t)s * n * m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    extern __shared__ double sh[];
    double* sig = sh;                                // [n]
    int* order = reinterpret_cast<int*>(sig + n);    // [n]
    for (int c = wave; c < n; c += nwave) {
        const double* a = a_base + (size_t)c * m;
        double ss = 0.0;
        for (int i = lane; i < m; i += 64) ss += a[i] * a[i];
        ss = wave_sum(ss);
        if (lane == 0) sig[c] = sqrt(ss);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        int rank = 0;
        for (int d = 0; d < n; ++d)
            rank += (sig[d] > sig[c]) || (sig[d] == sig[c] && d < c);
        order[rank] = c;
    }
    __syncthreads();
    for (int b = wave; b < n; b += nwave) {
        const int c = order[b];
        const double* a = a_base + (size_t)c * m;
        const double inv = sig[c] > 0.0 ? 1.0 / sig[c] : 0.0;
        double amax = 0.0;
        for (int i = lane; i < m; i += 64) amax = fmax(amax, fabs(a[i]));
        amax = wave_max(amax);
        int first = m;
        for (int i = lane; i < m; i += 64)
            if (fabs(a[i]) >= amax - 1e-12 * amax) first = min(first, i);
        first = wave_min_int(first);
        const double sgn = (first < m && a[first] < 0.0) ? -inv : inv;
        double* u = ub + ((size_t)s * n + b) * m;
        for (int i = lane; i < m; i += 64) u[i] = a[i] * sgn;
        if (lane == 0) sv[(size_t)s * n + b] = sig[c];
    }
    if (threadIdx.x == 0) {
        double smax = 0.0;
        for (int c = 0; c < n; ++c) smax = fmax(smax, sig[c]);
        const double thr = fmax(sv_tol, smax * (double)max(m, n) * 2.220446049250313e-16);
        int kept = 0;
        for (int c = 0; c < n; ++c) kept += sig[c] > thr;
        flags[4 + s] = kept;
    }
}

// ---------------------------------------------------------------- step a3
// Loewdin: S = U^T U over the kept bath vectors; E = S - I.  One wave per
// pair i >= j (written to both triangles, the same bits); the largest |E| of
// the workgroup's four waves goes to emax in one atomic.
__global__ void k_overlap(int m, int n, const double* __restrict__ ub, double* __restrict__ e_out,
                          const int* flags, double* __restrict__ emax) {
    const int s = blockIdx.y;
    const int nb = flags[4 + s];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long pair = (long)blockIdx.x * (blockDim.x >> 6) + wave;
    const long npair = (long)n * (n + 1) / 2;
    double e = 0.0;
    if (pair < npair) {
        int i = (int)((sqrt(8.0 * (double)pair + 1.0) - 1.0) * 0.5);
        while ((long)i * (i + 1) / 2 > pair) --i;
        while ((long)(i + 1) * (i + 2) / 2 <= pair) ++i;
        const int j = (int)(pair - (long)i * (i + 1) / 2);
        double acc = 0.0;
        if (i < nb && j < nb) {
            const double* a = ub + ((size_t)s * n + i) * m;
            const double* b = ub + ((size_t)s * n + j) * m;
            for (int r = lane; r < m; r += 64) acc += a[r] * b[r];
            acc = wave_sum(acc);
        }
        e = (i < nb && j < nb) ? acc - (i == j) : 0.0;
        if (lane == 0) {
            e_out[((size_t)s * n + i) * n + j] = e;
            e_out[((size_t)s * n + j) * n + i] = e;
        }
    }
    __shared__ double wmax[4];
    if (lane == 0) wmax[wave] = fabs(e);
    __syncthreads();
    if (threadIdx.x == 0) atomic_max_nonneg(emax, fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3])));
}

// C <- C S^{-1/2} with S = I + E, |E| ~ 1e-15:  S^{-1/2} = I - E/2 + O(E^2).
// Writes C^R[s][R][mu][col] for every supercell orbital (R, mu) and column.
__global__ void k_assemble_cr(int nsup, int nimp, int n, int ldc, int m,
                              const int* __restrict__ imp, const int* __restrict__ envpos,
                              const double* __restrict__ ub, const double* __restrict__ e_mat,
                              const int* flags, double* __restrict__ cr) {
    const int s = blockIdx.z;
    const int col = blockIdx.y;
    const int sup = blockIdx.x * blockDim.x + threadIdx.x;
    if (sup >= nsup) return;
    double v = 0.0;
    if (col < nimp) {
        v = (imp[col] == sup) ? 1.0 : 0.0;
    } else {
        const int b = col - nimp;
        const int nb = flags[4 + s];
        const int r = envpos[sup];
        if (b < nb && r >= 0) {
            const double* e = e_mat + (size_t)s * n * n;
            double corr = 0.0;
            for (int i = 0; i < nb; ++i) corr += ub[((size_t)s * n + i) * m + r] * e[i * n + b];
            v = ub[((size_t)s * n + b) * m + r] - 0.5 * corr;
        }
    }
    cr[((size_t)s * nsup + sup) * ldc + col] = v;
}

// C^k[s][k][mu][i] = sum_R exp(-i k.R) C^R[s][R][mu][i]
__global__ void k_cr_to_ck(Mesh mesh, int nao, int ldc, const double* __restrict__ cr,
                           double2* __restrict__ ck) {
    const int s = blockIdx.z, k = blockIdx.y;
    const int per = nao * ldc;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per) return;
    double re = 0.0, im = 0.0;
    for (int r = 0; r < mesh.nk; ++r) {
        const double c = cr[((size_t)s * mesh.nk + r) * per + e];
        const double2 p = phase_kR(mesh, k, r);
        re += p.x * c;
        im -= p.y * c;
    }
    ck[((size_t)s * mesh.nk + k) * per + e] = make_double2(re, im);
}

// out[s][k] = a[k] (nao x nao) * b[s][k] (nao x ldc), complex FP64.
__global__ void k_compose_ao_lo(int nk, int nao, int ldc, const double2* __restrict__ a,
                                const double2* __restrict__ b, double2* __restrict__ out) {
    const int s = blockIdx.z, k = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nao * ldc) return;
    const int mu = e / ldc, i = e % ldc;
    const double2* ak = a + (size_t)k * nao * nao + (size_t)mu * nao;
    const double2* bk = b + ((size_t)s * nk + k) * nao * ldc;
    double re = 0.0, im = 0.0;
    for (int nu = 0; nu < nao; ++nu) {
        double2 x = ak[nu], y = bk[(size_t)nu * ldc + i];
        re += x.x * y.x - x.y * y.y;
        im += x.x * y.y + x.y * y.x;
    }
    out[((size_t)s * nk + k) * nao * ldc + e] = make_double2(re, im);
}

// ---------------------------------------------------------------- host side
struct BathPlan {
    Mesh mesh;
    int nao, nspin, nimp, nval, nenv, ldc, nsup;
};

constexpr int BATH_MAX_SWEEPS = 60;

struct BathWs {
    double* dm_r;
    int* flags;        // [0] status bits, [4+s] kept bath
    int* rots;         // [sweep][s] rotations applied by each sweep (at most BATH_MAX_SWEEPS)
    double* scal;      // [0] max |Im gamma^R|, [1] max |S - I|
    int* env;
    int* cols;
    int* imp;
    int* envpos;
    double* mt;
    double* ub;
    double* emat;
    double* cr;
    double2* ck_lo;
};

static BathWs carve_bath(Carve& cv, const BathPlan& p, bool with_ao_lo) {
    BathWs w;
    w.dm_r = cv.take<double>((size_t)p.nspin * p.mesh.nk * p.nao * p.nao);
    w.flags = cv.take<int>(16);
    w.rots = cv.take<int>(2 * BATH_MAX_SWEEPS);
    w.scal = cv.take<double>(4);
    // the four index lists back to back: one upload
    w.env = cv.take<int>((size_t)p.nenv + p.nval + p.nimp + p.nsup);
    w.cols = w.env + p.nenv;
    w.imp = w.cols + p.nval;
    w.envpos = w.imp + p.nimp;
    w.mt = cv.take<double>((size_t)p.nspin * p.nval * p.nenv);
    w.ub = cv.take<double>((size_t)p.nspin * p.nval * p.nenv);
    w.emat = cv.take<double>((size_t)p.nspin * p.nval * p.nval);
    w.cr = cv.take<double>((size_t)p.nspin * p.nsup * p.ldc);
    w.ck_lo = with_ao_lo ? cv.take<double2>((size_t)p.nspin * p.nsup * p.ldc) : nullptr;
    return w;
}

size_t bath_workspace_bytes(const dmet_lattice* lat, int nimp, int nval) {
    BathPlan p;
    p.mesh = make_mesh(lat->kmesh);
    p.nao = lat->nao;
    p.nspin = lat->nspin;
    p.nimp = nimp;
    p.nval = nval;
    p.nsup = p.mesh.nk * p.nao;
    p.nenv = p.nsup - nimp;
    p.ldc = nimp + nval;
    Carve cv(nullptr, 0);
    carve_bath(cv, p, true);
    return cv.bytes();
}

dmet_status build_bath(const dmet_lattice* lat, const double2* dm_k, int nimp, const int* imp_idx,
                       int nval, const int* val_idx, double sv_tol, const double2* c_ao_lo,
                       double2* c_k, double* sv, int* neo, double* max_imag, void* ws, size_t ws_bytes,
                       hipStream_t st) {
    BathPlan p;
    p.mesh = make_mesh(lat->kmesh);
    p.nao = lat->nao;
    p.nspin = lat->nspin;
    p.nimp = nimp;
    p.nval = nval;
    p.nsup = p.mesh.nk * p.nao;
    p.nenv = p.nsup - nimp;
    p.ldc = nimp + nval;

    // host index lists: impurity, SVD columns, environment rows (supercell order)
    std::vector<int> imp(nimp), cols(nval), env, envpos(p.nsup, -1);
    std::vector<char> is_imp(p.nsup, 0);
    for (int i = 0; i < nimp; ++i) {
        imp[i] = imp_idx ? imp_idx[i] : i;
        if (imp[i] < 0 || imp[i] >= p.nsup) return fail(DMET_E_ARG, "imp_idx entry out of range");
        if (is_imp[imp[i]]) return fail(DMET_E_ARG, "imp_idx has a repeated orbital");
        is_imp[imp[i]] = 1;
    }
    for (int c = 0; c < nval; ++c) {
        int v = val_idx ? val_idx[c] : c;
        if (v < 0 || v >= nimp) return fail(DMET_E_ARG, "val_idx entry out of range");
        cols[c] = imp[v];
    }
    for (int r = 0; r < p.nsup; ++r)
        if (!is_imp[r]) {
            envpos[r] = (int)env.size();
            env.push_back(r);
        }
    if ((int)env.size() != p.nenv) return fail(DMET_E_ARG, "impurity list inconsistent");
    // an empty environment (the impurity is the whole supercell, e.g. one
    // k-point with every orbital in the impurity) has no bath; a non-empty one
    // must have at least as many orbitals as the SVD has columns
    if (p.nenv > 0 && p.nenv < nval) return fail(DMET_E_ARG, "fewer environment orbitals than SVD columns");

    Carve cv(ws, ws_bytes);
    BathWs w = carve_bath(cv, p, c_ao_lo != nullptr);
    if (cv.bytes() > ws_bytes) return fail(DMET_E_WORKSPACE, "build_bath workspace too small");

    {
        std::vector<int> lists;
        lists.reserve(env.size() + cols.size() + imp.size() + envpos.size());
        for (const std::vector<int>* v : {&env, &cols, &imp, &envpos}) lists.insert(lists.end(), v->begin(), v->end());
        DMET_HIP(hipMemcpyAsync(w.env, lists.data(), sizeof(int) * lists.size(), hipMemcpyHostToDevice, st));
    }
    fill_zero(w.flags, 16 * sizeof(int), st);
    fill_zero(w.rots, 2 * BATH_MAX_SWEEPS * sizeof(int), st);
    fill_zero(w.scal, 4 * sizeof(double), st);

    const int nn = p.nao * p.nao;
    k_dm_real<<<dim3((nn + 255) / 256, p.mesh.nk, p.nspin), 256, 0, st>>>(p.mesh, p.nao, dm_k, w.dm_r,
                                                                          w.flags, w.scal);
    DMET_LAUNCH_CHECK("k_dm_real");
    if (p.nenv > 0) {
        k_build_m<<<dim3((p.nenv + 255) / 256, nval, p.nspin), 256, 0, st>>>(
            p.mesh, p.nao, p.nenv, nval, w.env, w.cols, w.dm_r, w.mt);
        DMET_LAUNCH_CHECK("k_build_m");
    }
    if (p.nenv > 0) {
        // sweeps of np - 1 rounds until a sweep applies no rotation, at most
        // 60; the counts are read back after six sweeps, then after every two
        // (a sweep that follows one without rotation returns at once)
        const double tol = fmax(1e-15, sqrt((double)p.nenv) * 2.220446049250313e-16);
        const int np = nval + (nval & 1);
        // block form when the 2 JB columns of a block pair fit in LDS
        const int mp = p.nenv + (p.nenv & 1);
        const int JB = mp <= jb_maxm(8) ? 8 : 4;
        const bool blocked = mp <= jb_maxm(4);
        const int nb = (nval + JB - 1) / JB, nbp = nb + (nb & 1);
        const size_t lds = (size_t)2 * JB * mp * sizeof(double);
        const void* kblk = JB == 8 ? (const void*)k_jacobi_block<8> : (const void*)k_jacobi_block<4>;
        if (blocked) DMET_HIP(hipFuncSetAttribute(kblk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        bool converged = false;
        // at most 60 sweeps; DMET_SVD_MAX_SWEEPS lowers the limit (to force the
        // non-convergence status from the host)
        int max_sweeps = BATH_MAX_SWEEPS;
        if (const char* e = getenv("DMET_SVD_MAX_SWEEPS"))
            max_sweeps = std::min(BATH_MAX_SWEEPS, std::max(1, atoi(e)));
        for (int s0 = 0; s0 < max_sweeps && !converged;) {
            const int s1 = std::min(max_sweeps, s0 + (s0 == 0 ? 6 : 2));
            for (int sweep = s0; sweep < s1; ++sweep) {
                int* rot = w.rots + 2 * sweep;
                const int* prev = sweep > 0 ? w.rots + 2 * (sweep - 1) : nullptr;
                if (blocked) {
                    for (int round = 0; round < nbp - 1; ++round) {
                        if (JB == 8)
                            k_jacobi_block<8><<<dim3(nbp / 2, p.nspin), 512, lds, st>>>(
                                p.nenv, nval, nbp, round, w.mt, tol, rot, prev, w.flags);
                        else
                            k_jacobi_block<4><<<dim3(nbp / 2, p.nspin), 256, lds, st>>>(
                                p.nenv, nval, nbp, round, w.mt, tol, rot, prev, w.flags);
                    }
                    DMET_LAUNCH_CHECK("k_jacobi_block");
                } else {
                    for (int round = 0; round < np - 1; ++round)
                        k_jacobi_round<<<dim3(np / 2, p.nspin), 256, 0, st>>>(p.nenv, nval, np, round, w.mt, tol,
                                                                               rot, prev, w.flags);
                    DMET_LAUNCH_CHECK("k_jacobi_round");
                }
            }
            int h_rot[2 * BATH_MAX_SWEEPS], f0 = 0;
            DMET_HIP(hipMemcpyAsync(h_rot, w.rots + 2 * s0, sizeof(int) * 2 * (s1 - s0), hipMemcpyDeviceToHost, st));
            DMET_HIP(hipMemcpyAsync(&f0, w.flags, sizeof(int), hipMemcpyDeviceToHost, st));
            DMET_HIP(hipStreamSynchronize(st));
            if (f0 & FLAG_NONFINITE) return fail(DMET_E_NONFINITE, "non-finite entry in dm_k");
            for (int sweep = s0; sweep < s1 && !converged; ++sweep) {
                converged = true;
                for (int sp = 0; sp < p.nspin; ++sp)
                    if (h_rot[2 * (sweep - s0) + sp] != 0) converged = false;
            }
            s0 = s1;
        }
        if (!converged)
            return fail(DMET_E_NOCONV, "Jacobi SVD did not converge in " + std::to_string(max_sweeps) + " sweeps");
        const size_t shm = (size_t)nval * (sizeof(double) + sizeof(int));
        k_svd_finalize<<<p.nspin, 1024, shm, st>>>(p.nenv, nval, w.mt, w.ub, sv, sv_tol, w.flags);
        DMET_LAUNCH_CHECK("k_svd_finalize");
        const int ovl_blocks = (nval * (nval + 1) / 2 + 3) / 4;
        k_overlap<<<dim3(ovl_blocks, p.nspin), 256, 0, st>>>(p.nenv, nval, w.ub, w.emat, w.flags, w.scal + 1);
        DMET_LAUNCH_CHECK("k_overlap");
    } else {
        // no bath: the kept count (flags[4 + s]) stays 0, singular values are 0
        if (nval > 0) fill_zero(sv, (size_t)p.nspin * nval * sizeof(double), st);
    }
    k_assemble_cr<<<dim3((p.nsup + 255) / 256, p.ldc, p.nspin), 256, 0, st>>>(
        p.nsup, nimp, nval, p.ldc, p.nenv, w.imp, w.envpos, w.ub, w.emat, w.flags, w.cr);
    DMET_LAUNCH_CHECK("k_assemble_cr");
    const int per = p.nao * p.ldc;
    double2* ck_out = c_ao_lo ? w.ck_lo : c_k;
    k_cr_to_ck<<<dim3((per + 255) / 256, p.mesh.nk, p.nspin), 256, 0, st>>>(p.mesh, p.nao, p.ldc, w.cr,
                                                                             ck_out);
    DMET_LAUNCH_CHECK("k_cr_to_ck");
    if (c_ao_lo) {
        k_compose_ao_lo<<<dim3((per + 255) / 256, p.mesh.nk, p.nspin), 256, 0, st>>>(
            p.mesh.nk, p.nao, p.ldc, c_ao_lo, w.ck_lo, c_k);
        DMET_LAUNCH_CHECK("k_compose_ao_lo");
    }
    int flags[16];
    double scal[4];
    DMET_HIP(hipMemcpyAsync(flags, w.flags, sizeof(flags), hipMemcpyDeviceToHost, st));
    DMET_HIP(hipMemcpyAsync(scal, w.scal, sizeof(scal), hipMemcpyDeviceToHost, st));
    DMET_HIP(hipStreamSynchronize(st));
    if (flags[0] & FLAG_NONFINITE) return fail(DMET_E_NONFINITE, "non-finite entry in dm_k");
    if (flags[0] & FLAG_NOCONV) return fail(DMET_E_NOCONV, "Jacobi SVD did not converge in 60 sweeps");
    if (scal[1] > 1e-6) return fail(DMET_E_NOCONV, "bath vectors lost orthogonality (|S - I| > 1e-6)");
    for (int s = 0; s < p.nspin; ++s) {
        if (flags[4 + s] == 0 && p.nenv > 0)
            return fail(DMET_E_RANK, "no singular value above max(sv_tol, rounding level): no bath orbital");
        neo[s] = nimp + flags[4 + s];
    }
    if (max_imag) *max_imag = scal[0];
    return DMET_OK;
}

// ---------------------------------------------------------------- no-allocation entry
// Device scratch of build_bath_noalloc: a file-scope array, one copy per GPU,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device array: its device address is looked up once per
// device with hipGetSymbolAddress and only that address is handed to kernels.
// Every call on a device shares the array and leaves the last call's contents
// in it (build_bath clears the flags it accumulates into); calls that overlap
// on one device race.
static __device__ __align__(256) unsigned char scratch[BATH_SCRATCH_MAX];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};
}  // namespace

dmet_status build_bath_noalloc(const dmet_lattice* lat, const double2* dm_k, int nimp, const int* imp_idx,
                               int nval, const int* val_idx, double sv_tol, const double2* c_ao_lo,
                               double2* c_k, double* sv, int* neo, double* max_imag, hipStream_t st) {
    BathPlan p;
    p.mesh = make_mesh(lat->kmesh);
    p.nao = lat->nao;
    p.nspin = lat->nspin;
    p.nimp = nimp;
    p.nval = nval;
    p.nsup = p.mesh.nk * p.nao;
    p.nenv = p.nsup - nimp;
    p.ldc = nimp + nval;
    Carve cv(nullptr, 0);
    carve_bath(cv, p, c_ao_lo != nullptr);
    if (cv.bytes() > BATH_SCRATCH_MAX)
        return fail(DMET_E_WORKSPACE, "dmet_build_bath_noalloc: this bath needs " + std::to_string(cv.bytes()) +
                                          " bytes of scratch, more than the " + std::to_string(BATH_SCRATCH_MAX) +
                                          " bytes it holds; call dmet_build_bath with a workspace");
    int dev = 0;
    DMET_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(DMET_E_UNSUPPORTED, "device ordinal above 63");
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* a = nullptr;
            DMET_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
            if (!a) return fail(DMET_E_HIP, "hipGetSymbolAddress returned a null scratch address");
            g_scratch_ptr[dev] = a;
        }
        ptr = g_scratch_ptr[dev];
    }
    return build_bath(lat, dm_k, nimp, imp_idx, nval, val_idx, sv_tol, c_ao_lo, c_k, sv, neo, max_imag, ptr,
                      BATH_SCRATCH_MAX, st);
}

}  // namespace dmet
