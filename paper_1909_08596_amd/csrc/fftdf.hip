// Plane-wave (FFTDF) embedding ERIs, App. B, Eq. "FFTDF" and Alg. 2.
//
// The grid points r of the reference cell play the role of the fitting
// functions: the transform of Alg. 1 (FP64, or the split-bf16 transform of the
// reduced forms) turns the AO pair densities
// (r|mu k, nu k-q) into the real rows Z_r = w_q (Re X, Im X) of the embedded
// pair densities X(q)[r][ij] (q and -q combined as for GDF).  For each q the
// rows are Fourier transformed over the grid with the phase of q,
//   W(G) = sum_r exp(+i (q+G).r) X(r),
// one axis at a time (a separable 3-D DFT; each output sums the n_d points of
// its line, the phases read from a table of the L = N_d n_d roots of unity of
// the supercell axis held in LDS), and scaled by
// dV sqrt(4 pi / (Omega |q+G|^2)) into two real rows (Re W, Im W) per G (FP64).
// The contraction of those rows gives the ERIs: FP64, or on split-bf16 parts of
// the rows, split over the rows when there are few output tiles.
// The DFT runs in fractional
// coordinates, so only |q+G|^2 (through the reciprocal vectors) and Omega see
// the shape of the cell.
#include <math.h>

#include <algorithm>

#include <vector>

#include "common.h"
#include "eri.h"

namespace dmet {
namespace {

constexpr int PW_MAXL = 8192;    // N_d n_d roots of unity per supercell axis (128 KB of LDS)

struct PwAxis {
    int n[3];          // grid
    int axis;          // axis transformed by this pass
    int nmesh, m;      // k-mesh size and q coordinate along the axis
};

struct PwScale {
    int n[3], nmesh[3], m[3];
    double b[3][3];    // reciprocal vectors of the reference cell (rows), a_c . b_d = 2 pi delta_cd
    double dv, omega;
};

// dV sqrt(4 pi / (Omega |q+G|^2)) for the grid frequency x (0 at q+G = 0):
// q + G = sum_d (j_d / N_d) b_d with j_d the supercell frequency in FFT order
__device__ inline double pw_scale(const PwScale& k, const int x[3]) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        const long L = (long)k.nmesh[d] * k.n[d], j = (long)k.nmesh[d] * x[d] + k.m[d];
        const long jp = j <= (L - 1) / 2 ? j : j - L;   // supercell FFT order
        const double f = (double)jp / (double)k.nmesh[d];
        for (int c = 0; c < 3; ++c) v[c] += f * k.b[d][c];
    }
    const double k2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    return k2 > 0.0 ? k.dv * sqrt(4.0 * M_PI / (k.omega * k2)) : 0.0;
}

// Reciprocal vectors (rows of 2 pi (A^-1)^T, A the lattice vectors as rows)
// and |det A|, by cofactors.
void reciprocal(const double (&a)[3][3], double (&b)[3][3], double& vol) {
    const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                       a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                       a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    // b_d = 2 pi (a_{d+1} x a_{d+2}) / det
    for (int d = 0; d < 3; ++d) {
        const double* u = a[(d + 1) % 3];
        const double* w = a[(d + 2) % 3];
        b[d][0] = 2.0 * M_PI * (u[1] * w[2] - u[2] * w[1]) / det;
        b[d][1] = 2.0 * M_PI * (u[2] * w[0] - u[0] * w[2]) / det;
        b[d][2] = 2.0 * M_PI * (u[0] * w[1] - u[1] * w[0]) / det;
    }
    vol = fabs(det);
}

// One axis of W: out[.., g, ..][p] = sum_t exp(+2 pi i (N g + m) t / (N n)) in[.., t, ..][p]
// over a [x0][x1][x2][pair] layout.  IN: 0 complex buffer, 1 real rows
// (row zrow0 + r), 2 interleaved Re/Im rows (row zrow0 + 2 r + part), rows of
// type T (FP64, or FP32 from the split-bf16 transform).  OUT: 0 complex buffer,
// 1 scaled rows zg0 + 2 G + part.  The sums run in FP64, t in increasing order.
// A thread takes one line along the axis and one pair: it reads the line's
// inputs once per PW_GT outputs (consecutive pairs in the lanes: coalesced) and
// the twiddle of an (output, term) is the same in every lane (an LDS broadcast).
constexpr int PW_GT = 16;

template <int IN, int OUT, class T = double>
__global__ void __launch_bounds__(256) k_pw_axis(PwAxis ax, int npair, const double2* __restrict__ cin,
                                                 const T* __restrict__ zin, size_t zrow0, size_t ldz,
                                                 double2* __restrict__ cout, double* __restrict__ zout, size_t zg0,
                                                 PwScale ks) {
    extern __shared__ double2 tw[];   // tw[j] = exp(2 pi i j / L), L = N_d n_d entries
    const int nd = ax.n[ax.axis];
    const int L = ax.nmesh * nd;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)j / (double)L, &s, &c);
        tw[j] = make_double2(c, s);
    }
    __syncthreads();
    const int n1 = ax.n[1], n2 = ax.n[2];
    const long n12 = (long)n1 * n2;
    const long stride = ax.axis == 0 ? n12 : (ax.axis == 1 ? n2 : 1);
    const long total = (long)ax.n[0] * n12 / nd * npair;   // lines x pairs
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int p = (int)(e % npair);
        const long line = e / npair;
        // grid coordinates of the line's first point (coordinate `axis` = 0)
        int x[3];
        if (ax.axis == 0) {
            x[0] = 0;
            x[1] = (int)(line / n2);
            x[2] = (int)(line % n2);
        } else if (ax.axis == 1) {
            x[0] = (int)(line / n2);
            x[1] = 0;
            x[2] = (int)(line % n2);
        } else {
            x[0] = (int)(line / n1);
            x[1] = (int)(line % n1);
            x[2] = 0;
        }
        const long base = (long)x[0] * n12 + (long)x[1] * n2 + x[2];
        for (int g0 = 0; g0 < nd; g0 += PW_GT) {
            double re[PW_GT], im[PW_GT];
            int ph[PW_GT], step[PW_GT];
#pragma unroll
            for (int u = 0; u < PW_GT; ++u) {
                re[u] = 0.0;
                im[u] = 0.0;
                ph[u] = 0;
                // the phase of term t is (N g + m) t mod L, advanced exactly in integers
                step[u] = (ax.nmesh * (g0 + u) + ax.m) % L;
            }
            for (int t = 0; t < nd; ++t) {
                const long rt = base + (long)t * stride;
                double vr, vi;
                if (IN == 0) {
                    const double2 v = cin[rt * npair + p];
                    vr = v.x;
                    vi = v.y;
                } else if (IN == 1) {
                    vr = (double)zin[(zrow0 + rt) * ldz + p];
                    vi = 0.0;
                } else {
                    vr = (double)zin[(zrow0 + 2 * rt) * ldz + p];
                    vi = (double)zin[(zrow0 + 2 * rt + 1) * ldz + p];
                }
#pragma unroll
                for (int u = 0; u < PW_GT; ++u) {
                    const double2 w = tw[ph[u]];
                    ph[u] += step[u];
                    ph[u] -= ph[u] >= L ? L : 0;
                    re[u] += w.x * vr - w.y * vi;
                    im[u] += w.x * vi + w.y * vr;
                }
            }
#pragma unroll
            for (int u = 0; u < PW_GT; ++u) {
                const int g = g0 + u;
                if (g < nd) {
                    const long r = base + (long)g * stride;
                    if (OUT == 0) {
                        cout[r * npair + p] = make_double2(re[u], im[u]);
                    } else {
                        int xg[3] = {x[0], x[1], x[2]};
                        xg[ax.axis] = g;
                        const double sc = pw_scale(ks, xg);
                        zout[(zg0 + 2 * r) * ldz + p] = sc * re[u];
                        zout[(zg0 + 2 * r + 1) * ldz + p] = sc * im[u];
                    }
                }
            }
        }
    }
}

struct PwDims {
    size_t nr, eri_ws, zr, buf, zg, part;   // zr in elements of the row type; eri_ws, part in bytes
    int zrows_g, krows_p, ldz;
    bool split;                               // split-bf16 transform and contraction
};

PwDims pw_dims(const EriPlan& p) {
    PwDims d;
    d.split = p.prec == DMET_BF16X6_3M || p.prec == DMET_BF16X3_3M;
    d.nr = (size_t)p.naux;
    d.zrows_g = (int)(2 * d.nr * p.qblocks.size());
    d.krows_p = (d.zrows_g + 15) / 16 * 16;
    d.ldz = (p.npair + 1) / 2 * 2;
    d.eri_ws = d.split ? lp_transform_workspace(p) : eri_f64_workspace(p);
    d.zr = (size_t)p.nspin * p.zrows * p.npair;
    d.buf = d.nr * p.npair;
    d.zg = (size_t)p.nspin * d.krows_p * d.ldz;
    d.part = d.split ? lp_rows_contract_workspace(p.prec, p.nspin, p.npair, d.krows_p)
                     : contract_f64_workspace(p.nspin, p.npair, d.krows_p) * sizeof(double);
    return d;
}

}  // namespace

size_t fftdf_workspace(const EriPlan& p) {
    PwDims d = pw_dims(p);
    Carve cv(nullptr, 0);
    cv.take<char>(d.eri_ws);
    if (d.split) cv.take<float>(d.zr);
    else cv.take<double>(d.zr);
    cv.take<double2>(d.buf);
    cv.take<double2>(d.buf);
    cv.take<double>(d.zg);
    cv.take<char>(d.part);
    return cv.bytes();
}

dmet_status fftdf_eri(const EriPlan& p, const dmet_pw_grid* grid, const void* rho, const double* ck, double* eri_aa,
                      double* eri_bb, double* eri_ab, void* ws, size_t ws_bytes, hipStream_t st) {
    PwDims d = pw_dims(p);
    if (p.prec != DMET_FP64 && !d.split)
        return fail(DMET_E_UNSUPPORTED, "fftdf: FP64, BF16X6_3M or BF16X3_3M");
    Carve cv(ws, ws_bytes);
    void* ews = cv.take<char>(d.eri_ws);
    double* zr = d.split ? nullptr : cv.take<double>(d.zr);
    float* zf = d.split ? cv.take<float>(d.zr) : nullptr;
    double2* b1 = cv.take<double2>(d.buf);
    double2* b2 = cv.take<double2>(d.buf);
    double* zg = cv.take<double>(d.zg);
    void* part = cv.take<char>(d.part);
    if (cv.bytes() > ws_bytes) return fail(DMET_E_WORKSPACE, "fftdf workspace too small");
    for (int a = 0; a < 3; ++a)
        if ((long)grid->n[a] * p.mesh.n[a] > PW_MAXL)
            return fail(DMET_E_UNSUPPORTED, "fftdf: at most 8192 supercell grid points per axis (N_d n_d)");
    // embedded pair densities on the grid, real rows per q block (Alg. 1 transform)
    dmet_status s = d.split ? lp_transform(p, rho, ck, zf, ews, d.eri_ws, st)
                            : eri_f64(p, rho, ck, nullptr, nullptr, nullptr, ews, d.eri_ws, st, zr);
    if (s != DMET_OK) return s;
    PwScale ks;
    for (int a = 0; a < 3; ++a) {
        ks.n[a] = grid->n[a];
        ks.nmesh[a] = p.mesh.n[a];
    }
    reciprocal(grid->cell, ks.b, ks.omega);
    ks.dv = ks.omega / (double)d.nr;
    {   // root tables above 64 KB of LDS need the larger dynamic allocation
        int lmax = 0;
        for (int a = 0; a < 3; ++a) lmax = std::max(lmax, grid->n[a] * p.mesh.n[a] * (int)sizeof(double2));
        const void* ks6[6] = {(const void*)k_pw_axis<1, 0>,        (const void*)k_pw_axis<2, 0>,
                              (const void*)k_pw_axis<1, 0, float>, (const void*)k_pw_axis<2, 0, float>,
                              (const void*)k_pw_axis<0, 0>,        (const void*)k_pw_axis<0, 1>};
        for (const void* kf : ks6) DMET_HIP(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, lmax));
    }
    // one thread per line along the axis and pair
    auto nb = [&](int a) {
        return (unsigned)std::min<long>(((long)d.nr / grid->n[a] * p.npair + 255) / 256, 65535L * 4);
    };
    for (int sp = 0; sp < p.nspin; ++sp) {
        const double* zs = d.split ? nullptr : zr + (size_t)sp * p.zrows * p.npair;
        const float* zsf = d.split ? zf + (size_t)sp * p.zrows * p.npair : nullptr;
        double* zgs = zg + (size_t)sp * d.krows_p * d.ldz;
        if (d.krows_p > d.zrows_g)   // zero rows up to a multiple of 16 for the contraction
            fill_zero(zgs + (size_t)d.zrows_g * d.ldz, (size_t)(d.krows_p - d.zrows_g) * d.ldz * sizeof(double), st);
        for (size_t b = 0; b < p.qblocks.size(); ++b) {
            const QBlock& qb = p.qblocks[b];
            const int q2 = qb.q % p.mesh.n[2], q1 = (qb.q / p.mesh.n[2]) % p.mesh.n[1],
                      q0 = qb.q / (p.mesh.n[1] * p.mesh.n[2]);
            const int m[3] = {q0, q1, q2};
            for (int a = 0; a < 3; ++a) ks.m[a] = m[a];
            PwAxis ax;
            for (int a = 0; a < 3; ++a) ax.n[a] = grid->n[a];
            ProfScope ps("fftdf_dft", st);
            auto lds = [&](int a) { return (size_t)grid->n[a] * p.mesh.n[a] * sizeof(double2); };
            ax.axis = 0;
            ax.nmesh = p.mesh.n[0];
            ax.m = m[0];
            if (d.split && qb.self_conj)
                k_pw_axis<1, 0, float><<<nb(0), 256, lds(0), st>>>(ax, p.npair, nullptr, zsf, qb.zrow0, p.npair, b1,
                                                                nullptr, 0, ks);
            else if (d.split)
                k_pw_axis<2, 0, float><<<nb(0), 256, lds(0), st>>>(ax, p.npair, nullptr, zsf, qb.zrow0, p.npair, b1,
                                                                nullptr, 0, ks);
            else if (qb.self_conj)
                k_pw_axis<1, 0><<<nb(0), 256, lds(0), st>>>(ax, p.npair, nullptr, zs, qb.zrow0, p.npair, b1, nullptr, 0,
                                                         ks);
            else
                k_pw_axis<2, 0><<<nb(0), 256, lds(0), st>>>(ax, p.npair, nullptr, zs, qb.zrow0, p.npair, b1, nullptr, 0,
                                                         ks);
            ax.axis = 1;
            ax.nmesh = p.mesh.n[1];
            ax.m = m[1];
            k_pw_axis<0, 0, double><<<nb(1), 256, lds(1), st>>>(ax, p.npair, b1, nullptr, 0, p.npair, b2, nullptr, 0, ks);
            ax.axis = 2;
            ax.nmesh = p.mesh.n[2];
            ax.m = m[2];
            k_pw_axis<0, 1, double><<<nb(2), 256, lds(2), st>>>(ax, p.npair, b2, nullptr, 0, d.ldz, nullptr, zgs, 2 * d.nr * b,
                                                     ks);
            ps.stop();
            DMET_LAUNCH_CHECK("k_pw_axis");
        }
    }
    if (d.split)
        return lp_rows_contract(p.prec, p.nspin, p.npair, d.krows_p, zg, (size_t)d.krows_p * d.ldz, (size_t)d.ldz,
                                eri_aa, eri_bb, eri_ab, part, d.part, st);
    return contract_f64(p.nspin, p.npair, d.ldz, d.krows_p, zg, eri_aa, eri_bb, eri_ab, static_cast<double*>(part),
                        st);
}

}  // namespace dmet
