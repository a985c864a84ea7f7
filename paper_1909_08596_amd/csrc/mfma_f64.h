// FP64 MFMA tile helpers (v_mfma_f64_16x16x4f64), internal header.
#pragma once

#include "common.h"

namespace dmet {

typedef double d4 __attribute__((ext_vector_type(4)));

// 256 threads = 4 waves in a 2 x 2 grid; each wave owns a (BM/2) x (BN/2)
// block of 16 x 16 MFMA tiles.  Operands are staged in LDS K-major:
// As[k][m], Bs[k][n].
template <int BM, int BN, int BK>
struct F64Tile {
    static constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    static constexpr int LDA = BM + 2, LDB = BN + 2;
};

template <int BM, int BN, int BK>
__device__ inline void f64_mma(const double* As, const double* Bs, d4 (&acc)[BM / 32][BN / 32]) {
    using T = F64Tile<BM, BN, BK>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave >> 1) * T::WM, wn0 = (wave & 1) * T::WN;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        double a[T::TM], b[T::TN];
#pragma unroll
        for (int i = 0; i < T::TM; ++i) a[i] = As[kr * T::LDA + wm0 + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < T::TN; ++j) b[j] = Bs[kr * T::LDB + wn0 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < T::TM; ++i)
#pragma unroll
            for (int j = 0; j < T::TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// Visit the accumulator: fn(row, col, value) in tile-local coordinates.
// v_mfma_f64_16x16x4f64 result layout: register r of lane l holds
// D[4 r + l / 16][l % 16] (operands: A[l % 16][l / 16], B[l / 16][l % 16]).
template <int BM, int BN, int BK, class Fn>
__device__ inline void f64_visit(const d4 (&acc)[BM / 32][BN / 32], Fn fn) {
    using T = F64Tile<BM, BN, BK>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave >> 1) * T::WM, wn0 = (wave & 1) * T::WN;
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
        for (int j = 0; j < T::TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                fn(wm0 + i * 16 + r * 4 + (lane >> 4), wn0 + j * 16 + (lane & 15), acc[i][j][r]);
}

template <int BM, int BN>
__device__ inline void zero_acc(d4 (&acc)[BM / 32][BN / 32]) {
#pragma unroll
    for (int i = 0; i < BM / 32; ++i)
#pragma unroll
        for (int j = 0; j < BN / 32; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

}  // namespace dmet
