// Shared device/host helpers of libdmet (internal header).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "dmet.h"

namespace dmet {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
dmet_status fail(dmet_status st, const std::string& msg);
dmet_status hip_fail(hipError_t e, const char* what);

#define DMET_HIP(call)                                                    \
    do {                                                                  \
        hipError_t e__ = (call);                                          \
        if (e__ != hipSuccess) return ::dmet::hip_fail(e__, #call);       \
    } while (0)

#define DMET_LAUNCH_CHECK(what)                                           \
    do {                                                                  \
        hipError_t e__ = hipGetLastError();                               \
        if (e__ != hipSuccess) return ::dmet::hip_fail(e__, what);        \
    } while (0)

// ---------------------------------------------------------------- mesh
struct Mesh {
    int n[3];
    int nk;
};

inline Mesh make_mesh(const int kmesh[3]) {
    Mesh m;
    m.n[0] = kmesh[0];
    m.n[1] = kmesh[1];
    m.n[2] = kmesh[2];
    m.nk = kmesh[0] * kmesh[1] * kmesh[2];
    return m;
}

// Index of a - b (wrapped per axis) for row-major mesh indices a, b.
__host__ __device__ inline int mesh_sub(const Mesh& m, int a, int b) {
    int a2 = a % m.n[2], b2 = b % m.n[2];
    int a1 = (a / m.n[2]) % m.n[1], b1 = (b / m.n[2]) % m.n[1];
    int a0 = a / (m.n[1] * m.n[2]), b0 = b / (m.n[1] * m.n[2]);
    int d0 = (a0 - b0 + m.n[0]) % m.n[0];
    int d1 = (a1 - b1 + m.n[1]) % m.n[1];
    int d2 = (a2 - b2 + m.n[2]) % m.n[2];
    return (d0 * m.n[1] + d1) * m.n[2] + d2;
}

__host__ __device__ inline int mesh_neg(const Mesh& m, int a) { return mesh_sub(m, 0, a); }

// exp(i k.R) = exp(2 pi i sum_d n_d m_d / N_d).  The phase is reduced exactly
// in integers (numerator over N_k) before the sincos, so k.R never loses bits.
__device__ inline double2 phase_kR(const Mesh& m, int k, int r) {
    int k2 = k % m.n[2], r2 = r % m.n[2];
    int k1 = (k / m.n[2]) % m.n[1], r1 = (r / m.n[2]) % m.n[1];
    int k0 = k / (m.n[1] * m.n[2]), r0 = r / (m.n[1] * m.n[2]);
    long num = (long)k0 * r0 * (m.nk / m.n[0]) + (long)k1 * r1 * (m.nk / m.n[1]) +
               (long)k2 * r2 * (m.nk / m.n[2]);
    num %= m.nk;
    double s, c;
    sincospi(2.0 * (double)num / (double)m.nk, &s, &c);
    return make_double2(c, s);
}

// ---------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Carve {
    char* base;
    size_t cap;
    size_t used = 0;
    Carve(void* p, size_t n) : base(static_cast<char*>(p)), cap(n) {}
    template <class T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        if (base == nullptr) return nullptr;  // sizing pass
        return reinterpret_cast<T*>(base + off);
    }
    size_t bytes() const { return (used + 255) & ~size_t(255); }
};

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int wave_min_int(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// atomic max of a non-negative double (IEEE order == integer order for >= 0)
__device__ inline void atomic_max_nonneg(double* addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(addr),
              (unsigned long long)__double_as_longlong(v));
}

// status word written by device code (0 = ok), read by hosts that sync
enum DeviceFlag : int { FLAG_NONFINITE = 1, FLAG_NOCONV = 2 };

// Per-launch event timing (enabled by dmet_profile_enable).  Usage:
//   ProfScope ps("name", stream); kernel<<<...>>>; ps.stop();
struct ProfScope {
    int slot;
    hipStream_t st;
    ProfScope(const char* name, hipStream_t s);
    void stop();
};

// Suspends the profiler's event records (during a graph capture: events
// recorded into a graph cannot be timed).  Returns the previous state.
bool prof_suspend(bool on);

// small fill kernel (used instead of hipMemsetAsync so callers may capture)
void fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace dmet
