// Internal declarations of liblbmp: D3Q19 tables, error plumbing, handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/lbmp.h"

namespace lbmp {

// ---------------------------------------------------------------- lattice
// D3Q19 moving links (Sec. I of the paper: 19 velocities incl. rest). Link k
// and k^1 are opposite. Face links first (weight 1/18), then edge links (1/36).
constexpr int NL = 18;
__host__ __device__ constexpr int lcx(int k) {
    constexpr int t[NL] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[k];
}
__host__ __device__ constexpr int lcy(int k) {
    constexpr int t[NL] = {0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[k];
}
__host__ __device__ constexpr int lcz(int k) {
    constexpr int t[NL] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[k];
}
__host__ __device__ constexpr double lw(int k) { return k < 6 ? 1.0 / 18.0 : 1.0 / 36.0; }
constexpr double W_REST = 1.0 / 3.0;

__host__ __device__ inline int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
lbmp_status fail(lbmp_status st, const char* fmt, ...);

#define LBMP_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::lbmp::fail(LBMP_EDEVICE, "%s failed: %s (%s:%d)", #call,            \
                                hipGetErrorString(e_), __FILE__, __LINE__);              \
    } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided device workspace.
struct Carver {
    char* base;
    size_t cap, off = 0;
    Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        size_t bytes = align_up(count * sizeof(T));
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += bytes;
        return p;
    }
    bool fits() const { return off <= cap; }
};

// ---------------------------------------------------------------- handles
constexpr uint32_t FLOW_MAGIC = 0x4c42464cu;  // "LBFL"
constexpr uint32_t MP_MAGIC = 0x4c424d50u;    // "LBMP"

struct FlowLayout {
    uint8_t* solid;
    int8_t* cls;
    int32_t* slot;   // interface slot per node, -1 elsewhere
    int32_t* ilist;  // node index per interface slot (ascending)
    double* u;       // [3][N]
    int64_t* counts; // [2] fluid, interface
    uint32_t* blk;   // per-1024-node block counts / offsets, 2 arrays
};

struct lbmp_flow_impl;

}  // namespace lbmp

struct lbmp_flow {
    uint32_t magic;
    int nx, ny, nz, nbhd;
    int64_t N, nf, ni;
    lbmp::FlowLayout d;
    int converged;
    int64_t steps;
    double residual;
};

namespace lbmp {
lbmp_status build_geometry(const lbmp_geometry* g, Carver& c, FlowLayout& L, hipStream_t s,
                           int64_t* nf, int64_t* ni);
size_t geometry_bytes(int64_t N);
lbmp_status validate_geometry(const lbmp_geometry* g);
}  // namespace lbmp
