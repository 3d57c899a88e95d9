// Moment propagation with adsorption/desorption (Secs. II-III of the paper).
//
// Formulation on the device (the arithmetic of Eqs. 7, 9 and 10, rearranged
// for FP32 storage; the CPU oracle keeps the literal form):
//  * every propagated quantity X (density, first moments x, y, z) and its
//    adsorbed counterpart are stored as deviations from a reference
//    c_q * rho_ref (mobile) and c_q * Gamma_ref (adsorbed), where rho_ref and
//    Gamma_ref are the Eq. 11 weights and c_q = 1 for the density and the mean
//    velocity V_q for the first moments — the long-time limit of each field;
//  * the receiving node pulls Y = sum_i X(r - c_i) p_i(r - c_i) over a
//    receiver-indexed table pin[i][r] = p_i(r - c_i): an FP64 FMA chain in
//    the direct, box and z-march kernels; in the LDS-DMA and gathered-chunk
//    kernels three FP32 FMA chains in link order (links with c_ix = 0, +1,
//    -1), converted and added in that order (the stochastically rounded
//    inputs keep their round-to-nearest residuals from repeating);
//  * X' = ((fma(-X, sigma, X) - p_a X + p_d X_ads) + c_q rho_ref src) + Y
//    with sigma(r) = sum_i p_i(r) rounded once, and src(r) = sum_i pin_i(r) -
//    sum_i p_i(r) formed exactly from the stored probabilities (zero wherever
//    the Eq. 11 weights are stationary, e.g. slits with or without flow);
//  * adsorption and desorption fluxes p_a X, p_d X_ads are rounded once and
//    used on both sides, so Eqs. 9-10 exchange the same amount;
//  * the VACF sum of Eq. 12 and the conserved totals are accumulated in FP64
//    per block and reduced in a fixed order (bitwise reproducible).
//
// Batching: one launch advances every (geometry, species) pair. The logical
// block list is (geometry, tile, species group) with the group fastest; a
// tile is BLK lattice columns x K consecutive z-planes. Blocks are remapped
// so each XCD receives a contiguous range of logical blocks. The state time
// and ping-pong parity live in device memory, so a captured graph of steps
// can be replayed.
#include <sys/stat.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <cstdlib>
#include <cmath>
#include <map>
#include <tuple>
#include <type_traits>

#include "lbmp_internal.hpp"

namespace lbmp {

constexpr int BLK = 256;   // threads per block (4 waves)
constexpr int NRED = 8;    // FP64 sums per (species, step)
constexpr int KC = 16;     // FP64 constants per species for the DMA kernel
constexpr int SETUP_RED = 12;

template <typename T>
struct GeomDev {
    int nx, ny, nz, S;
    int64_t N, NI;
    int pb, zb, ngrp;          // plane blocks, z blocks, species groups
    int64_t ntile;             // tiles of the launched kernel variant
    int64_t blk0;              // first logical block of this geometry
    const int8_t* cls;
    const int32_t* slot;
    const T* pin;              // [18][N]
    const double* sig;         // [N] sum_i p_i(r), exact (FP64)
    const T* src;              // [N]
    const T* a;                // [3][N]
    T* X0;                     // [S][4][NC]
    T* X1;                     // [S][4][NC]
    T* Xa;                     // [S][4][NI]
    // compact storage (haloed LDS-DMA blocks): the fields and the link data
    // (pin, sig, src, a: each row's first NC entries) of fluid node n at
    // fidx[n] (-1 on solid nodes), NC = fluid nodes; dense otherwise: fidx
    // null, NC = N
    const int32_t* fidx;
    int64_t NC;
    // gathered chunks (variant 8): chunk c covers compact nodes
    // gch[c].x .. gch[c].x + gch[c].y - 1 (one per thread) and the halo
    // quads starting at the compact nodes ghsrc[gch[c].z .. + gch[c].w - 1];
    // node i's lattice index gnode[i], its
    // adsorbed-field index gaslot[i] (-1 off the interface) and, per link k,
    // the region slot of r - c_k in gnbr[k * NC + i]
    const int4* gch;
    const int32_t* ghsrc;
    const int32_t* gnode;
    const int32_t* gaslot;
    const uint16_t* gnbr;
    const T* coef;             // [S][4]
    const T* prob;             // [S][2] = p_a, p_d
    const double* kc;          // [S][KC]: p_a, p_d, c_0..c_3 (coef), -V_0..-V_2, FP64
    double* part;              // [S][ntile][NRED]
    double* series;            // [Tmax][S][NRED], entry t-1 holds time t
};

struct Ctl {
    int64_t t;      // time of the current state (1 after init)
    int64_t tmax;   // last recordable time
    uint32_t done;  // blocks of the series reduction finished in this step (0 between steps)
    // watchdog: first recorded time at which some species' total probability
    // (mobile + adsorbed, its recorded deviation from mass_ref) exceeded
    // drift_max in magnitude or was not finite; INT64_MAX while none has
    int64_t bad_t;
    double mass_ref;   // 0: totals recorded as deviations from the Eq. 11 weights; 1: as they are
    double drift_max;
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    // blockIdx b runs on XCD b % 8; give each XCD a contiguous logical range
    int64_t per = nb / 8, rem = nb % 8;
    int64_t x = b % 8, i = b / 8;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + i;
}

__device__ __forceinline__ int modp(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Fixed-order sum of NRED doubles over the BLK threads of a block; thread k < NRED
// of the block receives sum k in `res`.
__device__ __forceinline__ void block_sum8(double (&v)[NRED], double* lds, double& res) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NRED; ++k) lds[k * BLK + tid] = v[k];
    __syncthreads();
    const int k = tid >> 5, l = tid & 31;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < BLK / 32; ++j) s += lds[k * BLK + l * (BLK / 32) + j];
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 32);
    __syncthreads();
    if (l == 0) lds[k] = s;
    __syncthreads();
    res = tid < NRED ? lds[tid] : 0.0;
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ int find_geom(const GeomDev<T>* G, int ng, int64_t lb) {
    int lo = 0, hi = ng - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (G[mid].blk0 <= lb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Raw buffer access: a 128-bit resource per array (base, size in bytes); an
// offset at or beyond the size reads 0 and drops the store, which is how
// inactive lanes are masked without branches.
constexpr int OOB = 0x7ffffff0;
constexpr int RSRC_WORD3 = 0x00020000;  // gfx9-family raw buffer format word

__device__ __forceinline__ __amdgpu_buffer_rsrc_t mkrsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, RSRC_WORD3);
}
__device__ __forceinline__ float bload(float*, __amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bload(double*, __amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float bload(float*, __amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
__device__ __forceinline__ double bload(double*, __amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, int off, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, 0);
}
// Non-temporal (streaming) store: the LDS-DMA blocks' stepped fields, which
// no block reads again within the step, so that they leave the L2 to the
// halo rows and planes that neighbouring blocks do read (2.7 % faster on the
// batched slits; no gain for the gathered chunks, which keep plain stores).
__device__ __forceinline__ void bstore_nt(float v, __amdgpu_buffer_rsrc_t r, int off, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, 2);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, int off, int soff) {
    using v2u = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, off, soff, 0);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, int off) {
    using v2u = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, off, 0, 0);
}

// Counter-based random bits for stochastic rounding: one 32-bit hash per
// (node, step) seeds a xorshift32 stream (Marsaglia 2003) that is advanced once
// per stored value; runs are reproducible.
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    // integer finaliser of MurmurHash3
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t xorshift32(uint32_t& s) {
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    return s;
}
// Round v to FP32 stochastically: up (in magnitude) with probability equal to
// the discarded fraction of an FP32 unit in the last place, so the expected
// stored value is v. Adds 29 random bits below the FP32 mantissa of the FP64
// pattern and truncates them.
__device__ __forceinline__ float sround(double v, uint32_t r) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    b = (b + (r & 0x1fffffffu)) & ~(uint64_t)0x1fffffffu;
    return (float)__longlong_as_double((long long)b);
}
template <typename T> __device__ __forceinline__ T store_round(double v, uint32_t r);
template <> __device__ __forceinline__ float store_round<float>(double v, uint32_t r) { return sround(v, r); }
template <> __device__ __forceinline__ double store_round<double>(double v, uint32_t) { return v; }

// One propagation step for every (geometry, species) pair. Loads and stores
// are in the storage type T; the update itself is FP64 (an FMA chain for the
// arrivals, the exact FP64 sum of the departures), rounded once on store —
// stochastically for FP32 storage, so that no rounding direction repeats from
// step to step.
template <typename T, int K>
__global__ void __launch_bounds__(BLK) k_mp_step(const GeomDev<T>* __restrict__ geoms, int ngeom,
                                                 int gsz, int64_t nblocks, const Ctl* __restrict__ ctl) {
    __shared__ double lds[NRED * BLK];
    constexpr int E = (int)sizeof(T);
    T* const tag = nullptr;
    double* const dtag = nullptr;
    const int64_t lb = xcd_remap(blockIdx.x, nblocks);
    const int gi = find_geom(geoms, ngeom, lb);
    const GeomDev<T>& G = geoms[gi];
    const int64_t local = lb - G.blk0;
    const int grp = (int)(local % G.ngrp);
    const int64_t tile = local / G.ngrp;
    const int pbi = (int)(tile % G.pb), zbi = (int)(tile / G.pb);
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int N = (int)G.N, plane = nx * ny;
    const int p = pbi * BLK + threadIdx.x;
    const bool inplane = p < plane;
    const int x = inplane ? p % nx : 0, y = inplane ? p / nx : 0;
    const int z0 = zbi * K;
    const int xm = modp(x - 1, nx), xp = modp(x + 1, nx), ym = modp(y - 1, ny), yp = modp(y + 1, ny);
    // in-plane positions: 0 centre, 1 (x-1,y), 2 (x+1,y), 3 (x,y-1), 4 (x,y+1);
    // diagonals: 0 (x-1,y-1), 1 (x+1,y+1), 2 (x-1,y+1), 3 (x+1,y-1)
    const int o5[5] = {x + nx * y, xm + nx * y, xp + nx * y, x + nx * ym, x + nx * yp};
    const int od[4] = {xm + nx * ym, xp + nx * yp, xm + nx * yp, xp + nx * ym};
    int off5[K + 2][5], offd[K][4], offn[K], offa[K];
#pragma unroll
    for (int j = 0; j < K + 2; ++j) {
        const int zo = modp(z0 - 1 + j, nz) * plane;
#pragma unroll
        for (int c = 0; c < 5; ++c) off5[j][c] = inplane ? (zo + o5[c]) * E : OOB;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int zo = modp(z0 + j, nz) * plane;
#pragma unroll
        for (int c = 0; c < 4; ++c) offd[j][c] = inplane ? (zo + od[c]) * E : OOB;
    }
    const int64_t t = ctl->t;
    // per-node link data (FP64 in registers); inactive nodes read zeros
    bool act[K], isI[K];
    double pin[K][NL], sig[K], src[K], av[K][3];
    uint32_t rbase[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int n = modp(z0 + j, nz) * plane + o5[0];
        act[j] = inplane && (z0 + j < nz) && G.cls[n] != 0;
        const int sl = act[j] ? G.slot[n] : -1;
        isI[j] = sl >= 0;
        offn[j] = act[j] ? n * E : OOB;
        offa[j] = isI[j] ? sl * E : OOB;
        const int offn8 = act[j] ? n * 8 : OOB;
#pragma unroll
        for (int k = 0; k < NL; ++k)
            pin[j][k] = (double)bload(tag, mkrsrc(G.pin + (int64_t)k * N, (int64_t)N * E), offn[j]);
        sig[j] = bload(dtag, mkrsrc(G.sig, (int64_t)N * 8), offn8);
        src[j] = (double)bload(tag, mkrsrc(G.src, (int64_t)N * E), offn[j]);
#pragma unroll
        for (int g = 0; g < 3; ++g)
            av[j][g] = (double)bload(tag, mkrsrc(G.a + (int64_t)g * N, (int64_t)N * E), offn[j]);
        rbase[j] = hash32((uint32_t)n * 0x9e3779b9u ^ hash32((uint32_t)t ^ ((uint32_t)gi << 24)));
    }
    const T* Xin = (t & 1) ? G.X1 : G.X0;
    T* Xout = (t & 1) ? G.X0 : G.X1;
    const int s_begin = grp * gsz, s_end = min(G.S, s_begin + gsz);
    const int64_t ntile = G.ntile;
    const int64_t NI = G.NI;

    for (int s = s_begin; s < s_end; ++s) {
        const double pa = (double)G.prob[2 * s], pd = (double)G.prob[2 * s + 1];
        uint32_t rs[K];  // random stream of (node, step, species)
#pragma unroll
        for (int j = 0; j < K; ++j) rs[j] = hash32(rbase[j] ^ ((uint32_t)s * 0x632be5abu)) | 1u;
        double red[NRED];
#pragma unroll
        for (int k = 0; k < NRED; ++k) red[k] = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double cq = (double)G.coef[4 * s + q];
            const int64_t f = 4 * s + q;
            const auto rin = mkrsrc(Xin + f * N, (int64_t)N * E);
            const auto rout = mkrsrc(Xout + f * N, (int64_t)N * E);
            const auto rads = mkrsrc(G.Xa + f * NI, NI * E);
            double v5[K + 2][5], vd[K][4], xa[K];
#pragma unroll
            for (int j = 0; j < K + 2; ++j)
#pragma unroll
                for (int c = 0; c < 5; ++c) v5[j][c] = (double)bload(tag, rin, off5[j][c]);
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c) vd[j][c] = (double)bload(tag, rin, offd[j][c]);
#pragma unroll
            for (int j = 0; j < K; ++j) xa[j] = (double)bload(tag, rads, offa[j]);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                // arrivals (Eq. 7): source node r - c_k of link k
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < NL; ++k) {
                    const int dx = -lcx(k), dy = -lcy(k), dz = -lcz(k);
                    double v;
                    if (dz == 0 && dx != 0 && dy != 0) {
                        const int c = (dx < 0 && dy < 0) ? 0 : (dx > 0 && dy > 0) ? 1 : (dx < 0) ? 2 : 3;
                        v = vd[j][c];
                    } else {
                        const int c = dx < 0 ? 1 : dx > 0 ? 2 : dy < 0 ? 3 : dy > 0 ? 4 : 0;
                        v = v5[j + 1 + dz][c];
                    }
                    acc = __builtin_fma(v, pin[j][k], acc);
                }
                const double xc = v5[j + 1][0];
                const double fa = isI[j] ? pa * xc : 0.0;   // adsorption (Eq. 9)
                const double fd = pd * xa[j];               // desorption (Eq. 10); xa = 0 off the interface
                double nv = __builtin_fma(-xc, sig[j], xc); // the part that stays (Eq. 7)
                nv = __builtin_fma(cq, src[j], (nv - fa) + fd) + acc;
                const uint32_t r1 = xorshift32(rs[j]);
                bstore(store_round<T>(nv, r1), rout, offn[j]);
                bstore(store_round<T>((xa[j] + fa) - fd, (r1 >> 3) | (r1 << 29)), rads, offa[j]);
                const double xd = act[j] ? xc : 0.0;
                if (q == 0) {
                    red[3] += xd;
                    red[7] += xa[j];
                } else {
                    red[q - 1] = __builtin_fma(xd, av[j][q - 1], red[q - 1]);
                    red[3 + q] += xd + xa[j];
                }
            }
        }
        double r;
        block_sum8(red, lds, r);
        if (threadIdx.x < NRED)
            G.part[((int64_t)s * ntile + tile) * NRED + threadIdx.x] = r;
    }
}

// The same step with each field staged through LDS. A block owns a tile of
// TX x TY lattice columns and K consecutive z-planes; for every field (species,
// quantity) the block loads the tile plus a one-node periodic halo, a box of
// (K+2) x (TY+2) x (TX+2) values, into one of two LDS buffers while it updates
// the previous field from the other buffer. Link data stay in registers for
// all the fields of the block.
constexpr int TX = 64, TY = BLK / TX;

template <int K>
struct Box {
    static constexpr int PX = TX + 2, PY = TY + 2, PL = PX * PY, N = PL * (K + 2);
    static constexpr int LOADS = (N + BLK - 1) / BLK;
};

template <typename T, int K>
__global__ void __launch_bounds__(BLK) k_mp_step_box(const GeomDev<T>* __restrict__ geoms, int ngeom,
                                                     int gsz, int64_t nblocks, const Ctl* __restrict__ ctl) {
    using B = Box<K>;
    __shared__ T box[2][B::LOADS * BLK];
    __shared__ double lds[NRED * BLK];
    constexpr int E = (int)sizeof(T);
    T* const tag = nullptr;
    double* const dtag = nullptr;
    const int64_t lb = xcd_remap(blockIdx.x, nblocks);
    const int gi = find_geom(geoms, ngeom, lb);
    const GeomDev<T>& G = geoms[gi];
    const int64_t local = lb - G.blk0;
    const int grp = (int)(local % G.ngrp);
    const int64_t tile = local / G.ngrp;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int txi = (int)(tile % ntx), tyi = (int)((tile / ntx) % nty), zbi = (int)(tile / ((int64_t)ntx * nty));
    const int x0 = txi * TX, y0 = tyi * TY, z0 = zbi * K;
    const int N = (int)G.N, plane = nx * ny;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool inplane = x < nx && y < ny;
    // global offsets of this thread's share of the box (same for every field)
    int goff[B::LOADS];
#pragma unroll
    for (int i = 0; i < B::LOADS; ++i) {
        const int e = tid + i * BLK;
        if (e < B::N) {
            const int j = e / B::PL, r = e % B::PL, yy = r / B::PX, xx = r % B::PX;
            const int gx = modp(x0 - 1 + xx, nx), gy = modp(y0 - 1 + yy, ny), gz = modp(z0 - 1 + j, nz);
            goff[i] = (gz * plane + gy * nx + gx) * E;
        } else {
            goff[i] = OOB;
        }
    }
    const int64_t t = ctl->t;
    bool act[K], isI[K];
    int offn[K], offa[K];
    double pin[K][NL], sig[K], src[K], av[K][3];
    uint32_t rbase[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int n = modp(z0 + j, nz) * plane + (inplane ? y * nx + x : 0);
        act[j] = inplane && (z0 + j < nz) && G.cls[n] != 0;
        const int sl = act[j] ? G.slot[n] : -1;
        isI[j] = sl >= 0;
        offn[j] = act[j] ? n * E : OOB;
        offa[j] = isI[j] ? sl * E : OOB;
        const int offn8 = act[j] ? n * 8 : OOB;
#pragma unroll
        for (int k = 0; k < NL; ++k)
            pin[j][k] = (double)bload(tag, mkrsrc(G.pin + (int64_t)k * N, (int64_t)N * E), offn[j]);
        sig[j] = bload(dtag, mkrsrc(G.sig, (int64_t)N * 8), offn8);
        src[j] = (double)bload(tag, mkrsrc(G.src, (int64_t)N * E), offn[j]);
#pragma unroll
        for (int g = 0; g < 3; ++g)
            av[j][g] = (double)bload(tag, mkrsrc(G.a + (int64_t)g * N, (int64_t)N * E), offn[j]);
        rbase[j] = hash32((uint32_t)n * 0x9e3779b9u ^ hash32((uint32_t)t ^ ((uint32_t)gi << 24)));
    }
    const T* Xin = (t & 1) ? G.X1 : G.X0;
    T* Xout = (t & 1) ? G.X0 : G.X1;
    const int s_begin = grp * gsz, s_end = min(G.S, s_begin + gsz);
    const int nf = 4 * (s_end - s_begin);
    const int64_t ntile = G.ntile;
    const int64_t NI = G.NI;

    // prologue: field 0 into buffer 0
    T pre[B::LOADS];
    {
        const auto r0 = mkrsrc(Xin + (int64_t)(4 * s_begin) * N, (int64_t)N * E);
#pragma unroll
        for (int i = 0; i < B::LOADS; ++i) pre[i] = bload(tag, r0, goff[i]);
#pragma unroll
        for (int i = 0; i < B::LOADS; ++i) box[0][tid + i * BLK] = pre[i];
    }
    __syncthreads();

    double red[NRED];
    uint32_t rs[K];
    double pa = 0.0, pd = 0.0;
    for (int fi = 0; fi < nf; ++fi) {
        const int s = s_begin + fi / 4, q = fi % 4;
        const int64_t f = 4 * s + q;
        if (q == 0) {
            pa = (double)G.prob[2 * s];
            pd = (double)G.prob[2 * s + 1];
#pragma unroll
            for (int j = 0; j < K; ++j) rs[j] = hash32(rbase[j] ^ ((uint32_t)s * 0x632be5abu)) | 1u;
#pragma unroll
            for (int k = 0; k < NRED; ++k) red[k] = 0.0;
        }
        // prefetch the next field
        if (fi + 1 < nf) {
            const auto rn = mkrsrc(Xin + (f + 1) * N, (int64_t)N * E);
#pragma unroll
            for (int i = 0; i < B::LOADS; ++i) pre[i] = bload(tag, rn, goff[i]);
        }
        const auto rout = mkrsrc(Xout + f * N, (int64_t)N * E);
        const auto rads = mkrsrc(G.Xa + f * NI, NI * E);
        double xa[K];
#pragma unroll
        for (int j = 0; j < K; ++j) xa[j] = (double)bload(tag, rads, offa[j]);
        const double cq = (double)G.coef[f];
        const T* bx = box[fi & 1];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            // centre of node j in the box: plane j+1, row ly+1, column lx+1
            const int c0 = (j + 1) * B::PL + (ly + 1) * B::PX + (lx + 1);
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int o = -lcz(k) * B::PL - lcy(k) * B::PX - lcx(k);
                acc = __builtin_fma((double)bx[c0 + o], pin[j][k], acc);
            }
            const double xc = (double)bx[c0];
            const double fa = isI[j] ? pa * xc : 0.0;
            const double fd = pd * xa[j];
            double nv = __builtin_fma(-xc, sig[j], xc);
            nv = __builtin_fma(cq, src[j], (nv - fa) + fd) + acc;
            const uint32_t r1 = xorshift32(rs[j]);
            bstore(store_round<T>(nv, r1), rout, offn[j]);
            bstore(store_round<T>((xa[j] + fa) - fd, (r1 >> 3) | (r1 << 29)), rads, offa[j]);
            const double xd = act[j] ? xc : 0.0;
            if (q == 0) {
                red[3] += xd;
                red[7] += xa[j];
            } else {
                red[q - 1] = __builtin_fma(xd, av[j][q - 1], red[q - 1]);
                red[3 + q] += xd + xa[j];
            }
        }
        if (fi + 1 < nf) {
#pragma unroll
            for (int i = 0; i < B::LOADS; ++i) box[(fi + 1) & 1][tid + i * BLK] = pre[i];
        }
        if (q == 3) {
            double r;
            block_sum8(red, lds, r);   // synchronises the block
            if (tid < NRED) G.part[((int64_t)s * ntile + tile) * NRED + tid] = r;
        } else {
            __syncthreads();
        }
    }
}

// The step as a z-march. A block owns a tile of TX x TY lattice columns, a
// segment of consecutive z-planes and a group of G species (F = 4G fields).
// It keeps, for every field, the planes z-1, z, z+1 of the tile plus a
// one-node periodic halo in an LDS ring; plane z+2 is fetched from global
// memory while plane z is updated. Each field value is thus read from global
// memory once per step (plus the halo), the link data of a node once for all
// F fields, and the FP64 sums are reduced across the block once per species.
template <int F>
struct Ring {
    static constexpr int PX = TX + 2, PY = TY + 2, PL = PX * PY;  // one haloed plane
    static constexpr int LOADS = (PL + BLK - 1) / BLK;
};

template <typename T, int G>
__global__ void __launch_bounds__(BLK) k_mp_march(const GeomDev<T>* __restrict__ geoms, int ngeom,
                                                  int64_t nblocks, int zseg, const Ctl* __restrict__ ctl) {
    constexpr int F = 4 * G;
    using R = Ring<F>;
    constexpr size_t RING_BYTES = 3 * F * R::PL * sizeof(T);
    constexpr size_t RED_BYTES = NRED * BLK * sizeof(double);
    __shared__ __align__(16) char smem[RING_BYTES > RED_BYTES ? RING_BYTES : RED_BYTES];
    T* ring = reinterpret_cast<T*>(smem);  // [3][F][PL]
    constexpr int E = (int)sizeof(T);
    T* const tag = nullptr;
    double* const dtag = nullptr;
    const int64_t lb = xcd_remap(blockIdx.x, nblocks);
    const int gi = find_geom(geoms, ngeom, lb);
    const GeomDev<T>& Gm = geoms[gi];
    const int64_t local = lb - Gm.blk0;
    const int grp = (int)(local % Gm.ngrp);
    const int64_t tile = local / Gm.ngrp;
    const int nx = Gm.nx, ny = Gm.ny, nz = Gm.nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int txi = (int)(tile % ntx), tyi = (int)((tile / ntx) % nty), zsi = (int)(tile / ((int64_t)ntx * nty));
    const int x0 = txi * TX, y0 = tyi * TY;
    const int zs = zsi * zseg, ze = min(nz, zs + zseg);
    const int N = (int)Gm.N, plane = nx * ny;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool inplane = x < nx && y < ny;
    const int c0 = (ly + 1) * R::PX + (lx + 1);  // this thread's column in a haloed plane
    const int own = inplane ? y * nx + x : 0;
    int poff[R::LOADS];
#pragma unroll
    for (int i = 0; i < R::LOADS; ++i) {
        const int e = tid + i * BLK;
        poff[i] = e < R::PL ? modp(y0 - 1 + e / R::PX, ny) * nx + modp(x0 - 1 + e % R::PX, nx) : -1;
    }
    const int64_t t = ctl->t;
    const T* Xin = (t & 1) ? Gm.X1 : Gm.X0;
    T* Xout = (t & 1) ? Gm.X0 : Gm.X1;
    const int s0 = grp * G, ns = min(G, Gm.S - s0);
    const int NI = (int)Gm.NI;
    const uint32_t tseed = hash32((uint32_t)t ^ ((uint32_t)gi << 24));
    // one resource per array; field / link index in the scalar offset. Fields
    // beyond the group's species count read 0 and are never stored.
    const auto rin = mkrsrc(Xin + (int64_t)(4 * s0) * N, (int64_t)(4 * ns) * N * E);
    const auto rout = mkrsrc(Xout + (int64_t)(4 * s0) * N, (int64_t)(4 * ns) * N * E);
    const auto rads = mkrsrc(Gm.Xa + (int64_t)(4 * s0) * NI, (int64_t)(4 * ns) * NI * E);
    const auto rpin = mkrsrc(Gm.pin, (int64_t)NL * N * E);
    const auto ra = mkrsrc(Gm.a, (int64_t)3 * N * E);
    const auto rsig = mkrsrc(Gm.sig, (int64_t)N * 8);
    const auto rsrc = mkrsrc(Gm.src, (int64_t)N * E);
    const auto rcls = mkrsrc(Gm.cls, (int64_t)N);
    const auto rslot = mkrsrc(Gm.slot, (int64_t)N * 4);
    double pa[G], pd[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int s = min(s0 + g, Gm.S - 1);
        pa[g] = (double)Gm.prob[2 * s];
        pd[g] = (double)Gm.prob[2 * s + 1];
    }

    auto fetch = [&](int pz, T (&reg)[F][R::LOADS]) {
        const int zo = modp(pz, nz) * plane;
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
            for (int i = 0; i < R::LOADS; ++i)
                reg[f][i] = bload(tag, rin, (f < 4 * ns && poff[i] >= 0) ? (zo + poff[i]) * E : OOB, f * N * E);
    };
    auto stash = [&](int slot, const T (&reg)[F][R::LOADS]) {
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
            for (int i = 0; i < R::LOADS; ++i) {
                const int e = tid + i * BLK;
                if (e < R::PL) ring[(slot * F + f) * R::PL + e] = reg[f][i];
            }
    };
    // node classes two planes ahead, link data and adsorbed values one plane ahead
    auto cls_of = [&](int z) -> int {  // -1: no active node
        if (!inplane || z >= ze) return -1;
        const int n = z * plane + own;
        const int c = (int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(rcls, n, 0, 0);
        return c != 0 ? n : -1;
    };
    struct Link {
        T pin[NL], src, a[3];
        double sig;
        T xa[F];
        int n, sl;
    };
    auto load_link = [&](int n, int sl, Link& L) {
        const int on = n >= 0 ? n * E : OOB, oa = sl >= 0 ? sl * E : OOB;
#pragma unroll
        for (int k = 0; k < NL; ++k) L.pin[k] = bload(tag, rpin, on, k * N * E);
        L.sig = bload(dtag, rsig, n >= 0 ? n * 8 : OOB);
        L.src = bload(tag, rsrc, on);
#pragma unroll
        for (int g = 0; g < 3; ++g) L.a[g] = bload(tag, ra, on, g * N * E);
#pragma unroll
        for (int f = 0; f < F; ++f) L.xa[f] = bload(tag, rads, f < 4 * ns ? oa : OOB, f * NI * E);
        L.n = n;
        L.sl = sl;
    };
    auto slot_of = [&](int n) -> int {
        return n >= 0 ? (int)__builtin_amdgcn_raw_buffer_load_b32(rslot, n * 4, 0, 0) : -1;
    };

    T pre[F][R::LOADS];
    fetch(zs - 1, pre);
    stash(0, pre);
    fetch(zs, pre);
    stash(1, pre);
    fetch(zs + 1, pre);
    stash(2, pre);
    Link cur, nxt;
    int n1 = cls_of(zs + 1);         // node of plane zs+1
    {
        const int n0 = cls_of(zs);
        load_link(n0, slot_of(n0), cur);
    }
    int sl1 = slot_of(n1);
    __syncthreads();

    double red[G][NRED];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < NRED; ++k) red[g][k] = 0.0;

    for (int z = zs; z < ze; ++z) {
        const int sm = (z - zs) % 3, sc = (z - zs + 1) % 3, sp = (z - zs + 2) % 3;
        const bool more = z + 1 < ze;
        // in flight while plane z is updated: plane z+2 of every field, the
        // link data and adsorbed values of node z+1, the class of node z+2
        if (more) fetch(z + 2, pre);
        load_link(n1, sl1, nxt);
        const int n2 = cls_of(z + 2);
        const int sl2 = slot_of(n2);

        const bool act = cur.n >= 0, isI = cur.sl >= 0;
        const int offn = act ? cur.n * E : OOB, offa = isI ? cur.sl * E : OOB;
        double pin[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) pin[k] = (double)cur.pin[k];
        const double sig = cur.sig, src = (double)cur.src;
        const uint32_t rnode = hash32((uint32_t)(z * plane + own) * 0x9e3779b9u ^ tseed);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int s = s0 + g;
            const double pag = isI ? pa[g] : 0.0;
            uint32_t rs = hash32(rnode ^ ((uint32_t)s * 0x632be5abu)) | 1u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = 4 * g + q;
                const T* pm = ring + (sm * F + f) * R::PL;
                const T* pc = ring + (sc * F + f) * R::PL;
                const T* pp = ring + (sp * F + f) * R::PL;
                double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
                for (int k = 0; k < NL; ++k) {
                    const int o = c0 - lcy(k) * R::PX - lcx(k);
                    const T v = lcz(k) > 0 ? pm[o] : (lcz(k) < 0 ? pp[o] : pc[o]);
                    if (k & 1) acc1 = __builtin_fma((double)v, pin[k], acc1);
                    else acc0 = __builtin_fma((double)v, pin[k], acc0);
                }
                const double xc = (double)pc[c0];
                const double xa = (double)cur.xa[f];
                const double fa = pag * xc;
                const double fd = pd[g] * xa;
                double nv = __builtin_fma(-xc, sig, xc);
                nv = __builtin_fma((double)Gm.coef[4 * min(s, Gm.S - 1) + q], src, (nv - fa) + fd) + (acc0 + acc1);
                const uint32_t r1 = xorshift32(rs);
                const int so = f < 4 * ns ? 0 : OOB;  // partial group: no store
                bstore(store_round<T>(nv, r1), rout, offn | so, f * N * E);
                bstore(store_round<T>((xa + fa) - fd, (r1 >> 3) | (r1 << 29)), rads, offa | so, f * NI * E);
                const double xd = act ? xc : 0.0;
                if (q == 0) {
                    red[g][3] += xd;
                    red[g][7] += xa;
                } else {
                    red[g][q - 1] = __builtin_fma(xd, (double)cur.a[q - 1], red[g][q - 1]);
                    red[g][3 + q] += xd + xa;
                }
            }
        }
        __syncthreads();          // every read of plane z-1 is done
        if (more) stash(sm, pre); // plane z+2 takes its slot
        __syncthreads();
        cur = nxt;
        n1 = n2;
        sl1 = sl2;
    }
    // the ring is free: reuse it for the block sums
    double* lds = reinterpret_cast<double*>(smem);
    const int64_t ntile = Gm.ntile;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double r;
        block_sum8(red[g], lds, r);
        if (tid < NRED && g < ns) Gm.part[((int64_t)(s0 + g) * ntile + tile) * NRED + tid] = r;
    }
}

// ------------------------------------------------------------------ variant 3
// FP32 storage. A block owns a TX x (NH TY) tile of one z-plane: NH = 1 or 2
// reduction tiles of TX x TY nodes (4 waves each, with their own partial
// sums); a taller block re-reads fewer halo rows per node and synchronises
// twice as many waves per barrier. For every field (species, quantity) of the
// block, the stencil region — planes z-1, z and z+1 of the tile with a
// one-node periodic halo — and the tile's adsorbed values are copied by the
// buffer unit straight into LDS (buffer_load ... lds: lane i of a wave fills
// dword i of the wave's destination; a lane out of range writes 0), three
// fields ahead of the field being updated, through four LDS stages (stage =
// quantity q). Nothing passes
// through registers on its way in, so the tile's link data stay in registers
// for all the fields of the block. Tiles run x-fastest, then along y within
// bands of a few tiles, then along z, and the species groups of a tile are
// adjacent, so the blocks that read a plane, a row or a column as centre and
// as neighbour, and the blocks that share a tile's link data, are resident
// together. Waves without an interface node skip the sorption arithmetic.
// Variants 5 and 6 are the 8-wave blocks of variants 3 and 4 on lattices one
// tile wide (FR below).
constexpr int RX = TX + 2;                       // haloed row
// NH reduction tiles per block, stacked along y (ZX false: a TX x NH TY tile
// of one plane) or along z (ZX true: a TX x TY tile of NH consecutive planes).
// FR (full rows, lattices with nx = TX): the tile spans whole periodic rows,
// so the region has no x halo (x +- 1 wraps inside the row) and is copied in
// groups of 4 rows, one 16-byte copy per lane (lane i of a wave fills dwords
// 4i .. 4i+3 of the wave's destination).
template <int NH, bool ZX, bool FR = false>
struct DmaShape {
    static constexpr int DTY = ZX ? TY : NH * TY, DBLK = NH * BLK;  // block tile rows, threads
    static constexpr int NPL = ZX ? NH + 2 : 3;            // planes in the region
    static constexpr int RXS = FR ? TX : RX;              // region row length
    static constexpr int RROWS = NPL * (DTY + 2);         // region rows
    static constexpr int RREG = RROWS * RXS;              // planes z0-1 .. z0+NPL-2
    static constexpr int RLD = (RREG + DBLK - 1) / DBLK;  // 4-byte region loads per thread and field
    static constexpr int NW = DBLK / 64;                  // waves
    static constexpr int CPW = (RROWS + 4 * NW - 1) / (4 * NW);  // 16-byte row-group loads per wave and field
    static constexpr int NCP = FR ? CPW : RLD;            // region copies a wave issues per field
    // region dwords of a stage (FR: 4-row groups of every wave, the last ones
    // partly or wholly padding), then the adsorbed values of the tile
    static constexpr int REGION = FR ? NW * CPW * 4 * TX : RLD * DBLK;
    static constexpr int STAGE = REGION + DBLK;
    // Region layout: row-interleaved planes, element (hy, pz, hx) at
    // (NPL hy + pz) RXS + hx, so the 19 stencil values of a node lie within
    // (2 NPL + 2) RXS + 3 dwords of its (x-1, y-1, z-1) corner.
    __host__ __device__ static constexpr int at(int hy, int pz, int hx) { return (NPL * hy + pz) * RXS + hx; }
    // vector-memory operations a wave issues after a field's copy, up to the
    // wait for it: the copies of the next two fields and the stores of the
    // three before (with and without interface nodes in the wave; a field's
    // copy goes out right after the barrier three fields earlier, before that
    // field's update and store)
    static constexpr int WAIT_I = 2 * (NCP + 1) + 3 * 2, WAIT_N = 2 * NCP + 3;
    // waves without a node to update (lane compaction) copy and store nothing else
    static constexpr int WAIT_IDLE = 2 * NCP;
};
constexpr int DMA_GMAX = 64;                     // species per block
constexpr int NSUM = 5;                          // per-node block sums of a species

#define LBMP_LDS(p) ((__attribute__((address_space(3))) void*)(p))

// 16-byte LDS-DMA copy: lane i fills dwords 4i .. 4i+3 from dst. (Outside the
// kernel template: inside one, the host pass silently drops the launch stub.)
__device__ __forceinline__ void lds_copy16(__amdgpu_buffer_rsrc_t r, float* dst, int voff, int soff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, LBMP_LDS(dst), 16, voff, soff, 0, 0);
}
// s_waitcnt immediate: vmcnt(c), no expcnt wait, lgkmcnt(0)
#define LBMP_WAIT_VM_LGKM0(c) __builtin_amdgcn_s_waitcnt(((c) & 15) | ((((c) >> 4) & 3) << 14) | 0x0070)

// Block-wide barrier after this wave's LDS traffic has completed and at most
// n of its vector-memory operations (which complete in issue order) are
// outstanding. The empty asm statements keep the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void barrier_vm0() {
    asm volatile("" ::: "memory");
    LBMP_WAIT_VM_LGKM0(0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}
// The same with at most N outstanding; N a constant of the caller.
template <int N>
__device__ __forceinline__ void barrier_vm() {
    asm volatile("" ::: "memory");
    LBMP_WAIT_VM_LGKM0(N);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Lane permutation of an FP64 value (DPP on both halves); lanes without a
// source receive an unspecified value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Rotation of a wave by one lane: lane i receives lane i - 1 (ROR1) or i + 1
// (ROL1), mod 64.
constexpr int DPP_WAVE_ROL1 = 0x134, DPP_WAVE_ROR1 = 0x13C;
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
// The x-centred link of the row a link with an x component reads from (same
// y and z components), -1 for the node's own row.
__host__ __device__ constexpr int row_link(int k) {
    for (int j = 0; j < NL; ++j)
        if (lcx(j) == 0 && lcy(j) == lcy(k) && lcz(j) == lcz(k) && (lcy(k) != 0 || lcz(k) != 0)) return j;
    return -1;
}
static_assert(row_link(0) == -1 && row_link(6) == 2 && row_link(7) == 3 && row_link(12) == 5, "row links");

// Lane 15 of rows 0 and 2 broadcast to rows 1 and 3; rows 0 and 2 receive 0.
__device__ __forceinline__ double dpp_bcast15(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x142, 0xA, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x142, 0xA, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Four LDS stages as separate objects, so that the compiler's own tracking of
// LDS DMA can tell a stage being read from the stages still being filled.
struct Stages {
    float* p[4];
    template <int Q>
    __device__ __forceinline__ float* at() const { return p[Q]; }
};

// LC (lane compaction, haloed blocks only): the fluid nodes of the block are
// handed to its first threads in thread order, so that waves left without a
// node copy, synchronise and add block sums but skip the update arithmetic
// (porous media, where most lanes of a tile sit on solid nodes).
template <int NH, bool ZX, bool FR, bool LC = false>
__global__ void __launch_bounds__(NH * BLK) __attribute__((amdgpu_waves_per_eu(4))) k_mp_dma(const GeomDev<float>* __restrict__ geoms, int ngeom, int gsz,
                                               int64_t nblocks, const Ctl* __restrict__ ctl) {
    static_assert(!(LC && FR), "lane compaction needs the haloed region (a wave is not a row)");
    using SH = DmaShape<NH, ZX, FR>;
    constexpr int DTY = SH::DTY, DBLK = SH::DBLK, RREG = SH::RREG, RLD = SH::RLD, STAGE = SH::STAGE;
    constexpr int NCP = SH::NCP, REGION = SH::REGION;
    __shared__ __align__(16) float st0[STAGE];
    __shared__ __align__(16) float st1[STAGE];
    __shared__ __align__(16) float st2[STAGE];
    __shared__ __align__(16) float st3[STAGE];
    __shared__ __align__(16) double rl[NSUM * DBLK];  // per-node sums of a species
    __shared__ __align__(16) double l2[NH * NRED * 64]; // per half: partial sums of 4 nodes, by series slot
    float* const tag = nullptr;
    const int64_t lb = xcd_remap(blockIdx.x, nblocks);
    const int gi = find_geom(geoms, ngeom, lb);
    const GeomDev<float>& G = geoms[gi];
    const int64_t local = lb - G.blk0;
    const int grp = (int)(local % G.ngrp);
    const int64_t btile = local / G.ngrp;  // block tile; reduction tiles NH btile + half
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    // Block tiles in bands of YB tiles along y: band, then z, then y within
    // the band (the last band may be narrower), then x, so that the blocks
    // resident on one XCD at a time cover whole rows, a few tiles in y and
    // several in z, and share halo columns, rows and planes (and the cache
    // lines that a row's tiles split) in its L2.
    const int nzb = ZX ? (nz + NH - 1) / NH : nz;  // block positions along z
    const int nyt = (ny + DTY - 1) / DTY;           // block positions along y
    const int ntx = (nx + TX - 1) / TX;             // block positions along x
    constexpr int YB = 4;
    const int64_t per_band = (int64_t)YB * nzb * ntx;
    const int band = (int)(btile / per_band), bs = min(YB, nyt - band * YB);
    const int rr = (int)(btile - band * per_band);
    const int xt = rr % ntx, r2 = rr / ntx;
    const int z0 = (r2 / bs) * (ZX ? NH : 1);
    const int x0 = xt * TX, y0 = (band * YB + r2 % bs) * DTY;
    const int tid = threadIdx.x;
    // block position of thread t: x, row, plane
    auto pos_x = [](int t) { return t % TX; };
    auto pos_y = [](int t) { return ZX ? (t / TX) % TY : t / TX; };
    auto pos_z = [](int t) { return ZX ? t / BLK : 0; };
    const int wv = __builtin_amdgcn_readfirstlane(tid / 64);
    const int hf = wv >> 2, w4 = wv & 3;        // half of the block, wave within it
    const int64_t tile = NH * btile + hf;       // this wave's reduction tile
    const int N = (int)G.N, NI = (int)G.NI, plane = nx * ny, S = G.S;
    const int NC = (int)G.NC;  // nodes per stored field (fluid nodes when compact)
    const int32_t* const fidx = G.fidx;
    const int s0 = grp * gsz, s1 = min(S, s0 + gsz);
    const int64_t ntile = G.ntile;
    double* const part = G.part;
    // the thread's own node
    const int ox = x0 + pos_x(tid), oy = y0 + pos_y(tid), oz = z0 + pos_z(tid);
    const bool oin = ox < nx && oy < ny && oz < nz;
    const bool oact = oin && G.cls[oin ? oz * plane + oy * nx + ox : 0] != 0;
    if (!__syncthreads_or(oact)) {  // a tile without fluid: zero sums of every half
        for (int i = tid; i < NH * NRED * (s1 - s0); i += DBLK)
            part[((int64_t)(s0 + i / (NH * NRED)) * ntile + NH * btile + (i / NRED) % NH) * NRED + i % NRED] = 0.0;
        return;
    }
    // the node this thread updates: its own, or with LC the tid-th fluid node
    // of the block in thread order (none past the block's fluid count)
    __shared__ int lc_cnt[LC ? SH::NW : 1];
    __shared__ unsigned short lc_node[LC ? DBLK : 1];
    int at_t = tid;
    bool lc_has = true, idle = false;  // idle: wave-uniform, no node in the wave
    if constexpr (LC) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(oact);
        if ((tid & 63) == 0) lc_cnt[wv] = (int)__builtin_popcountll(m);
        __syncthreads();
        int base = 0, F = 0;
        for (int w = 0; w < SH::NW; ++w) {
            const int c = lc_cnt[w];
            base += w < wv ? c : 0;
            F += c;
        }
        const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (oact) lc_node[base + below] = (unsigned short)tid;
        __syncthreads();
        lc_has = tid < F;
        at_t = lc_has ? (int)lc_node[tid] : 0;
        idle = __builtin_amdgcn_readfirstlane(wv * 64 >= F ? 1 : 0) != 0;
    }
    const int lx = pos_x(at_t), ly = pos_y(at_t), zp = pos_z(at_t);  // updated node: x, row, plane in the block
    const int x = x0 + lx, y = y0 + ly, z = z0 + zp;
    const bool inplane = lc_has && x < nx && y < ny && z < nz;
    const int n = inplane ? z * plane + y * nx + x : 0;
    const bool act = inplane && G.cls[n] != 0;
    const int sl = act ? G.slot[n] : -1;
    const bool isI = sl >= 0;
    const bool anyI = __builtin_amdgcn_ballot_w64(isI) != 0;  // wave-uniform
    // fields and link data of node n at offn: its index among the fluid
    // nodes (compact storage) or n
    const int offa = isI ? sl * 4 : OOB;
    const int offn = act ? (fidx ? fidx[n] : n) * 4 : OOB;
    // this thread's share of the stencil region: element e = j * DBLK + tid,
    // or (FR) the 4 nodes from x = 4 (lane % 16) of row 4 g + lane / 16,
    // g = j NW + wave
    // (solid nodes hold zero fields and are never written: their elements are
    // masked like the padding, so the copy fetches fluid nodes only and the
    // out-of-range lanes write the same zeros; a 16-byte copy is masked when
    // its 4 nodes are solid)
    int voff[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) {
        if constexpr (FR) {
            const int r = 4 * (j * SH::NW + wv) + (tid & 63) / 16, hx = 4 * (tid & 15);
            const int hy = r / SH::NPL, pz = r % SH::NPL;
            const int m = r < SH::RROWS ? modp(z0 - 1 + pz, nz) * plane + modp(y0 - 1 + hy, ny) * nx + hx : 0;
            const bool any = r < SH::RROWS && (G.cls[m] | G.cls[m + 1] | G.cls[m + 2] | G.cls[m + 3]) != 0;
            voff[j] = any ? m * 4 : OOB;
        } else {
            const int e = j * DBLK + tid;
            const int hy = e / (SH::NPL * RX), pz = (e / RX) % SH::NPL, hx = e % RX;
            const int m = e < RREG ? modp(z0 - 1 + pz, nz) * plane + modp(y0 - 1 + hy, ny) * nx + modp(x0 - 1 + hx, nx) : 0;
            voff[j] = (e < RREG && G.cls[m] != 0) ? (fidx ? fidx[m] : m) * 4 : OOB;
        }
    }
    float pin[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) pin[k] = bload(tag, mkrsrc(G.pin + (int64_t)k * N, (int64_t)N * 4), offn);
    if constexpr (FR) {
        // full rows: a lane forms the arrivals over +x links for the lane at
        // x + 1 and over -x links for the lane at x - 1, so it holds their
        // probabilities of those links
#pragma unroll
        for (int k = 0; k < NL; ++k)
            if (lcx(k) > 0) pin[k] = dpp_f32<DPP_WAVE_ROL1>(pin[k]);
            else if (lcx(k) < 0) pin[k] = dpp_f32<DPP_WAVE_ROR1>(pin[k]);
    }
    const double sig = __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(mkrsrc(G.sig, (int64_t)N * 8), act ? offn * 2 : OOB, 0, 0));
    const double src = (double)bload(tag, mkrsrc(G.src, (int64_t)N * 4), offn);
    float av[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) av[g] = bload(tag, mkrsrc(G.a + (int64_t)g * N, (int64_t)N * 4), offn);
    // per-node VACF weights without a branch on the node's class
    const double actd = act ? 1.0 : 0.0;
    double avd[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) avd[g] = act ? (double)av[g] : 0.0;
    const int64_t t = ctl->t;
    const uint32_t rbase = hash32((uint32_t)n * 0x9e3779b9u ^ hash32((uint32_t)t ^ ((uint32_t)gi << 24)));
    const float* const Xin = (t & 1) ? G.X1 : G.X0;
    float* const Xout = (t & 1) ? G.X0 : G.X1;
    float* const Xa = G.Xa;
    // species constants in FP64, uniform: scalar loads into register pairs
    const __attribute__((address_space(4))) double* const kc =
        (const __attribute__((address_space(4))) double*)G.kc;
    const Stages stg{{st0, st1, st2, st3}};

    // Buffer resources span the 4 fields of one species; the field of quantity
    // q sits at soffset q * (bytes per field). The range check applies to
    // voffset + soffset + immediate: a masked offset (OOB) stays beyond the
    // range and OOB + 3 fields + 4 KB does not wrap (the host keeps 16 N + 4 KB
    // and 16 N_I + 4 KB below OOB for this kernel).
    const int NB = NC * 4, NIB = NI * 4;  // bytes per stored field
    const int64_t sN = 4 * (int64_t)NC, sNI = 4 * (int64_t)NI;
    // The immediate offset of an LDS-DMA load moves both the memory address and
    // the LDS destination, so copies whose destinations lie within 4 KB share
    // one LDS base (M0): copy j (and the adsorbed values, as copy RLD) goes to
    // base j / GJ at immediate (j % GJ) * DBLK * 4, taken back from its memory
    // offset; the resources start 4 KB below the species so that offset stays
    // non-negative.
    constexpr int GJ = FR ? 1 : 4096 / (DBLK * 4);  // copies per LDS base
    int vo[NCP];
#pragma unroll
    for (int j = 0; j < NCP; ++j) vo[j] = voff[j] == OOB ? OOB : voff[j] + 4096 - (FR ? 0 : (j % GJ) * DBLK * 4);
    const int voa = offa == OOB ? OOB : offa + 4096 - (FR ? 0 : (RLD % GJ) * DBLK * 4);
    static_assert(NCP <= 5, "copies are unrolled for at most 5 region loads");
    auto issue = [&](auto qpc, auto anyc, const float* ib, const float* iab) {
        constexpr int qp = decltype(qpc)::value;  // quantity (and stage) of the copied field
        const auto rin = mkrsrc(reinterpret_cast<const char*>(ib) - 4096, 4 * (int64_t)NB + 4096);
        float* dst = stg.at<qp>() + wv * 64;
        auto copy = [&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (FR && j < NCP)  // row group j NW + wv, 256 dwords
                lds_copy16(rin, stg.at<qp>() + (j * SH::NW + wv) * 4 * TX, vo[j], qp * NB);
            else if constexpr (!FR && j < NCP)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, LBMP_LDS(dst + (j / GJ) * GJ * DBLK), 4, vo[j],
                                                         qp * NB, (j % GJ) * DBLK * 4, 0);
        };
        copy(std::integral_constant<int, 0>());
        copy(std::integral_constant<int, 1>());
        copy(std::integral_constant<int, 2>());
        copy(std::integral_constant<int, 3>());
        copy(std::integral_constant<int, 4>());
        if constexpr (decltype(anyc)::value) {
            const auto rina = mkrsrc(reinterpret_cast<const char*>(iab) - 4096, 4 * (int64_t)NIB + 4096);
            if constexpr (FR)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rina, LBMP_LDS(stg.at<qp>() + REGION + wv * 64), 4, voa,
                                                         qp * NIB, 0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rina, LBMP_LDS(dst + (RLD / GJ) * GJ * DBLK), 4, voa,
                                                         qp * NIB, (RLD % GJ) * DBLK * 4, 0);
        }
    };
    // Block sums of a species in a fixed order, one step per field barrier.
    // Per node: the drift-corrected VACF terms X_g (a_g - V_g) - V_g X_ads,g
    // (g = x, y, z; their sum is sum X_g a_g - V_g E_g(t), E_g the stored
    // total of the first moment), and the mobile and adsorbed density. They
    // enter rl at the species' end; at q = 1 of the next species wave w folds
    // sum w, and a quarter of sum 4, into partials of 4 nodes (l2); at q = 0
    // of the species after that, wave w adds up slots 2w and 2w+1 (2
    // partials per lane, then over 32 lanes) and stores them: VACF terms in
    // slots 0-2, mobile density in 3, zeros in 4-6 (the drift term is
    // already in 0-2), adsorbed density in 7. None of this branches, and the
    // steps sit where the compiler keeps track of which LDS DMA is in flight
    // (after a branch, or before the first stage read of a species, it
    // otherwise waits for all of it). With nothing pending nothing is
    // stored.
    const int ln = tid & 63;
    auto fold = [&]() {
        // pair (partial of sum w over nodes 4 ln..4 ln+3, partial of sum 4 over
        // nodes 64 w + 4 (ln % 16) ..+3), one store: a second LDS store in a
        // row makes the compiler wait for all DMA in flight
        const double* p = rl + w4 * DBLK + hf * BLK + ln * 4;
        const double* p4 = rl + 4 * DBLK + wv * 64 + (ln & 15) * 4;  // wv * 64 = hf * BLK + w4 * 64
        using d2 = double __attribute__((ext_vector_type(2)));
        d2 v;
        v.x = ((p[0] + p[1]) + p[2]) + p[3];
        v.y = ((p4[0] + p4[1]) + p4[2]) + p4[3];
        *reinterpret_cast<d2*>(l2 + hf * (NRED * 64) + 2 * (w4 * 64 + ln)) = v;
    };
    auto finish = [&](int s) {
        const int k = 2 * w4 + (ln >> 5), j = ln & 31;
        // slots 0-3: partials 2j, 2j+1 of sum k; slot 7: partials 2j, 2j+1
        // of sum 4 (partial i from wave i / 16, lane i % 16)
        const int i0 = k < 4 ? 2 * (k * 64 + 2 * j) : 2 * ((j >> 3) * 64 + ((2 * j) & 15)) + 1;
        const double* l2h = l2 + hf * (NRED * 64);
        double v = l2h[i0] + l2h[i0 + 2];
        v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
        v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
        v += dpp_f64<0x124>(v);   // row_ror:4
        v += dpp_f64<0x128>(v);   // row_ror:8: every lane holds its row's sum
        v += dpp_bcast15(v);      // rows 1 and 3 add the sum of rows 0 and 2
        if (k >= 4 && k < 7) v = 0.0;
        // a buffer store: a flat store would also count as LDS traffic and
        // make the next LDS read wait for every DMA in flight
        bstore(v, mkrsrc(part + (int64_t)max(s, 0) * ntile * NRED, ntile * NRED * 8),
               (j == 31 && s >= 0) ? (int)(tile * NRED + k) * 8 : OOB);
    };

    // region index of (x-1, y-1, z-1); FR: of (x, y-1, z-1)
    const int cb = SH::at(ly, zp, lx);
    int pend = -1, pend2 = -1;  // species with per-node sums in rl, with partials in l2
    using T_ = std::true_type;
    using F_ = std::false_type;
    // anyc: the wave has interface nodes (wave-uniform; both paths pass the
    // same barriers). firstc / lastc: the block's first / last species, whose
    // first / last two fields wait for every copy in flight (fewer operations
    // follow their copies than the steady-state wait counts assume).
    auto run = [&](auto anyc, auto idlec) {
        constexpr bool ANYI = decltype(anyc)::value;
        constexpr bool IDLE = decltype(idlec)::value;  // no node in the wave: no update, no stores
        static_assert(!(IDLE && ANYI), "an idle wave has no interface node");
        const float* in_s = Xin + (int64_t)s0 * sN;  // species s of the input fields
        const float* ina_s = Xa + (int64_t)s0 * sNI;
        float* out_s = Xout + (int64_t)s0 * sN;
        float* outa_s = Xa + (int64_t)s0 * sNI;
        issue(std::integral_constant<int, 0>(), anyc, in_s, ina_s);
        issue(std::integral_constant<int, 1>(), anyc, in_s, ina_s);
        issue(std::integral_constant<int, 2>(), anyc, in_s, ina_s);
        auto species = [&](int s, auto firstc, auto lastc) {
            constexpr bool FIRST = decltype(firstc)::value, LAST = decltype(lastc)::value;
            const float* const in_n = in_s + sN;  // species s + 1
            const float* const ina_n = ina_s + sNI;
            const auto rout = mkrsrc(out_s, 4 * (int64_t)NB);
            const auto rads = mkrsrc(outa_s, 4 * (int64_t)NIB);
            const double pa = kc[KC * s], pd = kc[KC * s + 1];
            double cq[4], w[3], nv[3];
#pragma unroll
            for (int q = 0; q < 4; ++q) cq[q] = kc[KC * s + 2 + q];
#pragma unroll
            for (int g = 0; g < 3; ++g) {
                nv[g] = kc[KC * s + 6 + g];
                w[g] = __builtin_fma(actd, nv[g], avd[g]);  // av + nv, 0 off the fluid
            }
            double red[NSUM];
#pragma unroll
            for (int k = 0; k < NSUM; ++k) red[k] = 0.0;
            auto field = [&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const int f = 4 * s + q;
                // field f has landed for the whole block once this wave has at
                // most the operations issued after it outstanding: the loads of
                // f+1, f+2 and the stores of f-3, f-2, f-1 (2 (NCP + 1) + 3 * 2
                // with interface nodes in the wave, 2 NCP + 3 without); the
                // block's first three and last two fields have fewer behind them
                if constexpr ((FIRST && q < 3) || (LAST && q >= 2)) barrier_vm0();
                else if constexpr (IDLE) barrier_vm<SH::WAIT_IDLE>();
                else if constexpr (ANYI) barrier_vm<SH::WAIT_I>();
                else barrier_vm<SH::WAIT_N>();
                if constexpr (q == 0) {
                    finish(pend2);
                    pend2 = -1;
                }
                if constexpr (q == 1) {
                    fold();
                    pend2 = pend;
                    pend = -1;
                }
                // field f + 3 (quantity 3 of this species, or quantity q - 1 of the
                // next) into the stage of field f - 1, which every wave has read
                // before this barrier
                if constexpr (q == 0) issue(std::integral_constant<int, 3>(), anyc, in_s, ina_s);
                else if constexpr (!LAST) issue(std::integral_constant<int, q - 1>(), anyc, in_n, ina_n);
                if constexpr (!IDLE) {  // an idle wave updates no node
                    // one live base offset: addresses derived from it are not
                    // hoisted out of the loop (each would hold a register for the
                    // whole loop)
                    int cbb = 4 * cb;
                    asm volatile("" : "+v"(cbb));
                    // volatile: one ds_read_b32 per value, its stencil offset in the
                    // instruction's immediate (merged pairs need a base register each)
                    using lvf = const volatile __attribute__((address_space(3))) float;
                    lvf* const sb = (lvf*)((const __attribute__((address_space(3))) char*)stg.at<q>() + cbb);
                    // all values first, then the arithmetic; v[k] is the value at
                    // r - c_k (FR: for a link with an x component, the value at
                    // r - c_k + x-hat * c_kx, the lane's own column of that row)
                    float v[NL], c0;
                    if constexpr (FR) {
                        c0 = sb[SH::at(1, 1, 0)];
    #pragma unroll
                        for (int k = 0; k < NL; ++k)
                            if (lcx(k) == 0) v[k] = sb[SH::at(1 - lcy(k), 1 - lcz(k), 0)];
    #pragma unroll
                        for (int k = 0; k < NL; ++k)
                            if (lcx(k) != 0) v[k] = row_link(k) < 0 ? c0 : v[row_link(k)];
                    } else {
                        c0 = sb[SH::at(1, 1, 1)];
    #pragma unroll
                        for (int k = 0; k < NL; ++k) v[k] = sb[SH::at(1 - lcy(k), 1 - lcz(k), 1 - lcx(k))];
                    }
                    const double xc = (double)c0;
                    double stay = __builtin_fma(-xc, sig, xc);  // the part that stays (Eq. 7)
                    stay = __builtin_fma(cq[q], src, stay);
                    // arrivals from r - c_k (Eq. 7): three FP32 chains in link order,
                    // over the links with c_kx = 0, +1 and -1
                    float a0 = 0.0f, ap = 0.0f, am = 0.0f;
    #pragma unroll
                    for (int k = 0; k < NL; ++k) {
                        if (lcx(k) == 0) a0 = __builtin_fmaf(v[k], pin[k], a0);
                        else if (lcx(k) > 0) ap = __builtin_fmaf(v[k], pin[k], ap);
                        else am = __builtin_fmaf(v[k], pin[k], am);
                    }
                    if constexpr (FR) {
                        // a wave is one periodic row (lane = x): the lane formed the
                        // +x and -x chains of the lanes beside it (pin holds their
                        // probabilities there), and a rotation of the wave by one
                        // lane hands each its sum
                        ap = dpp_f32<DPP_WAVE_ROR1>(ap);
                        am = dpp_f32<DPP_WAVE_ROL1>(am);
                    }
                    double nvx = ((stay + (double)a0) + (double)ap) + (double)am;
                    const uint32_t r = rbase + (uint32_t)f * 0x9e3779b9u;
                    if constexpr (q == 0) red[3] += act ? xc : 0.0;
                    else red[q - 1] = __builtin_fma(xc, w[q - 1], red[q - 1]);
                    if constexpr (ANYI) {  // sorption (Eqs. 9, 10) where the wave has interface nodes
                        const double xa = (double)stg.at<q>()[REGION + tid];
                        const double fa = isI ? pa * xc : 0.0, fd = pd * xa;
                        nvx = (nvx - fa) + fd;
                        bstore_nt(sround((xa + fa) - fd, (r >> 3) | (r << 29)), rads, offa, q * NIB);
                        if constexpr (q == 0) red[4] += xa;
                        else red[q - 1] = __builtin_fma(nv[q - 1], xa, red[q - 1]);
                    }
                    bstore_nt(sround(nvx, r), rout, offn, q * NB);
                }
            };
            field(std::integral_constant<int, 0>());
            field(std::integral_constant<int, 1>());
            field(std::integral_constant<int, 2>());
            field(std::integral_constant<int, 3>());
#pragma unroll
            for (int k = 0; k < NSUM; ++k) rl[k * DBLK + tid] = red[k];
            pend = s;
            in_s = in_n;
            ina_s = ina_n;
            out_s += sN;
            outa_s += sNI;
        };
        if (s1 - s0 == 1) {
            species(s0, T_(), T_());
        } else {
            species(s0, T_(), F_());
            for (int s = s0 + 1; s < s1 - 1; ++s) species(s, F_(), F_());
            species(s1 - 1, F_(), T_());
        }
    };
    if (idle) run(F_(), T_());
    else if (anyI) run(T_(), F_());
    else run(F_(), F_());
    barrier_vm0();
    finish(pend2);
    barrier_vm0();
    fold();
    barrier_vm0();
    finish(pend);
}


// ------------------------------------------------------------------ gathered chunks
// Variant 8: a block updates one chunk of up to GCH fluid nodes that are
// consecutive in the compact storage, whose order (tiles of 32 x 4 x 4 lattice
// nodes, fluid nodes in lattice order within a tile) keeps a chunk spatially
// compact. Per field the buffer unit copies, in 16-byte quads (4 consecutive
// compact values, one quad per thread), the chunk's own values (one
// contiguous range) and those of its halo (the fluid nodes outside the chunk
// that its nodes pull from, covered by a precomputed list of quad starts)
// into an LDS region; each thread then reads its 18 arrivals at precomputed
// region slots (links from solid nodes read a slot the copy leaves at zero).
// Every thread has a fluid node, whatever the porosity, and only runs of
// fluid values are copied. The arithmetic, its order and the rounding bits
// are those of the LDS-DMA blocks, so the stored fields are bitwise the same.
// NH = 1 or 2: blocks of 256 or 512 threads (nodes per chunk, region quads)
template <int NH>
struct GatherShape {
    static constexpr int DBLK = NH * BLK;                 // nodes per chunk, threads per block
    static constexpr int NQ = DBLK;                       // region quads: one copy per thread and field
    static constexpr int REG = 4 * NQ;                    // region slots: chunk, halo quads, zeros
    static constexpr int ZSLOT = REG - 1;                 // in the last quad, never copied: reads 0
};
constexpr int GCH = 2 * BLK;                     // the largest chunk
constexpr int GTX = 32, GTY = 4, GTZ = 4;        // ordering tiles (compact storage)

template <int NH>
__global__ void __launch_bounds__(NH * BLK) __attribute__((amdgpu_waves_per_eu(4))) k_mp_gather(
    const GeomDev<float>* __restrict__ geoms, int ngeom, int gsz, int64_t nblocks, const Ctl* __restrict__ ctl) {
    using GS = GatherShape<NH>;
    constexpr int DBLK = GS::DBLK, NCP = 1, REGION = GS::REG, STAGE = GS::REG + DBLK;
    constexpr int GZSLOT = GS::ZSLOT;
    constexpr int NW = DBLK / 64;
    constexpr int WAIT_I = 2 * (NCP + 1) + 3 * 2, WAIT_N = 2 * NCP + 3, WAIT_IDLE = 2 * NCP;
    __shared__ __align__(16) float st0[STAGE];
    __shared__ __align__(16) float st1[STAGE];
    __shared__ __align__(16) float st2[STAGE];
    __shared__ __align__(16) float st3[STAGE];
    __shared__ __align__(16) double rl[NSUM * DBLK];
    __shared__ __align__(16) double l2[NH * NRED * 64];
    float* const tag = nullptr;
    const int64_t lb = xcd_remap(blockIdx.x, nblocks);
    const int gi = find_geom(geoms, ngeom, lb);
    const GeomDev<float>& G = geoms[gi];
    const int64_t local = lb - G.blk0;
    const int grp = (int)(local % G.ngrp);
    const int64_t chunk = local / G.ngrp;
    const int4 ch = G.gch[chunk];
    const int cbase = ch.x, C = ch.y, hoff = ch.z, H = ch.w;
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid / 64);
    const int hf = wv >> 2, w4 = wv & 3;
    const int64_t tile = NH * chunk + hf;         // reduction tiles: the halves (NH = 2) of the chunk
    const int NI = (int)G.NI, S = G.S;
    const int NC = (int)G.NC;
    const int s0 = grp * gsz, s1 = min(S, s0 + gsz);
    const int64_t ntile = G.ntile;
    double* const part = G.part;
    const bool act = tid < C;
    const bool idle = __builtin_amdgcn_readfirstlane(wv * 64 >= C ? 1 : 0) != 0;
    const int i = cbase + (act ? tid : 0);        // compact index of the node
    const int n = act ? G.gnode[i] : 0;           // its lattice index
    const int sl = act ? G.gaslot[i] : -1;
    const bool isI = sl >= 0;
    const bool anyI = __builtin_amdgcn_ballot_w64(isI) != 0;
    const int offa = isI ? sl * 4 : OOB;
    const int offn = act ? i * 4 : OOB;
    // region quad tid (slots 4 tid .. 4 tid + 3): chunk nodes 4 tid .. 4 tid + 3,
    // halo quad tid - Cq, or nothing (H counts the halo quads)
    const int Cq = (C + 3) >> 2;
    const int voff = tid < Cq ? (cbase + 4 * tid) * 4 : (tid < Cq + H ? G.ghsrc[hoff + tid - Cq] * 4 : OOB);
    // byte offsets of the 18 arrivals in the region
    int nba[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) nba[k] = act ? 4 * (int)G.gnbr[(int64_t)k * NC + i] : 4 * GZSLOT;
    float pin[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) pin[k] = bload(tag, mkrsrc(G.pin + (int64_t)k * G.N, (int64_t)G.N * 4), offn);
    const double sig = __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(mkrsrc(G.sig, G.N * 8), act ? offn * 2 : OOB, 0, 0));
    const double src = (double)bload(tag, mkrsrc(G.src, G.N * 4), offn);
    float av[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) av[g] = bload(tag, mkrsrc(G.a + (int64_t)g * G.N, G.N * 4), offn);
    const double actd = act ? 1.0 : 0.0;
    double avd[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) avd[g] = act ? (double)av[g] : 0.0;
    const int64_t t = ctl->t;
    const uint32_t rbase = hash32((uint32_t)n * 0x9e3779b9u ^ hash32((uint32_t)t ^ ((uint32_t)gi << 24)));
    const float* const Xin = (t & 1) ? G.X1 : G.X0;
    float* const Xout = (t & 1) ? G.X0 : G.X1;
    float* const Xa = G.Xa;
    const __attribute__((address_space(4))) double* const kc =
        (const __attribute__((address_space(4))) double*)G.kc;
    const Stages stg{{st0, st1, st2, st3}};
    const int NB = NC * 4, NIB = NI * 4;
    const int64_t sN = 4 * (int64_t)NC, sNI = 4 * (int64_t)NI;
    const int vo = voff == OOB ? OOB : voff + 4096;
    const int voa = offa == OOB ? OOB : offa + 4096;
    auto issue = [&](auto qpc, auto anyc, const float* ib, const float* iab) {
        constexpr int qp = decltype(qpc)::value;
        // 16 bytes beyond the species' 4 fields: a quad that starts at one of
        // the last 3 compact nodes reaches past its field (values no slot uses;
        // the storage continues beyond the last species)
        const auto rin = mkrsrc(reinterpret_cast<const char*>(ib) - 4096, 4 * (int64_t)NB + 4096 + 16);
        lds_copy16(rin, stg.at<qp>() + wv * 256, vo, qp * NB);  // wave wv: quads 64 wv .. 64 wv + 63
        if constexpr (decltype(anyc)::value) {
            const auto rina = mkrsrc(reinterpret_cast<const char*>(iab) - 4096, 4 * (int64_t)NIB + 4096);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rina, LBMP_LDS(stg.at<qp>() + REGION + wv * 64), 4, voa,
                                                     qp * NIB, 0, 0);
        }
    };
    const int ln = tid & 63;
    auto fold = [&]() {
        const double* p = rl + w4 * DBLK + hf * BLK + ln * 4;
        const double* p4 = rl + 4 * DBLK + wv * 64 + (ln & 15) * 4;
        using d2 = double __attribute__((ext_vector_type(2)));
        d2 v;
        v.x = ((p[0] + p[1]) + p[2]) + p[3];
        v.y = ((p4[0] + p4[1]) + p4[2]) + p4[3];
        *reinterpret_cast<d2*>(l2 + hf * (NRED * 64) + 2 * (w4 * 64 + ln)) = v;
    };
    auto finish = [&](int s) {
        const int k = 2 * w4 + (ln >> 5), j = ln & 31;
        const int i0 = k < 4 ? 2 * (k * 64 + 2 * j) : 2 * ((j >> 3) * 64 + ((2 * j) & 15)) + 1;
        const double* l2h = l2 + hf * (NRED * 64);
        double v = l2h[i0] + l2h[i0 + 2];
        v += dpp_f64<0xB1>(v);
        v += dpp_f64<0x4E>(v);
        v += dpp_f64<0x124>(v);
        v += dpp_f64<0x128>(v);
        v += dpp_bcast15(v);
        if (k >= 4 && k < 7) v = 0.0;
        bstore(v, mkrsrc(part + (int64_t)max(s, 0) * ntile * NRED, ntile * NRED * 8),
               (j == 31 && s >= 0) ? (int)(tile * NRED + k) * 8 : OOB);
    };
    int pend = -1, pend2 = -1;
    using T_ = std::true_type;
    using F_ = std::false_type;
    auto run = [&](auto anyc, auto idlec) {
        constexpr bool ANYI = decltype(anyc)::value;
        constexpr bool IDLE = decltype(idlec)::value;
        static_assert(!(IDLE && ANYI), "an idle wave has no interface node");
        const float* in_s = Xin + (int64_t)s0 * sN;
        const float* ina_s = Xa + (int64_t)s0 * sNI;
        float* out_s = Xout + (int64_t)s0 * sN;
        float* outa_s = Xa + (int64_t)s0 * sNI;
        issue(std::integral_constant<int, 0>(), anyc, in_s, ina_s);
        issue(std::integral_constant<int, 1>(), anyc, in_s, ina_s);
        issue(std::integral_constant<int, 2>(), anyc, in_s, ina_s);
        auto species = [&](int s, auto firstc, auto lastc) {
            constexpr bool FIRST = decltype(firstc)::value, LAST = decltype(lastc)::value;
            const float* const in_n = in_s + sN;
            const float* const ina_n = ina_s + sNI;
            const auto rout = mkrsrc(out_s, 4 * (int64_t)NB);
            const auto rads = mkrsrc(outa_s, 4 * (int64_t)NIB);
            const double pa = kc[KC * s], pd = kc[KC * s + 1];
            double cq[4], w[3], nv[3];
#pragma unroll
            for (int q = 0; q < 4; ++q) cq[q] = kc[KC * s + 2 + q];
#pragma unroll
            for (int g = 0; g < 3; ++g) {
                nv[g] = kc[KC * s + 6 + g];
                w[g] = __builtin_fma(actd, nv[g], avd[g]);
            }
            double red[NSUM];
#pragma unroll
            for (int k = 0; k < NSUM; ++k) red[k] = 0.0;
            auto field = [&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const int f = 4 * s + q;
                if constexpr ((FIRST && q < 3) || (LAST && q >= 2)) barrier_vm0();
                else if constexpr (IDLE) barrier_vm<WAIT_IDLE>();
                else if constexpr (ANYI) barrier_vm<WAIT_I>();
                else barrier_vm<WAIT_N>();
                if constexpr (q == 0) {
                    finish(pend2);
                    pend2 = -1;
                }
                if constexpr (q == 1) {
                    fold();
                    pend2 = pend;
                    pend = -1;
                }
                // field f + 3 (quantity 3 of this species, or quantity q - 1 of the
                // next) into the stage of field f - 1, which every wave has read
                // before this barrier
                if constexpr (q == 0) issue(std::integral_constant<int, 3>(), anyc, in_s, ina_s);
                else if constexpr (!LAST) issue(std::integral_constant<int, q - 1>(), anyc, in_n, ina_n);
                if constexpr (!IDLE) {
                    using lvc = const volatile __attribute__((address_space(3))) char;
                    lvc* const sb = (lvc*)stg.at<q>();
                    float v[NL];
                    const float c0 = *(const volatile __attribute__((address_space(3))) float*)(sb + 4 * tid);
#pragma unroll
                    for (int k = 0; k < NL; ++k)
                        v[k] = *(const volatile __attribute__((address_space(3))) float*)(sb + nba[k]);
                    const double xc = (double)c0;
                    double stay = __builtin_fma(-xc, sig, xc);  // the part that stays (Eq. 7)
                    stay = __builtin_fma(cq[q], src, stay);
                    // arrivals from r - c_k (Eq. 7): the LDS-DMA blocks' three FP32
                    // chains, over the links with c_kx = 0, +1 and -1
                    float a0 = 0.0f, ap = 0.0f, am = 0.0f;
#pragma unroll
                    for (int k = 0; k < NL; ++k) {
                        if (lcx(k) == 0) a0 = __builtin_fmaf(v[k], pin[k], a0);
                        else if (lcx(k) > 0) ap = __builtin_fmaf(v[k], pin[k], ap);
                        else am = __builtin_fmaf(v[k], pin[k], am);
                    }
                    double nvx = ((stay + (double)a0) + (double)ap) + (double)am;
                    const uint32_t r = rbase + (uint32_t)f * 0x9e3779b9u;
                    if constexpr (q == 0) red[3] += act ? xc : 0.0;
                    else red[q - 1] = __builtin_fma(xc, w[q - 1], red[q - 1]);
                    if constexpr (ANYI) {  // sorption (Eqs. 9, 10)
                        const double xa = (double)stg.at<q>()[REGION + tid];
                        const double fa = isI ? pa * xc : 0.0, fd = pd * xa;
                        nvx = (nvx - fa) + fd;
                        bstore(sround((xa + fa) - fd, (r >> 3) | (r << 29)), rads, offa, q * NIB);
                        if constexpr (q == 0) red[4] += xa;
                        else red[q - 1] = __builtin_fma(nv[q - 1], xa, red[q - 1]);
                    }
                    bstore(sround(nvx, r), rout, offn, q * NB);
                }
            };
            field(std::integral_constant<int, 0>());
            field(std::integral_constant<int, 1>());
            field(std::integral_constant<int, 2>());
            field(std::integral_constant<int, 3>());
#pragma unroll
            for (int k = 0; k < NSUM; ++k) rl[k * DBLK + tid] = red[k];
            pend = s;
            in_s = in_n;
            ina_s = ina_n;
            out_s += sN;
            outa_s += sNI;
        };
        if (s1 - s0 == 1) {
            species(s0, T_(), T_());
        } else {
            species(s0, T_(), F_());
            for (int s = s0 + 1; s < s1 - 1; ++s) species(s, F_(), F_());
            species(s1 - 1, F_(), T_());
        }
    };
    if (idle) run(F_(), T_());
    else if (anyI) run(T_(), F_());
    else run(F_(), F_());
    barrier_vm0();
    finish(pend2);
    barrier_vm0();
    fold();
    barrier_vm0();
    finish(pend);
}

// Lattices with many tiles: chunks of RCH tile partials of every
// (geometry, species) summed by one block each, in a fixed order, into
// chunk[work][chunk][NRED]; k_mp_reduce then adds the chunks.
constexpr int RCH = 2048;

template <typename T>
__global__ void __launch_bounds__(BLK) k_mp_reduce_chunks(const GeomDev<T>* __restrict__ geoms,
                                                          const int32_t* __restrict__ work, int nch,
                                                          double* __restrict__ chunk) {
    __shared__ double lds[NRED * BLK];
    const int w = blockIdx.x / nch, c = blockIdx.x % nch;
    const int gi = work[2 * w], s = work[2 * w + 1];
    const GeomDev<T>& G = geoms[gi];
    const int64_t ntile = G.ntile;
    using gdp = const __attribute__((address_space(1))) double*;  // global loads, not flat
    const gdp P = (gdp)(G.part + (int64_t)s * ntile * NRED);
    const int64_t i0 = (int64_t)c * RCH, i1 = min(ntile, i0 + RCH);
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; ++k) acc[k] = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BLK)
#pragma unroll
        for (int k = 0; k < NRED; ++k) acc[k] += P[i * NRED + k];
    double r;
    block_sum8(acc, lds, r);
    if (threadIdx.x < NRED) chunk[((int64_t)w * nch + c) * NRED + threadIdx.x] = r;
}

// Sum the block partials (or, with nch > 0, the chunk sums) of every
// (geometry, species) into the series at the current time, in a fixed order,
// one block of RED_T threads per pair, then advance the time: the partials of
// a pair are read as one flat array (thread i adds entries i, i + RED_T, ...,
// all of sum i % NRED, in turn into eight accumulators), the 32 threads of
// each sum are added by a fixed tree, and the last block to finish moves the
// state time on (every block has read it by then).
constexpr int RED_T = 256;

template <typename T>
__global__ void __launch_bounds__(RED_T) k_mp_reduce(const GeomDev<T>* __restrict__ geoms, int ngeom,
                                                     const int32_t* __restrict__ work, int nwork, int nch,
                                                     const double* __restrict__ chunk, Ctl* __restrict__ ctl) {
    static_assert(RED_T % (64 * 1) == 0 && 64 % NRED == 0, "a thread's entries belong to one sum");
    __shared__ double wsum[RED_T / 64][NRED];
    __shared__ bool last;
    const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t t = ctl->t;
    const int gi = work[2 * w], s = work[2 * w + 1];
    const GeomDev<T>& G = geoms[gi];
    const int64_t ntile = nch > 0 ? nch : G.ntile;
    // global address space: flat loads would also count as LDS traffic and
    // serialise the loads below
    using gdp = const __attribute__((address_space(1))) double*;
    const gdp P = (gdp)(nch > 0 ? chunk + (int64_t)w * nch * NRED : G.part + (int64_t)s * G.ntile * NRED);
    const int64_t len = ntile * NRED;
    // eight loads in flight per thread, then their sums (eight accumulators)
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    int64_t i = tid;
    for (; i + 7 * RED_T < len; i += 8 * RED_T) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = P[i + u * RED_T];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += x[u];
    }
#pragma unroll
    for (int u = 0; u < 7; ++u)
        if (i + u * RED_T < len) acc[u] += P[i + u * RED_T];
    double v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    // lanes l, l ^ 8, l ^ 16, ... hold the same sum (l % 8)
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < NRED) wsum[wv][lane] = v;
    __syncthreads();
    if (tid < NRED && t <= ctl->tmax) {
        double r = wsum[0][tid];
#pragma unroll
        for (int k = 1; k < RED_T / 64; ++k) r += wsum[k][tid];
        G.series[((t - 1) * G.S + s) * NRED + tid] = r;
    }
    if (tid == 0 && t <= ctl->tmax) {
        // total probability of the species (slots 3 and 7, summed as above)
        double m = wsum[0][3], a = wsum[0][7];
#pragma unroll
        for (int k = 1; k < RED_T / 64; ++k) {
            m += wsum[k][3];
            a += wsum[k][7];
        }
        if (!(fabs(m + a - ctl->mass_ref) <= ctl->drift_max))
            atomicMin(reinterpret_cast<unsigned long long*>(&ctl->bad_t), (unsigned long long)t);
    }
    // time advance by the last block
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        last = atomicAdd(&ctl->done, 1u) == (unsigned)(gridDim.x - 1);
    }
    __syncthreads();
    if (last && tid == 0) {
        ctl->done = 0;
        ctl->t = t + 1;
    }
}


// ------------------------------------------------------------------ set-up
// Link probabilities of Eq. 8 (local equilibrium), FP64, per node and link;
// zero on solid nodes and for links into solid nodes. bmu (nullable): the
// tracer's excess chemical potential beta mu^ex per node; the diffusive term
// then carries Q = exp(-(bmu(r + c_i) - bmu(r)) / 2) (Q = 1 without it).
__global__ void k_pout(const int8_t* __restrict__ cls, const double* __restrict__ u, int nx, int ny,
                       int nz, double lam, const double* __restrict__ bmu, double* __restrict__ pout) {
    const int64_t N = (int64_t)nx * ny * nz;
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
    const double ux = u[n], uy = u[N + n], uz = u[2 * N + n];
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int k = 0; k < NL; ++k) {
        double p = 0.0;
        if (cls[n] != 0) {
            int64_t m = modp(x + lcx(k), nx) + (int64_t)nx * (modp(y + lcy(k), ny) + (int64_t)ny * modp(z + lcz(k), nz));
            if (cls[m] != 0) {
                double cu = lcx(k) * ux + lcy(k) * uy + lcz(k) * uz;
                const double Q = bmu ? exp(-0.5 * (bmu[m] - bmu[n])) : 1.0;
                p = lw(k) * (0.5 * lam * Q + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            }
        }
        pout[(int64_t)k * N + n] = p;
    }
}

// Stored tables and per-node set-up values. Sums of stored (rounded) link
// probabilities are formed in FP64, so sigma and src describe exactly the
// chain the stored table propagates.
// w (nullable): relative Eq. 11 weight exp(-beta mu^ex) of every node (1
// without an excess chemical potential); sums over r below are weighted by it.
// setup partials per block: [0..2] sum_r w a_g, [3..5] sum_r w sum_i p_i c_ig^2,
// [6] min p_i, [7] max |u|, [8] min stay (bulk), [9] min stay (interface),
// [10] sum of w over fluid nodes, [11] sum of w over interfacial nodes.
template <typename T>
__global__ void k_links(const int8_t* __restrict__ cls, const double* __restrict__ pout,
                        const double* __restrict__ u, int nx, int ny, int nz, const double* __restrict__ w,
                        T* __restrict__ pin, double* __restrict__ sig, T* __restrict__ src, T* __restrict__ a,
                        double* __restrict__ b64, double* __restrict__ src64,
                        double* __restrict__ part) {
    __shared__ double lds[SETUP_RED * BLK];
    const int64_t N = (int64_t)nx * ny * nz;
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[SETUP_RED] = {0, 0, 0, 0, 0, 0, INFINITY, 0.0, INFINITY, INFINITY, 0, 0};
    if (n < N) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        const bool fl = cls[n] != 0;
        double sout = 0.0, sin = 0.0, ag[3] = {0, 0, 0}, bg[3] = {0, 0, 0}, c2[3] = {0, 0, 0};
        for (int k = 0; k < NL; ++k) {
            const double po = (double)(T)pout[(int64_t)k * N + n];
            sout += po;
            ag[0] += po * lcx(k);
            ag[1] += po * lcy(k);
            ag[2] += po * lcz(k);
            c2[0] += po * lcx(k) * lcx(k);
            c2[1] += po * lcy(k) * lcy(k);
            c2[2] += po * lcz(k) * lcz(k);
            int64_t m = modp(x - lcx(k), nx) + (int64_t)nx * (modp(y - lcy(k), ny) + (int64_t)ny * modp(z - lcz(k), nz));
            const T pt = fl ? (T)pout[(int64_t)k * N + m] : T(0);
            pin[(int64_t)k * N + n] = pt;
            const double wpt = (w ? w[m] : 1.0) * (double)pt;  // weighted arrival from r - c_k
            sin += wpt;
            bg[0] += wpt * lcx(k);
            bg[1] += wpt * lcy(k);
            bg[2] += wpt * lcz(k);
            if (fl && cls[m] != 0) v[6] = fmin(v[6], pout[(int64_t)k * N + n]);
        }
        sig[n] = fl ? sout : 0.0;
        // weighted arrivals minus departures of the stored table, both summed
        // exactly: zero wherever the Eq. 11 weights are stationary for that table
        const double wn = w ? w[n] : 1.0;
        const double s64 = fl ? sin - wn * sout : 0.0;
        src[n] = (T)s64;
        src64[n] = s64;
        for (int g = 0; g < 3; ++g) {
            a[(int64_t)g * N + n] = fl ? (T)ag[g] : T(0);
            b64[(int64_t)g * N + n] = fl ? bg[g] : 0.0;
        }
        if (fl) {
            for (int g = 0; g < 3; ++g) {
                v[g] = wn * ag[g];
                v[3 + g] = wn * c2[g];
            }
            const double uu = sqrt(u[n] * u[n] + u[N + n] * u[N + n] + u[2 * N + n] * u[2 * N + n]);
            v[7] = uu;
            if (cls[n] == 2) v[9] = 1.0 - sout; else v[8] = 1.0 - sout;
            v[10] = wn;
            v[11] = cls[n] == 2 ? wn : 0.0;
        }
    }
    const int tid = threadIdx.x;
    for (int k = 0; k < SETUP_RED; ++k) lds[k * BLK + tid] = v[k];
    __syncthreads();
    if (tid < SETUP_RED) {
        double r = lds[tid * BLK];
        for (int j = 1; j < BLK; ++j) {
            double w = lds[tid * BLK + j];
            if (tid == 6 || tid == 8 || tid == 9) r = fmin(r, w);
            else if (tid == 7) r = fmax(r, w);
            else r += w;
        }
        part[(int64_t)blockIdx.x * SETUP_RED + tid] = r;
    }
}

__global__ void k_setup_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    const int k = threadIdx.x;
    if (k >= SETUP_RED || blockIdx.x != 0) return;
    double r = part[k];
    for (int b = 1; b < nb; ++b) {
        double w = part[(int64_t)b * SETUP_RED + k];
        if (k == 6 || k == 8 || k == 9) r = fmin(r, w);
        else if (k == 7) r = fmax(r, w);
        else r += w;
    }
    out[k] = r;
}

// State at t = 1 (deviations): density rho_ref*src; first moments
// rho_ref*(b_q - V_q w); adsorbed density 0; adsorbed first moments
// -V_q Gamma_ref w (w the relative Eq. 11 weight of the node, 1 when null).
template <typename T>
__global__ void k_init_state(const int8_t* __restrict__ cls, const int32_t* __restrict__ ilist,
                             int64_t N, int64_t NI, int S, const double* __restrict__ spc,
                             const double* __restrict__ b64, const double* __restrict__ src64,
                             const double* __restrict__ w, const int32_t* __restrict__ fidx, int64_t NC,
                             const int32_t* __restrict__ aperm, T* __restrict__ X, T* __restrict__ Xa) {
    // spc per species: rho_ref, Gamma_ref, V0, V1, V2; fields dense (fidx
    // null, NC = N) or compact (node n at fidx[n], solid nodes not stored)
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    const double rr = spc[5 * s], gr = spc[5 * s + 1];
    if (n < N && (!fidx || fidx[n] >= 0)) {
        const bool fl = cls[n] != 0;
        const int64_t i = fidx ? fidx[n] : n;
        const double wn = w ? w[n] : 1.0;
        X[(int64_t)(4 * s) * NC + i] = fl ? (T)(rr * src64[n]) : T(0);
        for (int q = 1; q < 4; ++q)
            X[(int64_t)(4 * s + q) * NC + i] =
                fl ? (T)(rr * b64[(int64_t)(q - 1) * N + n] - rr * spc[5 * s + 1 + q] * wn) : T(0);
    }
    if (n < NI) {
        // interface slot n; its adsorbed fields at aperm[n] (variant 8) or n
        const double wn = w ? w[ilist[n]] : 1.0;
        const int64_t ia = aperm ? aperm[n] : n;
        Xa[(int64_t)(4 * s) * NI + ia] = T(0);
        for (int q = 1; q < 4; ++q) Xa[(int64_t)(4 * s + q) * NI + ia] = (T)(-spc[5 * s + 1 + q] * gr * wn);
    }
}

// Uptake start: density 1/N_F on every fluid node (the first-moment fields of
// each species stay zero).
template <typename T>
__global__ void k_init_uptake(const int8_t* __restrict__ cls, int64_t N, double rho0,
                              const int32_t* __restrict__ fidx, int64_t NC, T* __restrict__ X) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (n < N && (!fidx || fidx[n] >= 0))
        X[(int64_t)(4 * s) * NC + (fidx ? fidx[n] : n)] = cls[n] != 0 ? (T)rho0 : T(0);
}

// Time series of Z_g and D_g (discrete Eq. 3 about the mean drift) for one
// geometry, one thread per (species, direction), compensated summation.
// Z(t) = V^2 + sum_r dP a - E(t) V, where E(t) = sum dP + sum dP_ads is the
// total of the first-moment deviations (zero in exact arithmetic; the term
// removes the rounding drift of the stored total from the VACF).
__global__ void k_vacf_series(const double* __restrict__ series, int S, int64_t T, int64_t stride,
                              const double* __restrict__ spc0, double* __restrict__ Zo,
                              double* __restrict__ Do) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * S) return;
    const int s = i / 3, g = i % 3;
    const double V = spc0[4 * s + g];
    const double z0 = spc0[(int64_t)S * 4 + 3 * s + g];
    double* Z = Zo + (int64_t)i * stride;
    double* D = Do + (int64_t)i * stride;
    Z[0] = z0;
    double sum = 0.5 * (z0 - V * V), comp = 0.0;
    D[0] = sum;
    for (int64_t t = 1; t <= T; ++t) {
        const double* e = series + ((t - 1) * S + s) * NRED;
        const double c = e[g] - e[4 + g] * V;
        Z[t] = V * V + c;
        const double tt = sum + c;
        comp += fabs(sum) >= fabs(c) ? (sum - tt) + c : (c - tt) + sum;
        sum = tt;
        D[t] = sum + comp;
    }
}

// ------------------------------------------------------------------ host side
struct TuneKey {
    int prec;
    std::vector<int64_t> shape;
    bool operator<(const TuneKey& o) const { return std::tie(prec, shape) < std::tie(o.prec, o.shape); }
};
struct TuneVal {
    int K, gsz, variant;
};
static std::map<TuneKey, TuneVal> g_tune_cache;

struct GeomHost {
    const lbmp_flow* flow;
    int S;
    int64_t N, NI, nf;
    double lam;
    std::vector<double> pa, pd, rho_ref, gam_ref;
    double A[3], B[3];
    double min_p, max_u, min_stay_bulk, min_stay_iface, pa_max;
    std::vector<double> V, Z0;  // [S][3]
    // charged tracers: beta mu^ex per node (empty: neutral) and the relative
    // Eq. 11 weights exp(-(beta mu^ex - its minimum over fluid nodes)); the
    // weighted fluid and interfacial totals (N_F and N_I when neutral)
    std::vector<double> bmu, w;
    double sumw_f = 0.0, sumw_i = 0.0;
    int64_t ntile_max;
    // device buffers
    void *pin, *sig, *src, *a, *X0, *X1, *Xa, *coef, *prob;
    double *part, *series, *spc, *spc0, *kc, *zout, *dout;
    int32_t* fidx;  // [N] index of a fluid node among the fluid nodes in lattice order, -1 on solid
    std::vector<int32_t> fidx_h;  // host copy
    // gathered chunks (variant 8): the compact order of their fields (gidx,
    // tiles of 32 x 4 x 4 nodes), chunk table, halo quads, neighbour slots, lattice
    // index and adsorbed-field index per compact node, adsorbed-field index
    // per interface slot (aperm); host copies of gidx and aperm
    int32_t *gidx, *gnode, *gaslot, *ghsrc, *aperm;
    int4* gch;
    uint16_t* gnbr;
    int64_t nch = 0;
    int gnh = 2;  // threads per block / 256 of the chunk tables (LBMP_GATHER_NH, default 2)
    bool gather_ok = false;
    std::vector<int32_t> gidx_h, aperm_h;
};

}  // namespace lbmp

struct lbmp_mp {
    uint32_t magic;
    int prec, ngeom;
    int64_t tmax, steps;
    hipStream_t stream;
    std::vector<lbmp::GeomHost> g;
    void* geoms_dev;
    lbmp::Ctl* ctl;
    int32_t* work;
    int nwork;
    double* chunk;   // [nwork][nch_max][NRED] chunk sums of the series reduction
    int nch_max, nch;
    double* setup_tmp;
    int K, gsz, variant;  // variant 0: direct loads, 1: LDS-staged box, 2: z-march, 3-7: LDS DMA, 8: gathered chunks (FP32)
    int uptake;           // out-of-equilibrium density propagation (no VACF)
    int64_t nblocks;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace lbmp {
namespace {

constexpr int GRAPH_CHUNK = 64;

// chunks reserved per geometry: twice the count of full chunks of the
// smaller block (256 nodes)
int64_t gather_chunk_cap(int64_t nf) { return 2 * ((std::max<int64_t>(nf, 1) + BLK - 1) / BLK); }

int64_t ntile_for(const lbmp_flow* f, int K, int variant) {
    const int64_t zb = (f->nz + K - 1) / K;  // K = z-planes per tile (z-segment for variant 2)
    // variant 8: up to two reduction tiles (halves) per chunk; chunks are cut
    // shorter where their halo would not fit, up to the capacity reserved
    if (variant == 8) return 2 * gather_chunk_cap(f->nf);
    // variant 3: K reduction tiles (TX x TY) per block of TX x (K TY), one z-plane
    // (variant 5: the same with full rows)
    if (variant == 3 || variant == 5)
        return K * (int64_t)((f->nx + TX - 1) / TX) * ((f->ny + K * TY - 1) / (K * TY)) * f->nz;
    // variant 4 (6: full rows, 7: lane compaction): K reduction tiles (TX x TY) per block of K planes
    if (variant == 4 || variant == 6 || variant == 7) return K * (int64_t)((f->nx + TX - 1) / TX) * ((f->ny + TY - 1) / TY) * ((f->nz + K - 1) / K);
    if (variant >= 1) return (int64_t)((f->nx + TX - 1) / TX) * ((f->ny + TY - 1) / TY) * zb;
    return (((int64_t)f->nx * f->ny + BLK - 1) / BLK) * zb;
}

// set-up scratch: pout 18 N | b64 3 N | src64 N | block partials | final sums |
// bmu N | w N (the last two survive the compaction of the link tables, which
// reuses the head of the region)
int64_t setup_doubles(int64_t N) { return 24 * N + ((N + BLK - 1) / BLK) * SETUP_RED + SETUP_RED; }
double* setup_bmu(double* base, int64_t N) { return base + 22 * N + ((N + BLK - 1) / BLK) * SETUP_RED + SETUP_RED; }

template <typename T>
void carve_geom(GeomHost& g, Carver& c, int64_t tmax) {
    const int64_t N = g.N, NIa = std::max<int64_t>(g.NI, 1);
    const size_t S = (size_t)g.S;
    g.pin = c.take<T>(18 * N);
    g.sig = c.take<double>(N);
    g.src = c.take<T>(N);
    g.a = c.take<T>(3 * N);
    g.X0 = c.take<T>(S * 4 * N);
    g.X1 = c.take<T>(S * 4 * N);
    g.Xa = c.take<T>(S * 4 * NIa);
    g.fidx = c.take<int32_t>(N);
    {
        const int64_t NF = std::max<int64_t>(g.nf, 1), nch = gather_chunk_cap(NF);
        g.gidx = c.take<int32_t>(N);
        g.gnode = c.take<int32_t>(NF);
        g.gaslot = c.take<int32_t>(NF);
        g.gch = c.take<int4>(nch);
        g.ghsrc = c.take<int32_t>(nch * GatherShape<1>::REG);
        g.gnbr = c.take<uint16_t>(NL * NF);
        g.aperm = c.take<int32_t>(NIa);
    }
    g.coef = c.take<T>(S * 4);
    g.prob = c.take<T>(S * 2);
    g.part = c.take<double>(S * g.ntile_max * NRED);
    g.series = c.take<double>((size_t)std::max<int64_t>(tmax, 1) * S * NRED);
    g.spc = c.take<double>(S * 5);
    g.spc0 = c.take<double>(S * 7);
    g.kc = c.take<double>(S * KC);
    g.zout = c.take<double>(S * 3 * (tmax + 1));
    g.dout = c.take<double>(S * 3 * (tmax + 1));
}

// Carves the whole workspace; with a null base it only measures.
lbmp_status carve_all(lbmp_mp* h, Carver& c) {
    h->geoms_dev = c.take<char>(sizeof(GeomDev<double>) * h->ngeom);
    h->ctl = c.take<Ctl>(1);
    int64_t setup = 0;
    int nw = 0;
    for (auto& g : h->g) {
        if (h->prec == LBMP_FP32) carve_geom<float>(g, c, h->tmax); else carve_geom<double>(g, c, h->tmax);
        setup = std::max(setup, setup_doubles(g.N));
        nw += g.S;
    }
    h->setup_tmp = c.take<double>(setup);
    h->work = c.take<int32_t>(2 * (size_t)nw);
    h->nwork = nw;
    int64_t tmx = 1;
    for (auto& g : h->g) tmx = std::max(tmx, g.ntile_max);
    h->nch_max = (int)((tmx + RCH - 1) / RCH);
    h->chunk = c.take<double>((size_t)nw * h->nch_max * NRED);
    return LBMP_OK;
}

lbmp_status resolve_lambda(const lbmp_species& sp, double* lam) {
    bool has_db = std::isfinite(sp.D_b), has_dl = std::isfinite(sp.Delta);
    if (has_db == has_dl) return fail(LBMP_EINVAL, "give exactly one of D_b and Delta (the other NaN)");
    if (has_db) {
        if (!(sp.D_b > 0)) return fail(LBMP_EINVAL, "D_b must be positive");
        *lam = 12.0 * sp.D_b;
    } else {
        if (!(sp.Delta >= 0.0 && sp.Delta < 1.0)) return fail(LBMP_EINVAL, "Delta must be in [0, 1)");
        *lam = 3.0 * (1.0 - sp.Delta);
    }
    return LBMP_OK;
}

lbmp_status validate_species(const lbmp_species& sp, int gi, bool uptake) {
    if (sp.n_species < 1) return fail(LBMP_EINVAL, "geometry %d: n_species must be >= 1", gi);
    if (!sp.k_a || !sp.k_d) return fail(LBMP_EINVAL, "geometry %d: rate arrays are NULL", gi);
    for (int s = 0; s < sp.n_species; ++s) {
        if (!(sp.k_a[s] >= 0.0) || !std::isfinite(sp.k_a[s]))
            return fail(LBMP_EINVAL, "geometry %d: k_a[%d] must be finite and >= 0", gi, s);
        if (uptake ? !(sp.k_d[s] >= 0.0 && sp.k_d[s] <= 1.0) : !(sp.k_d[s] > 0.0 && sp.k_d[s] <= 1.0))
            return fail(LBMP_EINVAL,
                        uptake ? "geometry %d: k_d[%d] must be in [0, 1]"
                               : "geometry %d: k_d[%d] must be in (0, 1] (irreversible sorption has no "
                                 "equilibrium VACF; use the uptake calls)",
                        gi, s);
    }
    double lam;
    return resolve_lambda(sp, &lam);
}

lbmp_mp* make_handle(const lbmp_flow* const* flows, const lbmp_species* species, int n_geom, int precision,
                     int64_t tmax) {
    auto* h = new lbmp_mp();
    h->magic = MP_MAGIC;
    h->prec = precision;
    h->ngeom = n_geom;
    h->tmax = tmax;
    h->steps = 0;
    h->g.resize(n_geom);
    for (int gi = 0; gi < n_geom; ++gi) {
        GeomHost& g = h->g[gi];
        g.flow = flows[gi];
        g.S = species[gi].n_species;
        g.N = g.flow->N;
        g.NI = g.flow->ni;
        g.nf = g.flow->nf;
        g.ntile_max = std::max({ntile_for(g.flow, 1, 0), ntile_for(g.flow, 1, 1), ntile_for(g.flow, 1, 3),
                                ntile_for(g.flow, 2, 3), ntile_for(g.flow, 2, 4), ntile_for(g.flow, 4, 6),
                                ntile_for(g.flow, 2, 8)});
    }
    return h;
}

template <typename T>
void launch_step_kernel(lbmp_mp* h, hipStream_t s) {
    auto* G = static_cast<const GeomDev<T>*>(h->geoms_dev);
    dim3 grid((unsigned)h->nblocks);
    if (h->variant >= 3) {
        if constexpr (std::is_same<T, float>::value) {
            if (h->variant == 4) k_mp_dma<2, true, false><<<grid, 2 * BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else if (h->variant == 5) k_mp_dma<2, false, true><<<grid, 2 * BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else if (h->variant == 6 && h->K == 4) k_mp_dma<4, true, true><<<grid, 4 * BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else if (h->variant == 6) k_mp_dma<2, true, true><<<grid, 2 * BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else if (h->variant == 7) k_mp_dma<2, true, false, true><<<grid, 2 * BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else if (h->variant == 8 && h->g[0].gnh == 1) k_mp_gather<1><<<grid, BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else if (h->variant == 8) k_mp_gather<2><<<grid, 2 * BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else if (h->K == 2) k_mp_dma<2, false, false><<<grid, 2 * BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
            else k_mp_dma<1, false, false><<<grid, BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
        }
        return;
    }
    if (h->variant == 2) {
        switch (h->gsz) {
            case 1: k_mp_march<T, 1><<<grid, BLK, 0, s>>>(G, h->ngeom, h->nblocks, h->K, h->ctl); break;
            case 2: k_mp_march<T, 2><<<grid, BLK, 0, s>>>(G, h->ngeom, h->nblocks, h->K, h->ctl); break;
            default: k_mp_march<T, 4><<<grid, BLK, 0, s>>>(G, h->ngeom, h->nblocks, h->K, h->ctl); break;
        }
        return;
    }
    if (h->variant == 1) {
        if (h->K == 1) k_mp_step_box<T, 1><<<grid, BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
        else k_mp_step_box<T, 2><<<grid, BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl);
        return;
    }
    switch (h->K) {
        case 1: k_mp_step<T, 1><<<grid, BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl); break;
        default: k_mp_step<T, 2><<<grid, BLK, 0, s>>>(G, h->ngeom, h->gsz, h->nblocks, h->ctl); break;
    }
}

template <typename T>
void launch_step_tail(lbmp_mp* h, hipStream_t s) {
    auto* G = static_cast<const GeomDev<T>*>(h->geoms_dev);
    if (h->nch > 1)
        k_mp_reduce_chunks<T><<<(unsigned)(h->nwork * h->nch), BLK, 0, s>>>(G, h->work, h->nch, h->chunk);
    k_mp_reduce<T><<<(unsigned)h->nwork, RED_T, 0, s>>>(G, h->ngeom, h->work, h->nwork, h->nch > 1 ? h->nch : 0,
                                                         h->chunk, h->ctl);
}

template <typename T>
void launch_step(lbmp_mp* h, hipStream_t s) {
    launch_step_kernel<T>(h, s);
    launch_step_tail<T>(h, s);
}

void do_steps(lbmp_mp* h, int64_t n, hipStream_t s) {
    for (int64_t i = 0; i < n; ++i) {
        if (h->prec == LBMP_FP32) launch_step<float>(h, s); else launch_step<double>(h, s);
    }
}

// The haloed LDS-DMA blocks store the fields of fluid nodes only (a porous
// medium's solid nodes would otherwise share cache lines with its fluid ones
// and be fetched and written back with them); the other variants, and the
// full-row blocks, whose 16-byte copies take 4 consecutive nodes, keep the
// dense layout.
bool compact_fields(const lbmp_mp* h) {
    return h->variant == 3 || h->variant == 4 || h->variant == 7 || h->variant == 8;
}
// node -> compact index map of the chosen variant (null: dense fields)
const int32_t* cidx(const lbmp_mp* h, const GeomHost& g) {
    return !compact_fields(h) ? nullptr : (h->variant == 8 ? g.gidx : g.fidx);
}

// Fill the device geometry table for the current (K, gsz).
template <typename T>
lbmp_status upload_geoms(lbmp_mp* h) {
    std::vector<GeomDev<T>> v(h->ngeom);
    int64_t blk = 0;
    for (int gi = 0; gi < h->ngeom; ++gi) {
        GeomHost& g = h->g[gi];
        const lbmp_flow* f = g.flow;
        GeomDev<T>& d = v[gi];
        d.nx = f->nx; d.ny = f->ny; d.nz = f->nz; d.S = g.S;
        d.N = g.N; d.NI = std::max<int64_t>(g.NI, 1);
        d.pb = (int)(((int64_t)f->nx * f->ny + BLK - 1) / BLK);
        d.zb = (f->nz + h->K - 1) / h->K;
        d.ngrp = (g.S + h->gsz - 1) / h->gsz;
        d.ntile = h->variant == 8 ? g.gnh * g.nch : ntile_for(f, h->K, h->variant);
        d.blk0 = blk;
        // variants 3-7: one block per K tiles; variant 8: one per chunk
        blk += (h->variant == 8 ? g.nch : (h->variant >= 3 ? d.ntile / h->K : d.ntile)) * d.ngrp;
        d.cls = f->d.cls; d.slot = f->d.slot;
        d.pin = (const T*)g.pin; d.sig = (const double*)g.sig; d.src = (const T*)g.src; d.a = (const T*)g.a;
        d.X0 = (T*)g.X0; d.X1 = (T*)g.X1; d.Xa = (T*)g.Xa;
        d.fidx = cidx(h, g);
        d.gch = g.gch; d.ghsrc = g.ghsrc; d.gnode = g.gnode; d.gaslot = g.gaslot; d.gnbr = g.gnbr;
        d.NC = compact_fields(h) ? g.nf : g.N;
        d.coef = (const T*)g.coef; d.prob = (const T*)g.prob;
        d.kc = g.kc;
        d.part = g.part; d.series = g.series;
    }
    h->nblocks = blk;
    int64_t tmx = 1;
    for (const auto& d : v) tmx = std::max(tmx, d.ntile);
    h->nch = (int)((tmx + RCH - 1) / RCH);  // chunked series reduction when > 1
    LBMP_HIP(hipMemcpyAsync(h->geoms_dev, v.data(), sizeof(GeomDev<T>) * v.size(), hipMemcpyHostToDevice, h->stream));
    LBMP_HIP(hipStreamSynchronize(h->stream));
    return LBMP_OK;
}

lbmp_status upload(lbmp_mp* h) { return h->prec == LBMP_FP32 ? upload_geoms<float>(h) : upload_geoms<double>(h); }

// The z-march kernel addresses a group's fields and the link table through
// one 32-bit buffer range each.
// The LDS-DMA kernel addresses the 4 fields of a species (and 4 KB below them)
// through one buffer resource: 16 bytes a node (interface node) plus 4 KB must
// stay below the masking offset.
bool dma_fits(const lbmp_mp* h) {
    for (const auto& g : h->g)
        if ((int64_t)16 * g.N + 4096 >= (int64_t)OOB || (int64_t)16 * g.NI + 4096 >= (int64_t)OOB) return false;
    return true;
}

// Full-row LDS-DMA blocks (variants 5, 6) need every geometry one tile wide.
bool full_rows(const lbmp_mp* h) {
    for (const auto& g : h->g)
        if (g.flow->nx != TX) return false;
    return true;
}

bool march_fits(const lbmp_mp* h, int G) {
    const int64_t es = h->prec == LBMP_FP32 ? 4 : 8;
    for (const auto& g : h->g) {
        const int64_t big = std::max<int64_t>((int64_t)4 * std::min(G, g.S) * g.N, (int64_t)NL * g.N) * es;
        if (big >= (int64_t)INT32_MAX - 64) return false;
    }
    return true;
}

// ---- on-disk tuning cache: one JSON object per line,
// {"key": "...", "variant": v, "K": k, "species_per_block": g, "ms": t}; the
// key names the build, the precision and every geometry's shape, fluid and
// interfacial node counts and species count; the last line with a key wins.
// File: $LBMP_TUNE_CACHE, else $HOME/.cache/lbmp/tune.jsonl; LBMP_TUNE_CACHE
// set to an empty string turns it off. Unreadable or unwritable files are
// ignored (the tuner then times the candidates).
std::string tune_cache_path() {
    if (const char* p = getenv("LBMP_TUNE_CACHE")) return p;
    if (const char* home = getenv("HOME")) return std::string(home) + "/.cache/lbmp/tune.jsonl";
    return "";
}

std::string tune_key_string(const lbmp_mp* h) {
    std::string k = "build " __DATE__ " " __TIME__ "; fp" + std::to_string(h->prec);
    for (const auto& g : h->g)
        k += "; " + std::to_string(g.flow->nx) + "x" + std::to_string(g.flow->ny) + "x" + std::to_string(g.flow->nz) +
             " nf " + std::to_string(g.nf) + " ni " + std::to_string(g.NI) + " S " + std::to_string(g.S);
    return k;
}

bool tune_cache_read(const std::string& key, TuneVal* out) {
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return false;
    const std::string needle = "{\"key\": \"" + key + "\", ";
    char line[4096];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        if (strncmp(line, needle.c_str(), needle.size()) != 0) continue;
        TuneVal v;
        double ms = 0.0;
        if (sscanf(line + needle.size(), "\"variant\": %d, \"K\": %d, \"species_per_block\": %d, \"ms\": %lf",
                   &v.variant, &v.K, &v.gsz, &ms) == 4) {
            *out = v;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void tune_cache_write(const std::string& key, const TuneVal& v, double ms) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        // create the directory chain (best effort)
        for (size_t i = 1; i <= slash; ++i)
            if (path[i] == '/' || i == slash) mkdir(path.substr(0, i == slash ? slash : i).c_str(), 0755);
    }
    FILE* f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"variant\": %d, \"K\": %d, \"species_per_block\": %d, \"ms\": %.6f}\n",
            key.c_str(), v.variant, v.K, v.gsz, ms);
    fclose(f);
}

// Whether a (variant, K, species per block) choice is allowed for the handle.
bool tile_allowed(const lbmp_mp* h, int v, int K, int gs) {
    const bool ok01 = (v == 0 || v == 1) && (K == 1 || K == 2) && gs >= 1;
    const bool ok2 = v == 2 && K >= 1 && (gs == 1 || gs == 2 || gs == 4) && march_fits(h, gs);
    bool gather = true;
    for (const auto& g : h->g) gather = gather && g.gather_ok;
    const bool ok3 = ((v == 3 && (K == 1 || K == 2)) || ((v == 4 || v == 7) && K == 2) ||
                      ((v == 5 || v == 6) && K == 2 && full_rows(h)) || (v == 6 && K == 4 && full_rows(h)) ||
                      (v == 8 && K == 2 && gather)) &&
                     gs >= 1 && gs <= DMA_GMAX && h->prec == LBMP_FP32 && dma_fits(h);
    return ok01 || ok2 || ok3;
}

// Pick (K, species per block) by timing steps of each candidate on the
// set-up tables before the state exists: a short screening run of every
// candidate, then a longer steady-state run (warm caches and clocks) of the
// fastest few. Results are cached per (precision, shapes) for the life of the
// process and on disk (see tune_cache_path).
lbmp_status autotune(lbmp_mp* h) {
    TuneKey key{h->prec, {}};
    int64_t work = 0;
    int maxS = 0;
    for (auto& g : h->g) {
        key.shape.insert(key.shape.end(), {g.flow->nx, g.flow->ny, g.flow->nz, g.S, g.nf, g.NI});
        work += g.nf * g.S;
        maxS = std::max(maxS, g.S);
    }
    // LBMP_TILE="variant,K,species_per_block" pins the choice (tests, experiments)
    if (const char* env = getenv("LBMP_TILE")) {
        int v = 0, K = 1, gs = 1;
        const int nread = sscanf(env, "%d,%d,%d", &v, &K, &gs);
        if (nread == 3 && tile_allowed(h, v, K, gs)) {
            h->variant = v;
            h->K = K;
            h->gsz = v == 2 ? gs : std::min(gs, std::max(1, maxS));
            return upload(h);
        }
        return fail(LBMP_EINVAL, "LBMP_TILE must be 'variant,K,species_per_block': variant 0|1 with K 1|2, "
                                 "variant 2 with K = z-segment and 1|2|4 species per block, or variant 3 "
                                 "(FP32 only) with K = 1 or 2 (block height in 64 x 4 tiles), or variant 4 (FP32 only) with K = 2 "
                                 "(z-planes per block), or variants 5, 6 (variants 3, 4 with full rows: FP32, nx = 64 in every "
                                 "geometry) with K = 2, or variant 7 (variant 4 with lane compaction, FP32) with K = 2, "
                                 "or variant 8 (gathered chunks, FP32) with K = 2; at most 64 species per block for 3-8");
    }
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
        h->K = it->second.K;
        h->gsz = it->second.gsz;
        h->variant = it->second.variant;
        return upload(h);
    }
    const std::string skey = tune_key_string(h);
    {
        TuneVal dv;
        if (tune_cache_read(skey, &dv) && tile_allowed(h, dv.variant, dv.K, dv.gsz)) {
            h->K = dv.K;
            h->gsz = dv.variant == 2 ? dv.gsz : std::min(dv.gsz, std::max(1, maxS));
            h->variant = dv.variant;
            g_tune_cache[key] = {h->K, h->gsz, h->variant};
            return upload(h);
        }
    }
    if (work < (1 << 16)) {  // launch-bound sizes: one block per tile, all species
        h->K = 1;
        h->gsz = maxS;
        h->variant = 0;
        g_tune_cache[key] = {h->K, h->gsz, h->variant};
        return upload(h);
    }
    std::vector<TuneVal> cand;
    for (int v : {0, 1})
        for (int K : {1, 2})
            for (int gs : {1, 2, 4, 8, 16, 32, 64})
                if (gs <= maxS || gs == 1) cand.push_back({K, gs, v});
    int maxz = 0;
    for (auto& g : h->g) maxz = std::max(maxz, g.flow->nz);
    for (int zs : {8, 16, 32, 64})
        for (int gs : {1, 2, 4})
            if ((gs <= maxS || gs == 1) && zs <= std::max(8, maxz) && march_fits(h, gs))
                cand.push_back({zs, gs, 2});
    if (h->prec == LBMP_FP32 && dma_fits(h))
        for (int gs : {2, 4, 8, 16, 32, 64})
            for (int K : {1, 2}) {
                if (gs <= maxS || gs == 2) cand.push_back({K, gs, 3});
                if (K == 2 && (gs <= maxS || gs == 2)) {
                    cand.push_back({K, gs, 4});
                    cand.push_back({K, gs, 7});
                }
                if (K == 2 && (gs <= maxS || gs == 2) && full_rows(h)) {
                    cand.push_back({K, gs, 5});
                    cand.push_back({K, gs, 6});
                }
                if (K == 2 && (gs <= maxS || gs == 2) && tile_allowed(h, 8, 2, gs)) cand.push_back({K, gs, 8});
            }
    hipEvent_t e0, e1;
    LBMP_HIP(hipEventCreate(&e0));
    LBMP_HIP(hipEventCreate(&e1));
    // time `reps` steps of candidate c after `warm` untimed ones (ms per step)
    auto time_cand = [&](const TuneVal& c, int warm, int reps, float* ms) -> lbmp_status {
        h->K = c.K;
        h->gsz = c.gsz;
        h->variant = c.variant;
        lbmp_status st = upload(h);
        if (st != LBMP_OK) return st;
        do_steps(h, warm, h->stream);
        LBMP_HIP(hipEventRecord(e0, h->stream));
        do_steps(h, reps, h->stream);
        LBMP_HIP(hipEventRecord(e1, h->stream));
        LBMP_HIP(hipEventSynchronize(e1));
        LBMP_HIP(hipEventElapsedTime(ms, e0, e1));
        *ms /= (float)reps;
        return LBMP_OK;
    };
    // screening: one untimed and three timed steps per candidate
    std::vector<std::pair<float, TuneVal>> scored;
    for (auto c : cand) {
        float ms = 0;
        lbmp_status st = time_cand(c, 1, 3, &ms);
        if (st != LBMP_OK) return st;
        scored.push_back({ms, c});
    }
    std::stable_sort(scored.begin(), scored.end(),
                     [](const std::pair<float, TuneVal>& a, const std::pair<float, TuneVal>& b) { return a.first < b.first; });
    // steady state: the fastest four again, each after about 50 ms of untimed
    // steps (clocks and caches settle), over about 20 ms of timed steps
    float best = INFINITY;
    TuneVal bv = scored.front().second;
    const size_t nfin = std::min<size_t>(4, scored.size());
    for (size_t i = 0; i < nfin; ++i) {
        const float per = std::max(scored[i].first, 1e-3f);
        const int warm = std::max(5, std::min(400, (int)(50.0f / per)));
        const int reps = std::max(5, std::min(200, (int)(20.0f / per)));
        float ms = 0;
        lbmp_status st = time_cand(scored[i].second, warm, reps, &ms);
        if (st != LBMP_OK) return st;
        if (ms < best) {
            best = ms;
            bv = scored[i].second;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->K = bv.K;
    h->gsz = bv.gsz;
    h->variant = bv.variant;
    g_tune_cache[key] = bv;
    tune_cache_write(skey, bv, best);
    return upload(h);
}

// Link tables for one geometry (and the FP64 per-node values of the initial
// state in setup_tmp).
template <typename T>
lbmp_status build_links(lbmp_mp* h, GeomHost& g, hipStream_t s, double* fin_host) {
    const lbmp_flow* f = g.flow;
    const int64_t N = f->N;
    double* pout = h->setup_tmp;
    double* b64 = pout + 18 * N;
    double* src64 = b64 + 3 * N;
    double* part = src64 + N;
    const unsigned nb = (unsigned)((N + BLK - 1) / BLK);
    double* fin = part + (size_t)nb * SETUP_RED;
    double* bmu = nullptr;
    double* w = nullptr;
    if (!g.bmu.empty()) {
        bmu = setup_bmu(h->setup_tmp, N);
        w = bmu + N;
        LBMP_HIP(hipMemcpyAsync(bmu, g.bmu.data(), N * 8, hipMemcpyHostToDevice, s));
        LBMP_HIP(hipMemcpyAsync(w, g.w.data(), N * 8, hipMemcpyHostToDevice, s));
    }
    k_pout<<<nb, BLK, 0, s>>>(f->d.cls, f->d.u, f->nx, f->ny, f->nz, g.lam, bmu, pout);
    k_links<T><<<nb, BLK, 0, s>>>(f->d.cls, pout, f->d.u, f->nx, f->ny, f->nz, w, (T*)g.pin, (double*)g.sig,
                                  (T*)g.src, (T*)g.a, b64, src64, part);
    k_setup_final<<<1, 64, 0, s>>>(part, nb, fin);
    LBMP_HIP(hipGetLastError());
    if (fin_host) {
        LBMP_HIP(hipMemcpyAsync(fin_host, fin, SETUP_RED * 8, hipMemcpyDeviceToHost, s));
        LBMP_HIP(hipStreamSynchronize(s));
    }
    return LBMP_OK;
}

// Species constants: Eq. 11 weights, mean velocity, Z(0), probabilities.
template <typename T>
lbmp_status species_constants(lbmp_mp* h, GeomHost& g, const double* r, hipStream_t s) {
    const int S = g.S;
    for (int k = 0; k < 3; ++k) {
        g.A[k] = r[k];
        g.B[k] = r[3 + k];
    }
    g.min_p = r[6];
    g.max_u = r[7];
    g.min_stay_bulk = r[8];
    g.min_stay_iface = r[9];
    g.sumw_f = r[10];  // sums of 1 over the fluid and interfacial nodes when neutral: N_F, N_I exactly
    g.sumw_i = r[11];
    std::vector<double> spc(S * 5), spc0(S * 7, 0.0);
    std::vector<T> coef(S * 4), prob(S * 2);
    std::vector<double> kc(S * KC, 0.0);
    g.rho_ref.resize(S);
    g.gam_ref.resize(S);
    g.V.assign(3 * S, 0.0);
    g.Z0.assign(3 * S, 0.0);
    g.pa_max = 0.0;
    for (int sp = 0; sp < S; ++sp) {
        // uptake mode stores absolute densities (no reference, no source)
        const double Kr = h->uptake ? 0.0 : g.pa[sp] / g.pd[sp];
        const double Zp = g.sumw_f + g.sumw_i * Kr;
        const double rr = h->uptake ? 0.0 : 1.0 / Zp, gr = Kr / Zp;
        g.rho_ref[sp] = rr;
        g.gam_ref[sp] = gr;
        spc[5 * sp] = rr;
        spc[5 * sp + 1] = gr;
        for (int k = 0; k < 3; ++k) {
            g.V[3 * sp + k] = rr * g.A[k];
            g.Z0[3 * sp + k] = rr * g.B[k];
            spc[5 * sp + 2 + k] = g.V[3 * sp + k];
            spc0[4 * sp + k] = g.V[3 * sp + k];
            spc0[(size_t)S * 4 + 3 * sp + k] = g.Z0[3 * sp + k];
        }
        coef[4 * sp] = (T)rr;
        for (int k = 0; k < 3; ++k) coef[4 * sp + 1 + k] = (T)(rr * g.V[3 * sp + k]);
        prob[2 * sp] = (T)g.pa[sp];
        prob[2 * sp + 1] = (T)g.pd[sp];
        kc[KC * sp] = g.pa[sp];
        kc[KC * sp + 1] = g.pd[sp];
        kc[KC * sp + 2] = rr;
        for (int k = 0; k < 3; ++k) {
            kc[KC * sp + 3 + k] = rr * g.V[3 * sp + k];
            kc[KC * sp + 6 + k] = -g.V[3 * sp + k];
        }
        if (g.NI > 0) g.pa_max = std::max(g.pa_max, g.pa[sp]);
    }
    const double min_stay = std::min(g.min_stay_bulk, g.min_stay_iface - g.pa_max);
    if (min_stay < 0.0)
        return fail(LBMP_EPROB, "negative stay probability %.3e (sum p_i + p_a > 1)", min_stay);
    LBMP_HIP(hipMemcpyAsync(g.spc, spc.data(), spc.size() * 8, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.spc0, spc0.data(), spc0.size() * 8, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.coef, coef.data(), coef.size() * sizeof(T), hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.prob, prob.data(), prob.size() * sizeof(T), hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.kc, kc.data(), kc.size() * 8, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipStreamSynchronize(s));
    return LBMP_OK;
}

// rows x N values (row stride N) -> the fluid nodes' values at the head of
// each row, in lattice order
template <typename V>
__global__ void k_gather_fluid(const int32_t* __restrict__ fidx, int64_t N, const V* __restrict__ in,
                               V* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = blockIdx.y;
    if (n < N && fidx[n] >= 0) out[r * N + fidx[n]] = in[r * N + n];
}

// Link tables of geometry g in compact storage, through the set-up scratch
// (free once the state is initialised).
template <typename T>
lbmp_status compact_links(lbmp_mp* h, GeomHost& g, hipStream_t s) {
    const int64_t N = g.N;
    auto one = [&](void* buf, int rows, size_t es, auto tag) -> lbmp_status {
        using V = decltype(tag);
        V* tmp = reinterpret_cast<V*>(h->setup_tmp);
        dim3 grid((unsigned)((N + BLK - 1) / BLK), (unsigned)rows);
        k_gather_fluid<V><<<grid, BLK, 0, s>>>(cidx(h, g), N, static_cast<const V*>(buf), tmp);
        LBMP_HIP(hipGetLastError());
        LBMP_HIP(hipMemcpyAsync(buf, tmp, (size_t)rows * N * es, hipMemcpyDeviceToDevice, s));
        return LBMP_OK;
    };
    lbmp_status st = one(g.pin, NL, sizeof(T), T());
    if (st == LBMP_OK) st = one(g.sig, 1, sizeof(double), double());
    if (st == LBMP_OK) st = one(g.src, 1, sizeof(T), T());
    if (st == LBMP_OK) st = one(g.a, 3, sizeof(T), T());
    return st;
}

// Index of every fluid node among the fluid nodes in lattice order (-1 on
// solid nodes), the address of its fields in compact storage.
lbmp_status build_fidx(GeomHost& g, hipStream_t s) {
    std::vector<int8_t> cls(g.N);
    LBMP_HIP(hipMemcpyAsync(cls.data(), g.flow->d.cls, g.N, hipMemcpyDeviceToHost, s));
    LBMP_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> fi(g.N);
    int64_t c = 0;
    for (int64_t n = 0; n < g.N; ++n) fi[n] = cls[n] ? (int32_t)c++ : -1;
    if (c != g.nf) return fail(LBMP_ESTATE, "fluid node count %lld differs from the flow's %lld", (long long)c,
                               (long long)g.nf);
    LBMP_HIP(hipMemcpyAsync(g.fidx, fi.data(), g.N * 4, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipStreamSynchronize(s));
    g.fidx_h = std::move(fi);
    return LBMP_OK;
}

// Tables of the gathered-chunk blocks (variant 8) for geometry g. The compact
// order runs over tiles of GTX x GTY x GTZ lattice nodes and, within a
// tile, over its fluid nodes in lattice order; chunk c takes compact
// nodes base .. base + C - 1 (C up to the block's threads). Its halo, the
// fluid nodes outside the chunk its nodes pull from (r - c_k), is covered by
// quads of 4 consecutive compact nodes, each started at the lowest halo node
// the quads before it leave out; each node's 18 arrivals get their region
// slot: the chunk node's own position, 4 (ceil(C / 4) + q) + offset for a
// halo node in quad q, the zero slot for a solid r - c_k. A chunk whose quads
// exceed the region even when cut short leaves gather_ok false (the tuner
// then does not offer the variant for the workload).
lbmp_status build_gather(GeomHost& g, hipStream_t s) {
    g.gather_ok = false;
    const lbmp_flow* f = g.flow;
    const int nx = f->nx, ny = f->ny, nz = f->nz;
    const int64_t N = g.N;
    std::vector<int8_t> cls(N);
    std::vector<int32_t> slot(N);
    LBMP_HIP(hipMemcpyAsync(cls.data(), f->d.cls, N, hipMemcpyDeviceToHost, s));
    LBMP_HIP(hipMemcpyAsync(slot.data(), f->d.slot, N * 4, hipMemcpyDeviceToHost, s));
    LBMP_HIP(hipStreamSynchronize(s));
    // tiles of GTX x GTY x GTZ nodes, x fastest then y, z; long in x, so that
    // the halo a chunk pulls across its y and z faces comes in runs of up to
    // GTX consecutive compact nodes (whole cache lines) and its x faces are small
    // LBMP_GATHER_TILE="tx,ty,tz" overrides the tile shape (experiments)
    int gtx = GTX, gty = GTY, gtz = GTZ;
    if (const char* e = getenv("LBMP_GATHER_TILE")) {
        int a = 0, b = 0, c = 0;
        if (sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a > 0 && b > 0 && c > 0) {
            gtx = a;
            gty = b;
            gtz = c;
        }
    }
    std::vector<int32_t> gidx(N, -1), gnode;
    gnode.reserve(g.nf);
    for (int tz = 0; tz < nz; tz += gtz)
        for (int ty = 0; ty < ny; ty += gty)
            for (int tx = 0; tx < nx; tx += gtx)
                for (int z = tz; z < std::min(nz, tz + gtz); ++z)
                    for (int y = ty; y < std::min(ny, ty + gty); ++y)
                        for (int x = tx; x < std::min(nx, tx + gtx); ++x) {
                            const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                            if (cls[n]) {
                                gidx[n] = (int32_t)gnode.size();
                                gnode.push_back((int32_t)n);
                            }
                        }
    const int64_t NF = (int64_t)gnode.size();
    if (NF != g.nf) return fail(LBMP_ESTATE, "fluid node count %lld differs from the flow's %lld", (long long)NF,
                                (long long)g.nf);
    std::vector<int32_t> gaslot(NF, -1), aperm(std::max<int64_t>(g.NI, 1), 0);
    int32_t ai = 0;
    for (int64_t i = 0; i < NF; ++i)
        if (cls[gnode[i]] == 2) {
            gaslot[i] = ai;
            aperm[slot[gnode[i]]] = ai++;
        }
    g.gnh = 2;
    if (const char* e = getenv("LBMP_GATHER_NH")) g.gnh = atoi(e) == 1 ? 1 : 2;
    const int64_t CH = (int64_t)g.gnh * BLK;                      // nodes per chunk, region quads
    const int64_t ZS = g.gnh == 1 ? GatherShape<1>::ZSLOT : GatherShape<2>::ZSLOT;
    const int64_t cap = gather_chunk_cap(NF);
    std::vector<int4> chs;
    std::vector<int32_t> hsrc, halo, hq, pos(NF, -1);
    std::vector<uint16_t> nbr((size_t)NL * NF);
    auto from = [&](int64_t n, int k) {  // lattice index of r - c_k (periodic)
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        return (int64_t)wrapi(x - lcx(k), nx) + (int64_t)nx * (wrapi(y - lcy(k), ny) + (int64_t)ny * wrapi(z - lcz(k), nz));
    };
    auto halo_of = [&](int64_t base, int64_t C) {
        halo.clear();
        for (int64_t i = base; i < base + C; ++i)
            for (int k = 0; k < NL; ++k) {
                const int64_t m = from(gnode[i], k);
                if (!cls[m]) continue;
                const int32_t j = gidx[m];
                if (j < base || j >= base + C) halo.push_back(j);
            }
        std::sort(halo.begin(), halo.end());
        halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
        hq.clear();
        for (const int32_t h : halo)
            if (hq.empty() || h >= hq.back() + 4) hq.push_back(h);
    };
    // quads the region holds for chunk nodes and halo (the last quad stays zero)
    auto quads = [&](int64_t C) { return (C + 3) / 4 + (int64_t)hq.size(); };
    for (int64_t base = 0; base < NF;) {
        // the longest chunk (up to CH nodes, in steps of 64) whose quads fit
        int64_t C = std::min<int64_t>(CH, NF - base);
        halo_of(base, C);
        while (quads(C) > CH - 1 && C > 64) {
            C = std::max<int64_t>(64, C - 64);
            halo_of(base, C);
        }
        const int64_t Cq = (C + 3) / 4, H = (int64_t)hq.size();
        if (quads(C) > CH - 1 || (int64_t)chs.size() >= cap || (int64_t)hsrc.size() + H > cap * GatherShape<1>::REG)
            return LBMP_OK;  // does not fit the reserved tables: variant not offered
        for (size_t e = 0, q = 0; e < halo.size(); ++e) {
            while (q + 1 < hq.size() && hq[q + 1] <= halo[e]) ++q;
            pos[halo[e]] = (int32_t)(4 * (Cq + (int64_t)q) + (halo[e] - hq[q]));
        }
        for (int64_t i = base; i < base + C; ++i)
            for (int k = 0; k < NL; ++k) {
                const int64_t m = from(gnode[i], k);
                int32_t sl = (int32_t)ZS;
                if (cls[m]) {
                    const int32_t j = gidx[m];
                    sl = (j >= base && j < base + C) ? (int32_t)(j - base) : pos[j];
                }
                nbr[(size_t)k * NF + i] = (uint16_t)sl;
            }
        for (const int32_t h : halo) pos[h] = -1;
        chs.push_back(make_int4((int)base, (int)C, (int)hsrc.size(), (int)H));
        hsrc.insert(hsrc.end(), hq.begin(), hq.end());
        base += C;
    }
    const int64_t nch = (int64_t)chs.size();
    LBMP_HIP(hipMemcpyAsync(g.gidx, gidx.data(), N * 4, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.gnode, gnode.data(), NF * 4, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.gaslot, gaslot.data(), NF * 4, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.gch, chs.data(), nch * sizeof(int4), hipMemcpyHostToDevice, s));
    if (!hsrc.empty()) LBMP_HIP(hipMemcpyAsync(g.ghsrc, hsrc.data(), hsrc.size() * 4, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.gnbr, nbr.data(), nbr.size() * 2, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipMemcpyAsync(g.aperm, aperm.data(), aperm.size() * 4, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipStreamSynchronize(s));
    g.nch = nch;
    g.gidx_h = std::move(gidx);
    g.aperm_h = std::move(aperm);
    g.gather_ok = true;
    return LBMP_OK;
}

// The state at t = 1 lives in the odd buffer X1; X0 starts at zero. In uptake
// mode X1 holds the start tau = 0: density 1/N_F on every fluid node, first
// moments and adsorbed densities zero.
template <typename T>
lbmp_status init_state(lbmp_mp* h, GeomHost& g, hipStream_t s) {
    const int64_t N = g.N;
    double* b64 = h->setup_tmp + 18 * N;
    double* src64 = b64 + 3 * N;
    LBMP_HIP(hipMemsetAsync(g.X0, 0, (size_t)g.S * 4 * N * sizeof(T), s));
    if (h->uptake) {
        LBMP_HIP(hipMemsetAsync(g.X1, 0, (size_t)g.S * 4 * N * sizeof(T), s));
        LBMP_HIP(hipMemsetAsync(g.Xa, 0, (size_t)g.S * 4 * std::max<int64_t>(g.NI, 1) * sizeof(T), s));
        dim3 grid((unsigned)((N + BLK - 1) / BLK), (unsigned)g.S);
        k_init_uptake<T><<<grid, BLK, 0, s>>>(g.flow->d.cls, N, 1.0 / (double)g.nf, cidx(h, g),
                                              compact_fields(h) ? g.nf : N, (T*)g.X1);
        LBMP_HIP(hipGetLastError());
        return LBMP_OK;
    }
    dim3 grid((unsigned)((std::max<int64_t>(N, g.NI) + BLK - 1) / BLK), (unsigned)g.S);
    const double* w = g.bmu.empty() ? nullptr : setup_bmu(h->setup_tmp, N) + N;
    k_init_state<T><<<grid, BLK, 0, s>>>(g.flow->d.cls, g.flow->d.ilist, N, g.NI, g.S, g.spc, b64, src64, w,
                                         cidx(h, g), compact_fields(h) ? g.nf : N,
                                         h->variant == 8 ? g.aperm : nullptr, (T*)g.X1, (T*)g.Xa);
    LBMP_HIP(hipGetLastError());
    return LBMP_OK;
}

template <typename T>
lbmp_status setup_all(lbmp_mp* h, hipStream_t s) {
    double r[SETUP_RED];
    for (auto& g : h->g) {
        lbmp_status st = build_links<T>(h, g, s, r);
        if (st != LBMP_OK) return st;
        st = species_constants<T>(h, g, r, s);
        if (st != LBMP_OK) return st;
        st = build_fidx(g, s);
        if (st != LBMP_OK) return st;
        if (h->prec == LBMP_FP32) {
            st = build_gather(g, s);
            if (st != LBMP_OK) return st;
        }
        LBMP_HIP(hipMemsetAsync(g.X0, 0, (size_t)g.S * 4 * g.N * sizeof(T), s));
        LBMP_HIP(hipMemsetAsync(g.X1, 0, (size_t)g.S * 4 * g.N * sizeof(T), s));
        LBMP_HIP(hipMemsetAsync(g.Xa, 0, (size_t)g.S * 4 * std::max<int64_t>(g.NI, 1) * sizeof(T), s));
    }
    std::vector<int32_t> work;
    for (int gi = 0; gi < h->ngeom; ++gi)
        for (int sp = 0; sp < h->g[gi].S; ++sp) {
            work.push_back(gi);
            work.push_back(sp);
        }
    LBMP_HIP(hipMemcpyAsync(h->work, work.data(), work.size() * 4, hipMemcpyHostToDevice, s));
    // LBMP_MASS_DRIFT_MAX overrides the watchdog threshold (tests force it)
    double drift_max = LBMP_MASS_DRIFT_MAX;
    if (const char* e = getenv("LBMP_MASS_DRIFT_MAX")) drift_max = atof(e);
    Ctl c0{1, h->tmax, 0u, INT64_MAX, h->uptake ? 1.0 : 0.0, drift_max};
    LBMP_HIP(hipMemcpyAsync(h->ctl, &c0, sizeof c0, hipMemcpyHostToDevice, s));
    LBMP_HIP(hipStreamSynchronize(s));
    lbmp_status st = autotune(h);
    if (st != LBMP_OK) return st;
    // tuning advanced the device time and wrote the buffers: start over
    LBMP_HIP(hipMemcpyAsync(h->ctl, &c0, sizeof c0, hipMemcpyHostToDevice, s));
    for (auto& g : h->g) {
        st = build_links<T>(h, g, s, nullptr);
        if (st != LBMP_OK) return st;
        st = init_state<T>(h, g, s);
        if (st != LBMP_OK) return st;
        if (compact_fields(h)) {
            st = compact_links<T>(h, g, s);
            if (st != LBMP_OK) return st;
        }
    }
    LBMP_HIP(hipStreamSynchronize(s));
    return LBMP_OK;
}

lbmp_status check_mp(const lbmp_mp* h) {
    if (!h || h->magic != MP_MAGIC) return fail(LBMP_ESTATE, "invalid moment-propagation handle");
    return LBMP_OK;
}

// The watchdog's verdict over the steps run so far (the stream is synchronised
// by the caller).
lbmp_status check_watchdog(lbmp_mp* h) {
    Ctl c;
    LBMP_HIP(hipMemcpy(&c, h->ctl, sizeof c, hipMemcpyDeviceToHost));
    if (c.bad_t <= h->steps)
        return fail(LBMP_ENUMERIC, "total probability of a species left 1 by more than %.1e (or became non-finite) "
                                   "at step %lld", c.drift_max, (long long)c.bad_t);
    return LBMP_OK;
}

}  // namespace
}  // namespace lbmp

using namespace lbmp;

extern "C" lbmp_status mp_workspace_bytes(const lbmp_flow* const* flows, const lbmp_species* species,
                                          int n_geom, int precision, int64_t max_steps_recorded,
                                          size_t* bytes) {
    if (!flows || !species || n_geom < 1 || !bytes) return fail(LBMP_EINVAL, "bad arguments");
    if (precision != LBMP_FP32 && precision != LBMP_FP64) return fail(LBMP_EINVAL, "precision must be 32 or 64");
    if (max_steps_recorded < 0) return fail(LBMP_EINVAL, "max_steps_recorded must be >= 0");
    for (int gi = 0; gi < n_geom; ++gi) {
        if (!flows[gi] || flows[gi]->magic != FLOW_MAGIC) return fail(LBMP_ESTATE, "flow %d is not a valid handle", gi);
        if (species[gi].n_species < 1) return fail(LBMP_EINVAL, "geometry %d: n_species must be >= 1", gi);
        // per-node tables are addressed with 32-bit byte offsets, the widest
        // (the FP64 departure sums) at 8 bytes a node, and the masking offset
        // must lie beyond every table
        if (flows[gi]->N * 8 > (int64_t)OOB)
            return fail(LBMP_EINVAL, "geometry %d: %lld nodes exceed the per-field limit of %lld", gi,
                        (long long)flows[gi]->N, (long long)(OOB / 8));
    }
    lbmp_mp* h = make_handle(flows, species, n_geom, precision, max_steps_recorded);
    Carver c(nullptr, ~size_t(0));
    carve_all(h, c);
    *bytes = c.off;
    delete h;
    return LBMP_OK;
}

namespace {
// beta_mu_ex (nullable, and per geometry nullable): excess chemical potential
// of the tracers of a geometry, beta mu^ex per node (host, N doubles; values
// on solid nodes are ignored).
lbmp_status mp_create(const lbmp_flow* const* flows, const lbmp_species* species, const double* const* beta_mu_ex,
                      int n_geom, int precision, int64_t max_steps_recorded, void* dev_ws, size_t ws_bytes,
                      void* hip_stream, bool uptake, lbmp_mp** out) {
    if (!out) return fail(LBMP_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    lbmp_status st = mp_workspace_bytes(flows, species, n_geom, precision, max_steps_recorded, &need);
    if (st != LBMP_OK) return st;
    if (!dev_ws || ws_bytes < need) return fail(LBMP_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
    for (int gi = 0; gi < n_geom; ++gi) {
        st = validate_species(species[gi], gi, uptake);
        if (st != LBMP_OK) return st;
    }
    lbmp_mp* h = make_handle(flows, species, n_geom, precision, max_steps_recorded);
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->uptake = uptake ? 1 : 0;
    for (int gi = 0; gi < n_geom; ++gi) {
        GeomHost& g = h->g[gi];
        resolve_lambda(species[gi], &g.lam);
        g.pa.assign(species[gi].k_a, species[gi].k_a + g.S);  // p_a = k_a dt / dx
        g.pd.assign(species[gi].k_d, species[gi].k_d + g.S);  // p_d = k_d dt
        if (beta_mu_ex && beta_mu_ex[gi]) {
            const double* b = beta_mu_ex[gi];
            std::vector<int8_t> cls(g.N);
            hipError_t e = hipMemcpy(cls.data(), g.flow->d.cls, g.N, hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                delete h;
                return fail(LBMP_EDEVICE, "hipMemcpy of the node classes failed: %s", hipGetErrorString(e));
            }
            double bmin = INFINITY;
            for (int64_t n = 0; n < g.N; ++n) {
                if (!cls[n]) continue;
                if (!std::isfinite(b[n])) {
                    delete h;
                    return fail(LBMP_EINVAL, "geometry %d: beta_mu_ex is not finite at fluid node %lld", gi,
                                (long long)n);
                }
                bmin = std::min(bmin, b[n]);
            }
            // relative weights exp(-(beta mu^ex - min)): at most 1, the
            // normalisation absorbs the shift
            g.bmu.assign(g.N, 0.0);
            g.w.assign(g.N, 0.0);
            for (int64_t n = 0; n < g.N; ++n)
                if (cls[n]) {
                    g.bmu[n] = b[n];
                    g.w[n] = std::exp(-(b[n] - bmin));
                }
        }
    }
    Carver c(dev_ws, ws_bytes);
    carve_all(h, c);
    if (!c.fits()) {
        delete h;
        return fail(LBMP_ENOMEM, "workspace too small");
    }
    st = precision == LBMP_FP32 ? setup_all<float>(h, h->stream) : setup_all<double>(h, h->stream);
    if (st != LBMP_OK) {
        delete h;
        return st;
    }
    *out = h;
    return LBMP_OK;
}
}  // namespace

extern "C" lbmp_status mp_init(const lbmp_flow* const* flows, const lbmp_species* species, int n_geom,
                               int precision, int64_t max_steps_recorded, void* dev_ws, size_t ws_bytes,
                               void* hip_stream, lbmp_mp** out) {
    return mp_create(flows, species, nullptr, n_geom, precision, max_steps_recorded, dev_ws, ws_bytes, hip_stream,
                     false, out);
}

extern "C" lbmp_status mp_init_charged(const lbmp_flow* const* flows, const lbmp_species* species,
                                       const double* const* beta_mu_ex, int n_geom, int precision,
                                       int64_t max_steps_recorded, void* dev_ws, size_t ws_bytes, void* hip_stream,
                                       lbmp_mp** out) {
    if (!beta_mu_ex) return fail(LBMP_EINVAL, "beta_mu_ex is NULL (use mp_init for neutral tracers)");
    return mp_create(flows, species, beta_mu_ex, n_geom, precision, max_steps_recorded, dev_ws, ws_bytes,
                     hip_stream, false, out);
}

extern "C" lbmp_status mp_uptake_init(const lbmp_flow* const* flows, const lbmp_species* species, int n_geom,
                                      int precision, int64_t max_steps_recorded, void* dev_ws, size_t ws_bytes,
                                      void* hip_stream, lbmp_mp** out) {
    return mp_create(flows, species, nullptr, n_geom, precision, max_steps_recorded, dev_ws, ws_bytes, hip_stream,
                     true, out);
}

extern "C" lbmp_status mp_uptake(lbmp_mp* h, int geom, int64_t t0, int64_t count, double* mobile,
                                 double* adsorbed) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (!h->uptake) return fail(LBMP_ESTATE, "not an uptake handle (made by mp_init)");
    if (geom < 0 || geom >= h->ngeom) return fail(LBMP_EINVAL, "geometry index %d out of range", geom);
    // the sums of the state at tau are recorded by the step that reads it
    if (t0 < 0 || count < 0 || t0 + count > h->steps)
        return fail(LBMP_EINVAL, "times %lld..%lld not recorded (0..%lld)", (long long)t0,
                    (long long)(t0 + count - 1), (long long)(h->steps - 1));
    GeomHost& g = h->g[geom];
    const int S = g.S;
    std::vector<double> ser((size_t)count * S * NRED);
    if (count > 0)
        LBMP_HIP(hipMemcpyAsync(ser.data(), g.series + t0 * S * NRED, ser.size() * 8, hipMemcpyDeviceToHost,
                                h->stream));
    LBMP_HIP(hipStreamSynchronize(h->stream));
    st = check_watchdog(h);
    if (st != LBMP_OK) return st;
    for (int sp = 0; sp < S; ++sp)
        for (int64_t i = 0; i < count; ++i) {
            if (mobile) mobile[sp * count + i] = ser[(i * S + sp) * NRED + 3];
            if (adsorbed) adsorbed[sp * count + i] = ser[(i * S + sp) * NRED + 7];
        }
    for (size_t i = 0; i < ser.size(); ++i)
        if (!std::isfinite(ser[i])) return fail(LBMP_ENUMERIC, "non-finite value in the recorded totals");
    return LBMP_OK;
}

extern "C" lbmp_status mp_step_n(lbmp_mp* h, int64_t n_steps) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (n_steps < 0) return fail(LBMP_EINVAL, "n_steps must be >= 0");
    if (h->steps + n_steps > h->tmax)
        return fail(LBMP_ESTATE, "%lld steps would exceed max_steps_recorded = %lld",
                    (long long)(h->steps + n_steps), (long long)h->tmax);
    hipStream_t s = h->stream;
    int64_t left = n_steps;
    // replay a captured chunk of steps when the stream can be captured
    if (s != nullptr && left >= 2 * GRAPH_CHUNK) {
        if (!h->gexec) {
            LBMP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            do_steps(h, GRAPH_CHUNK, s);
            LBMP_HIP(hipStreamEndCapture(s, &h->graph));
            LBMP_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
        }
        while (left >= GRAPH_CHUNK) {
            LBMP_HIP(hipGraphLaunch(h->gexec, s));
            left -= GRAPH_CHUNK;
        }
    }
    do_steps(h, left, s);
    LBMP_HIP(hipGetLastError());
    h->steps += n_steps;
    return LBMP_OK;
}

extern "C" lbmp_status mp_steps_done(const lbmp_mp* h, int64_t* t) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (!t) return fail(LBMP_EINVAL, "t is NULL");
    *t = h->steps;
    return LBMP_OK;
}

extern "C" lbmp_status mp_vacf(lbmp_mp* h, int geom, int64_t t0, int64_t count, double* Z, double* D,
                               double* mass, double* vbar) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (h->uptake) return fail(LBMP_ESTATE, "an uptake handle records totals only (mp_uptake)");
    if (geom < 0 || geom >= h->ngeom) return fail(LBMP_EINVAL, "geometry index %d out of range", geom);
    if (t0 < 0 || count < 0 || t0 + count - 1 > h->steps)
        return fail(LBMP_EINVAL, "times %lld..%lld not recorded (0..%lld)", (long long)t0,
                    (long long)(t0 + count - 1), (long long)h->steps);
    GeomHost& g = h->g[geom];
    hipStream_t s = h->stream;
    const int S = g.S;
    const int64_t stride = h->tmax + 1;
    if ((Z || D) && count > 0) {
        k_vacf_series<<<(3 * S + 63) / 64, 64, 0, s>>>(g.series, S, h->steps, stride, g.spc0, g.zout, g.dout);
        LBMP_HIP(hipGetLastError());
        if (Z)
            LBMP_HIP(hipMemcpy2DAsync(Z, count * 8, g.zout + t0, stride * 8, count * 8, 3 * (size_t)S,
                                      hipMemcpyDeviceToHost, s));
        if (D)
            LBMP_HIP(hipMemcpy2DAsync(D, count * 8, g.dout + t0, stride * 8, count * 8, 3 * (size_t)S,
                                      hipMemcpyDeviceToHost, s));
    }
    std::vector<double> last;
    if (mass && h->steps > 0) {
        last.resize((size_t)S * NRED);
        LBMP_HIP(hipMemcpyAsync(last.data(), g.series + (h->steps - 1) * S * NRED, last.size() * 8,
                                hipMemcpyDeviceToHost, s));
    }
    LBMP_HIP(hipStreamSynchronize(s));
    st = check_watchdog(h);
    if (st != LBMP_OK) return st;
    if (mass)
        for (int sp = 0; sp < S; ++sp) {
            mass[2 * sp] = g.rho_ref[sp] * g.sumw_f + (last.empty() ? 0.0 : last[sp * NRED + 3]);
            mass[2 * sp + 1] = g.gam_ref[sp] * g.sumw_i + (last.empty() ? 0.0 : last[sp * NRED + 7]);
        }
    if (vbar)
        for (int i = 0; i < 3 * S; ++i) vbar[i] = g.V[i];
    const size_t n = (size_t)3 * S * count;
    for (size_t i = 0; i < n; ++i)
        if ((Z && !std::isfinite(Z[i])) || (D && !std::isfinite(D[i])))
            return fail(LBMP_ENUMERIC, "non-finite value in the recorded series");
    if (mass)
        for (int i = 0; i < 2 * S; ++i)
            if (!std::isfinite(mass[i])) return fail(LBMP_ENUMERIC, "non-finite total probability");
    return LBMP_OK;
}

extern "C" lbmp_status mp_stats(const lbmp_mp* h, int geom, lbmp_stats* out) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (geom < 0 || geom >= h->ngeom || !out) return fail(LBMP_EINVAL, "bad geometry index or output");
    const GeomHost& g = h->g[geom];
    out->n_nodes = g.N;
    out->n_fluid = g.nf;
    out->n_iface = g.NI;
    out->lambda = g.lam;
    out->min_p = g.min_p;
    out->max_cell_peclet = g.max_u / (g.lam / 12.0);
    out->min_stay = std::min(g.min_stay_bulk, g.min_stay_iface - g.pa_max);
    for (int k = 0; k < 3; ++k) out->mean_velocity[k] = g.A[k] / (double)g.nf;
    out->tile_k = h->K;
    out->species_per_block = h->gsz;
    out->kernel_variant = h->variant;
    return LBMP_OK;
}

extern "C" lbmp_status mp_state(lbmp_mp* h, int geom, int species, double* X, double* Xads) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (geom < 0 || geom >= h->ngeom) return fail(LBMP_EINVAL, "geometry index out of range");
    GeomHost& g = h->g[geom];
    if (species < 0 || species >= g.S) return fail(LBMP_EINVAL, "species index out of range");
    const int64_t N = g.N, NI = g.NI, NIa = std::max<int64_t>(NI, 1);
    const int64_t t = h->steps + 1;
    const size_t es = h->prec == LBMP_FP32 ? 4 : 8;
    // fields of fluid nodes only (in lattice order) with the haloed LDS-DMA blocks
    const int64_t NC = compact_fields(h) ? g.nf : N;
    const char* base = static_cast<const char*>((t & 1) ? g.X1 : g.X0) + (size_t)species * 4 * NC * es;
    const char* abase = static_cast<const char*>(g.Xa) + (size_t)species * 4 * NIa * es;
    std::vector<char> hx(4 * NC * es), ha(4 * NIa * es);
    std::vector<int8_t> cls(N);
    std::vector<int32_t> ilist(NIa);
    LBMP_HIP(hipMemcpyAsync(hx.data(), base, hx.size(), hipMemcpyDeviceToHost, h->stream));
    LBMP_HIP(hipMemcpyAsync(ha.data(), abase, ha.size(), hipMemcpyDeviceToHost, h->stream));
    LBMP_HIP(hipMemcpyAsync(cls.data(), g.flow->d.cls, N, hipMemcpyDeviceToHost, h->stream));
    if (NI > 0) LBMP_HIP(hipMemcpyAsync(ilist.data(), g.flow->d.ilist, NI * 4, hipMemcpyDeviceToHost, h->stream));
    LBMP_HIP(hipStreamSynchronize(h->stream));
    auto at = [&](const std::vector<char>& v, size_t i) {
        return es == 4 ? (double)reinterpret_cast<const float*>(v.data())[i]
                       : reinterpret_cast<const double*>(v.data())[i];
    };
    const double rr = g.rho_ref[species], gr = g.gam_ref[species];
    // where node n's fields and interface slot i's adsorbed fields are stored
    const std::vector<int32_t>* map = !compact_fields(h) ? nullptr : (h->variant == 8 ? &g.gidx_h : &g.fidx_h);
    const bool perm = h->variant == 8;
    for (int q = 0; q < 4; ++q) {
        const double cq = q == 0 ? 1.0 : g.V[3 * species + q - 1];
        for (int64_t n = 0; n < N; ++n) {
            const double wn = g.w.empty() ? 1.0 : g.w[n];
            if (X) X[q * N + n] = cls[n] ? at(hx, q * NC + (map ? (*map)[n] : n)) + cq * rr * wn : 0.0;
        }
        if (Xads) {
            for (int64_t n = 0; n < N; ++n) Xads[q * N + n] = 0.0;
            for (int64_t i = 0; i < NI; ++i)
                Xads[q * N + ilist[i]] =
                    at(ha, q * NIa + (perm ? g.aperm_h[i] : i)) + cq * gr * (g.w.empty() ? 1.0 : g.w[ilist[i]]);
        }
    }
    return LBMP_OK;
}

// ---------------------------------------------------------------- checkpoint
// A checkpoint holds the state at the last step: for every geometry the
// stored (deviation) fields of every species in the storage precision, fluid
// nodes in lattice order, the adsorbed fields in interface-list order, the
// recorded per-step sums, and the watchdog's state; a fingerprint of the
// set-up (shapes, node counts, rates, Eq. 11 references, mean velocities,
// Z(0)) guards against loading it into a handle of another workload. The
// canonical order does not depend on the step kernel the tuner chose.
namespace lbmp {
namespace {

constexpr uint64_t CKP_MAGIC = 0x31504B43504D424CULL;  // "LBMPCKP1" little-endian
struct CkpHeader {
    uint64_t magic, fingerprint, payload;
    int64_t steps, bad_t;
    int32_t prec, ngeom, uptake, pad;
};

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ULL;
    }
    return h;
}

uint64_t ckp_fingerprint(const lbmp_mp* h) {
    uint64_t f = 1469598103934665603ULL;
    const int32_t head[3] = {h->prec, h->ngeom, h->uptake};
    f = fnv1a(f, head, sizeof head);
    for (const auto& g : h->g) {
        const int64_t dims[7] = {g.flow->nx, g.flow->ny, g.flow->nz, g.N, g.NI, g.nf, g.S};
        f = fnv1a(f, dims, sizeof dims);
        f = fnv1a(f, &g.lam, sizeof g.lam);
        for (const auto* v : {&g.pa, &g.pd, &g.rho_ref, &g.gam_ref, &g.V, &g.Z0, &g.bmu})
            f = fnv1a(f, v->data(), v->size() * sizeof(double));
    }
    return f;
}

size_t ckp_payload(const lbmp_mp* h, int64_t steps) {
    const size_t es = h->prec == LBMP_FP32 ? 4 : 8;
    size_t b = 0;
    for (const auto& g : h->g)
        b += (size_t)g.S * 4 * ((size_t)g.nf + (size_t)g.NI) * es + (size_t)steps * g.S * NRED * 8;
    return b;
}

// device position of the field value of lattice node n (-1 on solid nodes)
// and of interface slot i's adsorbed value
struct CkpMaps {
    std::vector<int64_t> node;  // fluid nodes in lattice order -> device index
    std::vector<int64_t> slot;  // interface slots -> device index
};
lbmp_status ckp_maps(const lbmp_mp* h, const GeomHost& g, CkpMaps& m) {
    std::vector<int8_t> cls(g.N);
    LBMP_HIP(hipMemcpyAsync(cls.data(), g.flow->d.cls, g.N, hipMemcpyDeviceToHost, h->stream));
    LBMP_HIP(hipStreamSynchronize(h->stream));
    const std::vector<int32_t>* map = !compact_fields(h) ? nullptr : (h->variant == 8 ? &g.gidx_h : &g.fidx_h);
    m.node.clear();
    m.node.reserve(g.nf);
    for (int64_t n = 0; n < g.N; ++n)
        if (cls[n]) m.node.push_back(map ? (int64_t)(*map)[n] : n);
    if ((int64_t)m.node.size() != g.nf) return fail(LBMP_ESTATE, "fluid node count differs from the set-up");
    m.slot.resize(g.NI);
    for (int64_t i = 0; i < g.NI; ++i) m.slot[i] = h->variant == 8 ? g.aperm_h[i] : i;
    return LBMP_OK;
}

}  // namespace
}  // namespace lbmp

extern "C" lbmp_status mp_checkpoint_bytes(const lbmp_mp* h, size_t* bytes) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (!bytes) return fail(LBMP_EINVAL, "bytes is NULL");
    *bytes = sizeof(CkpHeader) + ckp_payload(h, h->steps);
    return LBMP_OK;
}

extern "C" lbmp_status mp_save(lbmp_mp* h, void* host_buf, size_t bytes) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    const size_t need = sizeof(CkpHeader) + ckp_payload(h, h->steps);
    if (!host_buf || bytes < need) return fail(LBMP_EINVAL, "checkpoint buffer of %zu bytes, need %zu", bytes, need);
    LBMP_HIP(hipStreamSynchronize(h->stream));
    Ctl c;
    LBMP_HIP(hipMemcpy(&c, h->ctl, sizeof c, hipMemcpyDeviceToHost));
    CkpHeader hd{CKP_MAGIC, ckp_fingerprint(h), need - sizeof(CkpHeader), h->steps, c.bad_t, h->prec, h->ngeom,
                 h->uptake, 0};
    char* out = static_cast<char*>(host_buf);
    memcpy(out, &hd, sizeof hd);
    out += sizeof hd;
    const size_t es = h->prec == LBMP_FP32 ? 4 : 8;
    const int64_t t = h->steps + 1;  // the current state's time: its fields are in X1 when t is odd
    for (auto& g : h->g) {
        CkpMaps m;
        st = ckp_maps(h, g, m);
        if (st != LBMP_OK) return st;
        const int64_t NC = compact_fields(h) ? g.nf : g.N, NIa = std::max<int64_t>(g.NI, 1);
        std::vector<char> hx((size_t)g.S * 4 * NC * es), ha((size_t)g.S * 4 * NIa * es);
        LBMP_HIP(hipMemcpyAsync(hx.data(), (t & 1) ? g.X1 : g.X0, hx.size(), hipMemcpyDeviceToHost, h->stream));
        LBMP_HIP(hipMemcpyAsync(ha.data(), g.Xa, ha.size(), hipMemcpyDeviceToHost, h->stream));
        LBMP_HIP(hipStreamSynchronize(h->stream));
        for (int64_t f = 0; f < (int64_t)g.S * 4; ++f)
            for (int64_t k = 0; k < g.nf; ++k, out += es) memcpy(out, hx.data() + (f * NC + m.node[k]) * es, es);
        for (int64_t f = 0; f < (int64_t)g.S * 4; ++f)
            for (int64_t i = 0; i < g.NI; ++i, out += es) memcpy(out, ha.data() + (f * NIa + m.slot[i]) * es, es);
        const size_t sb = (size_t)h->steps * g.S * NRED * 8;
        if (sb) LBMP_HIP(hipMemcpy(out, g.series, sb, hipMemcpyDeviceToHost));
        out += sb;
    }
    return LBMP_OK;
}

extern "C" lbmp_status mp_load(lbmp_mp* h, const void* host_buf, size_t bytes) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (!host_buf || bytes < sizeof(CkpHeader)) return fail(LBMP_EINVAL, "checkpoint buffer too small");
    CkpHeader hd;
    memcpy(&hd, host_buf, sizeof hd);
    if (hd.magic != CKP_MAGIC) return fail(LBMP_EINVAL, "not a moment-propagation checkpoint");
    if (hd.prec != h->prec || hd.ngeom != h->ngeom || hd.uptake != h->uptake || hd.fingerprint != ckp_fingerprint(h))
        return fail(LBMP_EINVAL, "checkpoint of another workload (geometries, species, precision or mode differ)");
    if (hd.steps < 0 || hd.steps > h->tmax)
        return fail(LBMP_ESTATE, "checkpoint at step %lld beyond max_steps_recorded = %lld", (long long)hd.steps,
                    (long long)h->tmax);
    const size_t payload = ckp_payload(h, hd.steps);
    if (hd.payload != payload || bytes < sizeof hd + payload)
        return fail(LBMP_EINVAL, "checkpoint buffer of %zu bytes, need %zu", bytes, sizeof hd + payload);
    LBMP_HIP(hipStreamSynchronize(h->stream));
    const char* in = static_cast<const char*>(host_buf) + sizeof hd;
    const size_t es = h->prec == LBMP_FP32 ? 4 : 8;
    const int64_t t = hd.steps + 1;
    for (auto& g : h->g) {
        CkpMaps m;
        st = ckp_maps(h, g, m);
        if (st != LBMP_OK) return st;
        const int64_t NC = compact_fields(h) ? g.nf : g.N, NIa = std::max<int64_t>(g.NI, 1);
        // solid nodes (dense fields) and unused slots stay zero
        std::vector<char> hx((size_t)g.S * 4 * NC * es, 0), ha((size_t)g.S * 4 * NIa * es, 0);
        for (int64_t f = 0; f < (int64_t)g.S * 4; ++f)
            for (int64_t k = 0; k < g.nf; ++k, in += es) memcpy(hx.data() + (f * NC + m.node[k]) * es, in, es);
        for (int64_t f = 0; f < (int64_t)g.S * 4; ++f)
            for (int64_t i = 0; i < g.NI; ++i, in += es) memcpy(ha.data() + (f * NIa + m.slot[i]) * es, in, es);
        LBMP_HIP(hipMemcpy((t & 1) ? g.X1 : g.X0, hx.data(), hx.size(), hipMemcpyHostToDevice));
        LBMP_HIP(hipMemcpy(g.Xa, ha.data(), ha.size(), hipMemcpyHostToDevice));
        const size_t sb = (size_t)hd.steps * g.S * NRED * 8;
        if (sb) LBMP_HIP(hipMemcpy(g.series, in, sb, hipMemcpyHostToDevice));
        in += sb;
    }
    Ctl c;
    LBMP_HIP(hipMemcpy(&c, h->ctl, sizeof c, hipMemcpyDeviceToHost));
    c.t = t;
    c.done = 0;
    c.bad_t = hd.bad_t;
    LBMP_HIP(hipMemcpy(h->ctl, &c, sizeof c, hipMemcpyHostToDevice));
    h->steps = hd.steps;
    return LBMP_OK;
}

extern "C" lbmp_status mp_profile_steps(lbmp_mp* h, int64_t n_steps, double* ms_step_kernel,
                                        double* ms_total) {
    lbmp_status st = check_mp(h);
    if (st != LBMP_OK) return st;
    if (n_steps < 1) return fail(LBMP_EINVAL, "n_steps must be >= 1");
    if (h->steps + n_steps > h->tmax)
        return fail(LBMP_ESTATE, "%lld steps would exceed max_steps_recorded = %lld",
                    (long long)(h->steps + n_steps), (long long)h->tmax);
    hipStream_t s = h->stream;
    std::vector<hipEvent_t> ev(2 * n_steps + 2);
    for (auto& e : ev) LBMP_HIP(hipEventCreate(&e));
    LBMP_HIP(hipEventRecord(ev[2 * n_steps], s));
    for (int64_t i = 0; i < n_steps; ++i) {
        LBMP_HIP(hipEventRecord(ev[2 * i], s));
        if (h->prec == LBMP_FP32) launch_step_kernel<float>(h, s); else launch_step_kernel<double>(h, s);
        LBMP_HIP(hipEventRecord(ev[2 * i + 1], s));
        if (h->prec == LBMP_FP32) launch_step_tail<float>(h, s); else launch_step_tail<double>(h, s);
    }
    LBMP_HIP(hipEventRecord(ev[2 * n_steps + 1], s));
    LBMP_HIP(hipEventSynchronize(ev[2 * n_steps + 1]));
    double ks = 0.0;
    for (int64_t i = 0; i < n_steps; ++i) {
        float ms = 0.f;
        LBMP_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
        ks += ms;
    }
    float tot = 0.f;
    LBMP_HIP(hipEventElapsedTime(&tot, ev[2 * n_steps], ev[2 * n_steps + 1]));
    for (auto& e : ev) (void)hipEventDestroy(e);
    h->steps += n_steps;
    if (ms_step_kernel) *ms_step_kernel = ks;
    if (ms_total) *ms_total = tot;
    return LBMP_OK;
}

extern "C" void mp_free(lbmp_mp* h) {
    if (!h || h->magic != MP_MAGIC) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->magic = 0;
    delete h;
}
