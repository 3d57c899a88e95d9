// Node classification (solid / fluid / interfacial) and the compacted
// interfacial-node list. Interfacial nodes are the fluid nodes where
// adsorption can happen (Sec. II of the paper, node classes of Eq. 11).
#include <cstdarg>

#include "lbmp_internal.hpp"

namespace lbmp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

lbmp_status fail(lbmp_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

constexpr int CBLK = 1024;  // nodes per counting block

// cls: 0 solid, 1 fluid, 2 interfacial fluid (a solid node among the first
// `nlinks` D3Q19 neighbours, periodic wrap).
__global__ void k_classify(const uint8_t* __restrict__ solid, int8_t* __restrict__ cls, int nx,
                           int ny, int nz, int nlinks) {
    int64_t N = (int64_t)nx * ny * nz;
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (solid[n]) {
        cls[n] = 0;
        return;
    }
    int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
    bool iface = false;
    for (int k = 0; k < nlinks; ++k) {
        int xx = wrapi(x + lcx(k), nx), yy = wrapi(y + lcy(k), ny), zz = wrapi(z + lcz(k), nz);
        iface |= solid[xx + (int64_t)nx * (yy + (int64_t)ny * zz)] != 0;
    }
    cls[n] = iface ? 2 : 1;
}

// Per 1024-node block: number of fluid and of interfacial nodes.
__global__ void k_count(const int8_t* __restrict__ cls, int64_t N, uint32_t* __restrict__ nflu,
                        uint32_t* __restrict__ nifc) {
    __shared__ uint32_t sf[CBLK / 64], si[CBLK / 64];
    int64_t n = (int64_t)blockIdx.x * CBLK + threadIdx.x;
    int8_t c = n < N ? cls[n] : 0;
    uint64_t bf = __ballot(c != 0), bi = __ballot(c == 2);
    int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        sf[w] = __popcll(bf);
        si[w] = __popcll(bi);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int k = 0; k < CBLK / 64; ++k) {
            a += sf[k];
            b += si[k];
        }
        nflu[blockIdx.x] = a;
        nifc[blockIdx.x] = b;
    }
}

// Exclusive scan of the per-block interfacial counts (one block); totals out.
__global__ void k_scan_blocks(const uint32_t* __restrict__ nflu, uint32_t* __restrict__ nifc,
                              int nb, int64_t* __restrict__ totals) {
    __shared__ uint64_t part[256];
    __shared__ uint64_t fpart[256];
    int t = threadIdx.x;
    // each thread owns a contiguous chunk
    int chunk = (nb + 255) / 256;
    int lo = t * chunk, hi = min(nb, lo + chunk);
    uint64_t s = 0, f = 0;
    for (int k = lo; k < hi; ++k) {
        s += nifc[k];
        f += nflu[k];
    }
    part[t] = s;
    fpart[t] = f;
    __syncthreads();
    if (t == 0) {
        uint64_t acc = 0, facc = 0;
        for (int k = 0; k < 256; ++k) {
            uint64_t v = part[k];
            part[k] = acc;
            acc += v;
            facc += fpart[k];
        }
        totals[0] = (int64_t)facc;
        totals[1] = (int64_t)acc;
    }
    __syncthreads();
    uint64_t acc = part[t];
    for (int k = lo; k < hi; ++k) {
        uint32_t v = nifc[k];
        nifc[k] = (uint32_t)acc;
        acc += v;
    }
}

// slot[n] = rank of n among interfacial nodes (ascending node index), -1 else.
__global__ void k_scatter(const int8_t* __restrict__ cls, int64_t N, const uint32_t* __restrict__ boff,
                          int32_t* __restrict__ slot, int32_t* __restrict__ ilist) {
    __shared__ uint32_t wcount[CBLK / 64];
    int64_t n = (int64_t)blockIdx.x * CBLK + threadIdx.x;
    bool is = n < N && cls[n] == 2;
    uint64_t b = __ballot(is);
    int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    uint32_t below = __popcll(b & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wcount[w] = __popcll(b);
    __syncthreads();
    uint32_t off = boff[blockIdx.x];
    for (int k = 0; k < w; ++k) off += wcount[k];
    if (n < N) {
        if (is) {
            slot[n] = (int32_t)(off + below);
            ilist[off + below] = (int32_t)n;
        } else {
            slot[n] = -1;
        }
    }
}

size_t geometry_bytes(int64_t N) {
    size_t nb = (size_t)((N + CBLK - 1) / CBLK);
    return align_up(N) + align_up(N) + align_up(4 * N) + align_up(4 * N) + align_up(24 * N) +
           align_up(16) + 2 * align_up(4 * nb);
}

lbmp_status validate_geometry(const lbmp_geometry* g) {
    if (!g) return fail(LBMP_EINVAL, "geometry is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0)
        return fail(LBMP_EINVAL, "lattice sizes must be positive (got %d %d %d)", g->nx, g->ny, g->nz);
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    if (N > (int64_t)INT32_MAX) return fail(LBMP_EINVAL, "lattice has more than 2^31-1 nodes");
    if (!g->solid) return fail(LBMP_EINVAL, "solid mask is NULL");
    if (g->iface_nbhd != 0 && g->iface_nbhd != 6 && g->iface_nbhd != 18)
        return fail(LBMP_EINVAL, "iface_nbhd must be 0, 6 or 18");
    const int n[3] = {g->nx, g->ny, g->nz};
    bool any_fluid = false;
    for (int64_t i = 0; i < N; ++i) {
        if (g->solid[i] > 1) return fail(LBMP_EINVAL, "solid mask values must be 0 or 1");
        any_fluid |= g->solid[i] == 0;
    }
    if (!any_fluid) return fail(LBMP_EINVAL, "geometry has no fluid node");
    for (int d = 0; d < 3; ++d) {
        if (g->periodic[d]) continue;
        for (int side = 0; side < 2; ++side) {
            int fixed = side ? n[d] - 1 : 0;
            for (int z = 0; z < g->nz; ++z)
                for (int y = 0; y < g->ny; ++y)
                    for (int x = 0; x < g->nx; ++x) {
                        int c[3] = {x, y, z};
                        if (c[d] != fixed) continue;
                        if (!g->solid[x + (int64_t)g->nx * (y + (int64_t)g->ny * z)])
                            return fail(LBMP_EINVAL,
                                        "axis %d is not periodic but its boundary plane has a fluid node",
                                        d);
                    }
        }
    }
    return LBMP_OK;
}

lbmp_status build_geometry(const lbmp_geometry* g, Carver& c, FlowLayout& L, hipStream_t s,
                           int64_t* nf, int64_t* ni) {
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    int nb = (int)((N + CBLK - 1) / CBLK);
    L.solid = c.take<uint8_t>(N);
    L.cls = c.take<int8_t>(N);
    L.slot = c.take<int32_t>(N);
    L.ilist = c.take<int32_t>(N);
    L.u = c.take<double>(3 * N);
    L.counts = c.take<int64_t>(2);
    L.blk = c.take<uint32_t>(nb);
    uint32_t* blk2 = c.take<uint32_t>(nb);
    if (!c.fits()) return fail(LBMP_ENOMEM, "flow workspace too small");
    LBMP_HIP(hipMemcpyAsync(L.solid, g->solid, N, hipMemcpyHostToDevice, s));
    int nlinks = g->iface_nbhd == 6 ? 6 : 18;
    k_classify<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(L.solid, L.cls, g->nx, g->ny, g->nz, nlinks);
    LBMP_HIP(hipGetLastError());
    k_count<<<nb, CBLK, 0, s>>>(L.cls, N, L.blk, blk2);
    k_scan_blocks<<<1, 256, 0, s>>>(L.blk, blk2, nb, L.counts);
    k_scatter<<<nb, CBLK, 0, s>>>(L.cls, N, blk2, L.slot, L.ilist);
    LBMP_HIP(hipGetLastError());
    int64_t h[2];
    LBMP_HIP(hipMemcpyAsync(h, L.counts, sizeof h, hipMemcpyDeviceToHost, s));
    LBMP_HIP(hipStreamSynchronize(s));
    *nf = h[0];
    *ni = h[1];
    return LBMP_OK;
}

}  // namespace lbmp

extern "C" const char* lbmp_last_error(void) { return lbmp::g_err; }
extern "C" const char* lbmp_version(void) { return "lbmp 0.1 (gfx950)"; }
