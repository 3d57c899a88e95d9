// Steady fluid flow by the lattice-Boltzmann equation (Eq. 6 of the paper):
// D3Q19 BGK, Guo forcing, half-way bounce-back, FP64, fused pull-stream +
// collide, one thread per fluid node, SoA populations [19][N_F] ping-pong
// over the fluid nodes only (in lattice order, through a lattice -> compact
// index map), so that no lane idles on a solid node and no solid value is
// moved; velocities stay on the dense lattice.
//
// The stored state is the post-collision population. A step gathers the
// post-collision populations of the upstream neighbours (or the reflected
// population of the node itself when the upstream node is solid), forms the
// density and the force-corrected velocity u = (sum f c)/rho + g/2, and
// relaxes towards the equilibrium with the Guo source term.
#include <mutex>
#include <vector>

#include "lbmp_internal.hpp"

namespace lbmp {

struct BGKParams {
    double tau, gx, gy, gz;
};

__device__ inline void bgk_collide(double f[19], const BGKParams& P, double& rho, double& ux,
                                   double& uy, double& uz) {
    double r = 0, jx = 0, jy = 0, jz = 0;
    r = f[0];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        double v = f[k + 1];
        r += v;
        jx += v * lcx(k);
        jy += v * lcy(k);
        jz += v * lcz(k);
    }
    rho = r;
    ux = jx / r + 0.5 * P.gx;
    uy = jy / r + 0.5 * P.gy;
    uz = jz / r + 0.5 * P.gz;
    const double Fx = r * P.gx, Fy = r * P.gy, Fz = r * P.gz;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double uF = ux * Fx + uy * Fy + uz * Fz;
    const double om = 1.0 / P.tau, pre = 1.0 - 0.5 / P.tau;
    // rest population
    {
        double feq = W_REST * r * (1.0 - 1.5 * uu);
        double S = pre * W_REST * (-3.0 * uF);
        f[0] = f[0] - om * (f[0] - feq) + S;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        double cu = lcx(k) * ux + lcy(k) * uy + lcz(k) * uz;
        double cF = lcx(k) * Fx + lcy(k) * Fy + lcz(k) * Fz;
        double feq = lw(k) * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        double S = pre * lw(k) * (3.0 * (cF - uF) + 9.0 * cu * cF);
        f[k + 1] = f[k + 1] - om * (f[k + 1] - feq) + S;
    }
}

// Start at rest: equilibrium with rho = 1, u = 0, then one collision with the
// force; the velocity slots of the residual history start at zero on solid
// nodes (the step kernel writes fluid nodes only).
__global__ void k_bgk_init(const uint8_t* __restrict__ solid, const int32_t* __restrict__ gidx,
                           double* __restrict__ fo, int64_t N, int64_t NF, BGKParams P, double* __restrict__ u0,
                           double* __restrict__ u1, double* __restrict__ u2) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (solid[n]) {
        for (int d = 0; d < 3; ++d) u0[d * N + n] = u1[d * N + n] = u2[d * N + n] = 0.0;
        return;
    }
    const int64_t i = gidx[n];
    double f[19];
    f[0] = W_REST;
#pragma unroll
    for (int k = 0; k < NL; ++k) f[k + 1] = lw(k);
    double rho, ux, uy, uz;
    bgk_collide(f, P, rho, ux, uy, uz);
    for (int k = 0; k < 19; ++k) fo[k * NF + i] = f[k];
    u0[n] = ux;
    u0[N + n] = uy;
    u0[2 * N + n] = uz;
}

// One step for fluid node i (lattice index gnode[i]): pull from the upstream
// neighbours through the compact map gidx (-1 on solid nodes: the node's own
// reflected population instead), collide, store; velocity on the lattice.
__global__ void k_bgk_step(const int32_t* __restrict__ gnode, const int32_t* __restrict__ gidx,
                           const double* __restrict__ fi, double* __restrict__ fo, int64_t NF, int nx, int ny,
                           int nz, BGKParams P, double* __restrict__ uout) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NF) return;
    const int64_t n = gnode[i];
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
    double f[19];
    f[0] = fi[i];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        int xs = wrapi(x - lcx(k), nx), ys = wrapi(y - lcy(k), ny), zs = wrapi(z - lcz(k), nz);
        const int32_t j = gidx[xs + (int64_t)nx * (ys + (int64_t)ny * zs)];
        f[k + 1] = j < 0 ? fi[(int64_t)((k ^ 1) + 1) * NF + i] : fi[(int64_t)(k + 1) * NF + j];
    }
    double rho, ux, uy, uz;
    bgk_collide(f, P, rho, ux, uy, uz);
#pragma unroll
    for (int k = 0; k < 19; ++k) fo[(int64_t)k * NF + i] = f[k];
    if (uout) {
        uout[n] = ux;
        uout[N + n] = uy;
        uout[2 * N + n] = uz;
    }
}

// Block maxima of |ubar(t) - ubar(t-1)| and |ubar(t)| over all components,
// ubar(t) = (u(t) + u(t-1))/2, from the velocities of the last three steps.
__global__ void k_resid(const double* __restrict__ u2, const double* __restrict__ u1,
                        const double* __restrict__ u0, int64_t N, double* __restrict__ part) {
    __shared__ double sd[256], sm[256];
    double d = 0.0, m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = 0.5 * (u0[i] + u1[i]), b = 0.5 * (u1[i] + u2[i]);
        d = fmax(d, fabs(a - b));
        m = fmax(m, fabs(a));
    }
    sd[threadIdx.x] = d;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
            sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sd[0];
        part[2 * blockIdx.x + 1] = sm[0];
    }
}

// Reported velocity: average of the last two steps.
__global__ void k_uavg(const double* __restrict__ u1, const double* __restrict__ u0, int64_t n3,
                       double* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) out[i] = 0.5 * (u0[i] + u1[i]);
}

__global__ void k_resid_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double d = 0.0, m = 0.0;
    for (int k = 0; k < nb; ++k) {
        d = fmax(d, part[2 * k]);
        m = fmax(m, part[2 * k + 1]);
    }
    out[0] = d;
    out[1] = m;
}

__global__ void k_zero_solid_u(const uint8_t* __restrict__ solid, double* __restrict__ u, int64_t N) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (solid[n]) u[n] = u[N + n] = u[2 * N + n] = 0.0;
}

constexpr int RES_BLOCKS = 512;

static size_t scratch_bytes_for(int64_t N) {
    return 2 * align_up(19 * 8 * (size_t)N) + 3 * align_up(24 * (size_t)N) +
           align_up(2 * 8 * RES_BLOCKS) + align_up(16) + 2 * align_up(4 * (size_t)N);
}

}  // namespace lbmp

using namespace lbmp;

extern "C" lbmp_status lb_flow_workspace_bytes(const lbmp_geometry* g, size_t* persistent,
                                               size_t* scratch_out) {
    if (!g || g->nx <= 0 || g->ny <= 0 || g->nz <= 0)
        return fail(LBMP_EINVAL, "invalid geometry");
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    if (persistent) *persistent = align_up(sizeof(lbmp_flow)) + geometry_bytes(N);
    if (scratch_out) *scratch_out = scratch_bytes_for(N);
    return LBMP_OK;
}

static lbmp_status make_flow(const lbmp_geometry* g, void* dev_ws, size_t ws_bytes, hipStream_t s,
                             lbmp_flow** out) {
    lbmp_status st = validate_geometry(g);
    if (st != LBMP_OK) return st;
    if (!dev_ws) return fail(LBMP_EINVAL, "workspace is NULL");
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    Carver c(dev_ws, ws_bytes);
    c.take<char>(sizeof(lbmp_flow));  // reserved, keeps layouts aligned with the query
    auto* f = new lbmp_flow();
    f->magic = FLOW_MAGIC;
    f->nx = g->nx;
    f->ny = g->ny;
    f->nz = g->nz;
    f->nbhd = g->iface_nbhd == 6 ? 6 : 18;
    f->N = N;
    st = build_geometry(g, c, f->d, s, &f->nf, &f->ni);
    if (st != LBMP_OK) {
        delete f;
        return st;
    }
    f->converged = 1;
    f->steps = 0;
    f->residual = 0.0;
    *out = f;
    return LBMP_OK;
}

// The solve of lb_flow_solve and lb_flow_solve_static: populations, velocity
// history and residual partials in dev_scratch (scratch_bytes long); nothing
// in dev_scratch needs to start at zero.
static lbmp_status flow_solve(const lbmp_geometry* g, double tau, const double force[3], double tol,
                              int64_t max_steps, int check_every, void* dev_ws, size_t ws_bytes,
                              void* dev_scratch, size_t scratch_bytes, void* hip_stream, lbmp_flow** out,
                              int64_t* steps_done, double* residual) {
    if (!out) return fail(LBMP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(LBMP_EINVAL, "tau must exceed 1/2");
    if (!force || !std::isfinite(force[0]) || !std::isfinite(force[1]) || !std::isfinite(force[2]))
        return fail(LBMP_EINVAL, "force must be finite");
    if (max_steps < 1) return fail(LBMP_EINVAL, "max_steps must be >= 1");
    if (!(tol >= 0.0)) return fail(LBMP_EINVAL, "tol must be >= 0");
    if (check_every < 0) return fail(LBMP_EINVAL, "check_every must be >= 0");
    int ce = check_every == 0 ? 100 : check_every;
    lbmp_status st = validate_geometry(g);
    if (st != LBMP_OK) return st;
    size_t need_p = 0, need_s = 0;
    st = lb_flow_workspace_bytes(g, &need_p, &need_s);
    if (st != LBMP_OK) return st;
    if (ws_bytes < need_p || scratch_bytes < need_s || !dev_scratch)
        return fail(LBMP_ENOMEM, "workspace %zu/%zu bytes, need %zu/%zu", ws_bytes, scratch_bytes,
                    need_p, need_s);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    lbmp_flow* f = nullptr;
    st = make_flow(g, dev_ws, ws_bytes, s, &f);
    if (st != LBMP_OK) return st;
    const int64_t N = f->N;
    Carver c(dev_scratch, scratch_bytes);
    double* fa = c.take<double>(19 * N);
    double* fb = c.take<double>(19 * N);
    // velocities of the last three steps, slot = step % 3
    double* U[3] = {c.take<double>(3 * N), c.take<double>(3 * N), c.take<double>(3 * N)};
    double* part = c.take<double>(2 * RES_BLOCKS);
    double* res = c.take<double>(2);
    int32_t* gidx = c.take<int32_t>(N);
    int32_t* gnode = c.take<int32_t>(N);
    // compact order of the fluid nodes (lattice order) from the host mask
    const int64_t NF = f->nf;
    {
        std::vector<int32_t> gi((size_t)N), gn;
        gn.reserve((size_t)NF);
        for (int64_t n = 0; n < N; ++n) {
            gi[n] = g->solid[n] ? -1 : (int32_t)gn.size();
            if (!g->solid[n]) gn.push_back((int32_t)n);
        }
        if ((int64_t)gn.size() != NF) {
            delete f;
            return fail(LBMP_ESTATE, "fluid node count %lld differs from the classification's %lld",
                        (long long)gn.size(), (long long)NF);
        }
        LBMP_HIP(hipMemcpyAsync(gidx, gi.data(), (size_t)N * 4, hipMemcpyHostToDevice, s));
        LBMP_HIP(hipMemcpyAsync(gnode, gn.data(), (size_t)NF * 4, hipMemcpyHostToDevice, s));
        LBMP_HIP(hipStreamSynchronize(s));
    }
    BGKParams P{tau, force[0], force[1], force[2]};
    const unsigned nb = (unsigned)((N + 255) / 256), nbf = (unsigned)((NF + 255) / 256);
    k_bgk_init<<<nb, 256, 0, s>>>(f->d.solid, gidx, fa, N, NF, P, U[0], U[1], U[2]);
    LBMP_HIP(hipGetLastError());
    double resv = INFINITY;
    int64_t step = 0;
    int conv = 0;
    while (step < max_steps) {
        const int64_t sn = step + 1;
        const bool check = sn >= 2 && (sn % ce) == 0;
        // u is needed at a check step and the two steps before it, and at the
        // last two steps (the reported velocity)
        const bool need = check || ((sn + 1) % ce) == 0 || ((sn + 2) % ce) == 0 || sn + 1 >= max_steps;
        double* uo = need ? U[sn % 3] : nullptr;
        k_bgk_step<<<nbf, 256, 0, s>>>(gnode, gidx, fa, fb, NF, f->nx, f->ny, f->nz, P, uo);
        std::swap(fa, fb);
        step = sn;
        if (check) {
            k_resid<<<RES_BLOCKS, 256, 0, s>>>(U[(sn - 2) % 3], U[(sn - 1) % 3], U[sn % 3], N, part);
            k_resid_final<<<1, 64, 0, s>>>(part, RES_BLOCKS, res);
            double h[2];
            LBMP_HIP(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s));
            LBMP_HIP(hipStreamSynchronize(s));
            resv = h[1] > 0.0 ? h[0] / h[1] : h[0];
            if (!std::isfinite(resv)) {
                delete f;
                return fail(LBMP_ENUMERIC, "flow solve produced a non-finite velocity at step %lld",
                            (long long)sn);
            }
            if (resv < tol) {
                conv = 1;
                break;
            }
        }
    }
    LBMP_HIP(hipGetLastError());
    {
        // step >= 1: u(step) and u(step-1) were both written (u(0) by the init)
        const int64_t n3 = 3 * N;
        k_uavg<<<(unsigned)((n3 + 255) / 256), 256, 0, s>>>(U[(step - 1) % 3], U[step % 3], n3, f->d.u);
        LBMP_HIP(hipGetLastError());
    }
    LBMP_HIP(hipStreamSynchronize(s));
    f->converged = conv;
    f->steps = step;
    f->residual = resv;
    if (steps_done) *steps_done = step;
    if (residual) *residual = resv;
    *out = f;
    if (!conv) return fail(LBMP_ENOTCONV, "flow not converged after %lld steps (residual %.3e)",
                           (long long)step, resv);
    return LBMP_OK;
}

extern "C" lbmp_status lb_flow_solve(const lbmp_geometry* g, double tau, const double force[3],
                                     double tol, int64_t max_steps, int check_every, void* dev_ws,
                                     size_t ws_bytes, void* dev_scratch, size_t scratch_bytes,
                                     void* hip_stream, lbmp_flow** out, int64_t* steps_done,
                                     double* residual) {
    return flow_solve(g, tau, force, tol, max_steps, check_every, dev_ws, ws_bytes, dev_scratch, scratch_bytes,
                      hip_stream, out, steps_done, residual);
}

// ---------------------------------------------------------------- no-allocation solve
// lb_flow_solve_static takes its scratch from a file-scope device array
// instead of a caller workspace, for callers that cannot allocate device
// memory. Each GPU holds its own copy of the array (at its own address) until
// the process ends; the host-side name is not a device address, so the
// address is taken once per device with hipGetSymbolAddress and used from
// then on.
namespace lbmp {
static __device__ __align__(256) unsigned char scratch[LBMP_STATIC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES];  // per device, null until first use there

static lbmp_status static_scratch(void** ptr) {
    int dev = -1;
    LBMP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBMP_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBMP_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return LBMP_OK;
}
}  // namespace lbmp

extern "C" lbmp_status lb_flow_solve_static(const lbmp_geometry* g, double tau, const double force[3],
                                            double tol, int64_t max_steps, int check_every, void* dev_ws,
                                            size_t ws_bytes, void* hip_stream, lbmp_flow** out,
                                            int64_t* steps_done, double* residual) {
    if (!out) return fail(LBMP_EINVAL, "out is NULL");
    *out = nullptr;
    lbmp_status st = validate_geometry(g);
    if (st != LBMP_OK) return st;
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    const size_t need = scratch_bytes_for(N);
    if (need > (size_t)LBMP_STATIC_SCRATCH_BYTES)
        return fail(LBMP_ENOMEM, "lattice of %lld nodes needs %zu scratch bytes; the static scratch holds %zu "
                    "(at most %lld nodes)", (long long)N, need, (size_t)LBMP_STATIC_SCRATCH_BYTES,
                    (long long)lb_flow_static_max_nodes());
    void* p = nullptr;
    st = static_scratch(&p);
    if (st != LBMP_OK) return st;
    return flow_solve(g, tau, force, tol, max_steps, check_every, dev_ws, ws_bytes, p,
                      (size_t)LBMP_STATIC_SCRATCH_BYTES, hip_stream, out, steps_done, residual);
}

extern "C" int64_t lb_flow_static_max_nodes(void) {
    // scratch_bytes_for is 384 bytes per node plus alignment and the residual
    // partials; the largest N that fits
    int64_t lo = 0, hi = (int64_t)LBMP_STATIC_SCRATCH_BYTES / 384 + 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (scratch_bytes_for(mid) <= (size_t)LBMP_STATIC_SCRATCH_BYTES) lo = mid; else hi = mid - 1;
    }
    return lo;
}

extern "C" lbmp_status lb_flow_from_velocity(const lbmp_geometry* g, const double* u_host,
                                             void* dev_ws, size_t ws_bytes, void* hip_stream,
                                             lbmp_flow** out) {
    if (!out) return fail(LBMP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!u_host) return fail(LBMP_EINVAL, "velocity is NULL");
    lbmp_status st = validate_geometry(g);
    if (st != LBMP_OK) return st;
    size_t need_p = 0;
    st = lb_flow_workspace_bytes(g, &need_p, nullptr);
    if (st != LBMP_OK) return st;
    if (ws_bytes < need_p) return fail(LBMP_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need_p);
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    for (int64_t i = 0; i < 3 * N; ++i)
        if (!std::isfinite(u_host[i]) && !g->solid[i % N])
            return fail(LBMP_EINVAL, "velocity is not finite at a fluid node");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    lbmp_flow* f = nullptr;
    st = make_flow(g, dev_ws, ws_bytes, s, &f);
    if (st != LBMP_OK) return st;
    LBMP_HIP(hipMemcpyAsync(f->d.u, u_host, 24 * (size_t)N, hipMemcpyHostToDevice, s));
    k_zero_solid_u<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(f->d.solid, f->d.u, N);
    LBMP_HIP(hipGetLastError());
    LBMP_HIP(hipStreamSynchronize(s));
    *out = f;
    return LBMP_OK;
}

extern "C" lbmp_status lb_flow_velocity(const lbmp_flow* f, double* u_host) {
    if (!f || f->magic != FLOW_MAGIC) return fail(LBMP_ESTATE, "invalid flow handle");
    if (!u_host) return fail(LBMP_EINVAL, "output is NULL");
    LBMP_HIP(hipMemcpy(u_host, f->d.u, 24 * (size_t)f->N, hipMemcpyDeviceToHost));
    return LBMP_OK;
}

extern "C" lbmp_status lb_flow_classes(const lbmp_flow* f, int8_t* cls_host, int64_t* n_fluid,
                                       int64_t* n_iface) {
    if (!f || f->magic != FLOW_MAGIC) return fail(LBMP_ESTATE, "invalid flow handle");
    if (cls_host) LBMP_HIP(hipMemcpy(cls_host, f->d.cls, (size_t)f->N, hipMemcpyDeviceToHost));
    if (n_fluid) *n_fluid = f->nf;
    if (n_iface) *n_iface = f->ni;
    return LBMP_OK;
}

extern "C" void lb_flow_free(lbmp_flow* f) {
    if (f && f->magic == FLOW_MAGIC) {
        f->magic = 0;
        delete f;
    }
}
