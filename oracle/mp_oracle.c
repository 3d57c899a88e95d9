/*
 * FP64 CPU oracle for lattice-Boltzmann moment propagation with adsorption
 * and desorption (Levesque, Duvail, Pagonabarraga, Frenkel, Rotenberg,
 * "Accounting for adsorption and desorption in Lattice Boltzmann
 * simulations", arXiv:1303.2470).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference the GPU
 * path is checked against. Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load it; the product path never does. It shares
 * no code, table or constant with the GPU library.
 *
 * Everything is double precision, one node at a time, in the paper's "stay"
 * form of the propagation (Sec. II, Eq. 7) with no flux or deviation
 * rewriting. Global sums use Neumaier compensated summation over fixed
 * chunks, so results do not depend on the OpenMP thread count.
 *
 * Readings of the paper taken here (the paper is silent or ambiguous):
 *  - D3Q19 with weights 1/3, 1/18, 1/36 and c_s^2 = 1/3 (Sec. I: "19 values").
 *  - Links from or into a solid node carry no probability (Sec. II: the
 *    quantity is propagated between fluid nodes); the tracer stays instead.
 *  - In Eq. 8 f_i/rho is the equilibrium distribution at the local density
 *    and (force-corrected) velocity, so
 *      p_i = w_i (lambda/2 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2),  Q = 1.
 *  - At an interface node the stay probability of Eq. 7 also loses p_a, so
 *    that Eqs. 9-10 conserve probability; adsorption uses the pre-step mobile
 *    quantity and desorbed quantity re-enters at the same node (one
 *    simultaneous Markov step).
 *  - Interface nodes: fluid nodes with at least one solid node among their
 *    18 D3Q19 neighbours (6 face neighbours as an option), periodic wrap.
 *  - Initial weights (Eq. 11, no excess chemical potential): 1/Z on every
 *    fluid node for the mobile part, (p_a/p_d)/Z adsorbed on interface nodes,
 *    Z = N_F + N_I p_a/p_d. The first-moment quantities start as the
 *    velocity-weighted first hop out of these weights.
 *  - Fluid: BGK with Guo forcing (force density rho*g), half-way bounce-back,
 *    velocity u = (sum f c + F/2)/rho.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q19 19

/* D3Q19 velocities: rest, 6 face links, 12 edge links; opposite links are
 * stored next to each other (1<->2, 3<->4, ...). */
static const int CX[Q19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W[Q19] = {1.0 / 3,
                              1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

static long wrap(long a, long n) { a %= n; return a < 0 ? a + n : a; }

/* node index of r + c_i (periodic) */
static long neighbour(int nx, int ny, int nz, long n, int i)
{
    long x = n % nx, y = (n / nx) % ny, z = n / ((long)nx * ny);
    return wrap(x + CX[i], nx) + (long)nx * (wrap(y + CY[i], ny) + (long)ny * wrap(z + CZ[i], nz));
}

/* ---- deterministic compensated sum ------------------------------------ */
#define CHUNK 4096
static void neumaier_add(double* s, double* c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v; else *c += (v - t) + *s;
    *s = t;
}
static double nsum(const double* a, long n)
{
    long nch = (n + CHUNK - 1) / CHUNK;
    if (nch == 0) return 0.0;
    double* part = (double*)malloc(sizeof(double) * nch);
    #pragma omp parallel for schedule(static) if (n > 32768)
    for (long k = 0; k < nch; ++k) {
        double s = 0.0, c = 0.0;
        long hi = (k + 1) * CHUNK < n ? (k + 1) * CHUNK : n;
        for (long j = k * CHUNK; j < hi; ++j) neumaier_add(&s, &c, a[j]);
        part[k] = s + c;
    }
    double s = 0.0, c = 0.0;
    for (long k = 0; k < nch; ++k) neumaier_add(&s, &c, part[k]);
    free(part);
    return s + c;
}

/* ---- node classes ------------------------------------------------------ */
/* cls[n]: 0 solid, 1 fluid away from the wall, 2 interfacial fluid node. */
int orc_classify(int nx, int ny, int nz, const uint8_t* solid, int nbhd, int8_t* cls)
{
    long N = (long)nx * ny * nz;
    int last = (nbhd == 6) ? 6 : 18;
    #pragma omp parallel for schedule(static) if (N > 32768)
    for (long n = 0; n < N; ++n) {
        if (solid[n]) { cls[n] = 0; continue; }
        int iface = 0;
        for (int i = 1; i <= last; ++i)
            if (solid[neighbour(nx, ny, nz, n, i)]) iface = 1;
        cls[n] = iface ? 2 : 1;
    }
    return 0;
}

/* ---- link probabilities (Eq. 8) ---------------------------------------- */
/* p[i*N + n] = probability to leave n along c_i, i = 1..18; p[0..N-1] = 0.
 * u: [3][N] velocity, or NULL for a fluid at rest.
 * bmu: [N] excess chemical potential beta mu^ex(r) of the tracer (e.g. its
 * charge times the electrostatic potential, over k_B T), or NULL (neutral).
 * The diffusive term of Eq. 8 carries the factor
 *   Q_i(r) = exp(-(beta mu^ex(r + c_i) - beta mu^ex(r)) / 2),
 * so that at rest rho(r) p_i(r) = rho(r + c_i) p_-i(r + c_i) for the
 * Boltzmann weights rho ~ exp(-beta mu^ex) of Eq. 11 (detailed balance);
 * Q = 1 for a neutral tracer. */
int orc_links_charged(int nx, int ny, int nz, const uint8_t* solid, const double* u,
                      double lambda, const double* bmu, double* p)
{
    long N = (long)nx * ny * nz;
    #pragma omp parallel for schedule(static) if (N > 32768)
    for (long n = 0; n < N; ++n) {
        double ux = u ? u[n] : 0.0, uy = u ? u[N + n] : 0.0, uz = u ? u[2 * N + n] : 0.0;
        double uu = ux * ux + uy * uy + uz * uz;
        p[n] = 0.0;
        for (int i = 1; i < Q19; ++i) {
            long m = neighbour(nx, ny, nz, n, i);
            if (solid[n] || solid[m]) { p[(long)i * N + n] = 0.0; continue; }
            double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
            double Q = bmu ? exp(-0.5 * (bmu[m] - bmu[n])) : 1.0;
            p[(long)i * N + n] = W[i] * (0.5 * lambda * Q + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        }
    }
    return 0;
}

int orc_links(int nx, int ny, int nz, const uint8_t* solid, const double* u,
              double lambda, double* p)
{
    return orc_links_charged(nx, ny, nz, solid, u, lambda, NULL, p);
}

/* ---- one propagation step (Eqs. 7, 9, 10) ------------------------------ */
/* X: mobile quantity on all nodes; Xa: adsorbed quantity (meaningful on
 * interface nodes only, zero elsewhere). Writes Xn, Xan. */
int orc_step(int nx, int ny, int nz, const int8_t* cls, const double* p,
             double pa, double pd, const double* X, const double* Xa,
             double* Xn, double* Xan)
{
    long N = (long)nx * ny * nz;
    #pragma omp parallel for schedule(static) if (N > 32768)
    for (long n = 0; n < N; ++n) {
        if (cls[n] == 0) { Xn[n] = 0.0; Xan[n] = 0.0; continue; }
        int iface = (cls[n] == 2);
        /* Eq. 7: arrivals from neighbours + the part that did not move */
        double leave = 0.0;
        for (int i = 1; i < Q19; ++i) leave += p[(long)i * N + n];
        double stay = 1.0 - leave - (iface ? pa : 0.0);
        double v = X[n] * stay;
        for (int i = 1; i < Q19; ++i) {
            long src = neighbour(nx, ny, nz, n, opposite(i)); /* r - c_i */
            v += X[src] * p[(long)i * N + src];
        }
        if (iface) {
            v += pd * Xa[n];                         /* Eq. 10 */
            Xan[n] = pa * X[n] + (1.0 - pd) * Xa[n]; /* Eq. 9 */
        } else {
            Xan[n] = 0.0;
        }
        Xn[n] = v;
    }
    return 0;
}

/* ---- propagate a given (X, Xa) pair T steps in place -------------------- */
/* bmu: beta mu^ex per node for a charged tracer (orc_links_charged), or NULL */
int orc_propagate_charged(int nx, int ny, int nz, const uint8_t* solid, const double* u,
                          double lambda, double pa, double pd, int nbhd, const double* bmu,
                          long T, double* X, double* Xa)
{
    long N = (long)nx * ny * nz;
    int8_t* cls = (int8_t*)malloc(N);
    double* p = (double*)malloc(sizeof(double) * Q19 * N);
    double* Y = (double*)malloc(sizeof(double) * N);
    double* Ya = (double*)malloc(sizeof(double) * N);
    orc_classify(nx, ny, nz, solid, nbhd, cls);
    orc_links_charged(nx, ny, nz, solid, u, lambda, bmu, p);
    for (long t = 0; t < T; ++t) {
        orc_step(nx, ny, nz, cls, p, pa, pd, X, Xa, Y, Ya);
        memcpy(X, Y, sizeof(double) * N);
        memcpy(Xa, Ya, sizeof(double) * N);
    }
    free(cls); free(p); free(Y); free(Ya);
    return 0;
}

int orc_propagate(int nx, int ny, int nz, const uint8_t* solid, const double* u,
                  double lambda, double pa, double pd, int nbhd, long T,
                  double* X, double* Xa)
{
    return orc_propagate_charged(nx, ny, nz, solid, u, lambda, pa, pd, nbhd, NULL, T, X, Xa);
}

/* ---- Uptake out of equilibrium (density propagated; Eqs. 7, 9, 10) ------ */
/* The density as the propagated quantity, from a uniform mobile density
 * 1/N_F on the fluid nodes and no adsorbed density; p_d = 0 (irreversible
 * adsorption) is allowed. Outputs, for t = 0..T: mobile[t] and adsorbed[t],
 * the total mobile and adsorbed densities. Returns -1 when the lattice has no
 * fluid node. */
int orc_uptake(int nx, int ny, int nz, const uint8_t* solid, const double* u,
               double lambda, double pa, double pd, int nbhd, long T,
               double* mobile, double* adsorbed)
{
    long N = (long)nx * ny * nz;
    int8_t* cls = (int8_t*)malloc(N);
    double* p = (double*)malloc(sizeof(double) * Q19 * N);
    double* X = (double*)malloc(sizeof(double) * N);
    double* Xa = (double*)malloc(sizeof(double) * N);
    double* Y = (double*)malloc(sizeof(double) * N);
    double* Ya = (double*)malloc(sizeof(double) * N);
    orc_classify(nx, ny, nz, solid, nbhd, cls);
    orc_links(nx, ny, nz, solid, u, lambda, p);
    long nf = 0;
    for (long n = 0; n < N; ++n) nf += cls[n] != 0;
    if (nf == 0) { free(cls); free(p); free(X); free(Xa); free(Y); free(Ya); return -1; }
    for (long n = 0; n < N; ++n) { X[n] = cls[n] != 0 ? 1.0 / (double)nf : 0.0; Xa[n] = 0.0; }
    for (long t = 0; t <= T; ++t) {
        mobile[t] = nsum(X, N);
        adsorbed[t] = nsum(Xa, N);
        if (t == T) break;
        orc_step(nx, ny, nz, cls, p, pa, pd, X, Xa, Y, Ya);
        memcpy(X, Y, sizeof(double) * N);
        memcpy(Xa, Ya, sizeof(double) * N);
    }
    free(cls); free(p); free(X); free(Xa); free(Y); free(Ya);
    return 0;
}

/* ---- VACF by moment propagation (Eqs. 5, 11, 12) ------------------------ */
/* Outputs, for t = 0..T:
 *   Z[g*(T+1) + t]   velocity autocorrelation in direction g (x, y, z);
 *   mass[0*(T+1)+t]  total mobile density, mass[1*(T+1)+t] total adsorbed;
 *   mom[g*(T+1)+t]   sum of P_g + P_ads,g (t >= 1; mom[.][0] = V_g).
 * V[g] is the mean velocity sum_r rho_0(r) a_g(r).
 * qmask selects the propagated pairs: bit 0 density, bits 1..3 x, y, z
 * moments (unselected outputs are left as zero).
 * Returns 0, or -1 when the lattice has no fluid node or p_d <= 0. */
/* bmu: [N] beta mu^ex(r) (charged tracers: Eq. 8 with the Q_i of
 * orc_links_charged, Eq. 11 with the factor exp(-beta mu^ex)), or NULL. */
int orc_vacf_charged(int nx, int ny, int nz, const uint8_t* solid, const double* u,
                     double lambda, double pa, double pd, int nbhd, const double* bmu,
                     long T, int qmask, double* Z, double* V, double* mass, double* mom)
{
    long N = (long)nx * ny * nz;
    if (pd <= 0.0) return -1;
    int8_t* cls = (int8_t*)malloc(N);
    double* p = (double*)malloc(sizeof(double) * Q19 * N);
    double* tmp = (double*)malloc(sizeof(double) * N);
    orc_classify(nx, ny, nz, solid, nbhd, cls);
    orc_links_charged(nx, ny, nz, solid, u, lambda, bmu, p);

    long nf = 0, ni = 0;
    for (long n = 0; n < N; ++n) { nf += cls[n] != 0; ni += cls[n] == 2; }
    if (nf == 0) { free(cls); free(p); free(tmp); return -1; }
    double K = pa / pd;                      /* Gamma/rho at equilibrium (Eq. 11) */
    /* Eq. 11: weight exp(-beta mu^ex(r)) of a mobile tracer at a fluid node,
     * times (1 + K) on interfacial nodes; Zpart normalises the total to 1 */
    double* rho0 = (double*)malloc(sizeof(double) * N);
    for (long n = 0; n < N; ++n) tmp[n] = cls[n] ? (bmu ? exp(-bmu[n]) : 1.0) : 0.0;
    double sF = nsum(tmp, N);
    for (long n = 0; n < N; ++n) if (cls[n] != 2) tmp[n] = 0.0;
    double sI = nsum(tmp, N);
    double Zpart = sF + sI * K;
    for (long n = 0; n < N; ++n) rho0[n] = cls[n] ? (bmu ? exp(-bmu[n]) : 1.0) / Zpart : 0.0;

    /* a_g(r) = sum_i p_i(r) c_ig: mean displacement of a mobile tracer at r */
    double* a = (double*)calloc(3 * N, sizeof(double));
    for (long n = 0; n < N; ++n)
        for (int i = 1; i < Q19; ++i) {
            a[n] += p[(long)i * N + n] * CX[i];
            a[N + n] += p[(long)i * N + n] * CY[i];
            a[2 * N + n] += p[(long)i * N + n] * CZ[i];
        }

    long T1 = T + 1;
    memset(Z, 0, sizeof(double) * 3 * T1);
    memset(mass, 0, sizeof(double) * 2 * T1);
    memset(mom, 0, sizeof(double) * 3 * T1);

    /* mean velocity and Z(0) = <v_g(0)^2> over the initial weights */
    for (int g = 0; g < 3; ++g) {
        const int* cg = g == 0 ? CX : (g == 1 ? CY : CZ);
        for (long n = 0; n < N; ++n) tmp[n] = cls[n] ? rho0[n] * a[g * N + n] : 0.0;
        V[g] = nsum(tmp, N);
        for (long n = 0; n < N; ++n) {
            double s = 0.0;
            if (cls[n])
                for (int i = 1; i < Q19; ++i) s += p[(long)i * N + n] * cg[i] * cg[i];
            tmp[n] = cls[n] ? rho0[n] * s : 0.0;
        }
        Z[g * T1] = nsum(tmp, N);
        mom[g * T1] = V[g];
    }

    double* X = (double*)malloc(sizeof(double) * N);
    double* Xa = (double*)malloc(sizeof(double) * N);
    double* Y = (double*)malloc(sizeof(double) * N);
    double* Ya = (double*)malloc(sizeof(double) * N);

    for (int q = 0; q < 4; ++q) {
        if (!(qmask & (1 << q))) continue;
        if (q == 0) {
            /* density: the initial weights themselves */
            for (long n = 0; n < N; ++n) {
                X[n] = cls[n] ? rho0[n] : 0.0;
                Xa[n] = cls[n] == 2 ? K * rho0[n] : 0.0;
            }
            mass[0] = nsum(X, N);
            mass[T1] = nsum(Xa, N);
            /* t = 1 */
            orc_step(nx, ny, nz, cls, p, pa, pd, X, Xa, Y, Ya);
            memcpy(X, Y, sizeof(double) * N);
            memcpy(Xa, Ya, sizeof(double) * N);
        } else {
            /* P_g(r, 1): probability to arrive at r after one step, weighted by
             * the displacement of that step; adsorption/desorption moves nothing,
             * so P_ads,g(., 1) = 0. */
            const int* cg = q == 1 ? CX : (q == 2 ? CY : CZ);
            for (long n = 0; n < N; ++n) {
                double v = 0.0;
                if (cls[n])
                    for (int i = 1; i < Q19; ++i) {
                        long src = neighbour(nx, ny, nz, n, opposite(i));
                        if (cls[src]) v += rho0[src] * p[(long)i * N + src] * cg[i];
                    }
                X[n] = v;
                Xa[n] = 0.0;
            }
        }
        for (long t = 1; t <= T; ++t) {
            if (q == 0) {
                mass[t] = nsum(X, N);
                mass[T1 + t] = nsum(Xa, N);
            } else {
                int g = q - 1;
                for (long n = 0; n < N; ++n) tmp[n] = X[n] * a[g * N + n];
                Z[g * T1 + t] = nsum(tmp, N);       /* Eq. 12 */
                double s1 = nsum(X, N), s2 = nsum(Xa, N);
                mom[g * T1 + t] = s1 + s2;
            }
            if (t == T) break;
            orc_step(nx, ny, nz, cls, p, pa, pd, X, Xa, Y, Ya);
            memcpy(X, Y, sizeof(double) * N);
            memcpy(Xa, Ya, sizeof(double) * N);
        }
    }
    free(X); free(Xa); free(Y); free(Ya); free(a); free(rho0);
    free(cls); free(p); free(tmp);
    return 0;
}

int orc_vacf(int nx, int ny, int nz, const uint8_t* solid, const double* u,
             double lambda, double pa, double pd, int nbhd, long T, int qmask,
             double* Z, double* V, double* mass, double* mom)
{
    return orc_vacf_charged(nx, ny, nz, solid, u, lambda, pa, pd, nbhd, NULL, T, qmask,
                            Z, V, mass, mom);
}

/* ---- steady BGK flow (Eq. 6) -------------------------------------------- */
/* D3Q19 BGK, relaxation time tau, Guo forcing with force density rho*g,
 * half-way bounce-back at solid nodes, periodic otherwise. Starts at rest
 * with rho = 1. The velocity u(t) = (sum f c + F/2)/rho is formed after every
 * step; the reported velocity is the average of two consecutive steps,
 * ubar(t) = (u(t) + u(t-1))/2, which removes the step-to-step sign flip of
 * fluid nodes enclosed by solid (bounce-back returns all their momentum).
 * Every `check_every` steps (t >= 2) the change max|ubar(t)-ubar(t-1)| /
 * max|ubar(t)| is compared with tol.
 * Outputs u[3][N] = ubar at the last step and rho[N] (zero on solid nodes).
 * Returns 0 when converged, 1 when max_steps was reached first, -1 when the
 * lattice has no fluid node. */
static void bgk_macro(long N, const uint8_t* solid, const double* f, const double* g,
                      double* rho, double* u)
{
    #pragma omp parallel for schedule(static) if (N > 32768)
    for (long n = 0; n < N; ++n) {
        if (solid[n]) { rho[n] = 0; u[n] = u[N + n] = u[2 * N + n] = 0; continue; }
        double r = 0, jx = 0, jy = 0, jz = 0;
        for (int i = 0; i < Q19; ++i) {
            double fi = f[(long)i * N + n];
            r += fi; jx += fi * CX[i]; jy += fi * CY[i]; jz += fi * CZ[i];
        }
        rho[n] = r;
        u[n] = jx / r + 0.5 * g[0];
        u[N + n] = jy / r + 0.5 * g[1];
        u[2 * N + n] = jz / r + 0.5 * g[2];
    }
}

int orc_bgk(int nx, int ny, int nz, const uint8_t* solid, double tau, const double* g,
            double tol, long max_steps, int check_every, double* u, double* rho,
            long* steps_done, double* resid)
{
    long N = (long)nx * ny * nz;
    long nf = 0;
    for (long n = 0; n < N; ++n) nf += !solid[n];
    if (nf == 0) return -1;
    double* f = (double*)calloc((size_t)Q19 * N, sizeof(double));
    double* fs = (double*)calloc((size_t)Q19 * N, sizeof(double));
    /* velocities of the last three steps: um2 = u(t-2), um1 = u(t-1), uc = u(t) */
    double* um2 = (double*)calloc(3 * (size_t)N, sizeof(double));
    double* um1 = (double*)calloc(3 * (size_t)N, sizeof(double));
    double* uc = (double*)calloc(3 * (size_t)N, sizeof(double));
    for (long n = 0; n < N; ++n)
        if (!solid[n]) for (int i = 0; i < Q19; ++i) f[(long)i * N + n] = W[i];
    bgk_macro(N, solid, f, g, rho, uc);

    int status = 1;
    double res = INFINITY;
    long step = 0;
    while (step < max_steps) {
        /* collision with Guo forcing */
        #pragma omp parallel for schedule(static) if (N > 32768)
        for (long n = 0; n < N; ++n) {
            if (solid[n]) continue;
            double r = 0, jx = 0, jy = 0, jz = 0;
            for (int i = 0; i < Q19; ++i) {
                double fi = f[(long)i * N + n];
                r += fi; jx += fi * CX[i]; jy += fi * CY[i]; jz += fi * CZ[i];
            }
            double Fx = r * g[0], Fy = r * g[1], Fz = r * g[2];
            double ux = (jx + 0.5 * Fx) / r, uy = (jy + 0.5 * Fy) / r, uz = (jz + 0.5 * Fz) / r;
            double uu = ux * ux + uy * uy + uz * uz;
            for (int i = 0; i < Q19; ++i) {
                double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
                double feq = W[i] * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                double cF = CX[i] * Fx + CY[i] * Fy + CZ[i] * Fz;
                double uF = ux * Fx + uy * Fy + uz * Fz;
                double S = (1.0 - 0.5 / tau) * W[i] * (3.0 * (cF - uF) + 9.0 * cu * cF);
                double fi = f[(long)i * N + n];
                fs[(long)i * N + n] = fi - (fi - feq) / tau + S;
            }
        }
        /* streaming (pull) with half-way bounce-back */
        #pragma omp parallel for schedule(static) if (N > 32768)
        for (long n = 0; n < N; ++n) {
            if (solid[n]) continue;
            for (int i = 0; i < Q19; ++i) {
                long src = neighbour(nx, ny, nz, n, opposite(i));
                f[(long)i * N + n] = solid[src] ? fs[(long)opposite(i) * N + n]
                                                : fs[(long)i * N + src];
            }
        }
        ++step;
        double* t = um2; um2 = um1; um1 = uc; uc = t;
        bgk_macro(N, solid, f, g, rho, uc);
        if (check_every > 0 && step >= 2 && step % check_every == 0) {
            double du = 0.0, um = 0.0;
            for (long n = 0; n < 3 * N; ++n) {
                double a = 0.5 * (uc[n] + um1[n]), b = 0.5 * (um1[n] + um2[n]);
                if (fabs(a - b) > du) du = fabs(a - b);
                if (fabs(a) > um) um = fabs(a);
            }
            res = um > 0.0 ? du / um : du;
            if (res < tol) { status = 0; break; }
        }
    }
    for (long n = 0; n < 3 * N; ++n) u[n] = 0.5 * (uc[n] + um1[n]);
    *steps_done = step;
    *resid = res;
    free(f); free(fs); free(um2); free(um1); free(uc);
    return status;
}

/* number of OpenMP threads the oracle runs on */
int orc_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* run the following calls on n OpenMP threads (results do not depend on it) */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#endif
    return orc_threads();
}
