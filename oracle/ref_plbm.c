/*
 * ref_plbm.c -- plain FP64 CPU oracle of the parametric lattice Boltzmann
 * method (Shim, "Parametric Lattice Boltzmann Method", arXiv:1402.5487).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library and must never
 * be linked into it.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * (the oracle/build.py script does exactly this).  IEEE binary64,
 * round-to-nearest-even, no fused multiply-add contraction.
 *
 * What it computes, in the paper's own order:
 *   - c_ij: coefficient of v^(j-1) of the Lagrange interpolating polynomial
 *     through (v_k, delta_ik)  (Sec. 2.1, Eq. rdr and the text after it);
 *   - mu_n: n-th moment of the 1D Maxwell-Boltzmann distribution
 *     (Sec. 2.1; closed forms in Table tableAccuracy);
 *   - r_i = sum_j c_ij mu_(j-1)  (Eq. rdr), tensor product in 2D (Sec. 2.1
 *     last paragraph, Sec. 2.4);
 *   - f_eq_i = rho r_i  (Eq. eqdist);
 *   - one SRT step in push form,
 *       f_i(x + v_i, t + 1) = (1 - omega) f_i(x, t) + omega f_eq_i(x, t)
 *     (Eq. srt), with periodic wrap in 2D and zero-gradient ghost nodes in 1D.
 *
 * Readings of what the paper leaves open (each is listed in the design notes):
 *   - discrete moments: rho = sum f, rho u = sum f v,
 *     d rho theta = sum f |v - u|^2 with one temperature shared by all axes
 *     (consistent with the (d/2) rho theta internal energy of Eq. ns);
 *   - lattice units: dx = dt = 1, integer velocities;
 *   - 2D population index k = i + q1d * j (i: x velocity, j: y velocity);
 *   - the state is the pre-collision f(x, t) at integer t, as in Eq. srt;
 *   - 1D zero-gradient ends: 3 ghost nodes per end receive, every step, the
 *     post-collision populations of the nearest interior node, and streaming
 *     then reads from them.
 *
 * Layout: f[k * ny * nx + y * nx + x] (1D: ny = 1).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_MAXQ 8
#define REF_GHOST 3

/* ------------------------------------------------------------------ */
/* Lagrange coefficients (Sec. 2.1, Eq. rdr)                            */
/* ------------------------------------------------------------------ */

/* c[i*q + j] = coefficient of v^j in L_i(v) = prod_{k != i} (v - v_k)/(v_i - v_k).
 * The polynomial is expanded factor by factor.  Returns 0, or -1 for q out of
 * range or two equal velocities. */
int ref_lagrange_coeffs(int q, const double *v, double *c)
{
    if (q < 1 || q > REF_MAXQ || !v || !c) return -1;
    for (int i = 0; i < q; ++i)
        for (int k = i + 1; k < q; ++k)
            if (v[i] == v[k]) return -1;
    for (int i = 0; i < q; ++i) {
        double poly[REF_MAXQ + 1];
        for (int j = 0; j <= q; ++j) poly[j] = 0.0;
        poly[0] = 1.0;                  /* running product, degree deg */
        int deg = 0;
        double denom = 1.0;
        for (int k = 0; k < q; ++k) {
            if (k == i) continue;
            /* multiply by (v - v_k) */
            double next[REF_MAXQ + 1];
            for (int j = 0; j <= q; ++j) next[j] = 0.0;
            for (int j = 0; j <= deg; ++j) {
                next[j + 1] += poly[j];
                next[j] -= v[k] * poly[j];
            }
            deg += 1;
            for (int j = 0; j <= deg; ++j) poly[j] = next[j];
            denom *= (v[i] - v[k]);
        }
        for (int j = 0; j < q; ++j) c[i * q + j] = poly[j] / denom;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Maxwell-Boltzmann moments (Sec. 2.1; Table tableAccuracy)            */
/* ------------------------------------------------------------------ */

static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

/* mu_n = integral v^n F(v) dv for the 1D Gaussian of mean u and variance
 * theta.  Written as the expectation of (u + sqrt(theta) Z)^n with Z standard
 * normal: mu_n = sum_{even m <= n} C(n, m) u^(n-m) theta^(m/2) (m-1)!!. */
void ref_maxwell_moments(double u, double theta, int nmax, double *mu)
{
    for (int n = 0; n <= nmax; ++n) {
        double s = 0.0;
        for (int m = 0; m <= n; m += 2) {
            double dfact = 1.0;                     /* (m-1)!! */
            for (int t = m - 1; t > 1; t -= 2) dfact *= (double)t;
            s += binom(n, m) * pow(u, (double)(n - m)) * pow(theta, 0.5 * m) * dfact;
        }
        mu[n] = s;
    }
}

/* r_i = sum_j c_ij mu_(j-1)  (Eq. rdr). */
void ref_weights_1d(int q, const double *c, double u, double theta, double *r)
{
    double mu[REF_MAXQ];
    ref_maxwell_moments(u, theta, q - 1, mu);
    for (int i = 0; i < q; ++i) {
        double s = 0.0;
        for (int j = 0; j < q; ++j) s += c[i * q + j] * mu[j];
        r[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Lattice helpers                                                       */
/* ------------------------------------------------------------------ */

static int to_shift(double v, int *s)
{
    double r = floor(v + 0.5);
    if (r != v) return -1;          /* streaming needs on-lattice velocities */
    *s = (int)r;
    return 0;
}

static int nq(int dim, int q1d) { return dim == 1 ? q1d : q1d * q1d; }

/* Moments of one node's populations fk[0..q-1] (reading: discrete moments).
 * flags bit 0 reverses the population summation order (used only to
 * measure the oracle's own rounding-order floor). */
static void node_moments(int dim, int q1d, const double *vel, const double *fk,
                         int flags, double *rho, double *ux, double *uy,
                         double *theta)
{
    int q = nq(dim, q1d);
    double s0 = 0.0, sx = 0.0, sy = 0.0;
    for (int t = 0; t < q; ++t) {
        int k = (flags & 1) ? q - 1 - t : t;
        double vx = vel[k % q1d];
        double vy = dim == 2 ? vel[k / q1d] : 0.0;
        s0 += fk[k];
        sx += fk[k] * vx;
        sy += fk[k] * vy;
    }
    double r = s0, u = sx / r, w = dim == 2 ? sy / r : 0.0;
    double e = 0.0;
    for (int t = 0; t < q; ++t) {
        int k = (flags & 1) ? q - 1 - t : t;
        double cx = vel[k % q1d] - u;
        double cy = dim == 2 ? vel[k / q1d] - w : 0.0;
        e += fk[k] * (cx * cx + cy * cy);
    }
    *rho = r;
    *ux = u;
    *uy = w;
    *theta = e / ((double)dim * r);
}

/* f_eq_k = rho r_i(ux, theta) r_j(uy, theta) with k = i + q1d j (2D) or
 * rho r_k(ux, theta) (1D)  (Eq. eqdist, Eq. rdr, tensor product). */
static void node_equilibrium(int dim, int q1d, const double *c, double rho,
                             double ux, double uy, double theta, double *feq)
{
    double rx[REF_MAXQ], ry[REF_MAXQ];
    ref_weights_1d(q1d, c, ux, theta, rx);
    if (dim == 1) {
        for (int i = 0; i < q1d; ++i) feq[i] = rho * rx[i];
        return;
    }
    ref_weights_1d(q1d, c, uy, theta, ry);
    for (int j = 0; j < q1d; ++j)
        for (int i = 0; i < q1d; ++i)
            feq[i + q1d * j] = rho * rx[i] * ry[j];
}

static int check_args(int dim, int nx, int ny, int q1d, const double *vel,
                      int *shift)
{
    if (dim != 1 && dim != 2) return -1;
    if (q1d < 1 || q1d > REF_MAXQ || nx < 1 || ny < 1) return -1;
    if (dim == 1 && ny != 1) return -1;
    for (int i = 0; i < q1d; ++i) {
        if (to_shift(vel[i], &shift[i])) return -1;
        if (abs(shift[i]) > REF_GHOST) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Public oracle entry points                                           */
/* ------------------------------------------------------------------ */

/* Equilibrium populations of the given fields: f(x, 0) = f_eq(x)
 * (initial populations reading).  uy is ignored in 1D. */
int ref_init(int dim, int nx, int ny, int q1d, const double *vel,
             const double *c, const double *rho, const double *ux,
             const double *uy, const double *theta, double *f)
{
    int shift[REF_MAXQ];
    if (check_args(dim, nx, ny, q1d, vel, shift)) return -1;
    int q = nq(dim, q1d);
    size_t n = (size_t)nx * ny;
    for (size_t p = 0; p < n; ++p) {
        double feq[REF_MAXQ * REF_MAXQ];
        node_equilibrium(dim, q1d, c, rho[p], ux[p], dim == 2 ? uy[p] : 0.0,
                         theta[p], feq);
        for (int k = 0; k < q; ++k) f[k * n + p] = feq[k];
    }
    return 0;
}

/* Advance f (pre-collision state, in place) by nsteps applications of
 * Eq. srt in push form: collide every node into a post-collision array, then
 * move population k of node x to node x + v_k.  bc: 0 periodic, 1
 * zero-gradient ghost ends (1D only). */
int ref_step_theta0(int dim, int nx, int ny, int q1d, const double *vel,
                    const double *c, double omega, int bc, double theta0,
                    double *f, int nsteps, int flags);

int ref_step(int dim, int nx, int ny, int q1d, const double *vel,
             const double *c, double omega, int bc, double *f, int nsteps,
             int flags)
{
    return ref_step_theta0(dim, nx, ny, q1d, vel, c, omega, bc, 0.0, f, nsteps, flags);
}

/* As ref_step; with theta0 > 0 the equilibrium is taken at the fixed
 * reference temperature theta0 instead of the local one: the isothermal
 * models of Sec. 2.3 (Eq. 1d3v, Table 3vel), whose second Maxwell moment is
 * mu_2 = theta0 + u^2. */
int ref_step_theta0(int dim, int nx, int ny, int q1d, const double *vel,
                    const double *c, double omega, int bc, double theta0,
                    double *f, int nsteps, int flags)
{
    int shift[REF_MAXQ];
    if (check_args(dim, nx, ny, q1d, vel, shift)) return -1;
    if (bc == 1 && dim != 1) return -1;
    if (bc != 0 && bc != 1) return -1;
    int q = nq(dim, q1d);
    size_t n = (size_t)nx * ny;
    double *post = malloc(sizeof(double) * q * n);
    /* 1D ghost layout: node x lives at x + REF_GHOST of a padded row. */
    double *pad = bc == 1 ? malloc(sizeof(double) * q * (nx + 2 * REF_GHOST)) : NULL;
    if (!post || (bc == 1 && !pad)) { free(post); free(pad); return -1; }

    for (int step = 0; step < nsteps; ++step) {
        /* collision: post = (1 - omega) f + omega f_eq */
        #pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                size_t p = (size_t)y * nx + x;
                double fk[REF_MAXQ * REF_MAXQ], feq[REF_MAXQ * REF_MAXQ];
                for (int k = 0; k < q; ++k) fk[k] = f[k * n + p];
                double rho, ux, uy, theta;
                node_moments(dim, q1d, vel, fk, flags, &rho, &ux, &uy, &theta);
                if (theta0 > 0.0) theta = theta0;
                node_equilibrium(dim, q1d, c, rho, ux, uy, theta, feq);
                for (int k = 0; k < q; ++k)
                    post[k * n + p] = (1.0 - omega) * fk[k] + omega * feq[k];
            }
        }
        /* streaming: f(x + v_k, t + 1)_k = post(x, t)_k */
        if (bc == 0) {
            #pragma omp parallel for schedule(static)
            for (int y = 0; y < ny; ++y) {
                for (int x = 0; x < nx; ++x) {
                    for (int k = 0; k < q; ++k) {
                        int sx = shift[k % q1d];
                        int sy = dim == 2 ? shift[k / q1d] : 0;
                        int xd = ((x + sx) % nx + nx) % nx;
                        int yd = ((y + sy) % ny + ny) % ny;
                        f[k * n + (size_t)yd * nx + xd] = post[k * n + (size_t)y * nx + x];
                    }
                }
            }
        } else {
            int w = nx + 2 * REF_GHOST;
            for (int k = 0; k < q; ++k) {
                for (int x = 0; x < nx; ++x) pad[k * w + x + REF_GHOST] = post[k * n + x];
                for (int g = 0; g < REF_GHOST; ++g) {
                    pad[k * w + g] = post[k * n + 0];
                    pad[k * w + nx + REF_GHOST + g] = post[k * n + nx - 1];
                }
            }
            for (int k = 0; k < q; ++k) {
                /* every padded node pushes; only arrivals on real nodes are kept */
                for (int xp = 0; xp < w; ++xp) {
                    int xd = xp - REF_GHOST + shift[k];
                    if (xd >= 0 && xd < nx) f[k * n + xd] = pad[k * w + xp];
                }
            }
        }
    }
    free(post);
    free(pad);
    return 0;
}

/* Moments rho, u, theta of every node of the pre-collision state f. */
int ref_moments(int dim, int nx, int ny, int q1d, const double *vel,
                const double *f, double *rho, double *ux, double *uy,
                double *theta, int flags)
{
    int shift[REF_MAXQ];
    if (check_args(dim, nx, ny, q1d, vel, shift)) return -1;
    int q = nq(dim, q1d);
    size_t n = (size_t)nx * ny;
    for (size_t p = 0; p < n; ++p) {
        double fk[REF_MAXQ * REF_MAXQ];
        for (int k = 0; k < q; ++k) fk[k] = f[k * n + p];
        double r, u, w, th;
        node_moments(dim, q1d, vel, fk, flags, &r, &u, &w, &th);
        rho[p] = r;
        ux[p] = u;
        if (uy) uy[p] = w;
        theta[p] = th;
    }
    return 0;
}

/* Neumaier-compensated global sums over all nodes of
 * (sum_k f, sum_k f vx, sum_k f vy, sum_k f |v|^2). */
int ref_sums(int dim, int nx, int ny, int q1d, const double *vel,
             const double *f, double *out)
{
    int shift[REF_MAXQ];
    if (check_args(dim, nx, ny, q1d, vel, shift)) return -1;
    int q = nq(dim, q1d);
    size_t n = (size_t)nx * ny;
    double s[4] = {0, 0, 0, 0}, comp[4] = {0, 0, 0, 0};
    for (size_t p = 0; p < n; ++p) {
        for (int k = 0; k < q; ++k) {
            double vx = vel[k % q1d];
            double vy = dim == 2 ? vel[k / q1d] : 0.0;
            double term[4] = {f[k * n + p], f[k * n + p] * vx,
                              f[k * n + p] * vy, f[k * n + p] * (vx * vx + vy * vy)};
            for (int m = 0; m < 4; ++m) {
                double t = s[m] + term[m];
                if (fabs(s[m]) >= fabs(term[m])) comp[m] += (s[m] - t) + term[m];
                else comp[m] += (term[m] - t) + s[m];
                s[m] = t;
            }
        }
    }
    for (int m = 0; m < 4; ++m) out[m] = s[m] + comp[m];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Three dimensions: the tensor product of the 1D rule over three axes  */
/* (Sec. 2.4: 125 velocities from the five of Eq. 1d5v), periodic.       */
/* Population k = i + q1d j + q1d^2 l moves with (v_i, v_j, v_l).       */
/* Layout f[k * nz * ny * nx + (z * ny + y) * nx + x].                   */
/* ------------------------------------------------------------------ */

#define REF_MAXQ3 (REF_MAXQ * REF_MAXQ * REF_MAXQ)

/* rho, u and theta with 3 rho theta = sum f |v - u|^2 (one temperature). */
static void node_moments3(int q1d, const double *vel, const double *fk, double *rho,
                          double *u, double *theta)
{
    int q = q1d * q1d * q1d;
    double s0 = 0.0, s[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < q; ++k) {
        double v[3] = {vel[k % q1d], vel[(k / q1d) % q1d], vel[k / (q1d * q1d)]};
        s0 += fk[k];
        for (int a = 0; a < 3; ++a) s[a] += fk[k] * v[a];
    }
    for (int a = 0; a < 3; ++a) u[a] = s[a] / s0;
    double e = 0.0;
    for (int k = 0; k < q; ++k) {
        double v[3] = {vel[k % q1d], vel[(k / q1d) % q1d], vel[k / (q1d * q1d)]};
        double c2 = 0.0;
        for (int a = 0; a < 3; ++a) c2 += (v[a] - u[a]) * (v[a] - u[a]);
        e += fk[k] * c2;
    }
    *rho = s0;
    *theta = e / (3.0 * s0);
}

/* f_eq_k = rho r_i(u_x, theta) r_j(u_y, theta) r_l(u_z, theta). */
static void node_equilibrium3(int q1d, const double *c, double rho, const double *u,
                              double theta, double *feq)
{
    double r[3][REF_MAXQ];
    for (int a = 0; a < 3; ++a) ref_weights_1d(q1d, c, u[a], theta, r[a]);
    for (int l = 0; l < q1d; ++l)
        for (int j = 0; j < q1d; ++j)
            for (int i = 0; i < q1d; ++i)
                feq[i + q1d * (j + q1d * l)] = rho * r[0][i] * r[1][j] * r[2][l];
}

static int check_args3(int nx, int ny, int nz, int q1d, const double *vel, int *shift)
{
    if (nx < 1 || ny < 1 || nz < 1 || q1d < 1 || q1d > REF_MAXQ) return -1;
    for (int i = 0; i < q1d; ++i)
        if (to_shift(vel[i], &shift[i])) return -1;
    return 0;
}

int ref_init3(int nx, int ny, int nz, int q1d, const double *vel, const double *c,
              const double *rho, const double *ux, const double *uy, const double *uz,
              const double *theta, double *f)
{
    int shift[REF_MAXQ];
    if (check_args3(nx, ny, nz, q1d, vel, shift)) return -1;
    int q = q1d * q1d * q1d;
    size_t n = (size_t)nx * ny * nz;
    double *feq = malloc(sizeof(double) * q);
    if (!feq) return -1;
    for (size_t p = 0; p < n; ++p) {
        double u[3] = {ux[p], uy[p], uz[p]};
        node_equilibrium3(q1d, c, rho[p], u, theta[p], feq);
        for (int k = 0; k < q; ++k) f[k * n + p] = feq[k];
    }
    free(feq);
    return 0;
}

/* nsteps applications of Eq. srt in push form, periodic in x, y and z. */
int ref_step3(int nx, int ny, int nz, int q1d, const double *vel, const double *c,
              double omega, double *f, int nsteps)
{
    int shift[REF_MAXQ];
    if (check_args3(nx, ny, nz, q1d, vel, shift)) return -1;
    int q = q1d * q1d * q1d;
    size_t n = (size_t)nx * ny * nz;
    double *post = malloc(sizeof(double) * q * n);
    if (!post) return -1;
    for (int step = 0; step < nsteps; ++step) {
        #pragma omp parallel for schedule(static)
        for (long long pp = 0; pp < (long long)n; ++pp) {
            size_t p = (size_t)pp;
            double fk[REF_MAXQ3], feq[REF_MAXQ3];
            for (int k = 0; k < q; ++k) fk[k] = f[k * n + p];
            double rho, u[3], theta;
            node_moments3(q1d, vel, fk, &rho, u, &theta);
            node_equilibrium3(q1d, c, rho, u, theta, feq);
            for (int k = 0; k < q; ++k) post[k * n + p] = (1.0 - omega) * fk[k] + omega * feq[k];
        }
        #pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    for (int k = 0; k < q; ++k) {
                        int xd = ((x + shift[k % q1d]) % nx + nx) % nx;
                        int yd = ((y + shift[(k / q1d) % q1d]) % ny + ny) % ny;
                        int zd = ((z + shift[k / (q1d * q1d)]) % nz + nz) % nz;
                        f[k * n + ((size_t)zd * ny + yd) * nx + xd] =
                            post[k * n + ((size_t)z * ny + y) * nx + x];
                    }
    }
    free(post);
    return 0;
}

int ref_moments3(int nx, int ny, int nz, int q1d, const double *vel, const double *f,
                 double *rho, double *ux, double *uy, double *uz, double *theta)
{
    int shift[REF_MAXQ];
    if (check_args3(nx, ny, nz, q1d, vel, shift)) return -1;
    int q = q1d * q1d * q1d;
    size_t n = (size_t)nx * ny * nz;
    for (size_t p = 0; p < n; ++p) {
        double fk[REF_MAXQ3], r, u[3], th;
        for (int k = 0; k < q; ++k) fk[k] = f[k * n + p];
        node_moments3(q1d, vel, fk, &r, u, &th);
        rho[p] = r;
        ux[p] = u[0];
        uy[p] = u[1];
        uz[p] = u[2];
        theta[p] = th;
    }
    return 0;
}

/* Compensated (sum f, sum f v_x, sum f v_y, sum f v_z, sum f |v|^2). */
int ref_sums3(int nx, int ny, int nz, int q1d, const double *vel, const double *f, double *out)
{
    int shift[REF_MAXQ];
    if (check_args3(nx, ny, nz, q1d, vel, shift)) return -1;
    int q = q1d * q1d * q1d;
    size_t n = (size_t)nx * ny * nz;
    double s[5] = {0, 0, 0, 0, 0}, comp[5] = {0, 0, 0, 0, 0};
    for (size_t p = 0; p < n; ++p) {
        for (int k = 0; k < q; ++k) {
            double v[3] = {vel[k % q1d], vel[(k / q1d) % q1d], vel[k / (q1d * q1d)]};
            double g = f[k * n + p];
            double term[5] = {g, g * v[0], g * v[1], g * v[2],
                              g * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2])};
            for (int m = 0; m < 5; ++m) {
                double t = s[m] + term[m];
                if (fabs(s[m]) >= fabs(term[m])) comp[m] += (s[m] - t) + term[m];
                else comp[m] += (term[m] - t) + s[m];
                s[m] = t;
            }
        }
    }
    for (int m = 0; m < 5; ++m) out[m] = s[m] + comp[m];
    return 0;
}

/* Threads the parallel loops above run on (1 without OpenMP). */
int ref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the threads of the parallel loops (n >= 1); the results do not depend
 * on it (each node and each push is computed by exactly one thread). */
void ref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
