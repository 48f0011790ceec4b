/* Host AddressSanitizer / UBSan run of the FP64 oracle: every entry point on
 * small lattices of several shapes, velocity sets and boundary modes,
 * including one-node and narrowest-periodic cases.  Exit status 0 means every
 * call returned 0 and the sanitizers found nothing. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int ref_lagrange_coeffs(int q, const double *v, double *c);
void ref_maxwell_moments(double u, double theta, int nmax, double *mu);
void ref_weights_1d(int q, const double *c, double u, double theta, double *r);
int ref_init(int dim, int nx, int ny, int q1d, const double *vel, const double *c, const double *rho,
             const double *ux, const double *uy, const double *theta, double *f);
int ref_step_theta0(int dim, int nx, int ny, int q1d, const double *vel, const double *c, double omega,
                    int bc, double theta0, double *f, int nsteps, int flags);
int ref_moments(int dim, int nx, int ny, int q1d, const double *vel, const double *f, double *rho, double *ux,
                double *uy, double *theta, int flags);
int ref_sums(int dim, int nx, int ny, int q1d, const double *vel, const double *f, double *out);
int ref_init3(int nx, int ny, int nz, int q1d, const double *vel, const double *c, const double *rho,
              const double *ux, const double *uy, const double *uz, const double *theta, double *f);
int ref_step3(int nx, int ny, int nz, int q1d, const double *vel, const double *c, double omega, double *f,
              int nsteps);
int ref_moments3(int nx, int ny, int nz, int q1d, const double *vel, const double *f, double *rho, double *ux,
                 double *uy, double *uz, double *theta);
int ref_sums3(int nx, int ny, int nz, int q1d, const double *vel, const double *f, double *out);

static int fails = 0;
#define CHECK(x) do { if ((x) != 0) { fprintf(stderr, "call failed: %s line %d\n", #x, __LINE__); ++fails; } } while (0)

static double frand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

static void run2(int dim, int nx, int ny, const double *v, int q1d, int bc, double theta0, unsigned seed)
{
    double c[64];
    CHECK(ref_lagrange_coeffs(q1d, v, c));
    const int q = dim == 1 ? q1d : q1d * q1d;
    const size_t n = (size_t)nx * ny;
    double *rho = malloc(n * sizeof(double)), *ux = malloc(n * sizeof(double));
    double *uy = malloc(n * sizeof(double)), *th = malloc(n * sizeof(double));
    double *f = malloc(n * q * sizeof(double)), *m = malloc(4 * n * sizeof(double));
    for (size_t p = 0; p < n; ++p) {
        rho[p] = 1.0 + 0.02 * (frand(&seed) - 0.5);
        ux[p] = 0.04 * (frand(&seed) - 0.5);
        uy[p] = 0.04 * (frand(&seed) - 0.5);
        th[p] = (theta0 > 0 ? theta0 : 0.5) * (1.0 + 0.02 * (frand(&seed) - 0.5));
    }
    CHECK(ref_init(dim, nx, ny, q1d, v, c, rho, ux, uy, th, f));
    CHECK(ref_step_theta0(dim, nx, ny, q1d, v, c, 1.3, bc, theta0, f, 3, 0));
    CHECK(ref_moments(dim, nx, ny, q1d, v, f, m, m + n, m + 2 * n, m + 3 * n, 0));
    double s[4];
    CHECK(ref_sums(dim, nx, ny, q1d, v, f, s));
    if (!isfinite(s[0])) ++fails;
    free(rho); free(ux); free(uy); free(th); free(f); free(m);
}

static void run3(int nx, int ny, int nz, unsigned seed)
{
    const double v[5] = {0, 1, -1, 3, -3};
    double c[25];
    CHECK(ref_lagrange_coeffs(5, v, c));
    const size_t n = (size_t)nx * ny * nz;
    double *a = malloc(5 * n * sizeof(double)), *f = malloc(125 * n * sizeof(double));
    for (size_t p = 0; p < 5 * n; ++p) a[p] = (p < n) ? 1.0 + 0.01 * frand(&seed) : (p >= 4 * n ? 0.5 : 0.02 * (frand(&seed) - 0.5));
    CHECK(ref_init3(nx, ny, nz, 5, v, c, a, a + n, a + 2 * n, a + 3 * n, a + 4 * n, f));
    CHECK(ref_step3(nx, ny, nz, 5, v, c, 1.4, f, 2));
    CHECK(ref_moments3(nx, ny, nz, 5, v, f, a, a + n, a + 2 * n, a + 3 * n, a + 4 * n));
    double s[5];
    CHECK(ref_sums3(nx, ny, nz, 5, v, f, s));
    free(a); free(f);
}

int main(void)
{
    const double v5[5] = {0, 1, -1, 3, -3}, v3[3] = {0, 1, -1}, v4[4] = {1, -1, 3, -3};
    const double v7[7] = {0, 1, -1, 2, -2, 3, -3}, va[3] = {0, 1, -2};
    double mu[9], r[8], c[64];
    ref_maxwell_moments(0.1, 0.4, 8, mu);
    CHECK(ref_lagrange_coeffs(7, v7, c));
    ref_weights_1d(7, c, 0.05, 0.9, r);
    run2(2, 3, 3, v5, 5, 0, 0.0, 1);
    run2(2, 7, 5, v5, 5, 0, 0.0, 2);
    run2(2, 1, 1, v5, 5, 0, 0.0, 3);
    run2(1, 1, 1, v5, 5, 1, 0.0, 4);
    run2(1, 9, 1, v5, 5, 1, 0.0, 5);
    run2(1, 12, 1, v5, 5, 0, 0.0, 6);
    run2(2, 4, 6, v3, 3, 0, 0.25, 7);
    run2(1, 5, 1, v3, 3, 1, 0.25, 8);
    run2(2, 5, 4, v4, 4, 0, 4.0 / 3.0, 9);
    run2(2, 6, 6, v7, 7, 0, 0.0, 10);
    run2(1, 4, 1, va, 3, 1, 0.25, 11);
    run3(3, 3, 3, 12);
    run3(5, 4, 3, 13);
    run3(1, 1, 1, 14);
    if (fails) fprintf(stderr, "%d failures\n", fails);
    return fails ? 1 : 0;
}
