// Host side of libplbm: the coefficient table, descriptor defaults and
// validation, status strings.  No device code lives here.
#include "plbm.h"
#include "plbm_internal.h"

#include <cmath>
#include <cstring>

extern "C" int plbm_coeffs(int q, const double *v, double *c)
{
    if (q < 1 || q > PLBM_MAX_Q1D || !v || !c) return PLBM_EINVAL;
    for (int i = 0; i < q; ++i)
        if (!std::isfinite(v[i])) return PLBM_EINVAL;
    for (int i = 0; i < q; ++i)
        for (int k = i + 1; k < q; ++k)
            if (v[i] == v[k]) return PLBM_ESINGULAR;

    // Appendix: R = V^-1 M with V[n][k] = v_k^n.  Row i of V^-1 holds the
    // coefficients c_i of r_i = sum_n c_in mu_n, so solve V X = I by Gaussian
    // elimination with partial pivoting on the augmented matrix [V | I].
    double a[PLBM_MAX_Q1D][2 * PLBM_MAX_Q1D];
    for (int n = 0; n < q; ++n) {
        for (int k = 0; k < q; ++k) {
            double p = 1.0;
            for (int e = 0; e < n; ++e) p *= v[k];
            a[n][k] = p;
        }
        for (int m = 0; m < q; ++m) a[n][q + m] = (n == m) ? 1.0 : 0.0;
    }
    for (int col = 0; col < q; ++col) {
        int piv = col;
        for (int r = col + 1; r < q; ++r)
            if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return PLBM_ESINGULAR;
        if (piv != col)
            for (int m = 0; m < 2 * q; ++m) std::swap(a[piv][m], a[col][m]);
        for (int r = col + 1; r < q; ++r) {
            double f = a[r][col] / a[col][col];
            if (f == 0.0) continue;
            for (int m = col; m < 2 * q; ++m) a[r][m] -= f * a[col][m];
        }
    }
    // back substitution: X = V^-1 (row n of X is column block of a)
    double x[PLBM_MAX_Q1D][PLBM_MAX_Q1D];
    for (int m = 0; m < q; ++m) {
        for (int r = q - 1; r >= 0; --r) {
            double s = a[r][q + m];
            for (int t = r + 1; t < q; ++t) s -= a[r][t] * x[t][m];
            x[r][m] = s / a[r][r];
        }
    }
    // X[k][n]: V X = I means sum_k v_k^n X[k][n'] = delta; row k of X is
    // r_k's coefficient vector: r_k = sum_n X[k][n] mu_n.
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) c[i * q + j] = x[i][j];

    // residual of the Lagrange property sum_j c_ij v_k^j = delta_ik
    double worst = 0.0, scale = 0.0;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) scale = std::fmax(scale, std::fabs(c[i * q + j]));
    for (int i = 0; i < q; ++i)
        for (int k = 0; k < q; ++k) {
            double s = 0.0, p = 1.0;
            for (int j = 0; j < q; ++j) { s += c[i * q + j] * p; p *= v[k]; }
            worst = std::fmax(worst, std::fabs(s - (i == k ? 1.0 : 0.0)));
        }
    if (!(worst <= 1e-9 * std::fmax(1.0, scale))) return PLBM_ESINGULAR;
    return PLBM_OK;
}

extern "C" int plbm_desc_default(plbm_desc *d, int dim, int nx, int ny,
                                 double omega, int storage)
{
    if (!d) return PLBM_EINVAL;
    std::memset(d, 0, sizeof(*d));
    d->dim = dim;
    d->nx = nx;
    d->ny = dim == 1 ? 1 : ny;
    d->nz = dim == 3 ? ny : 1;
    d->q1d = 5;
    d->bc = dim == 1 ? PLBM_BC_ZEROGRAD : PLBM_BC_PERIODIC;
    d->storage = storage;
    const double vel[5] = {0.0, 1.0, -1.0, 3.0, -3.0};
    for (int i = 0; i < 5; ++i) d->v[i] = vel[i];
    int rc = plbm_coeffs(5, d->v, d->c);
    if (rc != PLBM_OK) return rc;
    d->omega = omega;
    d->rho0 = 1.0;
    d->theta0 = 1.0 / 3.0;
    for (int k = 0; k < PLBM_MAX_Q1D * PLBM_MAX_Q1D; ++k) d->scale[k] = 1.0f;
    return plbm::validate(d);
}

extern "C" size_t plbm_elem_bytes(const plbm_desc *d)
{
    if (!d || plbm::validate(d) != PLBM_OK) return 0;
    switch (d->storage) {
    case PLBM_F64: return 8;
    case PLBM_F32: return 4;
    default: return 2;
    }
}

extern "C" size_t plbm_buffer_elems(const plbm_desc *d)
{
    if (!d || plbm::validate(d) != PLBM_OK) return 0;
    size_t q = (size_t)plbm::nq(d);
    if (d->dim == 1) return q * (size_t)(d->nx + 2 * PLBM_GHOST);
    if (d->dim == 3) return q * (size_t)d->nx * (size_t)d->ny * (size_t)d->nz;
    return q * (size_t)d->nx * (size_t)d->ny;
}

extern "C" const char *plbm_strerror(int status)
{
    switch (status) {
    case PLBM_OK: return "ok";
    case PLBM_EINVAL: return "invalid argument";
    case PLBM_ESINGULAR: return "velocity set is singular (duplicate velocities)";
    case PLBM_EHIP: return "HIP runtime error";
    case PLBM_ENONFINITE: return "non-finite invariants";
    case PLBM_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
    }
}

namespace plbm {

int nq(const plbm_desc *d)
{
    return d->dim == 1 ? d->q1d : (d->dim == 2 ? d->q1d * d->q1d : d->q1d * d->q1d * d->q1d);
}

int validate(const plbm_desc *d)
{
    if (!d) return PLBM_EINVAL;
    if (d->dim < 1 || d->dim > 3) return PLBM_EINVAL;
    if (d->dim < 3 && d->nz > 1) return PLBM_EINVAL;
    if (d->dim == 3 && d->nz < 1) return PLBM_EINVAL;
    if (d->q1d < 1 || d->q1d > PLBM_MAX_Q1D) return PLBM_EINVAL;
    if (d->nx < 1 || d->ny < 1) return PLBM_EINVAL;
    if (d->dim == 1 && d->ny != 1) return PLBM_EINVAL;
    if (!(d->omega > 0.0 && d->omega < 2.0)) return PLBM_EINVAL;
    if (d->storage < PLBM_F64 || d->storage > PLBM_BF16DEV) return PLBM_EINVAL;
    if (d->rounding != PLBM_ROUND_NEAREST && d->rounding != PLBM_ROUND_STOCHASTIC) return PLBM_EINVAL;
    if (d->rounding == PLBM_ROUND_STOCHASTIC && d->storage < PLBM_F16DEV) return PLBM_EINVAL;
    if (d->dim == 1 && d->bc != PLBM_BC_ZEROGRAD) return PLBM_EINVAL;
    if (d->dim >= 2 && d->bc != PLBM_BC_PERIODIC) return PLBM_EINVAL;
    // the kernels address a lattice row's population rows with 32-bit byte offsets
    if (d->dim >= 2 && d->nx > (1 << 26)) return PLBM_EINVAL;
    // node counts (and 1D grid sizes) stay within 2^30
    const double nodes = (double)d->nx * (double)d->ny * (double)(d->dim == 3 ? d->nz : 1);
    if (nodes > (double)(1u << 30)) return PLBM_EINVAL;
    int maxs = 0;
    for (int i = 0; i < d->q1d; ++i) {
        double r = std::floor(d->v[i] + 0.5);
        if (r != d->v[i] || std::fabs(r) > PLBM_GHOST) return PLBM_EINVAL;
        maxs = std::max(maxs, (int)std::fabs(r));
        for (int k = i + 1; k < d->q1d; ++k)
            if (d->v[i] == d->v[k]) return PLBM_ESINGULAR;
    }
    for (int i = 0; i < d->q1d * d->q1d; ++i)
        if (!std::isfinite(d->c[i])) return PLBM_EINVAL;
    if (d->dim == 2) {
        // periodic wrap with one correction needs n >= largest shift
        if (d->nx < maxs || d->ny < maxs) return PLBM_EINVAL;
        if ((double)d->nx * (double)d->ny > (double)(1u << 30)) return PLBM_EINVAL;
    }
    if (d->dim == 3) {
        if (d->nx < maxs || d->ny < maxs || d->nz < maxs) return PLBM_EINVAL;
        if ((double)d->nx * (double)d->ny * (double)d->nz > (double)(1u << 30)) return PLBM_EINVAL;
        if (d->storage >= PLBM_F16DEV) return PLBM_EUNSUPPORTED;
    }
    if (d->storage >= PLBM_F16DEV) {
        if (!(d->rho0 > 0.0) || !(d->theta0 > 0.0)) return PLBM_EINVAL;
        for (int k = 0; k < nq(d); ++k)
            if (!(d->scale[k] > 0.0f) || !std::isfinite(d->scale[k])) return PLBM_EINVAL;
    }
    return PLBM_OK;
}

} // namespace plbm
