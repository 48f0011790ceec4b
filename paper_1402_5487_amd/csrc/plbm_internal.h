// Internal declarations shared by the host and device translation units of
// libplbm (not part of the public ABI).
#pragma once
#include "plbm.h"

namespace plbm {
int nq(const plbm_desc *d);
int validate(const plbm_desc *d);

// Records a failed HIP call for plbm_last_hip_error (plbm_kernels.hip).
void note_hip_error(const char *what, int code);

// The isothermal three-velocity family (q1d = 3: D1Q3 and its tensor product
// D2Q9), plbm_q3.hip; the public plbm_init / plbm_step / plbm_moments forward
// to these.
int q3_init(const plbm_desc *d, const double *rho, const double *ux, const double *uy, void *f,
            void *stream);
int q3_step(const plbm_desc *d, void *f_a, void *f_b, int nsteps, double *sums, void *stream);
int q3_moments(const plbm_desc *d, const void *f, double *rho, double *ux, double *uy,
               double *theta, double *sums, void *stream);

// General on-lattice velocity sets (plbm_gen.hip): every dim-1/2 descriptor
// with q1d = 3..7 that the symmetric kernels do not take.  The public
// plbm_init / plbm_step / plbm_moments forward here when gen_handles is true.
bool gen_handles(const plbm_desc *d);
int gen_init(const plbm_desc *d, const double *rho, const double *ux, const double *uy,
             const double *theta, void *f, void *stream);
int gen_step(const plbm_desc *d, void *f_a, void *f_b, int nsteps, double *sums, void *stream);
int gen_moments(const plbm_desc *d, const void *f, double *rho, double *ux, double *uy,
                double *theta, double *sums, void *stream);

// The D3Q125 step (plbm_q125.hip); plbm_step forwards dim-3 descriptors here.
int q125_step(const plbm_desc *d, void *f_a, void *f_b, int nsteps, double *sums, void *stream);
} // namespace plbm
