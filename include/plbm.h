/*
 * plbm.h -- C ABI of libplbm, the MI355X (gfx950) implementation of the
 * fused collide-and-stream update of the parametric lattice Boltzmann method
 * (J. W. Shim, "Parametric Lattice Boltzmann Method", arXiv:1402.5487).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns a plbm_status; it never aborts and never throws
 *    across the ABI.  Arguments are validated on the host before any launch;
 *    an invalid call launches nothing.
 *  - "device pointer" arguments are HIP device allocations owned by the caller
 *    (typically torch tensors); the library never frees them and keeps no
 *    reference after the call returns.  "host pointer" arguments are ordinary
 *    host memory owned by the caller.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are asynchronous on that stream unless stated otherwise; a kernel fault
 *    is reported as PLBM_EHIP by the first later call that synchronises.
 *  - Velocities are in lattice units (dx = dt = 1) and must be integers for
 *    streaming.  The 1D rule uses q1d velocities in the paper's order
 *    (v_1 = 0, v_2,3 = +-a, v_4,5 = +-b, Sec. 2.4); the 2D model is the tensor
 *    product, population k = i + q1d * j moving with (v_i, v_j).  The device
 *    kernels take 3 to 7 distinct integer velocities with |v| <= 3 (which
 *    model a set selects: see plbm_desc); plbm_coeffs alone takes any real
 *    set of up to PLBM_MAX_Q1D velocities.
 *
 * Population layout in HBM (structure of arrays at row granularity)
 * ----------------------------------------------------------------------
 *  - dim 2: element (k, y, x) at (y * q + k) * nx + x with q = q1d^2: lattice
 *    row y stores the q population rows of nx nodes one after another, so a
 *    wave reads and writes contiguous runs of each population, and the rows
 *    a step touches for one output row are seven contiguous blocks.  Periodic
 *    in x and y.
 *  - dim 1: element (k, x) at k * (nx + 6) + x + 3: three ghost nodes on each
 *    side of the nx real nodes (zero-gradient ends, see plbm_step).
 *  - dim 3: element (k, z, y, x) at ((z * ny + y) * q + k) * nx + x with
 *    q = q1d^3: each lattice row (y, z) stores its q population rows one after
 *    another.  Periodic in x, y and z.
 *  - element type: double (PLBM_F64), float (PLBM_F32), or 16-bit deviations
 *    (PLBM_F16DEV: IEEE half, PLBM_BF16DEV: bfloat16) decoded as
 *    f_k = rho0 w_k + scale[k] * h_k with w_k = r_i(0, theta0) r_j(0, theta0).
 *    Scales are powers of two and equal within a symmetry class (the pair of
 *    speed magnitudes |v_i|, |v_j|); plbm_dev_scales chooses them.
 *  - A population buffer holds the POST-collision populations of the last
 *    completed step; the pre-collision state of Eq. srt at node x is obtained
 *    by pulling, f_k(x) = buffer_k(x - v_k).  plbm_init writes the buffer
 *    whose pull is the initial equilibrium.
 */
#ifndef PLBM_H
#define PLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum plbm_status {
    PLBM_OK = 0,
    PLBM_EINVAL = -1,        /* bad argument (range, null pointer, size) */
    PLBM_ESINGULAR = -2,     /* velocity set has duplicates / singular V */
    PLBM_EHIP = -3,          /* a HIP runtime call failed */
    PLBM_ENONFINITE = -4,    /* requested invariants are NaN or Inf */
    PLBM_EUNSUPPORTED = -5   /* valid but not implemented combination */
} plbm_status;

typedef enum plbm_bc {
    PLBM_BC_PERIODIC = 0,    /* dims 2 and 3 */
    PLBM_BC_ZEROGRAD = 1     /* dim 1: ghosts copy the edge node */
} plbm_bc;

typedef enum plbm_storage {
    PLBM_F64 = 0,
    PLBM_F32 = 1,
    PLBM_F16DEV = 2,
    PLBM_BF16DEV = 3
} plbm_storage;

/* Rounding of the stored 16-bit deviations h = (f - rho0 w) / scale.
 * NEAREST: round to nearest even.  STOCHASTIC: one of the two neighbouring
 * 16-bit values, the farther one with probability equal to the distance to
 * the nearer one in units of their spacing, so the stored value is unbiased;
 * the random bits hash the node, the population and the value, so results
 * stay deterministic and independent of how steps are split into calls.
 * Round to nearest loses every per-step change below half an ulp of the
 * deviation, which slows or stops slow viscous and thermal decay. */
typedef enum {
    PLBM_ROUND_NEAREST = 0,
    PLBM_ROUND_STOCHASTIC = 1
} plbm_rounding;

#define PLBM_MAX_Q1D 8
#define PLBM_GHOST 3          /* largest |velocity| the kernels stream */

/* Plain data describing one lattice.  Copied by value into every launch.
 * dim 3 is the tensor product of the 1D rule over three axes (Sec. 2.4:
 * D3Q125 from D1Q5), periodic, FP64 or FP32 storage; population
 * k = i + q1d j + q1d^2 l moves with (v_i, v_j, v_l).
 *
 * Which model a descriptor selects (dims 1 and 2):
 *  - q1d 5, v = (0, a, -a, b, -b): the thermal five-velocity model
 *    (Eq. 1d5v), every storage form;
 *  - q1d 3, v = (0, a, -a): the isothermal three-velocity family (Eq. 1d3v)
 *    at theta0, FP64 or FP32;
 *  - any other set of 3 to 7 distinct integer velocities (asymmetric sets,
 *    D1Q4, 6 or 7 velocities; Sec. 2.2): the general kernels, FP64 or FP32,
 *    with c checked against v (sum_n c_in v_k^n = delta_ik).  Up to four
 *    velocities the model is isothermal at theta0 (mu_n at the fixed
 *    temperature), from five on thermal (the local temperature). */
typedef struct plbm_desc {
    int32_t dim;              /* 1, 2 or 3 */
    int32_t nx, ny;           /* ny = 1 when dim = 1 */
    int32_t q1d;              /* velocities per axis (5 for D1Q5 / D2Q25) */
    int32_t bc;               /* plbm_bc */
    int32_t storage;          /* plbm_storage */
    double v[PLBM_MAX_Q1D];   /* 1D velocities, integers, |v| <= PLBM_GHOST */
    double c[PLBM_MAX_Q1D * PLBM_MAX_Q1D];  /* c[i*q1d + j], see plbm_coeffs */
    double omega;             /* relaxation constant, 0 < omega < 2 */
    double rho0, theta0;      /* deviation base state (16-bit storage); theta0
                                 is also the temperature of the isothermal models */
    float scale[PLBM_MAX_Q1D * PLBM_MAX_Q1D]; /* per-plane scale (16-bit) */
    int32_t nz;               /* dim 3: lattice depth; dims 1 and 2: 1 (0 is read as 1) */
    int32_t rounding;         /* plbm_rounding of the 16-bit deviations (0 for the
                                 other storage forms) */
} plbm_desc;

/*
 * plbm_coeffs -- coefficient table of the parametric equilibrium.
 * Sec. 2.1, Eq. rdr: r_i = sum_j c_ij mu_(j-1), with c_ij the coefficient of
 * degree j-1 of the Lagrange polynomial through (v_k, delta_ik); the Appendix
 * writes the same table as R = V^-1 M with V[n][k] = v_k^n.  Computed here by
 * Gaussian elimination with partial pivoting in FP64 on the host, followed by
 * a residual check of c V = I.
 *   q : number of velocities, 1..PLBM_MAX_Q1D
 *   v : host pointer, q velocities (any real values, pairwise distinct)
 *   c : host pointer, q*q doubles written row-major, c[i*q + j] = c_(i+1)(j+1)
 * Errors: PLBM_EINVAL (q out of range, null pointer, non-finite v),
 * PLBM_ESINGULAR (two equal velocities or a residual above 1e-9).
 * Host only, synchronous, thread-safe.
 */
int plbm_coeffs(int q, const double *v, double *c);

/*
 * plbm_desc_default -- fill *d for the D1Q5 {0, +-1, +-3} model (dim 1) or its
 * D2Q25 (dim 2) or D3Q125 (dim 3, depth nz = ny; set d->nz for another
 * depth) tensor product: velocities, c from plbm_coeffs, omega, boundary
 * (zero-gradient in 1D, periodic otherwise), storage, rho0 = 1,
 * theta0 = 1/3 and unit scales.  Host only.  PLBM_EINVAL on bad sizes.
 */
int plbm_desc_default(plbm_desc *d, int dim, int nx, int ny, double omega,
                      int storage);

/* Number of stored elements of one population buffer (see layout above),
 * or 0 if the descriptor is invalid.  Host only. */
size_t plbm_buffer_elems(const plbm_desc *d);

/* Bytes per stored population (8, 4 or 2), or 0 if invalid.  Host only. */
size_t plbm_elem_bytes(const plbm_desc *d);

/*
 * plbm_init -- populations of the initial state f(x, 0) = f_eq(x)
 * (Eq. eqdist with the tensor-product rule of Eq. rdr), written so that the
 * first pull of plbm_step or plbm_moments yields exactly that equilibrium.
 *   rho, ux, uy, theta : device pointers to nx*ny doubles (row-major, x
 *                        fastest); uy is ignored (may be NULL) when dim = 1.
 *   f                  : device pointer to plbm_buffer_elems(d) elements.
 * dim 3 descriptors take plbm_init3 instead (PLBM_EINVAL here).
 * Asynchronous on `stream`.  Errors: PLBM_EINVAL, PLBM_EUNSUPPORTED, PLBM_EHIP.
 */
int plbm_init(const plbm_desc *d, const double *rho, const double *ux,
              const double *uy, const double *theta, void *f, void *stream);

/*
 * plbm_init3 -- plbm_init for the D3Q125 model (dim 3, Sec. 2.4: the 1D
 * rule of Eq. rdr along each of three axes, f_eq_k = rho r_i(u_x) r_j(u_y)
 * r_l(u_z) for k = i + q1d j + q1d^2 l, one temperature theta).
 *   rho, ux, uy, uz, theta : device pointers to nx*ny*nz doubles, element
 *                            (z * ny + y) * nx + x.  All required.
 *   f                      : device pointer to plbm_buffer_elems(d) elements.
 * FP64 or FP32 storage, the symmetric five-velocity set.  Asynchronous on
 * `stream`.  Errors: PLBM_EINVAL (dim != 3, null pointers, bad descriptor),
 * PLBM_EUNSUPPORTED (16-bit storage or a non-symmetric set), PLBM_EHIP.
 */
int plbm_init3(const plbm_desc *d, const double *rho, const double *ux,
               const double *uy, const double *uz, const double *theta, void *f,
               void *stream);

/*
 * plbm_step -- nsteps applications of the SRT update, Eq. srt:
 *   f_i(x + v_i, t + 1) = (1 - omega) f_i(x, t) + omega f_eq_i(x, t),
 * each one a single fused pull kernel: gather f_k(x) = src_k(x - v_k), take
 * rho, u, theta, the Maxwell moments mu_0..mu_(q1d-1) per axis, the rule
 * r = C mu per axis, f_eq = rho r^x r^y, relax, and write dst at x.
 *   f_a, f_b : device pointers, two distinct buffers of plbm_buffer_elems(d)
 *              elements.  Step s reads f_a and writes f_b when s is even,
 *              the reverse when odd: the result is in f_a when nsteps is
 *              even and in f_b when it is odd.  nsteps >= 0.
 *   sums     : NULL, or a host pointer to 4 doubles (5 when dim = 3)
 *              receiving, after the last step, the FP64 sums over all nodes
 *              of the post-collision populations it wrote: sum f, sum f v_x,
 *              sum f v_y, sum f |v|^2 (mass, momenta, twice the energy) and,
 *              in 3D, sum f v_z as the fifth.  With periodic boundaries these
 *              are the invariants of the state after the call.  Asking for
 *              sums makes the call synchronise `stream`.
 * Boundaries: dims 2 and 3 periodic; dim 1 zero-gradient, i.e. each step the
 * three ghost nodes at each end receive the post-collision populations of
 * the nearest real node before streaming.  In 3D f_eq = rho r^x r^y r^z and
 * 3 rho theta = sum f |v - u|^2.
 * Without sums the call only launches kernels on `stream` (no allocation,
 * copy or synchronisation), so it can be recorded into a HIP graph.
 * Errors: PLBM_EINVAL (aliasing or null buffers, bad descriptor),
 * PLBM_EUNSUPPORTED (16-bit storage in 1D or 3D, a velocity set the
 * kernels do not take), PLBM_ENONFINITE (sums requested and not finite),
 * PLBM_EHIP.
 */
int plbm_step(const plbm_desc *d, void *f_a, void *f_b, int nsteps,
              double *sums, void *stream);

/*
 * plbm_step_fields -- plbm_step (without sums) whose first step also writes
 * the fields (rho, u_x, u_y, theta) of the state it reads, i.e. of the
 * state at the start of the call (Sec. 2: rho = sum f, rho u = sum f v,
 * 2 rho theta = sum f |v - u|^2 of the pulled populations, as
 * plbm_moments reports them).  They are the moments the collision itself
 * uses, so they cost no extra read: with FP64 storage they equal
 * plbm_moments bit for bit; with FP32 or 16-bit storage they are taken in
 * the step's FP32 arithmetic (plbm_moments sums in FP64).
 *   f_a, f_b, nsteps : as plbm_step, nsteps >= 1
 *   rho, ux, uy, theta : device FP64 planes of nx * ny values, row-major
 *              (ny, nx); any may be NULL (not written)
 * D2Q25 with the symmetric five-velocity set (dim 2) only; other
 * descriptors return PLBM_EUNSUPPORTED.  Launches kernels only (no
 * allocation or synchronisation).
 */
int plbm_step_fields(const plbm_desc *d, void *f_a, void *f_b, int nsteps, double *rho,
                     double *ux, double *uy, double *theta, void *stream);

/*
 * plbm_step_noalloc -- plbm_step without any device allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as plbm_step, for the descriptors of the symmetric five-velocity
 * model (D1Q5 and D2Q25, every storage form); other descriptors return
 * PLBM_EUNSUPPORTED.  The populations it writes are bitwise those of
 * plbm_step; the sums agree to FP64 rounding (their partial sums are grouped
 * differently).
 * Scratch: the partial sums of a call that asks for sums live in a
 * library-owned array in device memory, (8192 + 1) * 4 doubles (256 KiB),
 * held by every GPU the library runs on until the process ends.  Its device
 * address is looked up once per device, on the first call with that device
 * current; the stream must belong to the current device.  A 2D sums step
 * then runs at most 8192 workgroups, which walk all tiles.  Limit: a 1D
 * lattice with sums may have at most 8192 * 256 = 2,097,152 nodes
 * (PLBM_EINVAL beyond, before any launch); without sums no scratch is used
 * and plbm_step's limits apply.
 * Every call on one GPU shares that GPU's scratch and it keeps the last
 * call's contents: calls that ask for sums and overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.  Calls
 * without sums do not touch it.
 */
int plbm_step_noalloc(const plbm_desc *d, void *f_a, void *f_b, int nsteps,
                      double *sums, void *stream);

/*
 * plbm_moments -- macroscopic fields of the pre-collision state held by f
 * (pull, then rho = sum f, rho u = sum f v, 2 rho theta = sum f |v - u|^2 in
 * 2D and rho theta = sum f (v - u)^2 in 1D; one temperature for all axes).
 *   rho, ux, uy, theta : device pointers to nx*ny doubles, or NULL to skip
 *                        a field.
 *   sums               : NULL or a host pointer to 4 doubles: FP64 sums over
 *                        the nodes of that state (as for plbm_step).
 *                        Asking for sums synchronises `stream`.
 * dim 3 descriptors take plbm_moments3 instead (PLBM_EINVAL here).
 * Errors: PLBM_EINVAL, PLBM_EUNSUPPORTED, PLBM_ENONFINITE, PLBM_EHIP.
 */
int plbm_moments(const plbm_desc *d, const void *f, double *rho, double *ux,
                 double *uy, double *theta, double *sums, void *stream);

/*
 * plbm_moments3 -- plbm_moments for dim 3: rho, u = (ux, uy, uz) and theta
 * with 3 rho theta = sum f |v - u|^2 of the pre-collision state held by f.
 *   rho, ux, uy, uz, theta : device pointers to nx*ny*nz doubles (element
 *                            (z * ny + y) * nx + x), or NULL to skip a field.
 *   sums                   : NULL or a host pointer to 5 doubles, in the
 *                            order of plbm_step's 3D sums.  Asking for sums
 *                            synchronises `stream`.
 * Errors: PLBM_EINVAL, PLBM_EUNSUPPORTED, PLBM_ENONFINITE, PLBM_EHIP.
 */
int plbm_moments3(const plbm_desc *d, const void *f, double *rho, double *ux,
                  double *uy, double *uz, double *theta, double *sums, void *stream);

/*
 * plbm_dev_scales -- choose per-plane power-of-two scales for 16-bit
 * deviation storage from the initial fields: scale[k] = 2^e with e the
 * smallest integer such that max_x |f_eq_k(x) - rho0 w_k| <= 2^e * 2^10
 * (FP16: ample headroom below 65504 and well above the subnormal range),
 * and at least 2^-26 rho0 (rounded down to a power of two), so that the FP32
 * collision's rounding noise stays a small deviation even for an initial
 * state at rest.  The scales fit the initial fields: deviations growing
 * past about 64 times their initial maximum overflow FP16 (reported as
 * PLBM_ENONFINITE by the sums).  Writes d->scale.
 *   rho, ux, uy, theta : device pointers as for plbm_init.
 * Synchronises `stream`.  Errors: PLBM_EINVAL, PLBM_EHIP.
 */
int plbm_dev_scales(plbm_desc *d, const double *rho, const double *ux,
                    const double *uy, const double *theta, void *stream);

/* ------------------------------------------------------------------------
 * Batching form: many independent D2Q25 lattices advanced together.
 * Each lattice is the model of plbm_step (same velocity set and table) with
 * its own size and relaxation constant, FP32 storage, periodic boundaries.
 * One kernel launch per step walks a work list of tiles of every lattice;
 * plbm_batch_step replays a captured hipGraph of several such launches.
 * ------------------------------------------------------------------------ */
typedef struct plbm_batch plbm_batch;          /* opaque, owned by the library */

typedef struct plbm_lattice_spec {
    int32_t nx, ny;
    double omega;
} plbm_lattice_spec;

#define PLBM_BATCH_MAX_CLASSES 32

typedef struct plbm_batch_info {
    int32_t count;              /* lattices */
    int32_t tiles;              /* work-list entries */
    int32_t grid_mode;          /* 0: one workgroup per tile; k: k per CU */
    int32_t lds_bytes;          /* LDS reserved per workgroup (occupancy cap) */
    int32_t graph_steps;        /* launches per captured graph (0: no graph) */
    int32_t parity;             /* which of the two buffers holds the state */
    int64_t nodes;              /* total lattice nodes */
    int64_t pool_bytes;         /* device memory of all population buffers */
    int32_t classes;            /* size classes with a chosen tile shape */
    int32_t class_size[PLBM_BATCH_MAX_CLASSES];
    int32_t class_w[PLBM_BATCH_MAX_CLASSES];   /* tile width in nodes */
    int32_t class_r[PLBM_BATCH_MAX_CLASSES];   /* passes of 256/w rows */
} plbm_batch_info;

/*
 * plbm_batch_create -- allocate `count` lattices (two FP32 buffers each, one
 * device pool owned by the batch) described by specs[i] (host array) with
 * the velocity set and table of *proto (proto->storage must be PLBM_F32,
 * dim 2; its nx, ny, omega are ignored).  Tiles start at 256 x 1 until
 * plbm_batch_autotune chooses shapes.  Synchronous.  *out receives the handle.
 * Errors: PLBM_EINVAL (bad spec), PLBM_EUNSUPPORTED, PLBM_EHIP.
 */
int plbm_batch_create(const plbm_desc *proto, const plbm_lattice_spec *specs, int count,
                      plbm_batch **out);

/* Free the batch and its device memory (synchronises the device). */
int plbm_batch_destroy(plbm_batch *b);

/* Initialise lattice i to the equilibrium of its fields, as plbm_init
 * (rho, ux, uy, theta: device pointers to nx*ny doubles). Asynchronous. */
int plbm_batch_init(plbm_batch *b, int i, const double *rho, const double *ux,
                    const double *uy, const double *theta, void *stream);

/*
 * plbm_batch_autotune -- choose the tile shape of every size class
 * (max(nx, ny); width 64/128/256 nodes, 1/2/4/8 passes) from a few policies
 * (the narrowest width covering the class, 64-wide, 256-wide; one or two
 * passes), together with the grid mode and LDS occupancy cap, by timing
 * whole-batch launches.  cache_path (nullable) names a JSON file read first
 * (when it holds every class and the grid for this architecture nothing is
 * timed) and rewritten with the choices.  Overwrites every population
 * buffer (call before plbm_batch_init).  Synchronises `stream`.
 */
int plbm_batch_autotune(plbm_batch *b, const char *cache_path, void *stream);

/* Launches recorded per graph (even, 0..64; 0 disables graphs; default 8). */
int plbm_batch_set_graph_steps(plbm_batch *b, int steps);

/*
 * plbm_batch_step -- advance every lattice by nsteps applications of
 * Eq. srt (as plbm_step).  Whole groups of graph_steps steps replay the
 * captured graph (recorded on first use); the rest are direct launches.
 * Asynchronous on `stream`.
 */
int plbm_batch_step(plbm_batch *b, int nsteps, void *stream);

/* Moments (and optional host sums) of lattice i, as plbm_moments. */
int plbm_batch_moments(const plbm_batch *b, int i, double *rho, double *ux, double *uy,
                       double *theta, double *sums, void *stream);

/* Descriptor of lattice i (may be NULL) and its current population buffer
 * (device pointer, valid until the next step; may be NULL). */
int plbm_batch_lattice(const plbm_batch *b, int i, plbm_desc *desc, void **f);

/* Sizes, tiles and the tuned configuration. */
int plbm_batch_query(const plbm_batch *b, plbm_batch_info *info);

/* ------------------------------------------------------------------------
 * Learned closure: a 3-layer 3x3 convolutional network (25 -> 32 -> 32 -> 25
 * channels, ReLU, periodic padding; BF16 MFMA with FP32 accumulation) that
 * corrects a coarse D2Q25 lattice (FP32 or FP64 storage) after its
 * collide-and-stream step (Eq. srt).  Its output y, normalised by scales s,
 * becomes c = s * Ph y with Ph = I - B (B^T B)^-1 B^T, B = diag(s) Phi,
 * Phi_k = (1, v_x, v_y, |v|^2): node by node c carries no mass, momentum or
 * energy (the collision invariants), so streamed it only moves them between
 * nodes and the totals are conserved exactly.
 * Training compares, after the next streaming, the conserved densities the
 * correction adds with the one-step error of the plain coarse step against
 * restricted fine-lattice runs (plbm_restrict, plbm_closure_target).
 * ------------------------------------------------------------------------ */
typedef struct plbm_closure plbm_closure;      /* opaque, owns workspaces */

/* Flat FP32 parameter vector: for layer l = 0, 1, 2 at offset l * 9248,
 * weights W[tap][out][in] (9 x 32 x 32, tap = 3 * (dy + 1) + (dx + 1), the
 * input node is (y + dy, x + dx)) then the bias[32].  Channels are padded to
 * 32; the padded inputs of layer 0 and outputs of layer 2 must hold zeros. */
#define PLBM_CNN_LAYER_PARAMS 9248
#define PLBM_CNN_PARAMS (3 * PLBM_CNN_LAYER_PARAMS)

/*
 * plbm_closure_create -- workspaces for up to `frames` coarse lattices of
 * the shape of *coarse (dim 2, FP32 or FP64 storage, nx a multiple of 64,
 * ny at most 65535, whole-node velocities smaller than nx and ny) processed
 * together.
 * Synchronous.  Errors: PLBM_EINVAL, PLBM_EUNSUPPORTED, PLBM_EHIP.
 */
int plbm_closure_create(const plbm_desc *coarse, int frames, plbm_closure **out);
int plbm_closure_destroy(plbm_closure *c);

/* Normalisation (host arrays): network input (P_k - in_mean[k]) /
 * in_scale[k] and correction s_k * y_k with s_k = out_scale[k] (25 each);
 * moment_scale[4] = sigma_j of the loss (weights 1 / sigma_j^2 for rho,
 * j_x, j_y, E).  All must be finite, scales positive. */
int plbm_closure_set_norm(plbm_closure *c, const float *in_mean, const float *in_scale,
                          const float *out_scale, const float *moment_scale);

/*
 * plbm_closure_forward -- run the network on `frames` post-collision buffers
 * (post: host array of device pointers, each a population buffer of the
 * coarse lattice in its storage type) with parameters `params` (device,
 * PLBM_CNN_PARAMS floats).  noise: NULL, or device FP32 values added, times
 * noise_amp, to the normalised input, laid out [frame][k][y][x] (training
 * augmentation; the caller draws them).  Keeps the activations for
 * plbm_closure_backward and plbm_closure_apply.
 */
int plbm_closure_forward(plbm_closure *c, const float *params, const void *const *post,
                         int frames, const float *noise, float noise_amp, void *stream);

/*
 * plbm_closure_backward -- moment-form loss of the last forward pass and its
 * gradient with respect to `params`, written to `grads` (device,
 * PLBM_CNN_PARAMS floats).  With c = s * Ph y and m(x) = sum_k Phi_k
 * (c_k(x - v_k) - c_k(x)) (the conserved densities the correction brings to
 * node x after streaming, periodic, in flux form so their totals vanish),
 *   L = mean over nodes of [sum_j (m_j - d_j)^2 / sigma_j^2 + reg |Ph y|^2];
 * the moments fix 4 of a node's 21 free correction components and the
 * minimum-norm weight reg >= 0 selects the smallest correction.
 * target: host array of device pointers, one per frame, to d as four FP32
 * planes [j][y][x] (rho, j_x, j_y, E), e.g. from plbm_closure_target.
 * loss: NULL, or a host double receiving L (synchronises `stream`;
 * PLBM_ENONFINITE if not finite).
 */
int plbm_closure_backward(plbm_closure *c, const float *params, const float *const *target,
                          float reg, float *grads, double *loss, void *stream);

/* One Adam step (step count t >= 1) on device arrays of PLBM_CNN_PARAMS. */
int plbm_closure_adam(plbm_closure *c, float *params, const float *grads, float *m, float *v,
                      int t, float lr, float b1, float b2, float eps, void *stream);

/*
 * plbm_closure_apply -- give the last forward pass's correction to the same
 * post buffers, in place, in their storage type.  The correction c = s * Ph y
 * moves the conserved densities g(x) = sum_k Phi_k (c_k(x - v_k) - c_k(x)) between
 * nodes; apply hands them to the next step as a shift of the equilibrium,
 *   f <- f + f_eq(m + g) - f_eq(m)   (f = the pulled populations, m their
 *                                     moments; stored at x - v_k),
 * so each node's mass, momentum and energy become m + g exactly and its
 * non-equilibrium part is the plain step's.  Fallback: a node whose
 * normalised correction Ph y is not finite or exceeds `bound` in magnitude
 * in any component contributes nothing, and *skipped (device counter,
 * nullable) is incremented; a node whose shifted density or temperature
 * would not be positive keeps its populations.  Asynchronous.
 */
int plbm_closure_apply(plbm_closure *c, void *const *post, int frames, float bound,
                       unsigned *skipped, void *stream);

/* ------------------------------------------------------------------------
 * Training the closure through several coarse steps: reverse-mode
 * derivatives (vector-Jacobian products) of the step, of the apply and of a
 * loss on the rolled-out state.  An adjoint buffer holds dL/dP for a
 * population buffer P: FP64, the population layout of dim 2
 * ((y * 25 + k) * nx + x), caller-owned device memory.  With Phi_k =
 * (1, v_x, v_y, |v|^2), m = Phi^T f the conserved densities (rho, j_x, j_y,
 * E = sum f |v|^2) and F(m) the equilibrium of Eq. eqdist (r = C mu of
 * Eq. rdr at rho, u = j / rho, 2 theta = E / rho - |u|^2):
 * ------------------------------------------------------------------------ */

/*
 * plbm_step_vjp -- adjoint of one step of Eq. srt on the buffer convention:
 * for P' = (1 - omega) S + omega F(m(S)), S = pull(post),
 *   out = dL/dpost = push((1 - omega) lam + omega Phi J_F(m)^T lam),
 * with J_F the Jacobian of F (its derivatives from those of the Maxwell
 * moments, d mu_n/du = n mu_(n-1), d mu_n/dtheta = n (n-1)/2 mu_(n-2)).
 *   post : device, the buffer the step read (FP64 or FP32 storage)
 *   lam  : device FP64 adjoint buffer, dL/dP' of the buffer the step wrote
 *   out  : device FP64 adjoint buffer (written; must not alias lam)
 * D2Q25 (symmetric five-velocity set, dim 2, ny <= 65535) only; other
 * descriptors return PLBM_EUNSUPPORTED.  Asynchronous.
 */
int plbm_step_vjp(const plbm_desc *d, const void *post, const double *lam, double *out,
                  void *stream);

/*
 * plbm_closure_rollout_loss -- loss of rolled-out states against the truth
 *   L = scale sum_frames sum_x sum_j w_j (m_j(pull(post))(x) - cons_j(R)(x))^2
 * with w_j = 1 / sigma_j^2 from plbm_closure_set_norm's moment_scale and
 * cons(R) = (rho, rho u_x, rho u_y, rho (2 theta + |u|^2)) of the truth.
 *   post  : host array of `frames` device population buffers (the states)
 *   truth : host array of 4 * frames device FP64 planes (nx * ny each),
 *           (rho, u_x, u_y, theta) of frame 0, then frame 1, ...
 *   scale : > 0 (e.g. 1 / (steps * frames * nodes))
 *   lam   : NULL, or host array of `frames` FP64 adjoint buffers to which
 *           dL/dpost = push(Phi 2 scale w r) is added
 *   loss  : NULL, or a host double receiving L (synchronises `stream`;
 *           PLBM_ENONFINITE if not finite)
 */
int plbm_closure_rollout_loss(plbm_closure *c, void *const *post, const double *const *truth,
                              int frames, double scale, double *const *lam, double *loss,
                              void *stream);

/*
 * plbm_closure_apply_vjp -- adjoint of plbm_closure_apply (without its
 * fallback bound) for the buffers the last plbm_closure_forward read.  With
 * lam = dL/dpost' on entry (updated in place) and Lam = pull(lam):
 *   lam <- lam + push(Phi (J_F(m + g) - J_F(m))^T Lam)    (the state path)
 * and dL/dg = J_F(m + g)^T Lam is kept for plbm_closure_backward_vjp.  Nodes
 * the apply would leave unshifted pass nothing.
 *   post : the pre-apply buffers (as given to plbm_closure_forward)
 *   lam  : host array of `frames` FP64 adjoint buffers
 */
int plbm_closure_apply_vjp(plbm_closure *c, void *const *post, double *const *lam, int frames,
                           void *stream);

/*
 * plbm_closure_backward_vjp -- the network's part of the apply adjoint:
 * from dL/dg of the last plbm_closure_apply_vjp, dL/dy = Ph (s * dL/dc)
 * (plus the minimum-norm term reg), back through the three layers: the
 * parameter gradient is written to `grads` (device, PLBM_CNN_PARAMS floats)
 * or added to it when `accumulate` is non-zero, and, when lam is not NULL,
 * the gradient of the network input is added to the adjoint buffers
 * (lam += dL/dpost through the normalised input).  Asynchronous.
 */
int plbm_closure_backward_vjp(plbm_closure *c, const float *params, float reg, float *grads,
                              int accumulate, double *const *lam, void *stream);

/*
 * plbm_closure_rollout_vjp -- one backward step of training through
 * corrected coarse steps, fused: for step s of a segment, with Q_s the
 * state after the apply of step s, B_(s-1) the buffer the coarse step read
 * and A_(s-1) the buffer it wrote (the network's input, as given to the last
 * plbm_closure_forward), it computes what plbm_closure_rollout_loss (at
 * Q_s), plbm_closure_apply_vjp, plbm_closure_backward_vjp and plbm_step_vjp
 * compute in sequence, in two node passes instead of six (the three
 * in-place passes over the adjoint buffers become reads of per-node moment
 * cotangents; the loss's and the apply's moment cotangents are summed per
 * node before they are pushed, the same terms rounded in another order).
 *   coarse  : the coarse lattice's descriptor (its omega; shape, storage and
 *             velocities must be the closure's, else PLBM_EINVAL)
 *   params, reg, grads : as plbm_closure_backward_vjp; accumulate = 0 on
 *             the first call of a segment writes the parameter gradient and
 *             restarts the segment loss, non-zero adds to both
 *   after   : `frames` device buffers Q_s;  truth : 4 * frames FP64 planes
 *             as plbm_closure_rollout_loss;  scale > 0 as there
 *   pre     : the buffers A_(s-1) (must be those of the last forward)
 *   before  : the buffers B_(s-1) (needed only with lam_out)
 *   lam_in  : NULL (zero: the segment's last step), or `frames` FP64
 *             adjoint buffers dL/dQ_s from the later steps (read only)
 *   lam_out : NULL (the segment's first step: its adjoint is truncated), or
 *             `frames` FP64 adjoint buffers receiving dL/dQ_(s-1) (written;
 *             must not alias lam_in)
 *   loss    : NULL, or a host double receiving the segment loss accumulated
 *             since the last call with accumulate = 0 (synchronises
 *             `stream`; PLBM_ENONFINITE if not finite).  The partial sums
 *             live in the closure and plbm_closure_rollout_loss reuses
 *             them: do not interleave the two within a segment.
 * Asynchronous otherwise.
 */
int plbm_closure_rollout_vjp(plbm_closure *c, const plbm_desc *coarse, const float *params, float reg,
                             float *grads, int accumulate, void *const *after,
                             const double *const *truth, double scale, void *const *pre,
                             const void *const *before, const double *const *lam_in,
                             double *const *lam_out, int frames, double *loss, void *stream);

/* Device pointer and size of an internal buffer (for tests):
 * 0 input, 1 layer-1 output, 2 layer-2 output (bf16 NHWC x 32), 3 network
 * output (FP32 NHWC x 32), 4..6 gradients w.r.t. layer-3/2/1 outputs,
 * 7 the physical correction c (FP32 planes [frame][k][y][x]),
 * 8 dL/dm (FP32 [frame][y][x][j], j = mass, x and y momentum, energy),
 * 10 per-node moment cotangents of the last adjoint call (FP64
 * [frame][y][x][j]), 11 the gradient of the network input (FP32 NHWC x 32).
 * 9 is not a buffer (apply adds its equilibrium shift in place): PLBM_EINVAL. */
int plbm_closure_activation(const plbm_closure *c, int which, const void **ptr, size_t *bytes);

/*
 * plbm_closure_target -- the loss target of one frame: the one-step change
 * of the conserved densities cons = (rho, rho u_x, rho u_y, rho (2 theta +
 * |u|^2)) of the truth minus that of the plain coarse step,
 *   d = (cons(T1) - cons(T0)) - (cons(M1) - cons(M0)),
 * computed in FP64 and rounded once.  fields: host array of 16 device FP64
 * pointers, (rho, u_x, u_y, theta) of T0, T1, M0, M1 in that order, each
 * `nodes` long (1 to 2^30); out: device FP32, four planes of `nodes`.
 * Asynchronous.  Errors: PLBM_EINVAL (null pointers, nodes out of range).
 */
int plbm_closure_target(const double *const *fields, size_t nodes, float *out, void *stream);

/*
 * plbm_restrict -- block means over factor x factor fine nodes of rho,
 * rho u and rho (2 theta + |u|^2), returned as coarse (rho, u, theta).
 * All pointers are device FP64 arrays; fine fields fnx x fny (multiples of
 * factor, at most 65535 coarse rows).  Asynchronous.  Errors: PLBM_EINVAL.
 */
int plbm_restrict(const double *rho, const double *ux, const double *uy, const double *theta,
                  int fnx, int fny, int factor, double *crho, double *cux, double *cuy,
                  double *ctheta, void *stream);

/*
 * plbm_stream_copy -- measurement utility (not part of the method): copies
 * `bytes` from src to dst, 16 bytes per thread, one pass.  It calibrates the
 * achievable HBM bandwidth and the profiler's byte counters against a kernel
 * whose traffic is exactly 2 * bytes.
 *   src, dst : device pointers, 16-byte aligned, non-overlapping
 *   bytes    : a positive multiple of 16
 * Asynchronous on `stream`.  Errors: PLBM_EINVAL, PLBM_EHIP.
 */
int plbm_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Static description of a status code. */
const char *plbm_strerror(int status);

/* Text of the last HIP runtime error that made a call on this thread return
 * PLBM_EHIP ("" if none).  Owned by the library; valid until the next call
 * on the same thread. */
const char *plbm_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PLBM_H */
