/*
 * pse.h -- C ABI of the MI355X (gfx950) Positively-Split Ewald library for
 * Brownian dynamics of rigid spheres with stresslet constraints
 * (Fiore & Swan, arXiv 1709.06946).
 *
 * The library evaluates, on one GPU, the FTS grand mobility product
 * (Sec. II, Eqs. pairsums and WSops2), the split Brownian sampler
 * (Sec. III, Eq. split with the Lanczos real-space square root and the
 * analytic wave-space square root of Eq. FFTsqrt) and the stresslet-
 * constrained mid-point step (Sec. III.D and Appendix B).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: any consistent set; radius a, viscosity eta and kT come from the
 * parameters.  The periodic cell is a cube of side L, V = L^3.
 *
 * Positions: double x[N][3], device memory, any real values (they are
 *   wrapped into [0, L) internally; the caller's array is only written by
 *   pse_constrained_step).
 * Generalized force, 11 doubles per particle, particle-major:
 *   [F_x F_y F_z | L_x L_y L_z | s_1 .. s_5]
 * Generalized velocity, 11 doubles per particle:
 *   [U_x U_y U_z | Omega_x Omega_y Omega_z | e_1 .. e_5]
 *   The couplet is C = sum_q s_q Y_q - 1/2 eps.L (force index first), the
 *   velocity gradient D_ij = du_i/dx_j gives Omega = -1/2 eps:D and
 *   e_q = Y_q : D, with the orthonormal symmetric traceless basis
 *   Y_1 = (xy+yx)/sqrt2, Y_2 = (xz+zx)/sqrt2, Y_3 = (yz+zy)/sqrt2,
 *   Y_4 = (xx-yy)/sqrt2, Y_5 = (xx+yy-2zz)/sqrt6.  In these coordinates the
 *   11N x 11N grand mobility is a symmetric matrix.
 * Particle vectors are always double, whatever the handle's precision.
 *
 * Wave noise (optional caller-supplied Brownian noise for the wave-space
 *   square root): complex double psi[3][Ng][Ng][Ng/2+1] (interleaved re, im),
 *   device memory.  Index i of the z and y axes maps to wave number i for
 *   i < Ng/2 and i - Ng otherwise; the x index is kappa_x >= 0.  Only the
 *   canonical half space (kappa_x > 0; or kappa_x = 0, kappa_y > 0; or
 *   kappa_x = kappa_y = 0, kappa_z > 0) is read; psi(-k) = conj(psi(k)).
 *   Modes with a Nyquist index and k = 0 carry no noise.  Real and imaginary
 *   parts should be independent N(0, 1/2).
 *
 * Memory: every pointer argument is caller-owned device memory unless noted;
 *   the library never frees or keeps it after the call returns.  The handle
 *   owns all its workspace (grids, spectra, cell lists, Krylov bases).
 * Streams: all work runs on the stream given at creation (NULL = the
 *   library's own stream).  Calls of a synchronous handle return after the
 *   work has completed; calls of an asynchronous handle (params.async_calls)
 *   only enqueue it.  A handle is not re-entrant: use one handle per host
 *   thread.
 * Status: 0 = success; > 0 = warning with valid outputs; < 0 = error, outputs
 *   undefined.  No call aborts or throws; pse_last_error gives the message.
 */
#ifndef PSE_H
#define PSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PSE_OK = 0,
  PSE_WARN_NOT_CONVERGED = 1,   /* a Krylov solve stopped at its limit      */
  PSE_ERR_INVALID = -1,         /* invalid argument or parameter            */
  PSE_ERR_NOMEM = -2,           /* device allocation failed                 */
  PSE_ERR_HIP = -3,             /* HIP runtime error                        */
  PSE_ERR_NONFINITE = -4        /* NaN/Inf detected in an input or result   */
};

enum { PSE_FP64 = 0, PSE_MIXED = 1 };     /* pse_params.precision */
/* pse_mobility_apply parts; PSE_ES_BLOCK with either or both parts applies
 * only the stresslet-strain block M_ES (in's s components to out's e
 * components, the other components of out untouched) through the operator
 * the constrained step solves with (moment or derivative gridding). */
enum { PSE_REAL = 1u, PSE_WAVE = 2u, PSE_ES_BLOCK = 4u };

/* Input parameters.  Fields set to 0 are derived (see pse_derive). */
typedef struct pse_params {
  int64_t n;               /* number of particles N > 0                      */
  double box;              /* cubic cell side L > 4a                         */
  double radius;           /* sphere radius a > 0                            */
  double viscosity;        /* eta > 0                                        */
  double kT;               /* thermal energy > 0                             */
  double tol;              /* Ewald / quadrature tolerance eps, (0, 0.1]     */
  int32_t grid;            /* FFT grid points per side Ng (even, 2^j or
                              3*2^j, 8 <= Ng <= 1024); 0 = from tol         */
  int32_t support;         /* Gaussian support P (points per side); 0 = auto */
  double xi;               /* splitting parameter; 0 = from grid and tol     */
  double rcut;             /* real-space cutoff; 0 = auto                    */
  int32_t precision;       /* PSE_FP64 or PSE_MIXED                          */
  int32_t lanczos_maxit;   /* 0 = 100                                        */
  double lanczos_tol;      /* 0 = 1e-3                                       */
  int32_t gmres_restart;   /* 0 = 30                                         */
  int32_t gmres_maxit;     /* total GMRES iterations; 0 = 200                */
  double gmres_tol;        /* relative residual; 0 = 1e-6                    */
  int32_t refine_passes;   /* FP64 residual refinement passes (mixed); 0 = 3 */
  int32_t graphs;          /* 0: replay each constraint-operator application
                              from a captured hipGraph (captured on first use
                              per input/output pair); -1: launch eagerly     */
  int32_t deriv_gridding;  /* gridding of the wave-space products (Sec. II
                              in couplets C and velocity gradients D):
                              1 = every force, torque and stresslet
                              component gridded as its own moment and
                              transformed (up to eleven grids each way);
                              2 = forces and velocities on three moment
                              grids each, couplets (torques and stresslets
                              together) spread with the Gaussian's gradient
                              onto three grids and rotation and strain
                              interpolated with it from three more: at most
                              six grids each way, three each way for M_ES.
                              The gradient weights are corrected per
                              particle so that their discrete sum is zero
                              and their first moment exact, and the support
                              takes one more point when support = 0; falls
                              back to 1 when that support exceeds 10.
                              0 = library default: 2 while the stencil
                              points per grid point N (P+1)^3 / Ng^3 stay
                              at most 20, else 1                            */
  void *stream;            /* hipStream_t to run on, or NULL                 */
  int32_t async_calls;     /* 0: every call returns after its work has
                              completed; Krylov solves check convergence on
                              the host and stop at the first iteration that
                              meets the tolerance.
                              1: calls only enqueue work on the stream (no
                              host synchronisation, so a whole step can be
                              captured into a graph by the caller): every
                              Lanczos solve runs exactly lanczos_maxit
                              iterations (0 = 16) and every GMRES solve
                              exactly gmres_maxit (0 = 32, no restarts;
                              mixed handles: refine_passes passes, 0 = 1),
                              the result taken at the first iteration that
                              met the tolerance (the later ones are computed
                              and discarded); statistics and status are
                              written by the device (see pse_constrained_step);
                              the pair list keeps its creation capacity (pairs
                              beyond it are dropped and flagged). */
  double deform[9];        /* volume-preserving deformation A of the periodic
                              lattice (Sec. II.C.2), row-major; all zero =
                              the cube.  The lattice vectors are the columns
                              of L A (Lees-Edwards shear: A = [[1, gamma, 0],
                              [0, 1, 0], [0, 0, 1]]; planar extension:
                              diag(e, 1/e, 1)); det A must be 1.  The FFT
                              grid is the deformed lattice's, the Gaussian
                              support grows with lambda_max, the largest
                              eigenvalue of A^T A (Eq. bound), and the
                              constraint operator grids its five moments. */
} pse_params;

/* Derived quantities (Sec. II.C, Eq. bound and the Sec. II.C.1 cutoff). */
typedef struct pse_derived {
  int32_t grid;            /* Ng                                             */
  int32_t support;         /* P                                              */
  double xi;               /* splitting parameter                            */
  double eta_s;            /* Gaussian shape (h P xi / m)^2, < 1             */
  double m;                /* Gaussian width in standard deviations          */
  double h;                /* grid spacing L / Ng                            */
  double rcut;             /* real-space cutoff                              */
  int32_t cells;           /* cells per side of the real-space cell list     */
  int32_t lanczos_maxit, gmres_restart, gmres_maxit, refine_passes;
  double lanczos_tol, gmres_tol;
  int32_t deriv_gridding;  /* gridding in effect: 1 moments, 2 derivative */
  double lambda_max;       /* largest eigenvalue of A^T A (1 for the cube)   */
} pse_derived;

/* Krylov statistics of a step.  Synchronous handles write them to host
 * memory before returning; asynchronous handles write them from the device
 * (the pointer must be device memory or pinned host memory) and they are
 * valid once the stream has completed the call's work. */
typedef struct pse_stats {
  int32_t lanczos_iters;   /* Lanczos iterations of the real-space sqrt (for
                              asynchronous handles: the iteration whose
                              iterate was taken)                             */
  int32_t gmres_iters;     /* GMRES iterations, all refinement passes        */
  int32_t refine_passes;   /* FP64 refinement passes (mixed precision)       */
  int32_t converged;       /* 1 if every Krylov solve met its tolerance      */
  double lanczos_change;   /* last relative change of the Lanczos iterate    */
  double gmres_residual;   /* final relative residual of M_ES S = b (in the
                              precision of the last solve)                   */
  double fp64_residual;    /* FP64 relative residual after refinement, or -1 */
  int32_t status;          /* asynchronous handles: PSE_STATUS_* bits of
                              problems the device met (0 = none); 0 for
                              synchronous handles, which return errors      */
  int32_t reserved;
} pse_stats;

/* pse_stats.status bits. */
enum {
  PSE_STATUS_NONFINITE_POS = 1,  /* a non-finite position (taken as 0)       */
  PSE_STATUS_PAIR_OVERFLOW = 2   /* real-space pairs beyond the pair list's
                                    capacity were dropped                    */
};

/* step argument of pse_constrained_step / pse_rpy_step: take the noise
 * counter from the handle's device step counter and advance it (asynchronous
 * handles; a captured step then draws new noise on every replay). */
#define PSE_STEP_DEVICE UINT64_MAX

typedef struct pse_handle pse_handle;

/* Derive Ng, P, xi, eta_s, m, rcut and Krylov defaults from p without any
 * GPU work.  Rules (Sec. II.C, Eq. bound with lambda_max = 1, with the
 * quadrature tolerance tightened to eps/20 because the bound's constants are
 * unknown): P = ceil((2/pi) ln(40/eps)); m = 0.85 sqrt(pi P);
 * xi = pi Ng / (2 L sqrt(ln(1/eps) + 9)), so that the Hasimoto factor
 * exp(-k^2/4xi^2) is e^-9 eps at the Nyquist wave number;
 * eta_s = (h P xi / m)^2; rcut = 2a + sqrt(ln(1/eps))/xi, the real-space
 * functions decaying like exp(-xi^2 (r - 2a)^2) (Appendix A).
 * With these rules every block of the mobility product and of the wave-space
 * square root is within eps of the exact sums at eps = 1e-3 (checked against
 * the oracle).
 * Deformed lattices (params.deform): P = ceil(lambda_max (2/pi) ln(40/eps))
 * (Eq. bound: both error terms decay as exp(-pi P / (2 lambda_max)) at
 * m = sqrt(pi P), which needs lambda_max times the support for the same
 * error), xi divided by sqrt(lambda_max) (the shortest Nyquist wave vector of
 * the deformed reciprocal lattice is that much shorter), cells of the
 * real-space list from the cell's thinnest width.
 * Returns PSE_ERR_INVALID for inconsistent parameters (eta_s >= 1,
 * rcut > L/3, unsupported Ng, det A != 1, ...). */
int pse_derive(const pse_params *p, pse_derived *out);

/* Device bytes a handle with these parameters would allocate (host only). */
int pse_footprint_bytes(const pse_params *p, size_t *bytes);

/* Create a handle: validate, derive, allocate the library-owned workspace on
 * the current device and build the real-space function tables on the GPU. */
int pse_create(const pse_params *p, pse_handle **out);

/* Free the handle's device memory.  NULL is accepted. */
int pse_destroy(pse_handle *h);

/* Derived parameters of a live handle. */
int pse_get_derived(const pse_handle *h, pse_derived *out);

/* Grand mobility product (Eq. pairsums, WSops2):
 *   out = (M_r + M_w) in     for parts = PSE_REAL | PSE_WAVE,
 * or either part alone.  x: double[N][3]; in, out: double[N][11] in the
 * layouts above.  M_r is the neighbour-list sum of the real-space pair
 * functions (factor 1 - H) within rcut, M_w the Gaussian-gridded NUFFT
 * evaluation of the wave-space sum (factor H).  in and out must not
 * overlap. */
int pse_mobility_apply(pse_handle *h, const double *x, const double *in,
                       double *out, unsigned parts);

/* The same product for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): no
 * handle, and no hipMalloc, hipFree or allocating library call.  Parameters
 * are derived from *p as by pse_create (its Krylov and graph settings are
 * ignored); every buffer of the product (grids, tables, cell and pair lists)
 * is taken from a fixed static device scratch of 64 MiB per device, which
 * the library holds until the process ends.  x, in, out and parts as for
 * pse_mobility_apply, on p->stream (NULL: the null stream); the call returns
 * after the product has completed.  A product that does not fit the scratch
 * (roughly: grids above 64^3, or many thousands of particles) returns
 * PSE_ERR_NOMEM, with pse_last_error(NULL) saying so.  Every call on a device
 * shares that device's scratch: calls that overlap on one GPU (other host
 * threads, other streams) race and must be serialised by the caller.
 * Errors are reported through pse_last_error(NULL). */
int pse_mobility_apply_noalloc(const pse_params *p, const double *x, const double *in,
                               double *out, unsigned parts);

/* Split Brownian sampler (Eq. split): out_real = M_r^(1/2) psi_real by the
 * Lanczos iteration (relative change tolerance lanczos_tol), and
 * out_wave = M_w^(1/2) psi_wave by Eq. FFTsqrt (noise scaled, projected,
 * inverse FFT, interpolated).  Both unscaled (no sqrt(2kT/dt)).
 * psi_real: double[N][11] or NULL; psi_wave: wave-noise layout or NULL.
 * A NULL noise pointer draws the noise in-kernel from Philox-4x32-10 keyed by
 * (seed, counter).  out_real, out_wave: double[N][11], either may be NULL.
 * stats may be NULL.  Returns PSE_WARN_NOT_CONVERGED if Lanczos hit its
 * limit. */
int pse_brownian_sample(pse_handle *h, const double *x,
                        const double *psi_real, const double *psi_wave,
                        uint64_t seed, uint64_t counter,
                        double *out_real, double *out_wave, pse_stats *stats);

/* Optional inputs and outputs of pse_constrained_step (NULL = unused). */
typedef struct pse_step_io {
  const double *psi_real;  /* in:  double[N][11] real-space noise           */
  const double *psi_wave;  /* in:  wave noise (layout above)                */
  double *slip;            /* out: double[N][11] (U^B, Omega^B, E^B)        */
  double *stresslet;       /* out: double[N][5]  S at the mid-point         */
  double *velocity;        /* out: double[N][3]  U at the mid-point         */
} pse_step_io;

/* One stresslet-constrained mid-point step (Sec. III.D, Appendix B):
 *   (U^B, E^B) = sqrt(2 kT / dt) (M_r^(1/2) psi1 + M_w^(1/2) psi2)  at x_k
 *   x_{k+1/2}  = x_k + dt/2 U^B
 *   M_ES S     = -E^B - M_EF F^P         at x_{k+1/2}  (GMRES)
 *   U          = U^B + M_UF F^P + M_US S  at x_{k+1/2}
 *   x_{k+1}    = x_k + dt U      (written to x, wrapped into [0, L))
 * FL: double[N][6] deterministic force and torque F^P, or NULL for none.
 * Noise comes from io (if given) or from Philox keyed by (seed, step).
 * Returns PSE_WARN_NOT_CONVERGED if a Krylov solve hit its limit. */
int pse_constrained_step(pse_handle *h, double *x, const double *FL,
                         double dt, uint64_t seed, uint64_t step,
                         const pse_step_io *io, pse_stats *stats);

/* Switch a live handle between synchronous (async_calls = 0) and
 * asynchronous (1) calls.  For asynchronous calls, lanczos_iters (1 ..
 * lanczos_maxit of the handle), gmres_iters (1 .. its gmres_restart: the
 * basis holds every iteration) and refine_passes (>= 1, mixed handles) fix
 * the device-checked solves, and the pair list gets half its last length as
 * headroom (it cannot grow inside an asynchronous call).  The device step
 * counter of PSE_STEP_DEVICE is set to next_step.  Synchronises the stream.
 * Typical use: one synchronous step to learn the iteration counts, then
 * asynchronous steps with a little margin. */
int pse_set_krylov(pse_handle *h, int async_calls, int lanczos_iters, int gmres_iters,
                   int refine_passes, uint64_t next_step);

/* Wait until the handle's stream has completed all enqueued work. */
int pse_synchronize(pse_handle *h);

/* Graph-captured steps.  pse_step_graph_create captures `steps` constrained
 * steps of an asynchronous handle on its own stream (params.stream NULL)
 * into one executable graph: positions x (updated in place), forces FL (or
 * NULL), dt and seed are fixed; the noise counter is the handle's device step
 * counter (PSE_STEP_DEVICE), so every launch draws new noise; stats (device
 * or pinned host memory, or NULL) receives each step's statistics.  Nothing
 * runs at capture.  pse_step_graph_launch enqueues one replay on the handle's
 * stream (no host synchronisation); pse_step_graph_destroy waits for the
 * stream and frees the graph (the handle stays). */
typedef struct pse_step_graph pse_step_graph;
int pse_step_graph_create(pse_handle *h, double *x, const double *FL, double dt,
                          uint64_t seed, int steps, pse_stats *stats, pse_step_graph **out);
int pse_step_graph_launch(pse_step_graph *g);
int pse_step_graph_destroy(pse_step_graph *g);

/* ---- Unconstrained (RPY-level) PSE: forces only ----
 * The comparison system of the performance study (Sec. IV): the mobility
 * reduced to its force-velocity block M_UF (the periodic RPY tensor of the
 * positively split Ewald sum), three gridded components per product and no
 * constraint.  Same handle, kernels and precision as the FTS calls. */

/* U = M_UF F (parts as for pse_mobility_apply).  x: double[N][3];
 * F, U: double[N][3] device arrays (U overwritten). */
int pse_rpy_apply(pse_handle *h, const double *x, const double *F, double *U,
                  unsigned parts);

/* One Euler-Maruyama step with the split sampler restricted to the UF block
 * (the RPY tensor is divergence-free, so there is no drift term):
 *   U^B     = sqrt(2 kT / dt) ((M_r)_UF^(1/2) psi1 + (M_w)_UF^(1/2) psi2)  at x_k
 *   x_{k+1} = x_k + dt (M_UF F + U^B)   (written to x, wrapped into [0, L))
 * (M_r)_UF^(1/2) is the principal root of the real-space UF block (Lanczos);
 * the wave part maps the same three-component wave noise as the FTS sampler
 * through the velocity rows only.  F: double[N][3] or NULL.  io as for
 * pse_constrained_step, with psi_real double[N][3] (the first three of each
 * particle's Philox normals when NULL), slip double[N][3] = U^B and velocity
 * double[N][3] = M_UF F + U^B; stresslet is not used.  Returns
 * PSE_WARN_NOT_CONVERGED if Lanczos hit its limit. */
int pse_rpy_step(pse_handle *h, double *x, const double *F, double dt, uint64_t seed,
                 uint64_t step, const pse_step_io *io, pse_stats *stats);

/* Diagnostics of individual stages (used by the kernel tests). */
/* In-place unnormalized 3D FFT of ncomp complex double grids
 * data[ncomp][Ng][Ng][Ng] (z, y, x; x fastest) with the handle's grid and
 * precision (mixed handles convert to float and back).  direction -1:
 * sum f exp(-i k.x); +1: sum f exp(+i k.x).  1 <= ncomp <= 6. */
int pse_fft3d(pse_handle *h, double *data, int ncomp, int direction);

/* In-place real 3D FFT of ncomp grids with the transforms the mobility
 * product and the wave sampler run (Eq. WSops2), in the handle's precision
 * (mixed handles convert to float and back).  data holds ncomp blocks of
 * Ng^3 doubles.  direction -1: each block is a real grid g[z][y][x] (x
 * fastest) and is overwritten by its half spectrum
 * G[kz][ky][kx] = sum g exp(-i k.x) for kx < Ng/2, complex (re, im)
 * interleaved, the kx = Ng/2 column not stored; direction +1: the inverse,
 * g = sum_k G exp(+i k.x) (unnormalized) over the stored half spectrum and
 * its conjugates, the kx = Ng/2 column taken as zero.  1 <= ncomp <= 11. */
int pse_rfft3d(pse_handle *h, double *data, int ncomp, int direction);

/* Gaussian spreading of ncomp components of q (double[N][ncomp]) onto
 * ncomp real grids out[ncomp][Ng][Ng][Ng]: out_c(x_n) = sum_b K(x_n - x_b)
 * q_bc with K(r) = (2 xi^2 / (pi eta_s))^(3/2) exp(-2 xi^2 r^2 / eta_s)
 * truncated to the P^3 nearest grid points (Sec. II.C, Eq. quadapprox).
 * 1 <= ncomp <= 11. */
int pse_spread(pse_handle *h, const double *x, const double *q, int ncomp,
               double *grids);

/* Interpolation, the adjoint operation: out_bc = sum_n K(x_n - x_b)
 * g_c(x_n) for ncomp real grids g[ncomp][Ng][Ng][Ng]; out double[N][ncomp]. */
int pse_interpolate(pse_handle *h, const double *x, const double *grids,
                    int ncomp, double *out);

/* Stage timing (instrumentation).  With profiling on, every kernel launch
 * of the handle is bracketed by HIP events on the handle's stream and its
 * duration accumulated per stage, together with the stage's algorithmic
 * bytes (the data a launch must read or write at least once: the grids it
 * reads and writes, plus particle data).  pse_profile(h, 1) clears the
 * totals, times an empty bracket (two event records back to back: the time
 * the timestamps add, subtracted once from every bracket) and a bracket
 * around an empty one-thread kernel, and starts; pse_profile(h, 0) stops.
 * Stage names: spread, fft, kspace, interp, zero, real, cells, krylov,
 * noise; two last records (launches = 1) hold the empty bracket time
 * ("bracket", the subtracted one) and the empty-kernel bracket time
 * ("bracket_noop"). */
typedef struct pse_kernel_stat {
  const char *name;        /* static string owned by the library            */
  int64_t launches;
  double total_ms;
  double alg_bytes;        /* summed over the launches                      */
} pse_kernel_stat;

int pse_profile(pse_handle *h, int enable);

/* Copy up to max stage records to out (host memory); *count receives the
 * number written. */
int pse_profile_read(pse_handle *h, pse_kernel_stat *out, int max, int *count);

/* ------------------------------------------------------------------------
 * Serving: continuous admission of independent simulations onto one GPU.
 * Requests wait in a FIFO queue and are admitted when a worker slot is free
 * and their device footprint (pse_footprint_bytes plus their particle
 * arrays) fits in the remaining budget.  An admitted request owns a handle
 * on its own stream, keeps its state resident and runs all its steps
 * (pse_constrained_step with Philox noise keyed by (seed, step)); several
 * admitted requests run at once and their kernels overlap on the device.
 * The completion time of every step is recorded (per-step latency).  All
 * server functions are thread-safe.  Host arrays are copied at submission.
 */
typedef struct pse_server pse_server;

typedef struct pse_request {
  int64_t n;               /* particles                                       */
  double box, radius, viscosity, kT, tol;
  int32_t grid;            /* FFT grid (see pse_params.grid)                  */
  int32_t precision;       /* PSE_FP64 or PSE_MIXED                           */
  double gmres_tol;        /* 0 = library default                             */
  double lanczos_tol;      /* 0 = library default                             */
  int32_t steps;           /* mid-point steps to run                          */
  double dt;
  uint64_t seed;
  const double *x0;        /* host double[n][3] initial positions             */
  const double *FL;        /* host double[n][6] forces/torques, or NULL       */
} pse_request;

typedef struct pse_request_info {
  int64_t id;
  int32_t status;          /* 0 ok, >0 warning, <0 error code                 */
  int32_t steps_done;
  size_t bytes;            /* admitted footprint                              */
  double t_submit, t_admit, t_done;   /* seconds since server creation       */
} pse_request_info;

typedef struct pse_server_info {
  size_t budget, used, peak_used;
  int32_t active, peak_active, queued;
  int64_t completed, failed;
  double particle_steps;   /* sum of n * steps over completed requests        */
  double elapsed;          /* seconds since server creation                   */
} pse_server_info;

/* budget_bytes = 0: 90 % of the free device memory.  max_active worker
 * slots (1..64) on the current device. */
int pse_server_create(size_t budget_bytes, int max_active, pse_server **out);

/* Queue a request (non-blocking).  PSE_ERR_NOMEM if it can never fit. */
int pse_server_submit(pse_server *s, const pse_request *r, int64_t *id);

/* Block until the request has finished; info may be NULL. */
int pse_server_wait(pse_server *s, int64_t id, pse_request_info *info);

/* Final positions (host double[n][3]) and per-step latencies in ms (host
 * double[steps]) of a finished request; either pointer may be NULL. */
int pse_server_result(pse_server *s, int64_t id, double *x_out, double *step_ms);

/* Message of a failed request: the library's error text (the failing HIP
 * call or check and where it was made).  "" while the request has not
 * failed or for an unknown id; valid until the request is released. */
const char *pse_server_error(pse_server *s, int64_t id);

/* Forget a finished request. */
int pse_server_release(pse_server *s, int64_t id);

int pse_server_stats(pse_server *s, pse_server_info *out);

/* Run every queued request to completion, then stop the workers. */
int pse_server_destroy(pse_server *s);

/* Message for the last failure on this handle (or of the last failed create
 * when h is NULL).  Never NULL. */
const char *pse_last_error(const pse_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* PSE_H */
