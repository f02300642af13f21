/*
 * sa.h -- C ABI of the MI355X matrix-free global stability library.
 *
 * The library applies the linearised compressible Navier-Stokes operator
 * J(q0) (Section "Matrix free framework", eq. frechet: the operator N_lin
 * obtained by linearising N(q) about a base state q0) to perturbation
 * vectors, solves the Cayley systems (J - sigma I) x = b with restarted
 * GMRES (Section "Iterative solvers"), optionally right-preconditioned by a
 * block-Jacobi preconditioner (Section "Preconditioning"), and finds the
 * leading eigenpairs of J (eq. stability) with the implicitly restarted
 * Arnoldi method (Algorithm 1, eq. ritz_estimate) applied to the Cayley
 * transform C = (J - sigma I)^{-1} (J - mu I) (eq. cayley_transform,
 * eq. cayley_arnoldi).
 *
 * Conventions
 *  - Every pointer named *_dev is a device pointer (HIP memory on the
 *    context's device); *_host pointers are host memory.  The caller owns
 *    every buffer it passes; the library never frees caller memory.
 *  - Vectors are struct-of-arrays, x fastest:
 *        idx = ((var*Nz + k)*Ny + j)*Nx + i,
 *    var = (p, u, v, s) in 2D (Nz = 1) and (p, u, v, w, s) in 3D.
 *    n = nv*Nx*Ny*Nz entries.  Ny counts both wall rows (j = 0, Ny-1).
 *  - Perturbation vectors live in the interior subspace: the operator is
 *    P J P with P zeroing the wall rows; wall entries of inputs are ignored
 *    and wall entries of outputs are written as 0.
 *  - SA_F64 buffers are double*, SA_F32 buffers are float*.  SA_MIXED takes
 *    and returns double* and computes the inner work in float.
 *  - All work is ordered on the stream given to sa_create.  Calls that
 *    return host results (info / eigen structs) synchronise that stream
 *    first.  A context is not thread-safe; use one per host thread.
 *  - Return codes: 0 success; > 0 a result was produced but the requested
 *    tolerance was not met (the info struct tells which); < 0 an error, the
 *    outputs are unspecified and sa_last_error() describes it.
 */
#ifndef SA_H
#define SA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SA_OK = 0,
  SA_NOT_CONVERGED = 1, /* budget exhausted before the tolerance was met   */
  SA_EINVAL = -1,       /* bad argument (shape, size, null pointer, option) */
  SA_ENOMEM = -2,       /* device allocation failed                          */
  SA_EDEVICE = -3,      /* a HIP call failed                                 */
  SA_ESINGULAR = -4,    /* zero pivot in a block factorisation               */
  SA_ENONFINITE = -5,   /* NaN or Inf in an input or residual                */
  SA_ESTATE = -6        /* call out of order (e.g. apply before setup)       */
};

typedef enum { SA_F64 = 0, SA_F32 = 1, SA_MIXED = 2 } sa_prec;
typedef enum { SA_BC_PERIODIC = 0, SA_BC_WALL = 1 } sa_bc;
/* First derivatives of the discrete operator (Section "Governing equations",
 * last paragraph).  EXPLICIT: 6th-order central differences, 4th and 2nd
 * order on the two rows next to a wall.  COMPACT: the 6th-order compact
 * (tridiagonal) scheme of Lele the paper uses for its wave terms, on the
 * collocated grid, cyclic on periodic axes, with the 4th-order Pade row next
 * to a wall and the 3rd-order one-sided compact row at it.  Second
 * derivatives are the explicit ones in both. */
typedef enum { SA_SCHEME_EXPLICIT = 0, SA_SCHEME_COMPACT = 1 } sa_scheme;

typedef struct sa_ctx sa_ctx;

/* One base-flow problem (Section "Governing equations" and "Model problem").
 * The x (and z) axes are periodic with x_i = i Lx/Nx; the y axis is either
 * bounded by walls with y_j = -Ly/2 + j Ly/(Ny-1) (both walls on the grid)
 * or periodic.  Non-dimensional: rho_ref = T_ref = u_inf = delta = 1, so the
 * reference pressure is 1/(gamma M^2); mu_ref = 1/re (re <= 0: inviscid). */
typedef struct {
  int ndim;            /* 2 or 3                                        */
  int n[3];            /* Nx, Ny, Nz (Nz = 1 in 2D); each >= 7          */
  double len[3];       /* Lx, Ly, Lz                                    */
  int bc_y;            /* sa_bc of the y axis                           */
  double mach, re, pr, gamma, sutherland; /* sutherland = S/T_ref      */
  int scheme;          /* sa_scheme (0, the zero-initialised default:
                          explicit).  COMPACT computes each product
                          derivative-first, one system at a time, in a
                          context workspace of (ndim + 3)(ndim + 1) + 2 ndim
                          doubles per grid point; its kernels are not
                          autotuned (sa_get_jv_variant reports -1). */
  double stretch;      /* y-grid stretching beta >= 0 (Section "Model
                          problem": rows clustered where the velocity
                          gradients are largest).  0 (the zero-initialised
                          default): uniform rows.  beta > 0 needs walls in
                          y: the rows sit at y = (Ly/2) sinh(beta eta) /
                          sinh(beta), eta uniform on [-1, 1], and y
                          derivatives take the analytic metric (D_y =
                          D_eta / y', D_yy = D_etaeta / y'^2 - (y''/y'^2) D_y,
                          D_y the scheme's first derivative).  The
                          uniform-state kernels are not used then. */
} sa_problem;

typedef struct {
  int restart;         /* Krylov dimension m of GMRES(m); 1..128            */
  double tol;          /* stop when ||b - A x|| <= tol ||b||                */
  long max_matvec;     /* budget of operator applications (per system)      */
  int use_precond;     /* 1: right block-Jacobi preconditioning (after setup) */
  sa_prec prec;        /* F64: all FP64; F32: all FP32 (float buffers);
                          MIXED: FP64 iterative refinement around FP32 GMRES */
  double inner_tol;    /* MIXED: relative tolerance of each inner solve     */
  int max_outer;       /* MIXED: maximum refinement sweeps                  */
  int use_graph;       /* 1: each restart cycle (all its kernels, all shifts)
                          is captured once into a hipGraph and replayed; the
                          graph is cached in the context.  0: plain launches.
                          Results are identical either way.                 */
  int augment;         /* k >= 0: LGMRES(restart, k) (Section "Iterative
                          solvers": restart cycles augmented with error
                          approximations).  Each cycle runs `restart` Krylov
                          steps and then one step per stored correction of
                          the previous k cycles (newest first); a correction's
                          image under A is the difference of consecutive
                          residuals, so those steps cost no operator product.
                          0: plain GMRES(restart).  restart + k <= 128.     */
} sa_gmres_opts;

typedef struct {
  long iters;          /* Arnoldi steps (inner steps for MIXED)            */
  long matvecs;        /* operator applications (all precisions)           */
  long precond_applies;
  int cycles;          /* restart cycles (inner cycles for MIXED)          */
  int outer;           /* refinement sweeps (MIXED), else 0                */
  double relres;       /* final true relative residual (FP64 for MIXED)    */
  int status;          /* SA_OK or SA_NOT_CONVERGED for this system        */
} sa_gmres_info;

/* Preconditioners of the Cayley systems (Section "Preconditioning").
 * SA_PC_BLOCK_JACOBI: the paper's local block-Jacobi scheme, dense blocks of
 * bx x by x bz cells assembled from operator calls.
 * SA_PC_MEAN_FLOW: the operator of the base state averaged over the
 * periodic directions (x, and z in 3D), M(s) = P (J(q_bar) - s I) P, solved
 * exactly: it commutes with the periodic shifts, so it is solved mode by
 * mode in their Fourier basis, each mode's block banded in y and factored
 * by banded LU with partial pivoting (the Conclusions' direction of an
 * approximate operator built from operator calls).  Exact for bases that
 * do not vary along x and z; needs walls in y. */
typedef enum { SA_PC_BLOCK_JACOBI = 0, SA_PC_MEAN_FLOW = 1 } sa_pc_kind;

typedef struct {
  int bx, by, bz;          /* block size in cells (bz = 1 in 2D)          */
  double diag_add;         /* added to every block diagonal               */
  double noise_std;        /* std of the seeded N(0,1) noise added         */
  unsigned long long seed; /* Philox4x32-10 key for the noise             */
  sa_prec factor_prec;     /* SA_F32 (default use) or SA_F64 factors      */
  int kind;                /* sa_pc_kind; the block fields, diag_add,
                              noise_std and seed apply to block-Jacobi     */
} sa_precond_opts;

typedef struct {
  int nev;             /* wanted eigenpairs (1..32)                        */
  int ncv;             /* Arnoldi dimension m (nev+2 .. 64)               */
  double sigma, mu;    /* Cayley parameters                                */
  double tol;          /* tol_iram of the Ritz estimate test              */
  int max_restarts;
  sa_gmres_opts lin;   /* inner linear solves of the Cayley systems        */
} sa_eig_opts;

typedef struct {
  int nconv;           /* wanted Ritz pairs passing the Ritz estimate test */
  int restarts;
  long n_cayley;       /* Cayley applications (linear solves)             */
  long n_matvec;       /* operator applications, all inner solves          */
  long n_precond;
  double lam_re[32], lam_im[32];     /* eigenvalues of J (back-transformed) */
  double theta_re[32], theta_im[32]; /* Ritz values of C, by |theta|        */
  double ritz_est[32];               /* ||f_m|| |e_m^T y|                    */
  double resid[32];    /* ||J x - lam x|| / (|lam| ||x||) if vectors given   */
  double *evec_re_dev, *evec_im_dev; /* caller buffers of nev*n doubles or NULL */
  double wall_seconds; /* host wall time of this problem's solve              */
} sa_eig_result;

/* Context life cycle.  hip_stream is a hipStream_t (may be NULL: the null
 * stream).  *out is set to a new context or NULL on error. */
int sa_create(sa_ctx **out, void *hip_stream);
void sa_destroy(sa_ctx *ctx);
const char *sa_last_error(const sa_ctx *ctx);
/* Library version string. */
const char *sa_version(void);

/* Kernels of the operator product: a prefetching one (16 x 16 column tiles,
 * the next plane's loads in flight during the pointwise algebra) and a
 * plane-staging one (32 x 8 tiles, two waves per SIMD in FP32), each
 * marching over 32, 16, 4 or 1 z planes per workgroup (the shallow ones give
 * small 3D grids enough workgroups; in 2D the depth is irrelevant); and the
 * prefetching organisation specialised to base states whose pressure and
 * entropy are the same at every grid point (uniform thermodynamic state,
 * arbitrary velocity; sa_base_set detects this exactly): it reads only the
 * base-velocity data, and of those only the fields that vary in x or z
 * stream from memory.  On other base states the iso variants run the
 * precision's default kernel.  All give the same product to rounding. */
typedef enum {
  SA_JV_PREFETCH_Z32 = 0,
  SA_JV_PREFETCH_Z16 = 1,
  SA_JV_STAGE_Z16 = 2,
  SA_JV_STAGE_Z32 = 3,
  SA_JV_PREFETCH_Z4 = 4,
  SA_JV_PREFETCH_Z1 = 5,
  SA_JV_STAGE_Z4 = 6,
  SA_JV_STAGE_Z1 = 7,
  SA_JV_ISO_Z32 = 8,
  SA_JV_ISO_Z16 = 9,
  SA_JV_ISO_Z4 = 10,
  SA_JV_ISO_Z1 = 11,
  SA_JV_NVARIANTS = 12
} sa_jv_variant;

/* Set the base state q0 (eq. model_stabiity: J is linearised about q0).
 * q0_dev: nv*Npts doubles (wall rows included), copied into the context,
 * which also derives its FP32 shadow and pointwise thermodynamic fields.
 * Errors: SA_EINVAL (bad problem), SA_ENONFINITE (NaN/Inf or non-positive
 * pressure in q0), SA_ENOMEM. */
int sa_base_set(sa_ctx *ctx, const sa_problem *prob, const double *q0_dev);

/* Autotuning of the operator kernel.  sa_base_set times every sa_jv_variant
 * on the problem (a warm-up and three launches per variant and precision,
 * HIP events) and keeps the fastest per precision, unless a variant was
 * pinned with sa_set_jv_variant (variant -1 unpins and selects the
 * precision's default until the next sa_base_set; SA_JV_AUTOTUNE=0 in the
 * environment skips the timing).  sa_get_jv_variant returns the variant in
 * use (-1: default) and, if times_us is not NULL, fills
 * times_us[SA_JV_NVARIANTS] with the measured microseconds per launch (0
 * where not measured).  Errors:
 * SA_EINVAL (bad precision or variant). */
int sa_set_jv_variant(sa_ctx *ctx, sa_prec prec, int variant);
int sa_get_jv_variant(const sa_ctx *ctx, sa_prec prec, float *times_us);

/* y = (J(q0) - shift I) x for nrhs vectors stored one after another
 * (x_dev, y_dev: nrhs*n entries, double for SA_F64, float for SA_F32).
 * Section "Matrix free framework": the product N_lin x, computed exactly
 * (the tangent-linear of the discrete N) rather than by the finite quotient.
 * x and y must not overlap.  Errors: SA_ESTATE before sa_base_set,
 * SA_EINVAL (nrhs < 1, null pointer, SA_MIXED). */
int sa_op_apply(sa_ctx *ctx, sa_prec prec, int nrhs, const void *x_dev, void *y_dev,
                double shift);

/* Assemble and factor the preconditioner of opts->kind for nshift shifts.
 *
 * SA_PC_MEAN_FLOW: the base state is averaged over the periodic axes, its
 * operator's band coefficients are taken by 7 nv probes (operator calls on
 * the averaged base), and for every shift s and Fourier mode of the
 * periodic axes the mode's banded matrix (bandwidths 4 nv - 1, order
 * (Ny-2) nv) is factored by LU with partial pivoting in factor_prec, one
 * wavefront per (mode, shift), all in one launch.  The y axis must have
 * walls.  Memory, in complex entries of factor_prec per unknown of the
 * nshift (Nx/2+1) Nz (Ny-2) nv: 12 nv - 2 for the factorisation (L and U),
 * KU <= 8 nv - 1 for U packed to its common column extent, and with FP32
 * factors 4 nv - 1 + KU more for the step-pair copies the solve reads.
 *
 * SA_PC_BLOCK_JACOBI (Section "Preconditioning": blocks of the operator
 * assembled from operator calls).  Block b of shift s is
 *     B_b(s) = P_b J P_b^T + diag_add I + noise_std E_b - s I
 * on the block's interior DOFs, E_b seeded standard-normal (Philox4x32-10),
 * P_b the restriction to the block's DOFs; on its wall DOFs (which are not
 * unknowns of P J P) the block is the identity, with no noise or shift.
 * Blocks are extracted by coloured probing with the operator in the factor
 * precision (FP32 operator products for SA_F32 factors, FP64 for SA_F64),
 * formed in FP64 (unshifted blocks plus noise are kept in FP64 on the
 * device), rounded once to the factor precision and factored (LU with
 * partial pivoting), all blocks of all shifts in one launch.  Every axis
 * must be divisible by its block size, and along a periodic axis the block
 * count must be divisible by the probe colour count 1 + ceil(3/b);
 * nb = nv*bx*by*bz <= 128.  Errors: SA_ESTATE, SA_EINVAL, SA_ENOMEM,
 * SA_ESINGULAR (an exactly zero pivot; the factors are then unusable). */
int sa_precond_setup(sa_ctx *ctx, const sa_precond_opts *opts, int nshift,
                     const double *shifts_host);

/* z = P M(shift ishift)^{-1} r for nrhs vectors (double for SA_F64, float
 * for SA_F32): M the block diagonal of the block-Jacobi blocks, applied in
 * the factor precision, or the mean-flow operator (forward transforms,
 * banded substitutions with the factors converted to the vector precision,
 * inverse transforms; at most nshift vectors per call).  Wall entries of r
 * are ignored and those of z are 0.  Errors: SA_ESTATE before setup,
 * SA_EINVAL. */
int sa_precond_apply(sa_ctx *ctx, sa_prec prec, int ishift, int nrhs, const void *r_dev,
                     void *z_dev);

/* Solve (J - sigma_s I) x_s = b_s for nshift systems (eq. cayley_arnoldi's
 * linear system; Section "Iterative solvers": restarted GMRES or LGMRES, here
 * with classical Gram-Schmidt applied twice).  b_dev / x_dev hold nshift vectors
 * one after another; x is the initial guess on entry (zero it for x0 = 0)
 * and the solution on exit.  With use_precond, system s uses the factors of
 * shift s (nshift must equal the setup's).  info_host[nshift] is filled.
 * Returns SA_OK if every system converged, SA_NOT_CONVERGED otherwise. */
int sa_gmres_solve(sa_ctx *ctx, const sa_gmres_opts *opts, int nshift,
                   const double *sigma_host, const void *b_dev, void *x_dev,
                   sa_gmres_info *info_host);

/* Size of the device scratch array behind sa_gmres_solve_noalloc (one copy
 * per device, held until the process ends). */
#define SA_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* sa_gmres_solve for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same solve, argument
 * rules and results, but every workspace buffer (Krylov basis, small GMRES
 * state, reduction partials and counters) lives in a statically sized
 * device array of SA_NOALLOC_SCRATCH_BYTES instead of context-owned
 * allocations; the call performs no device allocation or free.  The caller
 * still passes b_dev and x_dev; the base state (and, with use_precond, the
 * factors) must already be set up by the allocating calls.  Restart cycles
 * run as plain launches (use_graph is ignored).  Every call on one device
 * shares that device's array and keeps the previous call's contents
 * (counters are cleared at the start of each call), so calls that overlap
 * on one device -- contexts on different streams -- race and must not be
 * issued concurrently.  Errors: those of sa_gmres_solve, and SA_EINVAL when
 * the workspace the solve needs, about (restart + augment + 2) * n * nshift
 * elements plus the small state, exceeds SA_NOALLOC_SCRATCH_BYTES. */
int sa_gmres_solve_noalloc(sa_ctx *ctx, const sa_gmres_opts *opts, int nshift,
                           const double *sigma_host, const void *b_dev, void *x_dev,
                           sa_gmres_info *info_host);

/* Leading eigenpairs of J for nprob problems (Algorithm 1 on the Cayley
 * transform; eigenvalues ordered by decreasing |theta|, theta = (lam - mu)/
 * (lam - sigma)).  ctxs[p] holds problem p's base state; v0_dev[p] its start
 * vector (n doubles).  res_host[nprob].  If all contexts share one stream
 * the problems run one after another; if their streams are pairwise
 * distinct they run concurrently, one host thread per problem (at most 16
 * at a time), so that the GPU overlaps their kernels.  Any other mix is
 * SA_EINVAL.  On an error the message of the failing problem is copied to
 * ctxs[0].  Returns SA_OK if all problems converged, SA_NOT_CONVERGED
 * otherwise. */
int sa_arnoldi_eigs(sa_ctx *const *ctxs, int nprob, const sa_eig_opts *opts,
                    const double *const *v0_dev, sa_eig_result *res_host);

#ifdef __cplusplus
}
#endif
#endif /* SA_H */
