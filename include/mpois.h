/*
 * mpois -- fast direct Poisson solver for MI355X (gfx950), C ABI.
 *
 * Solves the discrete Poisson equation  Lap(phi) = g  (Eq. 1 of the paper, in
 * 1, 2 or 3 dimensions) on a uniform box by the three-step method of
 * Section 2.1: forward transforms of Table 2 along every axis, division of
 * every coefficient by the sum of the per-axis eigenvalues (Section 2.3, from
 * Table 3 for the pseudo-spectral approximation or Table 4 for second-order
 * finite differences), and the backward transforms.
 *
 * Conventions common to all calls
 *  - Every function returns an mpois_status; 0 (MPOIS_OK) is success.  Output
 *    parameters are written only on success.
 *  - Arrays are C-contiguous, shape (n[0][, n[1][, n[2]]]), the last axis
 *    contiguous.  rhs and phi are device pointers owned by the caller.
 *  - Element type: double for MPOIS_F64 and MPOIS_F32_REFINE, float for
 *    MPOIS_F32.
 *  - Streams are passed as `void*` holding a hipStream_t (NULL = the default
 *    stream).  Execution is asynchronous on that stream; nothing is allocated
 *    and the host is not synchronised by mpois_execute / mpois_execute_batch.
 *  - A plan may be used by one stream at a time; distinct plans are
 *    independent.
 *
 * Environment variables read by the library
 *  - MPOIS_TUNE_CACHE=<file>: the autotuner's decisions are read from and
 *    appended to this file (keyed by gfx arch, CU count, HIP version and the
 *    library's build hash).
 *  - MPOIS_LOG=1: the autotuner prints every candidate's time and its choice.
 *  - MPOIS_TRACE=1: roctx ranges around the library's calls and the phases of
 *    a solve (solve, residual, batch solve, batch residual), for
 *    rocprofv3 --marker-trace.
 *  - Test hooks: MPOIS_NO_SPEC=1 (no kernels compiled for one transform),
 *    MPOIS_NO_PLANE=1 (no plane kernels), MPOIS_TUNE_VARIANT=k (the tuner
 *    times only radix plan k), MPOIS_FAULT_ALLOC=1 (device allocations fail).
 */
#ifndef MPOIS_H
#define MPOIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPOIS_OK = 0,
  MPOIS_ERR_INVALID = 1,        /* bad argument (shape, spacing, pointer, aliasing) */
  MPOIS_ERR_UNSUPPORTED = 2,    /* valid request this library does not implement */
  MPOIS_ERR_NOMEM = 3,          /* device allocation failed */
  MPOIS_ERR_DEVICE = 4,         /* no usable GPU, or a HIP call failed */
  MPOIS_ERR_NOT_CONVERGED = 5,  /* refinement ended above rtol (phi holds the last iterate) */
  MPOIS_ERR_NONFINITE = 6       /* the residual norm is NaN or infinite */
} mpois_status;

/* Boundary condition of one face.  Periodic must be on both faces of an axis;
 * Dirichlet and Neumann may differ between the two faces. */
typedef enum { MPOIS_PERIODIC = 0, MPOIS_DIRICHLET = 1, MPOIS_NEUMANN = 2 } mpois_bc;

/* Axis codes of the host helpers mpois_axis_eigenvalues / mpois_axis_plan: an
 * mpois_bc when both faces agree, else Dirichlet on the low face (index 0) and
 * Neumann on the high face (DN), or the reverse (ND).  Such an axis has the
 * eigenfunctions sin / cos((k+1/2) pi x/L) (beyond Tables 2-4 of the paper):
 * vertex grids transform by DST-III / DCT-III forward and DST-II / DCT-II
 * backward (unknowns: the interior nodes and the Neumann end node, L = n h),
 * staggered grids by DST-IV / DCT-IV both ways (L = n h); the finite-difference
 * eigenvalues are -(2 sin(pi (2k+1)/(4n))/h)^2. */
#define MPOIS_AXIS_DN 3
#define MPOIS_AXIS_ND 4

/* Grid of Section 2.1: vertex = the paper's "regular" grid (Dirichlet: interior
 * nodes x_j=(j+1)L/(n+1); Neumann: boundary nodes included, x_j=jL/(n-1));
 * staggered: x_j=(j+1/2)L/n.  Ignored on periodic axes (x_j=jL/n). */
typedef enum { MPOIS_VERTEX = 0, MPOIS_STAGGERED = 1 } mpois_grid;

/* Eigenvalues of Table 3 (pseudo-spectral) or Table 4 (2nd-order differences). */
typedef enum { MPOIS_SPECTRAL = 0, MPOIS_FD2 = 1 } mpois_approx;

/* Working precision: FP64; FP32; FP32 transforms with FP64 residual refinement
 * (finite differences only). */
typedef enum { MPOIS_F64 = 0, MPOIS_F32 = 1, MPOIS_F32_REFINE = 2 } mpois_prec;

/* Plan flags. */
#define MPOIS_FLAG_GRAPH 1u   /* capture the launch sequence once per (rhs, phi) pair and replay it */
#define MPOIS_FLAG_TUNE 2u    /* time the candidate kernel shapes at plan creation and keep the fastest */
#define MPOIS_FLAG_PROFILE 4u /* record an event after every launch of an execute (not captured) */
#define MPOIS_FLAG_F64_ARITH 8u /* MPOIS_F32_REFINE only: the transforms compute in FP64 on data that stays
                                   FP32 in memory (working array, residual); each stored value is then
                                   rounded relative to its own size, so a correction contracts the error
                                   by about the FP32 unit roundoff */

/* One grid.  ndim in 1..3; n[d] >= 1 (>= 2 on vertex axes with Neumann on both
 * faces); h[d] > 0 finite; bc[d][0] and bc[d][1] are the conditions of the low
 * face (index 0) and the high face of axis d (periodic on both or neither).
 * shift >= 0 is the Helmholtz sigma: the plan solves (Lap - sigma) phi = rhs
 * (0: Poisson); with sigma > 0 no problem is singular.  Entries beyond ndim are
 * ignored. */
typedef struct {
  int ndim;
  int64_t n[3];
  double h[3];
  int bc[3][2];   /* mpois_bc */
  int grid[3];    /* mpois_grid */
  double shift;   /* Helmholtz sigma >= 0 */
} mpois_grid_desc;

typedef struct mpois_plan_s* mpois_plan;

typedef struct {
  int iters;             /* FP32 solves performed by the last execute (1 + corrections) */
  double rel_resid;      /* ||g_c - L_h phi|| / ||g_c|| of the last result (FD plans; NaN otherwise) */
  double zero_mode_rhs;  /* weighted mean of g removed by the solve (0 when nonsingular) */
} mpois_info;

/* Build a plan for one grid (Sections 2.1-2.3, Tables 2-4).
 * approx: mpois_approx; prec: mpois_prec.  For MPOIS_F32_REFINE, max_iter is
 * the fixed number of FP64-residual corrections run by every execute (>= 1)
 * and rtol (>= 0; 0 disables the check) is compared with the relative residual
 * by mpois_get_info; both are ignored for the other precisions.
 * Allocates the plan's workspace and device tables on the current device.
 * Errors: INVALID (bad descriptor), UNSUPPORTED (spectral with refinement; an
 * axis no kernel shape can hold), DEVICE (no GPU), NOMEM. */
mpois_status mpois_plan_create(const mpois_grid_desc* grid, int approx, int prec, double rtol,
                               int max_iter, unsigned flags, mpois_plan* out);

/* Build one plan for `count` independent grids of the same ndim (1..2048),
 * solved together by mpois_execute_batch.  Same rules as mpois_plan_create
 * for every entry. */
mpois_status mpois_plan_create_batch(const mpois_grid_desc* grids, int count, int approx, int prec,
                                     double rtol, int max_iter, unsigned flags, mpois_plan* out);

/* Solve for one right-hand side: phi = Lap^{-1} rhs.  rhs is read-only;
 * rhs == phi (in place) is allowed except with MPOIS_F32_REFINE, which needs
 * rhs for the residual; partial overlap is INVALID.  When every axis is
 * periodic or Neumann the zero mode is set to zero: phi solves for g minus
 * its weighted mean (weights 1/2 on the end nodes of vertex Neumann axes, 1
 * elsewhere) and has zero weighted mean. */
mpois_status mpois_execute(mpois_plan plan, const void* rhs, void* phi, void* stream);

/* Solve for arrays that are views into larger arrays, e.g. the interior of a
 * halo-padded CFD field (Section 3: the right-hand side and the solution may
 * be a subset of a larger array with ghost cells).  rhs / phi point at element
 * (0, .., 0) of the grid; rhs_strides / phi_strides give ndim element strides,
 * row-major-like and non-overlapping: strides[ndim-1] >= 1 and strides[d] >=
 * strides[d+1] * n[d+1].  The views are read and written in place by the
 * first, last (and, for MPOIS_F64 / MPOIS_F32, every) sweep and by the
 * refinement residual; elements outside them are never touched.  rhs == phi
 * with equal strides is allowed except with MPOIS_F32_REFINE; overlapping
 * views otherwise are INVALID, as are bad strides.  Always enqueued eagerly
 * (the graph and profiling flags apply to mpois_execute).  mpois_get_info
 * reports on the views. */
mpois_status mpois_execute_view(mpois_plan plan, const void* rhs, const int64_t* rhs_strides, void* phi,
                                const int64_t* phi_strides, void* stream);

/* Projection step of an incompressible-flow solver (Section 5.1: the
 * pressure-correction step of each Runge-Kutta stage) on this plan's grid:
 *   Lap phi = div(u*) / adt,   u = u* - adt grad phi,   p = p + phi,
 * with second-order differences on the staggered (MAC) grid; adt is
 * alpha_k * dt of the stage (finite, > 0).
 * vel: host array of ndim device pointers; vel[d] is the velocity component
 *   normal to axis d, C order, the plan's shape except along axis d: n_d
 *   faces when that axis is periodic (face f on the low side of cell f, face
 *   n_d is face 0), n_d + 1 otherwise (faces 0 and n_d on the boundary).
 *   It holds u* on entry and the corrected velocity on return.  A Neumann
 *   boundary face keeps its value (no flux); on a Dirichlet face (phi = 0 on
 *   it) the gradient is +-2 phi / h from the adjacent cell.
 * p: pressure at the cells (plan shape, C order), updated in place.
 * phi: receives phi (plan shape, C order).
 * Every array has the plan's I/O type (float for MPOIS_F32, else double);
 * they are distinct device arrays that do not overlap (else INVALID).
 * Needs an MPOIS_FD2 plan without Helmholtz shift whose axes are all
 * periodic or staggered (else UNSUPPORTED).  When every axis is periodic or
 * Neumann, the mean of div(u*) is dropped (phi has zero mean) and the
 * corrected field keeps that mean as its divergence.
 * MPOIS_F64 / MPOIS_F32 plans form the divergence inside the first line pass
 * and correct p and the last axis's component inside the last; the other
 * components take one more kernel.  MPOIS_F32_REFINE plans form the
 * divergence into an FP64 array the plan allocates on its first call (NOMEM
 * if that fails), solve it with refinement and correct afterwards;
 * mpois_get_info then reports on that solve.  After an FP64 / FP32
 * projection mpois_get_info returns INVALID (no right-hand side array). */
mpois_status mpois_project(mpois_plan plan, void* const* vel, void* p, double adt, void* phi, void* stream);

/* Largest scratch the allocation-free execute uses (bytes per device). */
#define MPOIS_NOALLOC_SCRATCH_BYTES (65u << 20)

/* For callers that cannot allocate device memory while they run (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve as mpois_execute, but the scratch its kernels use -- the FP32
 * working array of an MPOIS_F32_REFINE plan (4 bytes per grid point), the
 * residual block partial sums and the reduced scalars -- lives in a static
 * device array of the library (MPOIS_NOALLOC_SCRATCH_BYTES, one copy per
 * device, held until the process ends) instead of the plan's workspace.
 * Allocates nothing and never synchronises; the plan's flags for graph
 * capture and profiling are ignored (it always enqueues its kernels).
 * Refinement plans up to 16,908,224 grid points (256^3 included) fit;
 * larger ones return UNSUPPORTED.  The plan must belong to the current device (else DEVICE).
 * All calls on one device share its scratch: calls that overlap in time on
 * one device (different streams, or other host threads) race and must be
 * serialised by the caller.  mpois_get_info reports on the last call. */
mpois_status mpois_execute_noalloc(mpois_plan plan, const void* rhs, void* phi, void* stream);

/* Solve every grid of a batch plan: rhs[i], phi[i] are the device arrays of
 * grid i (host arrays of `count` device pointers).  The work is ordered on
 * `stream`: within a sweep, the launches of different kernel shapes may run
 * on up to three streams the plan owns, forked from `stream` and joined back
 * to it by events, so work enqueued on `stream` afterwards sees the results
 * (and a capture of `stream` records them as parallel branches).  The
 * pointer arrays are validated and uploaded only when they change between
 * calls; with MPOIS_FLAG_GRAPH the whole sequence is captured once and
 * replayed. */
mpois_status mpois_execute_batch(mpois_plan plan, const void* const* rhs, void* const* phi, void* stream);

/* Residual report of the last execute (single-grid plans; for batch plans the
 * worst grid).  Synchronises `stream`.  Returns NOT_CONVERGED when rtol > 0 and
 * rel_resid > rtol, NONFINITE when the residual is not finite; *out is written
 * in both cases. */
mpois_status mpois_get_info(mpois_plan plan, void* stream, mpois_info* out);

/* Free the plan and everything it owns.  NULL is a no-op. */
mpois_status mpois_destroy(mpois_plan plan);

/* Device bytes owned by the plan (workspace and tables); 0 for NULL. */
size_t mpois_workspace_bytes(mpois_plan plan);

/* Per-launch timing of the last execute of a plan created with
 * MPOIS_FLAG_PROFILE: for launch i, ms[i] is the time between the end of the
 * previous launch (or the start of the execute) and its end, measured with HIP
 * events on the execute's stream; bytes[i] its algorithmic HBM bytes (each
 * input element read once, each output written once); kernel[i] the
 * line-transform kernel (generic shapes below 100, kernels specialised for
 * one transform from 200, plane kernels from 300), 100 for the residual, 101
 * for the reduction.
 * Writes min(cap, *count) entries; *count receives the number of launches.
 * Synchronises `stream`. */
mpois_status mpois_profile(mpois_plan plan, void* stream, int cap, double* ms, double* bytes, int* kernel,
                           int* count);

/* Static text for a status code. */
const char* mpois_status_string(mpois_status s);

/* Host-only helpers (no device needed). -------------------------------------- */

/* Check a descriptor as mpois_plan_create would, without touching the device. */
mpois_status mpois_validate(const mpois_grid_desc* grid, int approx, int prec, int max_iter);

/* lambda_k, k = 0..n-1, of one axis as used by the solver (Table 3 or 4,
 * unscaled, FP64), written to out[0..n-1].  bc: an axis code (mpois_bc or
 * MPOIS_AXIS_DN / MPOIS_AXIS_ND). */
mpois_status mpois_axis_eigenvalues(int bc, int grid, int approx, int64_t n, double h, double* out);

/* How one axis is transformed (bc: an axis code): forward/backward
 * line-transform kinds (0 real DFT to half-complex, 1 its inverse, 2 DCT-II,
 * 3 DCT-III, 4 DST-II, 5 DST-III, 6 DCT-I, 7 DST-I, 8 DST-IV, 9 DCT-IV),
 * complex DFT length M, work length P (P > M means a Bluestein convolution),
 * and the radices of the Stockham stages (up to `cap`; *nradix receives the
 * count). */
mpois_status mpois_axis_plan(int bc, int grid, int64_t n, int* kind_fwd, int* kind_bwd, int* M, int* P,
                             int* radices, int cap, int* nradix);

/* Shape of line-transform kernel `cfg` (the kernel ids reported by
 * mpois_profile): element size in bytes, line pairs per workgroup tile,
 * threads per workgroup, and the longest DFT work length -- or, for the
 * kernels specialised for one transform (ids 200 and up), its line length;
 * for the plane kernels that transform the last two axes of a small 3D grid
 * in one sweep (ids 300 and up: one workgroup per n x n plane), n / 2 pairs
 * and n.  INVALID if out of range. */
mpois_status mpois_kernel_shape(int cfg, int* elem_bytes, int* pairs, int* threads, int* max_len);

#ifdef __cplusplus
}
#endif

#endif /* MPOIS_H */
