/*
 * cs3d.h - C ABI of the MI355X direct solver for compact 27-point stencils.
 *
 * Method: Gonzales, Gryazin & Lee, "Scalable Algorithms for High-Order
 * Approximations on Three-Dimensional Compact Stencils" (arXiv 1912.03565).
 *
 * The solver computes U = A^{-1}(F - lift) for the 27-diagonal system of
 * eq. (stencil27) (Section 3.1): the weights (a, b, c, d) of plane offsets
 * -1, 0, +1 depend on the row's z index only.  Section 3.6 gives the solve:
 * a 2-D DST-I in x and y diagonalises every 9-point plane block, the modal
 * eigenvalues lambda = 4a cos(theta_n) cos(phi_m) + 2b cos(theta_n) +
 * 2c cos(phi_m) + d turn the system into N_x N_y independent tridiagonal
 * systems along z, each solved by LU without pivoting, and an inverse DST
 * returns U.
 *
 * Problem (Section 1, eq. problem/bc): u_xx + u_yy + u_zz + k(z)^2 u = f, or
 * the convection-diffusion equation u_xx + u_yy + u_zz + gamma u_z = f
 * (Section 3.5), on a box with N_alpha interior points and
 * h_alpha = L_alpha/(N_alpha+1) (Section 2); u = 0 on the x and y faces and
 * Dirichlet data g on the two z faces.  With desc.sides = CS3D_SIDES_NEUMANN the x and
 * y faces carry du/dn = 0 instead (the extension Section 1 mentions): the side nodes
 * are unknowns too, closed by even reflection, and a DCT-I replaces the DST-I.
 *
 * Conventions shared by every entry point:
 *  - Layout: x fastest.  Interior arrays hold nx*ny*nz doubles with point
 *    (i, j, l) (1-based) at (i-1) + nx*((j-1) + ny*(l-1)), the paper's row order.
 *    Closed-grid arrays hold (nx+2)*(ny+2)*(nz+2) doubles with point (i, j, l)
 *    (0-based, boundary included) at i + (nx+2)*(j + (ny+2)*l).  z-face data are
 *    closed planes of (nx+2)*(ny+2) doubles, ring included.
 *  - Neumann sides: the x and y side nodes are unknowns, so "interior" arrays hold
 *    (nx+2)*(ny+2)*nz doubles with node (i, j, l) (i, j 0-based, l 1-based) at
 *    i + (nx+2)*(j + (ny+2)*(l-1)); closed-grid arrays and z-face planes keep their
 *    shapes (every x/y node of the closed grid is then a point of the system).
 *  - Several right-hand sides are stored back to back (stride = one array).
 *  - Complex plans (desc.k2_im != NULL): nrhs counts complex right-hand sides and every
 *    complex array is planar, the real part followed by the imaginary part, each of the
 *    documented real shape; so f holds nrhs x 2 closed grids, u nrhs x 2 interior arrays,
 *    z-face data nrhs x 2 planes (right-hand side r: real part at array 2r, imaginary at
 *    2r+1).
 *  - Pointers named dev_* are device (HIP) pointers; everything else is host.
 *  - The caller owns every data buffer and the workspace; a plan owns only its
 *    small device tables.  Nothing is allocated during a solve.
 *  - All solve calls are asynchronous on the given HIP stream (NULL = default
 *    stream).  cs3d_get_stats synchronises that stream.
 *  - Errors are returned as cs3d_status codes; nothing aborts or throws.
 *  - A plan is not thread-safe; distinct plans are.
 */
#ifndef CS3D_H
#define CS3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs3d_plan_s* cs3d_plan;
typedef struct cs3d_batch_s* cs3d_batch;

typedef enum {
  CS3D_OK = 0,
  CS3D_E_INVAL = 1,          /* bad argument: null pointer, size, spacing, scheme */
  CS3D_E_NOMEM = 2,          /* a plan table could not be allocated */
  CS3D_E_DEVICE = 3,         /* a HIP call failed */
  CS3D_E_SINGULAR = 4,       /* a zero or non-finite pivot was met (from cs3d_get_stats) */
  CS3D_E_NOTCONVERGED = 5,   /* refinement did not reach its residual target */
  CS3D_E_UNSUPPORTED = 6,    /* valid request the library does not serve */
  CS3D_E_WORKSPACE = 7,      /* workspace missing or too small */
  CS3D_E_TOO_LARGE = 8       /* cs3d_solve_static: the solve needs more than its scratch */
} cs3d_status;

typedef enum {
  CS3D_HELM2 = 2,     /* 2nd-order 7-point Helmholtz, Section 3.2 (eq. scheme2) */
  CS3D_HELM4 = 4,     /* 4th-order compact Pade Helmholtz, Sections 2.1 and 3.3 */
  CS3D_HELM6 = 6,     /* 6th-order compact Helmholtz, Sections 2.1.1 and 3.4 (uniform h) */
  CS3D_CD4 = 14,      /* 4th-order compact convection-diffusion, Section 3.5 */
  CS3D_WEIGHTS = 99   /* any stencil of the class eq. stencil27: caller-given weights */
} cs3d_scheme;

typedef enum {
  CS3D_FP64 = 0,        /* every stage in FP64 */
  CS3D_MIXED_FP32 = 1   /* FP32 line transforms and FP32 intermediates in HBM, tridiagonal
                           LU arithmetic in FP64 (eigenvalues, pivots, c' and d' formed in
                           FP64; c' stored in FP64, d' rounded to FP32 between the forward
                           and the backward sweep, like the other FP32 intermediates), FP64
                           27-point residual (computed in FP64, handed to the FP32 correction
                           solve in FP32) and FP64 update of u */
} cs3d_precision;

/* Conditions on the x and y faces. */
enum {
  CS3D_SIDES_DIRICHLET = 0, /* u = 0 (Section 1, eq. bc); DST-I in x and y */
  CS3D_SIDES_NEUMANN = 1    /* du/dn = 0: the scheme's rows also on the side nodes, the
                               values beyond a side mirrored about it (u_{-1} = u_1,
                               likewise f); DCT-I in x and y.  Full order for solutions
                               whose odd normal derivatives vanish on the sides (the
                               cosine class), as the Dirichlet path's order asks the even
                               derivatives of f to vanish there.  FP64, real k, plans only;
                               nx + 2 and ny + 2 at most 1023 (FFT path where nx + 1 is a
                               power of two in 64..512, direct cosine sums otherwise) */
};

/* Conditions on the z faces. */
enum {
  CS3D_ZFACES_DIRICHLET = 0, /* u = g (the data of cs3d_solve lifted into rows 1 and nz) */
  CS3D_ZFACES_ROBIN = 1      /* alpha u_z + beta u = g (Section 1, eq. bc, real alpha, beta):
                                the z-face nodes z_0 and z_{nz+1} are unknowns too, so
                                interior arrays hold nz + 2 planes (z_0 .. z_{nz+1}); each
                                face node carries the scheme's row, the ghost plane beyond it
                                eliminated by u(z_0 - h) = u(z_0 + h) - 2h u_z - (h^3/3) u_zzz
                                with u_z from the condition and u_zzz from the equation
                                (fourth order near the faces: HELM2 keeps 2, HELM4 4, HELM6
                                drops to 4).  The modal systems keep N_z + 2 rows and only
                                their first and last rows change.  k2, k2_z (required) and
                                k2_zz then hold nz + 4 samples at z_{-1} .. z_{nz+2}.  HELM2 /
                                HELM4 / HELM6, FP64, real k, Dirichlet sides, plans only
                                (else E_UNSUPPORTED); cs3d_residual is unsupported */
};

typedef struct {
  int nx, ny, nz;          /* interior points per axis (Section 2); >= 1.  The FFT line
                              transform serves N+1 in {64,...,1024} (powers of two), a
                              direct sine-sum transform any other N <= 1024.  HELM6 needs
                              N >= 4 per axis (its fourth differences). */
  double hx, hy, hz;       /* grid steps > 0.  HELM6 requires hx == hy == hz (Section 2.1.1). */
  int scheme;              /* cs3d_scheme */
  const double* k2;        /* host, nz+2 samples of k(z)^2 at z_0..z_{nz+1}; Helmholtz schemes */
  const double* k2_z;      /* host, nz+2 samples of (k^2)_z; HELM6 only (analytic or O(h^4)) */
  const double* k2_zz;     /* host, nz+2 samples of (k^2)_zz; HELM6 only */
  double gamma;            /* convection coefficient; CD4 only */
  const double* weights;   /* host, nz*3*4 doubles: row l (0..nz-1), plane offset o (-1,0,+1 as
                              0,1,2), then (a, b, c, d) of eq. stencil27; CS3D_WEIGHTS only */
  int precision;           /* cs3d_precision */
  int refine_steps;        /* mixed precision: number of FP64 residual refinement steps (>= 0) */
  int max_rhs;             /* largest nrhs a solve will be called with (>= 1) */
  const double* k2_im;     /* host, nz+2 samples of Im k(z)^2, or NULL (real k).  Non-NULL makes
                              the plan complex (absorbing media; Section 1 allows complex k):
                              k2 then holds Re k^2, the weights, modal eigenvalues, tridiagonal
                              solves and every field are complex.  HELM2 / HELM4 / HELM6 with
                              CS3D_FP64 only (else E_UNSUPPORTED). */
  const double* k2_z_im;   /* host, nz+2 samples of Im (k^2)_z; complex HELM6 only */
  const double* k2_zz_im;  /* host, nz+2 samples of Im (k^2)_zz; complex HELM6 only */
  int sides;               /* CS3D_SIDES_DIRICHLET (0, the default of a zeroed desc) or
                              CS3D_SIDES_NEUMANN; Neumann with mixed precision, complex k or
                              a batch gives E_UNSUPPORTED, with nx + 2 or ny + 2 > 1023
                              E_INVAL */
  int zfaces;              /* CS3D_ZFACES_DIRICHLET (0, the default of a zeroed desc) or
                              CS3D_ZFACES_ROBIN */
  double robin_alpha[2];   /* Robin z faces: alpha of the faces z = L_z^l and z = L_z^r
                              (finite, non-zero) */
  double robin_beta[2];    /* Robin z faces: beta of the two faces (finite) */
} cs3d_desc;

typedef struct {
  double min_abs_pivot;    /* smallest |pivot| of the tridiagonal LU over the last solve */
  int64_t bad_pivots;      /* zero or non-finite pivots met in the last solve */
  int refine_done;         /* refinement steps performed by the last mixed solve */
  double residual_history[8]; /* FP64 ||F - A U||_2 / ||F||_2 after the initial solve and after
                                 each refinement step (mixed path; NaN where not computed) */
  double last_solve_ms;    /* device time of the last solve, from HIP events */
  double stage_ms[8];      /* mean device time per solve of each pass, over the solves since the
                              last cs3d_reset_timers (at most the last 128): FP64 path
                              [0] RHS operator, [1] x-DST, [2] y-DST + forward elimination,
                              [3] back substitution + inverse y-DST, [4] inverse x-DST */
  int stage_count;         /* number of passes reported in stage_ms */
  int timed_solves;        /* solves averaged into stage_ms */
} cs3d_stats;

/* Build a plan: the stencil weights of every row (Sections 3.2-3.5), modal cosine
 * tables and transform twiddles, uploaded once to small plan-owned device tables.
 * desc and the host arrays it points to are only read during this call.
 * Errors: E_INVAL (bad sizes, spacings, scheme, missing k2/k2_z/k2_zz/weights,
 * HELM6 with unequal h or N < 4), E_NOMEM, E_DEVICE. */
cs3d_status cs3d_plan_create(const cs3d_desc* desc, void* hip_stream, cs3d_plan* out_plan);

/* Free the plan's device tables.  NULL is accepted. */
cs3d_status cs3d_plan_destroy(cs3d_plan plan);

/* Bytes of device workspace a solve with nrhs right-hand sides needs (0 on error). */
size_t cs3d_workspace_bytes(cs3d_plan plan, int nrhs);

/* Hand the plan a caller-owned device workspace (256-byte aligned) that stays
 * valid until the next cs3d_set_workspace or cs3d_plan_destroy.
 * Errors: E_INVAL (NULL plan or pointer, misaligned). */
cs3d_status cs3d_set_workspace(cs3d_plan plan, void* dev_workspace, size_t bytes);

/* Solve for nrhs right-hand sides (1 <= nrhs <= max_rhs) from f on the closed grid.
 * The scheme's RHS operator is applied to f (Sections 3.2-3.5; the 6th-order one as
 * documented in the design notes), the z-face data are lifted into the first and last
 * rows through the plane-offset weights, and the solution is written to the interior
 * array dev_u.  dev_g_lo / dev_g_hi may be NULL (zero data).
 * Robin z faces (desc.zfaces = CS3D_ZFACES_ROBIN): dev_g_lo / dev_g_hi hold the data g of
 * alpha u_z + beta u = g (closed planes, zero ring), and dev_u receives nz + 2 planes, the
 * face nodes z_0 and z_{nz+1} included; f keeps its closed-grid shape.
 * Errors: E_INVAL (NULL plan, f or u; nrhs out of range; scheme CS3D_WEIGHTS, which has
 * no RHS operator - use cs3d_solve_assembled), E_WORKSPACE, E_DEVICE. */
cs3d_status cs3d_solve(cs3d_plan plan, int nrhs, const double* dev_f, const double* dev_g_lo,
                       const double* dev_g_hi, double* dev_u, void* hip_stream);

/* cs3d_solve for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same passes as cs3d_solve, with the
 * workspace in a static device array of CS3D_STATIC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends (the plan's own workspace, if set, is not
 * used or touched).  Call with the plan's device current.  No per-pass timing is recorded
 * (cs3d_get_stats still reports pivots, residuals and the solve time).  Nothing is
 * allocated: no hipMalloc/hipFree, no events, no library allocations.
 * Every call on one device shares that device's scratch: calls that overlap on a device
 * (other streams, other host threads, other plans) race and must be ordered by the caller.
 * The scratch keeps the last call's contents; no pass reads it before writing it.
 * Errors: as cs3d_solve, plus E_TOO_LARGE when cs3d_workspace_bytes(plan, nrhs) exceeds
 * CS3D_STATIC_SCRATCH_BYTES (64 MiB: for instance one FP64 right-hand side up to about 159^3). */
#define CS3D_STATIC_SCRATCH_BYTES (64u << 20)
cs3d_status cs3d_solve_static(cs3d_plan plan, int nrhs, const double* dev_f, const double* dev_g_lo,
                              const double* dev_g_hi, double* dev_u, void* hip_stream);

/* Solve A U = F for an interior right-hand side F already assembled by the caller
 * (any scheme; z-face data, if any, already lifted).  dev_F and dev_u are interior arrays.
 * Errors: as cs3d_solve. */
cs3d_status cs3d_solve_assembled(cs3d_plan plan, int nrhs, const double* dev_F, double* dev_u,
                                 void* hip_stream);

/* FP64 residual of eq. stencil27: dev_r = F - A U over the interior, with F the scheme's
 * RHS operator applied to dev_f (or dev_F itself when dev_f_is_assembled != 0) and the
 * z-face data taking the place of the boundary planes of U.
 * Errors: as cs3d_solve; E_UNSUPPORTED for complex plans. */
cs3d_status cs3d_residual(cs3d_plan plan, int nrhs, const double* dev_f, int dev_f_is_assembled,
                          const double* dev_g_lo, const double* dev_g_hi, const double* dev_u,
                          double* dev_r, void* hip_stream);

/* Statistics of the last solve on this plan; synchronises the plan's last stream.
 * Returns E_SINGULAR when the last solve met a zero or non-finite pivot (the stats are
 * still filled), E_NOTCONVERGED when a mixed solve ended above its residual target. */
cs3d_status cs3d_get_stats(cs3d_plan plan, cs3d_stats* out_stats);

/* Restart the per-pass timing average reported by cs3d_get_stats.  Errors: E_INVAL. */
cs3d_status cs3d_reset_timers(cs3d_plan plan);

/* Launch-shape choices.  Each has a default that needs no tuning; cs3d_autotune and
 * cs3d_batch_autotune time the candidates on the caller's data and keep the fastest.
 * zchunk, xpersist, yrhs, order and graph do not change the arithmetic (results are bitwise
 * the same for every value); ywpl selects another radix split of the y-line FFT, which
 * changes the rounding of the transform only, and pack runs other kernels with the same
 * arithmetic per line, whose results agree to rounding (the compiler may fuse multiplies
 * and adds differently there). */
typedef struct {
  int zchunk;    /* z-planes per workgroup of the z-marching passes (RHS operator and, on the
                    mixed path, the FP64 residual): 8..512, default 32, for nz >= 512
                    64 (FP64) or 128 (mixed) */
  int xpersist;  /* x passes of a plan: 1 = a resident set of workgroups walks all tiles
                    (default), 0 = one workgroup per tile */
  int ywpl;      /* y passes of a plan where N_y+1 is 512 or 1024: waves per line, 1 or 2
                    (default 2 for 1024, 1 otherwise; other sizes always use 1) */
  int order;     /* batches: 1 = members ordered by decreasing cost per work item in every
                    pass, so the longest items start first (default); 0 = order given */
  int graph;     /* batches: 1 = the passes of a solve are captured once into a HIP graph and
                    replayed (default); 0 = launched one by one, with per-pass timing */
  int yrhs;      /* y passes of a plan: right-hand sides per workgroup, 1, 2 or 4 (default 1
                    for FP64, 2 for mixed precision).
                    Their tridiagonal systems share the modal eigenvalues, the pivots and
                    each read of c'; transform sizes whose lanes hold 16 modes use 1. */
  int xwpl;      /* x passes of a plan where N_x+1 is 512 or 1024: waves per line, 1 or 2
                    (1024 threads per workgroup, half a line per lane); other sizes use 1 */
  int pack;      /* batches: 1 = in the x and y passes a wave carries 4 lines of a 64-point
                    or 2 lines of a 128-point transform (the lanes its FFT uses), 0 = one
                    line per wave (default: the packed kernels hold more registers, which
                    a batch of large members alone does not repay) */
} cs3d_tuning;

/* Current launch-shape choices of a plan.  Errors: E_INVAL (NULL argument). */
cs3d_status cs3d_get_tuning(cs3d_plan plan, cs3d_tuning* out);

/* Set the launch-shape choices of a plan (order, graph and pack are ignored).
 * Errors: E_INVAL (NULL argument or a field out of range). */
cs3d_status cs3d_set_tuning(cs3d_plan plan, const cs3d_tuning* tuning);

/* Time every candidate of each launch-shape choice on real solves of the caller's data
 * (reps timed solves per candidate after one warm-up solve; each choice is judged by the
 * device time of the passes it affects) and keep the fastest.  The arguments are those of
 * cs3d_solve; dev_u receives a solution.  Synchronises the stream.  *out_best (may be NULL)
 * receives the choice, *out_ms (may be NULL) the mean time of one solve with it.
 * Errors: as cs3d_solve; E_INVAL for reps < 1. */
cs3d_status cs3d_autotune(cs3d_plan plan, int nrhs, const double* dev_f, const double* dev_g_lo,
                          const double* dev_g_hi, double* dev_u, void* hip_stream, int reps,
                          cs3d_tuning* out_best, double* out_ms);

/* Batches: n independent problems, each with its own sizes, steps, scheme and
 * coefficients (desc[i]; max_rhs is ignored, every member takes one right-hand side,
 * precision must be CS3D_FP64, k must be real, scheme must not be CS3D_WEIGHTS), solved
 * together.  Every
 * pass of Section 3.6 (RHS operator and lift, x-DST, y-DST with forward elimination, back
 * substitution with inverse y-DST, inverse x-DST) is ONE launch over the work items of all
 * members (tiles, line groups), taken by a resident set of workgroups from a device work
 * list; the five launches are captured once into a HIP graph and replayed.  Each member
 * goes through the per-item code of a plan built from its desc (default y-line split).
 * The z-face data are zero.
 * Errors: E_INVAL (n < 1, NULL pointers, a desc rejected by cs3d_plan_create or
 * CS3D_WEIGHTS), E_UNSUPPORTED (mixed precision, complex k), E_NOMEM, E_DEVICE. */
cs3d_status cs3d_batch_create(int n, const cs3d_desc* descs, void* hip_stream, cs3d_batch* out);

/* Bytes of device workspace of the batch (the members' workspaces back to back). */
size_t cs3d_batch_workspace_bytes(cs3d_batch batch);

/* Caller-owned device workspace, 256-byte aligned, at least cs3d_batch_workspace_bytes.
 * Errors: E_INVAL (NULL, misaligned), E_WORKSPACE (too small). */
cs3d_status cs3d_batch_set_workspace(cs3d_batch batch, void* dev_workspace, size_t bytes);

/* Solve every member: dev_f[i] is member i's closed-grid f, dev_u[i] its interior solution
 * (device pointers; the two pointer arrays are host arrays of n entries, read during the
 * call).  Asynchronous on hip_stream.  When a pointer differs from the previous call the
 * member table is uploaded again on that stream before the launches; the captured graph is
 * kept.  Calls on one batch must be ordered (one stream, or synchronised by the caller).
 * Errors: E_INVAL (NULL argument or member pointer), E_WORKSPACE, E_DEVICE. */
cs3d_status cs3d_batch_solve(cs3d_batch batch, const double* const* dev_f, double* const* dev_u,
                             void* hip_stream);

/* Statistics of the last batch solve (synchronises): min |pivot| over all members and the
 * total count of bad pivots; last_solve_ms; stage_ms of the five passes when the last solve
 * was launched pass by pass (graph = 0), else stage_count = 0.  Returns E_SINGULAR when a
 * member met a zero or non-finite pivot. */
cs3d_status cs3d_batch_get_stats(cs3d_batch batch, cs3d_stats* out_stats);

/* Pivot statistics of member i of the last batch solve (min_abs_pivot, bad_pivots; the
 * timing fields are those of the batch).  Errors: E_INVAL (index out of range). */
cs3d_status cs3d_batch_member_stats(cs3d_batch batch, int i, cs3d_stats* out_stats);

/* Launch-shape choices of a batch (zchunk, order, graph, pack; xpersist, ywpl, yrhs and
 * xwpl are ignored: batch passes are always resident, use the default waves per line and
 * carry the one right-hand side of each member).  Setting them
 * rebuilds the work lists and drops the captured graph.
 * Errors: E_INVAL (NULL argument or a field out of range), E_DEVICE. */
cs3d_status cs3d_batch_get_tuning(cs3d_batch batch, cs3d_tuning* out);
cs3d_status cs3d_batch_set_tuning(cs3d_batch batch, const cs3d_tuning* tuning);

/* As cs3d_autotune for a batch: times zchunk, pack and order candidates with per-pass timing,
 * then enables graph replay.  The arguments are those of cs3d_batch_solve.
 * Errors: as cs3d_batch_solve; E_INVAL for reps < 1. */
cs3d_status cs3d_batch_autotune(cs3d_batch batch, const double* const* dev_f, double* const* dev_u,
                                void* hip_stream, int reps, cs3d_tuning* out_best, double* out_ms);

/* Free the batch's member tables, work lists and graph.  NULL is accepted. */
cs3d_status cs3d_batch_destroy(cs3d_batch batch);

/* Static text for a status code. */
const char* cs3d_status_str(cs3d_status status);

/* Library version string. */
const char* cs3d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CS3D_H */
