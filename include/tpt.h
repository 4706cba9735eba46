/*
 * tpt — tensor-product–Thomas direct solver for constant-coefficient
 * Poisson and Helmholtz equations on staggered, non-uniform 3-D Cartesian
 * grids, for one AMD Instinct MI355X (gfx950).
 *
 * Method (arXiv 2603.09528, §2.2): the 1-D second-order operators along x and
 * y (Eq. poisson-fd2 / tridiagonal-coefficients) are symmetrised by the
 * diagonal similarity T~ = D^{1/2} T D^{-1/2} (Eq. reverse-similarity-
 * transform), eigendecomposed once per grid (T~ = Q~ Λ Q~^T), and applied as
 * dense transforms Q^{-1} = Q~^T D^{1/2}, Q = D^{-1/2} Q~ (Eq. q-from-tildeq)
 * over all grid lines at once (one GEMM per direction, end of §2.2.2).  The
 * remaining z direction is solved line by line with the Thomas algorithm,
 * shifted by λ_x,i + λ_y,j (§2.2.2, solution steps 2.1–2.5).  Helmholtz uses
 * the same eigenvectors with a constant modal shift.  The pressure gauge of a
 * singular Poisson problem follows §3: the modal unknown whose final pivot
 * vanishes is set to zero.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Fields are contiguous row-major arrays u[k][j][i] (x fastest) of
 *   Nz*Ny*Nx elements, where N_d is the unknown count of direction d: the
 *   cell count n[d], or n[d]-1 for a face-located direction between two
 *   Dirichlet walls.  Several right-hand sides are stored back to back.
 * - Device pointers are HIP device memory on the current device.  The
 *   library never frees memory it did not allocate.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Solve calls are stream-ordered and return before the GPU finishes,
 *   except where stated.
 * - Every function returns an int: TPT_OK (0) on success, TPT_PENDING (1)
 *   for a server request still running, or a negative TPT_ERR_* code.
 *   Nothing is thrown across the ABI.  tpt_last_error() returns a message
 *   for the last failing call of the calling thread.  A device fault raised
 *   by an earlier asynchronous launch surfaces as TPT_ERR_HIP on a later call.
 */
#ifndef TPT_H
#define TPT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TPT_OK = 0,
    TPT_PENDING = 1,
    TPT_ERR_INVALID = -1,       /* bad argument (sizes, faces, BC pairing, NULL) */
    TPT_ERR_UNSUPPORTED = -2,   /* valid but not supported combination */
    TPT_ERR_OOM = -3,           /* device allocation failed / over budget */
    TPT_ERR_ALIAS = -4,         /* rhs and out overlap */
    TPT_ERR_NOT_CONVERGED = -5, /* refinement stopped above its tolerance */
    TPT_ERR_HIP = -6,           /* a HIP runtime call failed */
    TPT_ERR_WORKSPACE = -7      /* workspace too small */
};

/* Homogeneous boundary conditions, per direction and side (§2.2.1: the first
 * and last rows of T are modified by the boundary conditions; periodic
 * boundaries add cyclic corners).  Periodic must be set on both sides. */
enum { TPT_BC_PERIODIC = 0, TPT_BC_NEUMANN = 1, TPT_BC_DIRICHLET = 2 };
/* Location of the unknowns along a direction on the staggered grid (§2.1):
 * cell centres (pressure) or faces (the velocity component normal to them). */
enum { TPT_LOC_CENTER = 0, TPT_LOC_FACE = 1 };
/* Poisson: L phi = f (Eq. poi_ns).  Helmholtz: (I - alpha L) u = f
 * (Eq. helmholtz_ns with alpha = gamma nu dt / 2, implicit in x, y and z). */
enum { TPT_POISSON = 0, TPT_HELMHOLTZ = 1 };
/* Directions a Helmholtz plan treats implicitly (§2.1: the implicit diffusion
 * operator L_I holds all three directions, y and z, or z alone; §3: the same
 * pipeline serves them, yz without the x transforms, z with the tridiagonal
 * solve only): (I - alpha L_I) u = f.  Poisson plans are always XYZ; YZ and
 * Z plans are FP64 only. */
enum { TPT_IMPLICIT_XYZ = 0, TPT_IMPLICIT_YZ = 1, TPT_IMPLICIT_Z = 2,
       TPT_IMPLICIT_NONE = 3 /* L_I = 0, fully explicit diffusion: Navier-Stokes
                                substeps only (tpt_ns_create); plans reject it */ };
/* Arithmetic of the transforms.  FP64: everything in double precision.
 * MIXED_FP32: transforms in FP32 MFMA; MIXED_BF16X3: transforms as three
 * BF16 MFMA products (hi*hi + hi*lo + lo*hi) with FP32 accumulation.  Both
 * mixed modes refine in FP64 (residual, update, Thomas and the null-line pin
 * in double precision).  Input and output are FP64 in every mode. */
enum { TPT_FP64 = 0, TPT_MIXED_FP32 = 1, TPT_MIXED_BF16X3 = 2 };

/* Plan flags. */
enum {
    TPT_FLAG_HOST_ONLY = 1, /* build the host-side operators and eigenbases
                               only (no device memory, no GPU needed); such a
                               plan can be inspected but not solved */
    TPT_FLAG_DENSE_X = 2,   /* apply the x eigenbasis by dense GEMM even where a
                               fast transform applies (see tpt_plan_transforms) */
    TPT_FLAG_DENSE_Y = 4,   /* the same for y */
    TPT_FLAG_FUSE_XY = 8,   /* FP64 plans whose x is a fast transform and y a
                               GEMM: run the two as one fused pass per
                               direction (tpt_plan_fused).  Reads and writes
                               the field once instead of twice, but on gfx950
                               it is slower than the separate passes (the
                               row transforms inside the GEMM are not hidden
                               behind its MFMAs), so it is not the default */
    TPT_FLAG_SEQ_THOMAS = 16, /* solve the z lines with the sequential kernel
                               (one lane per line) instead of the partitioned
                               one (segments joined by an interface system);
                               periodic z always uses the sequential kernel */
    TPT_FLAG_NO_CHECK = 32  /* skip the right-hand-side check of every solve
                               (one extra read of rhs on the device); the
                               compat_defect and nonfinite fields of tpt_info
                               are then -1 */
};

/* How a plan applies the eigenbasis of x or y (tpt_plan_transforms). */
enum {
    TPT_XFORM_GEMM = 0,     /* dense eigenbasis product (MFMA GEMM) */
    TPT_XFORM_FFT = 1,      /* uniform periodic: real Fourier transform */
    TPT_XFORM_DCT = 2,      /* uniform Neumann-Neumann, cell centres: DCT-II */
    TPT_XFORM_DST = 3,      /* uniform Dirichlet-Dirichlet, cell centres: DST-II */
    TPT_XFORM_NONE = 4      /* not transformed: the direction is explicit (TPT_IMPLICIT_*) */
};

typedef struct tpt_plan_s *tpt_plan;
typedef struct tpt_batch_s *tpt_batch;
typedef struct tpt_server_s *tpt_server;
typedef struct tpt_ns_s *tpt_ns;

typedef struct {
    int n[3];               /* cells per direction x, y, z (>= 2) */
    const double *faces[3]; /* host arrays of n[d]+1 strictly increasing face
                               coordinates (copied; caller keeps ownership).
                               A periodic direction must be uniform only if
                               its analytic basis is wanted; any spacing works */
    int bc[3][2];           /* [direction][lower, upper], TPT_BC_*; periodic must be paired
                               (a periodic z makes the Thomas lines cyclic) */
    int loc[3];             /* TPT_LOC_*; FACE needs periodic or Dirichlet-Dirichlet */
    int kind;               /* TPT_POISSON or TPT_HELMHOLTZ */
    double alpha;           /* Helmholtz coefficient (> 0), ignored for Poisson */
    int precision;          /* TPT_FP64, TPT_MIXED_FP32, TPT_MIXED_BF16X3 */
    double rtol;            /* mixed modes (adaptive): stop after correction k when, for every
                               right-hand side, c_k = ||e_k|| / ||x_k|| <= rtol, or k >= 2 and the
                               observed contraction rho = c_k / c_{k-1} < 1 gives an estimated
                               remaining error c_k rho / (1 - rho) <= rtol (e_k: the k-th
                               correction, x_k: the iterate after it; default 1e-12 if <= 0) */
    int max_refine;         /* mixed modes: cap on corrections (default 8 if <= 0) */
    int fixed_refine;       /* mixed modes: >= 0 runs exactly this many corrections with
                               no host synchronisation (stream-ordered, capturable);
                               -1 = adaptive, which synchronises the stream once per correction */
    int nrhs;               /* right-hand sides per solve call (>= 1), stored back to back */
    int flags;              /* TPT_FLAG_* */
    int implicit;           /* TPT_IMPLICIT_* (Helmholtz; default XYZ) */
} tpt_plan_desc;

/* Result of the last solve of a plan (valid after the stream has been
 * synchronised).  With several right-hand sides each ratio is the largest
 * over them. */
typedef struct {
    int iters;              /* corrections applied (0 for FP64) */
    double rel_correction;  /* ||e_last||_2 / ||x||_2 (mixed modes), 0 for FP64 */
    double rel_residual;    /* ||f - A x||_2 / ||f||_2 at the last refinement residual (mixed), or -1 */
    int null_line;          /* index i + Nx*j of the pinned modal line, or -1 */
    double compat_defect;   /* singular Poisson plans (null_line >= 0): |sum dV f| / sum dV |f|
                               over the finite values of rhs, dV the control volumes (the left
                               null vector of the operator, §2.2.1: D T is symmetric).  The
                               share of f that the §3 pin absorbs; 0 for a compatible f up to
                               rounding, 0 for non-singular plans, -1 with TPT_FLAG_NO_CHECK */
    int nonfinite;          /* number of NaN / Inf values in rhs (the output is then not
                               meaningful), -1 with TPT_FLAG_NO_CHECK */
} tpt_info;

/* Fill a descriptor with defaults (FP64 Poisson, centre-located, Neumann, nrhs 1). */
void tpt_plan_desc_init(tpt_plan_desc *desc);

/* Build a plan: 1-D operators with their boundary rows (§2.2.1), eigenbases
 * of x and y (analytic on uniform periodic / Neumann / Dirichlet directions,
 * otherwise the library's own symmetric tridiagonal QL, with a dense
 * Householder reduction for cyclic operators; initialization steps 1.1–1.3 of
 * §2.2.2) and their device copies.  Eigenbases are cached on the device and
 * shared by plans with identical (faces, BC, location).  Synchronous.
 * Errors: TPT_ERR_INVALID, TPT_ERR_UNSUPPORTED, TPT_ERR_OOM, TPT_ERR_HIP. */
int tpt_plan_create(const tpt_plan_desc *desc, tpt_plan *out);
int tpt_plan_destroy(tpt_plan plan);

/* Unknown counts {Nx, Ny, Nz} of a plan. */
int tpt_plan_shape(tpt_plan plan, int shape[3]);

/* Bytes of device workspace one tpt_solve call needs (all nrhs included). */
int tpt_plan_workspace_bytes(tpt_plan plan, size_t *bytes);

/* Host copy of the eigen data of direction dir (0 = x, 1 = y): lam[N] (Λ)
 * and, if Qt is not NULL, Q~ as an N x N row-major array (Qt[i*N + p] is
 * component i of eigenvector p).  Works on host-only plans. */
int tpt_plan_eigen(tpt_plan plan, int dir, double *lam, double *Qt);

/* Host copy of the 1-D operator of direction dir (0, 1, 2): sub-diagonal a,
 * diagonal b, super-diagonal c and control volumes vol, N entries each (for a
 * periodic direction a[0] and c[N-1] are the cyclic corners). */
int tpt_plan_operator(tpt_plan plan, int dir, double *a, double *b, double *c, double *vol);

/* kinds[0], kinds[1]: TPT_XFORM_* used for x and y (NONE where the plan
 * leaves the direction explicit).  A direction gets a fast
 * transform (§3: a uniform direction may use FFT-based transforms) when its
 * analytic basis is one of the three listed, its unknown count is a power of
 * two in 8..2048, and its TPT_FLAG_DENSE_* flag is not set; otherwise GEMM. */
int tpt_plan_transforms(tpt_plan plan, int kinds[2]);

/* *fused = 1 when an FP64 solve of the plan applies the x fast transform
 * inside the y GEMM's operand loads (steps 2.1 + 2.2 and 2.4 + 2.5 of §2.2.2
 * as one pass each: the field is read and written once instead of twice);
 * this needs TPT_FLAG_FUSE_XY, x a fast transform with N_x = 128 or 256 and
 * y a GEMM with N_y a multiple of 128 (0 for host-only plans). */
int tpt_plan_fused(tpt_plan plan, int *fused);

/* Solve A x = rhs for the plan's nrhs right-hand sides.  rhs, out: device
 * FP64 fields (nrhs * Nz*Ny*Nx each); rhs is read only and must not overlap
 * out (TPT_ERR_ALIAS).  workspace: device memory of at least
 * tpt_plan_workspace_bytes, or NULL to use a buffer owned by the plan
 * (allocated on first use).  Stream-ordered; the adaptive mixed mode
 * (fixed_refine = -1) synchronises `stream` once per correction.  A singular
 * Poisson right-hand side is solved with the gauge of §3 (pinned final
 * modal unknown); an incompatible component is absorbed by that pin and
 * reported as tpt_info.compat_defect.  Unless TPT_FLAG_NO_CHECK, every solve
 * first reads rhs once on the device for that defect and for NaN / Inf
 * values (tpt_info.nonfinite); the solve itself proceeds either way. */
int tpt_solve(tpt_plan plan, const double *rhs, double *out, void *workspace,
              size_t workspace_bytes, void *stream);

/* Info of the plan's last solve (call after synchronising its stream). */
int tpt_solve_info(tpt_plan plan, tpt_info *info);

/* Residual of the plan's operator, r = f - A x: A the 7-point Kronecker sum
 * of §2.2.2 with the plan's boundary rows (L for Poisson, I - alpha L_I for
 * Helmholtz, L_I holding only the implicit directions), evaluated in FP64
 * and stored in FP32 — the residual the mixed-precision refinement forms
 * (§4.1 checks an FP64 solve's residual at round-off).  x, f: nrhs device
 * arrays of Nx*Ny*Nz doubles each (x fastest, the solve's layout); r: the
 * same count of floats, caller-owned.  Enqueued on stream; allocates
 * nothing.  TPT_ERR_INVALID for a NULL or host-only plan or a NULL array. */
int tpt_residual(tpt_plan plan, const double *x, const double *f, float *r, void *stream);

/* tpt_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is a static device array of tpt_static_workspace_capacity()
 * bytes (64 MiB) in the library's code object, one per GPU, held until the
 * process ends; the call allocates nothing (the caller still passes rhs and
 * out).  Same arguments, results and info as tpt_solve with workspace.
 * A plan whose tpt_plan_workspace_bytes exceeds the capacity is rejected
 * with TPT_ERR_WORKSPACE.  Every call on one GPU shares that GPU's array:
 * calls that overlap on a GPU (other streams or threads) race on it, so the
 * caller serialises them. */
int tpt_solve_noalloc(tpt_plan plan, const double *rhs, double *out, void *stream);
size_t tpt_static_workspace_capacity(void);

/* ---- projection step (§2.1 staggered grid; §4.1 divergence test) ---------- */

/* The plan must be the cell-centred pressure Poisson problem of the grid
 * (every loc TPT_LOC_CENTER, nrhs 1) with periodic or Neumann boundaries; a
 * Neumann direction is bounded by walls with no penetration.  Velocity
 * components live on the faces normal to them (§2.1), x fastest:
 * u (Nz, Ny, Nux), v (Nz, Nvy, Nx), w (Nwz, Ny, Nx), with N face unknowns
 * in a periodic direction (face m between cells m and m+1, the last one
 * wrapping to cell 0) and N - 1 between walls (the interior faces; the wall
 * faces carry zero normal velocity and are not stored).  Device FP64
 * arrays; stream-ordered; TPT_ERR_INVALID for another kind of plan. */

/* div = D(u, v, w): the net flux out of each cell over its volume,
 * (u_{i+1/2} - u_{i-1/2}) / dx_i + (same in y and z), dx_i the cell width
 * (the finite-volume divergence whose composition with the gradient below
 * is the operator of Eq. poisson-fd2).  div: (Nz, Ny, Nx). */
int tpt_divergence(tpt_plan plan, const double *u, const double *v, const double *w, double *div,
                   void *stream);
/* (u, v, w) -= G phi in place: on the face between cells m and m+1,
 * (phi_{m+1} - phi_m) / dx_{m+1/2}, dx_{m+1/2} the distance of the two cell
 * centres.  phi: (Nz, Ny, Nx). */
int tpt_gradient_update(tpt_plan plan, const double *phi, double *u, double *v, double *w, void *stream);
/* The projection: solve L phi = D u* with the plan (§3 gauge), then
 * u = u* - G phi, so that D u = 0 up to rounding (and, in the mixed modes,
 * the refinement tolerance).  u, v, w are updated in place; phi receives the
 * pressure correction.  workspace: device memory of at least
 * tpt_project_workspace_bytes (the divergence and the solve's workspace). */
int tpt_project_workspace_bytes(tpt_plan plan, size_t *bytes);
int tpt_project(tpt_plan plan, double *u, double *v, double *w, double *phi, void *workspace,
                size_t workspace_bytes, void *stream);

/* ---- Navier-Stokes Runge-Kutta substep (§2.1, Eq. rk3) -------------------- */

/* A time-stepping context on the grid of `pressure` (a plan accepted by
 * tpt_project: cell-centred Poisson, periodic or Neumann boundaries, where a
 * Neumann direction is bounded by no-slip, no-penetration walls), with
 * kinematic viscosity nu (>= 0), time step dt (> 0) and implicit directions
 * TPT_IMPLICIT_{NONE, Z, YZ, XYZ} (L_I of §2.1; NONE = fully explicit
 * diffusion).  For implicit diffusion (nu > 0 required) the context builds
 * the FP64 Helmholtz plans (I - c_k L_I) of the three velocity components
 * for the three substep coefficients c_k = gamma_k nu dt / 2 (nine plans,
 * the eigenbases shared through the cache).  The pressure plan must outlive
 * the context; its precision is that of the pressure solve.  A new dt needs
 * a new context.  TPT_ERR_INVALID for a bad plan or parameter. */
int tpt_ns_create(tpt_plan pressure, double nu, double dt, int implicit, tpt_ns *out);
int tpt_ns_destroy(tpt_ns ns);
/* Device workspace of tpt_ns_substep: three velocity-sized right-hand sides,
 * one pressure-sized divergence and the largest solve workspace. */
int tpt_ns_workspace_bytes(tpt_ns ns, size_t *bytes);
/* Substep k (1, 2 or 3) of Eq. rk3 with alpha_k = (8/15, 5/12, 3/4),
 * beta_k = (0, -17/60, -5/12), gamma_k = alpha_k + beta_k and
 * c = gamma_k nu dt / 2:
 *   E^k   = A u^k + nu L_E u^k
 *   u**   = u^k + dt [alpha_k E^k + beta_k E^{k-1} + gamma_k (-G P + nu L_I u^k)]
 *   (I - c L_I) u* = u** - c L_I u^k            (u* = u** when L_I = 0)
 *   L Phi = D u* / (gamma_k dt),  u^{k+1} = u* - gamma_k dt G Phi
 *   P^{k+1/2} = P^{k-1/2} + Phi - c L_I Phi
 * A u = -div(u (x) u) is the symmetry-preserving second-order finite-volume
 * advection (kinetic energy conserved for divergence-free u); L_E, L_I, G,
 * D are the staggered operators of tpt_project and of the plans.
 * u, v, w: device FP64 face velocities in the layouts of tpt_project, u^k in
 * and u^{k+1} out.  eu, ev, ew: the same shapes, E^{k-1} in (not read for
 * k = 1) and E^k out, carried by the caller from substep to substep.  p:
 * (Nz, Ny, Nx) pressure, P^{k-1/2} in and P^{k+1/2} out.  phi: (Nz, Ny, Nx),
 * receives Phi.  workspace: at least tpt_ns_workspace_bytes.  Stream-ordered;
 * allocates nothing.  Info of the pressure solve: tpt_solve_info(pressure). */
int tpt_ns_substep(tpt_ns ns, int k, double *u, double *v, double *w, double *eu, double *ev, double *ew,
                   double *p, double *phi, void *workspace, size_t workspace_bytes, void *stream);

/* ---- multi-problem batches (independent problems, uneven sizes) ---------- */

/* Group `count` plans (any sizes, same precision) into a batch whose solve
 * issues one launch per stage for all problems (a work list of tiles from
 * every problem), with GEMM tiles chosen by the autotuning table.  Plans must
 * outlive the batch.  Plans with nrhs > 1 are rejected. */
int tpt_batch_create(int count, const tpt_plan *plans, tpt_batch *out);
int tpt_batch_destroy(tpt_batch batch);
int tpt_batch_workspace_bytes(tpt_batch batch, size_t *bytes);
/* rhs[i], out[i]: device FP64 fields of plan i.  use_graph != 0 captures the
 * batch's launches once (per stream and pointer set) in a hipGraph and
 * replays it.  Stream-ordered; fixed-refinement mixed plans only
 * (adaptive ones are rejected with TPT_ERR_UNSUPPORTED). */
int tpt_batch_solve(tpt_batch batch, const double *const *rhs, double *const *out,
                    void *workspace, size_t workspace_bytes, void *stream, int use_graph);
/* Info of problem `index` of the batch's last solve (call after synchronising
 * its stream; reads a few bytes of the workspace, which must still hold them):
 * corrections, the last correction and residual ratios of mixed plans, and
 * the right-hand-side check (compat_defect, nonfinite) as for tpt_solve_info.
 * TPT_ERR_INVALID before the first solve or for an index out of range. */
int tpt_batch_info(tpt_batch batch, int index, tpt_info *info);

/* ---- autotuning of GEMM tiles and the Thomas kernel ------------------------ */

/* Time every compiled tile variant for the GEMM shapes of the given plans and
 * record the fastest per (shape class, precision) in the process-wide table;
 * for non-periodic z, likewise time the sequential and the partitioned Thomas
 * kernels (variants of tpt_thomas) on the plan's lines and record the fastest
 * per (precision, line count, line length).  Plans created before or after
 * use the table; plans with TPT_FLAG_SEQ_THOMAS keep the sequential kernel.
 * Needs the GPU; synchronous; allocates temporary device buffers. */
int tpt_autotune(int count, const tpt_plan *plans, void *stream);
/* Save / load the table as text (one "prec kind M N K variant" line per
 * entry; kind 0 x GEMM, 1 y GEMM, 2 Thomas with M = lines, N = nz). */
int tpt_autotune_save(const char *path);
int tpt_autotune_load(const char *path);

/* ---- serving loop ---------------------------------------------------------- */

/* A server admits solve requests while others run: a request waits until a
 * slot is free and its workspace fits in the HBM budget, then its stages are
 * launched on that slot's stream (requests admitted together share one
 * multi-problem launch per stage).  Eigenbases stay device-resident in the
 * plan cache.  max_slots concurrent requests, hbm_budget_bytes for request
 * workspaces (0 = 3/4 of the free memory at creation). */
int tpt_server_create(size_t hbm_budget_bytes, int max_slots, tpt_server *out);
/* Queue a request; rhs/out are device FP64 fields owned by the caller and
 * must stay valid until the request completes.  Returns at once. */
int tpt_server_submit(tpt_server server, tpt_plan plan, const double *rhs, double *out,
                      unsigned long long *ticket);
/* TPT_OK when done (times in seconds on a process-wide monotonic clock:
 * submit, admitted to a slot, finished on the GPU), TPT_PENDING if not yet.
 * info: corrections, the last correction and residual ratios of mixed plans,
 * and the right-hand-side check (compat_defect, nonfinite) of the request. */
int tpt_server_poll(tpt_server server, unsigned long long ticket, tpt_info *info,
                    double *t_submit, double *t_start, double *t_done);
/* Block until every submitted request has finished. */
int tpt_server_drain(tpt_server server);
int tpt_server_destroy(tpt_server server);

/* ---- kernel-level entry points (testing and measurement) ------------------ */

/* Batched Thomas solve (§2.2.2 step 2.3) on explicit inputs: for every line
 * l = i + nx*j of each of nsys systems,
 *   (sigma + tau*(lamx[i] + lamy[j] + T_z)) x = f,
 * T_z with sub-diagonal az, diagonal bz, super-diagonal cz (device, nz each);
 * with periodic_z != 0 the lines are cyclic: az[0] couples row 0 to x[nz-1]
 * and cz[nz-1] couples row nz-1 to x[0] (nz >= 2).  f, x: device FP64
 * [nsys][nz][ny][nx]; scratch: device FP64 of at least
 * 4 * nx * ny * nsys * ceil(nz / 16) elements (chunk checkpoints).
 * pin_line >= 0 sets the last unknown of that line to zero and drops its
 * last equation (§3 gauge).  f may equal x.
 * variant: -1 automatic (what plans use); 0 sequential (one lane per line,
 * the only kernel for cyclic lines); 1..17 partitioned (each line cut into
 * P segments of L planes solved in parallel and joined by a P-row interface
 * system, LB lines per block), (LB, P, L) = (64,4,8) (64,8,8) (32,8,8)
 * (64,8,16) (32,8,16) (16,8,16) (64,16,16) (32,16,16) (16,16,16) (64,8,32)
 * (32,8,32) (16,8,32) (16,32,16) (32,16,32) (16,16,32) (16,64,16)
 * (16,32,32), needing P*L >= nz and non-cyclic lines, else
 * TPT_ERR_INVALID.  The partitioned kernels use no scratch. */
int tpt_thomas(int nx, int ny, int nz, int nsys, const double *lamx, const double *lamy,
               const double *az, const double *bz, const double *cz, int periodic_z,
               double sigma, double tau, int pin_line, const double *f, double *x,
               double *scratch, int variant, void *stream);

/* Strided-batched GEMM with the library's MFMA kernels (the transform
 * kernels of §2.2.2 on explicit operands).  A is M x K row-major (lda = K);
 * b_nk = 0: C_b = A_b B_b with B stored K x N (ldb = N), the y-pass form;
 * b_nk = 1: C_b = A_b B_b^T with B stored N x K (ldb = K), the x-pass form.
 * C is M x N (ldc = N).  prec: TPT_FP64 (double operands), TPT_MIXED_FP32
 * (float) or TPT_MIXED_BF16X3 (float operands; the basis-side operand — B for
 * b_nk = 1, A for b_nk = 0 — is split once into bf16 planes in a temporary
 * device buffer, the other on the fly).  variant: tile shape 0..4 (128x128,
 * 64x128, 128x64, 64x64, 32x64); FP64 / FP32 only: 5 (128x128 with a 32-deep
 * K tile), 6 (128x128 persistent, four 64x64 waves), 7 (128x128 persistent,
 * eight 64x32 waves) — 6 and 7 need M, N multiples of 128 and K of 16; 8
 * (128x128 over eight 64x32 waves, any shape); or -1 for the tile table.  Batch strides in elements (0 = shared).  Synchronises
 * the stream for TPT_MIXED_BF16X3. */
int tpt_gemm(int prec, int b_nk, int variant, int M, int N, int K, int batch, const void *A,
             long long strideA, const void *B, long long strideB, void *C, long long strideC,
             void *stream);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every library kernel while enabled (process-wide). */
int tpt_timing_enable(int enable);
/* Synchronises the recorded events, then for each kernel kind k < *count
 * fills names (NUL-separated, up to names_len bytes), total_ms[k] and
 * launches[k]; *count becomes the number of kinds.  Clears the log. */
int tpt_timing_collect(int *count, char *names, size_t names_len, double *total_ms,
                       long long *launches);

const char *tpt_last_error(void);
const char *tpt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TPT_H */
