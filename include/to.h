/*
 * to.h -- C ABI of the MI355X (gfx950) voxel hex8 topology-optimisation hot
 * path: the SIMP-weighted linear-elasticity state solve, compliance and its
 * sensitivity, the density/sensitivity filters and the density -> signed
 * distance transfer of Jezek et al., "Sequential topology optimization: SIMP
 * initialization for level-set boundary refinement".
 *
 * Conventions for every call:
 *  - Plain C types only.  "d_" pointers are device (HBM) memory, "h_" pointers
 *    are host memory.  The caller owns every array; the library never frees
 *    caller memory.  The library owns the opaque context (and, when no
 *    workspace is passed to to_create, the device workspace it allocates).
 *  - Grid: nelx x nely x nelz cubic voxels of edge h.
 *      node     n = i + (nelx+1) * (j + (nely+1) * k)
 *      element  e = i + nelx * (j + nely * k)   (lower corner at node (i,j,k))
 *      DOF      3*n + c, c = 0:x 1:y 2:z (interleaved)
 *    nel = nelx*nely*nelz, nn = (nelx+1)(nely+1)(nelz+1), ndof = 3*nn.
 *  - Streams: all work is queued on the context's HIP stream (passed as a
 *    void* holding a hipStream_t; NULL = the default stream).  Calls that
 *    return host values (h_c, info, status of a solve) synchronise that stream.
 *  - Errors: every call returns a to_status.  Invalid arguments are rejected
 *    before anything is queued.  to_last_error(ctx) gives a message; with a
 *    NULL ctx it gives the calling thread's last error.  The context stays
 *    usable after any error.  One context per thread (not thread-safe).
 *  - Concurrency: contexts share no device state (each has its own workspace
 *    and stream; the one exception is the fixed array of
 *    to_density_to_sdf_noalloc), so calls on different contexts may overlap
 *    on the GPU, from one thread or several; the caller orders their streams
 *    where one call's output is another's input.
 */
#ifndef TO_H_
#define TO_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct to_ctx to_ctx;

typedef enum {
  TO_OK = 0,
  TO_E_INVALID = -1,    /* bad argument (sizes, NULL required pointer, x outside [0,1]) */
  TO_E_OOM = -2,        /* workspace too small or device allocation failed            */
  TO_E_HIP = -3,        /* a HIP runtime call failed                                  */
  TO_E_NOCONV = -4,     /* iteration cap reached; outputs hold the last iterate        */
  TO_E_NONFINITE = -5,  /* NaN/Inf in an input or produced during a solve             */
  TO_E_SINGULAR = -6,   /* CG breakdown (p^T K p <= 0): singular or indefinite system  */
  TO_E_BUSY = -7        /* serving: no slot or memory for the request right now        */
} to_status;

typedef enum {
  TO_BC_CANTILEVER = 0,
  TO_BC_MBB = 1,
  TO_BC_CUSTOM = 2,
  TO_BC_CANTILEVER_CORNERS = 3,
  TO_BC_MBB_STRIP = 4
} to_bc;

/* Arithmetic of the state solve.  FP64: Jacobi-PCG in float64 throughout.
 * FP32_REFINE: inner Jacobi-PCG with float32 vectors and float32 element
 * arithmetic, outer iterative refinement whose residual f - K u, norms and
 * solution update are float64.  FP32_REFINE_BF16: as FP32_REFINE with the
 * inner CG's preconditioned residual z stored in bfloat16 (search directions,
 * residual and iterate stay float32; float32 arithmetic and accumulation):
 * flexible CG, whose direction update keeps consecutive directions
 * K-conjugate under the rounding.  Fewer bytes per iteration, more
 * iterations; the float64 refinement sets the final accuracy. */
typedef enum { TO_PREC_FP64 = 0, TO_PREC_FP32_REFINE = 1, TO_PREC_FP32_REFINE_BF16 = 2 } to_prec;

typedef enum { TO_FILTER_DENS = 0, TO_FILTER_DENS_T = 1, TO_FILTER_SENS = 2 } to_filter_mode;

/* Statement of the state problem K(x) u = F (paper Sec. 2.1.1, Eq. 2) with the
 * modified SIMP modulus E_e = Emin + x_e^penal (E0 - Emin) (Eq. 1).
 * Built-in boundary conditions (z is the vertical axis):
 *   CANTILEVER: all DOFs fixed on the x = 0 face; total load -load_total in z
 *     along the bottom edge (i = nelx, k = 0) of the opposite face, as the
 *     consistent nodal shares of a uniform line load (end nodes carry half an
 *     interior node's share: -(load_total*w)/nely with w = 0.5 or 1).
 *   MBB: u_x = 0 on x = 0 (symmetry), u_z = 0 on the edge i = nelx, k = 0,
 *     u_y = 0 at node (0,0,0); the same line load on the edge i = 0, k = nelz.
 *   CUSTOM: fixed_mask (ndof bytes, nonzero = fixed) and load (ndof doubles)
 *     are host arrays read once by to_create.
 *   The paper's own variants (Secs. 4.2-4.3), with its geometry scaled to the
 *   grid (Ly = nely h, Lz = nelz h, r = min(Ly, Lz)/10):
 *   CANTILEVER_CORNERS: all DOFs fixed on the x = 0 nodes inside the four
 *     corner squares (y <= 0.3 Ly or y >= 0.7 Ly, and likewise z); load -z on
 *     the disc of radius r centred on the x = Lx face.
 *   MBB_STRIP: u_x = 0 on x = 0; u_z = 0 on the bottom nodes of the last
 *     element strip (k = 0, i >= nelx - 1); u_y = 0 at node (0,0,0); load -z
 *     on the half disc of radius r centred at (0, Ly/2, Lz) on the top face.
 *   A loaded region is the set of boundary-face quads whose centroid lies in
 *   it (on grids too coarse for any: the quads nearest its centre) under a
 *   uniform traction, so a node carries -(load_total c)/(4 nq) with c its
 *   tagged quads and nq their number.
 * Loads on fixed DOFs are ignored. */
typedef struct {
  int32_t nelx, nely, nelz;    /* voxels per axis, each >= 1                      */
  double h;                    /* voxel edge, > 0                                 */
  double E0, Emin, nu, penal;  /* E0 > 0, 0 <= Emin < E0, -1 < nu < 0.5, penal>=1 */
  int32_t bc;                  /* to_bc                                           */
  const uint8_t *fixed_mask;   /* CUSTOM only, host, ndof                         */
  const double *load;          /* CUSTOM only, host, ndof                         */
  double load_total;           /* built-in BCs: magnitude of the total load       */
  int32_t precision;           /* to_prec                                         */
  double rtol;                 /* stop when ||f - K u||_2 <= rtol ||f||_2 (float64) */
  int32_t max_iters;           /* cap on the total number of inner CG iterations  */
} to_problem;

typedef struct {
  int32_t outer_iters;   /* float64 residual evaluations after the first       */
  int32_t inner_iters;   /* CG iterations summed over all inner solves         */
  double rel_res;        /* final ||f - K u||_2 / ||f||_2, computed in float64  */
  double ms;             /* wall time of the call on the host, milliseconds     */
} to_solve_info;

/* Device workspace (bytes) a context for this problem needs.  Lets the caller
 * allocate it (e.g. as a torch uint8 tensor) and admit work by footprint.
 * Grid limits (TO_E_INVALID beyond them, here and in to_create): a float64
 * vector of 3 nn values below 2^31 bytes (nn < 89,478,486 nodes), and at most
 * 8192 product tiles of 31 x 7 nodes in x and y,
 * ceil((nelx + 1) / 31) * ceil((nely + 1) / 7) <= 8192. */
to_status to_workspace_size(const to_problem *prob, size_t *bytes);

/* Create a context.  d_workspace: caller-owned device memory of at least
 * to_workspace_size() bytes, 256-byte aligned, or NULL to let the library
 * allocate (and free, in to_destroy) its own.  stream: hipStream_t or NULL.
 * Precomputes the fixed-DOF mask and the load vector on the device. */
to_status to_create(const to_problem *prob, void *d_workspace, size_t bytes, void *stream,
                    to_ctx **out);
void to_destroy(to_ctx *ctx);                 /* NULL-safe */
const char *to_last_error(const to_ctx *ctx); /* valid until the next call on ctx */

/* State solve (Eq. 2): u = K(x)^{-1} F by Jacobi-preconditioned CG in the
 * context's precision, to rtol.  d_x: [nel] densities in [0,1] (Eq. 1 maps
 * them to moduli).  d_u0: [ndof] warm start or NULL (zero start).  d_u: [ndof]
 * output; fixed DOFs are exactly 0.  info: host, may be NULL.
 * Returns TO_E_NOCONV (d_u = last iterate, info filled) when max_iters is hit,
 * TO_E_SINGULAR on CG breakdown, TO_E_NONFINITE on NaN/Inf, TO_E_INVALID when
 * some x_e lies outside [0,1]. */
to_status to_solve(to_ctx *ctx, const double *d_x, const double *d_u0, double *d_u,
                   to_solve_info *info);

/* Compliance and its sensitivity (Eq. 2 and Eq. 3):
 *   h_c = F^T u  (host scalar, float64, deterministic reduction),
 *   d_dc[e] = -penal x_e^(penal-1) (E0 - Emin) u_e^T k0 u_e  (float64, [nel]),
 * with k0 the unit-modulus element stiffness.  d_dc may be NULL. */
to_status to_compliance_sensitivity(to_ctx *ctx, const double *d_x, const double *d_u, double *h_c,
                                     double *d_dc);

/* Filters (Sec. 2.1.3, Eq. 4), radius rmin in element units (> 0), weights
 * H = max(0, rmin - distance) over element centroids at distance < rmin,
 * truncated at the domain boundary and normalised per element:
 *   DENS   : out_e = sum_i H_ei V x_i / sum_i H_ei V            (d_in = x)
 *   DENS_T : out_j = sum_e H_ej V in_e / sum_i H_ei V           (adjoint of DENS)
 *   SENS   : out_e = sum_i (x_i/V) H_ei in_i / ((max(x_e,1e-3)/V) sum_i H_ei)  (Eq. 4;
 *            in = dc, d_x = densities, required)
 * d_x is ignored for DENS and DENS_T.  d_out must not alias d_in. */
to_status to_filter(to_ctx *ctx, double rmin, int32_t mode, const double *d_x, const double *d_in,
                    double *d_out);

/* Density -> signed distance (Secs. 3.2-3.4, Eqs. 25-30):
 *   rho_n : nodal densities; on a voxel grid the paper's local linear
 *           least-squares map (Eqs. 25-27, with its fallbacks) is the mean of
 *           the adjacent elements, summed in increasing element order;
 *   iso-surface rho_n = rho_t by marching tetrahedra on the six-tet (Kuhn)
 *           split of every voxel (a node is inside when rho_n >= rho_t);
 *   d      : exact minimum distance from every node to the triangles (Eqs. 28-29);
 *   phi    : -d where rho_n >= rho_t, +d elsewhere (Eq. 30); +/-inf when the
 *           surface is empty.
 *   vf     : per element, the volume fraction where the piecewise-linear
 *           interpolant of phi on the same split is < 0 (ersatz weight).
 * d_phi [nn] required; d_rho_nodes [nn] and d_vf [nel] may be NULL. */
to_status to_density_to_sdf(to_ctx *ctx, const double *d_x, double rho_t, double *d_phi,
                            double *d_rho_nodes, double *d_vf);

/* to_density_to_sdf for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, bit for bit, with the
 * triangles kept in a fixed device array of the library instead of a buffer
 * the context grows.  The array holds TO_NOALLOC_MAX_TRIANGLES triangles
 * (72 bytes each, 18.9 MB), one copy per GPU the library runs on, held until
 * the process ends.  A design whose iso-surface needs more is rejected with
 * TO_E_OOM after the counting pass (d_rho_nodes, if given, then holds the
 * nodal densities; d_phi and d_vf are untouched); to_last_triangle_count()
 * gives the number it needed.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (contexts on different streams or threads)
 * race and must be serialised by the caller.  No device memory is allocated
 * or freed (the context's workspace and pinned host scalars come from
 * to_create); on the host only an error path formats its message. */
#define TO_NOALLOC_MAX_TRIANGLES 262144
to_status to_density_to_sdf_noalloc(to_ctx *ctx, const double *d_x, double rho_t, double *d_phi,
                                    double *d_rho_nodes, double *d_vf);

/* Ersatz weights of a level set (Sec. 4.1: cut elements weighted by their
 * solid volume fraction): per element, the volume fraction where the
 * piecewise-linear interpolant of phi on the six-tet split is < 0 (the vf of
 * to_density_to_sdf, for any nodal phi).  d_phi [nn]; d_vf [nel] output.
 * Asynchronous. */
to_status to_volume_fraction(to_ctx *ctx, const double *d_phi, double *d_vf);

/* Optimality-criteria update of the densities: the design update of the
 * SIMP stage (Sec. 2.1 with the SIMP set-up of Sec. 4).  The paper names OC
 * without its parameters; this is the textbook scheme (Bendsoe and Sigmund):
 *   x_new_e = clamp(x_e (max(-dc_e, 0) / lam)^eta,
 *                   [max(0, x_e - move), min(1, x_e + move)])
 * (equal voxels: unit volume derivative), with lam by bisection on [0, 1e9]:
 * the midpoint is evaluated; the lower end moves up when
 * sum_e x_new_e > vf nel, else the upper end moves down; until
 * (l2 - l1) / (l1 + l2) <= 1e-3.  x_new is the design of the last midpoint
 * evaluated.  The volume sums are float64 in a fixed order, so the result is
 * reproducible run to run.
 *   d_x [nel] densities in [0,1]; d_dc [nel] sensitivities (filtered ones, in
 *   the SIMP loop; a positive value counts as 0); d_xnew [nel] output, may
 *   alias d_x but not d_dc.  0 < vf <= 1, 0 < move <= 1, 0 < eta <= 1.
 *   info: host, may be NULL.  Synchronises the context stream.
 * Errors, all before d_xnew is written: TO_E_NONFINITE (NaN/Inf in x or
 * dc), TO_E_INVALID (x outside [0,1], bad parameters), TO_E_NOCONV (no
 * multiplier within 200 midpoints: the volume target cannot be met from
 * above, e.g. every dc is 0). */
typedef struct {
  double lambda;       /* the multiplier of the returned design */
  double change;       /* max_e |x_new_e - x_e|  (Delta rho_max) */
  double volume;       /* mean of x_new: its volume fraction */
  int32_t bisections;  /* midpoints evaluated */
  int32_t reserved;
} to_oc_info;
to_status to_oc_update(to_ctx *ctx, const double *d_x, const double *d_dc, double vf, double move,
                       double eta, double *d_xnew, to_oc_info *info);

/* The SIMP loop of the paper's first stage (Sec. 2.1, set-up of Sec. 4).  Per
 * design iteration: the state solve (to_solve, warm-started from the previous
 * displacement), compliance and sensitivity (to_compliance_sensitivity), the
 * sensitivity filter of Eq. 4 at radius rmin (to_filter, SENS), and the OC
 * update (to_oc_update, in place); it stops once the largest density change
 * of an update is <= change_tol (Delta rho_max) or after max_iters updates.
 *   d_x [nel]: in: the start design (ignored when init_uniform != 0: then
 *     x = vf everywhere); out: the design after the last update.
 *   d_u [ndof]: out: the displacement of the last design solved (the one
 *     before the last update).
 *   d_work [2 nel]: device scratch.
 *   h_c_hist [max_iters]: host, may be NULL: compliance of each design solved.
 *   info: host, may be NULL.
 * A failing step returns its own status, with the design iteration named in
 * to_last_error; d_x then holds the last complete update. */
typedef struct {
  double vf;           /* target volume fraction, 0 < vf <= 1 (paper: 0.4) */
  double rmin;         /* sensitivity-filter radius, element units (paper: 2) */
  double move;         /* OC move limit (0.2) */
  double eta;          /* OC damping exponent (0.5) */
  double change_tol;   /* Delta rho_max stop (paper: 0.005 .. 0.08) */
  int32_t max_iters;   /* design iterations, >= 1 */
  int32_t init_uniform;
} to_simp_params;
typedef struct {
  int32_t iters;       /* design updates done */
  int32_t converged;   /* 1 when the Delta rho_max stop was met */
  int32_t inner_iters; /* inner CG iterations over all state solves */
  int32_t reserved;
  double c;            /* compliance of the last design solved */
  double change;       /* Delta rho_max of the last update */
  double volume;       /* volume fraction of the returned design */
  double ms;           /* wall time of the call */
} to_simp_info;
to_status to_simp(to_ctx *ctx, const to_simp_params *sp, double *d_x, double *d_u, double *d_work,
                  double *h_c_hist, to_simp_info *info);

/* Level-set evolution (Sec. 2.2.7): nsteps forward-Euler steps of the
 * Hamilton-Jacobi equation phi_t + v |grad phi| = 0 (Eq. 21) with the
 * first-order Godunov upwind stencil on the node grid, at
 * dt = gamma h / max|v| (the CFL bound of Eq. 22 times the CFL number gamma).
 * With D-, D+ the one-sided differences along each axis (across a box face
 * the difference is 0: the missing neighbour is the node itself):
 *   g+ = sqrt(sum_axes max(D-,0)^2 + min(D+,0)^2),
 *   g- = sqrt(sum_axes min(D-,0)^2 + max(D+,0)^2),
 *   phi <- phi - dt (max(v,0) g+ + min(v,0) g-).
 * d_phi [nn] in/out; d_v [nn] nodal normal speed, must not alias d_phi;
 * 0 < gamma <= 1; nsteps >= 0.  h_dt (host, may be NULL) receives dt (0 when
 * v = 0 everywhere: phi is left as it is).  TO_E_NONFINITE (NaN/Inf in phi or
 * v) is returned before phi is touched.  Asynchronous after the input check. */
to_status to_ls_advect(to_ctx *ctx, double *d_phi, const double *d_v, double gamma,
                       int32_t nsteps, double *h_dt);

/* Reinitialisation (Sec. 2.2.8): pseudo-steps of
 * phi_t + S(phi)(|grad phi| - 1) = 0 (Eq. 23) with the same stencil and the
 * smeared sign S = phi / sqrt(phi^2 + h^2 |grad phi|^2) (Eq. 24) taken from
 * the current phi at every pseudo-step (|grad phi| by central differences,
 * S = 0 where the root is 0):
 *   phi <- phi - gamma h (max(S,0)(g+ - 1) + min(S,0)(g- - 1)),
 * until the first pseudo-step whose largest |change| is < tol.
 * d_phi [nn] in/out; 0 < gamma <= 1; tol > 0; max_steps >= 1.  h_steps and
 * h_change (host, may be NULL): pseudo-steps taken and the last step's
 * largest change.  TO_E_NOCONV when max_steps pass without reaching tol (phi
 * holds the last iterate); TO_E_NONFINITE before phi is touched.
 * Synchronises the context stream. */
to_status to_ls_reinit(to_ctx *ctx, double *d_phi, double gamma, double tol, int32_t max_steps,
                       int32_t *h_steps, double *h_change);

/* Relaxed shape derivative (Sec. 2.2.5): the nodal vector of Eqs. 15-17,
 *   g_a = sum_e sum_q w_q h^3 N_a(q) (c_s s(q) + c_0) H'_eta(phi(q)) |grad phi(q)|,
 * over the 2x2x2 Gauss points q of every voxel, with phi and u trilinear on
 * it, s = sigma:eps = lambda (tr eps)^2 + 2 mu eps:eps at the solid's E0 and
 * nu, and H'_eta(t) = (1 + cos(pi t / eta)) / (2 eta) for |t| <= eta, else 0
 * (the derivative of Eq. 8).  (c_s, c_0) = (1, 0) gives J' (Eq. 15),
 * (0, -1/V_D) gives C' (Eq. 16), (1, (lambda - Lambda C)/V_D) gives L'
 * (Eqs. 17-18).
 * d_u [ndof] displacements (interleaved 3n + c; may be NULL when c_s == 0);
 * d_phi [nn] level set; d_g [nn] output, must not alias d_phi; eta > 0.
 * Deterministic (fixed summation order).  Asynchronous.  The first call on a
 * context allocates 64 bytes per element of device scratch (kept until
 * to_destroy; TO_E_OOM if that fails). */
to_status to_shape_rhs(to_ctx *ctx, const double *d_u, const double *d_phi, double eta,
                       double c_s, double c_0, double *d_g);

/* Hilbertian extension-regularisation (Sec. 2.2.6): solves
 * A_H v = g (Eq. 20), A_H = ell^2 K + M with the trilinear Laplacian and mass
 * of Eq. 19 on the voxel grid, and v = 0 on Gamma_N, the nodes where the
 * context's load vector has a non-zero component (the natural condition
 * elsewhere).  Jacobi-preconditioned CG in float64 from v = 0 to
 * ||r|| <= rtol ||g_free||.
 * d_g [nn] right-hand side; d_v [nn] output, must not alias d_g; ell >= 0;
 * 0 < rtol < 1; max_iters >= 1.  h_iters, h_rel (host, may be NULL): CG
 * iterations and the final relative residual.  TO_E_NOCONV at the cap (d_v =
 * last iterate), TO_E_SINGULAR on breakdown, TO_E_NONFINITE when d_g holds a
 * NaN or Inf (d_v untouched).  Synchronises the context stream. */
to_status to_hilbert_extend(to_ctx *ctx, double ell, const double *d_g, double *d_v, double rtol,
                            int32_t max_iters, int32_t *h_iters, double *h_rel);

/* Matrix-free operator of Eq. 2, y = K(x) u with the fixed DOFs zeroed on
 * input and identity rows on output (y_fixed = u_fixed), float64.
 * d_u, d_y: [ndof], must not alias.  d_x NULL reuses the moduli of the
 * previous call on this context (one kernel launch, for timing). */
to_status to_matvec(to_ctx *ctx, const double *d_x, const double *d_u, double *d_y);
/* The same operator with float32 vectors, float32 moduli and float32 element
 * arithmetic (the inner-CG product of TO_PREC_FP32_REFINE). */
to_status to_matvec_f32(to_ctx *ctx, const double *d_x, const float *d_u, float *d_y);

/* Serving (continuous batching).  A server owns one device allocation of
 * hbm_budget_bytes (an arena for per-request state), a private HIP stream of
 * default priority and a worker thread.  Requests are compliance +
 * sensitivity solves (TO_PREC_FP32_REFINE, built-in BCs, any grid size) that
 * are admitted in arrival order as soon as a slot (max_slots) and arena space
 * for the request's footprint are free; all admitted designs that are in an
 * inner CG solve advance together, one batched product launch and one
 * batched update launch per iteration.  A request's results do not depend on
 * which other requests share the batch.
 *   to_server_submit: h_x [nel] is copied; h_dc_out [nel] (may be NULL) must
 *     stay valid until the request is returned by to_server_poll.  Returns
 *     TO_E_OOM if the footprint can never fit the budget, TO_E_BUSY if the
 *     queue is full, TO_E_INVALID for other precisions or CUSTOM BCs.
 *   to_server_poll: non-blocking; returns up to cap finished requests (tag,
 *     compliance F^T u, status, latency from submit to completion in ms).
 *   to_server_wait_idle: blocks until nothing is queued or live, or the
 *     timeout passes (then TO_E_BUSY).
 *   Thread-safe: submit, poll, wait and stats may be called from any thread. */
typedef struct to_server to_server;
to_status to_server_create(size_t hbm_budget_bytes, int32_t max_slots, void *stream_unused,
                           to_server **out);
to_status to_server_submit(to_server *srv, const to_problem *prob, const double *h_x,
                           double *h_dc_out, uint64_t tag);
to_status to_server_poll(to_server *srv, uint64_t *tags, double *c, int32_t *status,
                         double *latency_ms, int32_t cap, int32_t *n);
to_status to_server_wait_idle(to_server *srv, double timeout_ms);
to_status to_server_stats(to_server *srv, int32_t *live, int32_t *queued, int64_t *ticks,
                          size_t *free_bytes);
const char *to_server_last_error(const to_server *srv);
void to_server_destroy(to_server *srv); /* NULL-safe; waits for the worker to stop */

/* Diagnostics.
 * to_last_energy_sum: sum_e E_e u_e^T k0 u_e of the last
 *   to_compliance_sensitivity call (equals F^T u at an exact solution).
 * to_last_triangle_count: triangles of the last to_density_to_sdf call.
 * to_profile: returns the accumulated HIP-event time (ms) and count of the
 *   inner-CG product launches recorded since the previous to_profile call,
 *   then resets them and turns recording on (enable != 0) or off.  While
 *   recording, one chunk of CG iterations in four runs as separate launches
 *   (not as a graph), and two of its product launches (one of each direction
 *   slot) carry start/stop events taken from the dispatch's own timestamps,
 *   without a system-scope fence.  Only launches of iterations before the
 *   CG's stop are counted.  The solve's results do not change. */
double to_last_energy_sum(const to_ctx *ctx);
int32_t to_last_triangle_count(const to_ctx *ctx);
to_status to_profile(to_ctx *ctx, int32_t enable, double *h_ms, int64_t *h_count);

#ifdef __cplusplus
}
#endif
#endif /* TO_H_ */
