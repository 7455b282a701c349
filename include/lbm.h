/*
 * lbm.h -- C ABI of the MI355X (gfx950) central-moment lattice Boltzmann
 * library liblbm.so.
 *
 * The library advances one advection-diffusion lattice h (internal energy
 * H = rho c_v T with c_v = 1) and, optionally, one hydrodynamic lattice f that
 * supplies the advecting velocity (one-way coupling; paper Sec. 2, Eqs.
 * f_0th_mom, f_1st_mom, h_0th_mom).  One call of lbm_step() performs, per step
 * and per node, pull-streaming, the boundary rules of Sec. 3 (BB/IBB on f,
 * ABB/IABB on h, EQ nodes, zero-gradient outlet) and the central-moment
 * collision of Sec. 2.1 (Eqs. raw_mom_def, cm_mom_def, H_cm_collision) with a
 * diagonal relaxation matrix, in one fused HIP kernel per step (D3Q27 with
 * listed boundary nodes: a bulk and a boundary kernel).
 *
 * Conventions
 *  - Ownership: every device buffer is owned by the caller and borrowed by the
 *    context; it must outlive the context (or the next call that replaces it).
 *    Host arrays are read during the call only.  The library never allocates
 *    device memory: lbm_workspace_bytes() tells the caller how much to provide.
 *  - Streams: every call is asynchronous on the stream given to lbm_create()
 *    except the ones marked "synchronises".  Device faults surface as
 *    LBM_EDEVICE at the next synchronising call.
 *  - Errors: calls return an lbm_status and never abort; lbm_last_error()
 *    returns a message that names the offending argument or index.
 *  - Threads: one context per stream; calls on one context must not overlap.
 *  - Layout: populations exchanged through this interface
 *    (lbm_get_populations, lbm_set_populations, the adjoint's lambda) are
 *    FP64 or arithmetic-type structure-of-arrays, index [i][z][y][x] with x
 *    fastest; node index n = x + nx (y + ny z).  The storage layout inside
 *    the workspace (node tiles, or planes for FP16) is private; snapshots of
 *    lbm_save_state() are opaque.
 *    Direction order i: D2Q9 (0,0),(1,0),(0,1),(1,1),(-1,0),(0,-1),(1,-1),
 *    (-1,1),(-1,-1) (the e_z = 0 subset of the D3Q27 order); D3Q27 is the
 *    order of Sec. 2.1.  Moment order of per-moment rates: Sec. 2.1 (D3Q27:
 *    000,100,010,001,110,101,011,200,020,002,120,102,210,201,012,021,111,
 *    220,202,022,211,121,112,122,212,221,222) and App. A for D2Q9
 *    (00,10,01,20,02,11,21,12,22).
 *  - Time: after lbm_init_equilibrium() the state is at time t = 0; each
 *    step advances t by one.  The canonical state at time t is the
 *    pre-collision, post-stream population set with all boundary rules of
 *    that step applied.  Internally the library stores the post-collision
 *    state of step t-1 and re-derives the canonical state when asked.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,       /* invalid argument; message names it */
  LBM_ENOMEM = -2,       /* workspace or table capacity too small */
  LBM_EDEVICE = -3,      /* HIP runtime error */
  LBM_ESTATE = -4,       /* call out of order (e.g. step before init) */
  LBM_EUNSUPPORTED = -5, /* combination not built */
  LBM_EDIVERGED = -6     /* non-finite value found by lbm_reduce() */
} lbm_status;

typedef enum { LBM_D2Q9 = 9, LBM_D3Q27 = 27 } lbm_lattice;

/* Storage type of the populations; arithmetic is FP64 for LBM_FP64 and
 * LBM_FP32_SR and FP32 otherwise.  The *_DEV types and LBM_FP16_SR store deviations g_i - w_i
 * g_ref from the rest equilibrium of the reference values rho_ref / H_ref.
 * LBM_FP32_SR stores FP32 values rounded stochastically from the FP64 result:
 * up or down to the two nearest FP32 values with probabilities set by the
 * distance to each, drawn from a hash of the updating node and the step and
 * the value's lattice and direction (deterministic for a given run, and the
 * same in the in-place and two-array layouts, which agree bit for bit).  A
 * steady state then does not accumulate the bias that rounding to nearest
 * repeats at every node and step.  No adjoint.
 * LBM_FP16_SR is LBM_FP16_DEV (FP32 arithmetic, FP16 deviations) with the
 * deviations rounded stochastically the same way (FP16 subnormals: to the
 * multiples of 2^-24 around them).  No adjoint. */
typedef enum {
  LBM_FP64 = 0,
  LBM_FP32 = 1,
  LBM_FP32_DEV = 2,
  LBM_FP16_DEV = 3,
  LBM_FP32_SR = 4,
  LBM_FP16_SR = 5
} lbm_storage;

/* Streaming layout: two arrays (AB) or one array updated in place (AA). */
typedef enum { LBM_STREAM_AB = 0, LBM_STREAM_AA = 1 } lbm_stream_mode;

/* Relaxation presets (Sec. 2.1.1).  s^H = 1/(3k + 1/2), s_nu = 1/(3 nu + 1/2).
 *  LBM_CM_SRT : every central moment at s^H (equal to BGK with the full
 *               equilibrium);
 *  LBM_CM_1ST : first-order moments at s^H, all others at 1;
 *  LBM_CM_TRT : moments of odd total order at s^H, even ones at 1
 *               (the paper's recommended kernel for h);
 *  LBM_CM_NS  : second-order moments at s_nu, all others at 1 (f lattice),
 *               with the trace of the diagonal block at s_bulk_f (default 1);
 *  LBM_CM_CUSTOM : rates taken from s_custom_f / s_custom_h. */
typedef enum {
  LBM_CM_SRT = 0,
  LBM_CM_1ST = 1,
  LBM_CM_TRT = 2,
  LBM_CM_NS = 3,
  LBM_CM_CUSTOM = 4
} lbm_relax;

/* Node flags: bits 0-3 type, bits 4-11 group (index into the group table). */
#define LBM_NODE_FLUID 0  /* ordinary node */
#define LBM_NODE_SOLID 1  /* wall interior: links into it are cut links */
#define LBM_NODE_EQ 2     /* populations replaced by the group equilibrium */
#define LBM_NODE_OUTLET 3 /* zero-gradient outlet (copies e_x < 0 from x - 1) */
#define LBM_FLAG(type, group) ((uint16_t)((type) | ((group) << 4)))
#define LBM_MAX_GROUPS 256

typedef enum { LBM_WALL_BB = 0, LBM_WALL_IBB = 1 } lbm_f_wall;   /* Eq. IBB */
typedef enum { LBM_WALL_ABB = 0, LBM_WALL_IABB = 1 } lbm_h_wall; /* Eq. IABB */

/* Boundary group.  For SOLID nodes: the wall schemes of links into the group
 * and the wall energy H_w of the IABB/ABB equilibrium term.  For EQ nodes:
 * the state (rho_w, u_w, H_w) the node is reset to.  Walls are at rest. */
typedef struct {
  int32_t f_scheme; /* lbm_f_wall */
  int32_t h_scheme; /* lbm_h_wall */
  double rho_w;
  double u_w[3];
  double H_w;
} lbm_group;

typedef struct {
  int32_t lattice;  /* lbm_lattice */
  int32_t nx, ny, nz; /* nz = 1 for D2Q9 */
  int32_t with_ns;  /* 1: evolve f and advect h with its velocity */
  int32_t storage;  /* lbm_storage */
  int32_t stream;   /* lbm_stream_mode */
  int32_t relax_f;  /* lbm_relax for f (with_ns only) */
  int32_t relax_h;  /* lbm_relax for h */
  int32_t u_mode;   /* advection-only: 0 uniform u0, 1 per-node field */
  int32_t with_source; /* 1: per-node source Q of h (App. D) */
  int32_t max_links;   /* capacity of the cut-link table */
  int32_t max_special; /* capacity of the boundary-node list */
  int32_t cumulant;    /* collision family per lattice: bit 0 h, bit 1 f use the
                        * cumulant collision (Eqs. H_cu_collision,
                        * hydro_cu_collision, source as in App. D) instead of
                        * central moments; the rates are those of relax_h /
                        * relax_f in cumulant order (LBM_CM_1ST for h is the
                        * paper's Cumulants-1st, LBM_CM_NS for f relaxes the
                        * second-order cumulants at s_nu).  The cumulant
                        * transform normalises by the zeroth moment, which must
                        * not vanish.  With those two presets every rate above
                        * order 2 (f) or order 1 (h) is 1, and the library
                        * runs a shorter transform that gives the same result
                        * to rounding; other rates run the full one. */
  double nu;        /* kinematic viscosity (lattice units), f lattice */
  double k;         /* conductivity / diffusivity (lattice units), h lattice */
  double rho_ref;   /* deviation reference of f (the *_DEV storages, LBM_FP16_SR) */
  double H_ref;     /* deviation reference of h */
  double u0[3];     /* uniform advection velocity (u_mode 0) */
  double s_custom_f[27]; /* per-moment rates, LBM_CM_CUSTOM */
  double s_custom_h[27];
  double s_bulk_f;  /* rate of the trace of f's diagonal second-order block
                     * (central moments 200 + 020 + 002, or the cumulants of
                     * the same indices): the bulk viscosity.  The deviatoric
                     * parts (differences of those moments) keep the diagonal
                     * rate of 200, i.e. s_nu under LBM_CM_NS.  0 selects 1 for
                     * LBM_CM_NS (the separate bulk rate of the cumulant f
                     * kernel of Geier et al. 2015, which the paper adopts)
                     * and no separate trace rate otherwise; a value in
                     * (0, 2) sets it (with LBM_CM_CUSTOM the custom rates of
                     * 200, 020 and 002 must then be equal).  Setting it to
                     * s_nu reproduces the diagonal relaxation. */
} lbm_params;

/* One cut link (Sec. 3): boundary node x_b, direction dir from x_b towards the
 * wall (x_b + e_dir is SOLID), group of that solid node, xf_solid = 1 when
 * x_f = x_b - e_dir is solid (a one-node gap), and q in (0, 1] the wall
 * distance as a fraction of e_dir.  In a gap, a link with q < 1/2 takes the
 * plain (A)BB rule, since the q <= 1/2 branch of Eqs. IBB and IABB reads x_f;
 * a link with q > 1/2 keeps the interpolated rule, whose branch reads only
 * x_b.  Sorted by (node, dir). */
typedef struct {
  int32_t node;
  int32_t dir;
  int32_t group;
  int32_t xf_solid;
  double q;
} lbm_link;

/* ---- host-only queries (no GPU needed) --------------------------------- */

/* Version string of the library. */
const char *lbm_version(void);

/* Bytes of device workspace lbm_create() needs for params p (0 if p is
 * invalid; the reason is then in lbm_last_error(NULL)). */
size_t lbm_workspace_bytes(const lbm_params *p);

/* Per-moment relaxation rates the library uses for p, in the moment order
 * above: s_f[27] and s_h[27] (entries past Q are 1), and *s_bulk_f the rate
 * of the trace of f's second-order block (0: none, the trace relaxes with
 * the diagonal rates).  Any output may be NULL. */
lbm_status lbm_relaxation_rates(const lbm_params *p, double *s_f, double *s_h, double *s_bulk_f);

/* Counts the cut links and the boundary-node records of a geometry (flags as
 * in lbm_set_geometry), the capacities max_links and max_special must hold.
 * A record is kept for every non-solid node with cut links and for the EQ and
 * OUTLET nodes the bulk threads do not handle: an EQ node is handled there when
 * it has no cut link and its group is below 252; an OUTLET node n when neither
 * it nor its upstream node n - 1 has a cut link, that node is FLUID, x != 0 and
 * n % 64 != 0.  In the AA layout a listed outlet's upstream node needs no
 * record of its own.  Either output may be NULL. */
lbm_status lbm_count_geometry(const lbm_params *p, const uint16_t *flags, int64_t *n_links,
                              int64_t *n_special);

/* Builds the cut-link table of a geometry on the host: flags[n], q[Q][n]
 * (read on cut links only; NULL means q = 1/2), groups[n_groups].  Writes at
 * most cap links to out, the total to *count.  Rejects q outside (0, 1] on a
 * cut link, a group index >= n_groups on a SOLID or EQ node, a type above 3,
 * an OUTLET node whose upstream node (x - 1, periodic in x) is SOLID and, in
 * the AA layout, one whose upstream node is not FLUID. */
lbm_status lbm_build_links(const lbm_params *p, const uint16_t *flags, const double *q,
                           int32_t n_groups, lbm_link *out, int64_t cap, int64_t *count);

/* Measurement aid, not part of the method: a streaming device-to-device copy
 * of `bytes` (a multiple of 16; both pointers 16-byte aligned, regions not
 * overlapping) with 16-byte non-temporal loads and stores, on
 * hip_stream (NULL = default), asynchronous.  blocks = 0 launches one 16-byte
 * vector per thread, blocks > 0 a grid-stride loop over that many 256-thread
 * blocks.  Its rate is the practical HBM ceiling against which the step
 * kernels are read (2 x bytes moved per call). */
lbm_status lbm_device_copy(void *dst_dev, const void *src_dev, size_t bytes, int32_t blocks, void *hip_stream);

/* Last error message of ctx (or of the calling thread when ctx is NULL). */
const char *lbm_last_error(const lbm_ctx *ctx);

/* ---- context ------------------------------------------------------------ */

/* Creates a context on the current HIP device.  workspace_dev: caller-owned
 * device buffer of lbm_workspace_bytes(p) bytes, 256-byte aligned.
 * hip_stream: a hipStream_t (NULL = default stream). */
lbm_status lbm_create(const lbm_params *p, void *workspace_dev, void *hip_stream, lbm_ctx **out);
void lbm_destroy(lbm_ctx *ctx);

/* Sets the geometry (default: every node FLUID, fully periodic).  flags[n] and
 * q[Q][n] are host arrays (see lbm_build_links); groups[n_groups] the group
 * table.  The node classes, link table and boundary-node list are built on the
 * host and copied into the workspace.  Must precede lbm_init_equilibrium(). */
lbm_status lbm_set_geometry(lbm_ctx *ctx, const uint16_t *flags, const double *q,
                            const lbm_group *groups, int32_t n_groups);

/* Copies the context's cut-link table to host memory (synchronises). */
lbm_status lbm_get_links(lbm_ctx *ctx, lbm_link *out, int64_t cap, int64_t *count);

/* Advection-only with u_mode = 1: borrowed per-node velocity field, device,
 * [3][n] in the arithmetic type (double for LBM_FP64 and LBM_FP32_SR, float otherwise).
 * With with_ns = 1 the field, when set, gives the velocity of EQ nodes. */
lbm_status lbm_set_velocity(lbm_ctx *ctx, const void *u_dev);

/* with_source = 1: borrowed per-node source Q of h, device, [n] in the
 * arithmetic type.  The collision adds (1 - s_000/2) Q to the zeroth central
 * moment and evaluates the equilibrium at H = sum h + Q/2 (App. D). */
lbm_status lbm_set_source(lbm_ctx *ctx, const void *Q_dev);

/* Equilibrium initial state at t = 0 from device FP64 fields rho[n] (may be
 * NULL = 1; ignored without f), u[3][n] (may be NULL = u0 or the velocity
 * field) and H[n].  The stored post-collision state is g^eq(x + e_i), so that
 * streaming gives g^eq in the bulk and boundary rules apply at t = 0. */
lbm_status lbm_init_equilibrium(lbm_ctx *ctx, const double *rho_dev, const double *u_dev,
                                const double *H_dev);

/* Advances nsteps time steps (Sec. 2.1 evolution equation). */
lbm_status lbm_step(lbm_ctx *ctx, int32_t nsteps);

/* Macroscopic fields of the canonical state at the current time into device
 * FP64 buffers (any may be NULL): rho[n], u[3][n] (the prescribed velocity in
 * advection-only mode), H[n] = sum h (+ Q/2 with a source).  Solid nodes
 * report 0. */
lbm_status lbm_macroscopic(lbm_ctx *ctx, double *rho_dev, double *u_dev, double *H_dev);

/* Population state as FP64 device arrays [Q][n]: which = 0 the canonical
 * (pre-collision) state at time t, which = 1 the stored post-collision state
 * of step t-1.  lattice 0 = f, 1 = h.  Solid nodes carry no state and read
 * as zeros. */
lbm_status lbm_get_populations(lbm_ctx *ctx, int32_t lattice, int32_t which, double *dst_dev);

/* Replaces the stored post-collision state (which = 1 layout) of one lattice
 * from a device FP64 array [Q][n] and sets the time to t.  With
 * LBM_FP32_SR or LBM_FP16_SR storage the values are rounded stochastically
 * with the draws of time t (the same t gives the same stored state). */
lbm_status lbm_set_populations(lbm_ctx *ctx, int32_t lattice, const double *src_dev, int64_t t);

/* FP64 reductions of the canonical state at the current time (synchronises):
 *   out[0] = sum rho, out[1] = sum H over non-solid nodes,
 *   out[2] = heat injected by the wall links of group `group` during the
 *            last step: sum over its links of h_opp(x_b, t) - h*_i(x_b, t-1)
 *            (Eq. heat_flux_thorough_heater),
 *   out[3 + j] = section flux sum_a e_ax h_a over the non-solid nodes of
 *            column x = columns[j] (Eq. heat_flux_section), j < n_columns.
 * nout must be >= 3 + n_columns.  Returns LBM_EDIVERGED if out[0] or out[1]
 * is not finite. */
lbm_status lbm_reduce(lbm_ctx *ctx, int32_t group, const int32_t *columns, int32_t n_columns,
                      double *out, int32_t nout);

/* lbm_reduce() for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same outputs, computed by the same kernels, with the scratch of the
 * reduction (first-pass partial sums, the device result vector and the
 * column list, 17,176 bytes) in a static device array that each GPU holds
 * once for the life of the process, instead of the context's workspace.  The
 * macroscopic pass still writes its per-node fields into the workspace the
 * caller gave lbm_create().  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call).  n_columns above 64, the array's capacity, is
 * LBM_EINVAL.  Calls on one GPU share that array: calls that overlap on one
 * GPU (from several threads or streams) race; every call overwrites what it
 * reads.  Synchronises. */
lbm_status lbm_reduce_noalloc(lbm_ctx *ctx, int32_t group, const int32_t *columns, int32_t n_columns, double *out,
                              int32_t nout);

/* Nusselt number of a heated body (Sec. 4.4: Nu = varsigma D / k with
 * varsigma = qdot / (pi D (T_wall - T_in)); heat fluxes of Eqs.
 * heat_flux_thorough_heater and heat_flux_section), in FP64 from the
 * reductions of lbm_reduce() (synchronises).  group: the heater's group;
 * x_in, x_out: the upstream and downstream section columns; k is the
 * context's conductivity.  Per unit depth (a D3Q27 lattice with nz layers
 * divides by nz).  out[5]:
 *   out[0] = Nu = qdot / (pi k (T_wall - T_in) nz),
 *            qdot = (q_s + q_out - q_in) / 2 (heater flux and the energy the
 *            flow gains between the sections, averaged; equal when steady),
 *   out[1] = Nu from the heater flux alone, q_s / (pi k (T_wall - T_in) nz),
 *   out[2] = q_s, out[3] = q_in, out[4] = q_out (as out[2..4] of lbm_reduce).
 * Returns LBM_EINVAL for nout < 5, k <= 0, T_wall == T_in or a column outside
 * [0, nx), and LBM_EDIVERGED as lbm_reduce() does. */
lbm_status lbm_nusselt(lbm_ctx *ctx, int32_t group, int32_t x_in, int32_t x_out, double T_wall, double T_in,
                       double *out, int32_t nout);

/* ---- discrete adjoint ----------------------------------------------------
 * Reverse mode of the advection-diffusion step with a source Q (App. D) for
 * contexts with with_ns = 0 and the central-moment collision of h, periodic
 * or with geometry (ABB/IABB walls of Eq. IABB, EQ nodes, outlets); other
 * contexts return LBM_EUNSUPPORTED.  Not in the paper: the reverse
 * step is the exact transpose of the forward step.  That step is affine in
 * (state, Q) for a prescribed velocity, so the reverse step needs no forward
 * state.  Solid nodes carry no state: their lambda is ignored on input and
 * zero on output.
 * lambda: adjoint of the canonical (pre-collision) state, device [Q][n] in
 * the arithmetic type (double for LBM_FP64 and LBM_FP32_SR, float otherwise); dJdQ: device
 * FP64 [n], an accumulator over all reverse steps. */

/* Objective J = 1/2 sum_x (H(x) - H_target(x))^2 over the non-solid nodes of
 * the canonical state at the current time (H = sum h + Q/2).  Writes lambda =
 * dJ/d(state) (every direction H - H_target, zero at solid nodes), sets
 * dJdQ = (H - H_target)/2 (the direct dependence through Q/2) and returns J
 * (synchronises).  H_target: device FP64 [n]. */
lbm_status lbm_objective(lbm_ctx *ctx, const double *H_target_dev, void *lambda_dev, void *dJdQ_dev,
                         double *J);

/* Objectives summed over several times (tracking H along the run): the two
 * halves of lbm_objective.  lbm_objective_residual writes resid = H -
 * H_target of the canonical state at the current time (zero at solid nodes)
 * and returns its J = 1/2 sum resid^2 (synchronises); lbm_adjoint_seed turns a
 * stored residual into the adjoint seed, lambda = resid in every direction and
 * dJdQ = resid / 2, added to what the buffers hold when accumulate != 0 and
 * written over it otherwise (lbm_objective = residual, then seed with
 * accumulate = 0).  A reverse sweep adds the seed of time t after the reverse
 * step that yields lambda at t; the residuals come from the forward states,
 * which a checkpointed sweep recomputes segment by segment.  resid: device
 * FP64 [n]; lambda, dJdQ as for lbm_objective.  Same contexts as the adjoint;
 * LBM_EINVAL for NULL buffers. */
lbm_status lbm_objective_residual(lbm_ctx *ctx, const double *H_target_dev, double *resid_dev, double *J);
lbm_status lbm_adjoint_seed(lbm_ctx *ctx, const double *resid_dev, void *lambda_dev, void *dJdQ_dev,
                            int32_t accumulate);

/* One reverse step: lambda_next = dJ/d(state at t+1) -> lambda_prev =
 * dJ/d(state at t), and dJdQ += dJ/dQ through the collision of step t
 * (may be NULL).  The two lambda buffers must be distinct.  Uses only the
 * context's parameters and velocity field, not its population state. */
lbm_status lbm_adjoint_step(lbm_ctx *ctx, const void *lambda_next_dev, void *lambda_prev_dev, void *dJdQ_dev);

/* Bytes of a raw state snapshot (populations in storage layout + header). */
size_t lbm_state_bytes(const lbm_ctx *ctx);

/* Raw snapshot of the stored state and time into / from a device buffer of
 * lbm_state_bytes() bytes (checkpoint / restart; same params required). */
lbm_status lbm_save_state(lbm_ctx *ctx, void *dst_dev);
lbm_status lbm_load_state(lbm_ctx *ctx, const void *src_dev);

/* Current time step of the context. */
int64_t lbm_time(const lbm_ctx *ctx);

/* Opt-in per-kernel timing of the next max_steps steps: HIP events are
 * recorded on the context's stream around each bulk and each boundary-node
 * launch.  lbm_profile_end() (synchronises) returns the summed kernel times in
 * milliseconds and the number of timed steps, and stops the timing. */
lbm_status lbm_profile_begin(lbm_ctx *ctx, int32_t max_steps);
lbm_status lbm_profile_end(lbm_ctx *ctx, double *bulk_ms, double *boundary_ms, int64_t *steps);

/* Waits for the context's stream (synchronises). */
lbm_status lbm_sync(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
