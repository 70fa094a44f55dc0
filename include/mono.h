/*
 * mono.h - C interface of libmono, an MI355X (gfx950) implementation of the
 * dual adaptive explicit time integration (DAETI) method for the cardiac
 * monodomain equation (Mountris & Pueyo, "A dual adaptive explicit time
 * integration algorithm for efficiently solving the cardiac monodomain
 * equation").
 *
 * Problem (paper Sec. 2, eq. 1):  dV/dt = -I_ion(V, y)/C + div(D grad V) in
 * Omega, with zero flux on the boundary.  Strang splitting (Sec. 2, eq. 2)
 * advances one outer step dt as B(dt/2) A(dt) B(dt/2):
 *   B: l forward Euler substeps of dt_ad = dt/(2l) of dV/dt = -M_L^-1 K V + s,
 *      with l from the Gershgorin step dt_s of eq. (3);
 *   A: every node advances its cell model with its own k substeps of dt/k,
 *      k = min(k0 + floor|dV/dt|, k_max), k0 = 5 if dV/dt > 0 else 1,
 *      k_max = floor(dt/dt0); gates by Rush-Larsen, the rest forward Euler.
 *
 * Conventions for every function:
 *   - The return value is a mono_status; MONO_OK is 0.  On failure
 *     mono_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).  No C++ exception crosses this interface.
 *   - NULL handles, NULL required pointers and bad sizes give MONO_EINVAL.
 *   - Host arrays passed in are read during the call only (copied); the
 *     library never keeps a pointer to caller memory except device buffers
 *     explicitly registered through mono_debug().
 *   - Device memory of a simulation is owned by the library and released by
 *     mono_destroy().  The HIP stream given at creation is borrowed: every
 *     kernel and copy of the simulation is enqueued on it.
 *   - Functions whose name says "async" only enqueue work; the others
 *     synchronise the stream before returning.
 *   - A non-finite V seen by the reaction kernel latches the simulation; the
 *     next synchronising call returns MONO_ENONFINITE and later stepping
 *     returns MONO_ESTATE until mono_set_state() rewrites V.
 *   - A simulation is not thread-safe; distinct simulations are independent.
 */
#ifndef MONO_H
#define MONO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mono_sim mono_sim;

typedef enum {
  MONO_OK = 0,
  MONO_EINVAL = -1,       /* bad argument or mesh                           */
  MONO_ENOMEM = -2,       /* device or host allocation failed               */
  MONO_EDEVICE = -3,      /* a HIP runtime call failed                      */
  MONO_ESTATE = -4,       /* call not valid in the simulation's state       */
  MONO_EUNSUPPORTED = -5, /* valid request the library does not implement   */
  MONO_ENONFINITE = -6    /* a NaN/Inf potential appeared during stepping   */
} mono_status;

typedef enum { MONO_F64 = 0, MONO_F32 = 1 } mono_precision;

/* Elements; the value is the number of element nodes, and with dim it
 * names the element.  Q1 (2^dim Gauss points): LINE2 x-,x+ (dim 1); QUAD4
 * (0,0) (1,0) (1,1) (0,1) in reference coordinates (dim 2); HEX8 the QUAD4
 * face at z- followed by the QUAD4 face at z+ (dim 3).  P1 simplices (one
 * point at the centroid, exact for their constant gradients; the lumped mass
 * of a node is the element's volume / (dim + 1)): TRI3 (dim 2) and TET4
 * (dim 3, the value of QUAD4 in 3D), any node order with positive
 * orientation (det [x1 - x0, ..., x_dim - x0] > 0). */
typedef enum {
  MONO_LINE2 = 2,
  MONO_TRI3 = 3,
  MONO_QUAD4 = 4,
  MONO_TET4 = 4,
  MONO_HEX8 = 8
} mono_element;

/* Cell models.  State 0 is always V.
 *  LINEAR   dV/dt = -g (V - E)                    params {g, E}, 1 state
 *  MS       Mitchell & Schaeffer (2003)           params {tau_in, tau_out,
 *           tau_open, tau_close, v_gate}, states {v, h}, v dimensionless
 *  TP06_EPI ten Tusscher & Panfilov (2006) epicardial, V in mV,
 *           params {Ko [mM], gNa, gCaL, gKr, gKs, gK1 scalings}, 19 states
 *           {V, K_i, Na_i, Ca_i, Ca_ss, Ca_SR, Rbar, m, h, j, xr1, xr2, xs,
 *            r, s, d, f, f2, fCass}
 *  TP06_TYPES the same with a transmural cell type per node in a 7th
 *           parameter row: 0 epicardial, 1 endocardial (G_to = 0.073, the
 *           endocardial s gate), 2 M cell (G_Ks = 0.098); heterogeneous
 *           tissue in one simulation.  In mono_backward the type row is
 *           a label: its gradient entry is 0.
 *  TP06_FIBRO myocytes and fibroblasts in one tissue (Sec. 3.2): 9 rows,
 *           those of TP06_EPI, then a node class (0 epicardial TP06
 *           myocyte, 1 fibroblast), then g_f [1/ms] and E_f [mV] of the
 *           fibroblasts' passive membrane dV/dt = -g_f (V - E_f) (defaults
 *           0.0216 and -49.6).  A fibroblast node keeps its other 18 state
 *           rows; its substep count follows the same k rule.  Any class
 *           other than 0 or 1 is EINVAL.  In mono_backward the class row is
 *           a label (gradient entry 0).                                     */
typedef enum {
  MONO_MODEL_LINEAR = 0,
  MONO_MODEL_MS = 1,
  MONO_MODEL_TP06_EPI = 2,
  MONO_MODEL_TP06_TYPES = 3,
  MONO_MODEL_TP06_FIBRO = 4
} mono_model;

/* DAETI: adaptive k and l (Sec. 2).  OSTAR: l = 1 (adaptive reaction only).
 * OST: k = l = 1 (the caller picks dt).  The comparison methods of Sec. 3. */
typedef enum { MONO_DAETI = 0, MONO_OSTAR = 1, MONO_OST = 2 } mono_method;

/* Storage of the diffusion operator.  ELL: general sparse rows (column index
 * + value per slot, slot-major).  STENCIL: the symmetric operator stored once
 * per edge at a fixed set of node-index offsets, usable when every edge
 * (i, j) of an instance has j - i in a set of at most 13 positive offsets
 * (structured node numbering).  AUTO picks STENCIL when it applies. */
enum { MONO_LAYOUT_AUTO = 0, MONO_LAYOUT_ELL = 1, MONO_LAYOUT_STENCIL = 2 };

/* Fields of mono_get_state / mono_set_state. */
enum {
  MONO_FIELD_V = 0,      /* transmembrane potential                         */
  MONO_FIELD_VPREV = 1,  /* V at the previous reaction entry                */
  MONO_FIELD_LAT = 2,    /* activation time [ms], FP64, -1 = not activated   */
  MONO_FIELD_K = 3,      /* reaction substeps k of the last step (get only)  */
  MONO_FIELD_APD = 4,    /* APD90 [ms], FP64 (get only), -1 = not measured;
                            needs mono_track_apd                             */
  MONO_FIELD_TUP = 5,    /* time of the steepest sampled upstroke [ms], FP64
                            (get only), -1 = not activated                   */
  MONO_FIELD_STATE0 = 16 /* + j: cell state j (j = 0 is V)                  */
};

typedef struct {
  int32_t dim;                  /* 1, 2 or 3                                    */
  int64_t n_nodes;
  const double *xyz;            /* n_nodes * dim node coordinates [cm]          */
  int32_t etype;                /* mono_element matching dim                    */
  int64_t n_elems;
  const int32_t *conn;          /* n_elems * etype 0-based node indices         */
  const double *D_elem;         /* n_elems * dim * dim symmetric positive
                                   definite diffusion tensors [cm^2/ms]         */
  const double *sigma_node;     /* n_nodes conductivity scales or NULL (= 1):
                                   off-diagonal K entries are multiplied by
                                   (sigma_i + sigma_j)/2, rows keep zero sum    */
  int32_t prec;                 /* mono_precision of V, states and operator     */
  void *stream;                 /* hipStream_t, borrowed; NULL = the library
                                   creates (and later destroys) its own stream  */
  int32_t n_instances;          /* >= 1; independent tissues concatenated       */
  const int64_t *inst_node_off; /* n_instances+1 node offsets, or NULL if 1;
                                   no element may join two instances            */
  int32_t layout;               /* MONO_LAYOUT_*                                 */
  int32_t sigma_device;         /* nonzero: sigma_node is device memory (FP64,
                                   ready when the call is made); the library
                                   copies it to the host for the FP64 assembly */
} mono_mesh_desc;

typedef struct {
  double dt_s;        /* eq. (3) stable diffusion step [ms] (per instance)     */
  double G_max;       /* max_i (k_ii + sum_j |k_ij|) / m_ii  [1/ms]            */
  double lambda_est;  /* power-iteration estimate of lambda_max(M_L^-1 K), or 0 */
  double dt_ad;       /* diffusion substep [ms] for the last prepared dt       */
  double dt;          /* outer step of the last prepare [ms]                   */
  double t;           /* simulated time of the current time level [ms]         */
  int64_t step;       /* index of the current time level                       */
  int64_t nnz;        /* stored nonzeros of K including the diagonal           */
  int32_t l;          /* diffusion substeps per half step                      */
  int32_t k_max;      /* reaction substep cap                                  */
  int32_t layout;     /* MONO_LAYOUT_ELL or MONO_LAYOUT_STENCIL in use          */
  int32_t n_instances;
  int32_t n_states;
  int32_t ell_width;  /* ELL slots per row, or stencil offsets per instance    */
  int32_t row_classes; /* distinct stencil rows of a single instance when the
                          diffusion can read rows by class (at most 65535
                          classes, and each row array under 2 GiB), else 0    */
  int32_t grid_rows;   /* 1 when the stencil offsets are those of a structured
                          grid numbered x fastest (row-sharing diffusion)      */
  int32_t diff_fused;  /* 1 when the grid is a whole 3D nx x ny x nz block
                          with no weight past its faces and row ends, so the
                          fused half-step diffusion (mono_launch.diff_fuse)
                          can run on it                                       */
  int32_t diff_launches; /* diffusion launches per half step under the current
                          launch shape and prepared l (0 before mono_prepare) */
} mono_info;

/* Assemble K and the row-sum lumped mass M_L of the FE diffusion problem
 * (Sec. 2, eq. 2b-c) in FP64 on the host, upload the chosen layout, and run
 * the Gershgorin kernel (eq. 3) in FP64 on the device.  Errors: EINVAL for a
 * bad description, an index out of range, a non-positive element Jacobian or
 * an element joining two instances; ENOMEM; EDEVICE. */
mono_status mono_create_mesh(const mono_mesh_desc *desc, mono_sim **out);

/* Choose the cell model.  params: n_params * n_nodes SoA, or NULL for the
 * model's defaults (uniform rows are stored once).  init_state: n_states *
 * n_nodes SoA or NULL for the model's published initial values.  dt0 [ms] is
 * the largest stable cell step: k_max = max(1, floor(dt/dt0)) (Sec. 2).
 * Resets time, V_prev (= V) and activation times.  Errors: EINVAL for an
 * unknown model, a wrong n_params, dt0 <= 0 or a TP06_TYPES cell type other
 * than 0, 1 or 2; ENOMEM; EDEVICE. */
mono_status mono_set_cell_model(mono_sim *sim, int32_t model, int32_t n_params,
                                const double *params, const double *init_state, double dt0);

/* Threshold of the activation-time detector (first upward crossing of the
 * V samples taken at reaction entry, linearly interpolated, FP64). */
mono_status mono_set_lat_threshold(mono_sim *sim, double v_threshold);

/* Add a stimulus: `amplitude` (dV/dt units) is added to the diffusion
 * right-hand side of the listed nodes for every substep whose start time tau
 * has t_on <= tau < t_on + duration.  At most 8 stimuli per simulation. */
mono_status mono_add_stimulus(mono_sim *sim, int64_t n, const int32_t *nodes, double t_on,
                              double duration, double amplitude);

/* Method flags.  dvdt_source 0: dV/dt = (V_entry - V_prev_entry)/dt (0 on
 * the first step); 1: the cell model's own dV/dt at reaction entry.
 * l_round 0: floor as in the paper; 1: ceiling (dt_ad <= dt_s). */
mono_status mono_set_method(mono_sim *sim, int32_t method, int32_t dvdt_source, int32_t l_round);

/* Advance n_outer_steps steps of size dt [ms] (async).  flags: bit 0
 * (MONO_STEP_EAGER) = launch kernels one by one instead of replaying a cached
 * HIP graph of graph_steps outer steps; bit 1 (MONO_STEP_TIMED) = launch one
 * by one, every step kernel with a start and a stop event that the command
 * processor records at the kernel's begin and end, and add the durations to
 * the totals read by MONO_DEBUG_KTIMES (this mode synchronises); bit 2
 * (MONO_STEP_CAPTURE) = only capture the graphs that a graph-mode call with
 * the same n_outer_steps and dt would replay (graph_steps steps and the
 * remainder), so that the call itself does no capture work; nothing runs. */
enum { MONO_STEP_EAGER = 1, MONO_STEP_TIMED = 2, MONO_STEP_CAPTURE = 4 };
mono_status mono_step(mono_sim *sim, int64_t n_outer_steps, double dt, uint32_t flags);

/* Copy `count` (= n_nodes) values of a field to host memory as FP64. */
mono_status mono_get_state(mono_sim *sim, int32_t field, double *host_dst, int64_t count);

/* Copy a field device-to-device in the simulation's precision (FP64 for
 * LAT, uint8 for K); async on the simulation's stream. */
mono_status mono_get_state_device_async(mono_sim *sim, int32_t field, void *dev_dst);

/* Overwrite a field from host FP64 values (V, VPREV, LAT, STATE0+j). */
mono_status mono_set_state(mono_sim *sim, int32_t field, const double *host_src, int64_t count);

/* Set the current time level (t = step * dt). */
mono_status mono_set_time_level(mono_sim *sim, int64_t step);

/* Prepare for outer step dt: l, dt_ad, k_max (also done by mono_step). */
mono_status mono_prepare(mono_sim *sim, double dt);

/* Diagnostics of instance `inst` (0-based). */
mono_status mono_get_info(mono_sim *sim, int32_t inst, mono_info *out);

/* Action-potential duration at 90 % repolarisation (APD90, paper Sec. 3.1
 * and Sec. 4, measured there from the time of the maximum upstroke
 * derivative), tracked per node from the same reaction-entry samples V_n at
 * t_n = (n + 1/2) dt that give the activation time.  For the first activation
 * of a node (first n with V_{n-1} < threshold <= V_n): V_rest = V_{n-1}; the
 * upstroke time is the midpoint of the sampled interval with the largest
 * slope (V_n - V_{n-1}) / dt from that interval on (the first such interval
 * on ties); V_90 = V_max - 0.9 (V_max - V_rest) with V_max the largest sample
 * since activation; repolarisation is the first interval after activation
 * with V_{n-1} >= V_90 > V_n, its time interpolated linearly; APD90 is the
 * repolarisation time minus the upstroke time.  Times and slopes in FP64 in
 * every precision.  on = 1 allocates the trackers (5 doubles per node) and
 * resets them (every node not activated), on = 0 frees them.  Tracking
 * follows ordinary steps (mono_step, mono_step_loss); the taped forward run
 * and the adjoint sweep do not update it, and snapshots do not carry it.
 * Errors: EINVAL, ESTATE (no model), ENOMEM. */
mono_status mono_track_apd(mono_sim *sim, int32_t on);

/* Normalised root-mean-square error of eq. (4):
 * sqrt(mean_i (u_hat_i - u_i)^2) / (max_i u_i - min_i u_i) over the n host
 * values (reference u, e.g. OST's LAT or APD90 per node); entries where either
 * value is negative (not measured) are left out of the mean and of the range.
 * *out = NaN when no entry is left or the range is 0.  Errors: EINVAL. */
mono_status mono_nrmse(const double *u_hat, const double *u, int64_t n, double *out);


/* Estimate lambda_max(M_L^-1 K) of every instance by `iters` FP64 power
 * iterations on the device (generalised Rayleigh quotient, a lower bound)
 * and check dt_ad < 2/lambda_est for the last prepared dt. */
mono_status mono_estimate_lambda(mono_sim *sim, int32_t iters);

/* Launch shapes of a simulation (defaults: 256, 1, 1, 256, 32, 0, 1, 1, 0, 0).  Block
 * sizes 128, 256 or 512 lanes (the FP32 reaction also 1024); rows per lane of the stencil diffusion kernel
 * 1, 2 or 4 (FP64: 1 or 2; ignored by the ELL layout); XCD remap 0/1 (deal
 * contiguous row ranges to each of the 8 XCDs); graph_steps 1..8192 outer
 * steps per captured HIP graph (a whole run can be one graph); react_sort
 * 0/1: every reaction workgroup first decides the k of all its nodes and
 * orders them by k in LDS, so that a wavefront runs one substep count where
 * it can; diff_classes 0/1 (default 1): where mono_info.row_classes > 0 the
 * stencil diffusion reads each row's weights and 1/m from a table of the
 * distinct rows through a 2-byte class id instead of per-row arrays, and
 * rows per lane (1, 2, 4, 8 or 16, any precision) count the rows each lane
 * sweeps in turn; diff_wave_rows 0/1 (default 1): with row classes on a
 * structured grid (mono_info.grid_rows) a wavefront loads each neighbouring
 * grid row once and passes x-neighbours between lanes; diff_fuse 0/1
 * (default 0): on a 3D structured grid that takes it (mono_info.diff_fused)
 * with row classes in use, up to 4 of the l substeps of a half step run in one
 * launch (temporal blocking: a workgroup marches z through a tile widened by
 * one node per fused substep on every side, keeping the intermediate levels
 * in LDS); a half step takes ceil(l / 4) such launches when l >= 2;
 * diff_fuse_planes 0..4096: z planes each workgroup of that kernel produces
 * (0 = chosen from the grid so that the launch fills the chip).
 * Results do not depend on the shape (bitwise, for finite potentials). */
typedef struct {
  int32_t diff_block;
  int32_t diff_rows_per_lane;
  int32_t diff_xcd_remap;
  int32_t react_block;
  int32_t graph_steps;
  int32_t react_sort;
  int32_t diff_classes;
  int32_t diff_wave_rows;
  int32_t diff_fuse;
  int32_t diff_fuse_planes;
} mono_launch;
mono_status mono_set_launch(mono_sim *sim, const mono_launch *cfg);
mono_status mono_get_launch(mono_sim *sim, mono_launch *out);

/* Replace the borrowed stream. */
mono_status mono_set_stream(mono_sim *sim, void *stream);

/* Wait for the simulation's stream; reports MONO_ENONFINITE if latched. */
mono_status mono_sync(mono_sim *sim);

/* Device memory hook (process-wide): every device buffer of a simulation is
 * then obtained from alloc(bytes, ctx) and returned with free_(ptr, ctx)
 * instead of hipMalloc / hipFree, e.g. so that a framework's caching
 * allocator owns it.  alloc must return device memory of the current device,
 * aligned to 256 bytes, or NULL (the calling function then fails with
 * MONO_ENOMEM); the library synchronises its stream before it frees a buffer.
 * Both NULL restores hipMalloc / hipFree.  Only while no simulation exists
 * (MONO_ESTATE otherwise); one NULL of the two is MONO_EINVAL. */
mono_status mono_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                               void (*free_)(void *ptr, void *ctx), void *ctx);

void mono_destroy(mono_sim *sim);
const char *mono_last_error(void);

/* Operations of one substep of a cell model at the given state and
 * parameters (host arrays of the model's sizes), counted on the reaction
 * kernel's own model code: out[7] = {add/sub, mul, div, exp, log, sqrt,
 * compare}.  The count follows the branches the state selects.  Host only. */
mono_status mono_model_flops(int32_t model, const double *state, const double *params,
                             int64_t *out);

/* Host evaluation, in FP64, of the reaction kernel's own model code: one
 * substep of length h applied to state[] in place, and the reverse-mode
 * product of that substep (lam: adjoint of the output in, of the input out;
 * gp[n_params]: parameter adjoints added).  clamp != 0 holds V fixed.  For
 * checking the adjoint against finite differences without a device. */
mono_status mono_model_substep_host(int32_t model, double *state, const double *params,
                                    double h, int32_t clamp);
mono_status mono_model_vjp_host(int32_t model, const double *state, const double *params,
                                double h, int32_t clamp, double *lam, double *gp);

/* Apply one phase of outer step `step` to the current state (testing the
 * kernels one launch at a time).  phase 0: diffusion substep `m` of the first
 * half step; 1: the reaction step; 2: diffusion substep `m` of the second
 * half step.  Synchronising. */
mono_status mono_apply_phase(mono_sim *sim, int32_t phase, int64_t step, int32_t m);

/* --- adjoint ---------------------------------------------------------------
 * Loss L = sum over outer steps n < n_steps and sensors q of
 * (V[nodes[q]] at reaction entry of step n - target[n * n + q])^2, with the
 * step index n absolute (time level n*dt); targets are copied.  Sensor nodes
 * must be distinct. */
mono_status mono_set_sensors(mono_sim *sim, int32_t n, const int32_t *nodes, const double *target,
                             int64_t n_steps);

/* Advance n_steps outer steps like mono_step (kernels launched one by one)
 * and copy V at the sensors at reaction entry of every step to host out
 * (n_steps x sensors, FP64): synthetic measurements for a loss target.
 * Synchronising; the targets given with the sensors are not used. */
mono_status mono_sample_sensors(mono_sim *sim, int64_t n_steps, double dt, double *out);

/* mono_sample_sensors for callers that cannot allocate device memory (code
 * that must not call hipMalloc: tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same samples, staged in a static
 * device buffer of the library (4 MiB per GPU, held until the process ends)
 * instead of a per-call allocation.  No allocation of any kind.  Limits and
 * errors: n_steps x sensors <= 524288 (EINVAL beyond); the simulation must
 * already be prepared for this dt (mono_prepare or an earlier step with the
 * same dt; ESTATE otherwise).  Every call on one GPU shares that GPU's
 * buffer: calls that overlap on one GPU (several threads, or several
 * simulations on different streams) race and must be serialised by the
 * caller.  Synchronising. */
mono_status mono_sample_sensors_noalloc(mono_sim *sim, int64_t n_steps, double dt, double *out);

/* Advance n_steps outer steps from the current time level like mono_step,
 * keeping snapshots of the state at segment starts (segments of ckpt_every
 * steps), and return the loss (FP64).  Synchronising.  Needs k_max <= 16.
 * EUNSUPPORTED with a clamped potential.  Memory: the snapshots (see
 * mono_set_checkpointing) plus a tape of one segment (ckpt_every steps of
 * diffusion inputs, reaction-entry states and substep counts). */
mono_status mono_forward_taped(mono_sim *sim, int64_t n_steps, double dt, int32_t ckpt_every,
                               double *loss);

/* Checkpoint schedule of the next mono_forward_taped (not in the paper,
 * which has no adjoint: the reverse sweep needs the state at the start of
 * every segment it reverses).
 *  MONO_CKPT_UNIFORM (default): a snapshot at every segment start; the
 *      reverse sweep recomputes each segment once (for its tape).
 *  MONO_CKPT_BINOMIAL: at most max_snapshots (>= 2) snapshot buffers, the
 *      run's start included; states in between are recomputed by forward
 *      advances of whole segments from an earlier snapshot, in the order
 *      that minimises the number of advances over recursive splits
 *      (binomial checkpointing, Griewank & Walther's revolve).  Gradients
 *      are bitwise those of the uniform schedule: every segment is reversed
 *      from the same state, in the same order.
 * EINVAL for another schedule or fewer than 2 snapshots. */
enum { MONO_CKPT_UNIFORM = 0, MONO_CKPT_BINOMIAL = 1 };
mono_status mono_set_checkpointing(mono_sim *sim, int32_t schedule, int32_t max_snapshots);

/* Figures of the last taped run's schedule into out[6]: {schedule, snapshot
 * buffers, segments, whole-segment forward advances of the last
 * mono_backward, snapshot bytes, segment tape bytes (two segment tapes in
 * the uniform schedule when memory allows: one segment is recomputed on a
 * second stream while the segment after it is reversed)}.  ESTATE before a
 * taped run. */
mono_status mono_checkpoint_info(mono_sim *sim, int64_t *out);

/* The number of whole-segment forward advances the binomial plan needs to
 * reverse n_segments with max_snapshots buffers (host only, no device).
 * EINVAL for fewer than 2 buffers when n_segments > 1. */
mono_status mono_checkpoint_plan(int64_t n_segments, int32_t max_snapshots, int64_t *advances);

/* Gradient of the last taped run's loss by a reverse sweep that recomputes
 * each segment from its checkpoint (the k each node took and l are held
 * fixed: the loss is piecewise smooth in the parameters).  grad_sigma[n_nodes]:
 * dL/dsigma_i of the per-node conductivity scales (of 1 where the mesh had
 * none); grad_params[n_params]: for each parameter row a, the derivative
 * with respect to a common multiplier of that row at 1,
 * sum_i p_i[a] dL/dp_i[a].  Either pointer may be NULL.  Leaves the state
 * where the taped run ended.  FP64 accumulation of both gradients. */
mono_status mono_backward(mono_sim *sim, double *grad_sigma, double *grad_params);

/* The sensitivity problem with its inputs and outputs in device memory (for
 * a differentiable caller whose tensors live on the GPU; the chain rule
 * through the scalings is applied here).
 *
 * mono_set_param_scalings: multiply parameter rows rows[0..n-1] (host array,
 * distinct, of the model's parameter rows; a cell-type or node-class row is
 * EINVAL) of every node by the scalings c[0..n-1] (device memory, FP64,
 * ready when the call is made; copied to the host, where uniform rows live
 * as kernel arguments), relative to the parameters of the last
 * mono_set_cell_model: a second call before the next mono_set_cell_model is
 * ESTATE; a scaling that is zero or not finite is EINVAL.  Per-node rows are
 * scaled on the device in the simulation precision.
 *
 * mono_forward_taped_device: mono_forward_taped writing the loss (FP64) to
 * device memory loss instead of the host; synchronising.
 *
 * mono_backward_device: mono_backward writing dL/dsigma (n_nodes FP64) to
 * device memory grad_sigma and, for the scalings of mono_set_param_scalings,
 * dL/dc_j = sum_i base_i[rows_j] dL/dp_i[rows_j] = grad_params[rows_j] / c_j
 * (n FP64, the same sums in the same order as mono_backward) to device
 * memory grad_scalings; either may be NULL (grad_scalings must be NULL when
 * no scalings were set: ESTATE).  Synchronising. */
mono_status mono_set_param_scalings(mono_sim *sim, int32_t n, const int32_t *rows,
                                    const double *scalings);
mono_status mono_forward_taped_device(mono_sim *sim, int64_t n_steps, double dt,
                                      int32_t ckpt_every, double *loss);
mono_status mono_backward_device(mono_sim *sim, double *grad_sigma, double *grad_scalings);

/* Test hooks.  `what`:
 *  MONO_DEBUG_KTRACE: arg -> mono_ktrace (device buffers n_steps x n_nodes,
 *      uint8, row = step - base_step): record the k each node picks and/or
 *      replay k from a given trace instead of the rule.  A replayed entry is
 *      clamped to [1, k_max] (and recorded as clamped in MONO_FIELD_K and in
 *      the adjoint's tape); steps outside the trace use the rule.
 *  MONO_DEBUG_VCLAMP: arg -> int32 (1 = the reaction leaves V unchanged).
 *  MONO_DEBUG_FORCE_L: arg -> int32 (l override for every instance, 0 = off).
 *  MONO_DEBUG_STATS: arg -> int64[4] {sum of k over nodes and steps, sum over
 *      wavefronts of 64 * max k, node-steps counted, node-steps at k_max}
 *      (synchronising; counters run only while enabled with arg int32 1 via
 *      MONO_DEBUG_STATS_ENABLE).
 *  MONO_DEBUG_KTIMES: arg -> double[5]; returns {diffusion kernel ms,
 *      diffusion launches, reaction kernel ms, reaction launches} of the
 *      MONO_STEP_TIMED steps so far; the totals are reset when arg[4] != 0
 *      on entry.
 *  MONO_DEBUG_TIME_DIFFUSION: arg -> double[2]; arg[0] = an even number R
 *      of repetitions on entry; runs R diffusion substeps (the first
 *      substep of the first half step at the current time level, alternating
 *      between the two potential buffers; where the half steps run fused,
 *      about R / l first half steps launched as stepping launches them, an
 *      even number of launches) captured in one HIP graph, timed by events
 *      around the graph launch, and returns the mean ms per substep in
 *      arg[1].  The potential is advanced by those R substeps:
 *      for benchmarking simulations only.  Synchronising; needs
 *      mono_prepare. */
enum {
  MONO_DEBUG_KTRACE = 1,
  MONO_DEBUG_VCLAMP = 2,
  MONO_DEBUG_FORCE_L = 3,
  MONO_DEBUG_STATS = 4,
  MONO_DEBUG_STATS_ENABLE = 5,
  MONO_DEBUG_KTIMES = 6,
  MONO_DEBUG_TIME_DIFFUSION = 7
};
typedef struct {
  int32_t mode;          /* bit 0 record, bit 1 replay; 0 = off          */
  uint8_t *record;       /* device, n_steps * n_nodes, or NULL            */
  const uint8_t *replay; /* device, n_steps * n_nodes, or NULL            */
  int64_t n_steps;
  int64_t base_step;
} mono_ktrace;
mono_status mono_debug(mono_sim *sim, int32_t what, void *arg);

#ifdef __cplusplus
}
#endif
#endif /* MONO_H */
