/*
 * pinn_jet.h - C ABI of the MI355X (gfx950) partial-jet PINN library.
 *
 * The library evaluates, for a tanh MLP u_theta(x) and a PDE residual r, the
 * derivative states the residual needs (the "partial jet"), the residual, the
 * mean-squared residual loss and its parameter gradient, following
 * Cao, Lu & Zhang, "Verified residual-specific explicit derivative kernels for
 * physics-informed learning and discretized PDE adjoints":
 *   - layer map z = W a + b, a = tanh(z)                          (Eq. 1)
 *   - derivative states: d_i z = W d_i a, d_i a = tanh'(z) d_i z   (Eq. 2)
 *     d_ii z = W d_ii a, d_ii a = tanh'' (d_i z)^2 + tanh' d_ii z  (Eq. 3)
 *     and the same recursion to order 4 for pure derivatives        (Sec. 2.2)
 *   - only the channels the residual needs are propagated, and all channels of
 *     a layer go through one stacked GEMM with the bias on the value only
 *                                                                    (Sec. 2.2)
 *   - residuals: viscous Burgers and Kuramoto-Sivashinsky (Sec. 3.1.1),
 *     steady incompressible Navier-Stokes (Eq. 16), and a 3-D heat equation;
 *   - the parameter gradient is reverse-mode differentiation of the scalar
 *     loss (Sec. 2.2, Sec. 3.1.1), here a hand-written adjoint.
 *
 * General conventions
 *   - All array arguments are DEVICE pointers unless marked "host".  Arrays are
 *     row-major.  The caller owns every buffer it passes; the library owns only
 *     the plan's workspace (allocated in pinn_plan_create, freed in
 *     pinn_plan_destroy).  The step calls (forward / residual / backward) do not
 *     allocate and may be captured into a HIP graph.
 *   - Calls are asynchronous and ordered on `stream` (a hipStream_t passed as
 *     void*, NULL = the default stream).  Nothing is synchronised.  A device
 *     fault surfaces at the caller's next synchronisation.
 *   - Every function returns a pinn_status; it never throws or aborts.  On a
 *     non-OK status pinn_last_error() holds a message (per host thread).  All
 *     argument checks happen on the host before any device work is enqueued,
 *     so a call that fails a check has no effect.
 *   - A plan is not safe to use from two host threads at once.
 */
#ifndef PINN_JET_H
#define PINN_JET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pinn_status;
enum {
  PINN_OK = 0,
  PINN_ERR_ARG = -1,         /* a NULL pointer, a size out of range, a shape mismatch */
  PINN_ERR_UNSUPPORTED = -2, /* valid request this build does not implement */
  PINN_ERR_NOMEM = -3,       /* device allocation failed */
  PINN_ERR_DEVICE = -4,      /* a HIP call failed */
  PINN_ERR_STATE = -5,       /* backward without the matching residual call */
  PINN_ERR_CAP = -6          /* save_cap_bytes below the minimum saved state */
};

/* PDE kinds.  Input ordering and channel order (the order of the jet channels
 * in every jets array) are fixed per kind:
 *   PINN_BURGERS_1D  inputs (x, t), output u, coef = {nu}
 *                    r = u_t + u u_x - nu u_xx            channels: u, u_t, u_x, u_xx
 *   PINN_NS2D_STEADY inputs (x, y), outputs (u, v, p), coef = {Re}
 *                    r_c = u_x + v_y
 *                    r_u = u u_x + v u_y + p_x - (u_xx + u_yy)/Re
 *                    r_v = u v_x + v v_y + p_y - (v_xx + v_yy)/Re      (Eq. 16)
 *                    residual rows in the order (r_c, r_u, r_v)
 *                    channels: value, d/dx, d/dy, d2/dx2, d2/dy2 (for every output)
 *   PINN_KS_1D       inputs (x, t), output u, coef = {alpha, beta, gamma}
 *                    r = u_t + alpha u u_x + beta u_xx + gamma u_xxxx
 *                    channels: u, u_t, u_x, u_xx, u_xxx, u_xxxx
 *   PINN_HEAT_3D     inputs (x, y, z, t), output u, coef = {kappa}
 *                    r = u_t - kappa (u_xx + u_yy + u_zz) - sin(pi x) sin(pi y) sin(pi z) e^-t
 *                    channels: u, u_t, u_x, u_y, u_z, u_xx, u_yy, u_zz
 *   PINN_ANISO_2D    inputs (x, y), output u, coef = {c}; a test operator with a
 *                    mixed derivative (Eq. 3 with i != j), not one of the paper's
 *                    problems: r = u_xx + 2 c u_xy + u_yy
 *                    channels: u, u_x, u_y, u_xx, u_yy, u_xy
 *   PINN_BURGERS_BC  inputs (x, t), output u, no coefficient: a value-channel
 *                    test operator, r = u + sin(pi x), the Dirichlet data of the
 *                    [-1, 1] Burgers workload at points on t = 0 and x = +-1.  It
 *                    is not the paper's Burgers loss, whose initial and periodic
 *                    boundary terms (u and u_x) are composite-loss segments of
 *                    the PINN_BURGERS_1D kind (pinn_jet_loss)
 *                    channels: u                                                   */
enum { PINN_BURGERS_1D = 1, PINN_NS2D_STEADY = 2, PINN_KS_1D = 3, PINN_HEAT_3D = 4, PINN_ANISO_2D = 5,
       PINN_BURGERS_BC = 6 };

/* Operand type of the hidden-layer GEMMs.  Accumulation, the activation jet,
 * its adjoint, the residual and the loss are always FP32. */
enum { PINN_FP32 = 0, PINN_BF16 = 1, PINN_FP16 = 2 };

/* Plan flags. */
enum {
  PINN_VERIFY_F64 = 1u /* also produce FP64 loss and gradient reductions */
};

/* Network: L = n_layers affine maps; dims[0] = number of inputs, dims[L] =
 * number of outputs, dims[1..L-1] = hidden width w (all equal; a multiple of 32,
 * 32 <= w <= 512).  W[l] is a device array of dims[l+1] x dims[l] floats, b[l]
 * of dims[l+1] floats.  tanh follows layers 0..L-2; layer L-1 is linear.
 * Requires L >= 2.  The parameter values may change between calls; the shapes
 * must match the plan's. */
typedef struct {
  int32_t n_layers;
  const int32_t *dims;     /* host, n_layers + 1 entries */
  const float *const *W;   /* host array of n_layers device pointers */
  const float *const *b;   /* host array of n_layers device pointers */
} pinn_net;

typedef struct {
  int32_t kind;    /* PINN_BURGERS_1D ... */
  double coef[4];  /* see the PDE kinds above; unused entries ignored */
} pinn_pde;

typedef struct pinn_plan_s *pinn_plan;
typedef struct pinn_batch_s *pinn_batch;
struct pinn_adam_s;

/* Creates a plan for one network shape, PDE kind and maximum point count: the
 * channel set of the kind (the on-demand partial jet of Sec. 2.2, only the
 * derivative states the residual needs), the saved-state schedule and the
 * device workspace of the step calls.
 *   prec            PINN_FP32 / PINN_BF16 / PINN_FP16
 *   flags           0 or PINN_VERIFY_F64
 *   save_cap_bytes  upper bound on the device bytes kept between
 *                   pinn_jet_residual and pinn_jet_backward (the saved layer
 *                   states); 0 = no bound (store every layer).  Under a bound
 *                   the plan stores a subset of layers and recomputes the rest
 *                   during backward (results are bitwise identical).
 *                   PINN_ERR_CAP if even the smallest checkpoint set exceeds it.
 * Allocates all device workspace on the current HIP device. */
pinn_status pinn_plan_create(const pinn_net *net, const pinn_pde *pde, int64_t max_points,
                             int32_t prec, uint32_t flags, size_t save_cap_bytes,
                             pinn_plan *out);
pinn_status pinn_plan_destroy(pinn_plan plan);

/* Bytes of saved layer state the plan keeps at max_points, and its total
 * device workspace (host outputs; either may be NULL). */
pinn_status pinn_plan_memory(pinn_plan plan, size_t *saved_bytes, size_t *workspace_bytes);

/* Forward partial-jet pass (Eq. 1-3 and the recursion of Sec. 2.2).
 *   x     N x d_in floats (point-major)
 *   jets  d_out x C x N floats: jets[(o*C + c)*N + n] is channel c of output o
 *         at point n, channels in the PDE kind's order.
 * 1 <= N <= max_points.  Invalidates the state saved by pinn_jet_residual. */
pinn_status pinn_jet_forward(pinn_plan plan, const pinn_net *net, const float *x, int64_t N,
                             float *jets, void *stream);

/* Forward pass (Eq. 1-3, the stacked-channel GEMM of Sec. 2.2), the PDE
 * residual of the kind (Sec. 3.1.1; Eq. 16 for Navier-Stokes) and the
 * mean-squared residual loss of the training runs (Sec. 3.1).  Saves the state
 * pinn_jet_backward needs.
 *   r         n_res x N floats (may be NULL)
 *   loss      1 float: sum over residual rows of (1/N) sum_n r^2 (may be NULL)
 *   loss_f64  1 double, the same reduction in FP64; requires PINN_VERIFY_F64
 *             (may be NULL)
 *   jets      optional d_out x C x N output as in pinn_jet_forward (may be NULL) */
pinn_status pinn_jet_residual(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                              const float *x, int64_t N, float *r, float *loss,
                              double *loss_f64, float *jets, void *stream);

/* Parameter gradient by reverse-mode differentiation of the loss, which the
 * paper keeps for training (Sec. 2.2, Sec. 3.1.1): here the hand-written
 * adjoint of the jet recursion of Eq. 1-3, layer by layer from the residual.
 * Must follow pinn_jet_residual on the same plan with the same net
 * parameter pointers, x and N (PINN_ERR_STATE otherwise), and with the
 * parameter values of that call: the operand-type copies of the hidden
 * weights that call made are reused, while the first and last layers and the
 * biases are read again.  The library cannot tell whether the values behind
 * the pointers changed in between; if they did, the result mixes the two sets
 * of parameters.  Run pinn_jet_residual again after any update.
 *   r_bar    n_res x N cotangent of r, or NULL for the loss gradient (2 r / N)
 *   dW, db   host arrays of n_layers device pointers shaped like W and b;
 *            overwritten with J^T r_bar (or dL/dtheta)
 *   dW_f64, db_f64  optional host arrays of device pointers receiving the same
 *            gradient reduced in FP64 (requires PINN_VERIFY_F64), or NULL.
 * The loss cotangent is scaled internally by a power of two of the order of
 * N (and the gradient by its inverse): this adds no rounding and keeps FP16
 * cotangents in range.  An explicit r_bar is used unscaled, so with FP16
 * operands its entries should not be far below 1e-3 of the residual scale. */
pinn_status pinn_jet_backward(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                              const float *x, int64_t N, const float *r_bar,
                              float *const *dW, float *const *db,
                              double *const *dW_f64, double *const *db_f64, void *stream);

/* The same for a cotangent of both outputs of pinn_jet_residual, formed on the
 * device: rbar = r_bar + (*loss_bar) 2 r / N.
 *   r_bar     n_res x N device array, or NULL (no cotangent of r)
 *   loss_bar  device pointer to one float, the cotangent of the loss, or NULL
 *             (none; with r_bar also NULL the loss gradient, *loss_bar = 1)
 * This is the backward of an autograd function returning (r, loss): no host
 * synchronisation is needed to read the loss cotangent.  With r_bar NULL the
 * loss cotangent is scaled internally as in pinn_jet_backward. */
pinn_status pinn_jet_backward_cot(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                                  const float *x, int64_t N, const float *r_bar, const float *loss_bar,
                                  float *const *dW, float *const *db,
                                  double *const *dW_f64, double *const *db_f64, void *stream);

/* Composite training loss (Sec. 3.1.1).  The paper's training runs combine
 * the PDE residual with initial-condition and boundary terms, each weighted,
 * and evaluate them in an "all-points batching" layout: the initial, boundary
 * and PDE points are concatenated, the network and its partial jet are
 * evaluated once on all of them, and the outputs are split afterwards to
 * assemble the loss terms.  A segment is one such term over a range of the
 * points:
 *   PINN_SEG_PDE        the plan's PDE residual at each point
 *   PINN_SEG_DIRICHLET  a data term u_o - g_o(x) at each point, for every
 *                       output o whose value bit (o * C) is set in mask; g_o:
 *                       PINN_DATA_ZERO 0, PINN_DATA_CONST param[o],
 *                       PINN_DATA_SIN param[0] sin(param[1] pi x_0),
 *                       PINN_DATA_VALUES values[k * d_out + o] at the
 *                       segment's k-th point (device array of count * d_out
 *                       floats: sampled initial data)
 *                       (initial conditions, no-slip walls, a moving lid)
 *   PINN_SEG_PERIODIC   consecutive point pairs (begin + 2k, begin + 2k + 1):
 *                       u_oc(first) - u_oc(second) for every output o and
 *                       channel c whose bit o * C + c is set in mask
 *                       (periodic boundary terms for u and its derivatives)
 * C is the kind's channel count; channel c of output o as in the jets array.
 * Each segment contributes weight * seg_loss, seg_loss being the mean over its
 * units (points, or pairs) of the sum of its squared terms.  Segments lie in
 * [0, N) and do not overlap; points outside every segment are evaluated but
 * do not enter the loss.  1 <= n_segments <= PINN_MAX_SEGMENTS. */
enum { PINN_SEG_PDE = 0, PINN_SEG_DIRICHLET = 1, PINN_SEG_PERIODIC = 2 };
enum { PINN_DATA_ZERO = 0, PINN_DATA_CONST = 1, PINN_DATA_SIN = 2, PINN_DATA_VALUES = 3 };
#define PINN_MAX_SEGMENTS 8
typedef struct {
  int32_t type;      /* PINN_SEG_* */
  int32_t data;      /* PINN_DATA_* (Dirichlet segments) */
  int64_t begin, count;
  double weight;     /* >= 0 */
  uint32_t mask;
  double param[4];
  const float *values; /* PINN_DATA_VALUES only (else ignored); read at every call */
} pinn_segment;

/* The composite loss: the forward pass over all N points, then each segment's
 * terms.  loss (1 float) receives sum_s weight_s seg_loss_s and seg_loss
 * (n_segments floats) the segments' own losses; either may be NULL.  Saves
 * the state pinn_jet_loss_backward needs (segments: host array).  Errors as
 * pinn_jet_residual; PINN_ERR_ARG for a malformed segment list. */
pinn_status pinn_jet_loss(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const pinn_segment *segments,
                          int32_t n_segments, const float *x, int64_t N, float *loss, float *seg_loss,
                          void *stream);
/* d loss / d theta of the composite loss, by reverse mode from every point's
 * output cotangent (a periodic pair's term reaches both of its points); the
 * same backward kernels as pinn_jet_backward.  Must follow pinn_jet_loss on the
 * same plan with the same segments, x, N and parameters (PINN_ERR_STATE). */
pinn_status pinn_jet_loss_backward(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                                   const pinn_segment *segments, int32_t n_segments, const float *x, int64_t N,
                                   float *const *dW, float *const *db, void *stream);

/* Modified MLP with a periodic input embedding: the network of the paper's
 * Kuramoto-Sivashinsky case (Sec. 3.1.1), where periodicity in x is imposed
 * by the input embedding; the paper adopts the architecture from earlier PINN
 * training work without writing it out.  The form computed:
 *   e(x) = (x_1 .. x_{d-1}, cos(w0 x_0), sin(w0 x_0), .., cos(M w0 x_0),
 *           sin(M w0 x_0)),  w0 = 2 pi / period,  de = d - 1 + 2 M
 *   U = tanh(W_U e + b_U),  V = tanh(W_V e + b_V),  h_1 = tanh(W_1 e + b_1)
 *   h_l = U + tanh(W_l h_{l-1} + b_l) (V - U)   elementwise, l = 2 .. hidden
 *   u = W_o h_hidden + b_o
 * pinn_plan_create_modified: FP32 operands only (PINN_ERR_UNSUPPORTED for
 * other precisions and for flags other than 0); kinds PINN_KS_1D and
 * PINN_BURGERS_1D (input x_0 periodic); width a multiple of 64 in [64, 256];
 * 2 <= hidden <= 16; 1 <= harmonics <= 8; period > 0.
 * Step calls on such a plan take a pinn_net with n_layers = hidden + 3 (dims
 * ignored; may be NULL) and W[l], b[l] in the order: U encoder (w x de),
 * V encoder (w x de), first layer (w x de), layers 2 .. hidden (w x w),
 * output (d_out x w).  Supported: pinn_jet_forward, pinn_jet_residual (no
 * loss_f64), pinn_jet_backward and pinn_jet_backward_cot (no FP64 outputs),
 * pinn_jet_loss, pinn_jet_loss_backward; the other plan calls return
 * PINN_ERR_UNSUPPORTED. */
typedef struct {
  int32_t hidden;
  int32_t width;
  int32_t harmonics;
  double period;
} pinn_modified;
pinn_status pinn_plan_create_modified(const pinn_modified *arch, const pinn_pde *pde, int64_t max_points,
                                      int32_t prec, uint32_t flags, pinn_plan *out);

/* Tunable launch parameters of a plan.  They change reduction order and
 * workgroup shapes, never the arithmetic: every setting is deterministic and
 * agrees with the others to rounding.
 *   dw_splits   number of split-K partials of each hidden-layer weight gradient
 *               (1 .. twice the plan's default); with the fused weight
 *               gradient, the persistent backward kernels run
 *               min(2 dw_splits, twice the default, 512, tiles) workgroups,
 *               one partial each
 *   fwd_points  points per workgroup of the whole-network forward kernel
 *               (0 = the default tiling; else 16, 32, or for 16-bit operands
 *               at widths 64-256 also 64, where each wave works on four
 *               16-point tiles and reuses every weight fragment across them)
 *   bwd_fused   1: hidden-layer weight gradients are accumulated inside the
 *               persistent backward layer kernels where the width allows
 *               (32, 64, 128); 0: separate split-K gradient kernels.  Default:
 *               1 for 16-bit operands where supported, else 0.
 *   bwd_points  the wide-layer backward kernel (widths >= 256, 16-bit
 *               operands): 0 = the default; 16 = 16 points per workgroup with
 *               the LDS chunks double-buffered (up to 8 channels); 32 or 64
 *               points per workgroup (up to 6 channels), each weight fragment
 *               then serving two or four 16-point tiles; 256 (width 256, up
 *               to 6 channels) = sixteen 16-point tiles per workgroup streamed
 *               through LDS with the weights held in registers and the next
 *               tile's loads in flight during the current tile's MFMAs. */
typedef struct {
  int32_t dw_splits;
  int32_t fwd_points;
  int32_t bwd_fused;
  int32_t bwd_points;
} pinn_tuning;
pinn_status pinn_plan_get_tuning(pinn_plan plan, pinn_tuning *tuning);
pinn_status pinn_plan_set_tuning(pinn_plan plan, const pinn_tuning *tuning);

/* Autotuner: times `reps` residual + backward steps (after one warm-up step)
 * for each candidate tuning on the caller's data, in two interleaved rounds,
 * keeps the candidate with the fastest round and returns it with its
 * milliseconds per step.  Synchronises the stream and
 * allocates temporary gradient buffers; invalidates the saved state.
 * Results are cached for the process, per (device architecture, PDE kind,
 * operand type, width, depth, point-count bucket ceil(log2 N)): a later call
 * with a cached key applies the cached choice without timing (the split count
 * is scaled to the plan's N) and returns the cached milliseconds. */
pinn_status pinn_plan_autotune(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                               int64_t N, int32_t reps, pinn_tuning *best, double *best_ms, void *stream);

/* The tuning cache of pinn_plan_autotune: drop every entry; the number of
 * entries; write it to / merge it from a text file (one entry per line:
 * arch kind prec w H nbucket split_mode fwd_points bwd_fused ms bwd_points;
 * lines without the last column load with bwd_points 0).
 * PINN_ERR_ARG on an unreadable or malformed file (nothing is merged). */
pinn_status pinn_tuning_cache_clear(void);
pinn_status pinn_tuning_cache_size(int64_t *entries);
pinn_status pinn_tuning_cache_save(const char *path);
pinn_status pinn_tuning_cache_load(const char *path);

/* Ensembles: many independent networks, each with its own width, depth, PDE
 * coefficients and point count, stepped together.  (The paper batches
 * collocation points within one network, Sec. 3.1.1; an ensemble of
 * networks is this library's extension of that batching.)
 *   pinn_batch_create   one plan per network (arguments as pinn_plan_create,
 *                       no save cap); nets[i], pdes[i], max_points[i] host arrays.
 *   pinn_batch_step     for every network i: residual, loss[i] (device array of
 *                       n floats) and the loss gradient into dW[i][l], db[i][l]
 *                       (host arrays of host arrays of device pointers).
 *                       The kernels are grouped across networks: at every
 *                       phase of the step one launch runs the same kernel
 *                       for all networks that are at that phase, each network
 *                       on its own grid of workgroups with its own argument
 *                       block (so each network's results are those of its
 *                       single-plan calls, bit for bit).  Networks of one
 *                       hidden width form a lane; lanes run on separate
 *                       streams forked from and joined into `stream`.  The
 *                       first call builds this schedule (a synchronous upload
 *                       of the argument blocks) and, with graphs on (the
 *                       default), captures it into one HIP graph; later calls
 *                       with the same pointers, sizes, coefficients and
 *                       tunings replay it.  Any change rebuilds it.
 *   pinn_batch_train_step  the same step followed by the Adam update of every
 *                       network (as pinn_adam_step; moments mW[i][l], vW[i][l],
 *                       mb[i][l], vb[i][l] per network, zero before step 1;
 *                       nets[i].W, b updated in place) and one advance of the
 *                       device step counter *step_dev (0 before the first
 *                       step), all in the same graph.
 *   pinn_batch_configure  the number of streams (1..16) and the flags:
 *                       PINN_BATCH_GRAPH captures the step into a graph;
 *                       PINN_BATCH_PER_NETWORK makes the lanes the streams
 *                       themselves, networks dealt to them longest first by
 *                       estimated work (without it: one lane per hidden
 *                       width, widths beyond the stream count sharing lanes);
 *                       PINN_BATCH_WIDTH_LANES (with PINN_BATCH_PER_NETWORK)
 *                       keeps each lane to networks of one width: every width
 *                       gets a lane, the remaining lanes go one at a time to
 *                       the width with the most estimated work per lane, and
 *                       each width's networks are dealt to its lanes longest
 *                       first (when there are fewer streams than widths, the
 *                       flag has no effect).
 *   pinn_batch_launches  grouped launches per step of the current schedule.
 *   pinn_batch_autotune  runs pinn_plan_autotune on every network (networks
 *                       sharing a cache key are timed once); then times
 *                       `reps` grouped steps with those tilings against the
 *                       same steps with every network on the tiling with the
 *                       most points per workgroup its shape allows (forward
 *                       64 points, fused weight gradient, wide backward 256
 *                       points, where supported) and keeps the faster; then
 *                       times width lanes on 1, 2 and 4 streams, per-network
 *                       lanes on 8 and 16, and per-network lanes by width on
 *                       8, 12 and 16, and keeps the fastest (best_streams
 *                       receives the stream count; pinn_batch_get_config the
 *                       flags). */
enum { PINN_BATCH_GRAPH = 1, PINN_BATCH_PER_NETWORK = 2, PINN_BATCH_WIDTH_LANES = 4 };
pinn_status pinn_batch_create(int32_t n, const pinn_net *nets, const pinn_pde *pdes, const int64_t *max_points,
                              int32_t prec, uint32_t flags, pinn_batch *out);
pinn_status pinn_batch_destroy(pinn_batch batch);
pinn_status pinn_batch_configure(pinn_batch batch, int32_t n_streams, int32_t use_graph);
/* The kernel class (PINN_K_*) of every grouped launch of the current
 * schedule, lane by lane in launch order, then the launches after the join;
 * *n_out receives the count (classes may be NULL to query it; PINN_ERR_ARG
 * when cap is below it).  With one lane this is the dispatch order of an
 * eager step, which ties per-dispatch profiler records to kernel classes. */
pinn_status pinn_batch_schedule_classes(pinn_batch batch, int32_t *classes, int64_t cap, int64_t *n_out);
/* The current stream count and PINN_BATCH_* flags (after pinn_batch_autotune). */
pinn_status pinn_batch_get_config(pinn_batch batch, int32_t *n_streams, int32_t *flags);
pinn_status pinn_batch_step(pinn_batch batch, const pinn_net *nets, const pinn_pde *pdes, const float *const *x,
                            const int64_t *N, float *loss, float *const *const *dW, float *const *const *db,
                            void *stream);
pinn_status pinn_batch_train_step(pinn_batch batch, const pinn_net *nets, const pinn_pde *pdes,
                                  const float *const *x, const int64_t *N, float *loss, float *const *const *dW,
                                  float *const *const *db, float *const *const *mW, float *const *const *vW,
                                  float *const *const *mb, float *const *const *vb, const struct pinn_adam_s *hp,
                                  int64_t *step_dev, void *stream);
pinn_status pinn_batch_launches(pinn_batch batch, int64_t *launches);
/* The tuning of network i (0 <= i < n), as pinn_plan_get_tuning; and its
 * replacement, as pinn_plan_set_tuning (the next step rebuilds the schedule). */
pinn_status pinn_batch_get_tuning(pinn_batch batch, int32_t i, pinn_tuning *tuning);
pinn_status pinn_batch_set_tuning(pinn_batch batch, int32_t i, const pinn_tuning *tuning);
/* Launch timing of one kernel class over a batch's steps, as
 * pinn_plan_profile: each grouped launch of that class is bracketed by a pair
 * of hipEvents on its lane's stream.  While a class is selected the steps run
 * without the graph (the same grouped launches, enqueued one by one). */
pinn_status pinn_batch_profile(pinn_batch batch, int32_t kernel_class);
pinn_status pinn_batch_profile_read(pinn_batch batch, double *total_ms, int64_t *launches);
pinn_status pinn_batch_autotune(pinn_batch batch, const pinn_net *nets, const pinn_pde *pdes,
                                const float *const *x, const int64_t *N, float *loss, float *const *const *dW,
                                float *const *const *db, int32_t reps, int32_t *best_streams, double *best_ms,
                                void *stream);

/* Optimizer step: Adam (Kingma & Ba, Algorithm 1), the optimizer of the
 * paper's training runs (full-batch Adam, Sec. 3.1), as one launch over every
 * parameter tensor of a network.  For each layer l and each element,
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   theta <- theta - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 * in FP32, in place on W[l], b[l] and the moment buffers.
 *   n_layers, dims   as in pinn_net (1 <= n_layers <= 16)
 *   W, b             host arrays of device pointers to the parameters
 *                    (written); dW, db the gradients (read), e.g. those of
 *                    pinn_jet_backward
 *   mW, vW, mb, vb   host arrays of device pointers to the first and second
 *                    moments, shaped like W and b, owned by the caller, zero
 *                    before step 1
 *   step             1, 2, ... (the bias corrections use it)
 *   hp               lr > 0, 0 <= beta1, beta2 < 1, eps > 0
 * Stream-ordered and asynchronous; allocates nothing, so it may be captured
 * into a graph with the step that produces the gradients.  PINN_ERR_ARG on a
 * NULL pointer, a bad shape or a bad hyperparameter (checked on the host). */
typedef struct pinn_adam_s {
  double lr, beta1, beta2, eps;
} pinn_adam;
pinn_status pinn_adam_step(int32_t n_layers, const int32_t *dims, float *const *W, float *const *b,
                           const float *const *dW, const float *const *db, float *const *mW, float *const *vW,
                           float *const *mb, float *const *vb, int64_t step, const pinn_adam *hp, void *stream);

/* One training-step graph of a plan: pinn_jet_residual (r, loss) followed by
 * pinn_jet_backward of the loss (r_bar = NULL) recorded into a HIP graph.
 * The graph is the standard route for callers that replay a fixed step:
 * one launch per step, no host work per step.
 *   pinn_graph_capture  validates like the two step calls, then records them
 *                       on a private stream (nothing executes) and instantiates
 *                       the graph.  r and loss may be NULL.  dW and db are host
 *                       arrays of device pointers as in pinn_jet_backward; the
 *                       pointer values (not the arrays) are kept.
 *   pinn_graph_launch   runs the step after the work already queued on
 *                       `stream`; work queued on `stream` afterwards waits for
 *                       it.  Each launch reads the current contents of W, b and
 *                       x and overwrites r, loss, dW and db.
 *   pinn_graph_destroy  releases the graph (not the plan).
 * The graph uses the plan's workspace and saved state: the plan must outlive
 * it, its tuning is frozen in the graph, and calls on the plan must not
 * overlap a launch on another stream.  Launch timing (pinn_plan_profile) is
 * switched off while capturing. */
typedef struct pinn_graph_s *pinn_graph;
pinn_status pinn_graph_capture(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                               int64_t N, float *r, float *loss, float *const *dW, float *const *db,
                               pinn_graph *out);
/* A training-step graph: the step above followed by the Adam update of
 * pinn_adam_step applied to the parameters net->W, net->b (updated in place by
 * every launch; the pointers in net must be writable), with the moments
 * mW, vW, mb, vb and hyperparameters hp as in pinn_adam_step.  The step count
 * lives in device memory: *step_dev (caller-owned int64, 0 before the first
 * launch) is the number of updates done; each launch uses *step_dev + 1 and
 * then advances it. */
pinn_status pinn_graph_capture_train(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                                     int64_t N, float *r, float *loss, float *const *dW, float *const *db,
                                     float *const *mW, float *const *vW, float *const *mb, float *const *vb,
                                     const pinn_adam *hp, int64_t *step_dev, pinn_graph *out);
pinn_status pinn_graph_launch(pinn_graph graph, void *stream);
pinn_status pinn_graph_destroy(pinn_graph graph);

/* Launch timing, a measurement aid for benchmarks.  pinn_plan_profile selects
 * one kernel class (0 = off) and clears the accumulator; from then on every
 * launch of that class made through this plan is bracketed by a pair of
 * hipEvents recorded on the call's stream.  pinn_plan_profile_read waits for
 * the recorded events and returns the summed kernel time (ms) and the number
 * of launches.  Do not enable it while capturing a HIP graph. */
enum {
  PINN_K_LAYER_FWD = 1,  /* hidden-layer GEMM + activation jet                  */
  PINN_K_LAYER_BWD = 2,  /* hidden-layer transposed GEMM + jet adjoint          */
  PINN_K_DW_HIDDEN = 3,  /* hidden-layer weight gradient (split-K partials)     */
  PINN_K_OUT_FWD = 4,    /* output layer + residual + loss partials             */
  PINN_K_OUT_BWD = 5,    /* residual adjoint + output layer adjoint             */
  PINN_K_SEED_FWD = 6,   /* first layer + activation jet                        */
  PINN_K_OTHER = 7,      /* casts, reductions, first/last layer gradients       */
  PINN_K_BWD_DW = 8      /* hidden-layer adjoint with its weight gradient fused */
};
pinn_status pinn_plan_profile(pinn_plan plan, int32_t kernel_class);
pinn_status pinn_plan_profile_read(pinn_plan plan, double *total_ms, int64_t *launches);

/* One residual + loss + loss-gradient step that allocates no device memory,
 * for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It computes what
 * pinn_jet_residual (r, loss) followed by pinn_jet_backward with r_bar = NULL
 * compute on a plan created for exactly N points with the default tuning, no
 * save cap and no flags, with the same kernels: the results are bit for bit
 * those of that plan.
 *   net, pde, prec, x, N   as in pinn_plan_create and pinn_jet_residual
 *   r, loss                as in pinn_jet_residual (either may be NULL)
 *   dW, db                 as in pinn_jet_backward (required)
 * Workspace: a static device array of PINN_NOALLOC_SCRATCH_BYTES (64 MiB)
 * that every GPU the library runs on holds until the process ends; its
 * device address is looked up once per device, on the first call made with
 * that device current.  The workspace grows with N and with the network
 * (about 10 KB per point for the 2-128x6-3 Navier-Stokes network, about
 * 1 KB per point for 2-32x3-1 Burgers); PINN_ERR_CAP when it exceeds the
 * array.  No part of the array has to start at zero: every workspace element
 * a call reads is written earlier in the same call.  All calls on one GPU
 * share its array, so calls that overlap on one GPU (from two host threads,
 * or on two streams with no ordering between them) race and give wrong
 * results; calls ordered on one stream are safe.  Stream-ordered and
 * asynchronous like the other step calls. */
#define PINN_NOALLOC_SCRATCH_BYTES (64u << 20)
pinn_status pinn_jet_step_noalloc(const pinn_net *net, const pinn_pde *pde, int32_t prec, const float *x,
                                  int64_t N, float *r, float *loss, float *const *dW, float *const *db,
                                  void *stream);

/* Message for the last non-OK status on this host thread ("" if none). */
const char *pinn_last_error(void);

/* Channel count for a PDE kind, and the number of residual rows (host). */
int32_t pinn_pde_channels(int32_t kind);
int32_t pinn_pde_residuals(int32_t kind);

#ifdef __cplusplus
}
#endif
#endif /* PINN_JET_H */
