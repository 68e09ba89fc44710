/*
 * FP64 CPU oracle for residual-specific partial-jet propagation through an MLP
 * (Cao, Lu & Zhang, "Verified residual-specific explicit derivative kernels ...",
 * Sec. 2.2, Eq. 1-3; residuals of Sec. 3.1.1 and Eq. 16).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library under paper_2606_29702_amd/.
 *
 * Conventions (all arrays row-major, all buffers owned by the caller):
 *   Network: L = n_layers affine maps, dims[0..L]; layer l (0-based) maps
 *     dims[l] -> dims[l+1].  theta packs, for l = 0..L-1, W_l (dims[l+1] x dims[l])
 *     followed by b_l (dims[l+1]).  The activation acts after layers 0..L-2;
 *     the last layer is linear.
 *   Channel set: C channels, channel 0 is the value.  Channel c > 0 is the pure
 *     derivative of order ch_ord[c] (1..4) along input direction ch_dir[c], or
 *     a mixed second derivative (ch_ord[c] = ORC_MIXED2, see below).
 *     For every (dir, k>1) channel the (dir, k-1) channel must also be present.
 *   Jets: d_out x C x N.   Residuals: n_res x N.
 *   Loss: sum over residual components of (1/N) sum_n r^2.
 *   Gradient: d(loss)/d(theta) packed like theta, or, when r_bar is given,
 *     the cotangent product J_theta^T r_bar (r_bar is n_res x N).
 */
#ifndef PINN_ORACLE_H
#define PINN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_ACT_TANH = 0,     /* the paper's activation */
  ORC_ACT_IDENTITY = 1, /* pins: the network is affine */
  ORC_ACT_SQUARE = 2,   /* pins: the network is a polynomial */
  ORC_ACT_CUBE = 3,
  ORC_ACT_SIN = 4       /* pins: derivatives cycle in closed form */
};

enum {
  ORC_PDE_NONE = 0,    /* jets only */
  ORC_PDE_BURGERS = 1, /* coef = {nu}; inputs (x, t); r = u_t + u u_x - nu u_xx */
  ORC_PDE_NS = 2,      /* coef = {Re}; inputs (x, y); outputs (u, v, p); Eq. 16 */
  ORC_PDE_KS = 3,      /* coef = {alpha, beta, gamma}; r = u_t + a u u_x + b u_xx + g u_xxxx */
  ORC_PDE_HEAT = 4,    /* coef = {kappa}; inputs (x, y, z, t);
                          r = u_t - kappa (u_xx + u_yy + u_zz) - sin(pi x) sin(pi y) sin(pi z) e^-t */
  ORC_PDE_ANISO = 5,   /* coef = {c}; inputs (x, y); r = u_xx + 2 c u_xy + u_yy: a test
                          operator with a mixed derivative (not one of the paper's problems) */
  ORC_PDE_BURGERS_BC = 6 /* inputs (x, t); r = u + sin(pi x): the Burgers initial condition
                            u(x, 0) = -sin(pi x) and boundary values u(+-1, t) = 0 at points on
                            those segments; value channel only */
};

/* Channel order code for a mixed second derivative d^2/dx_i dx_j (i < j, Eq. 3
 * with i != j): ch_ord = ORC_MIXED2 and ch_dir = 8 i + j.  Both first-order
 * channels (i, 1) and (j, 1) must be present. */
enum { ORC_MIXED2 = -2 };

/* Status: 0 ok, -1 bad argument, -2 channel set does not cover the PDE. */

/* Number of residual components of a PDE kind (0 for ORC_PDE_NONE). */
int orc_n_res(int pde_kind);

/* Full evaluation.  Any of jets, r, loss, grad may be NULL (not computed).
 * r_bar NULL means the cotangent of the loss (2 r / N).  n_threads <= 0 uses
 * the OpenMP default.  The result does not depend on the thread count: points
 * are processed in fixed chunks whose partial sums are added in chunk order. */
int orc_eval(int n_layers, const int *dims, const double *theta, int act,
             int pde_kind, const double *coef,
             int n_ch, const int *ch_dir, const int *ch_ord,
             int64_t N, const double *x,
             double *jets, double *r, double *loss,
             const double *r_bar, double *grad, int n_threads);

/* Complex-step directional derivative along delta in parameter space:
 * evaluates the forward pass at theta + i h delta in complex arithmetic and
 * returns Im(.)/h for the jets, the residuals and the loss (each may be NULL). */
int orc_eval_cs(int n_layers, const int *dims, const double *theta,
                const double *delta, double h, int act,
                int pde_kind, const double *coef,
                int n_ch, const int *ch_dir, const int *ch_ord,
                int64_t N, const double *x,
                double *djets, double *dr, double *dloss, int n_threads);

/* Composite training loss over segments of one point set (Sec. 3.1.1: the
 * initial-condition, boundary and PDE points are concatenated, the network is
 * evaluated once on all of them, and the outputs are split to assemble the
 * loss terms).  Segment s covers points [begin[s], begin[s] + count[s]) and
 * contributes weight[s] * seg_loss[s] to the loss, with seg_loss[s] the mean
 * over its units (points, or point pairs) of the sum of its squared residuals:
 *   ORC_SEG_PDE        the PDE residual of pde_kind at each point
 *   ORC_SEG_DIRICHLET  u_o - g_o(x) at each point for every output o whose
 *                      value bit (o * C) is set in mask[s]; g_o by data[s]:
 *                      ORC_DATA_ZERO 0, ORC_DATA_CONST param[s][o],
 *                      ORC_DATA_SIN param[s][0] sin(param[s][1] pi x_0)
 *   ORC_SEG_PERIODIC   point pairs (begin + 2k, begin + 2k + 1), count even:
 *                      u_oc(first) - u_oc(second) for every (o, c) whose bit
 *                      o * C + c is set in mask[s]
 * Segments must not overlap.  grad (may be NULL) receives d loss / d theta.
 * seg_loss has n_seg entries; loss and seg_loss may be NULL. */
enum { ORC_SEG_PDE = 0, ORC_SEG_DIRICHLET = 1, ORC_SEG_PERIODIC = 2 };
/* ORC_DATA_VALUES (modified-MLP evaluation only): g_o(x_n) = targets[n * d_out + o]. */
enum { ORC_DATA_ZERO = 0, ORC_DATA_CONST = 1, ORC_DATA_SIN = 2, ORC_DATA_VALUES = 3 };
int orc_eval_segments(int n_layers, const int *dims, const double *theta, int act, int pde_kind,
                      const double *coef, int n_ch, const int *ch_dir, const int *ch_ord, int64_t N,
                      const double *x, int n_seg, const int *seg_type, const int64_t *seg_begin,
                      const int64_t *seg_count, const double *seg_weight, const int *seg_mask,
                      const int *seg_data, const double *seg_param, double *seg_loss, double *loss,
                      double *grad, int n_threads);

/* Complex-step directional derivative of that loss along delta (theta space). */
int orc_eval_segments_cs(int n_layers, const int *dims, const double *theta, const double *delta, double h,
                         int act, int pde_kind, const double *coef, int n_ch, const int *ch_dir,
                         const int *ch_ord, int64_t N, const double *x, int n_seg, const int *seg_type,
                         const int64_t *seg_begin, const int64_t *seg_count, const double *seg_weight,
                         const int *seg_mask, const int *seg_data, const double *seg_param, double *dloss,
                         int n_threads);

/* Modified MLP with a periodic input embedding: the network of the paper's
 * Kuramoto-Sivashinsky case (Sec. 3.1.1), which the paper takes from earlier
 * PINN work without writing it out; the form evaluated here:
 *   embedding (periodic in x_0 with period `period`, omega = 2 pi / period,
 *   M harmonics; the other inputs pass through):
 *     e(x) = (x_1, .., x_{d-1}, cos(omega x_0), sin(omega x_0), ..,
 *             cos(M omega x_0), sin(M omega x_0)),   de = d - 1 + 2 M
 *   encoders  U = phi(W_U e + b_U),  V = phi(W_V e + b_V)
 *   layers    h_1 = phi(W_1 e + b_1);
 *             h_l = U + phi(W_l h_{l-1} + b_l) (V - U),  l = 2 .. H  (elementwise)
 *   output    u = W_o h_H + b_o
 * theta packs (W_U, b_U), (W_V, b_V), (W_1, b_1), .., (W_H, b_H), (W_o, b_o),
 * each W shaped (out, in): W_U, W_V, W_1 are w x de, W_2..W_H w x w, W_o dout x w.
 * The channel set is over the raw inputs (directions 0..d-1).  Jets: the
 * embedding's in closed form, products of jets by the Leibniz rule.
 * jets (dout x C x N) may be NULL.  With n_seg > 0 the segments define the
 * composite loss as in orc_eval_segments (plus ORC_DATA_VALUES with `targets`,
 * N x dout); with n_seg = 0, seg_loss, loss and grad must be NULL. */
int orc_mod_n_theta(int H, int w, int d, int M, double period, int dout, int64_t *n_theta);
int orc_eval_mod(int H, int w, int d, int M, double period, int dout, const double *theta, int act, int pde_kind,
                 const double *coef, int n_ch, const int *ch_dir, const int *ch_ord, int64_t N, const double *x,
                 double *jets, int n_seg, const int *seg_type, const int64_t *seg_begin, const int64_t *seg_count,
                 const double *seg_weight, const int *seg_mask, const int *seg_data, const double *seg_param,
                 const double *targets, double *seg_loss, double *loss, double *grad, int n_threads);
/* Complex-step directional derivative along delta of the jets and the loss. */
int orc_eval_mod_cs(int H, int w, int d, int M, double period, int dout, const double *theta, const double *delta,
                    double h, int act, int pde_kind, const double *coef, int n_ch, const int *ch_dir,
                    const int *ch_ord, int64_t N, const double *x, double *djets, int n_seg, const int *seg_type,
                    const int64_t *seg_begin, const int64_t *seg_count, const double *seg_weight,
                    const int *seg_mask, const int *seg_data, const double *seg_param, const double *targets,
                    double *dloss, int n_threads);

/* One Adam step (Kingma & Ba, Algorithm 1; the optimizer of the paper's
 * training runs, Sec. 3.1) on n parameters, in place:
 *   m <- b1 m + (1 - b1) g;   v <- b2 v + (1 - b2) g^2
 *   theta <- theta - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 * step counts from 1.  Status 0, or -1 for a bad argument. */
int orc_adam(int64_t n, double *theta, const double *g, double *m, double *v, int64_t step,
             double lr, double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
