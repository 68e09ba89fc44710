// Host-visible launchers of the gfx950 kernels.  All buffers are device
// pointers; every launcher enqueues on `st` and returns the launch status.
//
// Data layout in HBM (one network, N_pad = points rounded up to the point tile):
//   stack  [N_pad][C][w]  channel-major within a point, neuron index fastest;
//          the layer GEMM contracts over the neuron index, so every lane reads
//          8 consecutive elements (16 bytes in BF16/FP16) per MFMA operand.
//   S      [N_pad][C][w]  FP32 saved state of an activation layer:
//          S[n][0][j] = tanh(z_0), S[n][c][j] = z_c for the derivative channels.
//   W, WT  [w][w] operand-type copies of a hidden weight and of its transpose.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jet_math.hpp"

namespace pj {

enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP16 = 2 };
enum Kind { K_BURGERS = 1, K_NS = 2, K_KS = 3, K_HEAT = 4, K_ANISO = 5, K_BURGERS_BC = 6 };

constexpr int kPointTile = 128;  // N_pad granularity shared by all kernels

int op_size(int prec);

// W (fp32, rows x cols) -> Wop (operand type, same layout) and, if WTop is not
// null, its transpose (cols x rows).
hipError_t launch_cast(int prec, const float *W, int rows, int cols, void *Wop, void *WTop,
                       hipStream_t st);

// Casts of n hidden w x w weights in one launch (WTop and Wlo entries may be
// null).  Wlo receives the remainder W - Wop rounded to the operand type: for
// BF16 operands the forward GEMMs use the pair (Wop, Wlo), which carries
// about 16 significant bits of W instead of 8.
struct CastPack {
  const float *W[16];
  void *Wop[16];
  void *WTop[16];
  void *Wlo[16];
};
hipError_t launch_cast_all(int prec, const CastPack &pk, int n, int w, hipStream_t st);

// Layer 1: z = W1 x + b1 with the seeds d x / d x_i = e_i, then the activation
// jet.  S1 may be null (state not stored).
hipError_t launch_seed_fwd(int kind, int prec, const float *x, int64_t N, int64_t N_pad,
                           const float *W1, const float *b1, int w, void *A1, float *S1,
                           hipStream_t st);

// Hidden layer: Z = W A_in (+ b on the value channel), A_out = jet(Z); S_out
// (may be null) receives the FP32 state tanh(z_0), z_1 .. z_{C-1}.
// Wlo (may be null; required for BF16 operands) is the low part of the
// weight pair, as in CastPack.
hipError_t launch_layer_fwd(int kind, int prec, const void *A_in, const void *Wop, const void *Wlo, const float *b,
                            void *A_out, float *S_out, int64_t N_pad, int w, hipStream_t st);

// Hidden layer adjoint, producing Zbar of layer l-1 (see k_layer.hip):
//   abar = W_l^T Zbar_l (top = false) or W_L^T ubar (top = true, output layer);
//   z_{l-1} from S_in if given, else recomputed from A_prev with Wz, bz if
//   A_prev is given, else recomputed from x with W1, bz (first layer);
//   Zbar_{l-1} = jet_adjoint(abar, z_{l-1}).
struct LayerBwd {
  bool top;
  const void *Zb_in, *WT;       // !top
  const float *ubar, *WL;       // top
  const float *S_in;            // saved state, or null
  const void *A_prev, *Wz;      // recompute from the previous stack
  const float *bz;              // bias of layer l-1
  const float *x, *W1;          // recompute of the first layer
  int64_t N;
  void *Zb_out;
  int w;
  // first layer only (z from x): when non-null, the kernel writes the first
  // layer's weight-gradient partials seed_part[tile][w*DIN + w] (dW_1
  // row-major, then db_1; one partial per 16-point tile) instead of Zb_out
  float *seed_part = nullptr;
  // the wide-layer kernel (w >= 256): 0 the default, 16 the double-buffered
  // 16-point form, 32 / 64 points per workgroup, where wide_bwd_points_supported
  int points = 0;
  // top layer of a one-output network, where bwd_top_out_grad_supported
  // (fused backward) or wide_top_out_grad_supported (wide layer kernel): when
  // non-null, also the output layer's gradient partials out_part[g][w + 1]
  // (dW_L, then db_L), one per workgroup (fused) or per group of sixteen
  // 16-point tiles (wide, wide_top_out_grad_parts rows)
  float *out_part = nullptr;
};
bool wide_bwd_points_supported(int points, int C, int w, int prec);
bool wide_top_out_grad_supported(int points, int C, int w, int prec, int dout);
// Number of output-gradient partial rows the wide kernel writes.
int64_t wide_top_out_grad_parts(int64_t N_pad);
hipError_t launch_layer_bwd(int kind, int prec, const LayerBwd &L, int64_t N_pad, hipStream_t st);
// Whether launch_layer_bwd can produce seed_part for this shape.
bool seed_grad_fused_supported(int C, int w, int prec);

// Kernel-side argument block of the backward layer kernels.
enum { Z_FROM_S = 0, Z_FROM_GEMM = 1, Z_FROM_X = 2 };

struct BwdArgs {
  const void *Zb_in;   // [N_pad][C][w] operand type (!TOP)
  const void *WT;      // [w][w] transpose of W_l, operand type (!TOP)
  const float *ubar;   // [N_pad][DOUT][C] (TOP)
  const float *WL;     // [DOUT][w] (TOP)
  const float *S_in;   // [N_pad][C][w] (Z_FROM_S)
  const void *A_prev;  // [N_pad][C][w] operand type (Z_FROM_GEMM)
  const void *Wz;      // [w][w] operand type (Z_FROM_GEMM)
  const float *bz;     // [w] (Z_FROM_GEMM, Z_FROM_X)
  const float *x;      // [N][DIN] (Z_FROM_X)
  const float *W1;     // [w][DIN] (Z_FROM_X)
  int64_t N;
  void *Zb_out;        // [N_pad][C][w] operand type
  int w;
  float *seed_part;    // Z_FROM_X: first-layer gradient partials instead of Zb_out
  float *out_part;     // TOP, one output: output-layer gradient partials per 16-point tile
};


// Persistent backward layer kernel with the weight gradient of the layer it
// produces fused in (k_bwd_fused.hip).  Needs L.A_prev (the previous stack)
// even when L.S_in is given.  Writes `grid` partials part[g][w*w + w]
// (dW row-major, then db), summed by launch_reduce_parts2.
bool bwd_dw_fused_supported(int C, int w, int prec);
bool bwd_top_out_grad_supported(int C, int w, int prec, int dout);
hipError_t launch_bwd_dw(int kind, int prec, const LayerBwd &L, float *part, int64_t N_pad, int grid,
                         hipStream_t st);

// Whole-network forward pass for blocks of P points (k_fused_fwd.hip): seed
// layer, hidden layers, output layer, residual and one loss partial per block.
// Arrays are indexed by the 1-based layer number.  A[l], S[l], u_save,
// r_save, r, jets, loss_part may be null (not written).
constexpr int kMaxHidden = 16;
struct FusedFwdArgs {
  const float *x;
  int64_t N, N_pad;
  int w, H;
  int l_first, l_last;                  // hidden layers computed (1 <= l_first <= l_last <= H)
  const void *A_in;                     // stack of layer l_first - 1 (when l_first > 1)
  bool do_output;                       // output layer + residual (requires l_last == H)
  const float *W1, *b1;                 // layer 1 (fp32)
  const void *Wop[kMaxHidden + 1];      // layers 2..H, operand type
  const void *Wlo[kMaxHidden + 1];      // layers 2..H, low parts (BF16 operands only)
  const float *b[kMaxHidden + 1];       // layers 2..H
  const float *WL, *bL;                 // output layer (fp32)
  void *A[kMaxHidden + 1];              // saved stacks, layers 1..H
  float *S[kMaxHidden + 1];             // saved FP32 states, layers 1..H
  Coef k;
  float *jets, *r, *u_save, *r_save, *loss_part;
  double *loss_part64;
};
// Points per workgroup for the fused forward pass (32 or 16), or 0 when the
// block's stack does not fit in LDS (the layer-by-layer kernels are used).
int fused_fwd_points(int C, int w, int prec);
bool fused_fwd_fits(int P, int C, int w, int prec);
hipError_t launch_fwd_fused(int kind, int prec, const FusedFwdArgs &a, int P, hipStream_t st);

// Output layer, residual and per-block loss partial sums (16 points per block).
hipError_t launch_out_fwd(int kind, int prec, const void *A_H, const float *WL, const float *bL,
                          const float *x, int64_t N, int64_t N_pad, int w, Coef k, float *jets,
                          float *r, float *u_save, float *r_save, float *loss_part,
                          double *loss_part64, hipStream_t st);

// Deterministic sum of the loss partials; writes loss / N (fp32) and its FP64 twin.
hipError_t launch_loss_reduce(const float *part, const double *part64, int n_part, double inv_n,
                              float *loss, double *loss64, hipStream_t st);

// Residual adjoint at the outputs: ubar[n][o][c] = d<rbar, r>/d u_c[o] at
// point n, rbar = r_bar + lb * rbar_scale * r with lb = *loss_bar, or lb = 1
// when both r_bar and loss_bar are null (each may be null; zero on padded
// points).
hipError_t launch_out_adj(int kind, const float *u_save, const float *r_save, const float *r_bar,
                          const float *loss_bar, int64_t N, int64_t N_pad, float rbar_scale, Coef k, float *ubar,
                          hipStream_t st);

// Partial sums of the output layer's dW, db over chunks of points:
// part[chunk][d_out*w + d_out].
hipError_t launch_dw_out(int kind, int prec, const float *ubar, const void *A_H, int64_t N_pad,
                         int w, float *part, int n_chunks, hipStream_t st);

// Partial sums of the first layer's dW, db: part[chunk][w*d_in + w].
hipError_t launch_dw_seed(int kind, int prec, const void *Zb_1, const float *x, int64_t N,
                          int64_t N_pad, int w, float *part, int n_chunks, hipStream_t st);

// Split-K partials of a hidden layer's dW = sum_rows Zbar^T A (rows = points x
// channels) and of db = sum over value rows of Zbar, packed per split as
// part[split][w*w + w] (dW row-major, then db).  part_db must equal part + w*w.
int dw_tile(int w);  // dW workgroup tile edge (128, 64 or 32)
hipError_t launch_dw_hidden(int prec, int C, const void *Zb, const void *A_prev, int64_t N_pad, int w,
                            float *part, float *part_db, int splits, hipStream_t st);

// out[q] = scale * sum_s part[s * stride + q] for q < M1 + M2, summed in a
// fixed order (deterministic), scattered into two destinations: q < M1 goes
// to a[q], q >= M1 to b[q - M1] (packed dW/db partials).  FP32 results into
// a32/b32, FP64 sums of the same partials into a64/b64; each may be null.
// scale is a power of two (the inverse of the cotangent scaling), so it
// adds no rounding.  The kernel variant follows max(splits, select_splits).
hipError_t launch_reduce_parts2(const float *part, int splits, int64_t stride, int64_t M1,
                                int64_t M2, float *a32, float *b32, double *a64, double *b64,
                                hipStream_t st, float scale = 1.f, int select_splits = 0);

// Modified MLP with a periodic input embedding (k_mod.hip), FP32 operands.
constexpr int kModMaxHarmonics = 8;
constexpr int kModMaxDe = 1 + 2 * kModMaxHarmonics;  // embedding width for two inputs
struct ModArgs {
  const float *x;
  int64_t N, N_pad;
  int w, M, de;
  float omega;
  const float *WU, *bU, *WV, *bV, *W1, *b1;
  float *U, *V, *h1;
};
bool mod_kind_supported(int kind);
// U, V and h_1 from the embedding of x.
hipError_t launch_mod_enc(int kind, const ModArgs &m, hipStream_t st);
// Gated layer: h_out = U + tanh jet(W h_in + b) (V - U); S_out the state.
hipError_t launch_mod_layer(int kind, const float *h_in, const float *W, const float *b, const float *U,
                            const float *V, float *h_out, float *S_out, int64_t N_pad, int w, hipStream_t st);
// hbar = W^T zbar on every channel (WT = W^T, w x w).
hipError_t launch_mod_abar(int kind, const float *WT, const float *zbar, float *hbar, int64_t N_pad, int w,
                           hipStream_t st);
// Adjoint of a gated layer: Ubar, Vbar accumulated (set when top) and zbar;
// top: hbar = W_o^T ubar formed in the kernel.
hipError_t launch_mod_gate_bwd(int kind, bool top, const float *hbar, const float *ubar, const float *Wo,
                               const float *S, const float *U, const float *V, float *Ubar, float *Vbar,
                               float *zbar, int64_t N_pad, int w, hipStream_t st);
// Adjoint of h_1, U and V at their pre-activations: zb3 = 3 stacks (h_1, U, V),
// E = the embedding jets [N_pad][C][de].
hipError_t launch_mod_enc_bwd(int kind, const ModArgs &m, const float *h1bar, const float *Ubar, const float *Vbar,
                              float *zb3, float *E, hipStream_t st);
// Weight-gradient partials of h_1, U and V: part[layer][chunk][w*de + w].
hipError_t launch_mod_dw_enc(int kind, const float *zb3, const float *E, float *part, int64_t N_pad, int w, int de,
                             int n_chunks, hipStream_t st);

// Segments of a composite training loss over one point set (k_seg.hip).
constexpr int kMaxSegments = 8;
enum { SEG_PDE = 0, SEG_DIRICHLET = 1, SEG_PERIODIC = 2 };
enum { SEG_DATA_ZERO = 0, SEG_DATA_CONST = 1, SEG_DATA_SIN = 2, SEG_DATA_VALUES = 3 };
struct SegPack {
  int n;
  int type[kMaxSegments], data[kMaxSegments];
  int64_t begin[kMaxSegments], count[kMaxSegments];
  float weight[kMaxSegments];           // loss weights
  float cot[kMaxSegments];              // S * weight * 2 / units: the scaled cotangent factor
  unsigned mask[kMaxSegments];          // bit o * C + c: output o, channel c
  float param[kMaxSegments][4];         // data function parameters
  const float *values[kMaxSegments];    // SEG_DATA_VALUES: count x d_out targets (device)
  int blk_start[kMaxSegments + 1];      // loss-kernel workgroups of each segment (256 units each)
};
// Segment terms from the forward pass's outputs: partials per workgroup into
// part (blk_start[n] floats), then seg_loss[s] and the weighted loss (either
// may be null).
hipError_t launch_seg_loss(int kind, const SegPack &sp, const float *u_save, const float *r_save, const float *x,
                           int64_t N_pad, float *part, float *seg_loss, float *loss, hipStream_t st);
// Scaled cotangent of the loss at every point's outputs (zero outside the segments).
hipError_t launch_seg_adj(int kind, const SegPack &sp, const float *u_save, const float *r_save, const float *x,
                          int64_t N_pad, Coef k, float *ubar, hipStream_t st);

// One Adam step over up to kAdamSegs parameter tensors (k_adam.hip).
constexpr int kAdamSegs = 32;
struct AdamArgs {
  float *p[kAdamSegs];
  const float *g[kAdamSegs];
  float *m[kAdamSegs];
  float *v[kAdamSegs];
  int64_t n[kAdamSegs];
  int nseg;
  float lr, b1, b2, eps;
  int64_t step;             // 1, 2, ... when step_dev is null
  const int64_t *step_dev;  // else: steps completed so far, in device memory
};
hipError_t launch_adam(const AdamArgs &a, hipStream_t st);
hipError_t launch_step_count(int64_t *step, hipStream_t st);  // *step += 1

}  // namespace pj
