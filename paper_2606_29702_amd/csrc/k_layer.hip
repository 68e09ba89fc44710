// Host-side entry points of the hidden-layer kernels: the dispatch over PDE
// kinds (each kind's kernels are instantiated in its own translation unit,
// k_layer_<kind>.hip, so that they compile in parallel) and the tiling
// predicates.
#include "k_layer_impl.hpp"

namespace pj {

hipError_t launch_layer_fwd(int kind, int prec, const void *A_in, const void *Wop, const void *Wlo, const float *b,
                            void *A_out, float *S_out, int64_t N_pad, int w, hipStream_t st) {
  switch (kind) {
    case K_BURGERS: return layer_fwd_burgers(prec, A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    case K_NS: return layer_fwd_ns(prec, A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    case K_KS: return layer_fwd_ks(prec, A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    case K_HEAT: return layer_fwd_heat(prec, A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    case K_ANISO: return layer_fwd_aniso(prec, A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    case K_BURGERS_BC: return layer_fwd_burgers_bc(prec, A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    default: return hipErrorInvalidValue;
  }
}

bool wide_bwd_points_supported(int points, int C, int w, int prec) {
  if (prec == P_FP32 || w < 256 || w % 128 != 0) return false;
  if (points == 16) return C <= 8;  // the double-buffered 16-point kernel
  if (points == 256) return w == 256 && C <= 6;  // the streaming kernel with weights in registers
  return (points == 32 || points == 64) && C <= 6;
}

bool seed_grad_fused_supported(int C, int w, int prec) {
  const int osz = prec == P_FP32 ? 4 : 2;
  return (w >= 256 && w % 128 == 0) || (bwd_lds_cfg(C, w, osz, false).P > 0 && C * w * osz % 16 == 0);
}

bool wide_top_out_grad_supported(int points, int C, int w, int prec, int dout) {
  return points == 256 && w == 256 && C <= 6 && prec != P_FP32 && dout == 1;
}

// One partial row per workgroup group of sixteen 16-point tiles.
int64_t wide_top_out_grad_parts(int64_t N_pad) { return (N_pad / 16 + 15) / 16; }

hipError_t launch_layer_bwd(int kind, int prec, const LayerBwd &L, int64_t N_pad, hipStream_t st) {
  if (L.seed_part && (L.top || L.A_prev || !L.x)) return hipErrorInvalidValue;
  BwdArgs a{L.Zb_in, L.WT, L.ubar, L.WL, L.S_in, L.A_prev, L.Wz, L.bz, L.x, L.W1, L.N, L.Zb_out, L.w,
            L.seed_part, L.out_part};
  const int zsrc = L.S_in ? Z_FROM_S : (L.A_prev ? Z_FROM_GEMM : Z_FROM_X);
  switch (kind) {
    case K_BURGERS: return layer_bwd_burgers(prec, a, L.top, zsrc, N_pad, L.points, st);
    case K_NS: return layer_bwd_ns(prec, a, L.top, zsrc, N_pad, L.points, st);
    case K_KS: return layer_bwd_ks(prec, a, L.top, zsrc, N_pad, L.points, st);
    case K_HEAT: return layer_bwd_heat(prec, a, L.top, zsrc, N_pad, L.points, st);
    case K_ANISO: return layer_bwd_aniso(prec, a, L.top, zsrc, N_pad, L.points, st);
    case K_BURGERS_BC: return layer_bwd_burgers_bc(prec, a, L.top, zsrc, N_pad, L.points, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pj
