// Hidden-layer kernels instantiated for the Heat kind.
#include "k_layer_impl.hpp"

namespace pj {

hipError_t layer_fwd_heat(int prec, const void *A_in, const void *Wop, const void *Wlo, const float *b, void *A_out,
                   float *S_out, int64_t N_pad, int w, hipStream_t st) {
  return fwd_by_prec<PdeHeat>(prec, A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
}

hipError_t layer_bwd_heat(int prec, const BwdArgs &a, bool top, int zsrc, int64_t N_pad, int points, hipStream_t st) {
  return bwd_by_prec<PdeHeat>(prec, a, top, zsrc, N_pad, points, st);
}

}  // namespace pj
