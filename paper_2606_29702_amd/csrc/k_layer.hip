// Hidden-layer stacked-channel GEMM on MFMA with the activation jet (forward)
// or its adjoint (backward) fused into the epilogue.
//
// All channels of a layer share one weight matrix (Sec. 2.2: the states are
// stacked along the batch dimension and go through one GEMM).  Here the stack
// of a point block is [points][C][w]; a workgroup computes, for 32*WN points
// and 32*WJ output neurons, all C channels at once, so that every lane ends
// the contraction holding z_0 ... z_{C-1} of the same (neuron, point) pairs in
// registers and can apply the jet rules of Eq. 2-3 (and their adjoint)
// without another pass over memory.
//
// Tile: 4 waves; wave (wj, wn) owns neurons [32 wj, 32 wj + 32) x points
// [32 wn, 32 wn + 32) of the workgroup tile, i.e. 2 x 2 MFMA 16x16 output
// tiles per channel.  The contraction runs over the neuron index of the
// previous layer, 32 at a time.
#include "dev_common.hpp"
#include "kernels.hpp"

namespace pj {

template <class CH, class T, int WJ, bool BWD>
__global__ __launch_bounds__(256) void k_layer(const T *__restrict__ Bsrc, const T *__restrict__ Wop,
                                               const float *__restrict__ bias,
                                               const float *__restrict__ S_in, T *__restrict__ Out,
                                               float *__restrict__ S_out, int w) {
  using M = Mma<T>;
  constexpr int C = CH::C;
  constexpr int WN = 4 / WJ;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wj = wave % WJ, wn = wave / WJ;
  const int m0 = (blockIdx.y * WJ + wj) * 32;  // first output neuron of this wave
  const int64_t n0 = ((int64_t)blockIdx.x * WN + wn) * 32;  // first point of this wave
  const int r = lane & 15, g = lane >> 4;
  const int64_t ps = (int64_t)C * w;  // elements per point in a stack

  f32x4 acc[2][2][C];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < C; ++c) acc[a][b][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  const T *wp0 = Wop + (int64_t)(m0 + r) * w + 8 * g;
  const T *wp1 = wp0 + (int64_t)16 * w;
  const T *bp0 = Bsrc + (n0 + r) * ps + 8 * g;
  const T *bp1 = bp0 + 16 * ps;

  for (int k = 0; k < w; k += 32) {
    const typename M::frag a0 = M::load(wp0 + k);
    const typename M::frag a1 = M::load(wp1 + k);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const typename M::frag b0 = M::load(bp0 + c * w + k);
      const typename M::frag b1 = M::load(bp1 + c * w + k);
      M::mma(acc[0][0][c], a0, b0);
      M::mma(acc[0][1][c], a0, b1);
      M::mma(acc[1][0][c], a1, b0);
      M::mma(acc[1][1][c], a1, b1);
    }
  }

  // Epilogue: lane holds neurons mb..mb+3 of point n for every channel.
#pragma unroll
  for (int jt = 0; jt < 2; ++jt) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int64_t n = n0 + 16 * nt + r;
      const int mb = m0 + 16 * jt + 4 * g;
      float out[4][C];
      if constexpr (!BWD) {
        float sv[4][C];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float z[C], a[C];
#pragma unroll
          for (int c = 0; c < C; ++c) z[c] = acc[jt][nt][c][i];
          z[0] += bias[mb + i];
          float s;
          jet_forward<CH>(z, a, s);
          sv[i][0] = s;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            out[i][c] = a[c];
            if (c > 0) sv[i][c] = z[c];
          }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
          store4(Out + n * ps + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
          store4(S_out + n * ps + c * w + mb, sv[0][c], sv[1][c], sv[2][c], sv[3][c]);
        }
      } else {
        f32x4 sv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) sv[c] = *reinterpret_cast<const f32x4 *>(S_in + n * ps + c * w + mb);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float ab[C], zs[C], zb[C];
#pragma unroll
          for (int c = 0; c < C; ++c) {
            ab[c] = acc[jt][nt][c][i];
            zs[c] = sv[c][i];
          }
          jet_adjoint<CH>(ab, zs[0], zs, zb);
#pragma unroll
          for (int c = 0; c < C; ++c) out[i][c] = zb[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
          store4(Out + n * ps + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
      }
    }
  }
}

namespace {

template <class CH, class T, bool BWD>
hipError_t launch_layer_t(const void *Bsrc, const void *Wop, const float *bias, const float *S_in,
                          void *Out, float *S_out, int64_t N_pad, int w, hipStream_t st) {
  const int WJ = (w % 128 == 0) ? 4 : ((w % 64 == 0) ? 2 : 1);
  const int WN = 4 / WJ;
  dim3 grid((unsigned)(N_pad / (32 * WN)), (unsigned)(w / (32 * WJ)));
  const T *B = static_cast<const T *>(Bsrc);
  const T *Wp = static_cast<const T *>(Wop);
  T *O = static_cast<T *>(Out);
  if (WJ == 4)
    hipLaunchKernelGGL((k_layer<CH, T, 4, BWD>), grid, dim3(256), 0, st, B, Wp, bias, S_in, O, S_out, w);
  else if (WJ == 2)
    hipLaunchKernelGGL((k_layer<CH, T, 2, BWD>), grid, dim3(256), 0, st, B, Wp, bias, S_in, O, S_out, w);
  else
    hipLaunchKernelGGL((k_layer<CH, T, 1, BWD>), grid, dim3(256), 0, st, B, Wp, bias, S_in, O, S_out, w);
  return hipGetLastError();
}

template <class T, bool BWD>
hipError_t launch_layer_kind(int kind, const void *Bsrc, const void *Wop, const float *bias,
                             const float *S_in, void *Out, float *S_out, int64_t N_pad, int w,
                             hipStream_t st) {
  switch (kind) {
    case K_BURGERS: return launch_layer_t<ChBurgers, T, BWD>(Bsrc, Wop, bias, S_in, Out, S_out, N_pad, w, st);
    case K_NS: return launch_layer_t<ChNS, T, BWD>(Bsrc, Wop, bias, S_in, Out, S_out, N_pad, w, st);
    case K_KS: return launch_layer_t<ChKS, T, BWD>(Bsrc, Wop, bias, S_in, Out, S_out, N_pad, w, st);
    case K_HEAT: return launch_layer_t<ChHeat, T, BWD>(Bsrc, Wop, bias, S_in, Out, S_out, N_pad, w, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool BWD>
hipError_t launch_layer_prec(int kind, int prec, const void *Bsrc, const void *Wop, const float *bias,
                             const float *S_in, void *Out, float *S_out, int64_t N_pad, int w,
                             hipStream_t st) {
  switch (prec) {
    case P_FP32: return launch_layer_kind<float, BWD>(kind, Bsrc, Wop, bias, S_in, Out, S_out, N_pad, w, st);
    case P_BF16: return launch_layer_kind<bf16_t, BWD>(kind, Bsrc, Wop, bias, S_in, Out, S_out, N_pad, w, st);
    case P_FP16: return launch_layer_kind<f16_t, BWD>(kind, Bsrc, Wop, bias, S_in, Out, S_out, N_pad, w, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_layer_fwd(int kind, int prec, const void *A_in, const void *Wop, const float *b,
                            void *A_out, float *S_out, int64_t N_pad, int w, hipStream_t st) {
  return launch_layer_prec<false>(kind, prec, A_in, Wop, b, nullptr, A_out, S_out, N_pad, w, st);
}

hipError_t launch_layer_bwd(int kind, int prec, const void *Zb_in, const void *WTop,
                            const float *S_prev, void *Zb_out, int64_t N_pad, int w, hipStream_t st) {
  return launch_layer_prec<true>(kind, prec, Zb_in, WTop, nullptr, S_prev, Zb_out, nullptr, N_pad, w, st);
}

}  // namespace pj
