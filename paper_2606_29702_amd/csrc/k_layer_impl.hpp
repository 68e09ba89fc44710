// Hidden-layer kernels and their launch templates, included by the per-kind
// translation units (k_layer_<kind>.hip) that instantiate them and by
// k_layer.hip for the host-side configuration helpers.
#pragma once
// Hidden-layer stacked-channel GEMMs on MFMA with the activation jet (forward)
// or its adjoint (backward) fused into the epilogue.
//
// All channels of a layer share one weight matrix (Sec. 2.2: the states are
// stacked along the batch dimension and go through one GEMM).  A stack is
// stored [points][C][w]; a wave computes, for 32 output neurons and 16*NTN
// points, all C channels at once, so that every lane ends the contraction
// holding z_0 ... z_{C-1} of the same (neuron, point) pairs in registers and
// can apply the jet rules of Eq. 2-3 (and their adjoint) without another pass
// over memory.
//
// Workgroup: 4 waves, WJ of them side by side along the neurons and 4/WJ
// along the points.  Output tile per wave: 2 x NTN MFMA 16x16 tiles per
// channel; the contraction runs over the neuron index of the previous layer,
// 32 at a time, with operands read straight from global memory (L2-resident
// weights; each stack element is read by the WJ waves that share its points).
#include "dev_common.hpp"
#include "group.hpp"
#include "kernels.hpp"

namespace pj {

// Accumulates acc[jt][nt][c] += sum_k Wop[m0 + 16 jt + r][k] * B[n0 + 16 nt + r][c][k]
// over k in [0, w): the stacked-channel GEMM of one wave tile.
// With Wlo (the low parts of a BF16 weight pair) each product is the sum of
// the MFMAs with Wop and with Wlo.
template <class T, int C, int NTN, bool SPLIT = false>
__device__ __forceinline__ void stacked_gemm(f32x4 (&acc)[2][NTN][C], const T *__restrict__ Wop,
                                             const T *__restrict__ B, int m0, int64_t n0, int w, int lane,
                                             const T *__restrict__ Wlo = nullptr) {
  using M = Mma<T>;
  const int r = lane & 15, g = lane >> 4;
  const int64_t ps = (int64_t)C * w;
  const T *wp0 = Wop + (int64_t)(m0 + r) * w + 8 * g;
  const T *wp1 = wp0 + (int64_t)16 * w;
  const T *lp0 = SPLIT ? Wlo + (int64_t)(m0 + r) * w + 8 * g : nullptr;
  const T *lp1 = SPLIT ? lp0 + (int64_t)16 * w : nullptr;
  const T *bp = B + (n0 + r) * ps + 8 * g;
  for (int k = 0; k < w; k += 32) {
    const typename M::frag a0 = M::load(wp0 + k);
    const typename M::frag a1 = M::load(wp1 + k);
    typename M::frag l0, l1;
    if constexpr (SPLIT) {
      l0 = M::load(lp0 + k);
      l1 = M::load(lp1 + k);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
      for (int nt = 0; nt < NTN; ++nt) {
        const typename M::frag b = M::load(bp + nt * 16 * ps + c * w + k);
        M::mma(acc[0][nt][c], a0, b);
        M::mma(acc[1][nt][c], a1, b);
        if constexpr (SPLIT) {
          M::mma(acc[0][nt][c], l0, b);
          M::mma(acc[1][nt][c], l1, b);
        }
      }
    }
  }
}

template <int C, int NTN>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[2][NTN][C]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NTN; ++b)
#pragma unroll
      for (int c = 0; c < C; ++c) acc[a][b][c] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Forward hidden layer: Z = W A_in (+ b on the value channel), A_out = jet(Z);
// with STORE_S also the FP32 state S (tanh z_0 and the derivative channels).
template <class CH, class T, int WJ, bool STORE_S>
struct KLayerFwd {
  static constexpr int NT = 256;
  struct Args {
    const T * A_in;
    const T * Wop;
    const T * Wlo;
    const float * bias;
    T * A_out;
    float * S_out;
    int w;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const T *__restrict__ A_in = a_.A_in;
    const T *__restrict__ Wop = a_.Wop;
    const T *__restrict__ Wlo = a_.Wlo;
    const float *__restrict__ bias = a_.bias;
    T *__restrict__ A_out = a_.A_out;
    float *__restrict__ S_out = a_.S_out;
    int w = a_.w;
    constexpr int C = CH::C;
    constexpr int WN = 4 / WJ;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wj = wave % WJ, wn = wave / WJ;
    const int m0 = (vb.y * WJ + wj) * 32;
    const int64_t n0 = ((int64_t)vb.x * WN + wn) * 32;
    const int r = lane & 15, g = lane >> 4;
    const int64_t ps = (int64_t)C * w;

    f32x4 acc[2][2][C];
    zero_acc<C, 2>(acc);
    stacked_gemm<T, C, 2, __is_same(T, bf16_t)>(acc, Wop, A_in, m0, n0, w, lane, Wlo);

  #pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
  #pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int64_t n = n0 + 16 * nt + r;
        const int mb = m0 + 16 * jt + 4 * g;
        float out[4][C], sv[4][C];
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          float z[C], a[C], s;
  #pragma unroll
          for (int c = 0; c < C; ++c) z[c] = acc[jt][nt][c][i];
          z[0] += bias[mb + i];
          jet_forward<CH, sizeof(T) == 2>(z, a, s);
  #pragma unroll
          for (int c = 0; c < C; ++c) {
            out[i][c] = a[c];
            sv[i][c] = c == 0 ? s : z[c];
          }
        }
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          store4(A_out + n * ps + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
          if constexpr (STORE_S) store4(S_out + n * ps + c * w + mb, sv[0][c], sv[1][c], sv[2][c], sv[3][c]);
        }
      }
    }
  }
};

// Backward hidden layer.  Produces Zbar of layer l-1 for one tile:
//   abar  = W_l^T Zbar_l (MFMA)                      when !TOP
//         = W_L^T ubar   (output layer, d_out rows)  when TOP
//   z     = saved S                                  ZSRC == Z_FROM_S
//         = W_{l-1} A_{l-2} + b_{l-1} (MFMA recompute) ZSRC == Z_FROM_GEMM
//         = W_1 x + b_1 with the input seeds         ZSRC == Z_FROM_X
//   Zbar_{l-1} = jet_adjoint(abar, z).
template <class CH, class T, int WJ, int NTN, bool TOP, int DOUT, int ZSRC>
struct KLayerBwd {
  static constexpr int NT = 256;
  struct Args {
    BwdArgs args;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const BwdArgs &args = a_.args;
    constexpr int C = CH::C, D = CH::DIN;
    constexpr int WN = 4 / WJ;
    const int w = args.w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wj = wave % WJ, wn = wave / WJ;
    const int m0 = (vb.y * WJ + wj) * 32;
    const int64_t n0 = ((int64_t)vb.x * WN + wn) * (16 * NTN);
    const int r = lane & 15, g = lane >> 4;
    const int64_t ps = (int64_t)C * w;
    T *Zb_out = static_cast<T *>(args.Zb_out);

    f32x4 acc_a[2][NTN][C];
    zero_acc<C, NTN>(acc_a);
    if constexpr (!TOP)
      stacked_gemm<T, C, NTN>(acc_a, static_cast<const T *>(args.WT), static_cast<const T *>(args.Zb_in), m0, n0,
                              w, lane);
    f32x4 acc_z[2][NTN][C];
    if constexpr (ZSRC == Z_FROM_GEMM) {
      zero_acc<C, NTN>(acc_z);
      stacked_gemm<T, C, NTN>(acc_z, static_cast<const T *>(args.Wz), static_cast<const T *>(args.A_prev), m0, n0,
                              w, lane);
    }

  #pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
  #pragma unroll
      for (int nt = 0; nt < NTN; ++nt) {
        const int64_t n = n0 + 16 * nt + r;
        const int mb = m0 + 16 * jt + 4 * g;
        // z (pre-activation channels of layer l-1) for the 4 neurons of this lane,
        // with zz[i][0] replaced by s = tanh(z_0) and s1[i] = 1 - s^2
        constexpr bool FAST = sizeof(T) == 2;
        float zz[4][C], s1[4];
        if constexpr (ZSRC == Z_FROM_S) {
  #pragma unroll
          for (int c = 0; c < C; ++c) {
            const f32x4 v = *reinterpret_cast<const f32x4 *>(args.S_in + n * ps + c * w + mb);
  #pragma unroll
            for (int i = 0; i < 4; ++i) zz[i][c] = v[i];
          }
  #pragma unroll
          for (int i = 0; i < 4; ++i) s1[i] = (1.f - zz[i][0]) * (1.f + zz[i][0]);
        } else if constexpr (ZSRC == Z_FROM_GEMM) {
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
  #pragma unroll
            for (int c = 0; c < C; ++c) zz[i][c] = acc_z[jt][nt][c][i];
            const TanhS ts = tanh_eval<FAST>(zz[i][0] + args.bz[mb + i]);
            zz[i][0] = ts.s;
            s1[i] = ts.s1;
          }
        } else {
          float xin[D];
  #pragma unroll
          for (int q = 0; q < D; ++q) xin[q] = n < args.N ? args.x[n * D + q] : 0.f;
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int j = mb + i;
  #pragma unroll
            for (int c = 0; c < C; ++c) zz[i][c] = 0.f;
            float z0 = args.bz[j];
  #pragma unroll
            for (int q = 0; q < D; ++q) z0 += args.W1[j * D + q] * xin[q];
            const TanhS ts = tanh_eval<FAST>(z0);
            zz[i][0] = ts.s;
            s1[i] = ts.s1;
  #pragma unroll
            for (int d = 0; d < CH::NDIR; ++d) zz[i][CH::at(d, 1)] = args.W1[j * D + CH::in(d)];
          }
        }
        // abar for the same neurons
        float ab[4][C];
        if constexpr (TOP) {
          float ub[DOUT][C];
  #pragma unroll
          for (int o = 0; o < DOUT; ++o)
  #pragma unroll
            for (int c = 0; c < C; ++c) ub[o][c] = args.ubar[(n * DOUT + o) * C + c];
  #pragma unroll
          for (int i = 0; i < 4; ++i)
  #pragma unroll
            for (int c = 0; c < C; ++c) {
              float s = 0.f;
  #pragma unroll
              for (int o = 0; o < DOUT; ++o) s += args.WL[o * w + mb + i] * ub[o][c];
              ab[i][c] = s;
            }
        } else {
  #pragma unroll
          for (int i = 0; i < 4; ++i)
  #pragma unroll
            for (int c = 0; c < C; ++c) ab[i][c] = acc_a[jt][nt][c][i];
        }
        float out[4][C];
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          float zb[C];
          jet_adjoint<CH>(ab[i], zz[i][0], s1[i], zz[i], zb);
  #pragma unroll
          for (int c = 0; c < C; ++c) out[i][c] = zb[c];
        }
  #pragma unroll
        for (int c = 0; c < C; ++c)
          store4(Zb_out + n * ps + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
      }
    }
  }
};

// LDS-staged variant of k_layer_bwd for workgroups that cover every neuron
// of P points: the Zbar tile of layer l and, for the recompute, the stack tile
// of layer l-2 are copied into LDS with coalesced 16-byte loads (all issued
// before the first MFMA), then both GEMMs read their B operands from LDS.
// The tile split over waves is the one of the fused forward pass.
// Weight fragments of the first KP contraction steps (32 each) of a wave's TPW
// neuron tiles, loaded before the stack tiles are staged so that their L2
// latency is hidden behind the staging.
template <class T, int TPW, int KP>
struct WFrags {
  typename Mma<T>::frag f[TPW][KP];
};

template <class T, int TPW, int KP>
__device__ __forceinline__ void load_wfrags(WFrags<T, TPW, KP> &wf, const T *__restrict__ Wop, int jt0, int w,
                                            int lane) {
  const int r = lane & 15, g = lane >> 4;
  const T *wrow = Wop + (int64_t)(jt0 * 16 + r) * w + 8 * g;
#pragma unroll
  for (int kk = 0; kk < KP; ++kk)
#pragma unroll
    for (int t = 0; t < TPW; ++t)
      if (kk * 32 < w) wf.f[t][kk] = Mma<T>::load(wrow + (int64_t)t * 16 * w + kk * 32);
}

// acc[t][c] = rows (jt0 + t) * 16 .. + 15 of Wop (w x w) times the channel-c
// columns of the 16-point tile nt of the LDS stack.  The first KP steps use
// the preloaded fragments; further steps stream the weights from global
// memory one step ahead.
template <class T, int C, int TPW, int KP>
__device__ __forceinline__ void lds_gemm(f32x4 (&acc)[TPW][C], const WFrags<T, TPW, KP> &wf,
                                         const T *__restrict__ Wop, const T *stk, int pitch, int jt0, int nt, int w,
                                         int lane) {
  using M = Mma<T>;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const T *brow = stk + (nt * 16 + r) * pitch + 8 * g;
#pragma unroll
  for (int kk = 0; kk < KP; ++kk) {
    if (kk * 32 < w) {
      typename M::frag fb[C];
#pragma unroll
      for (int c = 0; c < C; ++c) fb[c] = M::load(brow + c * w + kk * 32);
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int c = 0; c < C; ++c) M::mma(acc[t][c], wf.f[t][kk], fb[c]);
    }
  }
  if (KP * 32 < w) {
    const T *wrow = Wop + (int64_t)(jt0 * 16 + r) * w + 8 * g;
    typename M::frag fa[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) fa[t] = M::load(wrow + (int64_t)t * 16 * w + KP * 32);
    for (int k = KP * 32; k < w; k += 32) {
      typename M::frag fb[C];
#pragma unroll
      for (int c = 0; c < C; ++c) fb[c] = M::load(brow + c * w + k);
      typename M::frag fn[TPW];
      const int kn = k + 32 < w ? k + 32 : k;
#pragma unroll
      for (int t = 0; t < TPW; ++t) fn[t] = M::load(wrow + (int64_t)t * 16 * w + kn);
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int c = 0; c < C; ++c) M::mma(acc[t][c], fa[t], fb[c]);
#pragma unroll
      for (int t = 0; t < TPW; ++t) fa[t] = fn[t];
    }
  }
}

// Epilogue of the backward layer kernels, per wave: the lane's point n and
// this wave's TPW neuron tiles starting at tile jt0.  z of the layer comes
// from the saved state, the recompute accumulators acc_z (plus the bias) or
// x; Abar from acc_a or, at the top, W_L^T ubar; then the jet adjoint.  Writes
// Zbar to Zb_out, or (first layer with seed_part) adds the first layer's
// gradient into the partial row `part_row`.
template <class CH, class T, int TPW, bool TOP, int DOUT, int ZSRC>
__device__ __forceinline__ void bwd_epilogue(const BwdArgs &args, const f32x4 (&acc_a)[TPW][CH::C],
                                             const f32x4 (&acc_z)[TPW][CH::C], int64_t n, int jt0,
                                             int64_t part_row, int lane, float *out_acc = nullptr) {
  constexpr int C = CH::C, D = CH::DIN;
  constexpr bool FAST = sizeof(T) == 2;
  const int w = args.w;
  const int r = lane & 15, g = lane >> 4;
  const int64_t ps = (int64_t)C * w;
  T *Zb_out = static_cast<T *>(args.Zb_out);
  // the point's inputs: for the first layer's z, or for its gradient
  float xin[D];
  if (ZSRC == Z_FROM_X || (ZSRC == Z_FROM_S && !TOP && args.seed_part)) {
#pragma unroll
    for (int q = 0; q < D; ++q) xin[q] = n < args.N ? args.x[n * D + q] : 0.f;
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int mb = (jt0 + t) * 16 + 4 * g;
    float zz[4][C], s1[4];
    if constexpr (ZSRC == Z_FROM_S) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const f32x4 v = *reinterpret_cast<const f32x4 *>(args.S_in + n * ps + c * w + mb);
#pragma unroll
        for (int i = 0; i < 4; ++i) zz[i][c] = v[i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) s1[i] = (1.f - zz[i][0]) * (1.f + zz[i][0]);
    } else if constexpr (ZSRC == Z_FROM_GEMM) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int c = 0; c < C; ++c) zz[i][c] = acc_z[t][c][i];
        const TanhS ts = tanh_eval<FAST>(zz[i][0] + args.bz[mb + i]);
        zz[i][0] = ts.s;
        s1[i] = ts.s1;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = mb + i;
#pragma unroll
        for (int c = 0; c < C; ++c) zz[i][c] = 0.f;
        float z0 = args.bz[j];
#pragma unroll
        for (int q = 0; q < D; ++q) z0 += args.W1[j * D + q] * xin[q];
        const TanhS ts = tanh_eval<FAST>(z0);
        zz[i][0] = ts.s;
        s1[i] = ts.s1;
#pragma unroll
        for (int d = 0; d < CH::NDIR; ++d) zz[i][CH::at(d, 1)] = args.W1[j * D + CH::in(d)];
      }
    }
    float ab[4][C];
    [[maybe_unused]] float ub[TOP ? DOUT : 1][C];
    if constexpr (TOP) {
#pragma unroll
      for (int o = 0; o < DOUT; ++o)
#pragma unroll
        for (int c = 0; c < C; ++c) ub[o][c] = args.ubar[(n * DOUT + o) * C + c];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          float sacc = 0.f;
#pragma unroll
          for (int o = 0; o < DOUT; ++o) sacc += args.WL[o * w + mb + i] * ub[o][c];
          ab[i][c] = sacc;
        }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < C; ++c) ab[i][c] = acc_a[t][c][i];
    }
    float out[4][C];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float zb[C];
      jet_adjoint<CH>(ab[i], zz[i][0], s1[i], zz[i], zb);
#pragma unroll
      for (int c = 0; c < C; ++c) out[i][c] = zb[c];
    }
    if constexpr (TOP && DOUT == 1 && ZSRC == Z_FROM_GEMM) {
      if (args.out_part) {
        // the output layer's gradient (one output): dW_L[j] = sum over the
        // points of sum_c ubar[n][c] a_H[n][c][j], the activation jet
        // recomputed from z_H.  With out_acc, this lane's terms are added to
        // the caller's accumulators (out_acc[t * 4 + i], db_L in
        // out_acc[TPW * 4]); otherwise the 16 points of the tile (the lanes r
        // of each lane group) are summed by a butterfly into the partial row
        // `part_row`, db_L with neuron tile 0.
        float *op = args.out_part + part_row * ((int64_t)w + 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float act[C];
          jet_forward_from<CH>(zz[i][0], s1[i], zz[i], act);
          float v = 0.f;
#pragma unroll
          for (int c = 0; c < C; ++c) v += ub[0][c] * act[c];
          if (out_acc) {
            out_acc[t * 4 + i] += v;
          } else {
            v = group_sum<16>(v);
            if (r == 0) op[mb + i] = v;
          }
        }
        if (out_acc) {
          if (t == 0) out_acc[TPW * 4] += ub[0][0];
        } else {
          const float v0 = group_sum<16>(ub[0][0]);
          if (jt0 + t == 0 && lane == 0) op[w] = v0;
        }
      }
    }
    if constexpr (ZSRC != Z_FROM_GEMM && !TOP) {
      if (args.seed_part) {
        // first-layer gradient of this tile instead of Zbar_1 (the seeds of
        // the input layer, reversed): dW_1[j][q] = sum over points of
        // zbar_0 x_q plus the first-order channel of direction q; db_1[j] =
        // sum of zbar_0.  The 16 points of the tile are the 16 lanes r of
        // each lane group, summed by a butterfly.
        float *sp = args.seed_part + part_row * ((int64_t)w * D + w);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v[D + 1];
#pragma unroll
          for (int q = 0; q < D; ++q) v[q] = out[i][0] * xin[q];
#pragma unroll
          for (int d = 0; d < CH::NDIR; ++d) v[CH::in(d)] += out[i][CH::at(d, 1)];
          v[D] = out[i][0];
#pragma unroll
          for (int e = 0; e <= D; ++e) v[e] = group_sum<16>(v[e]);
          if (r == 0) {
#pragma unroll
            for (int q = 0; q < D; ++q) sp[(mb + i) * D + q] = v[q];
            sp[(int64_t)w * D + mb + i] = v[D];
          }
        }
        continue;
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) store4(Zb_out + n * ps + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
  }
}

template <class CH, class T, int NW, int TPW, int P, bool TOP, int DOUT, int ZSRC>
struct KLayerBwdLds {
  static constexpr int NT = NW * 64;
  struct Args {
    BwdArgs args;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const BwdArgs &args = a_.args;
    constexpr int C = CH::C, D = CH::DIN;
    constexpr bool FAST = sizeof(T) == 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int w = args.w;
    const int pitch = C * w + 8;
    T *lds_b = reinterpret_cast<T *>(smem_raw);                         // Zbar_l tile
    T *lds_a = lds_b + (TOP ? 0 : P * pitch);                           // stack tile of layer l-2
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int64_t nb = (int64_t)vb.x * P;
    const int64_t ps = (int64_t)C * w;
    const int NJ = w / 16;
    const int tile0 = wave * TPW;
    const int nt = tile0 / NJ, jt0 = tile0 % NJ;
    // weight fragments of the first contraction steps, loaded first (16
    // registers per GEMM)
    constexpr int KP = (sizeof(T) == 2 ? 4 : 2) / TPW > 0 ? (sizeof(T) == 2 ? 4 : 2) / TPW : 1;
    WFrags<T, TPW, KP> wf_a, wf_z;
    if constexpr (!TOP) load_wfrags(wf_a, static_cast<const T *>(args.WT), jt0, w, lane);
    if constexpr (ZSRC == Z_FROM_GEMM) load_wfrags(wf_z, static_cast<const T *>(args.Wz), jt0, w, lane);
    // both tiles in one pass (Zbar_l first, then the stack of layer l-2), so that
    // a thread's loads of the two are in flight together
    {
      const T *zb_in = static_cast<const T *>(args.Zb_in) + nb * ps;
      const T *a_prev = static_cast<const T *>(args.A_prev) + nb * ps;
      if constexpr (!TOP && ZSRC == Z_FROM_GEMM)
        stage_rows<T, 12, true>(lds_b, zb_in, a_prev, P, C * w, pitch, tid, NW * 64);
      else if constexpr (!TOP)
        stage_rows<T, 12, false>(lds_b, zb_in, nullptr, P, C * w, pitch, tid, NW * 64);
      else if constexpr (ZSRC == Z_FROM_GEMM)
        stage_rows<T, 12, false>(lds_a, a_prev, nullptr, P, C * w, pitch, tid, NW * 64);
    }
    __syncthreads();

    f32x4 acc_a[TPW][C];
    if constexpr (!TOP)
      lds_gemm<T, C, TPW, KP>(acc_a, wf_a, static_cast<const T *>(args.WT), lds_b, pitch, jt0, nt, w, lane);
    f32x4 acc_z[TPW][C];
    if constexpr (ZSRC == Z_FROM_GEMM)
      lds_gemm<T, C, TPW, KP>(acc_z, wf_z, static_cast<const T *>(args.Wz), lds_a, pitch, jt0, nt, w, lane);

    bwd_epilogue<CH, T, TPW, TOP, DOUT, ZSRC>(args, acc_a, acc_z, nb + nt * 16 + r, jt0, vb.x, lane);
  }
};

// Backward layer kernel for wide layers (w >= 256), where a whole stack tile
// does not fit in LDS.  A workgroup of NW waves (TPW neuron tiles each)
// computes a P-point x 16 NW TPW-neuron output tile, P = 16 PTW: every wave
// takes all PTW point tiles, so each weight fragment it loads feeds PTW x C
// MFMAs.  The neuron tile is the fastest-varying part of the logical block
// index (xcd_order), so the workgroups that share a point tile run on one XCD
// and read its stack data into that XCD's L2 once.  The contraction (the
// neurons of the layer below) runs in chunks of KC: each chunk of the Zbar and A_{l-2}
// tiles ([point][channel][KC], rows padded by 8 elements) is staged through
// LDS with every thread's loads issued together, then feeds the Abar and z
// GEMMs.  The epilogue is that of the full-tile kernel.
template <class CH, class T, int NW, int TPW, int KC, bool TOP, int DOUT, int ZSRC, int PTW = 1>
struct KLayerBwdKc {
  static constexpr int NT = NW * 64;
  struct Args {
    BwdArgs args;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const BwdArgs &args = a_.args;
    using M = Mma<T>;
    constexpr int C = CH::C, P = 16 * PTW;
    constexpr int TILEN = NW * TPW * 16;
    constexpr int PITCH = C * KC + 8;
    constexpr bool ZB = !TOP, AZ = ZSRC == Z_FROM_GEMM;
    constexpr int P16 = 16 / (int)sizeof(T);       // elements per 16-byte piece
    constexpr int PPC = KC / P16;                  // pieces per (point, channel) row of a chunk
    constexpr int PIECES = P * C * PPC;            // pieces per tile chunk
    constexpr int PER_T = (PIECES + NW * 64 - 1) / (NW * 64);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds_b = reinterpret_cast<T *>(smem_raw);
    T *lds_a = lds_b + (ZB ? P * PITCH : 0);
    const int w = args.w;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ntn = w / TILEN;  // neuron tiles per point tile (consecutive workgroups)
    const int lb = xcd_order(vb);  // the neuron tiles of a point tile share an XCD's L2
    const int64_t ptile = lb / ntn;
    const int ntile = (int)(lb - ptile * ntn);
    const int64_t nb = ptile * P;
    const int jt0 = ntile * (TILEN / 16) + wave * TPW;
    const int64_t ps = (int64_t)C * w;
    const T *zb_src = static_cast<const T *>(args.Zb_in) + nb * ps;
    const T *a_src = static_cast<const T *>(args.A_prev) + nb * ps;
    const T *WT = static_cast<const T *>(args.WT);
    const T *Wz = static_cast<const T *>(args.Wz);
    f32x4 acc_a[PTW][TPW][C], acc_z[PTW][TPW][C];
  #pragma unroll
    for (int q = 0; q < PTW; ++q)
  #pragma unroll
      for (int t = 0; t < TPW; ++t)
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          acc_a[q][t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
          acc_z[q][t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    for (int k0 = 0; k0 < w; k0 += KC) {
      {
        uint4 vb[PER_T], va[PER_T];
  #pragma unroll
        for (int u = 0; u < PER_T; ++u) {
          const int q0 = tid + u * NW * 64;
          const int q = q0 < PIECES ? q0 : PIECES - 1;  // re-read the last piece (in bounds)
          const int p = q / (C * PPC), rem = q - p * (C * PPC), c = rem / PPC, j = rem - c * PPC;
          const int64_t goff = (int64_t)p * ps + (int64_t)c * w + k0 + j * P16;
          if (ZB) vb[u] = *reinterpret_cast<const uint4 *>(zb_src + goff);
          if (AZ) va[u] = *reinterpret_cast<const uint4 *>(a_src + goff);
        }
  #pragma unroll
        for (int u = 0; u < PER_T; ++u) {
          const int q = tid + u * NW * 64;
          if (q < PIECES) {
            const int p = q / (C * PPC), rem = q - p * (C * PPC), c = rem / PPC, j = rem - c * PPC;
            const int loff = p * PITCH + c * KC + j * P16;
            if (ZB) *reinterpret_cast<uint4 *>(lds_b + loff) = vb[u];
            if (AZ) *reinterpret_cast<uint4 *>(lds_a + loff) = va[u];
          }
        }
      }
      __syncthreads();
  #pragma unroll
      for (int kk = 0; kk < KC; kk += 32) {
        if constexpr (ZB) {
          typename M::frag fa[TPW];
  #pragma unroll
          for (int t = 0; t < TPW; ++t) fa[t] = M::load(WT + (int64_t)((jt0 + t) * 16 + r) * w + k0 + kk + 8 * g);
  #pragma unroll
          for (int q = 0; q < PTW; ++q) {
            typename M::frag fb[C];
  #pragma unroll
            for (int c = 0; c < C; ++c) fb[c] = M::load(lds_b + (q * 16 + r) * PITCH + c * KC + kk + 8 * g);
  #pragma unroll
            for (int t = 0; t < TPW; ++t)
  #pragma unroll
              for (int c = 0; c < C; ++c) M::mma(acc_a[q][t][c], fa[t], fb[c]);
          }
        }
        if constexpr (AZ) {
          typename M::frag fa[TPW];
  #pragma unroll
          for (int t = 0; t < TPW; ++t) fa[t] = M::load(Wz + (int64_t)((jt0 + t) * 16 + r) * w + k0 + kk + 8 * g);
  #pragma unroll
          for (int q = 0; q < PTW; ++q) {
            typename M::frag fb[C];
  #pragma unroll
            for (int c = 0; c < C; ++c) fb[c] = M::load(lds_a + (q * 16 + r) * PITCH + c * KC + kk + 8 * g);
  #pragma unroll
            for (int t = 0; t < TPW; ++t)
  #pragma unroll
              for (int c = 0; c < C; ++c) M::mma(acc_z[q][t][c], fa[t], fb[c]);
          }
        }
      }
      __syncthreads();  // the chunk buffers are restaged next
    }
  #pragma unroll
    for (int q = 0; q < PTW; ++q)
      bwd_epilogue<CH, T, TPW, TOP, DOUT, ZSRC>(args, acc_a[q], acc_z[q], nb + q * 16 + r, jt0, ptile * PTW + q, lane);
  }
};

// Staging of one point tile of the streaming wide kernel ([P][C][W] rows of
// Zbar and A_{l-2}): global loads into registers, then stores into the LDS
// tiles (rows padded by 8 elements).
template <class T, int C, int NT, int W, int P, int PER_T, bool ZB, bool AZ>
__device__ __forceinline__ void ks_load_unit(u32x4 (&rz)[PER_T], u32x4 (&ra)[PER_T], const T *zb_all, const T *a_all,
                                             int64_t nb, int64_t ps, int tid) {
  constexpr int P16 = 16 / (int)sizeof(T), PPR = C * W / P16, PIECES = P * PPR;
#pragma unroll
  for (int i = 0; i < PER_T; ++i) {
    const int q0 = tid + i * NT;
    const int q = q0 < PIECES ? q0 : PIECES - 1;  // re-read the last piece (in bounds)
    const int p = q / PPR, j = q - p * PPR;
    const int64_t goff = (nb + p) * ps + j * P16;
    if constexpr (ZB) rz[i] = *reinterpret_cast<const u32x4 *>(zb_all + goff);
    if constexpr (AZ) ra[i] = *reinterpret_cast<const u32x4 *>(a_all + goff);
  }
}

template <class T, int C, int NT, int W, int P, int PER_T, bool ZB, bool AZ>
__device__ __forceinline__ void ks_store_unit(const u32x4 (&rz)[PER_T], const u32x4 (&ra)[PER_T], T *lds_b, T *lds_a,
                                              int tid) {
  constexpr int P16 = 16 / (int)sizeof(T), PPR = C * W / P16, PIECES = P * PPR, PITCH = C * W + 8;
#pragma unroll
  for (int i = 0; i < PER_T; ++i) {
    const int q = tid + i * NT;
    if (q < PIECES) {
      const int p = q / PPR, j = q - p * PPR;
      const int loff = p * PITCH + j * P16;
      if constexpr (ZB) *reinterpret_cast<u32x4 *>(lds_b + loff) = rz[i];
      if constexpr (AZ) *reinterpret_cast<u32x4 *>(lds_a + loff) = ra[i];
    }
  }
}

// The backward layer at width W = 256 for 16-bit operands, streaming: a
// workgroup keeps its waves' weight fragments (16 rows of W^T and, for the z
// recompute, of W_z, over the whole contraction) in registers and works
// through PPW point tiles of P = 16 PTW points in turn.  Each point tile is
// staged whole (all W neurons of every channel) through one LDS buffer; the
// global loads of the next tile are issued before the current tile is
// multiplied, so that HBM traffic stays in flight during the MFMAs and the
// epilogue.  Logical block order as in KLayerBwdKc (the neuron tiles of a
// group of point tiles share an XCD).  The contraction runs in the same order
// as in KLayerBwdKc, so both give the same bits.
template <class CH, class T, int NW, int W, bool TOP, int DOUT, int ZSRC, int PTW, int PPW>
struct KLayerBwdKs {
  static constexpr int NT = NW * 64;
  struct Args {
    BwdArgs args;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const BwdArgs &args = a_.args;
    using M = Mma<T>;
    constexpr int C = CH::C, P = 16 * PTW, TPW = 1;
    constexpr int TILEN = NW * TPW * 16;
    constexpr int KS = W / 32;  // contraction steps
    constexpr int PITCH = C * W + 8;
    constexpr bool ZB = !TOP, AZ = ZSRC == Z_FROM_GEMM;
    constexpr int PER_T = (P * C * W * (int)sizeof(T) / 16 + NT - 1) / NT;  // 16-byte pieces per thread
    static_assert(sizeof(T) == 2 && W % 32 == 0, "shape");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds_b = reinterpret_cast<T *>(smem_raw);
    T *lds_a = lds_b + (ZB ? P * PITCH : 0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    constexpr int ntn = W / TILEN;
    const int lb = xcd_order(vb);
    const int64_t group = lb / ntn;
    const int ntile = (int)(lb - group * ntn);
    const int jt0 = ntile * (TILEN / 16) + wave * TPW;
    const int64_t n_ptiles = (args.N + kPointTile - 1) / kPointTile * (kPointTile / P);
    const int64_t pt0 = group * PPW;
    const int n_tiles = (int)(n_ptiles - pt0 < PPW ? n_ptiles - pt0 : PPW);
    if (n_tiles <= 0) return;  // uniform over the workgroup
    const int64_t ps = (int64_t)C * W;
    const T *WT = static_cast<const T *>(args.WT);
    const T *Wz = static_cast<const T *>(args.Wz);
    const T *zb_all = static_cast<const T *>(args.Zb_in);
    const T *a_all = static_cast<const T *>(args.A_prev);
    // the waves' weight rows over the whole contraction
    typename M::frag wa[ZB ? KS : 1], wz[AZ ? KS : 1];
  #pragma unroll
    for (int s = 0; s < KS; ++s) {
      if constexpr (ZB) wa[s] = M::load(WT + (int64_t)(jt0 * 16 + r) * W + s * 32 + 8 * g);
      if constexpr (AZ) wz[s] = M::load(Wz + (int64_t)(jt0 * 16 + r) * W + s * 32 + 8 * g);
    }
    u32x4 rz[PER_T], ra[PER_T];  // the next tile's pieces (a plain vector type keeps them in registers)
    ks_load_unit<T, C, NT, W, P, PER_T, ZB, AZ>(rz, ra, zb_all, a_all, pt0 * P, ps, tid);
    f32x4 acc_a[PTW][TPW][C], acc_z[PTW][TPW][C];
    // top layer, one output: the output layer's gradient over the
    // workgroup's tiles (this lane's neurons and point; db_L last)
    constexpr bool OUTG = TOP && DOUT == 1 && AZ;
    [[maybe_unused]] float oacc[OUTG ? TPW * 4 + 1 : 1];
    if constexpr (OUTG) {
  #pragma unroll
      for (int k = 0; k < TPW * 4 + 1; ++k) oacc[k] = 0.f;
    }
    for (int t = 0; t < n_tiles; ++t) {
      if (t > 0) __syncthreads();  // every wave is done with the previous tile's LDS data
      ks_store_unit<T, C, NT, W, P, PER_T, ZB, AZ>(rz, ra, lds_b, lds_a, tid);
      __syncthreads();
      if (t + 1 < n_tiles)  // in flight during this tile's MFMAs and epilogue
        ks_load_unit<T, C, NT, W, P, PER_T, ZB, AZ>(rz, ra, zb_all, a_all, (pt0 + t + 1) * P, ps, tid);
  #pragma unroll
      for (int q = 0; q < PTW; ++q)
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          acc_a[q][0][c] = f32x4{0.f, 0.f, 0.f, 0.f};
          acc_z[q][0][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
  #pragma unroll
      for (int s = 0; s < KS; ++s) {
        if constexpr (ZB) {
  #pragma unroll
          for (int q = 0; q < PTW; ++q) {
            typename M::frag fb[C];
  #pragma unroll
            for (int c = 0; c < C; ++c) fb[c] = M::load(lds_b + (q * 16 + r) * PITCH + c * W + s * 32 + 8 * g);
  #pragma unroll
            for (int c = 0; c < C; ++c) M::mma(acc_a[q][0][c], wa[s], fb[c]);
          }
        }
        if constexpr (AZ) {
  #pragma unroll
          for (int q = 0; q < PTW; ++q) {
            typename M::frag fb[C];
  #pragma unroll
            for (int c = 0; c < C; ++c) fb[c] = M::load(lds_a + (q * 16 + r) * PITCH + c * W + s * 32 + 8 * g);
  #pragma unroll
            for (int c = 0; c < C; ++c) M::mma(acc_z[q][0][c], wz[s], fb[c]);
          }
        }
      }
      const int64_t nb = (pt0 + t) * P;
  #pragma unroll
      for (int q = 0; q < PTW; ++q)
        bwd_epilogue<CH, T, TPW, TOP, DOUT, ZSRC>(args, acc_a[q], acc_z[q], nb + q * 16 + r, jt0,
                                                  (pt0 + t) * PTW + q, lane,
                                                  OUTG ? oacc : nullptr);
    }
    if constexpr (OUTG) {
      if (args.out_part) {  // one partial row per group of tiles, sums in a fixed order
        float *op = args.out_part + group * ((int64_t)W + 1);
  #pragma unroll
        for (int t = 0; t < TPW; ++t)
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float v = group_sum<16>(oacc[t * 4 + i]);
            if (r == 0) op[(jt0 + t) * 16 + 4 * g + i] = v;
          }
        const float v0 = group_sum<16>(oacc[TPW * 4]);
        if (jt0 == 0 && lane == 0) op[W] = v0;
      }
    }
  }
};

// The wide-layer kernel for 16-bit operands with its chunks double-buffered:
// two sets of chunk buffers are separate static LDS objects, and while one
// chunk feeds the GEMMs the next one streams into the other set with
// direct-to-LDS loads (one 1 KB-or-less wave load per point and tile: the C
// channel rows of KC elements of a point are contiguous in LDS).  A chunk's
// weight fragments are loaded before the next chunk's prefetch is issued,
// since the load counter completes in order.
template <class CH, class T, int NW, int KC, bool TOP, int DOUT, int ZSRC>
struct KLayerBwdKc2 {
  static constexpr int NT = NW * 64;
  struct Args {
    BwdArgs args;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const BwdArgs &args = a_.args;
    using M = Mma<T>;
    constexpr int C = CH::C, P = 16, TPW = 1;
    constexpr int TILEN = NW * TPW * 16;
    constexpr int PITCH = C * KC + 8;
    constexpr bool ZB = !TOP, AZ = ZSRC == Z_FROM_GEMM;
    constexpr int TILES = (ZB ? 1 : 0) + (AZ ? 1 : 0);
    constexpr int LPP = C * KC / 8;  // lanes (16-byte pieces) per point row of a chunk
    static_assert(sizeof(T) == 2 && LPP <= 64 && KC % 32 == 0, "chunk shape");
    // one LDS object per buffer and tile
    __shared__ __align__(16) T zbA[ZB ? P * PITCH : 8], azA[AZ ? P * PITCH : 8];
    __shared__ __align__(16) T zbB[ZB ? P * PITCH : 8], azB[AZ ? P * PITCH : 8];
    const int w = args.w;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ntn = w / TILEN;
    const int lb = xcd_order(vb);  // the neuron tiles of a point tile share an XCD's L2
    const int64_t ptile = lb / ntn;
    const int ntile = (int)(lb - ptile * ntn);
    const int64_t nb = ptile * P;
    const int jt0 = ntile * (TILEN / 16) + wave * TPW;
    const int64_t ps = (int64_t)C * w;
    const T *zb_src = static_cast<const T *>(args.Zb_in) + nb * ps;
    const T *a_src = static_cast<const T *>(args.A_prev) + nb * ps;
    const T *WT = static_cast<const T *>(args.WT);
    const T *Wz = static_cast<const T *>(args.Wz);
    // chunk k0 of both tiles into (zs, as): wave v loads the points v, v + NW, ...
    auto prefetch = [&](T *zs, T *as, int k0) __attribute__((always_inline)) {
      const int c = lane / (KC / 8), j = lane - c * (KC / 8);
      for (int p = wave; p < P; p += NW) {
        if (lane < LPP) {
          const int64_t goff = (int64_t)p * ps + (int64_t)c * w + k0 + 8 * j;
          if constexpr (ZB)
            __builtin_amdgcn_global_load_lds((const void *)(zb_src + goff),
                                             (__attribute__((address_space(3))) void *)(zs + p * PITCH), 16, 0, 0);
          if constexpr (AZ)
            __builtin_amdgcn_global_load_lds(
                (const void *)(a_src + goff),
                (__attribute__((address_space(3))) void *)(as + p * PITCH), 16, 0, 0);
        }
      }
    };
    f32x4 acc_a[TPW][C], acc_z[TPW][C];
  #pragma unroll
    for (int c = 0; c < C; ++c) {
      acc_a[0][c] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc_z[0][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const T *wra = WT + (int64_t)(jt0 * 16 + r) * w + 8 * g;
    const T *wrz = Wz + (int64_t)(jt0 * 16 + r) * w + 8 * g;
    // one chunk from (cz, ca) while the next one streams into (nz, na)
    auto chunk = [&](int k0, const T *cz, const T *ca, T *nz, T *na) __attribute__((always_inline)) {
      typename M::frag fa[KC / 32], fz[KC / 32];
  #pragma unroll
      for (int kk = 0; kk < KC / 32; ++kk) {
        if constexpr (ZB) fa[kk] = M::load(wra + k0 + 32 * kk);
        if constexpr (AZ) fz[kk] = M::load(wrz + k0 + 32 * kk);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_sched_barrier(0);  // the fragment loads stay ahead of the prefetch
      if (k0 + KC < w) prefetch(nz, na, k0 + KC);
      __builtin_amdgcn_sched_barrier(0);
  #pragma unroll
      for (int kk = 0; kk < KC / 32; ++kk) {
        if constexpr (ZB) {
          typename M::frag fb[C];
  #pragma unroll
          for (int c = 0; c < C; ++c) fb[c] = M::load(cz + r * PITCH + c * KC + 32 * kk + 8 * g);
  #pragma unroll
          for (int c = 0; c < C; ++c) M::mma(acc_a[0][c], fa[kk], fb[c]);
        }
        if constexpr (AZ) {
          typename M::frag fb[C];
  #pragma unroll
          for (int c = 0; c < C; ++c) fb[c] = M::load(ca + r * PITCH + c * KC + 32 * kk + 8 * g);
  #pragma unroll
          for (int c = 0; c < C; ++c) M::mma(acc_z[0][c], fz[kk], fb[c]);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // the next chunk has landed
      __syncthreads();                // and this one is consumed
    };
    prefetch(zbA, azA, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int k0 = 0; k0 < w;) {
      chunk(k0, zbA, azA, zbB, azB);
      k0 += KC;
      if (k0 >= w) break;
      chunk(k0, zbB, azB, zbA, azA);
      k0 += KC;
    }
    bwd_epilogue<CH, T, TPW, TOP, DOUT, ZSRC>(args, acc_a, acc_z, nb + r, jt0, ptile, lane);
  }
};

namespace {

template <class CH, class T>
hipError_t launch_fwd_t(const void *A_in, const void *Wop, const void *Wlo, const float *b, void *A_out,
                        float *S_out, int64_t N_pad, int w, hipStream_t st) {
  if (__is_same(T, bf16_t) && !Wlo) return hipErrorInvalidValue;  // BF16 needs the weight pair
  const int WJ = (w % 128 == 0) ? 4 : ((w % 64 == 0) ? 2 : 1);
  const int WN = 4 / WJ;
  dim3 grid((unsigned)(N_pad / (32 * WN)), (unsigned)(w / (32 * WJ)));
  const T *Ai = static_cast<const T *>(A_in);
  const T *Wp = static_cast<const T *>(Wop);
  const T *Wl = static_cast<const T *>(Wlo);
  T *Ao = static_cast<T *>(A_out);
#define PJ_FWD(WJV, SV) return launch_body<KLayerFwd<CH, T, WJV, SV>>({Ai, Wp, Wl, b, Ao, S_out, w}, grid, 0, st)
  if (S_out) {
    if (WJ == 4) PJ_FWD(4, true);
    if (WJ == 2) PJ_FWD(2, true);
    PJ_FWD(1, true);
  }
  if (WJ == 4) PJ_FWD(4, false);
  if (WJ == 2) PJ_FWD(2, false);
  PJ_FWD(1, false);
#undef PJ_FWD
}

// LDS-staged configuration (points per workgroup, waves, neuron tiles per
// wave) for the backward layer kernel, or P = 0 when the staged tiles would
// not fit the LDS and register budget.
struct BwdLdsCfg {
  int P, NW, TPW;
};
inline BwdLdsCfg bwd_lds_cfg(int C, int w, int osz, bool two_tiles) {
  const size_t tile = (size_t)16 * (C * w + 8) * osz;
  const size_t lds = tile * (two_tiles ? 2 : 1);
  if (lds > 100 * 1024) return {0, 0, 0};
  switch (w) {
    case 32: return {16, 2, 1};
    case 64: return {16, 4, 1};
    case 128: return {16, 4, 2};
    case 256: return {16, 8, 2};
    default: return {0, 0, 0};
  }
}

template <class CH, class T, bool TOP, int DOUT, int ZSRC>
hipError_t launch_bwd_t(const BwdArgs &a, int64_t N_pad, int points, hipStream_t st) {
  const int w = a.w;
  // output-layer gradient partials: formed by the streaming 256-wide kernel only
  if (a.out_part && !(TOP && DOUT == 1 && ZSRC == Z_FROM_GEMM && sizeof(T) == 2 && CH::C <= 6 && points == 256 &&
                      w == 256 && N_pad == (a.N + kPointTile - 1) / kPointTile * kPointTile))
    return hipErrorInvalidValue;
  // wide layers: neuron-tiled, contraction staged through LDS in chunks
  // 16-bit operands with 8 channels (one full wave load per point and tile),
  // or up to 8 with points == 16: the double-buffered form (slower than the
  // single-buffered one at 6 channels on KS: more registers, lower occupancy)
  if constexpr (sizeof(T) == 2 && CH::C <= 8) {
    if (w >= 256 && w % 128 == 0 && (CH::C == 8 || points == 16)) {
      const dim3 grid((unsigned)((N_pad / 16) * (w / 128)));
      return launch_body<KLayerBwdKc2<CH, T, 8, 64, TOP, DOUT, ZSRC>>({a}, grid, 0, st);
    }
  }
  if (w >= 256 && w % 128 == 0) {
    const int tiles = (TOP ? 0 : 1) + (ZSRC == Z_FROM_GEMM ? 1 : 0);
    // points per workgroup (wide_bwd_points): 32 or 64 share each weight
    // fragment across two or four point tiles (16-bit operands, up to 6
    // channels); chunks of 64 neurons at 64 points keep the LDS in bounds
    if constexpr (sizeof(T) == 2 && CH::C <= 6) {
      if (points == 256 && w == 256 && N_pad == (a.N + kPointTile - 1) / kPointTile * kPointTile) {
        // sixteen 16-point tiles per workgroup, weights in registers, staging pipelined
        const size_t lds = (size_t)tiles * 16 * (CH::C * 256 + 8) * sizeof(T);
        const dim3 grid((unsigned)((N_pad / 16 + 15) / 16 * (256 / 128)));
        return launch_body<KLayerBwdKs<CH, T, 8, 256, TOP, DOUT, ZSRC, 1, 16>>({a}, grid, lds, st);
      }
      if (points == 32) {
        const size_t lds = (size_t)tiles * 32 * (CH::C * 128 + 8) * sizeof(T);
        const dim3 grid((unsigned)((N_pad / 32) * (w / 128)));
        return launch_body<KLayerBwdKc<CH, T, 8, 1, 128, TOP, DOUT, ZSRC, 2>>({a}, grid, lds, st);
      }
      if (points == 64) {
        const size_t lds = (size_t)tiles * 64 * (CH::C * 64 + 8) * sizeof(T);
        const dim3 grid((unsigned)((N_pad / 64) * (w / 128)));
        return launch_body<KLayerBwdKc<CH, T, 8, 1, 64, TOP, DOUT, ZSRC, 4>>({a}, grid, lds, st);
      }
    }
    constexpr int KC = sizeof(T) == 2 ? 128 : 64;
    const size_t lds = (size_t)tiles * 16 * (CH::C * KC + 8) * sizeof(T);
    const dim3 grid((unsigned)((N_pad / 16) * (w / 128)));
    return launch_body<KLayerBwdKc<CH, T, 8, 1, KC, TOP, DOUT, ZSRC>>({a}, grid, lds, st);
  }
  const BwdLdsCfg cfg = bwd_lds_cfg(CH::C, w, (int)sizeof(T), !TOP && ZSRC == Z_FROM_GEMM);
  // the first-layer gradient partials are produced by the LDS-staged kernels only
  if (a.seed_part && !(cfg.P > 0 && CH::C * w * (int)sizeof(T) % 16 == 0)) return hipErrorInvalidValue;
  if (cfg.P > 0 && CH::C * w * (int)sizeof(T) % 16 == 0) {
    const int tiles = (TOP ? 0 : 1) + (ZSRC == Z_FROM_GEMM ? 1 : 0);
    const size_t lds = (size_t)tiles * cfg.P * (CH::C * w + 8) * sizeof(T);
    const dim3 grid((unsigned)(N_pad / cfg.P));
#define PJ_BWDL(NWV, TPWV) return launch_body<KLayerBwdLds<CH, T, NWV, TPWV, 16, TOP, DOUT, ZSRC>>({a}, grid, lds, st)
    if (cfg.NW == 2) PJ_BWDL(2, 1);
    if (cfg.NW == 4 && cfg.TPW == 1) PJ_BWDL(4, 1);
    if (cfg.NW == 4) PJ_BWDL(4, 2);
    PJ_BWDL(8, 2);
#undef PJ_BWDL
  }
  const int WJ = (w % 128 == 0) ? 4 : ((w % 64 == 0) ? 2 : 1);
  const int WN = 4 / WJ;
  // Two accumulator sets (abar and the recomputed z) at C = 8 do not fit with
  // two 16-point tiles per wave.  The tile does not depend on the source of z,
  // so the saved-state and recompute variants run the same GEMM tiling.
  constexpr int NTN = CH::C >= 8 ? 1 : 2;
  dim3 grid((unsigned)(N_pad / (16 * NTN * WN)), (unsigned)(w / (32 * WJ)));
#define PJ_BWD(WJV) return launch_body<KLayerBwd<CH, T, WJV, NTN, TOP, DOUT, ZSRC>>({a}, grid, 0, st)
  if (WJ == 4) PJ_BWD(4);
  if (WJ == 2) PJ_BWD(2);
  PJ_BWD(1);
#undef PJ_BWD
}

template <class PDE, class T>
hipError_t launch_bwd_kind(const BwdArgs &a, bool top, int zsrc, int64_t N_pad, int points, hipStream_t st) {
  using CH = typename PDE::CH;
  constexpr int DO = PDE::DOUT;
  if (top) {
    if (zsrc == Z_FROM_S) return launch_bwd_t<CH, T, true, DO, Z_FROM_S>(a, N_pad, points, st);
    if (zsrc == Z_FROM_GEMM) return launch_bwd_t<CH, T, true, DO, Z_FROM_GEMM>(a, N_pad, points, st);
    return launch_bwd_t<CH, T, true, DO, Z_FROM_X>(a, N_pad, points, st);
  }
  if (zsrc == Z_FROM_S) return launch_bwd_t<CH, T, false, DO, Z_FROM_S>(a, N_pad, points, st);
  if (zsrc == Z_FROM_GEMM) return launch_bwd_t<CH, T, false, DO, Z_FROM_GEMM>(a, N_pad, points, st);
  return launch_bwd_t<CH, T, false, DO, Z_FROM_X>(a, N_pad, points, st);
}

// Launches for one PDE kind, by operand type.
template <class PDE>
hipError_t fwd_by_prec(int prec, const void *A_in, const void *Wop, const void *Wlo, const float *b, void *A_out,
                       float *S_out, int64_t N_pad, int w, hipStream_t st) {
  using CH = typename PDE::CH;
  switch (prec) {
    case P_FP32: return launch_fwd_t<CH, float>(A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    case P_BF16: return launch_fwd_t<CH, bf16_t>(A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    case P_FP16: return launch_fwd_t<CH, f16_t>(A_in, Wop, Wlo, b, A_out, S_out, N_pad, w, st);
    default: return hipErrorInvalidValue;
  }
}

template <class PDE>
hipError_t bwd_by_prec(int prec, const BwdArgs &a, bool top, int zsrc, int64_t N_pad, int points, hipStream_t st) {
  switch (prec) {
    case P_FP32: return launch_bwd_kind<PDE, float>(a, top, zsrc, N_pad, points, st);
    case P_BF16: return launch_bwd_kind<PDE, bf16_t>(a, top, zsrc, N_pad, points, st);
    case P_FP16: return launch_bwd_kind<PDE, f16_t>(a, top, zsrc, N_pad, points, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// The per-kind entry points (one translation unit each).
#define PJ_LAYER_KIND_DECL(NAME)                                                                                    \
  hipError_t layer_fwd_##NAME(int prec, const void *A_in, const void *Wop, const void *Wlo, const float *b,         \
                              void *A_out, float *S_out, int64_t N_pad, int w, hipStream_t st);                     \
  hipError_t layer_bwd_##NAME(int prec, const BwdArgs &a, bool top, int zsrc, int64_t N_pad, int points,            \
                              hipStream_t st);
PJ_LAYER_KIND_DECL(burgers)
PJ_LAYER_KIND_DECL(ns)
PJ_LAYER_KIND_DECL(ks)
PJ_LAYER_KIND_DECL(heat)
PJ_LAYER_KIND_DECL(aniso)
PJ_LAYER_KIND_DECL(burgers_bc)
#undef PJ_LAYER_KIND_DECL

}  // namespace pj
