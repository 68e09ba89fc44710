// Whole-network forward pass for one block of P collocation points per
// workgroup: seed layer, every hidden layer (stacked-channel GEMM on MFMA with
// the activation jet in its epilogue), linear output layer, residual and the
// block's loss partial sum, in one launch.  The same kernel also recomputes a
// segment of layers l_first..l_last from a saved stack (checkpointed
// backward), so recomputed stacks are bit-for-bit the ones of the forward pass.
//
// The block's stack [P][C][w] lives in LDS for the whole pass (one row of
// C*w + 8 elements per point; the 8-element pad puts consecutive points on
// different LDS banks for the 16-byte operand reads).  Layer l reads its
// weights from global memory (L2-resident, shared by all workgroups), the
// stack from LDS, and writes the new stack back into the same LDS buffer
// after a barrier.  Global memory sees only x, the stacks saved for the
// backward pass (written once, coalesced), the optional FP32 states, and the
// per-point outputs.
//
// Wave layout: the P/16 x w/16 MFMA output tiles of a layer are split over NW
// waves, TPW consecutive neuron tiles of PTW consecutive 16-point tiles per
// wave, so that every B operand read from LDS feeds TPW MFMAs and every weight
// fragment PTW x C of them (more points per workgroup read the weights fewer
// times per point).
#include "dev_common.hpp"
#include "group.hpp"
#include "kernels.hpp"

namespace pj {

// Copy of the block's stack (P rows of C w elements, LDS pitch `pitch`) to
// global memory, where the rows are contiguous, in 16-byte pieces.  With
// per_row pieces per row and R = max(1, NT / per_row) rows per sweep, thread
// t owns piece columns t % per_row (+ NT, ...) of rows t / per_row (+ R, ...),
// so its addresses advance by constant strides.  Threads with t / per_row >= R
// idle.
template <class T, int NT, int P>
__device__ __forceinline__ void copy_out_rows(T *g, const T *lds, int row_elems, int pitch, int row0, int col) {
  constexpr int per16 = 16 / (int)sizeof(T);
  const int per_row = row_elems / per16;
  const int R = per_row <= NT ? NT / per_row : 1;
  if (row0 >= R) return;
  for (int row = row0; row < P; row += R)
    for (int c = col; c < per_row; c += NT)
      *reinterpret_cast<uint4 *>(g + row * row_elems + c * per16) =
          *reinterpret_cast<const uint4 *>(lds + row * pitch + c * per16);
}

template <class PDE, class T, int NW, int TPW, int P, int PTW = 1>
struct KFwdFused {
  static constexpr int NT = NW * 64;
  struct Args {
    FusedFwdArgs a;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const FusedFwdArgs &a = a_.a;
    using CH = typename PDE::CH;
    using M = Mma<T>;
    constexpr int C = CH::C, D = CH::DIN, DOUT = PDE::DOUT, NRES = PDE::NRES;
    constexpr int NT = NW * 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *stk = reinterpret_cast<T *>(smem_raw);
    __shared__ float red32[P];
    __shared__ double red64[P];

    const int w = a.w;
    const int pitch = C * w + 8;  // elements per point row in LDS
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int64_t nb = (int64_t)vb.x * P;
    const int64_t gps = (int64_t)C * w;  // elements per point in a global stack

    // Wave layout of every layer: this wave owns the TPW neuron tiles jt0 ..
    // jt0 + TPW - 1 of the PTW 16-point tiles nt0 .. nt0 + PTW - 1; lane (r, g)
    // holds point (nt0 + q) * 16 + r of tile q and, in neuron tile t, neurons
    // (jt0 + t) * 16 + 4 g + 0..3.
    const int NJ = w / 16;
    const int NG = NJ / TPW;  // neuron groups
    const int nt0 = (wave / NG) * PTW;
    const int jt0 = (wave % NG) * TPW;
    // this thread's place in the stack copy-out (row and 16-byte column)
    const int per_row16 = C * w * (int)sizeof(T) / 16;
    const int out_row0 = tid / per_row16, out_col = tid - out_row0 * per_row16;

    // ---- input of layer l_first: the seed layer from x, or a saved stack
    if (a.l_first == 1) {
      // layer 1: z = W1 x + b1, d z / d x_i = W1[:, i], then the jet
  #pragma unroll
      for (int qt = 0; qt < PTW; ++qt) {
      const int p_l = (nt0 + qt) * 16 + r;  // this lane's point within the block
      const int64_t n_l = nb + p_l;
      float xin[D];
  #pragma unroll
      for (int i = 0; i < D; ++i) xin[i] = n_l < a.N ? a.x[n_l * D + i] : 0.f;
  #pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int mb = (jt0 + t) * 16 + 4 * g;
        float out[4][C], sv[4][C];
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = mb + i;
          float z[C];
  #pragma unroll
          for (int c = 0; c < C; ++c) z[c] = 0.f;
          float z0 = a.b1[j];
  #pragma unroll
          for (int q = 0; q < D; ++q) z0 += a.W1[j * D + q] * xin[q];
          z[0] = z0;
  #pragma unroll
          for (int d = 0; d < CH::NDIR; ++d) z[CH::at(d, 1)] = a.W1[j * D + CH::in(d)];
          float act[C], sg;
          jet_forward<CH, sizeof(T) == 2>(z, act, sg);
  #pragma unroll
          for (int c = 0; c < C; ++c) {
            out[i][c] = act[c];
            sv[i][c] = c == 0 ? sg : z[c];
          }
        }
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          store4(stk + p_l * pitch + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
          if (a.S[1]) store4(a.S[1] + n_l * gps + c * w + mb, sv[0][c], sv[1][c], sv[2][c], sv[3][c]);
        }
      }
      }
      __syncthreads();
      if (a.A[1]) copy_out_rows<T, NT, P>(static_cast<T *>(a.A[1]) + nb * gps, stk, C * w, pitch, out_row0, out_col);
    } else {
      // the saved stack of layer l_first - 1, coalesced 16-byte pieces
      stage_rows<T, 8, false>(stk, static_cast<const T *>(a.A_in) + nb * gps, nullptr, P, C * w, pitch, tid, NT);
      __syncthreads();
    }

    // ---- hidden layers max(2, l_first) .. l_last
    // BF16 operands: W enters as the pair (W_hi, W_lo), two MFMAs per product,
    // so that the network evaluated is the FP32 one to about 16 bits (rounding
    // W itself to 8 bits changes the function enough to move the parameter
    // gradient by up to ~10% on deep networks); the stack stays one BF16 operand.
    constexpr bool SPLIT = __is_same(T, bf16_t);
    for (int l = a.l_first > 2 ? a.l_first : 2; l <= a.l_last; ++l) {
      const T *Wl = static_cast<const T *>(a.Wop[l]);
      const T *wrow = Wl + (int64_t)(jt0 * 16 + r) * w + 8 * g;
      const T *lrow = SPLIT ? static_cast<const T *>(a.Wlo[l]) + (int64_t)(jt0 * 16 + r) * w + 8 * g : nullptr;
      const T *brow = stk + (nt0 * 16 + r) * pitch + 8 * g;
      typename M::frag fa[TPW], fl[TPW];
  #pragma unroll
      for (int t = 0; t < TPW; ++t) {
        fa[t] = M::load(wrow + (int64_t)t * 16 * w);
        if constexpr (SPLIT) fl[t] = M::load(lrow + (int64_t)t * 16 * w);
      }
      f32x4 acc[PTW][TPW][C];
  #pragma unroll
      for (int qt = 0; qt < PTW; ++qt)
  #pragma unroll
        for (int t = 0; t < TPW; ++t)
  #pragma unroll
          for (int c = 0; c < C; ++c) acc[qt][t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int k = 0; k < w; k += 32) {
        typename M::frag fn[TPW];
        const int kn = k + 32 < w ? k + 32 : k;  // prefetch the next weight fragments
  #pragma unroll
        for (int t = 0; t < TPW; ++t) fn[t] = M::load(wrow + (int64_t)t * 16 * w + kn);
        typename M::frag fln[TPW];
        if constexpr (SPLIT)
  #pragma unroll
          for (int t = 0; t < TPW; ++t) fln[t] = M::load(lrow + (int64_t)t * 16 * w + kn);
  #pragma unroll
        for (int qt = 0; qt < PTW; ++qt) {
          typename M::frag fb[C];
  #pragma unroll
          for (int c = 0; c < C; ++c) fb[c] = M::load(brow + qt * 16 * pitch + c * w + k);
  #pragma unroll
          for (int t = 0; t < TPW; ++t)
  #pragma unroll
            for (int c = 0; c < C; ++c) M::mma(acc[qt][t][c], fa[t], fb[c]);
          if constexpr (SPLIT)
  #pragma unroll
            for (int t = 0; t < TPW; ++t)
  #pragma unroll
              for (int c = 0; c < C; ++c) M::mma(acc[qt][t][c], fl[t], fb[c]);
        }
        if constexpr (SPLIT)
  #pragma unroll
          for (int t = 0; t < TPW; ++t) fl[t] = fln[t];
  #pragma unroll
        for (int t = 0; t < TPW; ++t) fa[t] = fn[t];
      }
      __syncthreads();  // every wave has finished reading layer l-1's stack

      const float *bl = a.b[l];
      float *Sl = a.S[l];
  #pragma unroll
      for (int qt = 0; qt < PTW; ++qt) {
      const int p = (nt0 + qt) * 16 + r;
      const int64_t n = nb + p;
  #pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int mb = (jt0 + t) * 16 + 4 * g;
        float out[4][C], sv[4][C];
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          float z[C], act[C], s;
  #pragma unroll
          for (int c = 0; c < C; ++c) z[c] = acc[qt][t][c][i];
          z[0] += bl[mb + i];
          jet_forward<CH, sizeof(T) == 2>(z, act, s);
  #pragma unroll
          for (int c = 0; c < C; ++c) {
            out[i][c] = act[c];
            sv[i][c] = c == 0 ? s : z[c];
          }
        }
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          store4(stk + p * pitch + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
          if (Sl) store4(Sl + n * gps + c * w + mb, sv[0][c], sv[1][c], sv[2][c], sv[3][c]);
        }
      }
      }
      __syncthreads();  // layer l's stack complete in LDS

      if (a.A[l])  // coalesced copy of the block's stack to global memory
        copy_out_rows<T, NT, P>(static_cast<T *>(a.A[l]) + nb * gps, stk, C * w, pitch, out_row0, out_col);
    }

    // ---- output layer on MFMA, residual, loss partial.  Wave v < P / 16 takes
    // the point tile v: U_c = W_L A_c for every channel c, with W_L as the A
    // operand (rows = outputs, padded to 16 with zeros) and the stack as the B
    // operand.  For 16-bit stacks W_L enters as a pair of 16-bit parts (value
    // and remainder), which keeps the product at FP32-level accuracy.  Lane l
    // of the output tile holds point l % 16 and outputs 4 (l / 16) + 0..3, so
    // lanes 0..15 hold every output of their point.
    if (!a.do_output) return;
    static_assert(DOUT <= 4, "outputs per point");
    if (wave < P / 16) {
      const int pt = wave;
      f32x4 uacc[C];
  #pragma unroll
      for (int c = 0; c < C; ++c) uacc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
      const T *brow = stk + (pt * 16 + r) * pitch + 8 * g;
      for (int k = 0; k < w; k += 32) {
        float wv[8];
  #pragma unroll
        for (int e = 0; e < 8; ++e) wv[e] = r < DOUT ? a.WL[r * w + k + 8 * g + e] : 0.f;
        typename M::frag fb[C];
  #pragma unroll
        for (int c = 0; c < C; ++c) fb[c] = M::load(brow + c * w + k);
        if constexpr (sizeof(T) == 2) {
          typename M::frag whi, wlo;
  #pragma unroll
          for (int e = 0; e < 8; ++e) {
            const T h = static_cast<T>(wv[e]);
            whi[e] = h;
            wlo[e] = static_cast<T>(wv[e] - static_cast<float>(h));
          }
  #pragma unroll
          for (int c = 0; c < C; ++c) {
            M::mma(uacc[c], whi, fb[c]);
            M::mma(uacc[c], wlo, fb[c]);
          }
        } else {
          typename M::frag wf;
          wf.lo = f32x4{wv[0], wv[1], wv[2], wv[3]};
          wf.hi = f32x4{wv[4], wv[5], wv[6], wv[7]};
  #pragma unroll
          for (int c = 0; c < C; ++c) M::mma(uacc[c], wf, fb[c]);
        }
      }
      if (g == 0) {
        const int p = pt * 16 + r;
        const int64_t n = nb + p;
        float u[DOUT][C];
  #pragma unroll
        for (int o = 0; o < DOUT; ++o)
  #pragma unroll
          for (int c = 0; c < C; ++c) u[o][c] = uacc[c][o];
  #pragma unroll
        for (int o = 0; o < DOUT; ++o) u[o][0] += a.bL[o];
        const bool valid = n < a.N;
        float xin[D];
  #pragma unroll
        for (int i = 0; i < D; ++i) xin[i] = valid ? a.x[n * D + i] : 0.f;
        float rr[NRES];
        PDE::residual(u, xin, a.k, rr);
        float l32 = 0.f;
        double l64 = 0.0;
        if (valid) {
  #pragma unroll
          for (int e = 0; e < NRES; ++e) {
            l32 += rr[e] * rr[e];
            if (a.loss_part64) l64 += (double)rr[e] * (double)rr[e];
          }
        }
        red32[p] = l32;
        red64[p] = l64;
        if (a.u_save)
  #pragma unroll
          for (int o = 0; o < DOUT; ++o)
  #pragma unroll
            for (int c = 0; c < C; ++c) a.u_save[(n * DOUT + o) * C + c] = u[o][c];
        if (a.r_save)
  #pragma unroll
          for (int e = 0; e < NRES; ++e) a.r_save[e * a.N_pad + n] = valid ? rr[e] : 0.f;
        if (valid) {
          if (a.r)
  #pragma unroll
            for (int e = 0; e < NRES; ++e) a.r[e * a.N + n] = rr[e];
          if (a.jets)
  #pragma unroll
            for (int o = 0; o < DOUT; ++o)
  #pragma unroll
              for (int c = 0; c < C; ++c) a.jets[(int64_t)(o * C + c) * a.N + n] = u[o][c];
        }
      }
    }
    __syncthreads();
    if (tid == 0 && a.loss_part) {
      float s = 0.f;
      double sd = 0.0;
      for (int p = 0; p < P; ++p) {
        s += red32[p];
        sd += red64[p];
      }
      a.loss_part[vb.x] = s;
      if (a.loss_part64) a.loss_part64[vb.x] = sd;
    }
  }
};

namespace {

// LDS bytes of one block's stack.
size_t stack_lds(int P, int C, int w, int osz) { return (size_t)P * (C * w + 8) * osz; }

template <class PDE, class T>
hipError_t launch_fused_t(const FusedFwdArgs &a, int P, hipStream_t st) {
  constexpr int C = PDE::CH::C;
  const int w = a.w;
  if constexpr (__is_same(T, bf16_t))  // BF16 needs the weight pair of every GEMM layer
    for (int l = a.l_first > 2 ? a.l_first : 2; l <= a.l_last; ++l)
      if (!a.Wlo[l]) return hipErrorInvalidValue;
  const size_t lds = stack_lds(P, C, w, sizeof(T));
  const unsigned grid = (unsigned)(a.N_pad / P);
  // tiles per layer = (P/16) * (w/16); 4 per wave where possible
  const int tiles = (P / 16) * (w / 16);
#define PJ_FUSED(NWV, TPWV, PV) return launch_body<KFwdFused<PDE, T, NWV, TPWV, PV>>({a}, dim3(grid), lds, st)
#define PJ_FUSED_P(NWV, TPWV, PV, PTWV) \
  return launch_body<KFwdFused<PDE, T, NWV, TPWV, PV, PTWV>>({a}, dim3(grid), lds, st)
  if (P == 64) {  // 16-bit operands: four point tiles per wave
    if constexpr (sizeof(T) == 2) {
      if (tiles == 16) PJ_FUSED_P(4, 1, 64, 4);    // w = 64
      if (tiles == 32) PJ_FUSED_P(4, 2, 64, 4);    // w = 128
      if (tiles == 64) PJ_FUSED_P(8, 2, 64, 4);    // w = 256
    }
    return hipErrorInvalidValue;
  }
  if (P == 32) {
    if (tiles == 4) PJ_FUSED(4, 1, 32);          // w = 32
    if (tiles == 8) PJ_FUSED(4, 2, 32);          // w = 64
    if (tiles == 16) PJ_FUSED(4, 4, 32);         // w = 128
    if (tiles == 32) PJ_FUSED(8, 4, 32);         // w = 256
    return hipErrorInvalidValue;
  }
  if (tiles == 16) PJ_FUSED(4, 4, 16);           // w = 256
  if (tiles == 32) PJ_FUSED(8, 4, 16);           // w = 512
  if (tiles == 8) PJ_FUSED(4, 2, 16);            // w = 128
  return hipErrorInvalidValue;
#undef PJ_FUSED
#undef PJ_FUSED_P
}

}  // namespace

bool fused_fwd_fits(int P, int C, int w, int prec) {
  const size_t cap = 144 * 1024;
  const int tiles = (P / 16) * (w / 16);
  if (stack_lds(P, C, w, op_size(prec)) > cap) return false;
  if (P == 64) return prec != P_FP32 && (tiles == 16 || tiles == 32 || tiles == 64);
  if (P == 32) return tiles == 4 || tiles == 8 || tiles == 16 || tiles == 32;
  if (P == 16) return tiles == 8 || tiles == 16 || tiles == 32;
  return false;
}

// Default points per workgroup: 16 where that tiling exists (more
// workgroups in flight per CU; the faster choice measured on the NS
// workload), else 32; 0 when neither fits.
int fused_fwd_points(int C, int w, int prec) {
  if (fused_fwd_fits(16, C, w, prec)) return 16;
  if (fused_fwd_fits(32, C, w, prec)) return 32;
  return 0;
}

hipError_t launch_fwd_fused(int kind, int prec, const FusedFwdArgs &a, int P, hipStream_t st) {
  auto by_prec = [&](auto pde) -> hipError_t {
    using PDE = decltype(pde);
    switch (prec) {
      case P_FP32: return launch_fused_t<PDE, float>(a, P, st);
      case P_BF16: return launch_fused_t<PDE, bf16_t>(a, P, st);
      case P_FP16: return launch_fused_t<PDE, f16_t>(a, P, st);
      default: return hipErrorInvalidValue;
    }
  };
  switch (kind) {
    case K_BURGERS: return by_prec(PdeBurgers{});
    case K_NS: return by_prec(PdeNS{});
    case K_KS: return by_prec(PdeKS{});
    case K_HEAT: return by_prec(PdeHeat{});
    case K_ANISO: return by_prec(PdeAniso{});
    case K_BURGERS_BC: return by_prec(PdeBurgersBC{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pj
