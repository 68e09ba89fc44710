// Persistent backward layer kernel with the hidden-layer weight gradient fused
// in.  For activation layer m it produces, per block of 16 points,
//   abar_m   = W_{m+1}^T Zbar_{m+1}      (MFMA; or W_L^T ubar at the top)
//   z_m      = saved state, or W_m A_{m-1} + b_m recomputed on MFMA
//   Zbar_m   = jet_adjoint(abar_m, z_m)
// and accumulates dW_m += Zbar_m^T A_{m-1} and db_m += sum of the value rows
// of Zbar_m over all the blocks it processes, in registers.  Each workgroup
// loops over blocks of points and writes one partial dW_m, db_m at the end;
// the partials are summed in workgroup order by the reduction kernel.
//
// Both operands of the gradient are already in LDS: the previous stack A_{m-1}
// is staged for the recompute, and Zbar_m is written back into the LDS tile
// that held Zbar_{m+1} once the abar GEMM has consumed it.  The gradient
// contracts over the rows (point, channel) of the tile, 16 at a time
// (MFMA 16x16x16), with each lane gathering its 4 rows down a column.
#include "dev_common.hpp"
#include "group.hpp"
#include "kernels.hpp"

namespace pj {

typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4v __attribute__((ext_vector_type(4)));

// MFMA with a 16-long contraction: lane l supplies the 4 consecutive
// contraction elements 4*(l/16) .. 4*(l/16)+3 of row (l%16) of A and of
// column (l%16) of B.
template <class T>
struct Mma16;
template <>
struct Mma16<bf16_t> {
  using frag = bf16x4v;
  static __device__ __forceinline__ void mma(f32x4 &acc, const frag &a, const frag &b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
};
template <>
struct Mma16<f16_t> {
  using frag = f16x4v;
  static __device__ __forceinline__ void mma(f32x4 &acc, const frag &a, const frag &b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc, 0, 0, 0);
  }
};
// FP32: four 16x16x4 MFMAs; MFMA e pairs element e of every lane's fragments,
// so lane group g covers contraction indices 4g + e on both sides.
template <>
struct Mma16<float> {
  using frag = f32x4;
  static __device__ __forceinline__ void mma(f32x4 &acc, const frag &a, const frag &b) {
#pragma unroll
    for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], acc, 0, 0, 0);
  }
};

template <class T, int C, int TPW>
__device__ __forceinline__ void tile_gemm(f32x4 (&acc)[TPW][C], const T *__restrict__ Wop, const T *stk, int pitch,
                                          int jt0, int w, int lane) {
  using M = Mma<T>;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const T *wrow = Wop + (int64_t)(jt0 * 16 + r) * w + 8 * g;
  const T *brow = stk + r * pitch + 8 * g;
  typename M::frag fa[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) fa[t] = M::load(wrow + (int64_t)t * 16 * w);
  for (int k = 0; k < w; k += 32) {
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

template <class CH, class T, int W, int NW, int TPW, bool TOP, int DOUT, int ZSRC>
struct KBwdDw {
  static constexpr int NT = NW * 64;
  struct Args {
    BwdArgs args;
    float * part;
    int64_t n_tiles;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const BwdArgs &args = a_.args;
    float *__restrict__ part = a_.part;
    int64_t n_tiles = a_.n_tiles;
    using M16 = Mma16<T>;
    constexpr int C = CH::C, P = 16;
    constexpr bool FAST = sizeof(T) == 2;
    constexpr int pitch = C * W + 8;
    constexpr int JW = W / NW;      // gradient rows owned by one wave
    constexpr int JT = JW / 16, KT = W / 16;
    constexpr int ROWS = P * C;     // contraction rows per tile (multiple of 16)
    static_assert(JW % 16 == 0 && ROWS % 16 == 0, "tile shape");
    // 16-byte pieces per thread when staging both tiles: all in flight at once
    constexpr int SNB = (2 * P * C * W * (int)sizeof(T) / 16 + NW * 64 - 1) / (NW * 64);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds_b = reinterpret_cast<T *>(smem_raw);  // Zbar_{m+1}, then Zbar_m
    T *lds_a = lds_b + P * pitch;                // A_{m-1}
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    constexpr int64_t ps = (int64_t)C * W;
    const int jt0 = wave * TPW;  // neuron tiles of this wave in the layer GEMMs (one 16-point tile)

    f32x4 dacc[JT][KT];
  #pragma unroll
    for (int a = 0; a < JT; ++a)
  #pragma unroll
      for (int b = 0; b < KT; ++b) dacc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float db = 0.f;

    for (int64_t tile = vb.x; tile < n_tiles; tile += vb.gx) {
      const int64_t nb = tile * P;
      if constexpr (!TOP)
        stage_rows<T, SNB, true>(lds_b, static_cast<const T *>(args.Zb_in) + nb * ps,
                                static_cast<const T *>(args.A_prev) + nb * ps, P, C * W, pitch, tid, NW * 64);
      else
        stage_rows<T, SNB, false>(lds_a, static_cast<const T *>(args.A_prev) + nb * ps, nullptr, P, C * W, pitch, tid,
                                 NW * 64);
      __syncthreads();

      f32x4 acc_a[TPW][C];
      if constexpr (!TOP) tile_gemm<T, C, TPW>(acc_a, static_cast<const T *>(args.WT), lds_b, pitch, jt0, W, lane);
      f32x4 acc_z[TPW][C];
      if constexpr (ZSRC == Z_FROM_GEMM)
        tile_gemm<T, C, TPW>(acc_z, static_cast<const T *>(args.Wz), lds_a, pitch, jt0, W, lane);
      __syncthreads();  // the Zbar_{m+1} tile is consumed; it now receives Zbar_m

      const int64_t n = nb + r;
      T *Zb_out = static_cast<T *>(args.Zb_out);
  #pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int mb = (jt0 + t) * 16 + 4 * g;
        float zz[4][C], s1[4];
        if constexpr (ZSRC == Z_FROM_S) {
  #pragma unroll
          for (int c = 0; c < C; ++c) {
            const f32x4 v = *reinterpret_cast<const f32x4 *>(args.S_in + n * ps + c * W + mb);
  #pragma unroll
            for (int i = 0; i < 4; ++i) zz[i][c] = v[i];
          }
  #pragma unroll
          for (int i = 0; i < 4; ++i) s1[i] = (1.f - zz[i][0]) * (1.f + zz[i][0]);
        } else {
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
  #pragma unroll
            for (int c = 0; c < C; ++c) zz[i][c] = acc_z[t][c][i];
            const TanhS ts = tanh_eval<FAST>(zz[i][0] + args.bz[mb + i]);
            zz[i][0] = ts.s;
            s1[i] = ts.s1;
          }
        }
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
              float sacc = 0.f;
  #pragma unroll
              for (int o = 0; o < DOUT; ++o) sacc += args.WL[o * W + mb + i] * ub[o][c];
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
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          store4(Zb_out + n * ps + c * W + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
          store4(lds_b + r * pitch + c * W + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
        }
      }
      __syncthreads();  // Zbar_m tile complete in LDS

      // db_m: value rows (channel 0) of the tile
      if (tid < W) {
  #pragma unroll
        for (int p = 0; p < P; ++p) db += to_f32(lds_b[p * pitch + tid]);
      }
      // dW_m += Zbar_m^T A_{m-1} over the tile's rows (point, channel), 16 rows
      // per step.  Below the top layer the steps stay rolled, which keeps the
      // gathered operands of a single step in registers (two waves per SIMD
      // instead of one); the top-layer variant keeps fewer accumulators live and
      // unrolls.
      auto dw_step = [&](int s) {
        int off[4];
  #pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 16 * s + 4 * g + e;
          off[e] = (row / C) * pitch + (row % C) * W;
        }
        typename M16::frag fa[JT], fb[KT];
        if constexpr (sizeof(T) == 2) {
          // LDS transpose read: within each group of 16 lanes, output lane
          // 4a + e receives element e of the 8-byte reads of lanes a, a + 4,
          // a + 8, a + 12.  Lane r of group g therefore reads row
          // 16 s + 4 g + r / 4 at columns 4 (r % 4) .. + 3 of the 16-column
          // tile, and receives column r of rows 16 s + 4 g .. + 3: its operand.
          const int row = 16 * s + 4 * g + (r >> 2);
          const int roff = (row / C) * pitch + (row % C) * W + 4 * (r & 3);
  #pragma unroll
          for (int jt = 0; jt < JT; ++jt) fa[jt] = lds_tr16<T>(lds_b + roff + wave * JW + jt * 16);
  #pragma unroll
          for (int kt = 0; kt < KT; ++kt) fb[kt] = lds_tr16<T>(lds_a + roff + kt * 16);
        } else {
  #pragma unroll
          for (int jt = 0; jt < JT; ++jt) {
            const int j = wave * JW + jt * 16 + r;
  #pragma unroll
            for (int e = 0; e < 4; ++e) fa[jt][e] = lds_b[off[e] + j];
          }
  #pragma unroll
          for (int kt = 0; kt < KT; ++kt) {
            const int k = kt * 16 + r;
  #pragma unroll
            for (int e = 0; e < 4; ++e) fb[kt][e] = lds_a[off[e] + k];
          }
        }
  #pragma unroll
        for (int jt = 0; jt < JT; ++jt)
  #pragma unroll
          for (int kt = 0; kt < KT; ++kt) M16::mma(dacc[jt][kt], fa[jt], fb[kt]);
      };
      if constexpr (TOP) {
  #pragma unroll
        for (int s = 0; s < ROWS / 16; ++s) dw_step(s);
      } else {
  #pragma unroll 1
        for (int s = 0; s < ROWS / 16; ++s) dw_step(s);
      }
      __syncthreads();  // before the next tile is staged over both buffers
    }

    float *pp = part + (int64_t)vb.x * ((int64_t)W * W + W);
  #pragma unroll
    for (int jt = 0; jt < JT; ++jt)
  #pragma unroll
      for (int kt = 0; kt < KT; ++kt)
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = wave * JW + jt * 16 + 4 * g + i;
          const int k = kt * 16 + r;
          pp[(int64_t)j * W + k] = dacc[jt][kt][i];
        }
    if (tid < W) pp[(int64_t)W * W + tid] = db;
  }
};

// Double-buffered form of k_bwd_dw for 16-bit operands, with z recomputed
// from A_{m-1}.  At the top layer only A_{H-1} is staged (abar = W_L^T ubar
// is one FP32 MFMA per neuron tile and channel), and the Zbar half of each
// buffer pair receives Zbar_H for the gradient.  The tiles are stored in LDS without row
// padding: 16-byte piece c of row p sits at piece position c ^ p of that row
// (rows of a multiple of 16 pieces), which keeps the 16 points of an MFMA
// operand read on different banks.  While a tile's jet adjoint and dW run,
// the next tile's Zbar_{m+1} and A_{m-1} stream into the other buffer pair
// with direct-to-LDS loads, so their HBM latency is hidden.  Every global load
// a tile waits on (weight fragments, biases) is issued before that prefetch,
// since the load counter completes in order.
// The double-buffered kernel applies to 16-bit operands when a row is a
// multiple of 16 pieces and the four tile buffers fit in 80 KB (two
// workgroups per CU).
template <class T>
constexpr bool bwd_db_ok(int C, int W) {
  return sizeof(T) == 2 && (C * W / 8) % 16 == 0 && 4 * 16 * C * W * 2 <= 80 * 1024;
}

template <class T, int C, int W>
struct SwzTile {
  static constexpr int RE = C * W;         // elements per row (one point)
  static constexpr int PER_ROW = RE / 8;   // 16-byte pieces per row
  static constexpr int ELEMS = 16 * RE;    // one 16-point tile
  static_assert(sizeof(T) == 2 && PER_ROW % 16 == 0, "swizzled tile shape");
  // element e of row p
  static __device__ __forceinline__ int at(int p, int e) { return p * RE + ((((e >> 3) ^ p)) << 3) + (e & 7); }
};

template <class T, int C, int W, int NW>
__device__ __forceinline__ void prefetch_tile(T *dst, const T *src, int wave, int lane) {
  using L = SwzTile<T, C, W>;
  constexpr int TOTAL = 16 * L::PER_ROW;  // pieces, a multiple of 256
#pragma unroll 1
  for (int q0 = 0; q0 < TOTAL; q0 += NW * 64) {
    const int qw = __builtin_amdgcn_readfirstlane(q0 + wave * 64);  // this wave's 64 pieces
    const int q = qw + lane;
    const int p = q / L::PER_ROW, cs = q - p * L::PER_ROW;
    // LDS piece q (row p, position cs) holds source piece cs ^ p of row p
    __builtin_amdgcn_global_load_lds((const void *)(src + p * L::RE + ((cs ^ p) << 3)),
                                     (__attribute__((address_space(3))) void *)(dst + qw * 8), 16, 0, 0);
  }
}

template <class T, int C, int TPW, int W>
__device__ __forceinline__ void swz_gemm(f32x4 (&acc)[TPW][C], const T *__restrict__ Wop, const T *stk, int jt0,
                                         int lane) {
  using M = Mma<T>;
  using L = SwzTile<T, C, W>;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const T *wrow = Wop + (int64_t)(jt0 * 16 + r) * W + 8 * g;
  const T *row = stk + r * L::RE;
  typename M::frag fa[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) fa[t] = M::load(wrow + (int64_t)t * 16 * W);
  // unrolled by two only: a full unroll hoists every operand read and costs
  // the second wave per SIMD
#pragma unroll 2
  for (int kk = 0; kk < W / 32; ++kk) {
    typename M::frag fb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) fb[c] = M::load(row + ((((c * W + kk * 32) >> 3) + g) ^ r) * 8);
    typename M::frag fn[TPW];
    const int kn = kk + 1 < W / 32 ? kk + 1 : kk;  // the next weight fragments
#pragma unroll
    for (int t = 0; t < TPW; ++t) fn[t] = M::load(wrow + (int64_t)t * 16 * W + kn * 32);
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int c = 0; c < C; ++c) M::mma(acc[t][c], fa[t], fb[c]);
#pragma unroll
    for (int t = 0; t < TPW; ++t) fa[t] = fn[t];
  }
}

template <class CH, class T, int W, int NW, int TPW, int DOUT, bool TOP>
struct KBwdDwDb {
  static constexpr int NT = NW * 64;
  struct Args {
    BwdArgs args;
    float * part;
    int64_t n_tiles;
    float * part_out;  // top layer: output-layer gradient partials, or null
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const BwdArgs &args = a_.args;
    float *__restrict__ part = a_.part;
    int64_t n_tiles = a_.n_tiles;
    float *__restrict__ part_out = a_.part_out;
    using M16 = Mma16<T>;
    using L = SwzTile<T, CH::C, W>;
    constexpr int C = CH::C, P = 16;
    constexpr int JW = W / NW;
    constexpr int JT = JW / 16, KT = W / 16;
    constexpr int ROWS = P * C;
    static_assert(JW % 16 == 0 && ROWS % 16 == 0, "tile shape");
    // two buffer pairs [Zbar][A] as separate objects, so that the compiler can
    // tell the pair being prefetched from the pair being read
    __shared__ __align__(16) T pair0[2 * L::ELEMS];
    __shared__ __align__(16) T pair1[2 * L::ELEMS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    constexpr int64_t ps = (int64_t)C * W;
    const int jt0 = wave * TPW;
    const T *Zb_in = static_cast<const T *>(args.Zb_in);
    const T *A_prev = static_cast<const T *>(args.A_prev);
    const T *WT = static_cast<const T *>(args.WT);
    const T *Wz = static_cast<const T *>(args.Wz);
    T *Zb_out = static_cast<T *>(args.Zb_out);

    f32x4 dacc[JT][KT];
  #pragma unroll
    for (int a = 0; a < JT; ++a)
  #pragma unroll
      for (int b = 0; b < KT; ++b) dacc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float db = 0.f;

    // top layer: this lane's W_L^T operand of each neuron tile, row r, output g
    [[maybe_unused]] float wl[TOP ? TPW : 1];
    // top layer of a one-output network, with part_out: the output layer's
    // gradient dW_L[j] = sum over points and channels of ubar[n][c] a_H[n][c][j],
    // with the activation jet a_H recomputed from z_H here (it is not read
    // back from the stack), for this lane's neurons; db_L in wave 0.  (More
    // outputs would cost the second wave per SIMD.)
    constexpr bool OUTG = TOP && DOUT == 1;
    [[maybe_unused]] float dwl[OUTG ? DOUT : 1][OUTG ? TPW : 1][4];
    [[maybe_unused]] float dbl[OUTG ? DOUT : 1];
    if constexpr (OUTG) {
  #pragma unroll
      for (int o = 0; o < DOUT; ++o) {
        dbl[o] = 0.f;
  #pragma unroll
        for (int t = 0; t < TPW; ++t)
  #pragma unroll
          for (int i = 0; i < 4; ++i) dwl[o][t][i] = 0.f;
      }
    }
    if constexpr (TOP) {
      static_assert(DOUT <= 4, "output contraction on one MFMA 16x16x4");
  #pragma unroll
      for (int t = 0; t < TPW; ++t) wl[t] = g < DOUT ? args.WL[g * W + (jt0 + t) * 16 + r] : 0.f;
    }

    if (vb.x < n_tiles) {
      const int64_t nb = (int64_t)vb.x * P;
      if constexpr (!TOP) prefetch_tile<T, C, W, NW>(pair0, Zb_in + nb * ps, wave, lane);
      prefetch_tile<T, C, W, NW>(pair0 + L::ELEMS, A_prev + nb * ps, wave, lane);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // one tile in buffer pair `cur`; the next one streams into pair `nxt`
    auto step = [&](int64_t tile, T *cur, T *nxt) __attribute__((always_inline)) {
      const int64_t nb = tile * P;
      T *zb_t = cur;
      T *a_t = cur + L::ELEMS;

      // the GEMMs (their weight fragments stream from L2 ahead of use)
      f32x4 acc_a[TPW][C], acc_z[TPW][C];
      [[maybe_unused]] float ubo[OUTG ? DOUT : 1][C];  // ubar of this lane's point (every lane)
      if constexpr (TOP) {
        // abar = W_L^T ubar contracts over the DOUT <= 4 outputs: one FP32
        // MFMA 16x16x4 per neuron tile and channel, output o = lane group g
        // (zero beyond DOUT).  The ubar loads are issued before the z GEMM.
        const int64_t n = nb + r;
        float ub[C];
        if constexpr (OUTG) {
  #pragma unroll
          for (int c = 0; c < C; ++c) {
            ubo[0][c] = args.ubar[n * C + c];
            ub[c] = g == 0 ? ubo[0][c] : 0.f;
          }
        } else {
  #pragma unroll
          for (int c = 0; c < C; ++c) ub[c] = g < DOUT ? args.ubar[(n * DOUT + g) * C + c] : 0.f;
        }
        swz_gemm<T, C, TPW, W>(acc_z, Wz, a_t, jt0, lane);
  #pragma unroll
        for (int t = 0; t < TPW; ++t)
  #pragma unroll
          for (int c = 0; c < C; ++c)
            acc_a[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(wl[t], ub[c], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      } else {
        swz_gemm<T, C, TPW, W>(acc_a, WT, zb_t, jt0, lane);
        swz_gemm<T, C, TPW, W>(acc_z, Wz, a_t, jt0, lane);
      }
      // tanh of the recomputed z_0 (with the bias, a global load) before the
      // prefetch below is issued: the load counter completes in order, so any
      // load waited on after the prefetch would wait for the prefetch too
      float sv[TPW][4], s1v[TPW][4];
  #pragma unroll
      for (int t = 0; t < TPW; ++t)
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const TanhS ts = tanh_eval<true>(acc_z[t][0][i] + args.bz[(jt0 + t) * 16 + 4 * g + i]);
          sv[t][i] = ts.s;
          s1v[t][i] = ts.s1;
        }
      __syncthreads();  // the Zbar_{m+1} tile is consumed; it now receives Zbar_m

      // the next tile streams into the other buffer pair during the adjoint and
      // dW; every load issued so far completes first, so that no later wait on
      // them also waits for the prefetch
      __builtin_amdgcn_s_waitcnt(0);
      const int64_t next = tile + vb.gx;
      if (next < n_tiles) {
        if constexpr (!TOP) prefetch_tile<T, C, W, NW>(nxt, Zb_in + next * P * ps, wave, lane);
        prefetch_tile<T, C, W, NW>(nxt + L::ELEMS, A_prev + next * P * ps, wave, lane);
      }

      const int64_t n = nb + r;
  #pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int mb = (jt0 + t) * 16 + 4 * g;
        float zz[4][C], s1[4];
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
  #pragma unroll
          for (int c = 1; c < C; ++c) zz[i][c] = acc_z[t][c][i];
          zz[i][0] = sv[t][i];
          s1[i] = s1v[t][i];
        }
        float out[4][C];
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          float ab[C], zb[C];
  #pragma unroll
          for (int c = 0; c < C; ++c) ab[c] = acc_a[t][c][i];
          jet_adjoint<CH>(ab, zz[i][0], s1[i], zz[i], zb);
  #pragma unroll
          for (int c = 0; c < C; ++c) out[i][c] = zb[c];
          if constexpr (OUTG) {
            if (part_out) {
              float act[C];
              jet_forward_from<CH>(zz[i][0], s1[i], zz[i], act);
  #pragma unroll
              for (int o = 0; o < DOUT; ++o) {
                float sacc = 0.f;
  #pragma unroll
                for (int c = 0; c < C; ++c) sacc += ubo[o][c] * act[c];
                dwl[o][t][i] += sacc;
              }
            }
          }
        }
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          store4(Zb_out + n * ps + c * W + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
          store4(zb_t + L::at(r, c * W + mb), out[0][c], out[1][c], out[2][c], out[3][c]);
        }
      }
      if constexpr (OUTG) {
        if (part_out && wave == 0 && g == 0)
  #pragma unroll
          for (int o = 0; o < DOUT; ++o) dbl[o] += ubo[o][0];
      }
      // Zbar_m tile complete in LDS.  A plain barrier after the LDS stores have
      // completed: a full __syncthreads() would also wait for the prefetch.
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
      __builtin_amdgcn_s_barrier();

      if (tid < W) {
  #pragma unroll
        for (int p = 0; p < P; ++p) db += to_f32(zb_t[L::at(p, tid)]);
      }
      // dW_m += Zbar_m^T A_{m-1}: 16 rows (point, channel) per step; LDS
      // transpose reads give each lane column r of rows 16 s + 4 g .. + 3
  #pragma unroll 1
      for (int s = 0; s < ROWS / 16; ++s) {
        const int row = 16 * s + 4 * g + (r >> 2);
        const int p = row / C, ch = row - p * C;
        const int half = 4 * (r & 1);
        typename M16::frag fa[JT], fb[KT];
  #pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          const int piece = ((ch * W + wave * JW + jt * 16) >> 3) + ((r & 3) >> 1);
          fa[jt] = lds_tr16<T>(zb_t + p * L::RE + ((piece ^ p) << 3) + half);
        }
  #pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const int piece = ((ch * W + kt * 16) >> 3) + ((r & 3) >> 1);
          fb[kt] = lds_tr16<T>(a_t + p * L::RE + ((piece ^ p) << 3) + half);
        }
  #pragma unroll
        for (int jt = 0; jt < JT; ++jt)
  #pragma unroll
          for (int kt = 0; kt < KT; ++kt) M16::mma(dacc[jt][kt], fa[jt], fb[kt]);
      }
      __builtin_amdgcn_s_waitcnt(0);  // the next tile has landed
      __syncthreads();                // and this tile's buffers are free
    };
    for (int64_t tile = vb.x; tile < n_tiles;) {
      step(tile, pair0, pair1);
      tile += vb.gx;
      if (tile >= n_tiles) break;
      step(tile, pair1, pair0);
      tile += vb.gx;
    }

    float *pp = part + (int64_t)vb.x * ((int64_t)W * W + W);
  #pragma unroll
    for (int jt = 0; jt < JT; ++jt)
  #pragma unroll
      for (int kt = 0; kt < KT; ++kt)
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = wave * JW + jt * 16 + 4 * g + i;
          const int k = kt * 16 + r;
          pp[(int64_t)j * W + k] = dacc[jt][kt][i];
        }
    if (tid < W) pp[(int64_t)W * W + tid] = db;
    if constexpr (OUTG) {
      if (part_out) {  // sums over the 16 points of the lane group, in a fixed order
        float *po = part_out + (int64_t)vb.x * (DOUT * W + DOUT);
  #pragma unroll
        for (int o = 0; o < DOUT; ++o)
  #pragma unroll
          for (int t = 0; t < TPW; ++t)
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float v = group_sum<16>(dwl[o][t][i]);
              if (r == 0) po[o * W + (jt0 + t) * 16 + 4 * g + i] = v;
            }
        if (wave == 0)
  #pragma unroll
          for (int o = 0; o < DOUT; ++o) {
            const float v = group_sum<16>(dbl[o]);
            if (lane == 0) po[DOUT * W + o] = v;
          }
      }
    }
  }
};

namespace {

template <class CH, class T, int W, bool TOP, int DOUT, int ZSRC>
hipError_t launch_w(const BwdArgs &a, float *part, int64_t n_tiles, int grid, float *part_out, hipStream_t st) {
  constexpr int NW = W == 32 ? 2 : (W == 256 ? 8 : 4);
  constexpr int TPW = (W / 16) / NW;
  if constexpr (ZSRC == Z_FROM_GEMM && bwd_db_ok<T>(CH::C, W))
    return (part_out && !(TOP && DOUT == 1))
               ? hipErrorInvalidValue
               : launch_body<KBwdDwDb<CH, T, W, NW, TPW, DOUT, TOP>>({a, part, n_tiles, part_out},
                                                                    dim3((unsigned)grid), 0, st);
  if (part_out) return hipErrorInvalidValue;  // only the double-buffered top layer forms them
  constexpr size_t lds = (size_t)2 * 16 * (CH::C * W + 8) * sizeof(T);
  return launch_body<KBwdDw<CH, T, W, NW, TPW, TOP, DOUT, ZSRC>>({a, part, n_tiles}, dim3((unsigned)grid), lds, st);
}

template <class PDE, class T>
hipError_t launch_kind(const BwdArgs &a, bool top, int zsrc, float *part, int64_t n_tiles, int grid,
                       float *part_out, hipStream_t st) {
  using CH = typename PDE::CH;
  constexpr int DO = PDE::DOUT;
#define PJ_W(WV)                                                                                    \
  if (a.w == WV) {                                                                                  \
    if (top)                                                                                        \
      return zsrc == Z_FROM_S ? launch_w<CH, T, WV, true, DO, Z_FROM_S>(a, part, n_tiles, grid, part_out, st)  \
                              : launch_w<CH, T, WV, true, DO, Z_FROM_GEMM>(a, part, n_tiles, grid, part_out, st); \
    return zsrc == Z_FROM_S ? launch_w<CH, T, WV, false, DO, Z_FROM_S>(a, part, n_tiles, grid, part_out, st)   \
                            : launch_w<CH, T, WV, false, DO, Z_FROM_GEMM>(a, part, n_tiles, grid, part_out, st); \
  }
  PJ_W(32) PJ_W(64) PJ_W(128)
#undef PJ_W
  return hipErrorInvalidValue;
}

}  // namespace

bool bwd_top_out_grad_supported(int C, int w, int prec, int dout) {
  return dout == 1 && prec != P_FP32 && (w == 32 || w == 64 || w == 128) && (C * w / 8) % 16 == 0 &&
         4 * 16 * C * w * 2 <= 80 * 1024;
}

bool bwd_dw_fused_supported(int C, int w, int prec) {
  if (w != 32 && w != 64 && w != 128) return false;
  const size_t lds = (size_t)2 * 16 * (C * w + 8) * op_size(prec);
  return lds <= 100 * 1024;
}

hipError_t launch_bwd_dw(int kind, int prec, const LayerBwd &L, float *part, int64_t N_pad, int grid,
                         hipStream_t st) {
  BwdArgs a{L.Zb_in, L.WT, L.ubar, L.WL, L.S_in, L.A_prev, L.Wz, L.bz, L.x, L.W1, L.N, L.Zb_out, L.w, nullptr, nullptr};
  const int zsrc = L.S_in ? Z_FROM_S : Z_FROM_GEMM;
  const int64_t n_tiles = N_pad / 16;
  auto by_prec = [&](auto pde) -> hipError_t {
    using PDE = decltype(pde);
    switch (prec) {
      case P_FP32: return launch_kind<PDE, float>(a, L.top, zsrc, part, n_tiles, grid, L.out_part, st);
      case P_BF16: return launch_kind<PDE, bf16_t>(a, L.top, zsrc, part, n_tiles, grid, L.out_part, st);
      case P_FP16: return launch_kind<PDE, f16_t>(a, L.top, zsrc, part, n_tiles, grid, L.out_part, st);
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
