// Hidden-layer weight gradient dW = sum over rows (point, channel) of
// zbar_row^T a_row, i.e. a GEMM whose contraction runs over N * C rows, split
// over `splits` workgroup columns (split-K).  Each split writes its own FP32
// partial; a separate kernel sums the partials in split order, so the result
// is deterministic.  db = sum over the value rows of zbar.
//
// The stacks are stored [rows][w] with the neuron index contiguous, so the
// contraction index is strided in memory.  A workgroup stages 32 rows x TILE
// columns of each operand through LDS (double-buffered: the next chunk's
// global loads are in flight while the current chunk is multiplied).  Each
// lane takes its 8 contraction elements down a column of the staged tile: two
// LDS transpose reads for 16-bit types, a gather for FP32.
#include "dev_common.hpp"
#include "group.hpp"
#include "kernels.hpp"

namespace pj {

template <class T, int TILE, int RC>
struct DwLayout {
  // Row pitch in elements.  16-bit types: the transpose reads of one 16-lane
  // group take 32 bytes from each of 4 consecutive rows; a pitch of
  // TILE + 16 elements (32 bytes past a multiple of 128) puts those rows 8
  // banks apart, so the group's 128 bytes fall in 32 distinct banks, and
  // keeps rows 16-byte aligned for whole-piece stores.  FP32: rows stay
  // 8-byte aligned and rows 8 apart fall 16 banks apart, so the four lane
  // groups of a column gather do not collide.
  static constexpr int pitch = TILE + (sizeof(T) == 2 ? 16 : 2);
  static constexpr int tile_elems = RC * pitch;         // RC rows staged per chunk
  static constexpr int per_row = TILE / 8;              // 8-element copies per row
  static constexpr int copies = RC * per_row;           // per operand per chunk
  static constexpr int per_thread = (copies + 255) / 256;
  static constexpr int words = (int)sizeof(T);          // 8-byte words per copy
};

template <class T>
__device__ __forceinline__ typename Mma<T>::frag gather_col(const T *p, int pitch);

template <>
__device__ __forceinline__ Mma<bf16_t>::frag gather_col<bf16_t>(const bf16_t *p, int pitch) {
  bf16x8 f;
#pragma unroll
  for (int e = 0; e < 8; ++e) f[e] = p[e * pitch];
  return f;
}
template <>
__device__ __forceinline__ Mma<f16_t>::frag gather_col<f16_t>(const f16_t *p, int pitch) {
  f16x8 f;
#pragma unroll
  for (int e = 0; e < 8; ++e) f[e] = p[e * pitch];
  return f;
}
template <>
__device__ __forceinline__ Mma<float>::frag gather_col<float>(const float *p, int pitch) {
  Mma<float>::frag f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    f.lo[e] = p[e * pitch];
    f.hi[e] = p[(e + 4) * pitch];
  }
  return f;
}

// The same operand by two LDS transpose reads (16-bit types): contraction
// rows k0 .. k0 + 3 and k0 + 4 .. k0 + 7 of column c0 + lane % 16.
template <class T>
__device__ __forceinline__ typename Mma<T>::frag tr_col(const T *tile, int pitch, int k0, int c0, int r) {
  const T *p = tile + (k0 + (r >> 2)) * pitch + c0 + 4 * (r & 3);
  const auto lo = lds_tr16<T>(p), hi = lds_tr16<T>(p + 4 * pitch);
  typename Mma<T>::frag f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    f[e] = lo[e];
    f[e + 4] = hi[e];
  }
  return f;
}

template <class T, int TILE, int RC>
struct KDwHidden {
  static constexpr int NT = 256;
  struct Args {
    const T * Zb;
    const T * A;
    int64_t rows_total;
    int64_t rows_per_split;
    int w;
    int C;
    float * part;
    float * part_db;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const T *__restrict__ Zb = a_.Zb;
    const T *__restrict__ A = a_.A;
    int64_t rows_total = a_.rows_total;
    int64_t rows_per_split = a_.rows_per_split;
    int w = a_.w;
    int C = a_.C;
    float *__restrict__ part = a_.part;
    float *__restrict__ part_db = a_.part_db;
    // Workgroup tile: TILE x TILE of dW; wave (wj, wk) owns a (TILE/2)^2 quarter,
    // i.e. NT x NT MFMA 16x16 tiles.  RC rows (a multiple of 32) are staged per chunk.
    using M = Mma<T>;
    using LY = DwLayout<T, TILE, RC>;
    constexpr int P = LY::pitch;
    constexpr int NT = TILE / 32;
    constexpr int H = TILE / 2;
    __shared__ __align__(16) T lds[2][2][LY::tile_elems];  // [buffer][Zbar, A][rows x pitch]
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wj = wave & 1, wk = wave >> 1;
    const int r16 = lane & 15, g = lane >> 4;
    // weight tile and split; the tiles of one split share an XCD's L2
    const int lb = xcd_order(vb), ntiles = vb.gx;
    const int nt_ = w / TILE, tile = lb % ntiles, bx_ = tile % nt_, by_ = tile / nt_, bz_ = lb / ntiles;
    const int j0 = bx_ * TILE, k0 = by_ * TILE;
    const int64_t rb = (int64_t)bz_ * rows_per_split;
    const int64_t re = rb + rows_per_split < rows_total ? rb + rows_per_split : rows_total;
    const bool do_db = by_ == 0;

    f32x4 acc[NT][NT];
  #pragma unroll
    for (int a = 0; a < NT; ++a)
  #pragma unroll
      for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float db = 0.f;

    uint2 stage[2][LY::per_thread][LY::words];
    auto fetch = [&](int64_t r0) {
  #pragma unroll
      for (int u = 0; u < LY::per_thread; ++u) {
        const int q = t + 256 * u;
        if (q < LY::copies) {
          const int row = q / LY::per_row, col = (q % LY::per_row) * 8;
          const uint2 *sz = reinterpret_cast<const uint2 *>(Zb + (r0 + row) * w + j0 + col);
          const uint2 *sa = reinterpret_cast<const uint2 *>(A + (r0 + row) * w + k0 + col);
          if constexpr (sizeof(T) == 2) {  // one 16-byte load per piece
            const uint4 vz = *reinterpret_cast<const uint4 *>(sz), va = *reinterpret_cast<const uint4 *>(sa);
            stage[0][u][0] = uint2{vz.x, vz.y};
            stage[0][u][1] = uint2{vz.z, vz.w};
            stage[1][u][0] = uint2{va.x, va.y};
            stage[1][u][1] = uint2{va.z, va.w};
          } else {
  #pragma unroll
            for (int v = 0; v < LY::words; ++v) {
              stage[0][u][v] = sz[v];
              stage[1][u][v] = sa[v];
            }
          }
        }
      }
    };
    auto commit = [&](int buf) {
  #pragma unroll
      for (int u = 0; u < LY::per_thread; ++u) {
        const int q = t + 256 * u;
        if (q < LY::copies) {
          const int row = q / LY::per_row, col = (q % LY::per_row) * 8;
  #pragma unroll
          for (int m = 0; m < 2; ++m) {
            if constexpr (sizeof(T) == 2) {  // one 16-byte store per piece
              *reinterpret_cast<uint4 *>(&lds[buf][m][row * P + col]) =
                  uint4{stage[m][u][0].x, stage[m][u][0].y, stage[m][u][1].x, stage[m][u][1].y};
            } else {
              uint2 *d = reinterpret_cast<uint2 *>(&lds[buf][m][row * P + col]);
  #pragma unroll
              for (int v = 0; v < LY::words; ++v) d[v] = stage[m][u][v];
            }
          }
        }
      }
    };

    if (rb < re) {
      fetch(rb);
      commit(0);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t r0 = rb; r0 < re; r0 += RC) {
      const bool more = r0 + RC < re;
      if (more) fetch(r0 + RC);
      const T *Zs = lds[buf][0];
      const T *As = lds[buf][1];
      if (do_db && t < TILE) {
        // rows r with r % C == 0 are value rows
        const int first = (int)((C - (r0 % C)) % C);
        for (int rr = first; rr < RC; rr += C) db += to_f32(Zs[rr * P + t]);
      }
  #pragma unroll
      for (int ks = 0; ks < RC / 32; ++ks) {
        typename M::frag fa[NT], fb[NT];
        if constexpr (sizeof(T) == 2) {
  #pragma unroll
          for (int jt = 0; jt < NT; ++jt) fa[jt] = tr_col<T>(Zs, P, 32 * ks + 8 * g, H * wj + 16 * jt, r16);
  #pragma unroll
          for (int kt = 0; kt < NT; ++kt) fb[kt] = tr_col<T>(As, P, 32 * ks + 8 * g, H * wk + 16 * kt, r16);
        } else {
  #pragma unroll
          for (int jt = 0; jt < NT; ++jt)
            fa[jt] = gather_col<T>(Zs + (32 * ks + 8 * g) * P + H * wj + 16 * jt + r16, P);
  #pragma unroll
          for (int kt = 0; kt < NT; ++kt)
            fb[kt] = gather_col<T>(As + (32 * ks + 8 * g) * P + H * wk + 16 * kt + r16, P);
        }
  #pragma unroll
        for (int jt = 0; jt < NT; ++jt)
  #pragma unroll
          for (int kt = 0; kt < NT; ++kt) M::mma(acc[jt][kt], fa[jt], fb[kt]);
      }
      if (more) commit(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }

    float *pp = part + (int64_t)bz_ * ((int64_t)w * w + w);
  #pragma unroll
    for (int jt = 0; jt < NT; ++jt)
  #pragma unroll
      for (int kt = 0; kt < NT; ++kt)
  #pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = j0 + H * wj + 16 * jt + 4 * g + i;
          const int k = k0 + H * wk + 16 * kt + r16;
          pp[(int64_t)j * w + k] = acc[jt][kt][i];
        }
    if (do_db && t < TILE) part_db[(int64_t)bz_ * ((int64_t)w * w + w) + j0 + t] = db;
  }
};

int dw_tile(int w) { return (w % 128 == 0) ? 128 : ((w % 64 == 0) ? 64 : 32); }

namespace {
template <class T>
hipError_t launch_dw_t(const T *Zb, const T *A, int64_t rows, int64_t rps, int w, int C, float *part,
                       float *part_db, int splits, hipStream_t st) {
  const int tile = dw_tile(w);
  // x: the (w/tile)^2 weight tiles, y: the splits
  dim3 grid((unsigned)((w / tile) * (w / tile)), (unsigned)splits);
  // 128-wide tiles stage 64 rows per chunk (more bytes in flight per workgroup)
  if (tile == 128 && rps % 64 == 0)
    return launch_body<KDwHidden<T, 128, 64>>({Zb, A, rows, rps, w, C, part, part_db}, grid, 0, st);
  if (tile == 128) return launch_body<KDwHidden<T, 128, 32>>({Zb, A, rows, rps, w, C, part, part_db}, grid, 0, st);
  if (tile == 64) return launch_body<KDwHidden<T, 64, 32>>({Zb, A, rows, rps, w, C, part, part_db}, grid, 0, st);
  return launch_body<KDwHidden<T, 32, 32>>({Zb, A, rows, rps, w, C, part, part_db}, grid, 0, st);
}
}  // namespace

hipError_t launch_dw_hidden(int prec, int C, const void *Zb, const void *A_prev, int64_t N_pad, int w,
                            float *part, float *part_db, int splits, hipStream_t st) {
  const int64_t rows = N_pad * C;
  int64_t rps = (rows + splits - 1) / splits;
  rps = (rps + 31) / 32 * 32;
  switch (prec) {
    case P_FP32:
      return launch_dw_t<float>((const float *)Zb, (const float *)A_prev, rows, rps, w, C, part, part_db, splits, st);
    case P_BF16:
      return launch_dw_t<bf16_t>((const bf16_t *)Zb, (const bf16_t *)A_prev, rows, rps, w, C, part, part_db, splits,
                                 st);
    case P_FP16:
      return launch_dw_t<f16_t>((const f16_t *)Zb, (const f16_t *)A_prev, rows, rps, w, C, part, part_db, splits, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pj
