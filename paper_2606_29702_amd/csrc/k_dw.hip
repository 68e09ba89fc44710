// Hidden-layer weight gradient dW = sum over rows (point, channel) of
// zbar_row^T a_row, i.e. a GEMM whose contraction runs over N * C rows, split
// over `splits` workgroup columns (split-K).  Each split writes its own FP32
// partial; a separate kernel sums the partials in split order, so the result
// is deterministic.  db = sum over the value rows of zbar.
//
// The stacks are stored [rows][w] with the neuron index contiguous, so the
// contraction index is strided in memory.  A workgroup stages 32 rows x 64
// columns of each operand through LDS and every lane then gathers its 8
// contraction elements down a column of the staged tile.
#include "dev_common.hpp"
#include "kernels.hpp"

namespace pj {

template <class T>
struct LdsPitch {
  // row pitch in elements: 8-byte aligned rows, padded to spread the column
  // gathers of the four lane groups over different banks
  static constexpr int value = 64 + 8 / (int)sizeof(T) * 2;
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

// Copy 8 consecutive elements (16 B for 16-bit types, 32 B for FP32) from
// global memory into an 8-byte aligned LDS row segment.
template <class T>
__device__ __forceinline__ void copy8(T *dst, const T *src) {
  constexpr int n64 = (int)sizeof(T);  // number of 8-byte words in 8 elements
  const uint2 *s = reinterpret_cast<const uint2 *>(src);
  uint2 *d = reinterpret_cast<uint2 *>(dst);
  uint2 tmp[n64];
#pragma unroll
  for (int i = 0; i < n64; ++i) tmp[i] = s[i];
#pragma unroll
  for (int i = 0; i < n64; ++i) d[i] = tmp[i];
}

template <class T, int TILE>
__global__ __launch_bounds__(256) void k_dw_hidden(const T *__restrict__ Zb, const T *__restrict__ A,
                                                   int64_t rows_total, int64_t rows_per_split, int w,
                                                   int C, float *__restrict__ part,
                                                   float *__restrict__ part_db) {
  // Workgroup tile: TILE x TILE of dW; wave (wj, wk) owns a (TILE/2)^2 quarter,
  // i.e. NT x NT MFMA 16x16 tiles.
  using M = Mma<T>;
  constexpr int P = LdsPitch<T>::value;
  constexpr int NT = TILE / 32;
  constexpr int H = TILE / 2;
  __shared__ __align__(16) T Zs[32 * P];
  __shared__ __align__(16) T As[32 * P];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wj = wave & 1, wk = wave >> 1;
  const int r16 = lane & 15, g = lane >> 4;
  const int j0 = blockIdx.x * TILE, k0 = blockIdx.y * TILE;
  const int64_t rb = (int64_t)blockIdx.z * rows_per_split;
  const int64_t re = rb + rows_per_split < rows_total ? rb + rows_per_split : rows_total;
  const bool do_db = blockIdx.y == 0;

  f32x4 acc[NT][NT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.f;

  // loader: 32 rows x TILE columns, 8 elements per thread
  constexpr int per_row = TILE / 8;
  const bool loader = t < 32 * per_row;
  const int lrow = t / per_row, lcol = (t % per_row) * 8;
  for (int64_t r0 = rb; r0 < re; r0 += 32) {
    if (loader) {
      copy8(Zs + lrow * P + lcol, Zb + (r0 + lrow) * w + j0 + lcol);
      copy8(As + lrow * P + lcol, A + (r0 + lrow) * w + k0 + lcol);
    }
    __syncthreads();
    if (do_db && t < TILE) {
      // rows r with r % C == 0 are value rows
      const int first = (int)((C - (r0 % C)) % C);
      for (int rr = first; rr < 32; rr += C) db += to_f32(Zs[rr * P + t]);
    }
    typename M::frag fa[NT], fb[NT];
#pragma unroll
    for (int jt = 0; jt < NT; ++jt) fa[jt] = gather_col<T>(Zs + (8 * g) * P + H * wj + 16 * jt + r16, P);
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) fb[kt] = gather_col<T>(As + (8 * g) * P + H * wk + 16 * kt + r16, P);
#pragma unroll
    for (int jt = 0; jt < NT; ++jt)
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) M::mma(acc[jt][kt], fa[jt], fb[kt]);
    __syncthreads();
  }

  float *pp = part + (int64_t)blockIdx.z * ((int64_t)w * w + w);
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
  if (do_db && t < TILE) part_db[(int64_t)blockIdx.z * ((int64_t)w * w + w) + j0 + t] = db;
}

namespace {
template <class T>
void launch_dw_t(const T *Zb, const T *A, int64_t rows, int64_t rps, int w, int C, float *part,
                 float *part_db, int splits, hipStream_t st) {
  if (w % 64 == 0) {
    dim3 grid((unsigned)(w / 64), (unsigned)(w / 64), (unsigned)splits);
    hipLaunchKernelGGL((k_dw_hidden<T, 64>), grid, dim3(256), 0, st, Zb, A, rows, rps, w, C, part, part_db);
  } else {
    dim3 grid((unsigned)(w / 32), (unsigned)(w / 32), (unsigned)splits);
    hipLaunchKernelGGL((k_dw_hidden<T, 32>), grid, dim3(256), 0, st, Zb, A, rows, rps, w, C, part, part_db);
  }
}
}  // namespace

hipError_t launch_dw_hidden(int prec, int C, const void *Zb, const void *A_prev, int64_t N_pad, int w,
                            float *part, float *part_db, int splits, hipStream_t st) {
  const int64_t rows = N_pad * C;
  int64_t rps = (rows + splits - 1) / splits;
  rps = (rps + 31) / 32 * 32;
  switch (prec) {
    case P_FP32:
      launch_dw_t<float>((const float *)Zb, (const float *)A_prev, rows, rps, w, C, part, part_db, splits, st);
      break;
    case P_BF16:
      launch_dw_t<bf16_t>((const bf16_t *)Zb, (const bf16_t *)A_prev, rows, rps, w, C, part, part_db, splits, st);
      break;
    case P_FP16:
      launch_dw_t<f16_t>((const f16_t *)Zb, (const f16_t *)A_prev, rows, rps, w, C, part, part_db, splits, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pj
