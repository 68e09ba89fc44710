// Device-side building blocks for gfx950: operand types, MFMA fragments and
// wave reductions.  Written for CDNA4 only (64-lane wavefronts).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pj {

typedef __bf16 bf16_t;
typedef _Float16 f16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// One MFMA step of the 16x16 output tile with K = 32 along the contraction.
// Lane l supplies 8 consecutive contraction elements starting at 8*(l/16) of
// row (l%16) of the A tile and of column (l%16) of the B tile; the output tile
// holds, in lane l, column (l%16) and rows 4*(l/16) + 0..3.
template <class T>
struct Mma;

template <>
struct Mma<bf16_t> {
  using frag = bf16x8;
  static __device__ __forceinline__ frag load(const bf16_t *p) {
    return *reinterpret_cast<const bf16x8 *>(p);
  }
  static __device__ __forceinline__ void mma(f32x4 &acc, const frag &a, const frag &b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
};

template <>
struct Mma<f16_t> {
  using frag = f16x8;
  static __device__ __forceinline__ frag load(const f16_t *p) {
    return *reinterpret_cast<const f16x8 *>(p);
  }
  static __device__ __forceinline__ void mma(f32x4 &acc, const frag &a, const frag &b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
  }
};

// FP32 operands: eight 16x16x4 MFMAs cover the same 32-long contraction.  MFMA
// e pairs element e of every lane's A and B fragments, so lane group g covers
// contraction indices 8g + e on both sides, the same set as the 16-bit forms.
template <>
struct Mma<float> {
  struct frag {
    f32x4 lo, hi;
  };
  static __device__ __forceinline__ frag load(const float *p) {
    frag f;
    f.lo = reinterpret_cast<const f32x4 *>(p)[0];
    f.hi = reinterpret_cast<const f32x4 *>(p)[1];
    return f;
  }
  static __device__ __forceinline__ void mma(f32x4 &acc, const frag &a, const frag &b) {
#pragma unroll
    for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[e], b.lo[e], acc, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[e], b.hi[e], acc, 0, 0, 0);
  }
};

template <class T>
__device__ __forceinline__ T to_op(float v) {
  return static_cast<T>(v);
}

// Store 4 consecutive values.
__device__ __forceinline__ void store4(float *p, float a, float b, float c, float d) {
  *reinterpret_cast<f32x4 *>(p) = f32x4{a, b, c, d};
}
__device__ __forceinline__ void store4(bf16_t *p, float a, float b, float c, float d) {
  *reinterpret_cast<bf16x4 *>(p) = bf16x4{(bf16_t)a, (bf16_t)b, (bf16_t)c, (bf16_t)d};
}
__device__ __forceinline__ void store4(f16_t *p, float a, float b, float c, float d) {
  *reinterpret_cast<f16x4 *>(p) = f16x4{(f16_t)a, (f16_t)b, (f16_t)c, (f16_t)d};
}

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(bf16_t v) { return static_cast<float>(v); }
__device__ __forceinline__ float to_f32(f16_t v) { return static_cast<float>(v); }

// Sum over the lanes of a group of `G` consecutive lanes (G a power of two <= 64).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
  return v;
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
  return v;
}

// 8-byte LDS transpose read of 16-bit elements (gfx950 ds_read_b64_tr_b16):
// within each group of 16 lanes, output lane 4a + e receives element e of the
// 8-byte reads of lanes a, a + 4, a + 8, a + 12 (checked on the GPU).  So when
// lane s of a group reads row k0 + s / 4 at columns c0 + 4 (s % 4) .. + 3,
// lane r receives column c0 + r of rows k0 .. k0 + 3: four consecutive
// contraction elements of an MFMA operand, from a tile stored row-major.
typedef short i16x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ auto lds_tr16(const T *p) {
  const i16x4 v =
      __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4 *)(const_cast<T *>(p)));
  if constexpr (__is_same(T, bf16_t))
    return __builtin_bit_cast(bf16x4, v);
  else
    return __builtin_bit_cast(f16x4, v);
}

// Row blocks moved between global memory, where the rows of a block are
// contiguous, and LDS, where row p starts at element p * pitch.  The unit is a
// 16-byte piece: piece q of a block sits at element q * (16 / sizeof(T)) in
// global memory and row(q) * (pitch - row_elems) further on in LDS.  A thread
// takes the pieces tid, tid + nthreads, ...; their rows are advanced by
// increments (one division per thread, none per piece).  Each thread issues
// NB reads before its NB writes, so that up to NB accesses are in flight.
// row_elems * sizeof(T) must be a multiple of 16 and every base address
// 16-byte aligned.
struct PieceWalk {
  int q, row, col;
  int per_row, step, drow, dcol;
  __device__ __forceinline__ PieceWalk(int q0, int step_, int per_row_)
      : q(q0), per_row(per_row_), step(step_) {
    row = q0 / per_row;
    col = q0 - row * per_row;
    drow = step / per_row;
    dcol = step - drow * per_row;
  }
  __device__ __forceinline__ void next() {
    q += step;
    row += drow;
    col += dcol;
    if (col >= per_row) {
      col -= per_row;
      ++row;
    }
  }
};

// Global -> LDS.  Block 0 (rows 0 .. rows-1 in LDS) comes from g0; with TWO,
// block 1 (LDS rows rows .. 2 rows - 1) comes from g1.
template <class T, int NB, bool TWO>
__device__ __forceinline__ void stage_rows(T *lds, const T *g0, const T *g1, int rows, int row_elems, int pitch,
                                           int tid, int nthreads) {
  constexpr int per16 = 16 / (int)sizeof(T);
  const int per_row = row_elems / per16;
  const int total0 = rows * per_row;
  const int total = TWO ? 2 * total0 : total0;
  const int pad = pitch - row_elems;
  PieceWalk it(tid, nthreads, per_row);
  while (it.q < total) {
    uint4 v[NB];
    int dst[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const bool live = it.q < total;
      const T *src = g0 + it.q * per16;
      if (TWO && it.q >= total0) src = g1 + (it.q - total0) * per16;
      v[u] = live ? *reinterpret_cast<const uint4 *>(src) : uint4{0u, 0u, 0u, 0u};
      dst[u] = live ? it.q * per16 + it.row * pad : -1;
      it.next();
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (dst[u] >= 0) *reinterpret_cast<uint4 *>(lds + dst[u]) = v[u];
  }
}

}  // namespace pj
