// Edge kernels of the partial-jet step: parameter casts, the seed (first)
// layer, the linear output layer with the residual and loss, their adjoints,
// the thin parameter-gradient reductions of the first and last layers, and the
// deterministic partial-sum reductions.  All HBM-bound; coalesced along the
// neuron index.
#include "dev_common.hpp"
#include "group.hpp"
#include "kernels.hpp"

namespace pj {

int op_size(int prec) { return prec == P_FP32 ? 4 : 2; }

// ------------------------------------------------------------------ casts
template <class T>
struct KCast {
  static constexpr int NT = 256;
  struct Args {
    const float * W;
    int rows;
    int cols;
    T * Wop;
    T * WTop;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const float *__restrict__ W = a_.W;
    int rows = a_.rows;
    int cols = a_.cols;
    T *__restrict__ Wop = a_.Wop;
    T *__restrict__ WTop = a_.WTop;
    const int64_t idx = (int64_t)vb.x * 256 + threadIdx.x;
    if (idx >= (int64_t)rows * cols) return;
    const int i = (int)(idx / cols), j = (int)(idx % cols);
    const float v = W[idx];
    Wop[idx] = static_cast<T>(v);
    if (WTop) WTop[(int64_t)j * rows + i] = static_cast<T>(v);
  }
};

hipError_t launch_cast(int prec, const float *W, int rows, int cols, void *Wop, void *WTop,
                       hipStream_t st) {
  const int64_t n = (int64_t)rows * cols;
  dim3 grid((unsigned)((n + 255) / 256));
  switch (prec) {
    case P_FP32:
      return launch_body<KCast<float>>({W, rows, cols, (float *)Wop, (float *)WTop}, grid, 0, st);
    case P_BF16:
      return launch_body<KCast<bf16_t>>({W, rows, cols, (bf16_t *)Wop, (bf16_t *)WTop}, grid, 0, st);
    case P_FP16:
      return launch_body<KCast<f16_t>>({W, rows, cols, (f16_t *)Wop, (f16_t *)WTop}, grid, 0, st);
    default: return hipErrorInvalidValue;
  }
}

// All hidden w x w weights in one launch: the y index of the grid selects the layer.
template <class T>
struct KCastAll {
  static constexpr int NT = 256;
  struct Args {
    CastPack pk;
    int w;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const CastPack &pk = a_.pk;
    int w = a_.w;
    const int l = vb.y;
    const int64_t idx = (int64_t)vb.x * 256 + threadIdx.x;
    if (idx >= (int64_t)w * w) return;
    const int i = (int)(idx / w), j = (int)(idx % w);
    const float v = pk.W[l][idx];
    const T hi = static_cast<T>(v);
    static_cast<T *>(pk.Wop[l])[idx] = hi;
    if (pk.WTop[l]) static_cast<T *>(pk.WTop[l])[(int64_t)j * w + i] = hi;
    if (pk.Wlo[l]) static_cast<T *>(pk.Wlo[l])[idx] = static_cast<T>(v - static_cast<float>(hi));
  }
};

hipError_t launch_cast_all(int prec, const CastPack &pk, int n, int w, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)(((int64_t)w * w + 255) / 256), (unsigned)n);
  switch (prec) {
    case P_FP32: return launch_body<KCastAll<float>>({pk, w}, grid, 0, st);
    case P_BF16: return launch_body<KCastAll<bf16_t>>({pk, w}, grid, 0, st);
    case P_FP16: return launch_body<KCastAll<f16_t>>({pk, w}, grid, 0, st);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------- seed layer
// Layer 1 takes the raw coordinates: its value pre-activation is W1 x + b1,
// its first-order derivative along input i is the column W1[:, i] (the seed
// d x / d x_i = e_i), and its higher derivatives vanish.  Thread = (point, neuron).
template <class CH, class T>
struct KSeedFwd {
  static constexpr int NT = 256;
  struct Args {
    const float * x;
    int64_t N;
    int64_t total;
    const float * W1;
    const float * b1;
    int w;
    T * A1;
    float * S1;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const float *__restrict__ x = a_.x;
    int64_t N = a_.N;
    int64_t total = a_.total;
    const float *__restrict__ W1 = a_.W1;
    const float *__restrict__ b1 = a_.b1;
    int w = a_.w;
    T *__restrict__ A1 = a_.A1;
    float *__restrict__ S1 = a_.S1;
    constexpr int C = CH::C, D = CH::DIN;
    const int64_t t = (int64_t)vb.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int64_t n = t / w;
    const int j = (int)(t % w);
    float z[C];
  #pragma unroll
    for (int c = 0; c < C; ++c) z[c] = 0.f;
    float z0 = b1[j];
  #pragma unroll
    for (int i = 0; i < D; ++i) z0 += W1[j * D + i] * (n < N ? x[n * D + i] : 0.f);
    z[0] = z0;
  #pragma unroll
    for (int d = 0; d < CH::NDIR; ++d) z[CH::at(d, 1)] = W1[j * D + CH::in(d)];
    float a[C], s;
    jet_forward<CH, sizeof(T) == 2>(z, a, s);
    const int64_t base = n * C * w + j;
  #pragma unroll
    for (int c = 0; c < C; ++c) {
      A1[base + (int64_t)c * w] = static_cast<T>(a[c]);
      if (S1) S1[base + (int64_t)c * w] = c == 0 ? s : z[c];
    }
  }
};

// ------------------------------------------------------- output + residual
// 16 lanes per point, 16 points per workgroup.  u[o][c] = W_L[o] . a_c (+ b_L
// on the value channel), then the residual, then the block's sum of r^2.
template <class PDE, class T>
struct KOutFwd {
  static constexpr int NT = 256;
  struct Args {
    const T * AH;
    const float * WL;
    const float * bL;
    const float * x;
    int64_t N;
    int64_t N_pad;
    int w;
    Coef k;
    float * jets;
    float * r;
    float * u_save;
    float * r_save;
    float * loss_part;
    double * loss_part64;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const T *__restrict__ AH = a_.AH;
    const float *__restrict__ WL = a_.WL;
    const float *__restrict__ bL = a_.bL;
    const float *__restrict__ x = a_.x;
    int64_t N = a_.N;
    int64_t N_pad = a_.N_pad;
    int w = a_.w;
    Coef k = a_.k;
    float *__restrict__ jets = a_.jets;
    float *__restrict__ r = a_.r;
    float *__restrict__ u_save = a_.u_save;
    float *__restrict__ r_save = a_.r_save;
    float *__restrict__ loss_part = a_.loss_part;
    double *__restrict__ loss_part64 = a_.loss_part64;
    using CH = typename PDE::CH;
    constexpr int C = CH::C, DOUT = PDE::DOUT, NRES = PDE::NRES, DIN = CH::DIN;
    __shared__ float red32[16];
    __shared__ double red64[16];
    const int q = threadIdx.x & 15, grp = threadIdx.x >> 4;
    const int64_t n = (int64_t)vb.x * 16 + grp;
    float u[DOUT][C];
  #pragma unroll
    for (int o = 0; o < DOUT; ++o)
  #pragma unroll
      for (int c = 0; c < C; ++c) u[o][c] = 0.f;
    const T *ap = AH + n * C * w;
    for (int kk = q; kk < w; kk += 16) {
      float wv[DOUT];
  #pragma unroll
      for (int o = 0; o < DOUT; ++o) wv[o] = WL[o * w + kk];
  #pragma unroll
      for (int c = 0; c < C; ++c) {
        const float av = to_f32(ap[c * w + kk]);
  #pragma unroll
        for (int o = 0; o < DOUT; ++o) u[o][c] += wv[o] * av;
      }
    }
  #pragma unroll
    for (int o = 0; o < DOUT; ++o) {
  #pragma unroll
      for (int c = 0; c < C; ++c) u[o][c] = group_sum<16>(u[o][c]);
      u[o][0] += bL[o];
    }
    const bool valid = n < N;
    float xin[DIN];
  #pragma unroll
    for (int i = 0; i < DIN; ++i) xin[i] = valid ? x[n * DIN + i] : 0.f;
    float rr[NRES];
    PDE::residual(u, xin, k, rr);
    float l32 = 0.f;
    double l64 = 0.0;
    if (valid) {
  #pragma unroll
      for (int e = 0; e < NRES; ++e) {
        l32 += rr[e] * rr[e];
        if (loss_part64) l64 += (double)rr[e] * (double)rr[e];
      }
    }
    if (q == 0) {
  #pragma unroll
      for (int o = 0; o < DOUT; ++o)
  #pragma unroll
        for (int c = 0; c < C; ++c) u_save[(n * DOUT + o) * C + c] = u[o][c];
  #pragma unroll
      for (int e = 0; e < NRES; ++e) r_save[e * N_pad + n] = valid ? rr[e] : 0.f;
      if (valid) {
        if (r)
  #pragma unroll
          for (int e = 0; e < NRES; ++e) r[e * N + n] = rr[e];
        if (jets)
  #pragma unroll
          for (int o = 0; o < DOUT; ++o)
  #pragma unroll
            for (int c = 0; c < C; ++c) jets[(int64_t)(o * C + c) * N + n] = u[o][c];
      }
      red32[grp] = l32;
      red64[grp] = l64;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      double sd = 0.0;
      for (int e = 0; e < 16; ++e) {
        s += red32[e];
        sd += red64[e];
      }
      loss_part[vb.x] = s;
      if (loss_part64) loss_part64[vb.x] = sd;
    }
  }
};

struct KLossReduce {
  static constexpr int NT = 256;
  struct Args {
    const float * part;
    const double * part64;
    int n_part;
    double inv_n;
    float * loss;
    double * loss64;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const float *__restrict__ part = a_.part;
    const double *__restrict__ part64 = a_.part64;
    int n_part = a_.n_part;
    double inv_n = a_.inv_n;
    float *__restrict__ loss = a_.loss;
    double *__restrict__ loss64 = a_.loss64;
    __shared__ float s32[256];
    __shared__ double s64[256];
    const int t = threadIdx.x;
    float a = 0.f;
    double b = 0.0;
    for (int i = t; i < n_part; i += 256) {
      a += part[i];
      if (part64) b += part64[i];
    }
    s32[t] = a;
    s64[t] = b;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
      if (t < m) {
        s32[t] += s32[t + m];
        s64[t] += s64[t + m];
      }
      __syncthreads();
    }
    if (t == 0) {
      if (loss) *loss = s32[0] * (float)inv_n;
      if (loss64) *loss64 = s64[0] * inv_n;
    }
  }
};

// ------------------------------------------------------ output adjoint
// ubar = d<rbar, r>/du by the residual adjoint; one thread per point.
template <class PDE>
struct KOutAdj {
  static constexpr int NT = 256;
  struct Args {
    const float * u_save;
    const float * r_save;
    const float * r_bar;
    const float * loss_bar;
    int64_t N;
    int64_t N_pad;
    float rbar_scale;
    Coef k;
    float * ubar;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const float *__restrict__ u_save = a_.u_save;
    const float *__restrict__ r_save = a_.r_save;
    const float *__restrict__ r_bar = a_.r_bar;
    const float *__restrict__ loss_bar = a_.loss_bar;
    int64_t N = a_.N;
    int64_t N_pad = a_.N_pad;
    float rbar_scale = a_.rbar_scale;
    Coef k = a_.k;
    float *__restrict__ ubar = a_.ubar;
    using CH = typename PDE::CH;
    constexpr int C = CH::C, DOUT = PDE::DOUT, NRES = PDE::NRES;
    const int64_t n = (int64_t)vb.x * 256 + threadIdx.x;
    if (n >= N_pad) return;
    const bool valid = n < N;
    float u[DOUT][C], ub[DOUT][C], rb[NRES];
  #pragma unroll
    for (int o = 0; o < DOUT; ++o)
  #pragma unroll
      for (int c = 0; c < C; ++c) u[o][c] = u_save[(n * DOUT + o) * C + c];
    // rbar = r_bar + lb * rbar_scale * r, lb = *loss_bar (1 when neither
    // cotangent is given: the loss gradient)
    const float lb = loss_bar ? *loss_bar : (r_bar ? 0.f : 1.f);
  #pragma unroll
    for (int e = 0; e < NRES; ++e)
      rb[e] = !valid ? 0.f : (r_bar ? r_bar[e * N + n] : 0.f) + lb * rbar_scale * r_save[e * N_pad + n];
    PDE::adjoint(u, rb, k, ub);
  #pragma unroll
    for (int o = 0; o < DOUT; ++o)
  #pragma unroll
      for (int c = 0; c < C; ++c) ubar[(n * DOUT + o) * C + c] = ub[o][c];
  }
};

// ------------------------------------------------ thin gradient reductions
// Output layer: dW_L[o][k] = sum_n sum_c ubar[n][o][c] a_H[n][c][k],
// db_L[o] = sum_n ubar[n][o][0].  Workgroup = one chunk of points.  A row
// (point, channel) of the stack is read by w/8 lanes, 8 neurons (16 bytes in
// BF16/FP16) each; the 256 / (w/8) row groups stride over the chunk's rows and
// their sums are added in group order through LDS.
template <class T>
__device__ __forceinline__ void load8f(const T *p, float (&v)[8]) {
  if constexpr (sizeof(T) == 2) {
    typedef T T8 __attribute__((ext_vector_type(8)));
    const T8 q = *reinterpret_cast<const T8 *>(p);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = static_cast<float>(q[e]);
  } else {
    const f32x4 lo = reinterpret_cast<const f32x4 *>(p)[0], hi = reinterpret_cast<const f32x4 *>(p)[1];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = lo[e];
      v[e + 4] = hi[e];
    }
  }
}

template <class PDE, class T>
struct KDwOut {
  static constexpr int NT = 256;
  struct Args {
    const float * ubar;
    const T * AH;
    int64_t N_pad;
    int w;
    float * part;
    int64_t pts_per_chunk;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const float *__restrict__ ubar = a_.ubar;
    const T *__restrict__ AH = a_.AH;
    int64_t N_pad = a_.N_pad;
    int w = a_.w;
    float *__restrict__ part = a_.part;
    int64_t pts_per_chunk = a_.pts_per_chunk;
    constexpr int C = PDE::CH::C, DOUT = PDE::DOUT;
    __shared__ float red[2048 * DOUT];  // (256 / (w/8)) groups x DOUT x w = 2048 * DOUT
    __shared__ float red_b[256 * DOUT];  // per row group: sum of ubar over value rows
    const int lpr = w / 8, rgs = 256 / lpr;
    const int q = threadIdx.x % lpr, rg = threadIdx.x / lpr;
    const int64_t nb = (int64_t)vb.x * pts_per_chunk;
    const int64_t ne = nb + pts_per_chunk < N_pad ? nb + pts_per_chunk : N_pad;
    const int rows = (int)(ne > nb ? (ne - nb) * C : 0);
    float acc[DOUT][8], accb[DOUT];
  #pragma unroll
    for (int o = 0; o < DOUT; ++o) {
      accb[o] = 0.f;
  #pragma unroll
      for (int e = 0; e < 8; ++e) acc[o][e] = 0.f;
    }
    if (rg < rgs) {
      // four rows per round, all loads issued before the arithmetic; rows past
      // the end re-read the round's first row (in bounds) and are not added
      constexpr int B = 4;
      for (int rr0 = rg; rr0 < rows; rr0 += B * rgs) {
        float a[B][8], u[B][DOUT];
        bool val[B];
  #pragma unroll
        for (int b = 0; b < B; ++b) {
          const int rr = rr0 + b * rgs < rows ? rr0 + b * rgs : rr0;
          const int64_t n = nb + rr / C;
          const int c = rr % C;
          val[b] = c == 0;
          load8f<T>(AH + (n * C + c) * w + 8 * q, a[b]);
  #pragma unroll
          for (int o = 0; o < DOUT; ++o) u[b][o] = ubar[(n * DOUT + o) * C + c];
        }
  #pragma unroll
        for (int b = 0; b < B; ++b) {
          if (rr0 + b * rgs < rows) {
  #pragma unroll
            for (int o = 0; o < DOUT; ++o) {
  #pragma unroll
              for (int e = 0; e < 8; ++e) acc[o][e] += u[b][o] * a[b][e];
              if (val[b]) accb[o] += u[b][o];  // db_L: value rows
            }
          }
        }
      }
  #pragma unroll
      for (int o = 0; o < DOUT; ++o)
  #pragma unroll
        for (int e = 0; e < 8; ++e) red[(rg * DOUT + o) * w + 8 * q + e] = acc[o][e];
      if (q == 0)
  #pragma unroll
        for (int o = 0; o < DOUT; ++o) red_b[rg * DOUT + o] = accb[o];
    }
    __syncthreads();
    const int64_t stride = (int64_t)DOUT * w + DOUT;
    float *pp = part + vb.x * stride;
    for (int idx = threadIdx.x; idx < DOUT * w; idx += 256) {
      float sum = 0.f;
      for (int g2 = 0; g2 < rgs; ++g2) sum += red[g2 * DOUT * w + idx];
      pp[idx] = sum;
    }
    if (threadIdx.x < DOUT) {
      float sum = 0.f;
      for (int g2 = 0; g2 < rgs; ++g2) sum += red_b[g2 * DOUT + threadIdx.x];
      pp[DOUT * w + threadIdx.x] = sum;
    }
  }
};

// First layer: dW_1[j][i] = sum_n (zbar_0[n][j] x[n][i] + zbar_{e_i}[n][j]),
// where zbar_{e_i} is the first-order channel along input i (its seed is the
// unit vector e_i); db_1[j] = sum_n zbar_0[n][j].  Same thread layout as above.
template <class CH, class T>
struct KDwSeed {
  static constexpr int NT = 256;
  struct Args {
    const T * Zb1;
    const float * x;
    int64_t N;
    int w;
    float * part;
    int64_t pts_per_chunk;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const T *__restrict__ Zb1 = a_.Zb1;
    const float *__restrict__ x = a_.x;
    int64_t N = a_.N;
    int w = a_.w;
    float *__restrict__ part = a_.part;
    int64_t pts_per_chunk = a_.pts_per_chunk;
    constexpr int C = CH::C, D = CH::DIN;
    __shared__ float red[256 * (D + 1)];
    const int span = w >= 256 ? 256 : w;
    const int nsub = 256 / span;
    const int sub = threadIdx.x / span;
    const int j = vb.y * 256 + threadIdx.x % span;
    const int64_t nb = (int64_t)vb.x * pts_per_chunk;
    const int64_t ne = nb + pts_per_chunk < N ? nb + pts_per_chunk : N;
    float acc[D + 1];
  #pragma unroll
    for (int i = 0; i <= D; ++i) acc[i] = 0.f;
    if (sub < nsub && j < w) {
      for (int64_t n = nb + sub; n < ne; n += nsub) {
        const T *zp = Zb1 + n * C * w + j;
        const float z0 = to_f32(zp[0]);
  #pragma unroll
        for (int i = 0; i < D; ++i) acc[i] += z0 * x[n * D + i];
  #pragma unroll
        for (int d = 0; d < CH::NDIR; ++d) acc[CH::in(d)] += to_f32(zp[(int64_t)CH::at(d, 1) * w]);
        acc[D] += z0;
      }
    }
  #pragma unroll
    for (int i = 0; i <= D; ++i) red[i * 256 + threadIdx.x] = acc[i];
    __syncthreads();
    if (threadIdx.x < span && j < w) {
      const int64_t stride = (int64_t)w * D + w;
      float *pp = part + vb.x * stride;
  #pragma unroll
      for (int i = 0; i <= D; ++i) {
        float s = 0.f;
        for (int q = 0; q < nsub; ++q) s += red[i * 256 + q * span + threadIdx.x];
        if (i < D)
          pp[j * D + i] = s;
        else
          pp[(int64_t)w * D + j] = s;
      }
    }
  }
};

// Deterministic sum over `splits` partial arrays.  A workgroup owns 256 / G
// outputs; thread (o, g) sums the splits g, g + G, g + 2G, ... of output o in
// order, and the G group sums are then added in g order.
template <int G>
struct KReduceG {
  static constexpr int NT = 256;
  struct Args {
    const float * part;
    int splits;
    int64_t stride;
    int64_t M1;
    int64_t M2;
    float * a32;
    float * b32;
    double * a64;
    double * b64;
    float scale;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const float *__restrict__ part = a_.part;
    int splits = a_.splits;
    int64_t stride = a_.stride;
    int64_t M1 = a_.M1;
    int64_t M2 = a_.M2;
    float *__restrict__ a32 = a_.a32;
    float *__restrict__ b32 = a_.b32;
    double *__restrict__ a64 = a_.a64;
    double *__restrict__ b64 = a_.b64;
    float scale = a_.scale;
    constexpr int OUTS = 256 / G;
    __shared__ float s32[256];
    __shared__ double s64[256];
    const int o = threadIdx.x % OUTS, g = threadIdx.x / OUTS;
    const int64_t q = (int64_t)vb.x * OUTS + o;
    const bool live = q < M1 + M2;
    const bool want64 = live && (q < M1 ? (a64 != nullptr) : (b64 != nullptr));
    float s = 0.f;
    double sd = 0.0;
    if (live) {
  #pragma unroll 4
      for (int sp = g; sp < splits; sp += G) {
        const float v = part[sp * stride + q];
        s += v;
        if (want64) sd += (double)v;
      }
    }
    s32[threadIdx.x] = s;
    s64[threadIdx.x] = sd;
    __syncthreads();
    if (g == 0 && live) {
      float t = 0.f;
      double td = 0.0;
      for (int k = 0; k < G; ++k) {
        t += s32[k * OUTS + o];
        td += s64[k * OUTS + o];
      }
      t *= scale;
      td *= (double)scale;
      if (q < M1) {
        if (a32) a32[q] = t;
        if (a64) a64[q] = td;
      } else {
        if (b32) b32[q - M1] = t;
        if (b64) b64[q - M1] = td;
      }
    }
  }
};

// The same sum with 16-byte loads.  A workgroup of NT threads owns COLS float4
// columns (4 * COLS consecutive outputs); thread (col, grp), col = tid % COLS,
// sums the splits grp, grp + G, ... (G = NT / COLS) of its column in order,
// and the G group sums are then added in group order.  Consecutive lanes read
// consecutive 16-byte pieces of one partial row.  Requires stride, M1 and
// M1 + M2 to be multiples of 4 and part 16-byte aligned.
template <int COLS, int NTH>
struct KReduceV4 {
  static constexpr int NT = NTH;
  struct Args {
    const float * part;
    int splits;
    int64_t stride;
    int64_t M1;
    int64_t M2;
    float * a32;
    float * b32;
    double * a64;
    double * b64;
    float scale;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const float *__restrict__ part = a_.part;
    int splits = a_.splits;
    int64_t stride = a_.stride;
    int64_t M1 = a_.M1;
    int64_t M2 = a_.M2;
    float *__restrict__ a32 = a_.a32;
    float *__restrict__ b32 = a_.b32;
    double *__restrict__ a64 = a_.a64;
    double *__restrict__ b64 = a_.b64;
    float scale = a_.scale;
    constexpr int G = NT / COLS;
    __shared__ f32x4 s32[NT];
    __shared__ double s64[NT][4];
    const int col = threadIdx.x % COLS, grp = threadIdx.x / COLS;
    const int64_t c4 = (int64_t)vb.x * COLS + col;
    const bool live = 4 * c4 < M1 + M2;
    const bool want64 = a64 != nullptr || b64 != nullptr;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    if (live) {
      const f32x4 *src = reinterpret_cast<const f32x4 *>(part) + c4;
      const int64_t st4 = stride / 4;
      if (want64) {
        for (int sp = grp; sp < splits; sp += G) {
          const f32x4 v = src[sp * st4];
          acc += v;
          d0 += (double)v[0];
          d1 += (double)v[1];
          d2 += (double)v[2];
          d3 += (double)v[3];
        }
      } else {
  #pragma unroll 4
        for (int sp = grp; sp < splits; sp += G) acc += src[sp * st4];
      }
    }
    s32[threadIdx.x] = acc;
    s64[threadIdx.x][0] = d0;
    s64[threadIdx.x][1] = d1;
    s64[threadIdx.x][2] = d2;
    s64[threadIdx.x][3] = d3;
    __syncthreads();
    if (grp == 0 && live) {
      f32x4 t = s32[col];
      double td[4] = {s64[col][0], s64[col][1], s64[col][2], s64[col][3]};
      for (int k = 1; k < G; ++k) {
        t += s32[k * COLS + col];
  #pragma unroll
        for (int e = 0; e < 4; ++e) td[e] += s64[k * COLS + col][e];
      }
  #pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t q = 4 * c4 + e;
        const float te = t[e] * scale;
        const double tde = td[e] * (double)scale;
        if (q < M1) {
          if (a32) a32[q] = te;
          if (a64) a64[q] = tde;
        } else {
          if (b32) b32[q - M1] = te;
          if (b64) b64[q - M1] = tde;
        }
      }
    }
  }
};

// ---------------------------------------------------------------- launchers
namespace {

template <class F>
hipError_t by_kind(int kind, F &&f) {
  switch (kind) {
    case K_BURGERS: return f(PdeBurgers{});
    case K_NS: return f(PdeNS{});
    case K_KS: return f(PdeKS{});
    case K_HEAT: return f(PdeHeat{});
    case K_ANISO: return f(PdeAniso{});
    case K_BURGERS_BC: return f(PdeBurgersBC{});
    default: return hipErrorInvalidValue;
  }
}

template <class F>
hipError_t by_prec(int prec, F &&f) {
  switch (prec) {
    case P_FP32: return f(float{});
    case P_BF16: return f(bf16_t{});
    case P_FP16: return f(f16_t{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_seed_fwd(int kind, int prec, const float *x, int64_t N, int64_t N_pad,
                           const float *W1, const float *b1, int w, void *A1, float *S1,
                           hipStream_t st) {
  const int64_t total = N_pad * w;
  dim3 grid((unsigned)((total + 255) / 256));
  return by_kind(kind, [&](auto pde) {
    using CH = typename decltype(pde)::CH;
    return by_prec(prec, [&](auto tv) {
      using T = decltype(tv);
      return launch_body<KSeedFwd<CH, T>>({x, N, total, W1, b1, w, static_cast<T *>(A1), S1}, grid, 0, st);
    });
  });
}

hipError_t launch_out_fwd(int kind, int prec, const void *A_H, const float *WL, const float *bL,
                          const float *x, int64_t N, int64_t N_pad, int w, Coef k, float *jets,
                          float *r, float *u_save, float *r_save, float *loss_part,
                          double *loss_part64, hipStream_t st) {
  dim3 grid((unsigned)(N_pad / 16));
  return by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    return by_prec(prec, [&](auto tv) {
      using T = decltype(tv);
      return launch_body<KOutFwd<PDE, T>>({static_cast<const T *>(A_H), WL, bL, x, N, N_pad, w, k, jets, r, u_save,
                                           r_save, loss_part, loss_part64},
                                          grid, 0, st);
    });
  });
}

hipError_t launch_loss_reduce(const float *part, const double *part64, int n_part, double inv_n,
                              float *loss, double *loss64, hipStream_t st) {
  return launch_body<KLossReduce>({part, part64, n_part, inv_n, loss, loss64}, dim3(1), 0, st);
}

hipError_t launch_out_adj(int kind, const float *u_save, const float *r_save, const float *r_bar,
                          const float *loss_bar, int64_t N, int64_t N_pad, float rbar_scale, Coef k, float *ubar,
                          hipStream_t st) {
  dim3 grid((unsigned)((N_pad + 255) / 256));
  return by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    return launch_body<KOutAdj<PDE>>({u_save, r_save, r_bar, loss_bar, N, N_pad, rbar_scale, k, ubar}, grid, 0, st);
  });
}

hipError_t launch_dw_out(int kind, int prec, const float *ubar, const void *A_H, int64_t N_pad,
                         int w, float *part, int n_chunks, hipStream_t st) {
  const int64_t ppc = (N_pad + n_chunks - 1) / n_chunks;  // chunks beyond N_pad write zeros
  dim3 grid((unsigned)n_chunks);
  return by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    return by_prec(prec, [&](auto tv) {
      using T = decltype(tv);
      return launch_body<KDwOut<PDE, T>>({ubar, static_cast<const T *>(A_H), N_pad, w, part, ppc}, grid, 0, st);
    });
  });
}

hipError_t launch_dw_seed(int kind, int prec, const void *Zb_1, const float *x, int64_t N,
                          int64_t /*N_pad*/, int w, float *part, int n_chunks, hipStream_t st) {
  const int64_t ppc = (N + n_chunks - 1) / n_chunks;
  dim3 grid((unsigned)n_chunks, (unsigned)((w + 255) / 256));
  return by_kind(kind, [&](auto pde) {
    using CH = typename decltype(pde)::CH;
    return by_prec(prec, [&](auto tv) {
      using T = decltype(tv);
      return launch_body<KDwSeed<CH, T>>({static_cast<const T *>(Zb_1), x, N, w, part, ppc}, grid, 0, st);
    });
  });
}

hipError_t launch_reduce_parts2(const float *part, int splits, int64_t stride, int64_t M1,
                                int64_t M2, float *a32, float *b32, double *a64, double *b64,
                                hipStream_t st, float scale, int select_splits) {
  const int64_t M = M1 + M2;
  // enough workgroups to keep many loads in flight: more threads per output
  // when there are few outputs or many splits.  The variant is chosen by
  // max(splits, select_splits), so that launches grouped together can use
  // one variant whatever their split counts.
  const int sel = splits > select_splits ? splits : select_splits;
  if (sel >= 64 && M >= 4096 && stride % 4 == 0 && M1 % 4 == 0 && M % 4 == 0 &&
      reinterpret_cast<uintptr_t>(part) % 16 == 0) {
    dim3 grid((unsigned)((M / 4 + 15) / 16));
    return launch_body<KReduceV4<16, 256>>({part, splits, stride, M1, M2, a32, b32, a64, b64, scale}, grid, 0, st);
  } else if (M * 4 < 256LL * 256 && sel >= 64) {
    dim3 grid((unsigned)((M + 7) / 8));
    return launch_body<KReduceG<32>>({part, splits, stride, M1, M2, a32, b32, a64, b64, scale}, grid, 0, st);
  } else if (sel >= 64) {
    dim3 grid((unsigned)((M + 15) / 16));
    return launch_body<KReduceG<16>>({part, splits, stride, M1, M2, a32, b32, a64, b64, scale}, grid, 0, st);
  } else {
    dim3 grid((unsigned)((M + 63) / 64));
    return launch_body<KReduceG<4>>({part, splits, stride, M1, M2, a32, b32, a64, b64, scale}, grid, 0, st);
  }
}

}  // namespace pj
