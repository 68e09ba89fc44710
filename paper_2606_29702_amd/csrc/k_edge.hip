// Edge kernels of the partial-jet step: parameter casts, the seed (first)
// layer, the linear output layer with the residual and loss, their adjoints,
// the thin parameter-gradient reductions of the first and last layers, and the
// deterministic partial-sum reductions.  All HBM-bound; coalesced along the
// neuron index.
#include "dev_common.hpp"
#include "kernels.hpp"

namespace pj {

int op_size(int prec) { return prec == P_FP32 ? 4 : 2; }

// ------------------------------------------------------------------ casts
template <class T>
__global__ __launch_bounds__(256) void k_cast(const float *__restrict__ W, int rows, int cols,
                                              T *__restrict__ Wop, T *__restrict__ WTop) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)rows * cols) return;
  const int i = (int)(idx / cols), j = (int)(idx % cols);
  const float v = W[idx];
  Wop[idx] = static_cast<T>(v);
  if (WTop) WTop[(int64_t)j * rows + i] = static_cast<T>(v);
}

hipError_t launch_cast(int prec, const float *W, int rows, int cols, void *Wop, void *WTop,
                       hipStream_t st) {
  const int64_t n = (int64_t)rows * cols;
  dim3 grid((unsigned)((n + 255) / 256));
  switch (prec) {
    case P_FP32:
      hipLaunchKernelGGL(k_cast<float>, grid, dim3(256), 0, st, W, rows, cols, (float *)Wop, (float *)WTop);
      break;
    case P_BF16:
      hipLaunchKernelGGL(k_cast<bf16_t>, grid, dim3(256), 0, st, W, rows, cols, (bf16_t *)Wop, (bf16_t *)WTop);
      break;
    case P_FP16:
      hipLaunchKernelGGL(k_cast<f16_t>, grid, dim3(256), 0, st, W, rows, cols, (f16_t *)Wop, (f16_t *)WTop);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------- seed layer
// Layer 1 takes the raw coordinates: its value pre-activation is W1 x + b1,
// its first-order derivative along input i is the column W1[:, i] (the seed
// d x / d x_i = e_i), and its higher derivatives vanish.  Thread = (point, neuron).
template <class CH, class T>
__global__ __launch_bounds__(256) void k_seed_fwd(const float *__restrict__ x, int64_t N, int64_t total,
                                                  const float *__restrict__ W1,
                                                  const float *__restrict__ b1, int w,
                                                  T *__restrict__ A1, float *__restrict__ S1) {
  constexpr int C = CH::C, D = CH::DIN;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
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
  jet_forward<CH>(z, a, s);
  const int64_t base = n * C * w + j;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    A1[base + (int64_t)c * w] = static_cast<T>(a[c]);
    S1[base + (int64_t)c * w] = c == 0 ? s : z[c];
  }
}

// ------------------------------------------------------- output + residual
// 16 lanes per point, 16 points per workgroup.  u[o][c] = W_L[o] . a_c (+ b_L
// on the value channel), then the residual, then the block's sum of r^2.
template <class PDE, class T>
__global__ __launch_bounds__(256) void k_out_fwd(const T *__restrict__ AH, const float *__restrict__ WL,
                                                 const float *__restrict__ bL, const float *__restrict__ x,
                                                 int64_t N, int64_t N_pad, int w, Coef k,
                                                 float *__restrict__ jets, float *__restrict__ r,
                                                 float *__restrict__ u_save, float *__restrict__ r_save,
                                                 float *__restrict__ loss_part,
                                                 double *__restrict__ loss_part64) {
  using CH = typename PDE::CH;
  constexpr int C = CH::C, DOUT = PDE::DOUT, NRES = PDE::NRES, DIN = CH::DIN;
  __shared__ float red32[16];
  __shared__ double red64[16];
  const int q = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t n = (int64_t)blockIdx.x * 16 + grp;
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
    loss_part[blockIdx.x] = s;
    if (loss_part64) loss_part64[blockIdx.x] = sd;
  }
}

__global__ __launch_bounds__(256) void k_loss_reduce(const float *__restrict__ part,
                                                     const double *__restrict__ part64, int n_part,
                                                     double inv_n, float *__restrict__ loss,
                                                     double *__restrict__ loss64) {
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

// ------------------------------------------------------ output adjoint
// ubar = d<rbar, r>/du (residual adjoint), abar_c = W_L^T ubar_c, then the
// jet adjoint of the last hidden layer.  16 lanes per point.
template <class PDE, class T>
__global__ __launch_bounds__(256) void k_out_bwd(const float *__restrict__ u_save,
                                                 const float *__restrict__ r_save,
                                                 const float *__restrict__ r_bar, int64_t N,
                                                 int64_t N_pad, float rbar_scale,
                                                 const float *__restrict__ WL,
                                                 const float *__restrict__ SH, int w, Coef k,
                                                 float *__restrict__ ubar, T *__restrict__ ZbH) {
  using CH = typename PDE::CH;
  constexpr int C = CH::C, DOUT = PDE::DOUT, NRES = PDE::NRES;
  const int q = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t n = (int64_t)blockIdx.x * 16 + grp;
  const bool valid = n < N;
  float u[DOUT][C], ub[DOUT][C], rb[NRES];
#pragma unroll
  for (int o = 0; o < DOUT; ++o)
#pragma unroll
    for (int c = 0; c < C; ++c) u[o][c] = u_save[(n * DOUT + o) * C + c];
#pragma unroll
  for (int e = 0; e < NRES; ++e)
    rb[e] = !valid ? 0.f : (r_bar ? r_bar[e * N + n] : rbar_scale * r_save[e * N_pad + n]);
  PDE::adjoint(u, rb, k, ub);
  if (q == 0)
#pragma unroll
    for (int o = 0; o < DOUT; ++o)
#pragma unroll
      for (int c = 0; c < C; ++c) ubar[(n * DOUT + o) * C + c] = ub[o][c];
  const float *sp = SH + n * C * w;
  T *zp = ZbH + n * C * w;
  for (int kk = q; kk < w; kk += 16) {
    float ab[C], zs[C], zb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < DOUT; ++o) s += WL[o * w + kk] * ub[o][c];
      ab[c] = s;
      zs[c] = sp[c * w + kk];
    }
    jet_adjoint<CH>(ab, zs[0], zs, zb);
#pragma unroll
    for (int c = 0; c < C; ++c) zp[c * w + kk] = static_cast<T>(zb[c]);
  }
}

// ------------------------------------------------ thin gradient reductions
// Output layer: dW_L[o][k] = sum_n sum_c ubar[n][o][c] a_H[n][c][k],
// db_L[o] = sum_n ubar[n][o][0].  Workgroup = (chunk of points, 256 neurons).
template <class PDE, class T>
__global__ __launch_bounds__(256) void k_dw_out(const float *__restrict__ ubar, const T *__restrict__ AH,
                                                int64_t N_pad, int w, float *__restrict__ part,
                                                int64_t pts_per_chunk) {
  constexpr int C = PDE::CH::C, DOUT = PDE::DOUT;
  const int kk = blockIdx.y * 256 + threadIdx.x;
  const int64_t nb = (int64_t)blockIdx.x * pts_per_chunk;
  const int64_t ne = nb + pts_per_chunk < N_pad ? nb + pts_per_chunk : N_pad;
  float acc[DOUT], accb[DOUT];
#pragma unroll
  for (int o = 0; o < DOUT; ++o) acc[o] = accb[o] = 0.f;
  for (int64_t n = nb; n < ne; ++n) {
    const float *ub = ubar + n * DOUT * C;
    if (kk < w) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const float a = to_f32(AH[(n * C + c) * w + kk]);
#pragma unroll
        for (int o = 0; o < DOUT; ++o) acc[o] += ub[o * C + c] * a;
      }
    }
#pragma unroll
    for (int o = 0; o < DOUT; ++o) accb[o] += ub[o * C];
  }
  const int64_t stride = (int64_t)DOUT * w + DOUT;
  float *pp = part + blockIdx.x * stride;
  if (kk < w)
#pragma unroll
    for (int o = 0; o < DOUT; ++o) pp[o * w + kk] = acc[o];
  if (blockIdx.y == 0 && threadIdx.x == 0)
#pragma unroll
    for (int o = 0; o < DOUT; ++o) pp[DOUT * w + o] = accb[o];
}

// First layer: dW_1[j][i] = sum_n (zbar_0[n][j] x[n][i] + zbar_{e_i}[n][j]),
// where zbar_{e_i} is the first-order channel along input i (its seed is the
// unit vector e_i); db_1[j] = sum_n zbar_0[n][j].
template <class CH, class T>
__global__ __launch_bounds__(256) void k_dw_seed(const T *__restrict__ Zb1, const float *__restrict__ x,
                                                 int64_t N, int w, float *__restrict__ part,
                                                 int64_t pts_per_chunk) {
  constexpr int C = CH::C, D = CH::DIN;
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= w) return;
  const int64_t nb = (int64_t)blockIdx.x * pts_per_chunk;
  const int64_t ne = nb + pts_per_chunk < N ? nb + pts_per_chunk : N;
  float acc[D], accb = 0.f;
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = 0.f;
  for (int64_t n = nb; n < ne; ++n) {
    const T *zp = Zb1 + n * C * w + j;
    const float z0 = to_f32(zp[0]);
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] += z0 * x[n * D + i];
#pragma unroll
    for (int d = 0; d < CH::NDIR; ++d) acc[CH::in(d)] += to_f32(zp[(int64_t)CH::at(d, 1) * w]);
    accb += z0;
  }
  const int64_t stride = (int64_t)w * D + w;
  float *pp = part + blockIdx.x * stride;
#pragma unroll
  for (int i = 0; i < D; ++i) pp[j * D + i] = acc[i];
  pp[(int64_t)w * D + j] = accb;
}

__global__ __launch_bounds__(256) void k_reduce_parts(const float *__restrict__ part, int splits,
                                                      int64_t stride, int64_t M1, int64_t M2,
                                                      float *__restrict__ a32, float *__restrict__ b32,
                                                      double *__restrict__ a64, double *__restrict__ b64) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= M1 + M2) return;
  const bool want64 = q < M1 ? (a64 != nullptr) : (b64 != nullptr);
  float s = 0.f;
  double sd = 0.0;
  for (int sp = 0; sp < splits; ++sp) {
    const float v = part[sp * stride + q];
    s += v;
    if (want64) sd += (double)v;
  }
  if (q < M1) {
    if (a32) a32[q] = s;
    if (a64) a64[q] = sd;
  } else {
    if (b32) b32[q - M1] = s;
    if (b64) b64[q - M1] = sd;
  }
}

// ---------------------------------------------------------------- launchers
namespace {

template <class F>
hipError_t by_kind(int kind, F &&f) {
  switch (kind) {
    case K_BURGERS: return f(PdeBurgers{});
    case K_NS: return f(PdeNS{});
    case K_KS: return f(PdeKS{});
    case K_HEAT: return f(PdeHeat{});
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
      hipLaunchKernelGGL((k_seed_fwd<CH, T>), grid, dim3(256), 0, st, x, N, total, W1, b1, w,
                         static_cast<T *>(A1), S1);
      return hipGetLastError();
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
      hipLaunchKernelGGL((k_out_fwd<PDE, T>), grid, dim3(256), 0, st, static_cast<const T *>(A_H),
                         WL, bL, x, N, N_pad, w, k, jets, r, u_save, r_save, loss_part, loss_part64);
      return hipGetLastError();
    });
  });
}

hipError_t launch_loss_reduce(const float *part, const double *part64, int n_part, double inv_n,
                              float *loss, double *loss64, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, st, part, part64, n_part, inv_n, loss, loss64);
  return hipGetLastError();
}

hipError_t launch_out_bwd(int kind, int prec, const float *u_save, const float *r_save,
                          const float *r_bar, int64_t N, int64_t N_pad, float rbar_scale,
                          const float *WL, const float *S_H, int w, Coef k, float *ubar,
                          void *Zb_H, hipStream_t st) {
  dim3 grid((unsigned)(N_pad / 16));
  return by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    return by_prec(prec, [&](auto tv) {
      using T = decltype(tv);
      hipLaunchKernelGGL((k_out_bwd<PDE, T>), grid, dim3(256), 0, st, u_save, r_save, r_bar, N, N_pad,
                         rbar_scale, WL, S_H, w, k, ubar, static_cast<T *>(Zb_H));
      return hipGetLastError();
    });
  });
}

hipError_t launch_dw_out(int kind, int prec, const float *ubar, const void *A_H, int64_t N_pad,
                         int w, float *part, int n_chunks, hipStream_t st) {
  const int64_t ppc = (N_pad + n_chunks - 1) / n_chunks;
  dim3 grid((unsigned)n_chunks, (unsigned)((w + 255) / 256));
  return by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    return by_prec(prec, [&](auto tv) {
      using T = decltype(tv);
      hipLaunchKernelGGL((k_dw_out<PDE, T>), grid, dim3(256), 0, st, ubar, static_cast<const T *>(A_H),
                         N_pad, w, part, ppc);
      return hipGetLastError();
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
      hipLaunchKernelGGL((k_dw_seed<CH, T>), grid, dim3(256), 0, st, static_cast<const T *>(Zb_1), x,
                         N, w, part, ppc);
      return hipGetLastError();
    });
  });
}

hipError_t launch_reduce_parts(const float *part, int splits, int64_t stride, int64_t M,
                               float *out32, double *out64, hipStream_t st) {
  return launch_reduce_parts2(part, splits, stride, M, 0, out32, nullptr, out64, nullptr, st);
}

hipError_t launch_reduce_parts2(const float *part, int splits, int64_t stride, int64_t M1,
                                int64_t M2, float *a32, float *b32, double *a64, double *b64,
                                hipStream_t st) {
  const int64_t M = M1 + M2;
  dim3 grid((unsigned)((M + 255) / 256));
  hipLaunchKernelGGL(k_reduce_parts, grid, dim3(256), 0, st, part, splits, stride, M1, M2, a32, b32,
                     a64, b64);
  return hipGetLastError();
}

}  // namespace pj
