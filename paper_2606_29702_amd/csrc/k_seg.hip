// Composite training loss over segments of one point set (Sec. 3.1.1: the
// initial-condition, boundary and PDE points are concatenated, the network is
// evaluated once on all of them, and the outputs are split to assemble the
// loss terms).  The forward pass has already left every point's outputs
// u_save[n][o][c] and its PDE residual r_save[e][n]; these kernels assemble
// the segments' terms and, for the backward pass, every point's cotangent.
//   PDE        the PDE residual at each point
//   DIRICHLET  u_o - g_o(x) for the outputs o in the mask (value channel)
//   PERIODIC   consecutive point pairs: u_oc(first) - u_oc(second) for the
//              (output, channel) pairs in the mask
// seg_loss[s] = (1 / units_s) sum over the segment's units (points, or pairs)
// of its squared terms; loss = sum_s weight_s seg_loss[s].
#include "dev_common.hpp"
#include "group.hpp"
#include "kernels.hpp"

namespace pj {

namespace {

__device__ __forceinline__ int seg_of(const SegPack &sp, int64_t n) {
  for (int s = 0; s < sp.n; ++s)
    if (n >= sp.begin[s] && n < sp.begin[s] + sp.count[s]) return s;
  return -1;
}

template <int DOUT>
__device__ __forceinline__ float seg_data(const SegPack &sp, int s, int o, float x0, int64_t n) {
  switch (sp.data[s]) {
    case SEG_DATA_CONST: return sp.param[s][o];
    case SEG_DATA_SIN: return sp.param[s][0] * sinpif(sp.param[s][1] * x0);
    case SEG_DATA_VALUES: return sp.values[s][(n - sp.begin[s]) * DOUT + o];
    default: return 0.f;
  }
}

}  // namespace

// Partial sums of the squared terms: workgroup b covers units
// [chunk * 256, chunk * 256 + 256) of the segment sp.blk_seg(b); one unit per
// thread, summed in a fixed tree order.
template <class PDE>
struct KSegLoss {
  static constexpr int NT = 256;
  struct Args {
    SegPack sp;
    const float *u_save, *r_save, *x;
    int64_t N_pad;
    float *part;  // one per workgroup
  };
  static __device__ __forceinline__ void run(const Args &a, VBlock vb) {
    using CH = typename PDE::CH;
    constexpr int C = CH::C, DOUT = PDE::DOUT, NRES = PDE::NRES, DIN = CH::DIN;
    __shared__ float red[NT];
    const SegPack &sp = a.sp;
    int s = 0;
    while (s + 1 < sp.n && vb.x >= sp.blk_start[s + 1]) ++s;
    const int64_t unit = (int64_t)(vb.x - sp.blk_start[s]) * NT + threadIdx.x;
    const int64_t units = sp.type[s] == SEG_PERIODIC ? sp.count[s] / 2 : sp.count[s];
    float v = 0.f;
    if (unit < units) {
      if (sp.type[s] == SEG_PDE) {
        const int64_t n = sp.begin[s] + unit;
#pragma unroll
        for (int e = 0; e < NRES; ++e) {
          const float r = a.r_save[e * a.N_pad + n];
          v += r * r;
        }
      } else if (sp.type[s] == SEG_DIRICHLET) {
        const int64_t n = sp.begin[s] + unit;
        const float x0 = a.x[n * DIN];
#pragma unroll
        for (int o = 0; o < DOUT; ++o)
          if (sp.mask[s] >> (o * C) & 1u) {
            const float r = a.u_save[(n * DOUT + o) * C] - seg_data<DOUT>(sp, s, o, x0, n);
            v += r * r;
          }
      } else {
        const int64_t na = sp.begin[s] + 2 * unit, nb = na + 1;
#pragma unroll
        for (int o = 0; o < DOUT; ++o)
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (sp.mask[s] >> (o * C + c) & 1u) {
              const float r = a.u_save[(na * DOUT + o) * C + c] - a.u_save[(nb * DOUT + o) * C + c];
              v += r * r;
            }
      }
    }
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int m = NT / 2; m >= 1; m >>= 1) {
      if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.part[vb.x] = red[0];
  }
};

// seg_loss[s] = (sum of the segment's partials in order) / units_s and
// loss = sum_s weight_s seg_loss[s] (one workgroup).
struct KSegReduce {
  static constexpr int NT = 64;
  struct Args {
    SegPack sp;
    const float *part;
    float *seg_loss;  // may be null
    float *loss;      // may be null
  };
  static __device__ __forceinline__ void run(const Args &a, VBlock) {
    __shared__ float segv[kMaxSegments];
    const SegPack &sp = a.sp;
    const int s = (int)threadIdx.x;
    if (s < sp.n) {
      float t = 0.f;
      for (int b = sp.blk_start[s]; b < sp.blk_start[s + 1]; ++b) t += a.part[b];
      const int64_t units = sp.type[s] == SEG_PERIODIC ? sp.count[s] / 2 : sp.count[s];
      t = t / (float)units;
      segv[s] = t;
      if (a.seg_loss) a.seg_loss[s] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0 && a.loss) {
      float l = 0.f;
      for (int q = 0; q < sp.n; ++q) l += sp.weight[q] * segv[q];
      *a.loss = l;
    }
  }
};

// Cotangent of the loss with respect to every point's outputs, scaled by the
// power of two S: ubar = S d loss / d u.  cot[s] = S * weight_s * 2 / units_s.
// Points outside every segment, and padded points, get zero.
template <class PDE>
struct KSegAdj {
  static constexpr int NT = 256;
  struct Args {
    SegPack sp;
    const float *u_save, *r_save, *x;
    int64_t N_pad;
    Coef k;
    float *ubar;
  };
  static __device__ __forceinline__ void run(const Args &a, VBlock vb) {
    using CH = typename PDE::CH;
    constexpr int C = CH::C, DOUT = PDE::DOUT, NRES = PDE::NRES, DIN = CH::DIN;
    const int64_t n = (int64_t)vb.x * NT + threadIdx.x;
    if (n >= a.N_pad) return;
    const SegPack &sp = a.sp;
    float ub[DOUT][C];
#pragma unroll
    for (int o = 0; o < DOUT; ++o)
#pragma unroll
      for (int c = 0; c < C; ++c) ub[o][c] = 0.f;
    const int s = seg_of(sp, n);
    if (s >= 0) {
      const float cot = sp.cot[s];
      if (sp.type[s] == SEG_PDE) {
        float u[DOUT][C], rb[NRES];
#pragma unroll
        for (int o = 0; o < DOUT; ++o)
#pragma unroll
          for (int c = 0; c < C; ++c) u[o][c] = a.u_save[(n * DOUT + o) * C + c];
#pragma unroll
        for (int e = 0; e < NRES; ++e) rb[e] = cot * a.r_save[e * a.N_pad + n];
        PDE::adjoint(u, rb, a.k, ub);
      } else if (sp.type[s] == SEG_DIRICHLET) {
        const float x0 = a.x[n * DIN];
#pragma unroll
        for (int o = 0; o < DOUT; ++o)
          if (sp.mask[s] >> (o * C) & 1u)
            ub[o][0] = cot * (a.u_save[(n * DOUT + o) * C] - seg_data<DOUT>(sp, s, o, x0, n));
      } else {
        const int64_t j = n - sp.begin[s];
        const int64_t na = n - (j & 1), nb = na + 1;  // the pair, first and second
        const float sign = (j & 1) ? -1.f : 1.f;
#pragma unroll
        for (int o = 0; o < DOUT; ++o)
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (sp.mask[s] >> (o * C + c) & 1u)
              ub[o][c] = sign * cot * (a.u_save[(na * DOUT + o) * C + c] - a.u_save[(nb * DOUT + o) * C + c]);
      }
    }
#pragma unroll
    for (int o = 0; o < DOUT; ++o)
#pragma unroll
      for (int c = 0; c < C; ++c) a.ubar[(n * DOUT + o) * C + c] = ub[o][c];
  }
};

namespace {
template <class F>
hipError_t seg_by_kind(int kind, F &&f) {
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
}  // namespace

hipError_t launch_seg_loss(int kind, const SegPack &sp, const float *u_save, const float *r_save, const float *x,
                           int64_t N_pad, float *part, float *seg_loss, float *loss, hipStream_t st) {
  hipError_t e = seg_by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    return launch_body<KSegLoss<PDE>>({sp, u_save, r_save, x, N_pad, part}, dim3((unsigned)sp.blk_start[sp.n]), 0,
                                      st);
  });
  if (e != hipSuccess) return e;
  return launch_body<KSegReduce>({sp, part, seg_loss, loss}, dim3(1), 0, st);
}

hipError_t launch_seg_adj(int kind, const SegPack &sp, const float *u_save, const float *r_save, const float *x,
                          int64_t N_pad, Coef k, float *ubar, hipStream_t st) {
  return seg_by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    return launch_body<KSegAdj<PDE>>({sp, u_save, r_save, x, N_pad, k, ubar},
                                     dim3((unsigned)((N_pad + 255) / 256)), 0, st);
  });
}

}  // namespace pj
