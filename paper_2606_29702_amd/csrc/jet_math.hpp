// Partial-jet arithmetic for one (neuron, point): the activation jet (Eq. 2-3
// and the pure-derivative recursion to order 4 of Sec. 2.2), its adjoint, and
// the PDE residuals with their adjoints.  FP32 throughout.
#pragma once
#include <hip/hip_runtime.h>

namespace pj {

// ---------------------------------------------------------------------------
// Channel sets.  Channel 0 is the value.  The derivative channels form one
// chain per input direction: at(d, k) is the channel holding the order-k pure
// derivative along chain d, whose input coordinate is in(d).
// ---------------------------------------------------------------------------

// Burgers, inputs (x, t): u, u_t, u_x, u_xx
struct ChBurgers {
  static constexpr int NMIX = 0;  // no mixed channels
  __host__ __device__ static constexpr int mix(int, int) { return 0; }
  static constexpr int C = 4, NDIR = 2, MAXK = 2, DIN = 2;
  __host__ __device__ static constexpr int K(int d) { return d == 0 ? 2 : 1; }
  __host__ __device__ static constexpr int at(int d, int k) {
    return k == 0 ? 0 : (d == 0 ? (k == 1 ? 2 : 3) : 1);
  }
  __host__ __device__ static constexpr int in(int d) { return d; }
};

// Navier-Stokes, inputs (x, y): value, d/dx, d/dy, d2/dx2, d2/dy2
struct ChNS {
  static constexpr int NMIX = 0;  // no mixed channels
  __host__ __device__ static constexpr int mix(int, int) { return 0; }
  static constexpr int C = 5, NDIR = 2, MAXK = 2, DIN = 2;
  __host__ __device__ static constexpr int K(int) { return 2; }
  __host__ __device__ static constexpr int at(int d, int k) {
    return k == 0 ? 0 : (k == 1 ? 1 + d : 3 + d);
  }
  __host__ __device__ static constexpr int in(int d) { return d; }
};

// Kuramoto-Sivashinsky, inputs (x, t): u, u_t, u_x, u_xx, u_xxx, u_xxxx
struct ChKS {
  static constexpr int NMIX = 0;  // no mixed channels
  __host__ __device__ static constexpr int mix(int, int) { return 0; }
  static constexpr int C = 6, NDIR = 2, MAXK = 4, DIN = 2;
  __host__ __device__ static constexpr int K(int d) { return d == 0 ? 4 : 1; }
  __host__ __device__ static constexpr int at(int d, int k) {
    return k == 0 ? 0 : (d == 0 ? 1 + k : 1);
  }
  __host__ __device__ static constexpr int in(int d) { return d; }
};

// Heat, inputs (x, y, z, t): u, u_t, u_x, u_y, u_z, u_xx, u_yy, u_zz
struct ChHeat {
  static constexpr int NMIX = 0;  // no mixed channels
  __host__ __device__ static constexpr int mix(int, int) { return 0; }
  static constexpr int C = 8, NDIR = 4, MAXK = 2, DIN = 4;
  __host__ __device__ static constexpr int K(int d) { return d == 3 ? 1 : 2; }
  __host__ __device__ static constexpr int at(int d, int k) {
    return k == 0 ? 0 : (d == 3 ? 1 : (k == 1 ? 2 + d : 5 + d));
  }
  __host__ __device__ static constexpr int in(int d) { return d; }
};

// Value only, inputs (x, t): the channel set of the initial and boundary
// data terms, which need no derivative.
struct ChValue2 {
  static constexpr int NMIX = 0;
  __host__ __device__ static constexpr int mix(int, int) { return 0; }
  static constexpr int C = 1, NDIR = 0, MAXK = 0, DIN = 2;
  __host__ __device__ static constexpr int K(int) { return 0; }
  __host__ __device__ static constexpr int at(int, int) { return 0; }
  __host__ __device__ static constexpr int in(int d) { return d; }
};

// Anisotropic test operator, inputs (x, y): u, u_x, u_y, u_xx, u_yy, u_xy.
// The last channel is a mixed second derivative (Eq. 3 with i != j): mix(m, 0)
// is its channel, mix(m, 1) and mix(m, 2) the first-order channels it pairs.
struct ChAniso {
  static constexpr int C = 6, NDIR = 2, MAXK = 2, DIN = 2;
  static constexpr int NMIX = 1;
  __host__ __device__ static constexpr int K(int) { return 2; }
  __host__ __device__ static constexpr int at(int d, int k) {
    return k == 0 ? 0 : (k == 1 ? 1 + d : 3 + d);
  }
  __host__ __device__ static constexpr int in(int d) { return d; }
  __host__ __device__ static constexpr int mix(int, int q) { return q == 0 ? 5 : (q == 1 ? 1 : 2); }
};

// tanh and its derivatives as polynomials in s = tanh(z), from ds/dz = 1 - s^2.
struct TanhDerivs {
  float s, s1, s2, s3, s4, s5;
};

// s = tanh(z) and s1 = 1 - s^2.
//  FAST (16-bit operand paths): from the identity tanh z = 1 - 2 / (e + 1),
//    e = exp(2z), with the hardware base-2 exponential and reciprocal; then
//    1 - s = 2 / (e + 1) and 1 + s = 2e / (e + 1), so 1 - s^2 = 4 e / (e + 1)^2
//    carries no cancellation for saturated neurons.  Absolute error a few
//    1e-7, far below the BF16/FP16 operand rounding.
//  otherwise (FP32 path): the device library tanhf, and (1 - s)(1 + s).
struct TanhS {
  float s, s1;
};
template <bool FAST>
__device__ __forceinline__ TanhS tanh_eval(float z) {
  TanhS t;
  if constexpr (FAST) {
    const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);  // exp(2z) = 2^(2 z log2 e)
    const float q = __builtin_amdgcn_rcpf(e + 1.f);
    t.s = 1.f - 2.f * q;
    t.s1 = e < 3.0e38f ? 4.f * (e * q) * q : 0.f;
  } else {
    t.s = tanhf(z);
    t.s1 = (1.f - t.s) * (1.f + t.s);
  }
  return t;
}

// Higher derivatives from s and s1 = 1 - s^2.
template <int MAXD>
__device__ __forceinline__ TanhDerivs tanh_derivs(float s, float s1) {
  TanhDerivs t;
  const float ss = s * s;
  t.s = s;
  t.s1 = s1;
  t.s2 = -2.f * s * s1;
  t.s3 = MAXD >= 3 ? s1 * (6.f * ss - 2.f) : 0.f;
  t.s4 = MAXD >= 4 ? s * s1 * (16.f - 24.f * ss) : 0.f;
  t.s5 = MAXD >= 5 ? s1 * (16.f + ss * (120.f * ss - 120.f)) : 0.f;
  return t;
}

// Activation jet from s = tanh(z_0), s1 = 1 - s^2 and the derivative
// channels z_c (c >= 1; z[0] is not read) -> a.
template <class CH>
__device__ __forceinline__ void jet_forward_from(float s, float s1, const float (&z)[CH::C], float (&a)[CH::C]) {
  const TanhDerivs t = tanh_derivs<CH::MAXK>(s, s1);
  a[0] = t.s;
#pragma unroll
  for (int d = 0; d < CH::NDIR; ++d) {
    const int K = CH::K(d);
    const float z1 = z[CH::at(d, 1)];
    a[CH::at(d, 1)] = t.s1 * z1;
    if (K >= 2) {
      const float z2 = z[CH::at(d, 2)];
      a[CH::at(d, 2)] = t.s2 * z1 * z1 + t.s1 * z2;
      if (K >= 3) {
        const float z3 = z[CH::at(d, 3)];
        a[CH::at(d, 3)] = t.s3 * z1 * z1 * z1 + 3.f * t.s2 * z1 * z2 + t.s1 * z3;
        if (K >= 4) {
          const float z4 = z[CH::at(d, 4)];
          a[CH::at(d, 4)] = t.s4 * (z1 * z1) * (z1 * z1) + 6.f * t.s3 * z1 * z1 * z2 +
                            t.s2 * (3.f * z2 * z2 + 4.f * z1 * z3) + t.s1 * z4;
        }
      }
    }
  }
  // mixed second derivatives: a_ij = s'' z_i z_j + s' z_ij
#pragma unroll
  for (int m = 0; m < CH::NMIX; ++m)
    a[CH::mix(m, 0)] = t.s2 * z[CH::mix(m, 1)] * z[CH::mix(m, 2)] + t.s1 * z[CH::mix(m, 0)];
}

// Activation jet: z (pre-activation channels, bias already in z[0]) -> a.
template <class CH, bool FAST = false>
__device__ __forceinline__ void jet_forward(const float (&z)[CH::C], float (&a)[CH::C], float &s_out) {
  const TanhS ts = tanh_eval<FAST>(z[0]);
  s_out = ts.s;
  jet_forward_from<CH>(ts.s, ts.s1, z, a);
}

// Adjoint of jet_forward.  Inputs: the cotangent ab of the activation jet,
// s = tanh(z_0), s1 = 1 - s^2 and the derivative channels zs[c] = z_c (c >= 1)
// of the forward pass.  Output: zb, the cotangent of the pre-activation channels.
// Each a_k of a chain depends on z_1..z_k directly and on z_0 through the
// tanh derivatives (d s_j / d z_0 = s_{j+1}).
template <class CH>
__device__ __forceinline__ void jet_adjoint(const float (&ab)[CH::C], float s, float s1, const float (&zs)[CH::C],
                                            float (&zb)[CH::C]) {
  const TanhDerivs t = tanh_derivs<CH::MAXK + 1>(s, s1);
  float zb0 = t.s1 * ab[0];
#pragma unroll
  for (int d = 0; d < CH::NDIR; ++d) {
    const int K = CH::K(d);
    const int c1 = CH::at(d, 1);
    const float z1 = zs[c1];
    const float ab1 = ab[c1];
    float g1 = t.s1 * ab1;
    zb0 += t.s2 * z1 * ab1;
    if (K >= 2) {
      const int c2 = CH::at(d, 2);
      const float z2 = zs[c2], ab2 = ab[c2];
      float g2 = t.s1 * ab2;
      g1 += 2.f * t.s2 * z1 * ab2;
      zb0 += (t.s3 * z1 * z1 + t.s2 * z2) * ab2;
      if (K >= 3) {
        const int c3 = CH::at(d, 3);
        const float z3 = zs[c3], ab3 = ab[c3];
        float g3 = t.s1 * ab3;
        g2 += 3.f * t.s2 * z1 * ab3;
        g1 += (3.f * t.s3 * z1 * z1 + 3.f * t.s2 * z2) * ab3;
        zb0 += (t.s4 * z1 * z1 * z1 + 3.f * t.s3 * z1 * z2 + t.s2 * z3) * ab3;
        if (K >= 4) {
          const int c4 = CH::at(d, 4);
          const float z4 = zs[c4], ab4 = ab[c4];
          zb[c4] = t.s1 * ab4;
          g3 += 4.f * t.s2 * z1 * ab4;
          g2 += (6.f * t.s3 * z1 * z1 + 6.f * t.s2 * z2) * ab4;
          g1 += (4.f * t.s4 * z1 * z1 * z1 + 12.f * t.s3 * z1 * z2 + 4.f * t.s2 * z3) * ab4;
          zb0 += (t.s5 * (z1 * z1) * (z1 * z1) + 6.f * t.s4 * z1 * z1 * z2 +
                  t.s3 * (3.f * z2 * z2 + 4.f * z1 * z3) + t.s2 * z4) * ab4;
        }
        zb[c3] = g3;
      }
      zb[c2] = g2;
    }
    zb[c1] = g1;
  }
  // adjoint of a_ij = s''(z_0) z_i z_j + s'(z_0) z_ij
#pragma unroll
  for (int m = 0; m < CH::NMIX; ++m) {
    const int cm = CH::mix(m, 0), ci = CH::mix(m, 1), cj = CH::mix(m, 2);
    const float abm = ab[cm];
    zb0 += (t.s3 * zs[ci] * zs[cj] + t.s2 * zs[cm]) * abm;
    zb[ci] += t.s2 * zs[cj] * abm;
    zb[cj] += t.s2 * zs[ci] * abm;
    zb[cm] = t.s1 * abm;
  }
  zb[0] = zb0;
}

// ---------------------------------------------------------------------------
// PDE residuals.  u[o][c]: output o, channel c.  coef as in the public header.
// ---------------------------------------------------------------------------
struct Coef {
  float c[4];
};

struct PdeBurgers {
  using CH = ChBurgers;
  static constexpr int DOUT = 1, NRES = 1;
  // r = u_t + u u_x - nu u_xx
  __device__ static void residual(const float (&u)[1][4], const float *, const Coef &k, float (&r)[1]) {
    r[0] = u[0][1] + u[0][0] * u[0][2] - k.c[0] * u[0][3];
  }
  __device__ static void adjoint(const float (&u)[1][4], const float (&rb)[1], const Coef &k,
                                 float (&ub)[1][4]) {
    ub[0][0] = rb[0] * u[0][2];
    ub[0][1] = rb[0];
    ub[0][2] = rb[0] * u[0][0];
    ub[0][3] = -k.c[0] * rb[0];
  }
};

struct PdeNS {
  using CH = ChNS;
  static constexpr int DOUT = 3, NRES = 3;
  // outputs (u, v, p); channels value, x, y, xx, yy; Eq. 16 in the order (r_c, r_u, r_v)
  __device__ static void residual(const float (&u)[3][5], const float *, const Coef &k, float (&r)[3]) {
    const float inv_re = 1.f / k.c[0];
    r[0] = u[0][1] + u[1][2];
    r[1] = u[0][0] * u[0][1] + u[1][0] * u[0][2] + u[2][1] - (u[0][3] + u[0][4]) * inv_re;
    r[2] = u[0][0] * u[1][1] + u[1][0] * u[1][2] + u[2][2] - (u[1][3] + u[1][4]) * inv_re;
  }
  __device__ static void adjoint(const float (&u)[3][5], const float (&rb)[3], const Coef &k,
                                 float (&ub)[3][5]) {
    const float inv_re = 1.f / k.c[0];
    const float rc = rb[0], ru = rb[1], rv = rb[2];
    // u: value, x, y, xx, yy
    ub[0][0] = ru * u[0][1] + rv * u[1][1];
    ub[0][1] = rc + ru * u[0][0];
    ub[0][2] = ru * u[1][0];
    ub[0][3] = -ru * inv_re;
    ub[0][4] = -ru * inv_re;
    // v
    ub[1][0] = ru * u[0][2] + rv * u[1][2];
    ub[1][1] = rv * u[0][0];
    ub[1][2] = rc + rv * u[1][0];
    ub[1][3] = -rv * inv_re;
    ub[1][4] = -rv * inv_re;
    // p enters through p_x and p_y only
    ub[2][0] = 0.f;
    ub[2][1] = ru;
    ub[2][2] = rv;
    ub[2][3] = 0.f;
    ub[2][4] = 0.f;
  }
};

struct PdeKS {
  using CH = ChKS;
  static constexpr int DOUT = 1, NRES = 1;
  // r = u_t + alpha u u_x + beta u_xx + gamma u_xxxx
  __device__ static void residual(const float (&u)[1][6], const float *, const Coef &k, float (&r)[1]) {
    r[0] = u[0][1] + k.c[0] * u[0][0] * u[0][2] + k.c[1] * u[0][3] + k.c[2] * u[0][5];
  }
  __device__ static void adjoint(const float (&u)[1][6], const float (&rb)[1], const Coef &k,
                                 float (&ub)[1][6]) {
    ub[0][0] = k.c[0] * rb[0] * u[0][2];
    ub[0][1] = rb[0];
    ub[0][2] = k.c[0] * rb[0] * u[0][0];
    ub[0][3] = k.c[1] * rb[0];
    ub[0][4] = 0.f;
    ub[0][5] = k.c[2] * rb[0];
  }
};

struct PdeHeat {
  using CH = ChHeat;
  static constexpr int DOUT = 1, NRES = 1;
  // r = u_t - kappa (u_xx + u_yy + u_zz) - sin(pi x) sin(pi y) sin(pi z) exp(-t)
  __device__ static void residual(const float (&u)[1][8], const float *x, const Coef &k, float (&r)[1]) {
    const float f = sinpif(x[0]) * sinpif(x[1]) * sinpif(x[2]) * expf(-x[3]);
    r[0] = u[0][1] - k.c[0] * (u[0][5] + u[0][6] + u[0][7]) - f;
  }
  __device__ static void adjoint(const float (&)[1][8], const float (&rb)[1], const Coef &k,
                                 float (&ub)[1][8]) {
    ub[0][0] = 0.f;
    ub[0][1] = rb[0];
    ub[0][2] = 0.f;
    ub[0][3] = 0.f;
    ub[0][4] = 0.f;
    ub[0][5] = -k.c[0] * rb[0];
    ub[0][6] = -k.c[0] * rb[0];
    ub[0][7] = -k.c[0] * rb[0];
  }
};

// Burgers initial and boundary data: r = u - g with g = -sin(pi x), which is
// the initial condition u(x, 0) = -sin(pi x) on t = 0 and vanishes on the
// walls x = +-1 (the points lie on those segments).
struct PdeBurgersBC {
  using CH = ChValue2;
  static constexpr int DOUT = 1, NRES = 1;
  __device__ static void residual(const float (&u)[1][1], const float *x, const Coef &, float (&r)[1]) {
    r[0] = u[0][0] + sinpif(x[0]);
  }
  __device__ static void adjoint(const float (&)[1][1], const float (&rb)[1], const Coef &, float (&ub)[1][1]) {
    ub[0][0] = rb[0];
  }
};

// Anisotropic test operator with a mixed derivative (not one of the paper's
// problems): r = u_xx + 2 c u_xy + u_yy.
struct PdeAniso {
  using CH = ChAniso;
  static constexpr int DOUT = 1, NRES = 1;
  __device__ static void residual(const float (&u)[1][6], const float *, const Coef &k, float (&r)[1]) {
    r[0] = u[0][3] + 2.f * k.c[0] * u[0][5] + u[0][4];
  }
  __device__ static void adjoint(const float (&)[1][6], const float (&rb)[1], const Coef &k, float (&ub)[1][6]) {
    ub[0][0] = 0.f;
    ub[0][1] = 0.f;
    ub[0][2] = 0.f;
    ub[0][3] = rb[0];
    ub[0][4] = rb[0];
    ub[0][5] = 2.f * k.c[0] * rb[0];
  }
};

}  // namespace pj
