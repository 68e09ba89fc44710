// Modified MLP with a periodic input embedding: the network of the paper's
// Kuramoto-Sivashinsky case (Sec. 3.1.1, which takes the architecture from
// earlier PINN training work).  FP32 operands.
//
//   embedding (periodic in x_0, omega = 2 pi / period, M harmonics; the other
//   inputs pass through):
//     e = (x_1 .. x_{d-1}, cos(omega x_0), sin(omega x_0), .., cos(M omega x_0), sin(M omega x_0))
//   encoders  U = tanh(W_U e + b_U),  V = tanh(W_V e + b_V)
//   layers    h_1 = tanh(W_1 e + b_1);  h_l = U + tanh(W_l h_{l-1} + b_l) (V - U),  l = 2 .. H
//   output    u = W_o h_H + b_o   (the plain path's output kernels)
//
// Jets of the embedding are closed forms (the k-th x_0-derivative of
// cos(f x_0) is f^k cos(f x_0 + k pi / 2)); the gated product's jets follow
// the Leibniz rule along each direction.  Stacks are [points][C][w] FP32.
#include "dev_common.hpp"
#include "group.hpp"
#include "jet_math.hpp"
#include "kernels.hpp"

namespace pj {

namespace {

constexpr float kBinom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};

// Jets of the elementwise product p q: (pq)_k = sum_j binom(k, j) p_j q_{k-j}
// along each chain (channel at(d, 0) is the value), and for a mixed channel
// (pq)_ij = p_ij q + p_i q_j + p_j q_i + p q_ij.
template <class CH>
__device__ __forceinline__ void jet_product(const float (&p)[CH::C], const float (&q)[CH::C], float (&o)[CH::C]) {
  o[0] = p[0] * q[0];
#pragma unroll
  for (int d = 0; d < CH::NDIR; ++d)
#pragma unroll
    for (int k = 1; k <= CH::MAXK; ++k)
      if (k <= CH::K(d)) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j <= k; ++j) s += kBinom[k][j] * p[CH::at(d, j)] * q[CH::at(d, k - j)];
        o[CH::at(d, k)] = s;
      }
#pragma unroll
  for (int m = 0; m < CH::NMIX; ++m) {
    const int cm = CH::mix(m, 0), ci = CH::mix(m, 1), cj = CH::mix(m, 2);
    o[cm] = p[cm] * q[0] + p[ci] * q[cj] + p[cj] * q[ci] + p[0] * q[cm];
  }
}

// Adjoint of jet_product: pb += d<ob, pq>/dp, qb += d<ob, pq>/dq.
template <class CH>
__device__ __forceinline__ void jet_product_adjoint(const float (&p)[CH::C], const float (&q)[CH::C],
                                                    const float (&ob)[CH::C], float (&pb)[CH::C],
                                                    float (&qb)[CH::C]) {
  pb[0] += ob[0] * q[0];
  qb[0] += ob[0] * p[0];
#pragma unroll
  for (int d = 0; d < CH::NDIR; ++d)
#pragma unroll
    for (int k = 1; k <= CH::MAXK; ++k)
      if (k <= CH::K(d)) {
        const float g = ob[CH::at(d, k)];
#pragma unroll
        for (int j = 0; j <= k; ++j) {
          const int cp = CH::at(d, j), cq = CH::at(d, k - j);
          pb[cp] += kBinom[k][j] * q[cq] * g;
          qb[cq] += kBinom[k][j] * p[cp] * g;
        }
      }
#pragma unroll
  for (int m = 0; m < CH::NMIX; ++m) {
    const int cm = CH::mix(m, 0), ci = CH::mix(m, 1), cj = CH::mix(m, 2);
    const float g = ob[cm];
    pb[cm] += g * q[0];
    qb[0] += g * p[cm];
    pb[ci] += g * q[cj];
    qb[cj] += g * p[ci];
    pb[cj] += g * q[ci];
    qb[ci] += g * p[cj];
    pb[0] += g * q[cm];
    qb[cm] += g * p[0];
  }
}

// The activation jet from the saved state (s = tanh z_0, z_1 .. z_{C-1}):
// the same arithmetic as jet_forward on the FP32 path.
template <class CH>
__device__ __forceinline__ void jet_from_state(float s, const float (&zs)[CH::C], float (&a)[CH::C]) {
  const TanhDerivs t = tanh_derivs<CH::MAXK>(s, (1.f - s) * (1.f + s));
  a[0] = s;
#pragma unroll
  for (int d = 0; d < CH::NDIR; ++d) {
    const int K = CH::K(d);
    const float z1 = zs[CH::at(d, 1)];
    a[CH::at(d, 1)] = t.s1 * z1;
    if (K >= 2) {
      const float z2 = zs[CH::at(d, 2)];
      a[CH::at(d, 2)] = t.s2 * z1 * z1 + t.s1 * z2;
      if (K >= 3) {
        const float z3 = zs[CH::at(d, 3)];
        a[CH::at(d, 3)] = t.s3 * z1 * z1 * z1 + 3.f * t.s2 * z1 * z2 + t.s1 * z3;
        if (K >= 4) {
          const float z4 = zs[CH::at(d, 4)];
          a[CH::at(d, 4)] = t.s4 * (z1 * z1) * (z1 * z1) + 6.f * t.s3 * z1 * z1 * z2 +
                            t.s2 * (3.f * z2 * z2 + 4.f * z1 * z3) + t.s1 * z4;
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < CH::NMIX; ++m)
    a[CH::mix(m, 0)] = t.s2 * zs[CH::mix(m, 1)] * zs[CH::mix(m, 2)] + t.s1 * zs[CH::mix(m, 0)];
}

// Jets of the embedding at one point: e[c][q], q < DE.  Inputs 1 .. DIN-1
// pass through; harmonic m of x_0 is the pair (cos, sin)(m omega x_0), whose
// k-th derivative along x_0 is (m omega)^k times the pair rotated by k
// quarter turns.
template <class CH, int MAXDE>
__device__ __forceinline__ void embed_jets(const float *xp, int M, float omega, float (&e)[CH::C][MAXDE]) {
  constexpr int C = CH::C, DIN = CH::DIN;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < MAXDE; ++q) e[c][q] = 0.f;
#pragma unroll
  for (int q = 1; q < DIN; ++q) e[0][q - 1] = xp[q];
#pragma unroll
  for (int d = 0; d < CH::NDIR; ++d)
    if (CH::in(d) >= 1) e[CH::at(d, 1)][CH::in(d) - 1] = 1.f;  // d x_i / d x_i
  const float x0 = xp[0];
  for (int m = 1; m <= M; ++m) {
    const float f = (float)m * omega;
    float sn, cs;
    sincosf(f * x0, &sn, &cs);
    const int q = DIN - 1 + 2 * (m - 1);
    e[0][q] = cs;
    e[0][q + 1] = sn;
#pragma unroll
    for (int d = 0; d < CH::NDIR; ++d)
      if (CH::in(d) == 0) {
        float amp = 1.f;
#pragma unroll
        for (int k = 1; k <= CH::MAXK; ++k)
          if (k <= CH::K(d)) {
            amp *= f;
            // rotate (cos, sin) by k quarter turns: (cos, sin) -> (-sin, cos) -> ...
            const int r = k & 3;
            const float c0 = r == 0 ? cs : (r == 1 ? -sn : (r == 2 ? -cs : sn));
            const float s0 = r == 0 ? sn : (r == 1 ? cs : (r == 2 ? -sn : -cs));
            e[CH::at(d, k)][q] = amp * c0;
            e[CH::at(d, k)][q + 1] = amp * s0;
          }
      }
  }
}

// z = W e (+ b on the value), W of shape (w, de), for neuron j.
template <class CH, int MAXDE>
__device__ __forceinline__ void embed_affine(const float (&e)[CH::C][MAXDE], int de, const float *W, const float *b,
                                             int j, float (&z)[CH::C]) {
#pragma unroll
  for (int c = 0; c < CH::C; ++c) z[c] = c == 0 ? b[j] : 0.f;
  for (int q = 0; q < de; ++q) {
    const float wq = W[j * de + q];
#pragma unroll
    for (int c = 0; c < CH::C; ++c) z[c] += wq * e[c][q];
  }
}

}  // namespace

// Encoders and the first hidden layer: U, V, h_1 at every (point, neuron).
template <class CH>
struct KModEnc {
  static constexpr int NT = 256;
  struct Args {
    ModArgs m;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const ModArgs &a = a_.m;
    constexpr int C = CH::C, DIN = CH::DIN;
    const int64_t t = (int64_t)vb.x * NT + threadIdx.x;
    if (t >= a.N_pad * a.w) return;
    const int64_t n = t / a.w;
    const int j = (int)(t - n * a.w);
    float xp[DIN];
#pragma unroll
    for (int i = 0; i < DIN; ++i) xp[i] = n < a.N ? a.x[n * DIN + i] : 0.f;
    float e[C][kModMaxDe];
    embed_jets<CH, kModMaxDe>(xp, a.M, a.omega, e);
    const int64_t base = n * C * a.w + j;
    const float *Ws[3] = {a.WU, a.WV, a.W1};
    const float *bs[3] = {a.bU, a.bV, a.b1};
    float *outs[3] = {a.U, a.V, a.h1};
#pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
      float z[C], act[C], s;
      embed_affine<CH, kModMaxDe>(e, a.de, Ws[layer], bs[layer], j, z);
      jet_forward<CH, false>(z, act, s);
#pragma unroll
      for (int c = 0; c < C; ++c) outs[layer][base + c * a.w] = act[c];
    }
  }
};

// Gated hidden layer l >= 2: z = W_l h_{l-1} (+ b on the value) on MFMA,
// Z = tanh jet(z), h_l = U + Z (V - U) with the Leibniz rule; saves the state
// (tanh z_0, z_1 .. z_{C-1}) for the adjoint.  Tiling as the plain layer
// kernel: 4 waves, 32 neurons x 32 points per wave.
template <class CH>
struct KModLayer {
  static constexpr int NT = 256;
  struct Args {
    const float *h_in, *W, *b, *U, *V;
    float *h_out, *S_out;
    int w;
  };
  static __device__ __forceinline__ void run(const Args &a, VBlock vb) {
    constexpr int C = CH::C, WJ = 2, WN = 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wj = wave % WJ, wn = wave / WJ;
    const int m0 = (vb.y * WJ + wj) * 32;
    const int64_t n0 = ((int64_t)vb.x * WN + wn) * 32;
    const int r = lane & 15, g = lane >> 4;
    const int w = a.w;
    const int64_t ps = (int64_t)C * w;
    f32x4 acc[2][2][C];
    zero_acc_mod<C, 2>(acc);
    stacked_gemm_mod<C, 2>(acc, a.W, a.h_in, m0, n0, w, lane);
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int64_t n = n0 + 16 * nt + r;
        const int mb = m0 + 16 * jt + 4 * g;
        float out[4][C], sv[4][C];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float z[C], act[C], s, u[C], dv[C], pr[C];
#pragma unroll
          for (int c = 0; c < C; ++c) z[c] = acc[jt][nt][c][i];
          z[0] += a.b[mb + i];
          jet_forward<CH, false>(z, act, s);
#pragma unroll
          for (int c = 0; c < C; ++c) {
            u[c] = a.U[n * ps + c * w + mb + i];
            dv[c] = a.V[n * ps + c * w + mb + i] - u[c];
          }
          jet_product<CH>(act, dv, pr);
#pragma unroll
          for (int c = 0; c < C; ++c) {
            out[i][c] = u[c] + pr[c];
            sv[i][c] = c == 0 ? s : z[c];
          }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
          store4(a.h_out + n * ps + c * w + mb, out[0][c], out[1][c], out[2][c], out[3][c]);
          store4(a.S_out + n * ps + c * w + mb, sv[0][c], sv[1][c], sv[2][c], sv[3][c]);
        }
      }
  }

  template <int CC, int NTN>
  static __device__ __forceinline__ void zero_acc_mod(f32x4 (&acc)[2][NTN][CC]) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < NTN; ++y)
#pragma unroll
        for (int c = 0; c < CC; ++c) acc[x][y][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // acc[jt][nt][c] += sum_k W[m0 + 16 jt + r][k] B[n0 + 16 nt + r][c][k]
  template <int CC, int NTN>
  static __device__ __forceinline__ void stacked_gemm_mod(f32x4 (&acc)[2][NTN][CC], const float *W, const float *B,
                                                          int m0, int64_t n0, int w, int lane) {
    using M = Mma<float>;
    const int r = lane & 15, g = lane >> 4;
    const int64_t ps = (int64_t)CC * w;
    const float *wp0 = W + (int64_t)(m0 + r) * w + 8 * g;
    const float *wp1 = wp0 + (int64_t)16 * w;
    const float *bp = B + (n0 + r) * ps + 8 * g;
    for (int k = 0; k < w; k += 32) {
      const M::frag a0 = M::load(wp0 + k);
      const M::frag a1 = M::load(wp1 + k);
#pragma unroll
      for (int c = 0; c < CC; ++c)
#pragma unroll
        for (int nt = 0; nt < NTN; ++nt) {
          const M::frag bf = M::load(bp + nt * 16 * ps + c * w + k);
          M::mma(acc[0][nt][c], a0, bf);
          M::mma(acc[1][nt][c], a1, bf);
        }
    }
  }
};

// Cotangent of the stack below a gated layer: hbar[n][c][k] = sum_j W_l[j][k]
// zbar_l[n][c][j], with WT = W_l^T; a plain stacked GEMM (no epilogue).
template <class CH>
struct KModAbar {
  static constexpr int NT = 256;
  struct Args {
    const float *WT, *zbar;
    float *hbar;
    int w;
  };
  static __device__ __forceinline__ void run(const Args &a, VBlock vb) {
    constexpr int C = CH::C, WJ = 2, WN = 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wj = wave % WJ, wn = wave / WJ;
    const int m0 = (vb.y * WJ + wj) * 32;
    const int64_t n0 = ((int64_t)vb.x * WN + wn) * 32;
    const int r = lane & 15, g = lane >> 4;
    const int64_t ps = (int64_t)C * a.w;
    f32x4 acc[2][2][C];
    KModLayer<CH>::template zero_acc_mod<C, 2>(acc);
    KModLayer<CH>::template stacked_gemm_mod<C, 2>(acc, a.WT, a.zbar, m0, n0, a.w, lane);
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int64_t n = n0 + 16 * nt + r;
        const int mb = m0 + 16 * jt + 4 * g;
#pragma unroll
        for (int c = 0; c < C; ++c)
          store4(a.hbar + n * ps + c * a.w + mb, acc[jt][nt][c][0], acc[jt][nt][c][1], acc[jt][nt][c][2],
                 acc[jt][nt][c][3]);
      }
  }
};

// Adjoint of gated layer l at one (point, neuron): from hbar_l (or, for the
// top layer, from the output cotangent ubar through W_o), accumulate Ubar and
// Vbar (set them on the top layer) and produce zbar_l.
//   h = U + Z D, D = V - U:  Ubar += hbar - Dbar,  Vbar += Dbar,
//   (Zbar, Dbar) = product adjoint,  zbar = tanh jet adjoint(Zbar).
template <class PDE, bool TOP>
struct KModGateBwd {
  static constexpr int NT = 256;
  struct Args {
    const float *hbar, *ubar, *Wo, *S, *U, *V;
    float *Ubar, *Vbar, *zbar;
    int64_t N_pad;
    int w;
  };
  static __device__ __forceinline__ void run(const Args &a, VBlock vb) {
    using CH = typename PDE::CH;
    constexpr int C = CH::C, DOUT = PDE::DOUT;
    const int64_t t = (int64_t)vb.x * NT + threadIdx.x;
    if (t >= a.N_pad * a.w) return;
    const int64_t n = t / a.w;
    const int j = (int)(t - n * a.w);
    const int64_t base = n * C * a.w + j;
    float hb[C], u[C], dv[C], zs[C], Z[C], Zb[C], Db[C], zb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if constexpr (TOP) {
        float s = 0.f;
#pragma unroll
        for (int o = 0; o < DOUT; ++o) s += a.Wo[o * a.w + j] * a.ubar[(n * DOUT + o) * C + c];
        hb[c] = s;
      } else {
        hb[c] = a.hbar[base + c * a.w];
      }
      u[c] = a.U[base + c * a.w];
      dv[c] = a.V[base + c * a.w] - u[c];
      zs[c] = a.S[base + c * a.w];
      Zb[c] = 0.f;
      Db[c] = 0.f;
    }
    const float s = zs[0];
    jet_from_state<CH>(s, zs, Z);
    jet_product_adjoint<CH>(Z, dv, hb, Zb, Db);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float ub = hb[c] - Db[c];
      if constexpr (TOP) {
        a.Ubar[base + c * a.w] = ub;
        a.Vbar[base + c * a.w] = Db[c];
      } else {
        a.Ubar[base + c * a.w] += ub;
        a.Vbar[base + c * a.w] += Db[c];
      }
    }
    jet_adjoint<CH>(Zb, s, (1.f - s) * (1.f + s), zs, zb);
#pragma unroll
    for (int c = 0; c < C; ++c) a.zbar[base + c * a.w] = zb[c];
  }
};

// Adjoint of the encoders and the first layer at one (point, neuron): their
// pre-activations are recomputed from the embedding; zbar of h_1, U and V
// into zb3[0..2], and the embedding jets of the point into E (by neuron 0).
template <class CH>
struct KModEncBwd {
  static constexpr int NT = 256;
  struct Args {
    ModArgs m;
    const float *h1bar, *Ubar, *Vbar;
    float *zb3, *E;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const ModArgs &a = a_.m;
    constexpr int C = CH::C, DIN = CH::DIN;
    const int64_t t = (int64_t)vb.x * NT + threadIdx.x;
    if (t >= a.N_pad * a.w) return;
    const int64_t n = t / a.w;
    const int j = (int)(t - n * a.w);
    float xp[DIN];
#pragma unroll
    for (int i = 0; i < DIN; ++i) xp[i] = n < a.N ? a.x[n * DIN + i] : 0.f;
    float e[C][kModMaxDe];
    embed_jets<CH, kModMaxDe>(xp, a.M, a.omega, e);
    if (j == 0)
      for (int c = 0; c < C; ++c)
        for (int q = 0; q < a.de; ++q) a_.E[(n * C + c) * a.de + q] = e[c][q];
    const int64_t base = n * C * a.w + j;
    const int64_t stack = a.N_pad * C * a.w;
    const float *Ws[3] = {a.W1, a.WU, a.WV};
    const float *bs[3] = {a.b1, a.bU, a.bV};
    const float *bars[3] = {a_.h1bar, a_.Ubar, a_.Vbar};
#pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
      float z[C], ab[C], zb[C];
      embed_affine<CH, kModMaxDe>(e, a.de, Ws[layer], bs[layer], j, z);
      const TanhS ts = tanh_eval<false>(z[0]);
#pragma unroll
      for (int c = 0; c < C; ++c) ab[c] = bars[layer][base + c * a.w];
      jet_adjoint<CH>(ab, ts.s, ts.s1, z, zb);
#pragma unroll
      for (int c = 0; c < C; ++c) a_.zb3[layer * stack + base + c * a.w] = zb[c];
    }
  }
};

// Partial sums of the weight gradients of the three embedding-fed layers:
// part[e][chunk][w*de + w] = sum over the chunk's points and the channels of
// zbar_e[n][c][j] * E[n][c][q] (q < de; q = de: the value channel alone, db).
template <class CH>
struct KModDwEnc {
  static constexpr int NT = 256;
  struct Args {
    const float *zb3, *E;
    float *part;
    int64_t N_pad, pts_per_chunk;
    int w, de, n_chunks;
  };
  static __device__ __forceinline__ void run(const Args &a, VBlock vb) {
    constexpr int C = CH::C;
    const int layer = vb.y, chunk = vb.x;
    const int64_t stack = a.N_pad * C * a.w;
    const float *zb = a.zb3 + layer * stack;
    const int64_t stride = (int64_t)a.w * a.de + a.w;
    float *pp = a.part + ((int64_t)layer * a.n_chunks + chunk) * stride;
    const int64_t nb = (int64_t)chunk * a.pts_per_chunk;
    const int64_t ne = nb + a.pts_per_chunk < a.N_pad ? nb + a.pts_per_chunk : a.N_pad;
    for (int q = threadIdx.x; q < stride; q += NT) {
      const bool is_b = q >= a.w * a.de;
      const int j = is_b ? q - a.w * a.de : q / a.de, i = is_b ? 0 : q - (q / a.de) * a.de;
      float s = 0.f;
      for (int64_t n = nb; n < ne; ++n) {
        if (is_b) {
          s += zb[n * C * a.w + j];
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) s += zb[(n * C + c) * a.w + j] * a.E[(n * C + c) * a.de + i];
        }
      }
      pp[q] = s;
    }
  }
};

namespace {
template <class F>
hipError_t mod_by_kind(int kind, F &&f) {
  switch (kind) {
    case K_KS: return f(PdeKS{});
    case K_BURGERS: return f(PdeBurgers{});
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

bool mod_kind_supported(int kind) { return kind == K_KS || kind == K_BURGERS; }

hipError_t launch_mod_enc(int kind, const ModArgs &m, hipStream_t st) {
  return mod_by_kind(kind, [&](auto pde) {
    using CH = typename decltype(pde)::CH;
    return launch_body<KModEnc<CH>>({m}, dim3((unsigned)((m.N_pad * m.w + 255) / 256)), 0, st);
  });
}

hipError_t launch_mod_layer(int kind, const float *h_in, const float *W, const float *b, const float *U,
                            const float *V, float *h_out, float *S_out, int64_t N_pad, int w, hipStream_t st) {
  return mod_by_kind(kind, [&](auto pde) {
    using CH = typename decltype(pde)::CH;
    return launch_body<KModLayer<CH>>({h_in, W, b, U, V, h_out, S_out, w},
                                      dim3((unsigned)(N_pad / 64), (unsigned)(w / 64)), 0, st);
  });
}

hipError_t launch_mod_abar(int kind, const float *WT, const float *zbar, float *hbar, int64_t N_pad, int w,
                           hipStream_t st) {
  return mod_by_kind(kind, [&](auto pde) {
    using CH = typename decltype(pde)::CH;
    return launch_body<KModAbar<CH>>({WT, zbar, hbar, w}, dim3((unsigned)(N_pad / 64), (unsigned)(w / 64)), 0,
                                     st);
  });
}

hipError_t launch_mod_gate_bwd(int kind, bool top, const float *hbar, const float *ubar, const float *Wo,
                               const float *S, const float *U, const float *V, float *Ubar, float *Vbar,
                               float *zbar, int64_t N_pad, int w, hipStream_t st) {
  return mod_by_kind(kind, [&](auto pde) {
    using PDE = decltype(pde);
    const dim3 grid((unsigned)((N_pad * w + 255) / 256));
    if (top)
      return launch_body<KModGateBwd<PDE, true>>({hbar, ubar, Wo, S, U, V, Ubar, Vbar, zbar, N_pad, w}, grid, 0,
                                                 st);
    return launch_body<KModGateBwd<PDE, false>>({hbar, ubar, Wo, S, U, V, Ubar, Vbar, zbar, N_pad, w}, grid, 0,
                                                st);
  });
}

hipError_t launch_mod_enc_bwd(int kind, const ModArgs &m, const float *h1bar, const float *Ubar, const float *Vbar,
                              float *zb3, float *E, hipStream_t st) {
  return mod_by_kind(kind, [&](auto pde) {
    using CH = typename decltype(pde)::CH;
    return launch_body<KModEncBwd<CH>>({m, h1bar, Ubar, Vbar, zb3, E},
                                       dim3((unsigned)((m.N_pad * m.w + 255) / 256)), 0, st);
  });
}

hipError_t launch_mod_dw_enc(int kind, const float *zb3, const float *E, float *part, int64_t N_pad, int w, int de,
                             int n_chunks, hipStream_t st) {
  return mod_by_kind(kind, [&](auto pde) {
    using CH = typename decltype(pde)::CH;
    const int64_t ppc = (N_pad + n_chunks - 1) / n_chunks;
    return launch_body<KModDwEnc<CH>>({zb3, E, part, N_pad, ppc, w, de, n_chunks}, dim3((unsigned)n_chunks, 3u),
                                      0, st);
  });
}

}  // namespace pj
