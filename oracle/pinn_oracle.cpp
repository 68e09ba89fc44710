/*
 * FP64 CPU oracle: plain per-point partial-jet forward pass, residual, loss and
 * reverse sweep for the parameter gradient.
 *
 * TEST INFRASTRUCTURE ONLY (see pinn_oracle.h).  Deliberately slow and direct:
 * one collocation point at a time, one dot product per (channel, neuron), no
 * blocking or fusion, so that each step can be read against the paper:
 *   - layer affine map and activation:             Eq. 1
 *   - first-order derivative states:                Eq. 2
 *   - second-order (pure) derivative states:        Eq. 3
 *   - higher orders by the same recursion:          Sec. 2.2 (text after Eq. 3);
 *     written here as the univariate Faa di Bruno formula along one direction
 *   - only the states the residual needs:           Sec. 2.2 ("on-demand partial jet")
 *   - residuals: Burgers and KS as in Sec. 3.1.1, Navier-Stokes Eq. 16,
 *     heat u_t - kappa Lap u - f (a workload of this library, not of the paper)
 *   - parameter gradient by reverse-mode differentiation of the scalar loss,
 *     which the paper keeps for training (Sec. 2.2, Sec. 3.1.1).
 */
#include "pinn_oracle.h"

#include <cmath>
#include <complex>
#include <type_traits>
#include <vector>
#include <omp.h>

namespace {

constexpr int kMaxCh = 16;
constexpr int kMaxDir = 8;
constexpr int kMaxOrder = 4;
constexpr int64_t kChunk = 64; /* points per deterministic partial sum */

using cplx = std::complex<double>;

struct ChannelSet {
  int C = 0;
  int dir[kMaxCh];
  int ord[kMaxCh];
  /* at[i][k]: channel index of d^k/dx_i^k, or -1.  at[i][0] = 0 (the value). */
  int at[kMaxDir][kMaxOrder + 1];
  int top[kMaxDir]; /* highest order present along direction i */
  /* mixed second-order channels d^2/dx_i dx_j (i < j), Eq. 3 with i != j:
     channel mix_c[m] with first-order partners mix_ci[m], mix_cj[m] */
  int n_mix = 0;
  int mix_c[kMaxCh], mix_ci[kMaxCh], mix_cj[kMaxCh];
};

int build_channels(int n_ch, const int *ch_dir, const int *ch_ord, int d_in, ChannelSet *cs) {
  if (n_ch < 1 || n_ch > kMaxCh || d_in < 1 || d_in > kMaxDir) return -1;
  cs->C = n_ch;
  for (int i = 0; i < kMaxDir; ++i) {
    cs->top[i] = 0;
    cs->at[i][0] = 0;
    for (int k = 1; k <= kMaxOrder; ++k) cs->at[i][k] = -1;
  }
  if (ch_ord[0] != 0) return -1;
  cs->dir[0] = -1;
  cs->ord[0] = 0;
  cs->n_mix = 0;
  int mix_i[kMaxCh], mix_j[kMaxCh];
  for (int c = 1; c < n_ch; ++c) {
    int i = ch_dir[c], k = ch_ord[c];
    if (k == ORC_MIXED2) { /* d^2 / dx_i dx_j, i < j, coded as ch_dir = i * 8 + j */
      const int mi = i / 8, mj = i % 8;
      if (i < 0 || mi >= mj || mj >= d_in) return -1;
      for (int m = 0; m < cs->n_mix; ++m)
        if (mix_i[m] == mi && mix_j[m] == mj) return -1; /* duplicate */
      cs->dir[c] = -1;
      cs->ord[c] = 2;
      mix_i[cs->n_mix] = mi;
      mix_j[cs->n_mix] = mj;
      cs->mix_c[cs->n_mix++] = c;
      continue;
    }
    if (i < 0 || i >= d_in || k < 1 || k > kMaxOrder) return -1;
    if (cs->at[i][k] != -1) return -1; /* duplicate */
    cs->dir[c] = i;
    cs->ord[c] = k;
    cs->at[i][k] = c;
  }
  for (int i = 0; i < d_in; ++i) {
    int k = 0;
    while (k + 1 <= kMaxOrder && cs->at[i][k + 1] >= 0) ++k;
    cs->top[i] = k;
    for (int kk = k + 1; kk <= kMaxOrder; ++kk)
      if (cs->at[i][kk] >= 0) return -1; /* order chain must be a prefix 1..k */
  }
  for (int m = 0; m < cs->n_mix; ++m) { /* a mixed channel needs both first-order channels */
    cs->mix_ci[m] = cs->at[mix_i[m]][1];
    cs->mix_cj[m] = cs->at[mix_j[m]][1];
    if (cs->mix_ci[m] < 0 || cs->mix_cj[m] < 0) return -1;
  }
  return 0;
}

/* Derivatives phi^(0..5)(z) of the activation. */
template <class T>
void act_derivs(int act, T z, T *p) {
  switch (act) {
    case ORC_ACT_TANH: {
      /* tanh' = 1 - tanh^2; each further derivative follows by differentiating
         a polynomial in s = tanh z and using ds/dz = 1 - s^2. */
      T s = std::tanh(z);
      T s1 = 1.0 - s * s;
      p[0] = s;
      p[1] = s1;
      p[2] = -2.0 * s * s1;
      p[3] = s1 * (6.0 * s * s - 2.0);
      p[4] = s * s1 * (16.0 - 24.0 * s * s);
      p[5] = s1 * (16.0 - 120.0 * s * s + 120.0 * s * s * s * s);
      break;
    }
    case ORC_ACT_IDENTITY:
      p[0] = z; p[1] = 1.0; p[2] = 0.0; p[3] = 0.0; p[4] = 0.0; p[5] = 0.0;
      break;
    case ORC_ACT_SQUARE:
      p[0] = z * z; p[1] = 2.0 * z; p[2] = 2.0; p[3] = 0.0; p[4] = 0.0; p[5] = 0.0;
      break;
    case ORC_ACT_CUBE:
      p[0] = z * z * z; p[1] = 3.0 * z * z; p[2] = 6.0 * z; p[3] = 6.0; p[4] = 0.0; p[5] = 0.0;
      break;
    default: { /* ORC_ACT_SIN */
      T sn = std::sin(z), cs = std::cos(z);
      p[0] = sn; p[1] = cs; p[2] = -sn; p[3] = -cs; p[4] = sn; p[5] = cs;
      break;
    }
  }
}

/* Order-k derivative of phi(z(x)) along one direction, from z_1..z_k (the
 * derivatives of the pre-activation along that direction) and phi^(j)(z_0).
 * q points at phi^(0): the formulas read q[1] = phi', q[2] = phi'', ...
 * Called with q shifted by one it gives the partial derivative of a_k with
 * respect to z_0, since d phi^(j)(z_0)/d z_0 = phi^(j+1)(z_0). */
template <class T>
T faa_di_bruno(int k, const T *q, const T *zz) {
  const T z1 = zz[1];
  switch (k) {
    case 1: return q[1] * z1;
    case 2: return q[2] * z1 * z1 + q[1] * zz[2];
    case 3: return q[3] * z1 * z1 * z1 + 3.0 * q[2] * z1 * zz[2] + q[1] * zz[3];
    default:
      return q[4] * z1 * z1 * z1 * z1 + 6.0 * q[3] * z1 * z1 * zz[2] +
             q[2] * (3.0 * zz[2] * zz[2] + 4.0 * z1 * zz[3]) + q[1] * zz[4];
  }
}

/* Partial derivative of a_k (formula above) with respect to z_m, 1 <= m <= k. */
template <class T>
T faa_di_bruno_dz(int k, int m, const T *q, const T *zz) {
  const T z1 = zz[1];
  if (m == k) return q[1];
  switch (k) {
    case 2: /* m = 1 */
      return 2.0 * q[2] * z1;
    case 3:
      if (m == 1) return 3.0 * q[3] * z1 * z1 + 3.0 * q[2] * zz[2];
      return 3.0 * q[2] * z1; /* m = 2 */
    default: /* k = 4 */
      if (m == 1) return 4.0 * q[4] * z1 * z1 * z1 + 12.0 * q[3] * z1 * zz[2] + 4.0 * q[2] * zz[3];
      if (m == 2) return 6.0 * q[3] * z1 * z1 + 6.0 * q[2] * zz[2];
      return 4.0 * q[2] * z1; /* m = 3 */
  }
}

/* The activation jet of one layer (Eq. 2-3 and the recursion): from the
 * pre-activation jets z (C x n, channel-major) to the activation's jets a. */
template <class T>
void act_jet(const ChannelSet &cs, int act, int d, const T *z, T *a, int n) {
  for (int i = 0; i < n; ++i) {
    T phi[6];
    act_derivs(act, z[i], phi);
    a[i] = phi[0];
    for (int dir = 0; dir < d; ++dir) {
      T zz[kMaxOrder + 1];
      zz[0] = z[i];
      for (int k = 1; k <= cs.top[dir]; ++k) zz[k] = z[(size_t)cs.at[dir][k] * n + i];
      for (int k = 1; k <= cs.top[dir]; ++k) a[(size_t)cs.at[dir][k] * n + i] = faa_di_bruno(k, phi, zz);
    }
    /* mixed second order (Eq. 3, i != j): a_ij = phi'' z_i z_j + phi' z_ij */
    for (int m = 0; m < cs.n_mix; ++m) {
      const T zi = z[(size_t)cs.mix_ci[m] * n + i], zj = z[(size_t)cs.mix_cj[m] * n + i];
      const T zij = z[(size_t)cs.mix_c[m] * n + i];
      a[(size_t)cs.mix_c[m] * n + i] = phi[2] * zi * zj + phi[1] * zij;
    }
  }
}

/* Adjoint of act_jet: from the cotangent abar of the activation's jets to the
 * cotangent zbar of the pre-activation jets (both C x n), at the jets z. */
void act_jet_adjoint(const ChannelSet &cs, int act, int d, const double *z, const double *abar, double *zbar,
                     int n) {
  const int C = cs.C;
  for (size_t q = 0; q < (size_t)C * n; ++q) zbar[q] = 0.0;
  for (int j = 0; j < n; ++j) {
    double phi[6];
    act_derivs(act, z[j], phi);
    double z0bar = phi[1] * abar[j]; /* a_0 = phi(z_0) */
    for (int dir = 0; dir < d; ++dir) {
      const int K = cs.top[dir];
      if (K == 0) continue;
      double zz[kMaxOrder + 1];
      zz[0] = z[j];
      for (int k = 1; k <= K; ++k) zz[k] = z[(size_t)cs.at[dir][k] * n + j];
      for (int k = 1; k <= K; ++k) {
        const double ab = abar[(size_t)cs.at[dir][k] * n + j];
        z0bar += faa_di_bruno(k, phi + 1, zz) * ab; /* a_k depends on z_0 through phi^(.) */
        for (int m = 1; m <= k; ++m) zbar[(size_t)cs.at[dir][m] * n + j] += faa_di_bruno_dz(k, m, phi, zz) * ab;
      }
    }
    /* adjoint of a_ij = phi''(z_0) z_i z_j + phi'(z_0) z_ij */
    for (int m = 0; m < cs.n_mix; ++m) {
      const double ab = abar[(size_t)cs.mix_c[m] * n + j];
      const double zi = z[(size_t)cs.mix_ci[m] * n + j], zj = z[(size_t)cs.mix_cj[m] * n + j];
      const double zij = z[(size_t)cs.mix_c[m] * n + j];
      z0bar += (phi[3] * zi * zj + phi[2] * zij) * ab;
      zbar[(size_t)cs.mix_ci[m] * n + j] += phi[2] * zj * ab;
      zbar[(size_t)cs.mix_cj[m] * n + j] += phi[2] * zi * ab;
      zbar[(size_t)cs.mix_c[m] * n + j] += phi[1] * ab;
    }
    zbar[j] = z0bar;
  }
}

/* The affine map of a layer on every channel (Eq. 1): z_c = W a_c, plus the
 * bias on the value only.  W is n_out x n_in; a is C x n_in, z is C x n_out. */
template <class T>
void affine_jet(int C, const T *W, const T *b, const T *a, T *z, int n_in, int n_out) {
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < n_out; ++i) {
      T s = (c == 0) ? b[i] : T(0);
      for (int j = 0; j < n_in; ++j) s += W[(size_t)i * n_in + j] * a[(size_t)c * n_in + j];
      z[(size_t)c * n_out + i] = s;
    }
}

/* Its adjoint: dW += zbar_c a_c^T over channels, db += zbar_0, and (abar not
 * NULL) abar_c = W^T zbar_c. */
void affine_jet_adjoint(int C, const double *W, const double *a, const double *zbar, double *gW, double *gb,
                        double *abar, int n_in, int n_out) {
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < n_out; ++i) {
      const double zb = zbar[(size_t)c * n_out + i];
      if (zb == 0.0) continue;
      for (int j = 0; j < n_in; ++j) gW[(size_t)i * n_in + j] += zb * a[(size_t)c * n_in + j];
    }
  for (int i = 0; i < n_out; ++i) gb[i] += zbar[i];
  if (!abar) return;
  for (size_t q = 0; q < (size_t)C * n_in; ++q) abar[q] = 0.0;
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < n_out; ++i) {
      const double zb = zbar[(size_t)c * n_out + i];
      for (int j = 0; j < n_in; ++j) abar[(size_t)c * n_in + j] += W[(size_t)i * n_in + j] * zb;
    }
}

struct NetView {
  int L;
  const int *dims;
  std::vector<int64_t> w_off, b_off;
  int64_t n_theta;
};

NetView make_view(int L, const int *dims) {
  NetView v;
  v.L = L;
  v.dims = dims;
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    v.w_off.push_back(off);
    off += (int64_t)dims[l + 1] * dims[l];
    v.b_off.push_back(off);
    off += dims[l + 1];
  }
  v.n_theta = off;
  return v;
}

/* Per-point state for the reverse sweep: a[l] = input of layer l (C x dims[l]),
 * z[l] = output of layer l before activation (C x dims[l+1]). */
template <class T>
struct PointWork {
  std::vector<std::vector<T>> a, z;
  void init(const NetView &nv, int C) {
    a.resize(nv.L);
    z.resize(nv.L);
    for (int l = 0; l < nv.L; ++l) {
      a[l].assign((size_t)C * nv.dims[l], T(0));
      z[l].assign((size_t)C * nv.dims[l + 1], T(0));
    }
  }
};

/* Forward partial-jet pass for one point (Eq. 1-3 and the recursion). */
template <class T>
void forward_point(const NetView &nv, const T *theta, const ChannelSet &cs, int act,
                   const double *xp, PointWork<T> &pw) {
  const int C = cs.C;
  const int d = nv.dims[0];
  /* Seeds: a^0 = x, d a^0 / d x_i = e_i, higher derivatives of the input vanish. */
  std::vector<T> &a0 = pw.a[0];
  for (size_t q = 0; q < a0.size(); ++q) a0[q] = T(0);
  for (int j = 0; j < d; ++j) a0[j] = T(xp[j]);
  for (int c = 1; c < C; ++c)
    if (cs.ord[c] == 1) a0[(size_t)c * d + cs.dir[c]] = T(1);

  for (int l = 0; l < nv.L; ++l) {
    const int n_in = nv.dims[l], n_out = nv.dims[l + 1];
    const T *W = theta + nv.w_off[l];
    const T *b = theta + nv.b_off[l];
    const std::vector<T> &a = pw.a[l];
    std::vector<T> &z = pw.z[l];
    /* The same W acts on every channel; the bias enters the value only. */
    for (int c = 0; c < C; ++c)
      for (int i = 0; i < n_out; ++i) {
        T s = (c == 0) ? b[i] : T(0);
        for (int j = 0; j < n_in; ++j) s += W[(size_t)i * n_in + j] * a[(size_t)c * n_in + j];
        z[(size_t)c * n_out + i] = s;
      }
    if (l == nv.L - 1) break; /* linear output layer */
    std::vector<T> &an = pw.a[l + 1];
    for (int i = 0; i < n_out; ++i) {
      T phi[6];
      act_derivs(act, z[i], phi);
      an[i] = phi[0];
      for (int dir = 0; dir < d; ++dir) {
        T zz[kMaxOrder + 1];
        zz[0] = z[i];
        for (int k = 1; k <= cs.top[dir]; ++k) zz[k] = z[(size_t)cs.at[dir][k] * n_out + i];
        for (int k = 1; k <= cs.top[dir]; ++k)
          an[(size_t)cs.at[dir][k] * n_out + i] = faa_di_bruno(k, phi, zz);
      }
      /* mixed second order (Eq. 3, i != j): a_ij = phi'' z_i z_j + phi' z_ij */
      for (int m = 0; m < cs.n_mix; ++m) {
        const T zi = z[(size_t)cs.mix_ci[m] * n_out + i], zj = z[(size_t)cs.mix_cj[m] * n_out + i];
        const T zij = z[(size_t)cs.mix_c[m] * n_out + i];
        an[(size_t)cs.mix_c[m] * n_out + i] = phi[2] * zi * zj + phi[1] * zij;
      }
    }
  }
}

/* Residual channel lookups.  Returns -2 when a needed channel is missing. */
struct PdeChannels {
  int u, ut, ux, uxx, uxxxx, uy, uyy, uz, uzz, uxy;
};

int pde_channels(int kind, int d_in, int d_out, const ChannelSet &cs, PdeChannels *pc) {
  auto need = [&](int dir, int k) { return (dir < d_in) ? cs.at[dir][k] : -1; };
  *pc = PdeChannels{0, -1, -1, -1, -1, -1, -1, -1, -1, -1};
  auto need_mix = [&](int i, int j) {
    for (int m = 0; m < cs.n_mix; ++m)
      if (cs.mix_ci[m] == cs.at[i][1] && cs.mix_cj[m] == cs.at[j][1]) return cs.mix_c[m];
    return -1;
  };
  switch (kind) {
    case ORC_PDE_NONE: return 0;
    case ORC_PDE_BURGERS:
      if (d_in != 2 || d_out != 1) return -1;
      pc->ux = need(0, 1); pc->uxx = need(0, 2); pc->ut = need(1, 1);
      return (pc->ux < 0 || pc->uxx < 0 || pc->ut < 0) ? -2 : 0;
    case ORC_PDE_NS:
      if (d_in != 2 || d_out != 3) return -1;
      pc->ux = need(0, 1); pc->uxx = need(0, 2); pc->uy = need(1, 1); pc->uyy = need(1, 2);
      return (pc->ux < 0 || pc->uxx < 0 || pc->uy < 0 || pc->uyy < 0) ? -2 : 0;
    case ORC_PDE_KS:
      if (d_in != 2 || d_out != 1) return -1;
      pc->ux = need(0, 1); pc->uxx = need(0, 2); pc->uxxxx = need(0, 4); pc->ut = need(1, 1);
      return (pc->ux < 0 || pc->uxx < 0 || pc->uxxxx < 0 || pc->ut < 0) ? -2 : 0;
    case ORC_PDE_HEAT:
      if (d_in != 4 || d_out != 1) return -1;
      pc->uxx = need(0, 2); pc->uyy = need(1, 2); pc->uzz = need(2, 2); pc->ut = need(3, 1);
      return (pc->uxx < 0 || pc->uyy < 0 || pc->uzz < 0 || pc->ut < 0) ? -2 : 0;
    case ORC_PDE_BURGERS_BC:
      if (d_in != 2 || d_out != 1) return -1;
      return 0;
    case ORC_PDE_ANISO:
      if (d_in != 2 || d_out != 1) return -1;
      pc->uxx = need(0, 2); pc->uyy = need(1, 2);
      if (pc->uxx < 0 || pc->uyy < 0) return -2;
      pc->uxy = need_mix(0, 1);
      return pc->uxy < 0 ? -2 : 0;
    default: return -1;
  }
}

/* Heat source f = sin(pi x) sin(pi y) sin(pi z) exp(-t). */
double heat_source(const double *xp) {
  const double pi = 3.14159265358979323846;
  return std::sin(pi * xp[0]) * std::sin(pi * xp[1]) * std::sin(pi * xp[2]) * std::exp(-xp[3]);
}

/* u(o, c) = output o, channel c, taken from the last layer's pre-activation. */
template <class T>
void residual_point(int kind, const double *coef, const PdeChannels &pc, const double *xp,
                    const std::vector<T> &u, int C, T *r) {
  auto U = [&](int o, int c) { return u[(size_t)c * (u.size() / C) + o]; };
  switch (kind) {
    case ORC_PDE_BURGERS: {
      const double nu = coef[0];
      r[0] = U(0, pc.ut) + U(0, 0) * U(0, pc.ux) - nu * U(0, pc.uxx);
      break;
    }
    case ORC_PDE_NS: { /* Eq. 16, outputs (u, v, p) = (0, 1, 2) */
      const double Re = coef[0];
      T u0 = U(0, 0), v0 = U(1, 0);
      r[0] = U(0, pc.ux) + U(1, pc.uy);
      r[1] = u0 * U(0, pc.ux) + v0 * U(0, pc.uy) + U(2, pc.ux) - (U(0, pc.uxx) + U(0, pc.uyy)) / Re;
      r[2] = u0 * U(1, pc.ux) + v0 * U(1, pc.uy) + U(2, pc.uy) - (U(1, pc.uxx) + U(1, pc.uyy)) / Re;
      break;
    }
    case ORC_PDE_KS: {
      const double al = coef[0], be = coef[1], ga = coef[2];
      r[0] = U(0, pc.ut) + al * U(0, 0) * U(0, pc.ux) + be * U(0, pc.uxx) + ga * U(0, pc.uxxxx);
      break;
    }
    case ORC_PDE_HEAT: {
      const double ka = coef[0];
      r[0] = U(0, pc.ut) - ka * (U(0, pc.uxx) + U(0, pc.uyy) + U(0, pc.uzz)) - heat_source(xp);
      break;
    }
    case ORC_PDE_ANISO: {
      const double c = coef[0];
      r[0] = U(0, pc.uxx) + 2.0 * c * U(0, pc.uxy) + U(0, pc.uyy);
      break;
    }
    case ORC_PDE_BURGERS_BC: {
      const double pi = 3.14159265358979323846;
      r[0] = U(0, 0) + std::sin(pi * xp[0]);
      break;
    }
    default: break;
  }
}

/* Cotangent of the residual with respect to the output jets: ubar(o, c) =
 * sum_k rbar_k d r_k / d u(o, c), by the chain rule on the formulas above. */
void residual_adjoint_point(int kind, const double *coef, const PdeChannels &pc,
                            const std::vector<double> &u, int C, const double *rbar,
                            std::vector<double> &ubar) {
  const size_t d_out = u.size() / C;
  auto U = [&](int o, int c) { return u[(size_t)c * d_out + o]; };
  auto UB = [&](int o, int c) -> double & { return ubar[(size_t)c * d_out + o]; };
  for (double &v : ubar) v = 0.0;
  switch (kind) {
    case ORC_PDE_BURGERS: {
      const double nu = coef[0];
      UB(0, pc.ut) += rbar[0];
      UB(0, 0) += rbar[0] * U(0, pc.ux);
      UB(0, pc.ux) += rbar[0] * U(0, 0);
      UB(0, pc.uxx) += -nu * rbar[0];
      break;
    }
    case ORC_PDE_NS: {
      const double Re = coef[0];
      const double rc = rbar[0], ru = rbar[1], rv = rbar[2];
      /* r_c = u_x + v_y */
      UB(0, pc.ux) += rc;
      UB(1, pc.uy) += rc;
      /* r_u = u u_x + v u_y + p_x - (u_xx + u_yy)/Re */
      UB(0, 0) += ru * U(0, pc.ux);
      UB(0, pc.ux) += ru * U(0, 0);
      UB(1, 0) += ru * U(0, pc.uy);
      UB(0, pc.uy) += ru * U(1, 0);
      UB(2, pc.ux) += ru;
      UB(0, pc.uxx) += -ru / Re;
      UB(0, pc.uyy) += -ru / Re;
      /* r_v = u v_x + v v_y + p_y - (v_xx + v_yy)/Re */
      UB(0, 0) += rv * U(1, pc.ux);
      UB(1, pc.ux) += rv * U(0, 0);
      UB(1, 0) += rv * U(1, pc.uy);
      UB(1, pc.uy) += rv * U(1, 0);
      UB(2, pc.uy) += rv;
      UB(1, pc.uxx) += -rv / Re;
      UB(1, pc.uyy) += -rv / Re;
      break;
    }
    case ORC_PDE_KS: {
      const double al = coef[0], be = coef[1], ga = coef[2];
      UB(0, pc.ut) += rbar[0];
      UB(0, 0) += al * rbar[0] * U(0, pc.ux);
      UB(0, pc.ux) += al * rbar[0] * U(0, 0);
      UB(0, pc.uxx) += be * rbar[0];
      UB(0, pc.uxxxx) += ga * rbar[0];
      break;
    }
    case ORC_PDE_HEAT: {
      const double ka = coef[0];
      UB(0, pc.ut) += rbar[0];
      UB(0, pc.uxx) += -ka * rbar[0];
      UB(0, pc.uyy) += -ka * rbar[0];
      UB(0, pc.uzz) += -ka * rbar[0];
      break;
    }
    case ORC_PDE_BURGERS_BC:
      UB(0, 0) += rbar[0];
      break;
    case ORC_PDE_ANISO: {
      const double c = coef[0];
      UB(0, pc.uxx) += rbar[0];
      UB(0, pc.uyy) += rbar[0];
      UB(0, pc.uxy) += 2.0 * c * rbar[0];
      break;
    }
    default: break;
  }
}

/* Reverse sweep for one point: given zbar of the last layer (the output jets'
 * cotangent), accumulate d/dtheta into g. */
void backward_point(const NetView &nv, const double *theta, const ChannelSet &cs, int act,
                    PointWork<double> &pw, std::vector<double> &zbar, double *g) {
  const int C = cs.C;
  const int d = nv.dims[0];
  std::vector<double> abar;
  for (int l = nv.L - 1; l >= 0; --l) {
    const int n_in = nv.dims[l], n_out = nv.dims[l + 1];
    const double *W = theta + nv.w_off[l];
    const std::vector<double> &a = pw.a[l];
    double *gW = g + nv.w_off[l];
    double *gb = g + nv.b_off[l];
    /* z_c = W a_c (+ b for c = 0):  dW += zbar_c a_c^T,  db += zbar_0 */
    for (int c = 0; c < C; ++c)
      for (int i = 0; i < n_out; ++i) {
        const double zb = zbar[(size_t)c * n_out + i];
        if (zb == 0.0) continue;
        for (int j = 0; j < n_in; ++j) gW[(size_t)i * n_in + j] += zb * a[(size_t)c * n_in + j];
      }
    for (int i = 0; i < n_out; ++i) gb[i] += zbar[i];
    if (l == 0) break; /* the input seeds do not depend on theta */
    /* abar_c = W^T zbar_c */
    abar.assign((size_t)C * n_in, 0.0);
    for (int c = 0; c < C; ++c)
      for (int i = 0; i < n_out; ++i) {
        const double zb = zbar[(size_t)c * n_out + i];
        for (int j = 0; j < n_in; ++j) abar[(size_t)c * n_in + j] += W[(size_t)i * n_in + j] * zb;
      }
    /* Adjoint of the activation jet of layer l-1 (whose output is a[l]). */
    const std::vector<double> &zp = pw.z[l - 1];
    std::vector<double> zbp((size_t)C * n_in, 0.0);
    for (int j = 0; j < n_in; ++j) {
      double phi[6];
      act_derivs(act, zp[j], phi);
      double z0bar = phi[1] * abar[j]; /* a_0 = phi(z_0) */
      for (int dir = 0; dir < d; ++dir) {
        const int K = cs.top[dir];
        if (K == 0) continue;
        double zz[kMaxOrder + 1];
        zz[0] = zp[j];
        for (int k = 1; k <= K; ++k) zz[k] = zp[(size_t)cs.at[dir][k] * n_in + j];
        for (int k = 1; k <= K; ++k) {
          const double ab = abar[(size_t)cs.at[dir][k] * n_in + j];
          z0bar += faa_di_bruno(k, phi + 1, zz) * ab; /* a_k depends on z_0 through phi^(.) */
          for (int m = 1; m <= k; ++m)
            zbp[(size_t)cs.at[dir][m] * n_in + j] += faa_di_bruno_dz(k, m, phi, zz) * ab;
        }
      }
      /* adjoint of a_ij = phi''(z_0) z_i z_j + phi'(z_0) z_ij */
      for (int m = 0; m < cs.n_mix; ++m) {
        const double ab = abar[(size_t)cs.mix_c[m] * n_in + j];
        const double zi = zp[(size_t)cs.mix_ci[m] * n_in + j], zj = zp[(size_t)cs.mix_cj[m] * n_in + j];
        const double zij = zp[(size_t)cs.mix_c[m] * n_in + j];
        z0bar += (phi[3] * zi * zj + phi[2] * zij) * ab;
        zbp[(size_t)cs.mix_ci[m] * n_in + j] += phi[2] * zj * ab;
        zbp[(size_t)cs.mix_cj[m] * n_in + j] += phi[2] * zi * ab;
        zbp[(size_t)cs.mix_c[m] * n_in + j] += phi[1] * ab;
      }
      zbp[j] = z0bar;
    }
    zbar.swap(zbp);
  }
}

struct Problem {
  NetView nv;
  ChannelSet cs;
  PdeChannels pc;
  int n_res;
};

int setup(int n_layers, const int *dims, int act, int pde_kind, int n_ch, const int *ch_dir,
          const int *ch_ord, int64_t N, Problem *P) {
  if (n_layers < 1 || !dims || N < 0 || act < 0 || act > ORC_ACT_SIN) return -1;
  for (int l = 0; l <= n_layers; ++l)
    if (dims[l] < 1) return -1;
  P->nv = make_view(n_layers, dims);
  if (build_channels(n_ch, ch_dir, ch_ord, dims[0], &P->cs)) return -1;
  int st = pde_channels(pde_kind, dims[0], dims[n_layers], P->cs, &P->pc);
  if (st) return st;
  P->n_res = orc_n_res(pde_kind);
  return 0;
}

int n_threads_or_default(int n) { return n > 0 ? n : omp_get_max_threads(); }

} /* namespace */

extern "C" int orc_n_res(int pde_kind) {
  switch (pde_kind) {
    case ORC_PDE_BURGERS: return 1;
    case ORC_PDE_NS: return 3;
    case ORC_PDE_KS: return 1;
    case ORC_PDE_HEAT: return 1;
    case ORC_PDE_ANISO: return 1;
    case ORC_PDE_BURGERS_BC: return 1;
    default: return 0;
  }
}

extern "C" int orc_eval(int n_layers, const int *dims, const double *theta, int act, int pde_kind,
                        const double *coef, int n_ch, const int *ch_dir, const int *ch_ord,
                        int64_t N, const double *x, double *jets, double *r, double *loss,
                        const double *r_bar, double *grad, int n_threads) {
  Problem P;
  int st = setup(n_layers, dims, act, pde_kind, n_ch, ch_dir, ch_ord, N, &P);
  if (st) return st;
  if (!theta || (N > 0 && !x)) return -1;
  if ((r || loss || grad) && P.n_res == 0) return -1; /* residual quantities need a PDE */
  const NetView &nv = P.nv;
  const int C = P.cs.C, d = dims[0], d_out = dims[n_layers], n_res = P.n_res;
  const int64_t n_chunks = (N + kChunk - 1) / kChunk;
  std::vector<double> chunk_loss(n_chunks > 0 ? n_chunks : 1, 0.0);
  std::vector<std::vector<double>> chunk_grad;
  if (grad) chunk_grad.assign(n_chunks, std::vector<double>());

#pragma omp parallel num_threads(n_threads_or_default(n_threads))
  {
    PointWork<double> pw;
    pw.init(nv, C);
    std::vector<double> rr(n_res > 0 ? n_res : 1), rb(n_res > 0 ? n_res : 1);
    std::vector<double> ubar((size_t)C * d_out), zbar;
#pragma omp for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
      double lsum = 0.0;
      if (grad) chunk_grad[ch].assign(nv.n_theta, 0.0);
      const int64_t n_end = std::min<int64_t>(N, (ch + 1) * kChunk);
      for (int64_t n = ch * kChunk; n < n_end; ++n) {
        const double *xp = x + n * d;
        forward_point(nv, theta, P.cs, act, xp, pw);
        const std::vector<double> &u = pw.z[nv.L - 1];
        if (jets)
          for (int o = 0; o < d_out; ++o)
            for (int c = 0; c < C; ++c) jets[((size_t)o * C + c) * N + n] = u[(size_t)c * d_out + o];
        if (n_res == 0) continue;
        residual_point(pde_kind, coef, P.pc, xp, u, C, rr.data());
        for (int k = 0; k < n_res; ++k) {
          if (r) r[(size_t)k * N + n] = rr[k];
          lsum += rr[k] * rr[k];
        }
        if (grad) {
          for (int k = 0; k < n_res; ++k)
            rb[k] = r_bar ? r_bar[(size_t)k * N + n] : 2.0 * rr[k] / (double)N;
          residual_adjoint_point(pde_kind, coef, P.pc, u, C, rb.data(), ubar);
          zbar = ubar;
          backward_point(nv, theta, P.cs, act, pw, zbar, chunk_grad[ch].data());
        }
      }
      chunk_loss[ch] = lsum;
    }
  }
  if (loss) {
    double s = 0.0;
    for (int64_t ch = 0; ch < n_chunks; ++ch) s += chunk_loss[ch];
    *loss = N > 0 ? s / (double)N : 0.0;
  }
  if (grad) {
    for (int64_t q = 0; q < nv.n_theta; ++q) grad[q] = 0.0;
    for (int64_t ch = 0; ch < n_chunks; ++ch)
      for (int64_t q = 0; q < nv.n_theta; ++q) grad[q] += chunk_grad[ch][q];
  }
  return 0;
}

namespace {

/* The segments of a composite loss, checked against the point set. */
struct Segments {
  int n;
  const int *type;
  const int64_t *begin, *count;
  const double *weight;
  const int *mask, *data;
  const double *param;
  const double *targets; /* N x d_out target values of ORC_DATA_VALUES segments, or NULL */
};

int check_segments(const Segments &S, int64_t N, int C, int d_out, int n_res) {
  if (S.n < 1 || !S.type || !S.begin || !S.count || !S.weight || !S.mask || !S.data || !S.param) return -1;
  std::vector<char> used((size_t)N, 0);
  for (int s = 0; s < S.n; ++s) {
    const int64_t b = S.begin[s], c = S.count[s];
    if (b < 0 || c < 1 || b + c > N) return -1;
    switch (S.type[s]) {
      case ORC_SEG_PDE:
        if (n_res == 0) return -1;
        break;
      case ORC_SEG_DIRICHLET:
        if (S.data[s] < ORC_DATA_ZERO || S.data[s] > ORC_DATA_VALUES) return -1;
        if (S.data[s] == ORC_DATA_VALUES && !S.targets) return -1;
        for (int q = 0; q < d_out * C; ++q)
          if ((S.mask[s] >> q & 1) && q % C != 0) return -1; /* values only */
        if (S.mask[s] == 0 || (S.mask[s] >> (d_out * C)) != 0) return -1;
        break;
      case ORC_SEG_PERIODIC:
        if (c % 2 != 0 || S.mask[s] == 0 || (S.mask[s] >> (d_out * C)) != 0) return -1;
        break;
      default: return -1;
    }
    for (int64_t n = b; n < b + c; ++n) {
      if (used[n]) return -1; /* overlapping segments */
      used[n] = 1;
    }
  }
  return 0;
}

/* Boundary or initial data g_o(x) of a Dirichlet segment at point n. */
double seg_data_value(const Segments &S, int s, int o, int64_t n, int d_out, const double *xp) {
  const double pi = 3.14159265358979323846;
  const double *param = S.param + 4 * s;
  switch (S.data[s]) {
    case ORC_DATA_CONST: return param[o];
    case ORC_DATA_SIN: return param[0] * std::sin(param[1] * pi * xp[0]);
    case ORC_DATA_VALUES: return S.targets[n * d_out + o];
    default: return 0.0;
  }
}

/* Loss terms from the outputs of all points (u[n] = d_out x C, channel-major
 * as in forward_point's last layer); with ubar, also d loss / d u per point. */
template <class T>
void segment_loss(const Segments &S, int pde_kind, const double *coef, const PdeChannels &pc, int C, int d_out,
                  int n_res, const double *x, int d, const std::vector<std::vector<T>> &u, T *seg_loss, T *loss,
                  std::vector<std::vector<double>> *ubar) {
  auto U = [&](int64_t n, int o, int c) { return u[n][(size_t)c * d_out + o]; };
  T total = T(0);
  std::vector<T> rr(n_res > 0 ? n_res : 1);
  std::vector<double> rb(n_res > 0 ? n_res : 1), ub((size_t)C * d_out);
  for (int s = 0; s < S.n; ++s) {
    const int64_t b = S.begin[s], cnt = S.count[s];
    const double w = S.weight[s];
    T acc = T(0);
    if (S.type[s] == ORC_SEG_PDE) {
      for (int64_t n = b; n < b + cnt; ++n) {
        residual_point(pde_kind, coef, pc, x + n * d, u[n], C, rr.data());
        for (int k = 0; k < n_res; ++k) acc += rr[k] * rr[k];
        if (ubar) { /* d (w / cnt sum r^2) / d u = the residual adjoint with rbar = 2 w r / cnt */
          for (int k = 0; k < n_res; ++k) rb[k] = 2.0 * w * std::real(rr[k]) / (double)cnt;
          std::vector<double> ur((size_t)C * d_out);
          for (size_t q = 0; q < ur.size(); ++q) ur[q] = std::real(u[n][q]);
          residual_adjoint_point(pde_kind, coef, pc, ur, C, rb.data(), ub);
          for (size_t q = 0; q < ub.size(); ++q) (*ubar)[n][q] += ub[q];
        }
      }
      acc = acc / (double)cnt;
    } else if (S.type[s] == ORC_SEG_DIRICHLET) {
      for (int64_t n = b; n < b + cnt; ++n)
        for (int o = 0; o < d_out; ++o) {
          if (!(S.mask[s] >> (o * C) & 1)) continue;
          const T r = U(n, o, 0) - seg_data_value(S, s, o, n, d_out, x + n * d);
          acc += r * r;
          if (ubar) (*ubar)[n][(size_t)0 * d_out + o] += 2.0 * w * std::real(r) / (double)cnt;
        }
      acc = acc / (double)cnt;
    } else { /* periodic pairs */
      const int64_t pairs = cnt / 2;
      for (int64_t k = 0; k < pairs; ++k) {
        const int64_t na = b + 2 * k, nb = na + 1;
        for (int o = 0; o < d_out; ++o)
          for (int c = 0; c < C; ++c) {
            if (!(S.mask[s] >> (o * C + c) & 1)) continue;
            const T r = U(na, o, c) - U(nb, o, c);
            acc += r * r;
            if (ubar) {
              const double g = 2.0 * w * std::real(r) / (double)pairs;
              (*ubar)[na][(size_t)c * d_out + o] += g;
              (*ubar)[nb][(size_t)c * d_out + o] -= g;
            }
          }
      }
      acc = acc / (double)pairs;
    }
    if (seg_loss) seg_loss[s] = acc;
    total += w * acc;
  }
  if (loss) *loss = total;
}

template <class T>
int eval_segments(int n_layers, const int *dims, const T *theta, int act, int pde_kind, const double *coef,
                  int n_ch, const int *ch_dir, const int *ch_ord, int64_t N, const double *x, const Segments &S,
                  T *seg_loss, T *loss, double *grad, int n_threads) {
  Problem P;
  int st = setup(n_layers, dims, act, pde_kind, n_ch, ch_dir, ch_ord, N, &P);
  if (st) return st;
  if (!theta || N < 1 || !x) return -1;
  const NetView &nv = P.nv;
  const int C = P.cs.C, d = dims[0], d_out = dims[n_layers];
  if (check_segments(S, N, C, d_out, P.n_res)) return -1;
  /* 1. the network and its partial jet at every point, all segments together */
  std::vector<std::vector<T>> u((size_t)N);
#pragma omp parallel num_threads(n_threads_or_default(n_threads))
  {
    PointWork<T> pw;
    pw.init(nv, C);
#pragma omp for schedule(dynamic, 64)
    for (int64_t n = 0; n < N; ++n) {
      forward_point(nv, theta, P.cs, act, x + n * d, pw);
      u[n] = pw.z[nv.L - 1];
    }
  }
  /* 2. split: each segment's terms and the weighted loss; d loss / d u */
  std::vector<std::vector<double>> ubar;
  if (grad) ubar.assign((size_t)N, std::vector<double>((size_t)C * d_out, 0.0));
  segment_loss<T>(S, pde_kind, coef, P.pc, C, d_out, P.n_res, x, d, u, seg_loss, loss, grad ? &ubar : nullptr);
  if constexpr (!std::is_same<T, double>::value) return 0; /* complex step: the loss only */
  if (!grad) return 0;
  /* 3. reverse mode, point by point from its cotangent, summed in chunk order */
  const int64_t n_chunks = (N + kChunk - 1) / kChunk;
  std::vector<std::vector<double>> chunk_grad((size_t)n_chunks);
#pragma omp parallel num_threads(n_threads_or_default(n_threads))
  {
    PointWork<double> pw;
    pw.init(nv, C);
    std::vector<double> zbar;
#pragma omp for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
      chunk_grad[ch].assign(nv.n_theta, 0.0);
      const int64_t n_end = std::min<int64_t>(N, (ch + 1) * kChunk);
      for (int64_t n = ch * kChunk; n < n_end; ++n) {
        bool any = false;
        for (double v : ubar[n]) any = any || v != 0.0;
        if (!any) continue;
        forward_point(nv, (const double *)theta, P.cs, act, x + n * d, pw);
        zbar = ubar[n];
        backward_point(nv, (const double *)theta, P.cs, act, pw, zbar, chunk_grad[ch].data());
      }
    }
  }
  for (int64_t q = 0; q < nv.n_theta; ++q) grad[q] = 0.0;
  for (int64_t ch = 0; ch < n_chunks; ++ch)
    for (int64_t q = 0; q < nv.n_theta; ++q) grad[q] += chunk_grad[ch][q];
  return 0;
}

/* ---- Modified MLP with a periodic input embedding (the KS network of
 * Sec. 3.1.1, an architecture the paper takes from earlier PINN training
 * work; the exact form used here is stated in pinn_oracle.h). */
struct ModView {
  int H, w, d, M, dout, de;
  double omega;
  /* layers: 0 = U encoder, 1 = V encoder, 2 = first hidden layer, 3 .. H+1 =
     hidden layers 2 .. H, H+2 = output layer */
  std::vector<int> n_in, n_out;
  std::vector<int64_t> w_off, b_off;
  int64_t n_theta;
};

int make_mod_view(int H, int w, int d, int M, double period, int dout, ModView *v) {
  if (H < 1 || w < 1 || d < 1 || d > kMaxDir || M < 1 || !(period > 0.0) || dout < 1) return -1;
  v->H = H;
  v->w = w;
  v->d = d;
  v->M = M;
  v->dout = dout;
  v->de = d - 1 + 2 * M;
  v->omega = 2.0 * 3.14159265358979323846 / period;
  v->n_in = {v->de, v->de, v->de};
  v->n_out = {w, w, w};
  for (int l = 2; l <= H; ++l) {
    v->n_in.push_back(w);
    v->n_out.push_back(w);
  }
  v->n_in.push_back(w);
  v->n_out.push_back(dout);
  int64_t off = 0;
  v->w_off.clear();
  v->b_off.clear();
  for (size_t l = 0; l < v->n_in.size(); ++l) {
    v->w_off.push_back(off);
    off += (int64_t)v->n_out[l] * v->n_in[l];
    v->b_off.push_back(off);
    off += v->n_out[l];
  }
  v->n_theta = off;
  return 0;
}

/* Jets of the embedding e(x) (C x de).  The inputs x_1 .. x_{d-1} pass
 * through (a first derivative along their own direction is 1, every other
 * derivative 0).  The harmonics depend on x_0 only:
 *   d^k/dx_0^k cos(m omega x_0) = (m omega)^k cos(m omega x_0 + k pi / 2),
 *   d^k/dx_0^k sin(m omega x_0) = (m omega)^k sin(m omega x_0 + k pi / 2);
 * mixed derivatives of the embedding vanish. */
void embed_jet(const ModView &v, const ChannelSet &cs, const double *xp, double *e) {
  const int de = v.de, C = cs.C;
  const double half_pi = 0.5 * 3.14159265358979323846;
  for (size_t q = 0; q < (size_t)C * de; ++q) e[q] = 0.0;
  for (int c = 0; c < C; ++c) {
    const int dir = cs.dir[c], k = cs.ord[c];
    if (c > 0 && dir < 0) continue; /* mixed: zero */
    for (int j = 1; j < v.d; ++j) {
      if (c == 0) e[j - 1] = xp[j];
      else if (dir == j && k == 1) e[(size_t)c * de + j - 1] = 1.0;
    }
    if (c > 0 && dir != 0) continue; /* the harmonics do not depend on x_1.. */
    for (int m = 1; m <= v.M; ++m) {
      const double f = m * v.omega, ph = f * xp[0] + k * half_pi;
      const double amp = std::pow(f, (double)k);
      e[(size_t)c * de + v.d - 1 + 2 * (m - 1)] = amp * std::cos(ph);
      e[(size_t)c * de + v.d - 1 + 2 * (m - 1) + 1] = amp * std::sin(ph);
    }
  }
}

double binom(int k, int j) {
  double r = 1.0;
  for (int i = 1; i <= j; ++i) r = r * (k - j + i) / i;
  return r;
}

/* Jets of the elementwise product p q (C x n each): the Leibniz rule along
 * each direction, (pq)_k = sum_j binom(k, j) p_j q_{k-j}, and for a mixed
 * channel (pq)_ij = p_ij q + p_i q_j + p_j q_i + p q_ij. */
template <class T>
void prod_jet(const ChannelSet &cs, int d, const T *p, const T *q, T *out, int n) {
  for (int i = 0; i < n; ++i) {
    auto P = [&](int c) { return p[(size_t)c * n + i]; };
    auto Q = [&](int c) { return q[(size_t)c * n + i]; };
    out[i] = P(0) * Q(0);
    for (int dir = 0; dir < d; ++dir)
      for (int k = 1; k <= cs.top[dir]; ++k) {
        T s = T(0);
        for (int j = 0; j <= k; ++j) s += binom(k, j) * P(cs.at[dir][j]) * Q(cs.at[dir][k - j]);
        out[(size_t)cs.at[dir][k] * n + i] = s;
      }
    for (int m = 0; m < cs.n_mix; ++m) {
      const int cij = cs.mix_c[m], ci = cs.mix_ci[m], cj = cs.mix_cj[m];
      out[(size_t)cij * n + i] = P(cij) * Q(0) + P(ci) * Q(cj) + P(cj) * Q(ci) + P(0) * Q(cij);
    }
  }
}

/* Adjoint of prod_jet: pbar += d<obar, pq>/dp, qbar += d<obar, pq>/dq. */
void prod_jet_adjoint(const ChannelSet &cs, int d, const double *p, const double *q, const double *obar,
                      double *pbar, double *qbar, int n) {
  for (int i = 0; i < n; ++i) {
    auto at = [&](int c) { return (size_t)c * n + i; };
    pbar[at(0)] += obar[at(0)] * q[at(0)];
    qbar[at(0)] += obar[at(0)] * p[at(0)];
    for (int dir = 0; dir < d; ++dir)
      for (int k = 1; k <= cs.top[dir]; ++k) {
        const double ob = obar[at(cs.at[dir][k])];
        for (int j = 0; j <= k; ++j) {
          const int cp = cs.at[dir][j], cq = cs.at[dir][k - j];
          pbar[at(cp)] += binom(k, j) * q[at(cq)] * ob;
          qbar[at(cq)] += binom(k, j) * p[at(cp)] * ob;
        }
      }
    for (int m = 0; m < cs.n_mix; ++m) {
      const int cij = cs.mix_c[m], ci = cs.mix_ci[m], cj = cs.mix_cj[m];
      const double ob = obar[at(cij)];
      pbar[at(cij)] += ob * q[at(0)];
      qbar[at(0)] += ob * p[at(cij)];
      pbar[at(ci)] += ob * q[at(cj)];
      qbar[at(cj)] += ob * p[at(ci)];
      pbar[at(cj)] += ob * q[at(ci)];
      qbar[at(ci)] += ob * p[at(cj)];
      pbar[at(0)] += ob * q[at(cij)];
      qbar[at(cij)] += ob * p[at(0)];
    }
  }
}

/* Per-point state of the modified MLP: embedding e; encoder pre-activations
 * and outputs; per hidden layer l the pre-activation z[l] and output h[l]
 * (l = 1: phi(W_1 e + b_1); l >= 2: zZ[l] -> Z[l] -> h[l] = U + Z (V - U));
 * D = V - U; the output jets out. */
template <class T>
struct ModWork {
  std::vector<T> e, zU, U, zV, V, D, out;
  std::vector<std::vector<T>> z, Z, h;
  void init(const ModView &v, int C) {
    e.assign((size_t)C * v.de, T(0));
    zU.assign((size_t)C * v.w, T(0));
    U = zU;
    zV = zU;
    V = zU;
    D = zU;
    out.assign((size_t)C * v.dout, T(0));
    z.assign(v.H + 1, zU);
    Z.assign(v.H + 1, zU);
    h.assign(v.H + 1, zU);
  }
};

template <class T>
void forward_point_mod(const ModView &v, const T *theta, const ChannelSet &cs, int act, const double *xp,
                       ModWork<T> &wk) {
  const int C = cs.C, w = v.w, de = v.de;
  std::vector<double> e((size_t)C * de);
  embed_jet(v, cs, xp, e.data());
  for (size_t q = 0; q < e.size(); ++q) wk.e[q] = T(e[q]);
  auto W = [&](int l) { return theta + v.w_off[l]; };
  auto B = [&](int l) { return theta + v.b_off[l]; };
  affine_jet(C, W(0), B(0), wk.e.data(), wk.zU.data(), de, w);
  act_jet(cs, act, v.d, wk.zU.data(), wk.U.data(), w);
  affine_jet(C, W(1), B(1), wk.e.data(), wk.zV.data(), de, w);
  act_jet(cs, act, v.d, wk.zV.data(), wk.V.data(), w);
  for (size_t q = 0; q < wk.D.size(); ++q) wk.D[q] = wk.V[q] - wk.U[q];
  affine_jet(C, W(2), B(2), wk.e.data(), wk.z[1].data(), de, w);
  act_jet(cs, act, v.d, wk.z[1].data(), wk.h[1].data(), w);
  std::vector<T> P((size_t)C * w);
  for (int l = 2; l <= v.H; ++l) {
    affine_jet(C, W(l + 1), B(l + 1), wk.h[l - 1].data(), wk.z[l].data(), w, w);
    act_jet(cs, act, v.d, wk.z[l].data(), wk.Z[l].data(), w);
    prod_jet(cs, v.d, wk.Z[l].data(), wk.D.data(), P.data(), w); /* Z (V - U) */
    for (size_t q = 0; q < P.size(); ++q) wk.h[l][q] = wk.U[q] + P[q];
  }
  affine_jet(C, W(v.H + 2), B(v.H + 2), wk.h[v.H].data(), wk.out.data(), w, v.dout);
}

/* Reverse sweep for one point from the output jets' cotangent ubar (C x dout). */
void backward_point_mod(const ModView &v, const double *theta, const ChannelSet &cs, int act, ModWork<double> &wk,
                        const double *ubar, double *g) {
  const int C = cs.C, w = v.w, de = v.de;
  const size_t S = (size_t)C * w;
  auto W = [&](int l) { return theta + v.w_off[l]; };
  auto gW = [&](int l) { return g + v.w_off[l]; };
  auto gB = [&](int l) { return g + v.b_off[l]; };
  std::vector<double> hbar(S), hprev(S), Ubar(S, 0.0), Vbar(S, 0.0), Zbar(S), Dbar(S), zbar(S);
  affine_jet_adjoint(C, W(v.H + 2), wk.h[v.H].data(), ubar, gW(v.H + 2), gB(v.H + 2), hbar.data(), w, v.dout);
  for (int l = v.H; l >= 2; --l) {
    /* h_l = U + Z_l D */
    for (size_t q = 0; q < S; ++q) {
      Ubar[q] += hbar[q];
      Zbar[q] = 0.0;
      Dbar[q] = 0.0;
    }
    prod_jet_adjoint(cs, v.d, wk.Z[l].data(), wk.D.data(), hbar.data(), Zbar.data(), Dbar.data(), w);
    for (size_t q = 0; q < S; ++q) { /* D = V - U */
      Ubar[q] -= Dbar[q];
      Vbar[q] += Dbar[q];
    }
    act_jet_adjoint(cs, act, v.d, wk.z[l].data(), Zbar.data(), zbar.data(), w);
    affine_jet_adjoint(C, W(l + 1), wk.h[l - 1].data(), zbar.data(), gW(l + 1), gB(l + 1), hprev.data(), w, w);
    hbar.swap(hprev);
  }
  act_jet_adjoint(cs, act, v.d, wk.z[1].data(), hbar.data(), zbar.data(), w);
  affine_jet_adjoint(C, W(2), wk.e.data(), zbar.data(), gW(2), gB(2), nullptr, de, w);
  act_jet_adjoint(cs, act, v.d, wk.zU.data(), Ubar.data(), zbar.data(), w);
  affine_jet_adjoint(C, W(0), wk.e.data(), zbar.data(), gW(0), gB(0), nullptr, de, w);
  act_jet_adjoint(cs, act, v.d, wk.zV.data(), Vbar.data(), zbar.data(), w);
  affine_jet_adjoint(C, W(1), wk.e.data(), zbar.data(), gW(1), gB(1), nullptr, de, w);
}

/* Jets at every point and, with segments, the composite loss and its gradient
 * (the structure of eval_segments: all points evaluated together, then split). */
template <class T>
int eval_mod(const ModView &v, const T *theta, int act, int pde_kind, const double *coef, int n_ch,
             const int *ch_dir, const int *ch_ord, int64_t N, const double *x, const Segments *S, T *jets,
             T *seg_loss, T *loss, double *grad, int n_threads) {
  ChannelSet cs;
  if (build_channels(n_ch, ch_dir, ch_ord, v.d, &cs)) return -1;
  PdeChannels pc;
  const int n_res = orc_n_res(pde_kind);
  if (n_res > 0) {
    const int st = pde_channels(pde_kind, v.d, v.dout, cs, &pc);
    if (st) return st;
  }
  if (!theta || N < 1 || !x) return -1;
  const int C = cs.C, d = v.d, d_out = v.dout;
  if (S && check_segments(*S, N, C, d_out, n_res)) return -1;
  std::vector<std::vector<T>> u((size_t)N);
#pragma omp parallel num_threads(n_threads_or_default(n_threads))
  {
    ModWork<T> wk;
    wk.init(v, C);
#pragma omp for schedule(dynamic, 64)
    for (int64_t n = 0; n < N; ++n) {
      forward_point_mod(v, theta, cs, act, x + n * d, wk);
      u[n] = wk.out;
    }
  }
  if (jets)
    for (int64_t n = 0; n < N; ++n)
      for (int o = 0; o < d_out; ++o)
        for (int c = 0; c < C; ++c) jets[((size_t)o * C + c) * N + n] = u[n][(size_t)c * d_out + o];
  if (!S) return 0;
  std::vector<std::vector<double>> ubar;
  if (grad) ubar.assign((size_t)N, std::vector<double>((size_t)C * d_out, 0.0));
  segment_loss<T>(*S, pde_kind, coef, pc, C, d_out, n_res, x, d, u, seg_loss, loss, grad ? &ubar : nullptr);
  if constexpr (!std::is_same<T, double>::value) return 0; /* complex step: the loss only */
  if (!grad) return 0;
  const int64_t n_chunks = (N + kChunk - 1) / kChunk;
  std::vector<std::vector<double>> chunk_grad((size_t)n_chunks);
#pragma omp parallel num_threads(n_threads_or_default(n_threads))
  {
    ModWork<double> wk;
    wk.init(v, C);
#pragma omp for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
      chunk_grad[ch].assign(v.n_theta, 0.0);
      const int64_t n_end = std::min<int64_t>(N, (ch + 1) * kChunk);
      for (int64_t n = ch * kChunk; n < n_end; ++n) {
        bool any = false;
        for (double q : ubar[n]) any = any || q != 0.0;
        if (!any) continue;
        forward_point_mod(v, (const double *)theta, cs, act, x + n * d, wk);
        backward_point_mod(v, (const double *)theta, cs, act, wk, ubar[n].data(), chunk_grad[ch].data());
      }
    }
  }
  for (int64_t q = 0; q < v.n_theta; ++q) grad[q] = 0.0;
  for (int64_t ch = 0; ch < n_chunks; ++ch)
    for (int64_t q = 0; q < v.n_theta; ++q) grad[q] += chunk_grad[ch][q];
  return 0;
}

} /* namespace */

extern "C" int orc_eval_segments(int n_layers, const int *dims, const double *theta, int act, int pde_kind,
                                 const double *coef, int n_ch, const int *ch_dir, const int *ch_ord, int64_t N,
                                 const double *x, int n_seg, const int *seg_type, const int64_t *seg_begin,
                                 const int64_t *seg_count, const double *seg_weight, const int *seg_mask,
                                 const int *seg_data, const double *seg_param, double *seg_loss, double *loss,
                                 double *grad, int n_threads) {
  const Segments S{n_seg, seg_type, seg_begin, seg_count, seg_weight, seg_mask, seg_data, seg_param, nullptr};
  return eval_segments<double>(n_layers, dims, theta, act, pde_kind, coef, n_ch, ch_dir, ch_ord, N, x, S,
                               seg_loss, loss, grad, n_threads);
}

extern "C" int orc_eval_segments_cs(int n_layers, const int *dims, const double *theta, const double *delta,
                                    double h, int act, int pde_kind, const double *coef, int n_ch,
                                    const int *ch_dir, const int *ch_ord, int64_t N, const double *x, int n_seg,
                                    const int *seg_type, const int64_t *seg_begin, const int64_t *seg_count,
                                    const double *seg_weight, const int *seg_mask, const int *seg_data,
                                    const double *seg_param, double *dloss, int n_threads) {
  if (!theta || !delta || !(h > 0.0) || !dloss || n_layers < 1 || !dims) return -1;
  const Segments S{n_seg, seg_type, seg_begin, seg_count, seg_weight, seg_mask, seg_data, seg_param, nullptr};
  const NetView nv = make_view(n_layers, dims);
  std::vector<cplx> th((size_t)nv.n_theta);
  for (int64_t q = 0; q < nv.n_theta; ++q) th[q] = cplx(theta[q], h * delta[q]);
  cplx l(0.0, 0.0);
  const int st = eval_segments<cplx>(n_layers, dims, th.data(), act, pde_kind, coef, n_ch, ch_dir, ch_ord, N, x,
                                     S, nullptr, &l, nullptr, n_threads);
  if (st) return st;
  *dloss = l.imag() / h;
  return 0;
}

extern "C" int orc_eval_cs(int n_layers, const int *dims, const double *theta, const double *delta,
                           double h, int act, int pde_kind, const double *coef, int n_ch,
                           const int *ch_dir, const int *ch_ord, int64_t N, const double *x,
                           double *djets, double *dr, double *dloss, int n_threads) {
  Problem P;
  int st = setup(n_layers, dims, act, pde_kind, n_ch, ch_dir, ch_ord, N, &P);
  if (st) return st;
  if (!theta || !delta || !(h > 0.0) || (N > 0 && !x)) return -1;
  if ((dr || dloss) && P.n_res == 0) return -1;
  const NetView &nv = P.nv;
  const int C = P.cs.C, d = dims[0], d_out = dims[n_layers], n_res = P.n_res;
  std::vector<cplx> th(nv.n_theta);
  for (int64_t q = 0; q < nv.n_theta; ++q) th[q] = cplx(theta[q], h * delta[q]);
  const int64_t n_chunks = (N + kChunk - 1) / kChunk;
  std::vector<cplx> chunk_loss(n_chunks > 0 ? n_chunks : 1, cplx(0.0, 0.0));

#pragma omp parallel num_threads(n_threads_or_default(n_threads))
  {
    PointWork<cplx> pw;
    pw.init(nv, C);
    std::vector<cplx> rr(n_res > 0 ? n_res : 1);
#pragma omp for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
      cplx lsum(0.0, 0.0);
      const int64_t n_end = std::min<int64_t>(N, (ch + 1) * kChunk);
      for (int64_t n = ch * kChunk; n < n_end; ++n) {
        const double *xp = x + n * d;
        forward_point(nv, th.data(), P.cs, act, xp, pw);
        const std::vector<cplx> &u = pw.z[nv.L - 1];
        if (djets)
          for (int o = 0; o < d_out; ++o)
            for (int c = 0; c < C; ++c)
              djets[((size_t)o * C + c) * N + n] = u[(size_t)c * d_out + o].imag() / h;
        if (n_res == 0) continue;
        residual_point(pde_kind, coef, P.pc, xp, u, C, rr.data());
        for (int k = 0; k < n_res; ++k) {
          if (dr) dr[(size_t)k * N + n] = rr[k].imag() / h;
          lsum += rr[k] * rr[k]; /* analytic square, not |r|^2 */
        }
      }
      chunk_loss[ch] = lsum;
    }
  }
  if (dloss) {
    cplx s(0.0, 0.0);
    for (int64_t ch = 0; ch < n_chunks; ++ch) s += chunk_loss[ch];
    *dloss = N > 0 ? (s / (double)N).imag() / h : 0.0;
  }
  return 0;
}

// Adam, one step, element by element in FP64 (Kingma & Ba, Algorithm 1).
extern "C" int orc_adam(int64_t n, double *theta, const double *g, double *m, double *v, int64_t step,
                        double lr, double b1, double b2, double eps) {
  if (n < 0 || step < 1 || !theta || !g || !m || !v) return -1;
  const double c1 = 1.0 - std::pow(b1, (double)step);
  const double c2 = 1.0 - std::pow(b2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mhat = m[i] / c1;
    const double vhat = v[i] / c2;
    theta[i] -= lr * mhat / (std::sqrt(vhat) + eps);
  }
  return 0;
}

extern "C" int orc_mod_n_theta(int H, int w, int d, int M, double period, int dout, int64_t *n_theta) {
  ModView v;
  if (!n_theta || make_mod_view(H, w, d, M, period, dout, &v)) return -1;
  *n_theta = v.n_theta;
  return 0;
}

extern "C" int orc_eval_mod(int H, int w, int d, int M, double period, int dout, const double *theta, int act,
                            int pde_kind, const double *coef, int n_ch, const int *ch_dir, const int *ch_ord,
                            int64_t N, const double *x, double *jets, int n_seg, const int *seg_type,
                            const int64_t *seg_begin, const int64_t *seg_count, const double *seg_weight,
                            const int *seg_mask, const int *seg_data, const double *seg_param,
                            const double *targets, double *seg_loss, double *loss, double *grad, int n_threads) {
  ModView v;
  if (make_mod_view(H, w, d, M, period, dout, &v)) return -1;
  const Segments S{n_seg, seg_type, seg_begin, seg_count, seg_weight, seg_mask, seg_data, seg_param, targets};
  if (n_seg == 0 && (seg_loss || loss || grad)) return -1;
  return eval_mod<double>(v, theta, act, pde_kind, coef, n_ch, ch_dir, ch_ord, N, x, n_seg ? &S : nullptr, jets,
                          seg_loss, loss, grad, n_threads);
}

extern "C" int orc_eval_mod_cs(int H, int w, int d, int M, double period, int dout, const double *theta,
                               const double *delta, double h, int act, int pde_kind, const double *coef, int n_ch,
                               const int *ch_dir, const int *ch_ord, int64_t N, const double *x, double *djets,
                               int n_seg, const int *seg_type, const int64_t *seg_begin, const int64_t *seg_count,
                               const double *seg_weight, const int *seg_mask, const int *seg_data,
                               const double *seg_param, const double *targets, double *dloss, int n_threads) {
  ModView v;
  if (make_mod_view(H, w, d, M, period, dout, &v) || !theta || !delta || !(h > 0.0)) return -1;
  if (n_seg == 0 && dloss) return -1;
  const Segments S{n_seg, seg_type, seg_begin, seg_count, seg_weight, seg_mask, seg_data, seg_param, targets};
  std::vector<cplx> th((size_t)v.n_theta);
  for (int64_t q = 0; q < v.n_theta; ++q) th[q] = cplx(theta[q], h * delta[q]);
  ChannelSet cs;
  if (build_channels(n_ch, ch_dir, ch_ord, d, &cs)) return -1;
  std::vector<cplx> jc(djets ? (size_t)dout * cs.C * N : 0);
  cplx l(0.0, 0.0);
  const int st = eval_mod<cplx>(v, th.data(), act, pde_kind, coef, n_ch, ch_dir, ch_ord, N, x,
                                n_seg ? &S : nullptr, djets ? jc.data() : nullptr, nullptr, dloss ? &l : nullptr,
                                nullptr, n_threads);
  if (st) return st;
  if (djets)
    for (size_t q = 0; q < jc.size(); ++q) djets[q] = jc[q].imag() / h;
  if (dloss) *dloss = l.imag() / h;
  return 0;
}
