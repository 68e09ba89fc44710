// Host side of the C ABI declared in include/pinn_jet.h: argument validation,
// plan and workspace management, and the kernel schedule of one forward,
// residual or backward call.
#include "pinn_jet.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace {

thread_local std::string g_err;

pinn_status fail(pinn_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
pinn_status fail(pinn_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

struct KindInfo {
  int din, dout, C, nres;
};

bool kind_info(int kind, KindInfo *ki) {
  switch (kind) {
    case PINN_BURGERS_1D: *ki = {2, 1, 4, 1}; return true;
    case PINN_NS2D_STEADY: *ki = {2, 3, 5, 3}; return true;
    case PINN_KS_1D: *ki = {2, 1, 6, 1}; return true;
    case PINN_HEAT_3D: *ki = {4, 1, 8, 1}; return true;
    default: return false;
  }
}

constexpr int kMaxLayers = 17;        // up to 16 hidden layers
constexpr int64_t kMaxPoints = int64_t(1) << 26;

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

pinn_status check_pde(const pinn_pde *pde, int kind_expected) {
  if (!pde) return fail(PINN_ERR_ARG, "pde is NULL");
  KindInfo ki;
  if (!kind_info(pde->kind, &ki)) return fail(PINN_ERR_ARG, "unknown PDE kind %d", pde->kind);
  if (kind_expected && pde->kind != kind_expected)
    return fail(PINN_ERR_ARG, "PDE kind %d differs from the plan's kind %d", pde->kind, kind_expected);
  const int ncoef = pde->kind == PINN_KS_1D ? 3 : 1;
  for (int i = 0; i < ncoef; ++i)
    if (!std::isfinite(pde->coef[i])) return fail(PINN_ERR_ARG, "PDE coefficient %d is not finite", i);
  if (pde->kind == PINN_NS2D_STEADY && !(pde->coef[0] > 0.0))
    return fail(PINN_ERR_ARG, "Reynolds number must be positive");
  return PINN_OK;
}

// Validates a network description against a PDE kind; returns its hidden width.
pinn_status check_net(const pinn_net *net, int kind, int *w_out) {
  if (!net) return fail(PINN_ERR_ARG, "net is NULL");
  const int L = net->n_layers;
  if (L < 2 || L > kMaxLayers) return fail(PINN_ERR_ARG, "n_layers = %d outside [2, %d]", L, kMaxLayers);
  if (!net->dims || !net->W || !net->b) return fail(PINN_ERR_ARG, "net dims, W or b is NULL");
  KindInfo ki;
  kind_info(kind, &ki);
  if (net->dims[0] != ki.din)
    return fail(PINN_ERR_ARG, "dims[0] = %d but the PDE has %d inputs", net->dims[0], ki.din);
  if (net->dims[L] != ki.dout)
    return fail(PINN_ERR_ARG, "dims[L] = %d but the PDE has %d outputs", net->dims[L], ki.dout);
  const int w = net->dims[1];
  for (int l = 1; l < L; ++l)
    if (net->dims[l] != w) return fail(PINN_ERR_UNSUPPORTED, "hidden widths must all be equal");
  if (w < 32 || w > 512 || w % 32 != 0)
    return fail(PINN_ERR_UNSUPPORTED, "hidden width %d is not a multiple of 32 in [32, 512]", w);
  for (int l = 0; l < L; ++l)
    if (!net->W[l] || !net->b[l]) return fail(PINN_ERR_ARG, "W[%d] or b[%d] is NULL", l, l);
  *w_out = w;
  return PINN_OK;
}

pinn_status hip_fail(hipError_t e, const char *what) {
  return fail(PINN_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

struct pinn_plan_s {
  int kind = 0, prec = 0;
  uint32_t flags = 0;
  int L = 0, H = 0, w = 0;
  KindInfo ki{};
  int64_t max_points = 0, npad_max = 0;
  size_t save_cap = 0;
  int device = 0;
  // FP32 operands keep the FP32 layer state for the adjoint; 16-bit operands
  // recompute it in the backward kernels (a second MFMA GEMM is cheaper than
  // writing and reading the state).
  bool store_S = false;

  // device workspace (indices are 1-based layer numbers; entry 0 unused)
  std::vector<void *> Wop, WTop;  // hidden layers 2..H, operand-type copies
  std::vector<void *> A;          // activation stacks, layers 1..H
  std::vector<float *> S;         // saved FP32 states, layers 1..H
  void *Zb[2] = {nullptr, nullptr};
  float *u_save = nullptr, *r_save = nullptr, *ubar = nullptr;
  float *loss_part = nullptr;
  double *loss_part64 = nullptr;
  float *part = nullptr;
  int dw_splits = 1, thin_chunks = 1;
  std::vector<void *> allocs;
  size_t saved_bytes = 0, ws_bytes = 0;

  // state saved by the latest residual call
  bool have_state = false;
  int64_t st_N = 0;
  const float *st_x = nullptr;
  std::vector<const float *> st_W, st_b;

  // launch timing of one kernel class (pinn_plan_profile)
  int prof_class = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;

  bool verify() const { return (flags & PINN_VERIFY_F64) != 0; }

  hipError_t alloc(void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) {
      allocs.push_back(*p);
      ws_bytes += bytes;
    }
    return e;
  }
  // Adds the elapsed times of all recorded event pairs and empties the pool.
  hipError_t harvest() {
    if (ev_used == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(ev_pool[ev_used - 1]);
    if (e) return e;
    for (size_t i = 0; i + 1 < ev_used; i += 2) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev_pool[i], ev_pool[i + 1]);
      if (e) return e;
      prof_ms += ms;
      ++prof_launches;
    }
    ev_used = 0;
    return hipSuccess;
  }
  ~pinn_plan_s() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void *p : allocs) (void)hipFree(p);
  }
};

namespace {

int dw_splits_for(int64_t npad, int C, int w) {
  const int tile = pj::dw_tile(w);
  const int64_t tiles = (int64_t)(w / tile) * (w / tile);
  const int64_t rows = npad * C;
  // about two workgroups per CU, at least 1024 rows per split
  int64_t s = (512 + tiles - 1) / tiles;
  s = std::min<int64_t>(s, std::max<int64_t>(1, rows / 1024));
  return (int)std::max<int64_t>(1, s);
}

// Runs one launch; when its kernel class is the one being profiled, brackets
// it with a pair of events on the same stream.
template <class F>
hipError_t timed(pinn_plan p, int cls, hipStream_t st, F &&launch) {
  if (p->prof_class != cls) return launch();
  if (p->ev_used + 2 > p->ev_pool.size()) {
    if (p->ev_pool.size() < 2048) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e) return e;
        p->ev_pool.push_back(ev);
      }
    } else {
      hipError_t e = p->harvest();
      if (e) return e;
    }
  }
  hipError_t e = hipEventRecord(p->ev_pool[p->ev_used], st);
  if (e) return e;
  e = launch();
  if (e) return e;
  e = hipEventRecord(p->ev_pool[p->ev_used + 1], st);
  p->ev_used += 2;
  return e;
}

pinn_status check_call(pinn_plan plan, const pinn_net *net, const float *x, int64_t N) {
  if (!plan) return fail(PINN_ERR_ARG, "plan is NULL");
  int w = 0;
  pinn_status st = check_net(net, plan->kind, &w);
  if (st) return st;
  if (net->n_layers != plan->L || w != plan->w)
    return fail(PINN_ERR_ARG, "network shape differs from the plan's");
  if (!x) return fail(PINN_ERR_ARG, "x is NULL");
  if (N < 1 || N > plan->max_points)
    return fail(PINN_ERR_ARG, "N = %lld outside [1, max_points = %lld]", (long long)N,
                (long long)plan->max_points);
  return PINN_OK;
}

pj::Coef coef_of(const pinn_pde *pde) {
  pj::Coef k;
  for (int i = 0; i < 4; ++i) k.c[i] = (float)pde->coef[i];
  return k;
}

// Forward pass through all layers; optionally the residual and the loss.
pinn_status run_forward(pinn_plan p, const pinn_net *net, const pinn_pde *pde, const float *x,
                        int64_t N, float *jets, float *r, float *loss, double *loss_f64,
                        bool save_state, hipStream_t st) {
  const int64_t npad = round_up(N, pj::kPointTile);
  const int w = p->w, H = p->H, L = p->L;
  hipError_t e;
  {
    pj::CastPack pk{};
    for (int l = 2; l <= H; ++l) {
      pk.W[l - 2] = net->W[l - 1];
      pk.Wop[l - 2] = p->Wop[l];
    }
    e = timed(p, PINN_K_OTHER, st, [&] { return pj::launch_cast_all(p->prec, pk, H - 1, w, st); });
    if (e) return hip_fail(e, "cast");
  }
  pinn_pde dflt0{};
  const pinn_pde *pd = pde;
  if (!pd) {
    dflt0.kind = p->kind;
    dflt0.coef[0] = 1.0;
    pd = &dflt0;
  }
  double *lp64 = p->verify() ? p->loss_part64 : nullptr;
  const int P = pj::fused_fwd_points(p->ki.C, w, p->prec);
  if (P > 0) {
    pj::FusedFwdArgs a{};
    a.x = x;
    a.N = N;
    a.N_pad = npad;
    a.w = w;
    a.H = H;
    a.W1 = net->W[0];
    a.b1 = net->b[0];
    for (int l = 2; l <= H; ++l) {
      a.Wop[l] = p->Wop[l];
      a.b[l] = net->b[l - 1];
    }
    a.WL = net->W[L - 1];
    a.bL = net->b[L - 1];
    for (int l = 1; l <= H; ++l) {
      a.A[l] = save_state ? p->A[l] : nullptr;
      a.S[l] = save_state ? p->S[l] : nullptr;
    }
    a.k = coef_of(pd);
    a.jets = jets;
    a.r = r;
    a.u_save = p->u_save;
    a.r_save = p->r_save;
    a.loss_part = p->loss_part;
    a.loss_part64 = lp64;
    e = timed(p, PINN_K_LAYER_FWD, st, [&] { return pj::launch_fwd_fused(p->kind, p->prec, a, P, st); });
    if (e) return hip_fail(e, "fused forward");
    if (loss || loss_f64) {
      e = timed(p, PINN_K_OTHER, st, [&] { return pj::launch_loss_reduce(p->loss_part, lp64, (int)(npad / P), 1.0 / (double)N, loss, loss_f64, st); });
      if (e) return hip_fail(e, "loss reduction");
    }
    return PINN_OK;
  }
  e = timed(p, PINN_K_SEED_FWD, st, [&] { return pj::launch_seed_fwd(p->kind, p->prec, x, N, npad, net->W[0], net->b[0], w, p->A[1], p->S[1], st); });
  if (e) return hip_fail(e, "seed layer");
  for (int l = 2; l <= H; ++l) {
    e = timed(p, PINN_K_LAYER_FWD, st, [&] { return pj::launch_layer_fwd(p->kind, p->prec, p->A[l - 1], p->Wop[l], net->b[l - 1], p->A[l], p->S[l],
                             npad, w, st); });
    if (e) return hip_fail(e, "hidden layer");
  }
  e = timed(p, PINN_K_OUT_FWD, st, [&] { return pj::launch_out_fwd(p->kind, p->prec, p->A[H], net->W[L - 1], net->b[L - 1], x, N, npad, w,
                         coef_of(pd), jets, r, p->u_save, p->r_save, p->loss_part, lp64, st); });
  if (e) return hip_fail(e, "output layer");
  if (loss || loss_f64) {
    e = timed(p, PINN_K_OTHER, st, [&] { return pj::launch_loss_reduce(p->loss_part, lp64, (int)(npad / 16), 1.0 / (double)N, loss, loss_f64, st); });
    if (e) return hip_fail(e, "loss reduction");
  }
  return PINN_OK;
}

}  // namespace

extern "C" {

const char *pinn_last_error(void) { return g_err.c_str(); }

int32_t pinn_pde_channels(int32_t kind) {
  KindInfo ki;
  return kind_info(kind, &ki) ? ki.C : 0;
}

int32_t pinn_pde_residuals(int32_t kind) {
  KindInfo ki;
  return kind_info(kind, &ki) ? ki.nres : 0;
}

pinn_status pinn_plan_create(const pinn_net *net, const pinn_pde *pde, int64_t max_points,
                             int32_t prec, uint32_t flags, size_t save_cap_bytes, pinn_plan *out) {
  g_err.clear();
  if (!out) return fail(PINN_ERR_ARG, "out is NULL");
  *out = nullptr;
  pinn_status st = check_pde(pde, 0);
  if (st) return st;
  int w = 0;
  st = check_net(net, pde->kind, &w);
  if (st) return st;
  if (prec != PINN_FP32 && prec != PINN_BF16 && prec != PINN_FP16)
    return fail(PINN_ERR_ARG, "unknown precision %d", prec);
  if (flags & ~(uint32_t)PINN_VERIFY_F64) return fail(PINN_ERR_ARG, "unknown flags 0x%x", flags);
  if (max_points < 1 || max_points > kMaxPoints)
    return fail(PINN_ERR_ARG, "max_points = %lld outside [1, %lld]", (long long)max_points,
                (long long)kMaxPoints);

  KindInfo ki;
  kind_info(pde->kind, &ki);
  const int L = net->n_layers, H = L - 1;
  const int64_t npad = round_up(max_points, pj::kPointTile);
  const size_t osz = (size_t)pj::op_size(prec);
  const size_t stack_elems = (size_t)npad * ki.C * w;
  const bool store_S = prec == PINN_FP32;
  const size_t saved = (size_t)H * stack_elems * (osz + (store_S ? sizeof(float) : 0));
  if (save_cap_bytes != 0 && save_cap_bytes < saved)
    return fail(PINN_ERR_CAP, "save_cap_bytes = %zu below the %zu bytes of saved layer state", save_cap_bytes,
                saved);

  pinn_plan p = new (std::nothrow) pinn_plan_s;
  if (!p) return fail(PINN_ERR_NOMEM, "host allocation failed");
  p->kind = pde->kind;
  p->prec = prec;
  p->flags = flags;
  p->L = L;
  p->H = H;
  p->w = w;
  p->ki = ki;
  p->max_points = max_points;
  p->npad_max = npad;
  p->save_cap = save_cap_bytes;
  p->saved_bytes = saved;
  p->store_S = store_S;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(PINN_ERR_DEVICE, "no HIP device");
  }
  p->Wop.assign(H + 1, nullptr);
  p->WTop.assign(H + 1, nullptr);
  p->A.assign(H + 1, nullptr);
  p->S.assign(H + 1, nullptr);
  hipError_t e = hipSuccess;
  auto A = [&](void **ptr, size_t bytes) {
    if (e == hipSuccess) e = p->alloc(ptr, bytes);
  };
  for (int l = 2; l <= H; ++l) {
    A(&p->Wop[l], (size_t)w * w * osz);
    A(&p->WTop[l], (size_t)w * w * osz);
  }
  for (int l = 1; l <= H; ++l) {
    A(&p->A[l], stack_elems * osz);
    if (store_S) A(reinterpret_cast<void **>(&p->S[l]), stack_elems * sizeof(float));
  }
  A(&p->Zb[0], stack_elems * osz);
  A(&p->Zb[1], stack_elems * osz);
  A(reinterpret_cast<void **>(&p->u_save), (size_t)npad * ki.dout * ki.C * sizeof(float));
  A(reinterpret_cast<void **>(&p->r_save), (size_t)npad * ki.nres * sizeof(float));
  A(reinterpret_cast<void **>(&p->ubar), (size_t)npad * ki.dout * ki.C * sizeof(float));
  A(reinterpret_cast<void **>(&p->loss_part), (size_t)(npad / 16) * sizeof(float));
  A(reinterpret_cast<void **>(&p->loss_part64), (size_t)(npad / 16) * sizeof(double));
  p->dw_splits = dw_splits_for(npad, ki.C, w);
  p->thin_chunks = (int)std::max<int64_t>(1, npad / 64);
  const size_t part_elems =
      std::max<size_t>((size_t)p->dw_splits * ((size_t)w * w + w),
                       (size_t)p->thin_chunks * std::max(ki.dout * w + ki.dout, w * ki.din + w));
  A(reinterpret_cast<void **>(&p->part), part_elems * sizeof(float));
  if (e != hipSuccess) {
    delete p;
    return fail(e == hipErrorOutOfMemory ? PINN_ERR_NOMEM : PINN_ERR_DEVICE, "workspace allocation: %s",
                hipGetErrorString(e));
  }
  *out = p;
  return PINN_OK;
}

pinn_status pinn_plan_destroy(pinn_plan plan) {
  g_err.clear();
  if (!plan) return fail(PINN_ERR_ARG, "plan is NULL");
  delete plan;
  return PINN_OK;
}

pinn_status pinn_plan_memory(pinn_plan plan, size_t *saved_bytes, size_t *workspace_bytes) {
  g_err.clear();
  if (!plan) return fail(PINN_ERR_ARG, "plan is NULL");
  if (saved_bytes) *saved_bytes = plan->saved_bytes;
  if (workspace_bytes) *workspace_bytes = plan->ws_bytes;
  return PINN_OK;
}

pinn_status pinn_plan_profile(pinn_plan plan, int32_t kernel_class) {
  g_err.clear();
  if (!plan) return fail(PINN_ERR_ARG, "plan is NULL");
  if (kernel_class < 0 || kernel_class > PINN_K_OTHER)
    return fail(PINN_ERR_ARG, "unknown kernel class %d", kernel_class);
  plan->prof_class = kernel_class;
  plan->ev_used = 0;
  plan->prof_ms = 0.0;
  plan->prof_launches = 0;
  return PINN_OK;
}

pinn_status pinn_plan_profile_read(pinn_plan plan, double *total_ms, int64_t *launches) {
  g_err.clear();
  if (!plan) return fail(PINN_ERR_ARG, "plan is NULL");
  hipError_t e = plan->harvest();
  if (e) return hip_fail(e, "event timing");
  if (total_ms) *total_ms = plan->prof_ms;
  if (launches) *launches = plan->prof_launches;
  return PINN_OK;
}

pinn_status pinn_jet_forward(pinn_plan plan, const pinn_net *net, const float *x, int64_t N,
                             float *jets, void *stream) {
  g_err.clear();
  pinn_status st = check_call(plan, net, x, N);
  if (st) return st;
  if (!jets) return fail(PINN_ERR_ARG, "jets is NULL");
  plan->have_state = false;
  return run_forward(plan, net, nullptr, x, N, jets, nullptr, nullptr, nullptr, false, (hipStream_t)stream);
}

pinn_status pinn_jet_residual(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                              const float *x, int64_t N, float *r, float *loss, double *loss_f64,
                              float *jets, void *stream) {
  g_err.clear();
  pinn_status st = check_call(plan, net, x, N);
  if (st) return st;
  st = check_pde(pde, plan->kind);
  if (st) return st;
  if (loss_f64 && !plan->verify()) return fail(PINN_ERR_ARG, "loss_f64 needs a PINN_VERIFY_F64 plan");
  plan->have_state = false;
  st = run_forward(plan, net, pde, x, N, jets, r, loss, loss_f64, true, (hipStream_t)stream);
  if (st) return st;
  plan->have_state = true;
  plan->st_N = N;
  plan->st_x = x;
  plan->st_W.assign(net->W, net->W + net->n_layers);
  plan->st_b.assign(net->b, net->b + net->n_layers);
  return PINN_OK;
}

pinn_status pinn_jet_backward(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                              const float *x, int64_t N, const float *r_bar, float *const *dW,
                              float *const *db, double *const *dW_f64, double *const *db_f64,
                              void *stream) {
  g_err.clear();
  pinn_status st = check_call(plan, net, x, N);
  if (st) return st;
  st = check_pde(pde, plan->kind);
  if (st) return st;
  pinn_plan p = plan;
  const int L = p->L, H = p->H, w = p->w;
  if (!dW || !db) return fail(PINN_ERR_ARG, "dW or db is NULL");
  for (int l = 0; l < L; ++l)
    if (!dW[l] || !db[l]) return fail(PINN_ERR_ARG, "dW[%d] or db[%d] is NULL", l, l);
  if ((dW_f64 || db_f64) && !p->verify())
    return fail(PINN_ERR_ARG, "FP64 gradients need a PINN_VERIFY_F64 plan");
  if ((dW_f64 == nullptr) != (db_f64 == nullptr))
    return fail(PINN_ERR_ARG, "dW_f64 and db_f64 must both be given or both be NULL");
  if (dW_f64)
    for (int l = 0; l < L; ++l)
      if (!dW_f64[l] || !db_f64[l]) return fail(PINN_ERR_ARG, "dW_f64[%d] or db_f64[%d] is NULL", l, l);
  if (!p->have_state || p->st_N != N || p->st_x != x ||
      !std::equal(p->st_W.begin(), p->st_W.end(), net->W) ||
      !std::equal(p->st_b.begin(), p->st_b.end(), net->b))
    return fail(PINN_ERR_STATE, "backward does not follow a residual call with the same x, N and parameters");

  hipStream_t s = (hipStream_t)stream;
  const int64_t npad = round_up(N, pj::kPointTile);
  const KindInfo &ki = p->ki;
  auto f64 = [&](double *const *arr, int l) -> double * { return arr ? arr[l] : nullptr; };
  hipError_t e;
  {
    pj::CastPack pk{};
    for (int l = 2; l <= H; ++l) {
      pk.W[l - 2] = net->W[l - 1];
      pk.Wop[l - 2] = p->Wop[l];
      pk.WTop[l - 2] = p->WTop[l];
    }
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_cast_all(p->prec, pk, H - 1, w, s); });
    if (e) return hip_fail(e, "cast");
  }
  // Source of z for the adjoint of activation layer m: the saved state, or a
  // recompute from the previous stack (m >= 2) or from x (m = 1).
  auto zsrc = [&](pj::LayerBwd &B, int m) {
    if (p->store_S) {
      B.S_in = p->S[m];
    } else if (m >= 2) {
      B.A_prev = p->A[m - 1];
      B.Wz = p->Wop[m];
      B.bz = net->b[m - 1];
    } else {
      B.x = x;
      B.W1 = net->W[0];
      B.bz = net->b[0];
    }
  };
  // Output layer: ubar, then zbar of layer H, then dW_L, db_L.
  e = timed(p, PINN_K_OUT_BWD, s, [&] { return pj::launch_out_adj(p->kind, p->u_save, p->r_save, r_bar, N, npad, (float)(2.0 / (double)N), coef_of(pde), p->ubar, s); });
  if (e) return hip_fail(e, "output adjoint");
  {
    pj::LayerBwd B{};
    B.top = true;
    B.ubar = p->ubar;
    B.WL = net->W[L - 1];
    B.N = N;
    B.w = w;
    B.Zb_out = p->Zb[H % 2];
    zsrc(B, H);
    e = timed(p, PINN_K_OUT_BWD, s, [&] { return pj::launch_layer_bwd(p->kind, p->prec, B, npad, s); });
    if (e) return hip_fail(e, "last hidden adjoint");
  }
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_dw_out(p->kind, p->prec, p->ubar, p->A[H], npad, w, p->part, p->thin_chunks, s); });
  if (e) return hip_fail(e, "output-layer gradient");
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->thin_chunks, (int64_t)ki.dout * w + ki.dout,
                               (int64_t)ki.dout * w, ki.dout, dW[L - 1], db[L - 1], f64(dW_f64, L - 1),
                               f64(db_f64, L - 1), s); });
  if (e) return hip_fail(e, "reduction");
  // Hidden layers H..2.
  for (int l = H; l >= 2; --l) {
    void *cur = p->Zb[l % 2], *prev = p->Zb[(l - 1) % 2];
    e = timed(p, PINN_K_DW_HIDDEN, s, [&] { return pj::launch_dw_hidden(p->prec, ki.C, cur, p->A[l - 1], npad, w, p->part, p->part + (size_t)w * w, p->dw_splits, s); });
    if (e) return hip_fail(e, "hidden-layer gradient");
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->dw_splits, (int64_t)w * w + w, (int64_t)w * w, w, dW[l - 1], db[l - 1], f64(dW_f64, l - 1), f64(db_f64, l - 1), s); });
    if (e) return hip_fail(e, "reduction");
    pj::LayerBwd B{};
    B.top = false;
    B.Zb_in = cur;
    B.WT = p->WTop[l];
    B.N = N;
    B.w = w;
    B.Zb_out = prev;
    zsrc(B, l - 1);
    e = timed(p, PINN_K_LAYER_BWD, s, [&] { return pj::launch_layer_bwd(p->kind, p->prec, B, npad, s); });
    if (e) return hip_fail(e, "hidden adjoint");
  }
  // First layer.
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_dw_seed(p->kind, p->prec, p->Zb[1], x, N, npad, w, p->part, p->thin_chunks, s); });
  if (e) return hip_fail(e, "first-layer gradient");
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->thin_chunks, (int64_t)w * ki.din + w, (int64_t)w * ki.din, w,
                               dW[0], db[0], f64(dW_f64, 0), f64(db_f64, 0), s); });
  if (e) return hip_fail(e, "reduction");
  return PINN_OK;
}

}  // extern "C"
