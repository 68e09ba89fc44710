// Host side of the C ABI declared in include/pinn_jet.h: argument validation,
// plan and workspace management, and the kernel schedule of one forward,
// residual or backward call.
#include "pinn_jet.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

#include "group.hpp"
#include "kernels.hpp"
#include "plan_region.hpp"

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
    case PINN_ANISO_2D: *ki = {2, 1, 6, 1}; return true;
    case PINN_BURGERS_BC: *ki = {2, 1, 1, 1}; return true;
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
  std::vector<void *> Wlo;        // low parts W - Wop of the BF16 weight pairs (BF16 only)
  std::vector<void *> A;          // activation stacks, layers 1..H (null: not materialized)
  std::vector<float *> S;         // saved FP32 states, layers 1..H (store_S only)
  // Checkpoint schedule: ckpt[l] means layer l's stack is kept from the
  // forward pass to the backward pass.  The other layers are recomputed
  // during backward, one segment (the layers between two checkpoints) at a
  // time, into the scratch slots.
  std::vector<char> ckpt;
  std::vector<void *> slot;
  std::vector<void *> ckpt_buf;   // owned buffers of the checkpoint layers
  void *Zb[2] = {nullptr, nullptr};
  float *u_save = nullptr, *r_save = nullptr, *ubar = nullptr;
  float *loss_part = nullptr;
  double *loss_part64 = nullptr;
  float *part = nullptr;
  int dw_splits = 1, thin_chunks = 1;
  int dw_splits_max = 1;   // partial buffer capacity (autotune candidates stay below it)
  int fwd_points = 0;      // fused forward points per workgroup; 0 = largest that fits
  int bwd_fused = 0;       // weight gradients inside the backward layer kernels when supported
  int bwd_points = 0;      // points per workgroup of the wide backward kernel; 0 = default (16)
  std::vector<void *> allocs;
  size_t saved_bytes = 0, ws_bytes = 0;
  // Workspace source: separate hipMalloc allocations (the default), consecutive
  // 256-byte aligned pieces of a caller-given device region (region != null;
  // nothing is allocated or freed), or no memory at all (measure: only the
  // bytes a region would need are counted).
  char *region = nullptr;
  size_t region_cap = 0, region_used = 0;
  bool measure = false;

  // modified MLP with periodic embedding (pinn_plan_create_modified); arch 0
  // is the plain MLP.  Layer l's stack h[l] (l = 1..H), gated-layer states
  // S[l] (l = 2..H), encoder stacks and the adjoint buffers; FP32 throughout.
  int arch = 0;
  int mod_M = 0, mod_de = 0;
  double mod_period = 0.0;
  float *mU = nullptr, *mV = nullptr, *mUbar = nullptr, *mVbar = nullptr;
  float *mhbar = nullptr, *mzbar = nullptr, *mzb3 = nullptr, *mE = nullptr, *mWscratch = nullptr;
  std::vector<float *> mh, mS, mWT;

  // segments of the latest pinn_jet_loss call (valid with have_state)
  bool have_seg = false;
  pj::SegPack seg{};
  double seg_scale = 1.0;
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
    if (measure || region) {
      const size_t sz = (bytes + 255) & ~size_t(255);
      *p = nullptr;
      if (region) {
        if (region_used + sz > region_cap) return hipErrorOutOfMemory;
        *p = region + region_used;
        region_used += sz;
      }
      ws_bytes += sz;
      return hipSuccess;
    }
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
  if (pj::current_recorder()) {  // recording (ensemble): tag the records with the class
    pj::current_record_class() = cls;
    const hipError_t e = launch();
    pj::current_record_class() = 0;
    return e;
  }
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
  if (plan->arch) {  // modified MLP: shapes are the plan's, the net carries the pointers
    if (!net) return fail(PINN_ERR_ARG, "net is NULL");
    if (net->n_layers != plan->L)
      return fail(PINN_ERR_ARG, "a modified-MLP net has hidden + 3 = %d layers, not %d", plan->L, net->n_layers);
    if (!net->W || !net->b) return fail(PINN_ERR_ARG, "net W or b is NULL");
    for (int l = 0; l < net->n_layers; ++l)
      if (!net->W[l] || !net->b[l]) return fail(PINN_ERR_ARG, "W[%d] or b[%d] is NULL", l, l);
  } else {
    int w = 0;
    pinn_status st = check_net(net, plan->kind, &w);
    if (st) return st;
    if (net->n_layers != plan->L || w != plan->w)
      return fail(PINN_ERR_ARG, "network shape differs from the plan's");
  }
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

// Hidden layers l_first..l_last starting from x (l_first = 1) or from A_in,
// the stack of layer l_first - 1; dest[l] / Sdest[l] (may be null) receive
// layer l's stack / FP32 state.  With `output`, also the output layer, the
// residual and the loss partials (l_last must be H).  Returns the number of
// loss partials in *n_part.
struct FwdOutputs {
  bool output = false;
  const pinn_pde *pde = nullptr;
  float *jets = nullptr, *r = nullptr;
};

pinn_status fwd_range(pinn_plan p, const pinn_net *net, const float *x, int64_t N, int64_t npad, int l_first,
                      int l_last, const void *A_in, void *const *dest, float *const *Sdest,
                      const FwdOutputs &o, int *n_part, hipStream_t st) {
  const int w = p->w, H = p->H, L = p->L;
  hipError_t e;
  pinn_pde dflt{};
  const pinn_pde *pd = o.pde;
  if (!pd) {
    dflt.kind = p->kind;
    dflt.coef[0] = 1.0;
    pd = &dflt;
  }
  double *lp64 = p->verify() ? p->loss_part64 : nullptr;
  int P = pj::fused_fwd_points(p->ki.C, w, p->prec);
  if (P > 0 && p->fwd_points > 0 && pj::fused_fwd_fits(p->fwd_points, p->ki.C, w, p->prec)) P = p->fwd_points;
  if (P > 0) {
    pj::FusedFwdArgs a{};
    a.x = x;
    a.N = N;
    a.N_pad = npad;
    a.w = w;
    a.H = H;
    a.l_first = l_first;
    a.l_last = l_last;
    a.A_in = A_in;
    a.do_output = o.output;
    a.W1 = net->W[0];
    a.b1 = net->b[0];
    for (int l = 2; l <= H; ++l) {
      a.Wop[l] = p->Wop[l];
      a.Wlo[l] = p->Wlo[l];
      a.b[l] = net->b[l - 1];
    }
    a.WL = net->W[L - 1];
    a.bL = net->b[L - 1];
    for (int l = l_first; l <= l_last; ++l) {
      a.A[l] = dest ? dest[l] : nullptr;
      a.S[l] = Sdest ? Sdest[l] : nullptr;
    }
    a.k = coef_of(pd);
    if (o.output) {
      a.jets = o.jets;
      a.r = o.r;
      a.u_save = p->u_save;
      a.r_save = p->r_save;
      a.loss_part = p->loss_part;
      a.loss_part64 = lp64;
    }
    e = timed(p, PINN_K_LAYER_FWD, st, [&] { return pj::launch_fwd_fused(p->kind, p->prec, a, P, st); });
    if (e) return hip_fail(e, "fused forward");
    if (n_part) *n_part = (int)(npad / P);
    return PINN_OK;
  }
  // layer by layer; layers without a destination go through two temporaries
  // (the adjoint ping-pong buffers, unused during a forward pass)
  const void *prev = A_in;
  for (int l = l_first; l <= l_last; ++l) {
    void *out = (dest && dest[l]) ? dest[l] : p->Zb[l % 2];
    float *S = Sdest ? Sdest[l] : nullptr;
    if (l == 1) {
      e = timed(p, PINN_K_SEED_FWD, st, [&] { return pj::launch_seed_fwd(p->kind, p->prec, x, N, npad, net->W[0], net->b[0], w, out, S, st); });
    } else {
      e = timed(p, PINN_K_LAYER_FWD, st, [&] { return pj::launch_layer_fwd(p->kind, p->prec, prev, p->Wop[l], p->Wlo[l], net->b[l - 1], out, S, npad, w, st); });
    }
    if (e) return hip_fail(e, "hidden layer");
    prev = out;
  }
  if (o.output) {
    e = timed(p, PINN_K_OUT_FWD, st, [&] { return pj::launch_out_fwd(p->kind, p->prec, prev, net->W[L - 1], net->b[L - 1], x, N, npad, w, coef_of(pd), o.jets, o.r, p->u_save, p->r_save, p->loss_part, lp64, st); });
    if (e) return hip_fail(e, "output layer");
    if (n_part) *n_part = (int)(npad / 16);
  }
  return PINN_OK;
}

pinn_status cast_weights(pinn_plan p, const pinn_net *net, bool transposed, hipStream_t st) {
  pj::CastPack pk{};
  for (int l = 2; l <= p->H; ++l) {
    pk.W[l - 2] = net->W[l - 1];
    pk.Wop[l - 2] = p->Wop[l];
    pk.WTop[l - 2] = transposed ? p->WTop[l] : nullptr;
    pk.Wlo[l - 2] = p->Wlo[l];
  }
  hipError_t e = timed(p, PINN_K_OTHER, st, [&] { return pj::launch_cast_all(p->prec, pk, p->H - 1, p->w, st); });
  return e ? hip_fail(e, "cast") : PINN_OK;
}

// Forward pass through all layers, the residual and the loss.  With
// save_state the checkpoint layers' stacks (and FP32 states) are kept.
pinn_status mod_forward(pinn_plan p, const pinn_net *net, const pinn_pde *pde, const float *x, int64_t N,
                        float *jets, float *r, float *loss, hipStream_t st);

// Whether the backward pass takes the fused weight-gradient path, and whether
// its top layer kernel also forms the output layer's gradient (then the top
// stack A_H is never read back, and the forward does not save it).
bool backward_fused(const pinn_plan p) {
  return p->bwd_fused && p->H >= 2 && pj::bwd_dw_fused_supported(p->ki.C, p->w, p->prec);
}
bool top_forms_out_grad(const pinn_plan p) {
  if (p->store_S || p->H < 2) return false;
  if (backward_fused(p)) return pj::bwd_top_out_grad_supported(p->ki.C, p->w, p->prec, p->ki.dout);
  return pj::wide_top_out_grad_supported(p->bwd_points, p->ki.C, p->w, p->prec, p->ki.dout);
}

pinn_status run_forward(pinn_plan p, const pinn_net *net, const pinn_pde *pde, const float *x,
                        int64_t N, float *jets, float *r, float *loss, double *loss_f64,
                        bool save_state, hipStream_t st) {
  if (p->arch) return mod_forward(p, net, pde, x, N, jets, r, loss, st);
  const int64_t npad = round_up(N, pj::kPointTile);
  const int H = p->H;
  // operand-type weights; a residual call (save_state) also makes the
  // transposed copies its backward pass uses
  pinn_status rs = cast_weights(p, net, save_state, st);
  if (rs) return rs;
  // stacks of non-checkpoint layers from an earlier backward are stale now
  for (int l = 1; l <= H; ++l)
    if (!p->ckpt[l]) p->A[l] = nullptr;
  std::vector<void *> dest(H + 1, nullptr);
  std::vector<float *> Sdest(H + 1, nullptr);
  if (save_state)
    for (int l = 1; l <= H; ++l) {
      dest[l] = p->ckpt[l] ? p->ckpt_buf[l] : nullptr;
      Sdest[l] = p->S[l];
    }
  if (save_state && top_forms_out_grad(p)) dest[H] = nullptr;
  FwdOutputs o;
  o.output = true;
  o.pde = pde;
  o.jets = jets;
  o.r = r;
  int n_part = 0;
  rs = fwd_range(p, net, x, N, npad, 1, H, nullptr, dest.data(), Sdest.data(), o, &n_part, st);
  if (rs) return rs;
  if (loss || loss_f64) {
    double *lp64 = p->verify() ? p->loss_part64 : nullptr;
    hipError_t e = timed(p, PINN_K_OTHER, st, [&] { return pj::launch_loss_reduce(p->loss_part, lp64, n_part, 1.0 / (double)N, loss, loss_f64, st); });
    if (e) return hip_fail(e, "loss reduction");
  }
  return PINN_OK;
}

// Stack of layer j (1 <= j <= H) for the backward pass: a checkpoint, or the
// segment of non-checkpoint layers around j recomputed into the scratch slots
// from the checkpoint below it (or from x).
pinn_status backward_stack(pinn_plan p, const pinn_net *net, const float *x, int64_t N, int64_t npad, int j,
                           const void **out, hipStream_t st) {
  if (p->A[j]) {
    *out = p->A[j];
    return PINN_OK;
  }
  const int H = p->H;
  int c = j - 1;
  while (c > 0 && !p->ckpt[c]) --c;
  int top = j;
  while (top + 1 <= H && !p->ckpt[top + 1]) ++top;
  for (int l = 1; l <= H; ++l)
    if (!p->ckpt[l]) p->A[l] = nullptr;  // the slots now hold this segment
  std::vector<void *> dest(H + 1, nullptr);
  for (int l = c + 1; l <= top; ++l) dest[l] = p->slot[l - c - 1];
  FwdOutputs o;
  pinn_status rs = fwd_range(p, net, x, N, npad, c + 1, top, c > 0 ? p->A[c] : nullptr, dest.data(), nullptr, o,
                             nullptr, st);
  if (rs) return rs;
  for (int l = c + 1; l <= top; ++l) p->A[l] = dest[l];
  *out = p->A[j];
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

}  // extern "C"

// Validates the arguments of a plan and builds it with its workspace taken
// as the plan's allocator says (see pinn_plan_s::alloc): hipMalloc when
// region is null and measure false; carved from [region, region + region_cap);
// or, with measure, only counted (the returned plan then owns no memory and
// is only good for its byte counts).
static pinn_status plan_build(const pinn_net *net, const pinn_pde *pde, int64_t max_points, int32_t prec,
                              uint32_t flags, size_t save_cap_bytes, char *region, size_t region_cap, bool measure,
                              pinn_plan *out) {
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
  // Checkpoint schedule.  No bound: every stack is kept (and, for FP32
  // operands, the FP32 layer states).  Under a bound: k = cap / stack stacks
  // are kept, at every s-th layer with s = ceil(H / (k + 1)); the FP32 states
  // are recomputed.
  const size_t stack_bytes = stack_elems * osz;
  const bool store_S = save_cap_bytes == 0 && prec == PINN_FP32;
  std::vector<char> ckpt(H + 1, 1);
  ckpt[0] = 0;
  if (save_cap_bytes != 0) {
    const size_t kmax = save_cap_bytes / stack_bytes;
    if (kmax < 1)
      return fail(PINN_ERR_CAP, "save_cap_bytes = %zu below one saved layer stack (%zu bytes)", save_cap_bytes,
                  stack_bytes);
    if (kmax < (size_t)H) {
      const int sgap = (H + (int)kmax) / ((int)kmax + 1);  // ceil(H / (k + 1))
      for (int l = 1; l <= H; ++l) ckpt[l] = (l % sgap == 0 && l < H) ? 1 : 0;
    }
  }
  int n_ckpt = 0, max_gap = 0;
  for (int l = 1, c = 0; l <= H + 1; ++l) {
    if (l == H + 1 || ckpt[l]) {
      max_gap = std::max(max_gap, l - c - 1);
      c = l;
    }
    if (l <= H && ckpt[l]) ++n_ckpt;
  }
  const size_t saved = (size_t)n_ckpt * stack_bytes + (store_S ? (size_t)H * stack_elems * sizeof(float) : 0);

  pinn_plan p = new (std::nothrow) pinn_plan_s;
  if (!p) return fail(PINN_ERR_NOMEM, "host allocation failed");
  p->kind = pde->kind;
  p->prec = prec;
  p->flags = flags;
  p->L = L;
  p->H = H;
  p->w = w;
  p->ki = ki;
  p->region = region;
  p->region_cap = region_cap;
  p->measure = measure;
  p->max_points = max_points;
  p->npad_max = npad;
  p->save_cap = save_cap_bytes;
  p->saved_bytes = saved;
  p->store_S = store_S;
  p->ckpt = ckpt;
  if (!measure && hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(PINN_ERR_DEVICE, "no HIP device");
  }
  p->Wop.assign(H + 1, nullptr);
  p->WTop.assign(H + 1, nullptr);
  p->Wlo.assign(H + 1, nullptr);
  p->A.assign(H + 1, nullptr);
  p->S.assign(H + 1, nullptr);
  hipError_t e = hipSuccess;
  auto A = [&](void **ptr, size_t bytes) {
    if (e == hipSuccess) e = p->alloc(ptr, bytes);
  };
  for (int l = 2; l <= H; ++l) {
    A(&p->Wop[l], (size_t)w * w * osz);
    A(&p->WTop[l], (size_t)w * w * osz);
    if (prec == PINN_BF16) A(&p->Wlo[l], (size_t)w * w * osz);
  }
  p->ckpt_buf.assign(H + 1, nullptr);
  for (int l = 1; l <= H; ++l) {
    if (ckpt[l]) {
      A(&p->ckpt_buf[l], stack_bytes);
      p->A[l] = p->ckpt_buf[l];
    }
    if (store_S) A(reinterpret_cast<void **>(&p->S[l]), stack_elems * sizeof(float));
  }
  p->slot.assign(max_gap, nullptr);
  for (int q = 0; q < max_gap; ++q) A(&p->slot[q], stack_bytes);
  A(&p->Zb[0], stack_elems * osz);
  A(&p->Zb[1], stack_elems * osz);
  A(reinterpret_cast<void **>(&p->u_save), (size_t)npad * ki.dout * ki.C * sizeof(float));
  A(reinterpret_cast<void **>(&p->r_save), (size_t)npad * ki.nres * sizeof(float));
  A(reinterpret_cast<void **>(&p->ubar), (size_t)npad * ki.dout * ki.C * sizeof(float));
  A(reinterpret_cast<void **>(&p->loss_part), (size_t)(npad / 16) * sizeof(float));
  A(reinterpret_cast<void **>(&p->loss_part64), (size_t)(npad / 16) * sizeof(double));
  p->dw_splits = dw_splits_for(npad, ki.C, w);
  p->dw_splits_max = 2 * p->dw_splits;
  // 16-bit operands: weight gradients fused into the backward layer kernels
  // where the width allows (the faster variant measured on the NS workload)
  p->bwd_fused = (prec != PINN_FP32 && pj::bwd_dw_fused_supported(ki.C, w, prec)) ? 1 : 0;
  p->thin_chunks = (int)std::max<int64_t>(1, npad / 64);
  const size_t part_elems = std::max<size_t>(
      std::max<size_t>((size_t)p->dw_splits_max * ((size_t)w * w + w + ki.dout * w + ki.dout),
                       (size_t)p->thin_chunks * std::max(ki.dout * w + ki.dout, w * ki.din + w)),
      (size_t)(npad / 16) * ((size_t)w * ki.din + w));  // first-layer partials, one per 16-point tile
  A(reinterpret_cast<void **>(&p->part), part_elems * sizeof(float));
  if (e != hipSuccess) {
    delete p;
    if (region && e == hipErrorOutOfMemory)
      return fail(PINN_ERR_CAP, "workspace does not fit the %zu-byte device region", region_cap);
    return fail(e == hipErrorOutOfMemory ? PINN_ERR_NOMEM : PINN_ERR_DEVICE, "workspace allocation: %s",
                hipGetErrorString(e));
  }
  *out = p;
  return PINN_OK;
}

namespace pj_host {

void set_error(const char *msg) { g_err = msg; }

pinn_status plan_region_bytes(const pinn_net *net, const pinn_pde *pde, int64_t max_points, int32_t prec,
                              size_t *bytes) {
  pinn_plan p = nullptr;
  pinn_status st = plan_build(net, pde, max_points, prec, 0, 0, nullptr, 0, true, &p);
  if (st) return st;
  *bytes = p->ws_bytes;
  delete p;
  return PINN_OK;
}

pinn_status plan_create_in_region(const pinn_net *net, const pinn_pde *pde, int64_t max_points, int32_t prec,
                                  void *region, size_t region_bytes, pinn_plan *out) {
  if (!region) return fail(PINN_ERR_ARG, "region is NULL");
  return plan_build(net, pde, max_points, prec, 0, 0, static_cast<char *>(region), region_bytes, false, out);
}

}  // namespace pj_host

extern "C" {

pinn_status pinn_plan_create(const pinn_net *net, const pinn_pde *pde, int64_t max_points,
                             int32_t prec, uint32_t flags, size_t save_cap_bytes, pinn_plan *out) {
  g_err.clear();
  return plan_build(net, pde, max_points, prec, flags, save_cap_bytes, nullptr, 0, false, out);
}

pinn_status pinn_plan_create_modified(const pinn_modified *arch, const pinn_pde *pde, int64_t max_points,
                                      int32_t prec, uint32_t flags, pinn_plan *out) {
  g_err.clear();
  if (!out) return fail(PINN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!arch) return fail(PINN_ERR_ARG, "arch is NULL");
  pinn_status st = check_pde(pde, 0);
  if (st) return st;
  if (!pj::mod_kind_supported(pde->kind))
    return fail(PINN_ERR_UNSUPPORTED, "the modified MLP supports the KS and Burgers kinds (input x_0 periodic)");
  if (prec != PINN_FP32) return fail(PINN_ERR_UNSUPPORTED, "the modified MLP runs with FP32 operands only");
  if (flags) return fail(PINN_ERR_UNSUPPORTED, "the modified MLP takes no flags");
  if (arch->hidden < 2 || arch->hidden > 16) return fail(PINN_ERR_UNSUPPORTED, "hidden = %d outside [2, 16]", arch->hidden);
  if (arch->width < 64 || arch->width > 256 || arch->width % 64)
    return fail(PINN_ERR_UNSUPPORTED, "width %d is not a multiple of 64 in [64, 256]", arch->width);
  if (arch->harmonics < 1 || arch->harmonics > pj::kModMaxHarmonics)
    return fail(PINN_ERR_UNSUPPORTED, "harmonics = %d outside [1, %d]", arch->harmonics, pj::kModMaxHarmonics);
  if (!(arch->period > 0.0) || !std::isfinite(arch->period)) return fail(PINN_ERR_ARG, "period must be positive");
  if (max_points < 1 || max_points > kMaxPoints)
    return fail(PINN_ERR_ARG, "max_points = %lld outside [1, %lld]", (long long)max_points, (long long)kMaxPoints);
  KindInfo ki;
  kind_info(pde->kind, &ki);
  const int H = arch->hidden, w = arch->width, C = ki.C;
  const int64_t npad = round_up(max_points, pj::kPointTile);
  pinn_plan p = new (std::nothrow) pinn_plan_s;
  if (!p) return fail(PINN_ERR_NOMEM, "host allocation failed");
  p->kind = pde->kind;
  p->prec = PINN_FP32;
  p->L = H + 3;
  p->H = H;
  p->w = w;
  p->ki = ki;
  p->max_points = max_points;
  p->npad_max = npad;
  p->arch = 1;
  p->mod_M = arch->harmonics;
  p->mod_de = ki.din - 1 + 2 * arch->harmonics;
  p->mod_period = arch->period;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(PINN_ERR_DEVICE, "no HIP device");
  }
  const size_t stack = (size_t)npad * C * w * sizeof(float);
  hipError_t e = hipSuccess;
  auto A = [&](float **ptr, size_t bytes) {
    void *q = nullptr;
    if (e == hipSuccess) e = p->alloc(&q, bytes);
    *ptr = static_cast<float *>(q);
  };
  A(&p->mU, stack);
  A(&p->mV, stack);
  A(&p->mUbar, stack);
  A(&p->mVbar, stack);
  A(&p->mhbar, stack);
  A(&p->mzbar, stack);
  A(&p->mzb3, 3 * stack);
  A(&p->mE, (size_t)npad * C * p->mod_de * sizeof(float));
  A(&p->mWscratch, (size_t)w * w * sizeof(float));
  p->mh.assign(H + 1, nullptr);
  p->mS.assign(H + 1, nullptr);
  p->mWT.assign(H + 1, nullptr);
  for (int l = 1; l <= H; ++l) A(&p->mh[l], stack);
  for (int l = 2; l <= H; ++l) {
    A(&p->mS[l], stack);
    A(&p->mWT[l], (size_t)w * w * sizeof(float));
  }
  A(&p->u_save, (size_t)npad * ki.dout * C * sizeof(float));
  A(&p->r_save, (size_t)npad * ki.nres * sizeof(float));
  A(&p->ubar, (size_t)npad * ki.dout * C * sizeof(float));
  A(&p->loss_part, (size_t)(npad / 16) * sizeof(float));
  p->dw_splits = dw_splits_for(npad, C, w);
  p->dw_splits_max = p->dw_splits;
  p->thin_chunks = (int)std::max<int64_t>(1, npad / 64);
  const size_t part_elems = std::max<size_t>(
      std::max<size_t>((size_t)p->dw_splits * ((size_t)w * w + w), (size_t)p->thin_chunks * (ki.dout * w + ki.dout)),
      (size_t)3 * p->thin_chunks * ((size_t)w * p->mod_de + w));
  A(&p->part, part_elems * sizeof(float));
  if (e != hipSuccess) {
    delete p;
    return fail(e == hipErrorOutOfMemory ? PINN_ERR_NOMEM : PINN_ERR_DEVICE, "workspace allocation: %s",
                hipGetErrorString(e));
  }
  p->saved_bytes = (size_t)(2 * H + 1) * stack;
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
  if (kernel_class < 0 || kernel_class > PINN_K_BWD_DW)
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
  plan->have_seg = false;
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
  plan->have_seg = false;
  st = run_forward(plan, net, pde, x, N, jets, r, loss, loss_f64, true, (hipStream_t)stream);
  if (st) return st;
  plan->have_state = true;
  plan->st_N = N;
  plan->st_x = x;
  plan->st_W.assign(net->W, net->W + net->n_layers);
  plan->st_b.assign(net->b, net->b + net->n_layers);
  return PINN_OK;
}

}  // extern "C"

namespace {

// Forward pass of a modified-MLP plan: embedding and encoders, the gated
// layers, then the plain path's output layer, residual and loss partials.
pinn_status mod_forward(pinn_plan p, const pinn_net *net, const pinn_pde *pde, const float *x, int64_t N,
                        float *jets, float *r, float *loss, hipStream_t st) {
  const int64_t npad = round_up(N, pj::kPointTile);
  const int H = p->H, L = p->L, w = p->w;
  pinn_pde dflt{};
  if (!pde) {
    dflt.kind = p->kind;
    dflt.coef[0] = 1.0;
    pde = &dflt;
  }
  pj::ModArgs m{x, N, npad, w, p->mod_M, p->mod_de, (float)(2.0 * M_PI / p->mod_period),
                net->W[0], net->b[0], net->W[1], net->b[1], net->W[2], net->b[2], p->mU, p->mV, p->mh[1]};
  hipError_t e = timed(p, PINN_K_SEED_FWD, st, [&] { return pj::launch_mod_enc(p->kind, m, st); });
  if (e) return hip_fail(e, "embedding and encoders");
  for (int l = 2; l <= H; ++l) {
    e = timed(p, PINN_K_LAYER_FWD, st, [&] { return pj::launch_mod_layer(p->kind, p->mh[l - 1], net->W[l + 1], net->b[l + 1], p->mU, p->mV, p->mh[l], p->mS[l], npad, w, st); });
    if (e) return hip_fail(e, "gated layer");
  }
  e = timed(p, PINN_K_OUT_FWD, st, [&] { return pj::launch_out_fwd(p->kind, PINN_FP32, p->mh[H], net->W[L - 1], net->b[L - 1], x, N, npad, w, coef_of(pde), jets, r, p->u_save, p->r_save, p->loss_part, nullptr, st); });
  if (e) return hip_fail(e, "output layer");
  if (loss) {
    e = timed(p, PINN_K_OTHER, st, [&] { return pj::launch_loss_reduce(p->loss_part, nullptr, (int)(npad / 16), 1.0 / (double)N, loss, nullptr, st); });
    if (e) return hip_fail(e, "loss reduction");
  }
  return PINN_OK;
}

// Backward pass of a modified-MLP plan from the output cotangent in p->ubar
// (scaled by 1 / inv_s): output layer, the gated layers top down (their weight
// gradients by the split-K kernel, the stack below through W^T), then the
// first layer and the two encoders.
pinn_status mod_backward(pinn_plan p, const pinn_net *net, const float *x, int64_t N, float *const *dW,
                         float *const *db, float inv_s, hipStream_t s) {
  const int64_t npad = round_up(N, pj::kPointTile);
  const int H = p->H, L = p->L, w = p->w, C = p->ki.C, dout = p->ki.dout, de = p->mod_de;
  hipError_t e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_dw_out(p->kind, PINN_FP32, p->ubar, p->mh[H], npad, w, p->part, p->thin_chunks, s); });
  if (e) return hip_fail(e, "output-layer gradient");
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->thin_chunks, (int64_t)dout * w + dout, (int64_t)dout * w, dout, dW[L - 1], db[L - 1], nullptr, nullptr, s, inv_s); });
  if (e) return hip_fail(e, "reduction");
  for (int l = H; l >= 2; --l) {
    e = timed(p, PINN_K_LAYER_BWD, s, [&] { return pj::launch_mod_gate_bwd(p->kind, l == H, p->mhbar, p->ubar, net->W[L - 1], p->mS[l], p->mU, p->mV, p->mUbar, p->mVbar, p->mzbar, npad, w, s); });
    if (e) return hip_fail(e, "gated-layer adjoint");
    e = timed(p, PINN_K_DW_HIDDEN, s, [&] { return pj::launch_dw_hidden(PINN_FP32, C, p->mzbar, p->mh[l - 1], npad, w, p->part, p->part + (size_t)w * w, p->dw_splits, s); });
    if (e) return hip_fail(e, "gated-layer gradient");
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->dw_splits, (int64_t)w * w + w, (int64_t)w * w, w, dW[l + 1], db[l + 1], nullptr, nullptr, s, inv_s); });
    if (e) return hip_fail(e, "reduction");
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_cast(PINN_FP32, net->W[l + 1], w, w, p->mWscratch, p->mWT[l], s); });
    if (e) return hip_fail(e, "transpose");
    e = timed(p, PINN_K_LAYER_BWD, s, [&] { return pj::launch_mod_abar(p->kind, p->mWT[l], p->mzbar, p->mhbar, npad, w, s); });
    if (e) return hip_fail(e, "gated-layer input adjoint");
  }
  pj::ModArgs m{x, N, npad, w, p->mod_M, de, (float)(2.0 * M_PI / p->mod_period),
                net->W[0], net->b[0], net->W[1], net->b[1], net->W[2], net->b[2], nullptr, nullptr, nullptr};
  e = timed(p, PINN_K_LAYER_BWD, s, [&] { return pj::launch_mod_enc_bwd(p->kind, m, p->mhbar, p->mUbar, p->mVbar, p->mzb3, p->mE, s); });
  if (e) return hip_fail(e, "encoder adjoint");
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_mod_dw_enc(p->kind, p->mzb3, p->mE, p->part, npad, w, de, p->thin_chunks, s); });
  if (e) return hip_fail(e, "encoder gradients");
  const int64_t stride = (int64_t)w * de + w;
  const int dst[3] = {2, 0, 1};  // zb3 holds h_1, U, V
  for (int q = 0; q < 3; ++q) {
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part + (size_t)q * p->thin_chunks * stride, p->thin_chunks, stride, (int64_t)w * de, w, dW[dst[q]], db[dst[q]], nullptr, nullptr, s, inv_s); });
    if (e) return hip_fail(e, "reduction");
  }
  return PINN_OK;
}

}  // namespace

// The backward pass for the cotangent rbar = r_bar + lb 2 r / N, with lb =
// *loss_bar, or lb = 1 when both are null (see pinn_jet_backward_cot).
// The layer description with the plan's wide-kernel tiling.
static pj::LayerBwd with_points(pj::LayerBwd B, pinn_plan p) {
  B.points = p->bwd_points;
  return B;
}

static pinn_status backward_impl(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                                 int64_t N, const float *r_bar, const float *loss_bar, float *const *dW,
                                 float *const *db, double *const *dW_f64, double *const *db_f64,
                                 void *stream, bool segments = false) {
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
  // The loss cotangent 2 r / N is scaled by S, the largest power of two not
  // above N / 2, so that the backward stacks hold values of the order of r:
  // with FP16 operands the unscaled cotangents fall below the normal range at
  // large N.  Every backward step is linear in the cotangent and power-of-two
  // scaling adds no rounding, so the reductions take out 1/S exactly and FP32
  // and BF16 results are those of the unscaled arithmetic.  An explicit r_bar
  // is used as given.
  double cot_scale = 1.0;
  if (segments) {
    cot_scale = p->seg_scale;  // chosen with the segments' weights and sizes
  } else if (!r_bar) {
    while (4.0 * cot_scale <= (double)N) cot_scale *= 2.0;
  }
  const float rbar_scale = (float)(2.0 * cot_scale / (double)N);
  const float inv_s = (float)(1.0 / cot_scale);
  // the cotangent at the outputs: the residual adjoint, or the segments'
  auto output_adjoint = [&]() -> hipError_t {
    if (segments)
      return timed(p, PINN_K_OUT_BWD, s, [&] { return pj::launch_seg_adj(p->kind, p->seg, p->u_save, p->r_save, x, npad, coef_of(pde), p->ubar, s); });
    return timed(p, PINN_K_OUT_BWD, s, [&] { return pj::launch_out_adj(p->kind, p->u_save, p->r_save, r_bar, loss_bar, N, npad, rbar_scale, coef_of(pde), p->ubar, s); });
  };
  if (p->arch) {
    const hipError_t e0 = output_adjoint();
    if (e0) return hip_fail(e0, "output adjoint");
    return mod_backward(p, net, x, N, dW, db, inv_s, s);
  }
  hipError_t e;
  // the operand-type weights W and W^T were made by the residual call
  pinn_status rs = PINN_OK;
  // Source of z for the adjoint of activation layer m: the saved state, or a
  // recompute from the stack of layer m - 1 (m >= 2) or from x (m = 1).
  auto zsrc = [&](pj::LayerBwd &B, int m) -> pinn_status {
    if (m == 1) B.x = x;  // also the inputs of the first layer's gradient
    if (p->store_S) {
      B.S_in = p->S[m];
    } else if (m >= 2) {
      const void *Am1 = nullptr;
      pinn_status r2 = backward_stack(p, net, x, N, npad, m - 1, &Am1, s);
      if (r2) return r2;
      B.A_prev = Am1;
      B.Wz = p->Wop[m];
      B.bz = net->b[m - 1];
    } else {
      B.x = x;
      B.W1 = net->W[0];
      B.bz = net->b[0];
    }
    return PINN_OK;
  };
  const bool fused = backward_fused(p);
  // layer 1's adjoint kernel also yields the first layer's gradient (H >= 2:
  // layer 1 is then a hidden-layer adjoint from zbar_2, not the top layer)
  const bool seed_fused = H >= 2 && pj::seed_grad_fused_supported(ki.C, w, p->prec);
  if (fused) {
    // Each backward layer kernel also produces the weight gradient of the
    // layer whose zbar it computes: dW_m from zbar_m and the stack of m - 1.
    // persistent workgroups, one weight-gradient partial each: twice the split
    // count (the default split count gives the partial buffer's capacity)
    const int grid = (int)std::min<int64_t>(std::min<int64_t>(npad / 16, std::min(2 * p->dw_splits, p->dw_splits_max)), 512);
    e = output_adjoint();
    if (e) return hip_fail(e, "output adjoint");
    auto layer = [&](pj::LayerBwd &B, int m, int cls) -> pinn_status {
      const void *Am1 = nullptr;
      pinn_status r2 = backward_stack(p, net, x, N, npad, m - 1, &Am1, s);
      if (r2) return r2;
      B.A_prev = Am1;
      if (p->store_S) {
        B.S_in = p->S[m];
      } else {
        B.Wz = p->Wop[m];
        B.bz = net->b[m - 1];
      }
      B.N = N;
      B.w = w;
      B.Zb_out = p->Zb[m % 2];
      hipError_t e2 = timed(p, cls, s, [&] { return pj::launch_bwd_dw(p->kind, p->prec, B, p->part, npad, grid, s); });
      if (e2) return hip_fail(e2, "backward layer");
      e2 = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, grid, (int64_t)w * w + w, (int64_t)w * w, w, dW[m - 1], db[m - 1], f64(dW_f64, m - 1), f64(db_f64, m - 1), s, inv_s); });
      return e2 ? hip_fail(e2, "reduction") : PINN_OK;
    };
    // the top layer's kernel also forms the output layer's gradient partials
    // where it is the double-buffered one (after the top layer's own partials)
    const bool out_fused = top_forms_out_grad(p);
    float *out_part = out_fused ? p->part + (size_t)grid * ((size_t)w * w + w) : nullptr;
    {
      pj::LayerBwd B{};
      B.top = true;
      B.ubar = p->ubar;
      B.WL = net->W[L - 1];
      B.out_part = out_part;
      rs = layer(B, H, PINN_K_OUT_BWD);
      if (rs) return rs;
    }
    if (out_fused) {
      e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(out_part, grid, (int64_t)ki.dout * w + ki.dout, (int64_t)ki.dout * w, ki.dout, dW[L - 1], db[L - 1], f64(dW_f64, L - 1), f64(db_f64, L - 1), s, inv_s); });
      if (e) return hip_fail(e, "reduction");
    } else {
      const void *AH = nullptr;
      rs = backward_stack(p, net, x, N, npad, H, &AH, s);
      if (rs) return rs;
      e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_dw_out(p->kind, p->prec, p->ubar, AH, npad, w, p->part, p->thin_chunks, s); });
      if (e) return hip_fail(e, "output-layer gradient");
      e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->thin_chunks, (int64_t)ki.dout * w + ki.dout, (int64_t)ki.dout * w, ki.dout, dW[L - 1], db[L - 1], f64(dW_f64, L - 1), f64(db_f64, L - 1), s, inv_s); });
      if (e) return hip_fail(e, "reduction");
    }
    for (int l = H; l >= 3; --l) {
      pj::LayerBwd B{};
      B.top = false;
      B.Zb_in = p->Zb[l % 2];
      B.WT = p->WTop[l];
      rs = layer(B, l - 1, PINN_K_BWD_DW);
      if (rs) return rs;
    }
    // zbar of layer 1 (its z comes from x; its gradient is the thin seed kernel's)
    pj::LayerBwd B{};
    B.top = false;
    B.Zb_in = p->Zb[0];
    B.WT = p->WTop[2];
    B.N = N;
    B.w = w;
    B.Zb_out = p->Zb[1];
    B.seed_part = seed_fused ? p->part : nullptr;
    rs = zsrc(B, 1);
    if (rs) return rs;
    e = timed(p, PINN_K_LAYER_BWD, s, [&] { return pj::launch_layer_bwd(p->kind, p->prec, with_points(B, p), npad, s); });
    if (e) return hip_fail(e, "hidden adjoint");
  } else {
  // Output layer: ubar, then zbar of layer H, then dW_L, db_L.
  e = output_adjoint();
  if (e) return hip_fail(e, "output adjoint");
  // the wide top layer's kernel also forms the output layer's gradient
  // partials (one per workgroup's sixteen tiles) where it is the streaming
  // 256-wide one
  const bool out_wide = top_forms_out_grad(p);
  {
    pj::LayerBwd B{};
    B.top = true;
    B.ubar = p->ubar;
    B.WL = net->W[L - 1];
    B.N = N;
    B.w = w;
    B.Zb_out = p->Zb[H % 2];
    B.out_part = out_wide ? p->part : nullptr;
    rs = zsrc(B, H);
    if (rs) return rs;
    e = timed(p, PINN_K_OUT_BWD, s, [&] { return pj::launch_layer_bwd(p->kind, p->prec, with_points(B, p), npad, s); });
    if (e) return hip_fail(e, "last hidden adjoint");
  }
  if (out_wide) {
    // one reduction variant for every point count, so that the networks of
    // an ensemble lane group into one launch here
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, (int)pj::wide_top_out_grad_parts(npad), (int64_t)w + 1, w, 1, dW[L - 1], db[L - 1], f64(dW_f64, L - 1), f64(db_f64, L - 1), s, inv_s, 64); });
    if (e) return hip_fail(e, "reduction");
  } else {
    const void *AH = nullptr;
    rs = backward_stack(p, net, x, N, npad, H, &AH, s);
    if (rs) return rs;
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_dw_out(p->kind, p->prec, p->ubar, AH, npad, w, p->part, p->thin_chunks, s); });
    if (e) return hip_fail(e, "output-layer gradient");
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->thin_chunks, (int64_t)ki.dout * w + ki.dout,
                                 (int64_t)ki.dout * w, ki.dout, dW[L - 1], db[L - 1], f64(dW_f64, L - 1),
                                 f64(db_f64, L - 1), s, inv_s); });
    if (e) return hip_fail(e, "reduction");
  }
  // Hidden layers H..2: dW_l, db_l from zbar_l and the stack of layer l - 1,
  // then zbar of layer l - 1.
  for (int l = H; l >= 2; --l) {
    void *cur = p->Zb[l % 2], *prev = p->Zb[(l - 1) % 2];
    const void *Al1 = nullptr;
    rs = backward_stack(p, net, x, N, npad, l - 1, &Al1, s);
    if (rs) return rs;
    e = timed(p, PINN_K_DW_HIDDEN, s, [&] { return pj::launch_dw_hidden(p->prec, ki.C, cur, Al1, npad, w, p->part, p->part + (size_t)w * w, p->dw_splits, s); });
    if (e) return hip_fail(e, "hidden-layer gradient");
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->dw_splits, (int64_t)w * w + w, (int64_t)w * w, w, dW[l - 1], db[l - 1], f64(dW_f64, l - 1), f64(db_f64, l - 1), s, inv_s); });
    if (e) return hip_fail(e, "reduction");
    pj::LayerBwd B{};
    B.top = false;
    B.Zb_in = cur;
    B.WT = p->WTop[l];
    B.N = N;
    B.w = w;
    B.Zb_out = prev;
    B.seed_part = (l == 2 && seed_fused) ? p->part : nullptr;
    rs = zsrc(B, l - 1);
    if (rs) return rs;
    e = timed(p, PINN_K_LAYER_BWD, s, [&] { return pj::launch_layer_bwd(p->kind, p->prec, with_points(B, p), npad, s); });
    if (e) return hip_fail(e, "hidden adjoint");
  }
  }
  // First layer: its gradient partials came out of the layer-1 adjoint kernel
  // (one per 16-point tile), or the separate kernel sums them from zbar_1.
  if (seed_fused) {
    e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, (int)(npad / 16), (int64_t)w * ki.din + w, (int64_t)w * ki.din, w,
                                 dW[0], db[0], f64(dW_f64, 0), f64(db_f64, 0), s, inv_s); });
    if (e) return hip_fail(e, "reduction");
    return PINN_OK;
  }
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_dw_seed(p->kind, p->prec, p->Zb[1], x, N, npad, w, p->part, p->thin_chunks, s); });
  if (e) return hip_fail(e, "first-layer gradient");
  e = timed(p, PINN_K_OTHER, s, [&] { return pj::launch_reduce_parts2(p->part, p->thin_chunks, (int64_t)w * ki.din + w, (int64_t)w * ki.din, w,
                               dW[0], db[0], f64(dW_f64, 0), f64(db_f64, 0), s, inv_s); });
  if (e) return hip_fail(e, "reduction");
  return PINN_OK;
}


extern "C" {

pinn_status pinn_jet_backward(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                              const float *x, int64_t N, const float *r_bar, float *const *dW,
                              float *const *db, double *const *dW_f64, double *const *db_f64,
                              void *stream) {
  g_err.clear();
  return backward_impl(plan, net, pde, x, N, r_bar, nullptr, dW, db, dW_f64, db_f64, stream);
}

pinn_status pinn_jet_backward_cot(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                                  int64_t N, const float *r_bar, const float *loss_bar, float *const *dW,
                                  float *const *db, double *const *dW_f64, double *const *db_f64,
                                  void *stream) {
  g_err.clear();
  return backward_impl(plan, net, pde, x, N, r_bar, loss_bar, dW, db, dW_f64, db_f64, stream);
}

}  // extern "C"

// Checks a segment list against the plan and N and packs it for the kernels:
// units, the cotangent scale S (a power of two that brings the largest
// per-unit cotangent weight * 2 / units to at most 1) and the loss kernel's
// workgroup ranges.
static pinn_status seg_pack(pinn_plan p, const pinn_segment *segs, int32_t n_seg, int64_t N, pj::SegPack *sp,
                            double *scale) {
  if (!segs) return fail(PINN_ERR_ARG, "segments is NULL");
  if (n_seg < 1 || n_seg > pj::kMaxSegments)
    return fail(PINN_ERR_ARG, "n_segments = %d outside [1, %d]", n_seg, pj::kMaxSegments);
  const int C = p->ki.C, dout = p->ki.dout;
  const uint64_t all_bits = (uint64_t(1) << (dout * C)) - 1;
  *sp = pj::SegPack{};
  sp->n = n_seg;
  double ratio = 1e300;  // min over segments of units / (2 weight)
  int blk = 0;
  for (int s = 0; s < n_seg; ++s) {
    const pinn_segment &g = segs[s];
    if (g.begin < 0 || g.count < 1 || g.begin + g.count > N)
      return fail(PINN_ERR_ARG, "segment %d: points [%lld, %lld) outside [0, N = %lld)", s, (long long)g.begin,
                  (long long)(g.begin + g.count), (long long)N);
    if (!std::isfinite(g.weight) || g.weight < 0.0) return fail(PINN_ERR_ARG, "segment %d: bad weight", s);
    for (int q = 0; q < 4; ++q)
      if (!std::isfinite(g.param[q])) return fail(PINN_ERR_ARG, "segment %d: parameter %d not finite", s, q);
    for (int t = 0; t < s; ++t)
      if (g.begin < segs[t].begin + segs[t].count && segs[t].begin < g.begin + g.count)
        return fail(PINN_ERR_ARG, "segments %d and %d overlap", t, s);
    int64_t units = g.count;
    switch (g.type) {
      case PINN_SEG_PDE: break;
      case PINN_SEG_DIRICHLET:
        if (g.data != PINN_DATA_ZERO && g.data != PINN_DATA_CONST && g.data != PINN_DATA_SIN &&
            g.data != PINN_DATA_VALUES)
          return fail(PINN_ERR_ARG, "segment %d: unknown data function %d", s, g.data);
        if (g.data == PINN_DATA_VALUES && !g.values)
          return fail(PINN_ERR_ARG, "segment %d: PINN_DATA_VALUES without values", s);
        if (g.mask == 0 || (uint64_t)g.mask > all_bits) return fail(PINN_ERR_ARG, "segment %d: bad mask", s);
        for (int q = 0; q < dout * C; ++q)
          if ((g.mask >> q & 1u) && q % C != 0)
            return fail(PINN_ERR_ARG, "segment %d: a data term constrains output values (channel 0) only", s);
        break;
      case PINN_SEG_PERIODIC:
        if (g.count % 2 != 0) return fail(PINN_ERR_ARG, "segment %d: periodic pairs need an even count", s);
        if (g.mask == 0 || (uint64_t)g.mask > all_bits) return fail(PINN_ERR_ARG, "segment %d: bad mask", s);
        units = g.count / 2;
        break;
      default: return fail(PINN_ERR_ARG, "segment %d: unknown type %d", s, g.type);
    }
    sp->type[s] = g.type;
    sp->data[s] = g.data;
    sp->begin[s] = g.begin;
    sp->count[s] = g.count;
    sp->weight[s] = (float)g.weight;
    sp->mask[s] = g.mask;
    for (int q = 0; q < 4; ++q) sp->param[s][q] = (float)g.param[q];
    sp->values[s] = g.type == PINN_SEG_DIRICHLET && g.data == PINN_DATA_VALUES ? g.values : nullptr;
    sp->blk_start[s] = blk;
    blk += (int)((units + 255) / 256);
    if (g.weight > 0.0) ratio = std::min(ratio, (double)units / (2.0 * g.weight));
  }
  sp->blk_start[n_seg] = blk;
  double S = 1.0;
  if (ratio < 1e300) {
    while (S * 2.0 <= ratio && S < 0x1p30) S *= 2.0;
    while (S > ratio && S > 0x1p-30) S *= 0.5;
  }
  for (int s = 0; s < n_seg; ++s) {
    const double units = segs[s].type == PINN_SEG_PERIODIC ? segs[s].count / 2 : segs[s].count;
    sp->cot[s] = (float)(S * segs[s].weight * 2.0 / units);
  }
  *scale = S;
  return PINN_OK;
}

extern "C" {

pinn_status pinn_jet_loss(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const pinn_segment *segs,
                          int32_t n_seg, const float *x, int64_t N, float *loss, float *seg_loss, void *stream) {
  g_err.clear();
  pinn_status st = check_call(plan, net, x, N);
  if (st) return st;
  st = check_pde(pde, plan->kind);
  if (st) return st;
  pj::SegPack sp;
  double S = 1.0;
  st = seg_pack(plan, segs, n_seg, N, &sp, &S);
  if (st) return st;
  // the loss partials (one per 256 units, at most N / 256 + 8) use the
  // gradient partial buffer, which holds at least 6 floats per point
  plan->have_state = false;
  plan->have_seg = false;
  hipStream_t s = (hipStream_t)stream;
  st = run_forward(plan, net, pde, x, N, nullptr, nullptr, nullptr, nullptr, true, s);
  if (st) return st;
  const int64_t npad = round_up(N, pj::kPointTile);
  hipError_t e = timed(plan, PINN_K_OTHER, s, [&] { return pj::launch_seg_loss(plan->kind, sp, plan->u_save, plan->r_save, x, npad, plan->part, seg_loss, loss, s); });
  if (e) return hip_fail(e, "segment loss");
  plan->have_state = true;
  plan->st_N = N;
  plan->st_x = x;
  plan->st_W.assign(net->W, net->W + net->n_layers);
  plan->st_b.assign(net->b, net->b + net->n_layers);
  plan->have_seg = true;
  plan->seg = sp;
  plan->seg_scale = S;
  return PINN_OK;
}

pinn_status pinn_jet_loss_backward(pinn_plan plan, const pinn_net *net, const pinn_pde *pde,
                                   const pinn_segment *segs, int32_t n_seg, const float *x, int64_t N,
                                   float *const *dW, float *const *db, void *stream) {
  g_err.clear();
  if (!plan) return fail(PINN_ERR_ARG, "plan is NULL");
  pj::SegPack sp;
  double S = 1.0;
  pinn_status st = seg_pack(plan, segs, n_seg, N, &sp, &S);
  if (st) return st;
  if (!plan->have_seg || std::memcmp(&sp, &plan->seg, sizeof sp) != 0)
    return fail(PINN_ERR_STATE, "loss backward does not follow pinn_jet_loss with the same segments");
  return backward_impl(plan, net, pde, x, N, nullptr, nullptr, dW, db, nullptr, nullptr, stream, true);
}

pinn_status pinn_plan_get_tuning(pinn_plan plan, pinn_tuning *t) {
  g_err.clear();
  if (!plan || !t) return fail(PINN_ERR_ARG, "plan or tuning is NULL");
  t->dw_splits = plan->dw_splits;
  t->fwd_points = plan->fwd_points;
  t->bwd_fused = plan->bwd_fused;
  t->bwd_points = plan->bwd_points;
  return PINN_OK;
}

pinn_status pinn_plan_set_tuning(pinn_plan plan, const pinn_tuning *t) {
  g_err.clear();
  if (!plan || !t) return fail(PINN_ERR_ARG, "plan or tuning is NULL");
  if (t->dw_splits < 1 || t->dw_splits > plan->dw_splits_max)
    return fail(PINN_ERR_ARG, "dw_splits = %d outside [1, %d]", t->dw_splits, plan->dw_splits_max);
  if (t->fwd_points != 0 && !pj::fused_fwd_fits(t->fwd_points, plan->ki.C, plan->w, plan->prec))
    return fail(PINN_ERR_ARG, "fwd_points = %d has no fused forward tiling at this width", t->fwd_points);
  if (t->bwd_fused != 0 && t->bwd_fused != 1) return fail(PINN_ERR_ARG, "bwd_fused must be 0 or 1");
  if (t->bwd_points != 0 && !pj::wide_bwd_points_supported(t->bwd_points, plan->ki.C, plan->w, plan->prec))
    return fail(PINN_ERR_ARG, "bwd_points = %d has no wide backward tiling at this width", t->bwd_points);
  plan->dw_splits = t->dw_splits;
  plan->fwd_points = t->fwd_points;
  plan->bwd_fused = t->bwd_fused;
  plan->bwd_points = t->bwd_points;
  plan->have_state = false;
  return PINN_OK;
}

}  // extern "C"

// Tuning cache: the autotuner's choice per (device architecture, PDE kind,
// operand type, width, depth, point-count bucket ceil(log2 N)).  The split
// count is kept relative to the plan's default (the candidates are half,
// once and twice the default), so an entry applies to every N of its bucket.
namespace {
struct TuneKey {
  std::string arch;
  int kind, prec, w, H, nbucket;
  bool operator<(const TuneKey &o) const {
    return std::tie(arch, kind, prec, w, H, nbucket) < std::tie(o.arch, o.kind, o.prec, o.w, o.H, o.nbucket);
  }
};
struct TuneVal {
  int split_mode;  // 0: half the default split count, 1: the default, 2: twice
  int fwd_points, bwd_fused;
  double ms;
  int bwd_points;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

std::string device_arch(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}

TuneKey tune_key(pinn_plan p, int64_t N) {
  int nb = 0;
  while ((int64_t(1) << nb) < N) ++nb;
  return TuneKey{device_arch(p->device), p->kind, p->prec, p->w, p->H, nb};
}
}  // namespace

extern "C" {

pinn_status pinn_plan_autotune(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                               int64_t N, int32_t reps, pinn_tuning *best, double *best_ms, void *stream) {
  g_err.clear();
  if (plan && plan->arch) return fail(PINN_ERR_UNSUPPORTED, "a modified-MLP plan has no tunings");
  pinn_status st = check_call(plan, net, x, N);
  if (st) return st;
  st = check_pde(pde, plan->kind);
  if (st) return st;
  if (reps < 1 || reps > 1000) return fail(PINN_ERR_ARG, "reps = %d outside [1, 1000]", reps);
  hipStream_t s = (hipStream_t)stream;
  pinn_plan p = plan;
  const TuneKey tk = tune_key(p, N);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(tk);
    if (it != g_tune.end()) {  // cached: apply without timing
      const int s0 = dw_splits_for(round_up(N, pj::kPointTile), p->ki.C, p->w);
      const int sp = it->second.split_mode == 0 ? std::max(1, s0 / 2)
                                                : (it->second.split_mode == 1 ? s0 : std::min(p->dw_splits_max, 2 * s0));
      p->dw_splits = std::max(1, std::min(sp, p->dw_splits_max));
      p->fwd_points = pj::fused_fwd_fits(it->second.fwd_points, p->ki.C, p->w, p->prec) ? it->second.fwd_points : 0;
      p->bwd_fused = it->second.bwd_fused && pj::bwd_dw_fused_supported(p->ki.C, p->w, p->prec) ? 1 : 0;
      p->bwd_points =
          pj::wide_bwd_points_supported(it->second.bwd_points, p->ki.C, p->w, p->prec) ? it->second.bwd_points : 0;
      p->have_state = false;
      if (best) *best = pinn_tuning{p->dw_splits, p->fwd_points, p->bwd_fused, p->bwd_points};
      if (best_ms) *best_ms = it->second.ms;
      return PINN_OK;
    }
  }
  // gradient outputs for the trial steps
  std::vector<void *> bufs;
  std::vector<float *> dW(p->L), db(p->L);
  hipError_t e = hipSuccess;
  for (int l = 0; l < p->L && e == hipSuccess; ++l) {
    void *a = nullptr, *b = nullptr;
    e = hipMalloc(&a, (size_t)net->dims[l] * net->dims[l + 1] * sizeof(float));
    if (e == hipSuccess) bufs.push_back(a), e = hipMalloc(&b, (size_t)net->dims[l + 1] * sizeof(float));
    if (e == hipSuccess) bufs.push_back(b);
    dW[l] = (float *)a;
    db[l] = (float *)b;
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  auto cleanup = [&]() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    for (void *q : bufs) (void)hipFree(q);
  };
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "autotune setup");
  }
  const pinn_tuning orig{p->dw_splits, p->fwd_points, p->bwd_fused, p->bwd_points};
  const int s0 = dw_splits_for(round_up(N, pj::kPointTile), p->ki.C, p->w);
  std::vector<pinn_tuning> cand;
  const bool can_fuse = pj::bwd_dw_fused_supported(p->ki.C, p->w, p->prec);
  for (int sp : {std::max(1, s0 / 2), s0, std::min(p->dw_splits_max, 2 * s0)})
    for (int fp : {0, 16, 32, 64})
    for (int bf : {0, 1})
    for (int bp : {0, 32, 64, 256}) {  // 16 (double-buffered) measured slower at 4 and 6 channels
      // 0 (layer-by-layer forward) only when no whole-network tiling exists
      const bool any_fused = pj::fused_fwd_points(p->ki.C, p->w, p->prec) > 0;
      if (fp == 0 ? any_fused : !pj::fused_fwd_fits(fp, p->ki.C, p->w, p->prec)) continue;
      if (bf == 1 && !can_fuse) continue;
      if (bp != 0 && !pj::wide_bwd_points_supported(bp, p->ki.C, p->w, p->prec)) continue;
      pinn_tuning t{sp, fp, bf, bp};
      bool dup = false;
      for (auto &c : cand)
        dup = dup || (c.dw_splits == t.dw_splits && c.fwd_points == t.fwd_points && c.bwd_fused == t.bwd_fused &&
                      c.bwd_points == t.bwd_points);
      if (!dup) cand.push_back(t);
    }
  // two interleaved timing rounds; a candidate's time is its faster round
  std::vector<double> cms(cand.size(), 1e300);
  for (int round = 0; round < 2 && st == PINN_OK && e == hipSuccess; ++round) {
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const pinn_tuning &c = cand[ci];
      p->dw_splits = c.dw_splits;
      p->fwd_points = c.fwd_points;
      p->bwd_fused = c.bwd_fused;
      p->bwd_points = c.bwd_points;
      for (int it = -1; it < reps && st == PINN_OK; ++it) {
        if (it == 0) e = hipEventRecord(t0, s);
        st = pinn_jet_residual(p, net, pde, x, N, nullptr, nullptr, nullptr, nullptr, stream);
        if (st == PINN_OK)
          st = pinn_jet_backward(p, net, pde, x, N, nullptr, dW.data(), db.data(), nullptr, nullptr, stream);
      }
      if (st != PINN_OK) break;
      e = hipEventRecord(t1, s);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e != hipSuccess) break;
      cms[ci] = std::min(cms[ci], (double)ms / reps);
    }
  }
  double bms = 1e300;
  pinn_tuning bt = orig;
  for (size_t ci = 0; ci < cand.size(); ++ci)
    if (cms[ci] < bms) {
      bms = cms[ci];
      bt = cand[ci];
    }
  cleanup();
  if (st != PINN_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "autotune timing");
  p->dw_splits = bt.dw_splits;
  p->fwd_points = bt.fwd_points;
  p->bwd_fused = bt.bwd_fused;
  p->bwd_points = bt.bwd_points;
  p->have_state = false;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[tk] = TuneVal{bt.dw_splits < s0 ? 0 : (bt.dw_splits == s0 ? 1 : 2), bt.fwd_points, bt.bwd_fused, bms,
                         bt.bwd_points};
  }
  if (best) *best = bt;
  if (best_ms) *best_ms = bms;
  return PINN_OK;
}

pinn_status pinn_tuning_cache_clear(void) {
  g_err.clear();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  return PINN_OK;
}

pinn_status pinn_tuning_cache_size(int64_t *entries) {
  g_err.clear();
  if (!entries) return fail(PINN_ERR_ARG, "entries is NULL");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  *entries = (int64_t)g_tune.size();
  return PINN_OK;
}

pinn_status pinn_tuning_cache_save(const char *path) {
  g_err.clear();
  if (!path) return fail(PINN_ERR_ARG, "path is NULL");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  FILE *f = fopen(path, "w");
  if (!f) return fail(PINN_ERR_ARG, "cannot write %s", path);
  fprintf(f, "# pinn tuning cache v2: arch kind prec w H nbucket split_mode fwd_points bwd_fused ms bwd_points\n");
  for (const auto &kv : g_tune)
    fprintf(f, "%s %d %d %d %d %d %d %d %d %.6g %d\n", kv.first.arch.c_str(), kv.first.kind, kv.first.prec,
            kv.first.w, kv.first.H, kv.first.nbucket, kv.second.split_mode, kv.second.fwd_points,
            kv.second.bwd_fused, kv.second.ms, kv.second.bwd_points);
  const bool ok = fclose(f) == 0;
  return ok ? PINN_OK : fail(PINN_ERR_ARG, "cannot write %s", path);
}

pinn_status pinn_tuning_cache_load(const char *path) {
  g_err.clear();
  if (!path) return fail(PINN_ERR_ARG, "path is NULL");
  FILE *f = fopen(path, "r");
  if (!f) return fail(PINN_ERR_ARG, "cannot read %s", path);
  std::map<TuneKey, TuneVal> got;
  char line[512];
  int lineno = 0;
  while (fgets(line, sizeof line, f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    char arch[64];
    TuneKey k;
    TuneVal v;
    v.bwd_points = 0;  // v1 lines have no wide-backward column
    const int got_n = sscanf(line, "%63s %d %d %d %d %d %d %d %d %lf %d", arch, &k.kind, &k.prec, &k.w, &k.H,
                             &k.nbucket, &v.split_mode, &v.fwd_points, &v.bwd_fused, &v.ms, &v.bwd_points);
    if ((got_n != 10 && got_n != 11) || v.split_mode < 0 || v.split_mode > 2 || (v.bwd_fused != 0 && v.bwd_fused != 1) ||
        (v.bwd_points != 0 && v.bwd_points != 16 && v.bwd_points != 32 && v.bwd_points != 64 &&
         v.bwd_points != 256)) {
      fclose(f);
      return fail(PINN_ERR_ARG, "%s:%d: malformed tuning cache entry", path, lineno);
    }
    k.arch = arch;
    got[k] = v;
  }
  fclose(f);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const auto &kv : got) g_tune[kv.first] = kv.second;
  return PINN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adam step over all parameters of a network.
// ---------------------------------------------------------------------------
// Validates the Adam arguments and fills the kernel argument block.
static pinn_status adam_args(int32_t n_layers, const int32_t *dims, float *const *W, float *const *b,
                             const float *const *dW, const float *const *db, float *const *mW, float *const *vW,
                             float *const *mb, float *const *vb, const pinn_adam *hp, pj::AdamArgs *a) {
  if (n_layers < 1 || 2 * n_layers > pj::kAdamSegs)
    return fail(PINN_ERR_ARG, "n_layers = %d outside [1, %d]", n_layers, pj::kAdamSegs / 2);
  if (!dims || !W || !b || !dW || !db || !mW || !vW || !mb || !vb || !hp)
    return fail(PINN_ERR_ARG, "NULL argument");
  if (!(hp->lr > 0.0) || !(hp->beta1 >= 0.0 && hp->beta1 < 1.0) || !(hp->beta2 >= 0.0 && hp->beta2 < 1.0) ||
      !(hp->eps > 0.0))
    return fail(PINN_ERR_ARG, "Adam hyperparameters out of range");
  *a = pj::AdamArgs{};
  for (int l = 0; l < n_layers; ++l) {
    if (dims[l] < 1 || dims[l + 1] < 1) return fail(PINN_ERR_ARG, "dims[%d..%d] must be positive", l, l + 1);
    if (!W[l] || !b[l] || !dW[l] || !db[l] || !mW[l] || !vW[l] || !mb[l] || !vb[l])
      return fail(PINN_ERR_ARG, "layer %d: NULL pointer", l);
    a->p[2 * l] = W[l];
    a->g[2 * l] = dW[l];
    a->m[2 * l] = mW[l];
    a->v[2 * l] = vW[l];
    a->n[2 * l] = (int64_t)dims[l] * dims[l + 1];
    a->p[2 * l + 1] = b[l];
    a->g[2 * l + 1] = db[l];
    a->m[2 * l + 1] = mb[l];
    a->v[2 * l + 1] = vb[l];
    a->n[2 * l + 1] = dims[l + 1];
  }
  a->nseg = 2 * n_layers;
  a->lr = (float)hp->lr;
  a->b1 = (float)hp->beta1;
  a->b2 = (float)hp->beta2;
  a->eps = (float)hp->eps;
  return PINN_OK;
}

extern "C" pinn_status pinn_adam_step(int32_t n_layers, const int32_t *dims, float *const *W, float *const *b,
                                      const float *const *dW, const float *const *db, float *const *mW,
                                      float *const *vW, float *const *mb, float *const *vb, int64_t step,
                                      const pinn_adam *hp, void *stream) {
  g_err.clear();
  pj::AdamArgs a;
  pinn_status st = adam_args(n_layers, dims, W, b, dW, db, mW, vW, mb, vb, hp, &a);
  if (st) return st;
  if (step < 1) return fail(PINN_ERR_ARG, "step = %lld, must be >= 1", (long long)step);
  a.step = step;
  a.step_dev = nullptr;
  const hipError_t e = pj::launch_adam(a, (hipStream_t)stream);
  return e ? hip_fail(e, "adam") : PINN_OK;
}

// ---------------------------------------------------------------------------
// One plan's step captured into a HIP graph.
// ---------------------------------------------------------------------------
struct pinn_graph_s {
  pinn_plan plan = nullptr;
  hipStream_t origin = nullptr;  // private capture and launch stream (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec = nullptr;
  ~pinn_graph_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (origin) (void)hipStreamDestroy(origin);
  }
};

// Records residual + loss-gradient backward (and, with `adam`, the Adam update
// and the step counter's advance) on a private stream and instantiates it.
static pinn_status graph_capture(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                                 int64_t N, float *r, float *loss, float *const *dW, float *const *db,
                                 const pj::AdamArgs *adam, int64_t *step_dev, pinn_graph *out) {
  if (!out) return fail(PINN_ERR_ARG, "out is NULL");
  *out = nullptr;
  pinn_status st = check_call(plan, net, x, N);
  if (st) return st;
  st = check_pde(pde, plan->kind);
  if (st) return st;
  if (!dW || !db) return fail(PINN_ERR_ARG, "dW or db is NULL");
  for (int l = 0; l < plan->L; ++l)
    if (!dW[l] || !db[l]) return fail(PINN_ERR_ARG, "dW[%d] or db[%d] is NULL", l, l);
  auto *gr = new pinn_graph_s();
  gr->plan = plan;
  hipError_t e = hipStreamCreateWithFlags(&gr->origin, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&gr->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&gr->ev_out, hipEventDisableTiming);
  if (e) {
    delete gr;
    return hip_fail(e, "graph stream");
  }
  plan->prof_class = 0;  // no event timing inside a graph
  e = hipStreamBeginCapture(gr->origin, hipStreamCaptureModeRelaxed);
  if (e) {
    delete gr;
    return hip_fail(e, "graph capture");
  }
  st = pinn_jet_residual(plan, net, pde, x, N, r, loss, nullptr, nullptr, gr->origin);
  if (st == PINN_OK)
    st = pinn_jet_backward(plan, net, pde, x, N, nullptr, dW, db, nullptr, nullptr, gr->origin);
  hipError_t ek = hipSuccess;
  if (st == PINN_OK && adam) {
    ek = pj::launch_adam(*adam, gr->origin);
    if (ek == hipSuccess) ek = pj::launch_step_count(step_dev, gr->origin);
  }
  const std::string msg = g_err;
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(gr->origin, &g);
  if (st || e || ek) {
    if (g) (void)hipGraphDestroy(g);
    delete gr;
    if (st) return fail(st, "%s", msg.c_str());
    return hip_fail(ek ? ek : e, "graph capture");
  }
  e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e) {
    delete gr;
    return hip_fail(e, "graph instantiate");
  }
  *out = gr;
  return PINN_OK;
}

extern "C" {

pinn_status pinn_graph_capture(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                               int64_t N, float *r, float *loss, float *const *dW, float *const *db,
                               pinn_graph *out) {
  g_err.clear();
  if (plan && plan->arch) return fail(PINN_ERR_UNSUPPORTED, "graph capture of a modified-MLP plan");
  return graph_capture(plan, net, pde, x, N, r, loss, dW, db, nullptr, nullptr, out);
}

pinn_status pinn_graph_capture_train(pinn_plan plan, const pinn_net *net, const pinn_pde *pde, const float *x,
                                     int64_t N, float *r, float *loss, float *const *dW, float *const *db,
                                     float *const *mW, float *const *vW, float *const *mb, float *const *vb,
                                     const pinn_adam *hp, int64_t *step_dev, pinn_graph *out) {
  g_err.clear();
  if (plan && plan->arch) return fail(PINN_ERR_UNSUPPORTED, "graph capture of a modified-MLP plan");
  if (!net || !step_dev) return fail(PINN_ERR_ARG, "net or step_dev is NULL");
  if (!out) return fail(PINN_ERR_ARG, "out is NULL");
  pj::AdamArgs a;
  // the net's parameters are the ones the replays update in place
  pinn_status st = adam_args(net->n_layers, net->dims, const_cast<float *const *>(net->W),
                             const_cast<float *const *>(net->b), dW, db, mW, vW, mb, vb, hp, &a);
  if (st) return st;
  a.step = 0;
  a.step_dev = step_dev;
  return graph_capture(plan, net, pde, x, N, r, loss, dW, db, &a, step_dev, out);
}

pinn_status pinn_graph_launch(pinn_graph gr, void *stream) {
  g_err.clear();
  if (!gr) return fail(PINN_ERR_ARG, "graph is NULL");
  hipStream_t caller = (hipStream_t)stream;
  hipError_t e = hipEventRecord(gr->ev_in, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(gr->origin, gr->ev_in, 0);
  if (e == hipSuccess) e = hipGraphLaunch(gr->exec, gr->origin);
  if (e == hipSuccess) e = hipEventRecord(gr->ev_out, gr->origin);
  if (e == hipSuccess) e = hipStreamWaitEvent(caller, gr->ev_out, 0);
  return e ? hip_fail(e, "graph launch") : PINN_OK;
}

pinn_status pinn_graph_destroy(pinn_graph gr) {
  g_err.clear();
  if (!gr) return fail(PINN_ERR_ARG, "graph is NULL");
  // launches already queued must not run on a destroyed graph
  const hipError_t e = hipStreamSynchronize(gr->origin);
  delete gr;
  return e ? hip_fail(e, "graph destroy") : PINN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Ensembles: many independent networks stepped together.
//
// Every member has its own plan.  A step first records, per member, the
// launches its residual, backward (and Adam) calls would make (the plan code
// runs unchanged with a Recorder installed), uploads all argument blocks to
// device memory once, and merges the members' launch lists into grouped
// launches: at each point the kernel body at the front of the most members is
// launched once for all of them (group.hpp), each member on its own virtual
// grid.  Members of one hidden width share a stream (a lane); lanes run
// concurrently.  The schedule is kept while the pointers, sizes and
// coefficients stay the same, and with graphs on it is captured into one HIP
// graph.  A member's results are those of its single-plan calls bit for bit.
// ---------------------------------------------------------------------------
namespace pj {
Recorder *&current_recorder() {
  static thread_local Recorder *r = nullptr;
  return r;
}
int &current_record_class() {
  static thread_local int c = 0;
  return c;
}
}  // namespace pj

namespace {

struct GroupedLaunch {
  pj::GroupTab tab;
  int cls = 0;  // kernel class of the launch sites
  int blocks = 0;
  size_t lds = 0;
  hipError_t (*launch)(const pj::GroupTab &, int, size_t, hipStream_t) = nullptr;
};

// Adam state of a training step over a batch (host arrays per member).
struct BatchTrain {
  float *const *const *mW, *const *const *vW, *const *const *mb, *const *const *vb;
  const pinn_adam *hp;
  int64_t *step_dev;
};

}  // namespace

struct pinn_batch_s {
  int n = 0;
  std::vector<pinn_plan> plans;
  std::vector<int> L, width;
  int n_streams = 4;                  // lanes at most
  std::vector<hipStream_t> streams;   // one per lane (default priority)
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr, ev_in = nullptr, ev_out = nullptr;
  hipStream_t origin = nullptr;       // capture origin
  bool use_graph = true;
  bool per_network = false;           // lanes: by hidden width, or networks balanced over the streams
  bool width_lanes = false;           // per-network lanes that each hold networks of one width
  hipGraphExec_t exec = nullptr;
  std::vector<const void *> key;      // every pointer and size baked into the schedule
  // the schedule
  std::vector<std::vector<GroupedLaunch>> lanes;
  std::vector<GroupedLaunch> tail;    // after the join (the Adam step counter)
  void *dev_args = nullptr;
  size_t dev_args_cap = 0;
  size_t n_launches = 0;              // grouped launches per step
  // launch timing of one kernel class (pinn_batch_profile): eager steps only
  int prof_class = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  ~pinn_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipEvent_t e : ev_join) (void)hipEventDestroy(e);
    for (hipEvent_t e : {ev_fork, ev_in, ev_out})
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    if (origin) (void)hipStreamDestroy(origin);
    if (dev_args) (void)hipFree(dev_args);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (pinn_plan p : plans) delete p;
  }
  hipError_t harvest() {
    if (ev_used == 0) return hipSuccess;
    for (size_t i = 0; i + 1 < ev_used; i += 2) {
      hipError_t e = hipEventSynchronize(ev_pool[i + 1]);
      if (e) return e;
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev_pool[i], ev_pool[i + 1]);
      if (e) return e;
      prof_ms += ms;
      ++prof_launches;
    }
    ev_used = 0;
    return hipSuccess;
  }
};

namespace {

constexpr int kMaxBatchStreams = 16;

hipError_t batch_streams(pinn_batch b, int n) {
  while ((int)b->streams.size() < n) {
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e) return e;
    b->streams.push_back(s);
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e) return e;
    b->ev_join.push_back(ev);
  }
  b->n_streams = n;
  return hipSuccess;
}

// Drops the schedule.  A step still running may read the argument table
// and the graph, so the batch's streams are drained first.
void invalidate(pinn_batch b) {
  if (b->exec || !b->lanes.empty()) {
    if (b->origin) (void)hipStreamSynchronize(b->origin);
    for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  }
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  b->key.clear();
  b->lanes.clear();
  b->tail.clear();
}

// Greedy merge of the members' launch records (in order per member) into
// grouped launches; the records' argument blocks sit at base + off[i][k].
void merge_lane(const std::vector<int> &members, const std::vector<std::vector<pj::LaunchRecord>> &recs,
                const std::vector<std::vector<size_t>> &off, char *base, std::vector<GroupedLaunch> &out) {
  std::vector<size_t> front(recs.size(), 0);
  for (;;) {
    // the body at the front of the most members (first seen on a tie)
    std::vector<const void *> keys;
    std::vector<int> counts;
    for (int i : members) {
      if (front[i] >= recs[i].size()) continue;
      const void *k = recs[i][front[i]].key;
      size_t q = 0;
      while (q < keys.size() && keys[q] != k) ++q;
      if (q == keys.size()) {
        keys.push_back(k);
        counts.push_back(0);
      }
      ++counts[q];
    }
    if (keys.empty()) break;
    const void *K = keys[std::max_element(counts.begin(), counts.end()) - counts.begin()];
    GroupedLaunch gl{};
    auto flush = [&]() {
      if (gl.tab.n > 0) out.push_back(gl);
      gl = GroupedLaunch{};
    };
    for (int i : members) {
      if (front[i] >= recs[i].size() || recs[i][front[i]].key != K) continue;
      const pj::LaunchRecord &r = recs[i][front[i]];
      if (gl.tab.n == pj::kGroupMax) flush();
      const int e = gl.tab.n++;
      gl.tab.start[e] = gl.blocks;
      gl.tab.gx[e] = r.gx;
      gl.tab.args[e] = base + off[i][front[i]];
      gl.blocks += r.gx * r.gy;
      gl.tab.start[e + 1] = gl.blocks;
      gl.lds = std::max(gl.lds, r.lds);
      gl.launch = r.launch_group;
      gl.cls = r.cls;
      ++front[i];
    }
    flush();
  }
}

// Records every member's step and builds the grouped schedule.
pinn_status batch_build(pinn_batch b, const pinn_net *nets, const pinn_pde *pdes, const float *const *x,
                        const int64_t *N, float *loss, float *const *const *dW, float *const *const *db,
                        const BatchTrain *train) {
  invalidate(b);
  std::vector<std::vector<pj::LaunchRecord>> recs(b->n);
  for (int i = 0; i < b->n; ++i) {
    pinn_plan p = b->plans[i];
    p->prof_class = 0;
    pj::Recorder rec;
    pj::current_recorder() = &rec;
    pinn_status st = pinn_jet_residual(p, &nets[i], &pdes[i], x[i], N[i], nullptr, loss + i, nullptr, nullptr,
                                       nullptr);
    if (st == PINN_OK)
      st = pinn_jet_backward(p, &nets[i], &pdes[i], x[i], N[i], nullptr, dW[i], db[i], nullptr, nullptr, nullptr);
    if (st == PINN_OK && train) {
      pj::AdamArgs a;
      st = adam_args(nets[i].n_layers, nets[i].dims, const_cast<float *const *>(nets[i].W),
                     const_cast<float *const *>(nets[i].b), dW[i], db[i], train->mW[i], train->vW[i], train->mb[i],
                     train->vb[i], train->hp, &a);
      if (st == PINN_OK) {
        a.step = 0;
        a.step_dev = train->step_dev;
        const hipError_t e = pj::launch_adam(a, nullptr);
        if (e) st = hip_fail(e, "adam");
      }
    }
    pj::current_recorder() = nullptr;
    if (st) {
      const std::string msg = g_err;
      return fail(st, "network %d: %s", i, msg.c_str());
    }
    recs[i] = std::move(rec.recs);
  }
  // a training step ends with one advance of the step counter, after every
  // member's update: recorded as one more launch list (entry n)
  if (train) {
    pj::Recorder rec;
    pj::current_recorder() = &rec;
    const hipError_t e2 = pj::launch_step_count(train->step_dev, nullptr);
    pj::current_recorder() = nullptr;
    if (e2) return hip_fail(e2, "step count");
    recs.push_back(std::move(rec.recs));
  }
  // argument blocks, 16-byte aligned, in one device buffer
  std::vector<std::vector<size_t>> off(recs.size());
  size_t total = 0;
  for (size_t i = 0; i < recs.size(); ++i)
    for (const pj::LaunchRecord &r : recs[i]) {
      off[i].push_back(total);
      total += (r.args.size() + 15) & ~size_t(15);
    }
  std::vector<unsigned char> host(std::max<size_t>(total, 16));
  for (size_t i = 0; i < recs.size(); ++i)
    for (size_t k = 0; k < recs[i].size(); ++k)
      std::memcpy(host.data() + off[i][k], recs[i][k].args.data(), recs[i][k].args.size());
  if (total > b->dev_args_cap) {
    if (b->dev_args) (void)hipFree(b->dev_args);
    b->dev_args = nullptr;
    b->dev_args_cap = 0;
    hipError_t e = hipMalloc(&b->dev_args, total);
    if (e) return hip_fail(e, "batch argument table");
    b->dev_args_cap = total;
  }
  hipError_t e = hipMemcpy(b->dev_args, host.data(), total, hipMemcpyHostToDevice);
  if (e) return hip_fail(e, "batch argument table");
  // lanes: one per hidden width (widths in increasing order), folded onto the
  // streams; or, per network, the networks dealt longest first to the lane
  // with the least estimated work (hidden-layer flops w^2 C H N); or, per
  // network by width, the lanes shared out to the widths (one each, the rest
  // one at a time to the width with the most work per lane) and each width's
  // networks dealt to its lanes the same way, so that a lane's networks run
  // the same kernels and group at every phase
  std::vector<std::vector<int>> members;
  std::vector<int> widths(b->width);
  std::sort(widths.begin(), widths.end());
  widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
  const int n_widths = (int)widths.size();
  if (b->per_network) {
    const int n_lanes = std::min(b->n, b->n_streams);
    std::vector<double> cost(b->n);
    std::vector<int> order(b->n);
    for (int i = 0; i < b->n; ++i) {
      const pinn_plan p = b->plans[i];
      cost[i] = (double)p->w * p->w * p->ki.C * p->H * (double)N[i];
      order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    // the lanes each width may use: all of them, or its share
    std::vector<int> lane0(n_widths, 0), nl(n_widths, n_lanes);
    if (b->width_lanes && n_lanes >= n_widths) {
      std::vector<double> work(n_widths, 0.0);
      std::vector<int> count(n_widths, 0);
      for (int i = 0; i < b->n; ++i) {
        const int wi = (int)(std::lower_bound(widths.begin(), widths.end(), b->width[i]) - widths.begin());
        work[wi] += cost[i];
        ++count[wi];
      }
      std::fill(nl.begin(), nl.end(), 1);
      for (int extra = n_lanes - n_widths; extra > 0; --extra) {
        int best = -1;
        for (int k = 0; k < n_widths; ++k)
          if (nl[k] < count[k] && (best < 0 || work[k] / nl[k] > work[best] / nl[best])) best = k;
        if (best < 0) break;
        ++nl[best];
      }
      for (int k = 1; k < n_widths; ++k) lane0[k] = lane0[k - 1] + nl[k - 1];
    }
    const int total = b->width_lanes && n_lanes >= n_widths ? lane0[n_widths - 1] + nl[n_widths - 1] : n_lanes;
    members.assign(total, {});
    std::vector<double> load(total, 0.0);
    for (int i : order) {
      int k = 0;
      if (b->width_lanes && n_lanes >= n_widths)
        k = (int)(std::lower_bound(widths.begin(), widths.end(), b->width[i]) - widths.begin());
      const int lo = b->width_lanes && n_lanes >= n_widths ? lane0[k] : 0;
      const int hi = b->width_lanes && n_lanes >= n_widths ? lane0[k] + nl[k] : total;
      const int l = (int)(std::min_element(load.begin() + lo, load.begin() + hi) - load.begin());
      members[l].push_back(i);
      load[l] += cost[i];
    }
    for (auto &m : members) std::sort(m.begin(), m.end());
  } else {
    const int n_lanes = std::min<int>(n_widths, b->n_streams);
    members.assign(n_lanes, {});
    for (int i = 0; i < b->n; ++i) {
      const int wi = (int)(std::lower_bound(widths.begin(), widths.end(), b->width[i]) - widths.begin());
      members[wi % n_lanes].push_back(i);
    }
  }
  const int n_lanes = (int)members.size();
  b->lanes.assign(n_lanes, {});
  b->n_launches = 0;
  char *base = static_cast<char *>(b->dev_args);
  for (int l = 0; l < n_lanes; ++l) {
    merge_lane(members[l], recs, off, base, b->lanes[l]);
    b->n_launches += b->lanes[l].size();
  }
  if (train) {
    merge_lane(std::vector<int>{b->n}, recs, off, base, b->tail);
    b->n_launches += b->tail.size();
  }
  return PINN_OK;
}

// Enqueues the schedule: fork from `origin` to the lanes, join back.
pinn_status batch_enqueue(pinn_batch b, hipStream_t origin) {
  hipError_t e = hipEventRecord(b->ev_fork, origin);
  if (e) return hip_fail(e, "fork");
  const int n_lanes = (int)b->lanes.size();
  for (int l = 0; l < n_lanes; ++l) {
    hipStream_t s = b->streams[l];
    e = hipStreamWaitEvent(s, b->ev_fork, 0);
    if (e) return hip_fail(e, "fork");
    for (const GroupedLaunch &g : b->lanes[l]) {
      const bool tm = b->prof_class != 0 && g.cls == b->prof_class;
      if (tm) {  // a pair of events around the launch, on its lane
        if (b->ev_used + 2 > b->ev_pool.size()) {
          if (b->ev_pool.size() >= 4096) {
            e = b->harvest();
            if (e) return hip_fail(e, "event timing");
          }
          while (b->ev_used + 2 > b->ev_pool.size()) {
            hipEvent_t ev;
            e = hipEventCreate(&ev);
            if (e) return hip_fail(e, "event timing");
            b->ev_pool.push_back(ev);
          }
        }
        e = hipEventRecord(b->ev_pool[b->ev_used], s);
        if (e) return hip_fail(e, "event timing");
      }
      e = g.launch(g.tab, g.blocks, g.lds, s);
      if (e) return hip_fail(e, "grouped launch");
      if (tm) {
        e = hipEventRecord(b->ev_pool[b->ev_used + 1], s);
        if (e) return hip_fail(e, "event timing");
        b->ev_used += 2;
      }
    }
    e = hipEventRecord(b->ev_join[l], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, b->ev_join[l], 0);
    if (e) return hip_fail(e, "join");
  }
  for (const GroupedLaunch &g : b->tail) {
    e = g.launch(g.tab, g.blocks, g.lds, origin);
    if (e) return hip_fail(e, "grouped launch");
  }
  return PINN_OK;
}

pinn_status batch_check(pinn_batch b, const pinn_net *nets, const pinn_pde *pdes, const float *const *x,
                        const int64_t *N, float *loss, float *const *const *dW, float *const *const *db,
                        std::vector<const void *> &key) {
  if (!nets || !pdes || !x || !N || !loss || !dW || !db) return fail(PINN_ERR_ARG, "a batch argument is NULL");
  key.push_back(loss);
  for (int i = 0; i < b->n; ++i) {
    pinn_status st = check_call(b->plans[i], &nets[i], x[i], N[i]);
    if (st == PINN_OK) st = check_pde(&pdes[i], b->plans[i]->kind);
    if (st) {
      std::string msg = g_err;
      return fail(st, "network %d: %s", i, msg.c_str());
    }
    if (!dW[i] || !db[i]) return fail(PINN_ERR_ARG, "network %d: dW or db is NULL", i);
    for (int l = 0; l < b->L[i]; ++l)
      if (!dW[i][l] || !db[i][l]) return fail(PINN_ERR_ARG, "network %d: dW[%d] or db[%d] is NULL", i, l, l);
    key.push_back(x[i]);
    key.push_back(reinterpret_cast<const void *>((intptr_t)N[i]));
    for (int q = 0; q < 4; ++q) {
      double c = pdes[i].coef[q];
      intptr_t bits;
      std::memcpy(&bits, &c, sizeof bits);
      key.push_back(reinterpret_cast<const void *>(bits));
    }
    for (int l = 0; l < b->L[i]; ++l) {
      key.push_back(nets[i].W[l]);
      key.push_back(nets[i].b[l]);
      key.push_back(dW[i][l]);
      key.push_back(db[i][l]);
    }
    // the tuning selects the kernels
    key.push_back(reinterpret_cast<const void *>((intptr_t)b->plans[i]->dw_splits));
    key.push_back(reinterpret_cast<const void *>((intptr_t)(b->plans[i]->fwd_points * 2 + b->plans[i]->bwd_fused)));
    key.push_back(reinterpret_cast<const void *>((intptr_t)b->plans[i]->bwd_points));
  }
  return PINN_OK;
}

pinn_status batch_run(pinn_batch b, const pinn_net *nets, const pinn_pde *pdes, const float *const *x,
                      const int64_t *N, float *loss, float *const *const *dW, float *const *const *db,
                      const BatchTrain *train, void *stream) {
  std::vector<const void *> key;
  pinn_status st = batch_check(b, nets, pdes, x, N, loss, dW, db, key);
  if (st) return st;
  if (train) {
    key.push_back(train->step_dev);
    for (int i = 0; i < b->n; ++i)
      for (int l = 0; l < b->L[i]; ++l) {
        key.push_back(train->mW[i][l]);
        key.push_back(train->vW[i][l]);
        key.push_back(train->mb[i][l]);
        key.push_back(train->vb[i][l]);
      }
    const double *h = &train->hp->lr;
    for (int q = 0; q < 4; ++q) {
      intptr_t bits;
      std::memcpy(&bits, h + q, sizeof bits);
      key.push_back(reinterpret_cast<const void *>(bits));
    }
  }
  key.push_back(reinterpret_cast<const void *>((intptr_t)b->n_streams));
  key.push_back(reinterpret_cast<const void *>((intptr_t)(b->per_network * 2 + b->width_lanes)));
  hipStream_t caller = (hipStream_t)stream;
  if (b->lanes.empty() || key != b->key) {
    st = batch_build(b, nets, pdes, x, N, loss, dW, db, train);
    if (st) return st;
    b->key = key;
  }
  if (!b->use_graph || b->prof_class != 0) return batch_enqueue(b, caller);
  hipError_t e;
  if (!b->exec) {
    e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeRelaxed);
    if (e) return hip_fail(e, "graph capture");
    st = batch_enqueue(b, b->origin);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->origin, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e) return hip_fail(e, "graph capture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e) return hip_fail(e, "graph instantiate");
  }
  e = hipEventRecord(b->ev_in, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->origin, b->ev_in, 0);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->origin);
  if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->origin);
  if (e == hipSuccess) e = hipStreamWaitEvent(caller, b->ev_out, 0);
  if (e) return hip_fail(e, "graph launch");
  return PINN_OK;
}

}  // namespace

extern "C" {

pinn_status pinn_batch_create(int32_t n, const pinn_net *nets, const pinn_pde *pdes, const int64_t *max_points,
                              int32_t prec, uint32_t flags, pinn_batch *out) {
  g_err.clear();
  if (!out) return fail(PINN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > 4096) return fail(PINN_ERR_ARG, "n = %d outside [1, 4096]", n);
  if (!nets || !pdes || !max_points) return fail(PINN_ERR_ARG, "nets, pdes or max_points is NULL");
  pinn_batch b = new (std::nothrow) pinn_batch_s;
  if (!b) return fail(PINN_ERR_NOMEM, "host allocation failed");
  for (int i = 0; i < n; ++i) {
    pinn_plan p = nullptr;
    pinn_status st = pinn_plan_create(&nets[i], &pdes[i], max_points[i], prec, flags, 0, &p);
    if (st) {
      std::string msg = g_err;
      delete b;
      return fail(st, "network %d: %s", i, msg.c_str());
    }
    b->plans.push_back(p);
    b->L.push_back(nets[i].n_layers);
    b->width.push_back(p->w);
  }
  b->n = n;
  hipError_t e = batch_streams(b, 4);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "batch streams");
  }
  *out = b;
  return PINN_OK;
}

pinn_status pinn_batch_destroy(pinn_batch b) {
  g_err.clear();
  if (!b) return fail(PINN_ERR_ARG, "batch is NULL");
  (void)hipStreamSynchronize(b->origin);
  for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  delete b;
  return PINN_OK;
}

pinn_status pinn_batch_configure(pinn_batch b, int32_t n_streams, int32_t use_graph) {
  g_err.clear();
  if (!b) return fail(PINN_ERR_ARG, "batch is NULL");
  if (n_streams < 1 || n_streams > kMaxBatchStreams)
    return fail(PINN_ERR_ARG, "n_streams = %d outside [1, %d]", n_streams, kMaxBatchStreams);
  if (use_graph & ~(PINN_BATCH_GRAPH | PINN_BATCH_PER_NETWORK | PINN_BATCH_WIDTH_LANES))
    return fail(PINN_ERR_ARG, "unknown batch flags 0x%x", use_graph);
  if ((use_graph & PINN_BATCH_WIDTH_LANES) && !(use_graph & PINN_BATCH_PER_NETWORK))
    return fail(PINN_ERR_ARG, "PINN_BATCH_WIDTH_LANES needs PINN_BATCH_PER_NETWORK");
  hipError_t e = batch_streams(b, n_streams);
  if (e) return hip_fail(e, "batch streams");
  b->use_graph = (use_graph & PINN_BATCH_GRAPH) != 0;
  b->per_network = (use_graph & PINN_BATCH_PER_NETWORK) != 0;
  b->width_lanes = (use_graph & PINN_BATCH_WIDTH_LANES) != 0;
  invalidate(b);
  return PINN_OK;
}

pinn_status pinn_batch_get_config(pinn_batch b, int32_t *n_streams, int32_t *flags) {
  g_err.clear();
  if (!b || !n_streams || !flags) return fail(PINN_ERR_ARG, "a pinn_batch_get_config argument is NULL");
  *n_streams = b->n_streams;
  *flags = (b->use_graph ? PINN_BATCH_GRAPH : 0) | (b->per_network ? PINN_BATCH_PER_NETWORK : 0) |
           (b->width_lanes ? PINN_BATCH_WIDTH_LANES : 0);
  return PINN_OK;
}

pinn_status pinn_batch_step(pinn_batch b, const pinn_net *nets, const pinn_pde *pdes, const float *const *x,
                            const int64_t *N, float *loss, float *const *const *dW, float *const *const *db,
                            void *stream) {
  g_err.clear();
  if (!b) return fail(PINN_ERR_ARG, "batch is NULL");
  return batch_run(b, nets, pdes, x, N, loss, dW, db, nullptr, stream);
}

pinn_status pinn_batch_train_step(pinn_batch b, const pinn_net *nets, const pinn_pde *pdes, const float *const *x,
                                  const int64_t *N, float *loss, float *const *const *dW, float *const *const *db,
                                  float *const *const *mW, float *const *const *vW, float *const *const *mb,
                                  float *const *const *vb, const struct pinn_adam_s *hp, int64_t *step_dev,
                                  void *stream) {
  g_err.clear();
  if (!b) return fail(PINN_ERR_ARG, "batch is NULL");
  if (!mW || !vW || !mb || !vb || !hp || !step_dev) return fail(PINN_ERR_ARG, "an Adam argument is NULL");
  for (int i = 0; i < b->n; ++i)
    if (!mW[i] || !vW[i] || !mb[i] || !vb[i]) return fail(PINN_ERR_ARG, "network %d: moment arrays NULL", i);
  BatchTrain t{mW, vW, mb, vb, hp, step_dev};
  return batch_run(b, nets, pdes, x, N, loss, dW, db, &t, stream);
}

pinn_status pinn_batch_profile(pinn_batch b, int32_t kernel_class) {
  g_err.clear();
  if (!b) return fail(PINN_ERR_ARG, "batch is NULL");
  if (kernel_class < 0 || kernel_class > PINN_K_BWD_DW)
    return fail(PINN_ERR_ARG, "unknown kernel class %d", kernel_class);
  b->prof_class = kernel_class;
  b->ev_used = 0;
  b->prof_ms = 0.0;
  b->prof_launches = 0;
  return PINN_OK;
}

pinn_status pinn_batch_profile_read(pinn_batch b, double *total_ms, int64_t *launches) {
  g_err.clear();
  if (!b) return fail(PINN_ERR_ARG, "batch is NULL");
  const hipError_t e = b->harvest();
  if (e) return hip_fail(e, "event timing");
  if (total_ms) *total_ms = b->prof_ms;
  if (launches) *launches = b->prof_launches;
  return PINN_OK;
}

pinn_status pinn_batch_get_tuning(pinn_batch b, int32_t i, pinn_tuning *t) {
  g_err.clear();
  if (!b || !t) return fail(PINN_ERR_ARG, "batch or tuning is NULL");
  if (i < 0 || i >= b->n) return fail(PINN_ERR_ARG, "network %d outside [0, %d)", i, b->n);
  return pinn_plan_get_tuning(b->plans[i], t);
}

pinn_status pinn_batch_set_tuning(pinn_batch b, int32_t i, const pinn_tuning *t) {
  g_err.clear();
  if (!b || !t) return fail(PINN_ERR_ARG, "batch or tuning is NULL");
  if (i < 0 || i >= b->n) return fail(PINN_ERR_ARG, "network %d outside [0, %d)", i, b->n);
  return pinn_plan_set_tuning(b->plans[i], t);  // the schedule key holds the tuning: the next step rebuilds
}

pinn_status pinn_batch_launches(pinn_batch b, int64_t *launches) {
  g_err.clear();
  if (!b || !launches) return fail(PINN_ERR_ARG, "batch or launches is NULL");
  *launches = (int64_t)b->n_launches;
  return PINN_OK;
}

pinn_status pinn_batch_schedule_classes(pinn_batch b, int32_t *classes, int64_t cap, int64_t *n_out) {
  g_err.clear();
  if (!b || !n_out) return fail(PINN_ERR_ARG, "batch or n_out is NULL");
  int64_t n = 0;
  auto put = [&](const GroupedLaunch &g) {
    if (classes && n < cap) classes[n] = g.cls;
    ++n;
  };
  for (const auto &lane : b->lanes)
    for (const GroupedLaunch &g : lane) put(g);
  for (const GroupedLaunch &g : b->tail) put(g);
  *n_out = n;
  if (classes && n > cap) return fail(PINN_ERR_ARG, "cap = %lld below the %lld launches", (long long)cap, (long long)n);
  return PINN_OK;
}

pinn_status pinn_batch_autotune(pinn_batch b, const pinn_net *nets, const pinn_pde *pdes, const float *const *x,
                                const int64_t *N, float *loss, float *const *const *dW, float *const *const *db,
                                int32_t reps, int32_t *best_streams, double *best_ms, void *stream) {
  g_err.clear();
  if (!b) return fail(PINN_ERR_ARG, "batch is NULL");
  if (reps < 1 || reps > 1000) return fail(PINN_ERR_ARG, "reps = %d outside [1, 1000]", reps);
  std::vector<const void *> key;
  pinn_status st = batch_check(b, nets, pdes, x, N, loss, dW, db, key);
  if (st) return st;
  // every member's tuning (point tiles, fused or separate weight gradient,
  // split count) from the plan autotuner, through its cache: members that
  // share width, depth and point-count bucket are timed once
  for (int i = 0; i < b->n; ++i) {
    st = pinn_plan_autotune(b->plans[i], &nets[i], &pdes[i], x[i], N[i], reps, nullptr, nullptr, stream);
    if (st) {
      const std::string msg = g_err;
      return fail(st, "network %d: %s", i, msg.c_str());
    }
  }
  hipStream_t caller = (hipStream_t)stream;
  hipEvent_t t0, t1;
  hipError_t e = hipEventCreate(&t0);
  if (e) return hip_fail(e, "autotune events");
  e = hipEventCreate(&t1);
  if (e) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "autotune events");
  }
  const int graph = b->use_graph ? PINN_BATCH_GRAPH : 0;
  // milliseconds per step of the current configuration (one untimed step first)
  auto time_steps = [&](double *ms_out) -> pinn_status {
    pinn_status s2 = PINN_OK;
    for (int it = -1; it < reps && s2 == PINN_OK; ++it) {
      if (it == 0) e = hipEventRecord(t0, caller);
      s2 = pinn_batch_step(b, nets, pdes, x, N, loss, dW, db, stream);
    }
    if (s2) return s2;
    e = hipEventRecord(t1, caller);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e) return hip_fail(e, "autotune timing");
    *ms_out = ms / reps;
    return PINN_OK;
  };
  // the member tilings: each network's own fastest, or every network on the
  // tiling with the most points per workgroup its shape allows (in grouped
  // launches the per-point cost counts, not a member's own latency), timed as
  // whole grouped steps
  {
    std::vector<pinn_tuning> own(b->n), wide(b->n);
    for (int i = 0; i < b->n; ++i) {
      const pinn_plan p = b->plans[i];
      own[i] = pinn_tuning{p->dw_splits, p->fwd_points, p->bwd_fused, p->bwd_points};
      wide[i] = own[i];
      if (pj::fused_fwd_fits(64, p->ki.C, p->w, p->prec)) wide[i].fwd_points = 64;
      if (pj::bwd_dw_fused_supported(p->ki.C, p->w, p->prec)) wide[i].bwd_fused = 1;
      if (pj::wide_bwd_points_supported(256, p->ki.C, p->w, p->prec)) wide[i].bwd_points = 256;
    }
    double ms_own = 1e300, ms_wide = 1e300;
    st = pinn_batch_configure(b, 8, graph | PINN_BATCH_PER_NETWORK);
    if (st == PINN_OK) st = time_steps(&ms_own);
    for (int i = 0; i < b->n && st == PINN_OK; ++i) st = pinn_plan_set_tuning(b->plans[i], &wide[i]);
    if (st == PINN_OK) st = time_steps(&ms_wide);
    if (st == PINN_OK && ms_own <= ms_wide)
      for (int i = 0; i < b->n && st == PINN_OK; ++i) st = pinn_plan_set_tuning(b->plans[i], &own[i]);
    if (st) {
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      return st;
    }
  }
  // then the number of lanes
  double bms = 1e300;
  int bs = b->n_streams,
      bmode = (b->per_network ? PINN_BATCH_PER_NETWORK : 0) | (b->width_lanes ? PINN_BATCH_WIDTH_LANES : 0);
  constexpr int PW = PINN_BATCH_PER_NETWORK | PINN_BATCH_WIDTH_LANES;
  const std::pair<int, int> cands[] = {{1, 0}, {2, 0}, {4, 0}, {8, PINN_BATCH_PER_NETWORK},
                                       {16, PINN_BATCH_PER_NETWORK}, {8, PW}, {12, PW}, {16, PW}};
  for (const auto &cand : cands) {
    const int ns = cand.first, mode = cand.second;
    double ms = 1e300;
    st = pinn_batch_configure(b, ns, graph | mode);
    if (st == PINN_OK) st = time_steps(&ms);
    if (st) break;
    if (ms < bms) {
      bms = ms;
      bs = ns;
      bmode = mode;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st) return st;
  st = pinn_batch_configure(b, bs, graph | bmode);
  if (st) return st;
  if (best_streams) *best_streams = bs;
  if (best_ms) *best_ms = bms;
  return PINN_OK;
}

}  // extern "C"
