// Walks the host paths of the C ABI on the stand-in runtime (fake_hip.cpp):
// the ensemble step as the benchmark drives it (autotune, timing, per-class
// launch timing, schedule queries, reconfiguration, destroy) under several
// synthetic-clock seeds, the ensemble training step, single plans of every
// PDE kind, operand type and tuning, composite losses, the modified MLP,
// graphs, the tuning cache, the no-allocation step and argument errors.
// Built with AddressSanitizer; any status other than the expected one, any
// sanitizer report or runtime violation fails the run.
//
// usage: driver ENSEMBLE_SHAPES CACHE_PATH
//   ENSEMBLE_SHAPES: one network per line, "N nu d0 d1 .. dL"
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pinn_jet.h"

extern "C" {
void fake_hip_set_seed(uint64_t seed);
uint64_t fake_hip_launches(void);
void fake_hip_live(size_t *streams, size_t *events, size_t *graphs, size_t *execs, size_t *allocs);
int fake_hip_capturing(void);
}

namespace {

int g_checks = 0;

void expect_status(pinn_status got, pinn_status want, const char *what, int line) {
  ++g_checks;
  if (got != want) {
    fprintf(stderr, "driver.cpp:%d: %s returned %d, expected %d (%s)\n", line, what, got, want, pinn_last_error());
    exit(1);
  }
}
#define OK(call) expect_status((call), PINN_OK, #call, __LINE__)
#define STATUS(call, want) expect_status((call), (want), #call, __LINE__)

void *dev_alloc(size_t bytes) {
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc(%zu) failed\n", bytes);
    exit(1);
  }
  return p;
}
void dev_free(void *p) { (void)hipFree(p); }

// A network's device buffers (contents never read on this runtime).
struct Net {
  std::vector<int32_t> dims;
  std::vector<float *> W, b, dW, db, mW, vW, mb, vb;
  pinn_net net{};
  float *x = nullptr, *r = nullptr, *loss = nullptr, *jets = nullptr;
  int64_t N = 0;
  int64_t *step = nullptr;

  Net(std::vector<int32_t> d, int64_t n, int C, int dout) : dims(std::move(d)), N(n) {
    const int L = (int)dims.size() - 1;
    for (auto *v : {&W, &b, &dW, &db, &mW, &vW, &mb, &vb}) v->resize(L);
    for (int l = 0; l < L; ++l) {
      const size_t nw = (size_t)dims[l] * dims[l + 1], nb = dims[l + 1];
      W[l] = (float *)dev_alloc(nw * 4), dW[l] = (float *)dev_alloc(nw * 4);
      mW[l] = (float *)dev_alloc(nw * 4), vW[l] = (float *)dev_alloc(nw * 4);
      b[l] = (float *)dev_alloc(nb * 4), db[l] = (float *)dev_alloc(nb * 4);
      mb[l] = (float *)dev_alloc(nb * 4), vb[l] = (float *)dev_alloc(nb * 4);
    }
    net = pinn_net{L, dims.data(), (const float *const *)W.data(), (const float *const *)b.data()};
    x = (float *)dev_alloc((size_t)std::max<int64_t>(n, 1) * dims[0] * 4);
    r = (float *)dev_alloc((size_t)std::max<int64_t>(n, 1) * dout * 4);
    jets = (float *)dev_alloc((size_t)std::max<int64_t>(n, 1) * dout * C * 4);
    loss = (float *)dev_alloc(64);
    step = (int64_t *)dev_alloc(8);
  }
  ~Net() {
    for (auto *v : {&W, &b, &dW, &db, &mW, &vW, &mb, &vb})
      for (float *p : *v) dev_free(p);
    for (void *p : {(void *)x, (void *)r, (void *)loss, (void *)jets, (void *)step}) dev_free(p);
  }
  Net(const Net &) = delete;
  Net &operator=(const Net &) = delete;
};

struct Kind {
  int kind, din, dout, C;
  double coef[4];
};
const Kind kKinds[] = {
    {PINN_BURGERS_1D, 2, 1, 4, {0.01}},       {PINN_NS2D_STEADY, 2, 3, 5, {100.0}},
    {PINN_KS_1D, 2, 1, 6, {5.0, 0.5, 0.005}}, {PINN_HEAT_3D, 4, 1, 8, {0.1}},
    {PINN_ANISO_2D, 2, 1, 6, {0.3}},          {PINN_BURGERS_BC, 2, 1, 1, {}},
};

pinn_pde pde_of(const Kind &k) {
  pinn_pde p{};
  p.kind = k.kind;
  for (int q = 0; q < 4; ++q) p.coef[q] = k.coef[q];
  return p;
}

std::vector<int32_t> mlp(int din, int w, int H, int dout) {
  std::vector<int32_t> d{din};
  for (int h = 0; h < H; ++h) d.push_back(w);
  d.push_back(dout);
  return d;
}

// ---------------------------------------------------------------- the ensemble, as the benchmark drives it
void ensemble(const char *path, int prec, uint64_t seed, int counter_window) {
  FILE *f = fopen(path, "r");
  if (!f) {
    fprintf(stderr, "cannot read %s\n", path);
    exit(1);
  }
  std::vector<Net *> nets;
  std::vector<pinn_pde> pdes;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    long long N;
    double nu;
    int consumed = 0;
    if (sscanf(line, "%lld %lf%n", &N, &nu, &consumed) != 2) continue;
    std::vector<int32_t> d;
    const char *s = line + consumed;
    int v, c2;
    while (sscanf(s, "%d%n", &v, &c2) == 1) d.push_back(v), s += c2;
    nets.push_back(new Net(d, N, 4, 1));
    pinn_pde p{};
    p.kind = PINN_BURGERS_1D;
    p.coef[0] = nu;
    pdes.push_back(p);
  }
  fclose(f);
  const int n = (int)nets.size();
  std::vector<pinn_net> nv(n);
  std::vector<const float *> xs(n);
  std::vector<int64_t> Ns(n), maxp(n);
  std::vector<float *const *> dWs(n), dbs(n), mWs(n), vWs(n), mbs(n), vbs(n);
  for (int i = 0; i < n; ++i) {
    nv[i] = nets[i]->net;
    xs[i] = nets[i]->x;
    Ns[i] = maxp[i] = nets[i]->N;
    dWs[i] = nets[i]->dW.data(), dbs[i] = nets[i]->db.data();
    mWs[i] = nets[i]->mW.data(), vWs[i] = nets[i]->vW.data();
    mbs[i] = nets[i]->mb.data(), vbs[i] = nets[i]->vb.data();
  }
  float *loss = (float *)dev_alloc(4 * n);
  fake_hip_set_seed(seed);
  OK(pinn_tuning_cache_clear());
  pinn_batch b = nullptr;
  OK(pinn_batch_create(n, nv.data(), pdes.data(), maxp.data(), prec, 0, &b));
  int32_t best_streams = 0;
  double best_ms = 0;
  OK(pinn_batch_autotune(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(), dbs.data(), 3,
                         &best_streams, &best_ms, nullptr));
  for (int k = 0; k < 3; ++k) OK(pinn_batch_step(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(),
                                                 dbs.data(), nullptr));
  int32_t ns = 0, fl = 0;
  OK(pinn_batch_get_config(b, &ns, &fl));
  // per-class launch timing with the lanes on one stream
  OK(pinn_batch_configure(b, 1, fl & ~PINN_BATCH_PER_NETWORK));
  for (int cls = 1; cls <= 8; ++cls) {
    OK(pinn_batch_profile(b, cls));
    OK(pinn_batch_step(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(), dbs.data(), nullptr));
    double ms;
    int64_t launches;
    OK(pinn_batch_profile_read(b, &ms, &launches));
  }
  OK(pinn_batch_profile(b, 0));
  OK(pinn_batch_configure(b, ns, fl));
  OK(pinn_batch_step(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(), dbs.data(), nullptr));
  for (int i = 0; i < n; ++i) {
    pinn_tuning t;
    OK(pinn_batch_get_tuning(b, i, &t));
    OK(pinn_batch_set_tuning(b, i, &t));
    pinn_tuning bad = t;
    bad.bwd_points = 48;
    STATUS(pinn_batch_set_tuning(b, i, &bad), PINN_ERR_ARG);
  }
  STATUS(pinn_batch_set_tuning(b, n, nullptr), PINN_ERR_ARG);
  int64_t launches = 0;
  OK(pinn_batch_launches(b, &launches));
  if (counter_window) {
    OK(pinn_batch_configure(b, 1, 0));
    OK(pinn_batch_step(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(), dbs.data(), nullptr));
    int64_t nc = 0;
    OK(pinn_batch_schedule_classes(b, nullptr, 0, &nc));
    std::vector<int32_t> cls(nc);
    OK(pinn_batch_schedule_classes(b, cls.data(), nc, &nc));
    if (nc > 1) STATUS(pinn_batch_schedule_classes(b, cls.data(), nc - 1, &nc), PINN_ERR_ARG);
    for (int k = 0; k < counter_window; ++k)
      OK(pinn_batch_step(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(), dbs.data(), nullptr));
  }
  // the training step (Adam in the graph)
  OK(pinn_batch_configure(b, 4, PINN_BATCH_GRAPH | PINN_BATCH_PER_NETWORK));
  pinn_adam hp{1e-3, 0.9, 0.999, 1e-8};
  int64_t *step = (int64_t *)dev_alloc(8);
  for (int k = 0; k < 2; ++k)
    OK(pinn_batch_train_step(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(), dbs.data(),
                             mWs.data(), vWs.data(), mbs.data(), vbs.data(), &hp, step, nullptr));
  // every lane configuration
  for (int s : {1, 2, 3, 4, 5, 8, 12, 16})
    for (int flags : {0, 1, 2, 3, 6, 7}) {
      OK(pinn_batch_configure(b, s, flags));
      OK(pinn_batch_step(b, nv.data(), pdes.data(), xs.data(), Ns.data(), loss, dWs.data(), dbs.data(), nullptr));
    }
  STATUS(pinn_batch_configure(b, 17, 0), PINN_ERR_ARG);
  STATUS(pinn_batch_configure(b, 2, 4), PINN_ERR_ARG);  // width lanes without per-network lanes
  STATUS(pinn_batch_configure(b, 2, 8), PINN_ERR_ARG);
  OK(pinn_batch_destroy(b));
  dev_free(step);
  dev_free(loss);
  for (Net *p : nets) delete p;
}

// ---------------------------------------------------------------- single plans
void run_plan(const Kind &k, int prec, int w, int H, int64_t N, uint32_t flags, size_t cap) {
  Net nt(mlp(k.din, w, H, k.dout), N, k.C, k.dout);
  pinn_pde pde = pde_of(k);
  pinn_plan p = nullptr;
  const pinn_status cs = pinn_plan_create(&nt.net, &pde, N, prec, flags, cap, &p);
  if (cs == PINN_ERR_UNSUPPORTED || cs == PINN_ERR_CAP) return;
  OK(cs);
  size_t saved = 0, work = 0;
  OK(pinn_plan_memory(p, &saved, &work));
  double *l64 = (flags & PINN_VERIFY_F64) ? (double *)dev_alloc(8) : nullptr;
  std::vector<double *> dW64, db64;
  if (flags & PINN_VERIFY_F64)
    for (int l = 0; l < H + 1; ++l) {
      dW64.push_back((double *)dev_alloc((size_t)nt.dims[l] * nt.dims[l + 1] * 8));
      db64.push_back((double *)dev_alloc((size_t)nt.dims[l + 1] * 8));
    }
  auto step = [&]() {
    OK(pinn_jet_residual(p, &nt.net, &pde, nt.x, N, nt.r, nt.loss, l64, nt.jets, nullptr));
    OK(pinn_jet_backward(p, &nt.net, &pde, nt.x, N, nullptr, nt.dW.data(), nt.db.data(),
                         dW64.empty() ? nullptr : dW64.data(), db64.empty() ? nullptr : db64.data(), nullptr));
  };
  OK(pinn_jet_forward(p, &nt.net, nt.x, N, nt.jets, nullptr));
  STATUS(pinn_jet_backward(p, &nt.net, &pde, nt.x, N, nullptr, nt.dW.data(), nt.db.data(), nullptr, nullptr, nullptr),
         PINN_ERR_STATE);
  step();
  OK(pinn_jet_residual(p, &nt.net, &pde, nt.x, N, nt.r, nt.loss, nullptr, nullptr, nullptr));
  OK(pinn_jet_backward_cot(p, &nt.net, &pde, nt.x, N, nt.r, nt.loss, nt.dW.data(), nt.db.data(), nullptr, nullptr,
                           nullptr));
  // every tuning the plan accepts
  pinn_tuning t0;
  OK(pinn_plan_get_tuning(p, &t0));
  for (int sp : {1, t0.dw_splits, 2 * t0.dw_splits})
    for (int fp : {0, 16, 32, 64})
      for (int bf : {0, 1})
        for (int bp : {0, 16, 32, 64}) {
          pinn_tuning t{sp, fp, bf, bp};
          const pinn_status s = pinn_plan_set_tuning(p, &t);
          if (s == PINN_OK) step();
          else STATUS(s, PINN_ERR_ARG);
        }
  OK(pinn_plan_set_tuning(p, &t0));
  // composite losses on the kinds that have boundary data
  if (k.kind == PINN_BURGERS_1D || k.kind == PINN_NS2D_STEADY) {
    const int64_t a = N / 2, c = N / 4;
    float *vals = (float *)dev_alloc((size_t)std::max<int64_t>(N, 1) * k.dout * 4);
    std::vector<pinn_segment> segs;
    segs.push_back(pinn_segment{PINN_SEG_PDE, 0, 0, a, 1.0, 0, {}, nullptr});
    segs.push_back(pinn_segment{PINN_SEG_DIRICHLET, PINN_DATA_SIN, a, c, 10.0, 1, {1.0, 3.14159, 0, 0}, nullptr});
    const int64_t rest = N - a - c, v = rest / 2, per = (rest - v) / 2 * 2;
    uint32_t values_mask = 0;  // the value channel of every output
    for (int o = 0; o < k.dout; ++o) values_mask |= 1u << (o * k.C);
    segs.push_back(pinn_segment{PINN_SEG_DIRICHLET, PINN_DATA_VALUES, a + c, v, 2.0, values_mask, {}, vals});
    if (k.kind == PINN_BURGERS_1D)
      segs.push_back(pinn_segment{PINN_SEG_PERIODIC, 0, a + c + v, per, 1.0, 3, {}, nullptr});
    std::vector<pinn_segment> use;
    for (auto &s : segs)
      if (s.count > 0) use.push_back(s);
    float *seg_loss = (float *)dev_alloc(64);
    if (!use.empty()) {
      OK(pinn_jet_loss(p, &nt.net, &pde, use.data(), (int)use.size(), nt.x, N, nt.loss, seg_loss, nullptr));
      OK(pinn_jet_loss_backward(p, &nt.net, &pde, use.data(), (int)use.size(), nt.x, N, nt.dW.data(), nt.db.data(),
                                nullptr));
    }
    pinn_segment bad = segs[0];
    bad.count = N + 1;
    STATUS(pinn_jet_loss(p, &nt.net, &pde, &bad, 1, nt.x, N, nt.loss, seg_loss, nullptr), PINN_ERR_ARG);
    dev_free(seg_loss);
    dev_free(vals);
  }
  // autotune, graphs, launch timing
  pinn_tuning best;
  double ms;
  if (N > 0) {
    OK(pinn_plan_autotune(p, &nt.net, &pde, nt.x, N, 2, &best, &ms, nullptr));
    OK(pinn_plan_autotune(p, &nt.net, &pde, nt.x, N, 2, &best, &ms, nullptr));  // from the cache
    pinn_graph g = nullptr;
    OK(pinn_graph_capture(p, &nt.net, &pde, nt.x, N, nt.r, nt.loss, nt.dW.data(), nt.db.data(), &g));
    for (int k2 = 0; k2 < 3; ++k2) OK(pinn_graph_launch(g, nullptr));
    OK(pinn_graph_destroy(g));
    pinn_adam hp{1e-3, 0.9, 0.999, 1e-8};
    OK(pinn_graph_capture_train(p, &nt.net, &pde, nt.x, N, nt.r, nt.loss, nt.dW.data(), nt.db.data(), nt.mW.data(),
                                nt.vW.data(), nt.mb.data(), nt.vb.data(), &hp, nt.step, &g));
    OK(pinn_graph_launch(g, nullptr));
    OK(pinn_graph_destroy(g));
    OK(pinn_adam_step(H + 1, nt.dims.data(), nt.W.data(), nt.b.data(), (const float *const *)nt.dW.data(),
                      (const float *const *)nt.db.data(), nt.mW.data(), nt.vW.data(), nt.mb.data(), nt.vb.data(), 1,
                      &hp, nullptr));
  }
  for (int cls = 1; cls <= 8; ++cls) {
    OK(pinn_plan_profile(p, cls));
    step();
    int64_t n_l;
    OK(pinn_plan_profile_read(p, &ms, &n_l));
  }
  OK(pinn_plan_profile(p, 0));
  // argument errors
  STATUS(pinn_jet_residual(p, &nt.net, &pde, nt.x, N + 1, nt.r, nt.loss, nullptr, nullptr, nullptr), PINN_ERR_ARG);
  STATUS(pinn_jet_residual(p, &nt.net, &pde, nullptr, N, nt.r, nt.loss, nullptr, nullptr, nullptr), PINN_ERR_ARG);
  pinn_pde other = pde;
  other.kind = k.kind == PINN_BURGERS_1D ? PINN_KS_1D : PINN_BURGERS_1D;
  STATUS(pinn_jet_residual(p, &nt.net, &other, nt.x, N, nt.r, nt.loss, nullptr, nullptr, nullptr), PINN_ERR_ARG);
  OK(pinn_plan_destroy(p));
  if (l64) dev_free(l64);
  for (double *q : dW64) dev_free(q);
  for (double *q : db64) dev_free(q);
}

// ---------------------------------------------------------------- the modified MLP
void run_modified(int kind, int hidden, int width, int M, int64_t N) {
  const Kind &k = kind == PINN_KS_1D ? kKinds[2] : kKinds[0];
  pinn_pde pde = pde_of(k);
  pinn_modified arch{hidden, width, M, 6.283185307179586};
  pinn_plan p = nullptr;
  OK(pinn_plan_create_modified(&arch, &pde, N, PINN_FP32, 0, &p));
  const int de = 1 + 2 * M;
  Net nt(mlp(2, width, hidden, 1), N, k.C, 1);
  // parameter list: U, V, first layer (w x de), layers 2..hidden (w x w), output (1 x w)
  std::vector<float *> W, bb;
  for (int e = 0; e < 3; ++e) W.push_back((float *)dev_alloc((size_t)width * de * 4)), bb.push_back((float *)dev_alloc(width * 4));
  for (int e = 1; e < hidden; ++e) W.push_back((float *)dev_alloc((size_t)width * width * 4)), bb.push_back((float *)dev_alloc(width * 4));
  W.push_back((float *)dev_alloc(width * 4)), bb.push_back((float *)dev_alloc(4));
  std::vector<float *> dW, db;
  for (size_t e = 0; e < W.size(); ++e) dW.push_back((float *)dev_alloc((size_t)width * std::max(width, de) * 4)),
                                         db.push_back((float *)dev_alloc(width * 4));
  pinn_net net{hidden + 3, nullptr, (const float *const *)W.data(), (const float *const *)bb.data()};
  OK(pinn_jet_forward(p, &net, nt.x, N, nt.jets, nullptr));
  OK(pinn_jet_residual(p, &net, &pde, nt.x, N, nt.r, nt.loss, nullptr, nt.jets, nullptr));
  OK(pinn_jet_backward(p, &net, &pde, nt.x, N, nullptr, dW.data(), db.data(), nullptr, nullptr, nullptr));
  float *vals = (float *)dev_alloc((size_t)N * 4);
  pinn_segment segs[2] = {{PINN_SEG_PDE, 0, 0, N - N / 4, 1.0, 0, {}, nullptr},
                          {PINN_SEG_DIRICHLET, PINN_DATA_VALUES, N - N / 4, N / 4, 3.0, 1, {}, vals}};
  float *seg_loss = (float *)dev_alloc(64);
  OK(pinn_jet_loss(p, &net, &pde, segs, 2, nt.x, N, nt.loss, seg_loss, nullptr));
  OK(pinn_jet_loss_backward(p, &net, &pde, segs, 2, nt.x, N, dW.data(), db.data(), nullptr));
  STATUS(pinn_plan_autotune(p, &net, &pde, nt.x, N, 2, nullptr, nullptr, nullptr), PINN_ERR_UNSUPPORTED);
  pinn_graph g = nullptr;
  STATUS(pinn_graph_capture(p, &net, &pde, nt.x, N, nt.r, nt.loss, dW.data(), db.data(), &g), PINN_ERR_UNSUPPORTED);
  pinn_net short_net{hidden + 2, nullptr, (const float *const *)W.data(), (const float *const *)bb.data()};
  STATUS(pinn_jet_residual(p, &short_net, &pde, nt.x, N, nt.r, nt.loss, nullptr, nullptr, nullptr), PINN_ERR_ARG);
  OK(pinn_plan_destroy(p));
  for (auto *v : {&W, &bb, &dW, &db})
    for (float *q : *v) dev_free(q);
  dev_free(vals);
  dev_free(seg_loss);
}

// ---------------------------------------------------------------- the no-allocation step
void run_noalloc() {
  const Kind &k = kKinds[0];
  pinn_pde pde = pde_of(k);
  for (int prec : {PINN_FP32, PINN_BF16}) {
    for (int64_t N : {1, 300, 4096}) {
      Net nt(mlp(2, 32, 3, 1), N, k.C, 1);
      OK(pinn_jet_step_noalloc(&nt.net, &pde, prec, nt.x, N, nt.r, nt.loss, nt.dW.data(), nt.db.data(), nullptr));
    }
    Net big(mlp(2, 32, 3, 1), 1 << 20, k.C, 1);
    STATUS(pinn_jet_step_noalloc(&big.net, &pde, prec, big.x, 1 << 20, big.r, big.loss, big.dW.data(), big.db.data(),
                                 nullptr),
           PINN_ERR_CAP);
  }
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s ENSEMBLE_SHAPES CACHE_PATH\n", argv[0]);
    return 2;
  }
  // the ensemble as the benchmark drives it, under several clocks (the
  // autotuners then choose different tilings and lane layouts)
  for (uint64_t seed : {0ull, 1ull, 2ull, 3ull}) ensemble(argv[1], PINN_BF16, seed, 3);
  ensemble(argv[1], PINN_FP16, 5, 0);
  ensemble(argv[1], PINN_FP32, 6, 0);
  fprintf(stderr, "ensemble paths done (%d checks)\n", g_checks);
  // single plans
  for (const Kind &k : kKinds)
    for (int prec : {PINN_FP32, PINN_BF16, PINN_FP16})
      for (int w : {32, 64, 128, 256, 512}) {
        if (w == 512 && k.kind != PINN_HEAT_3D && k.kind != PINN_BURGERS_1D) continue;
        run_plan(k, prec, w, 3, 4099, 0, 0);
        if (w == 64 || w == 256) {
          run_plan(k, prec, w, 5, 1, 0, 0);
          run_plan(k, prec, w, 2, 200, PINN_VERIFY_F64, 0);
          run_plan(k, prec, w, 6, 3000, 0, (size_t)3000 * w * k.C * 4 * 2);  // checkpointed
        }
      }
  fprintf(stderr, "single-plan paths done (%d checks)\n", g_checks);
  for (int kind : {PINN_KS_1D, PINN_BURGERS_1D})
    for (int w : {64, 128, 256}) run_modified(kind, 3, w, kind == PINN_KS_1D ? 1 : 2, 777);
  run_modified(PINN_KS_1D, 6, 64, 8, 4608);
  // the tuning cache round trip
  int64_t entries = 0, entries2 = 0;
  OK(pinn_tuning_cache_size(&entries));
  OK(pinn_tuning_cache_save(argv[2]));
  OK(pinn_tuning_cache_clear());
  OK(pinn_tuning_cache_load(argv[2]));
  OK(pinn_tuning_cache_size(&entries2));
  if (entries != entries2 || entries == 0) {
    fprintf(stderr, "tuning cache round trip: %lld entries saved, %lld loaded\n", (long long)entries,
            (long long)entries2);
    return 1;
  }
  run_noalloc();
  size_t streams, events, graphs, execs, allocs;
  fake_hip_live(&streams, &events, &graphs, &execs, &allocs);
  if (streams || events || graphs || execs || allocs > 1 || fake_hip_capturing()) {
    fprintf(stderr, "left behind: %zu streams, %zu events, %zu graphs, %zu executable graphs, %zu allocations\n",
            streams, events, graphs, execs, allocs);
    return 1;
  }
  fprintf(stderr, "host paths OK: %d checks, %llu kernel launches checked\n", g_checks,
          (unsigned long long)fake_hip_launches());
  return 0;
}
