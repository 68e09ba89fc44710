// A stand-in for the HIP runtime that lets the library's host code run on a
// machine without a GPU, built with AddressSanitizer: plan and workspace
// management, the kernel schedules, the ensemble's recorded and grouped
// launches, graph capture, the autotuners and the tuning cache.  Kernels do
// not run.  Instead every launch is checked:
//   - the function was registered, the grid and block are non-empty and within
//     the hardware limits, dynamic LDS is at most 160 KiB and above 64 KiB only
//     after hipFuncSetAttribute raised the function's limit;
//   - a grouped launch's member table is well formed (ranges that tile the
//     grid, virtual grid widths that divide the ranges) and every member's
//     argument block lies in a live device allocation.
// Device memory is an inaccessible (PROT_NONE) address range that is never
// reused, so a host dereference of a device pointer faults, and a launch or
// copy that names freed memory is reported.  Events carry a synthetic clock
// (each launch advances it by a cost derived from its grid and a seed), so the
// autotuners pick different candidates under different seeds.
//
// Violations print "FAKE_HIP VIOLATION: ..." and abort.  With FAKE_HIP_TRACE
// set to a file name, every launch is also listed there (kernel, grid, block,
// dynamic LDS).
#include <hip/hip_runtime.h>
#include <cxxabi.h>
#include <sys/mman.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>

#include "group.hpp"

namespace {

[[noreturn]] void violation(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void violation(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  fprintf(stderr, "FAKE_HIP VIOLATION: ");
  vfprintf(stderr, fmt, ap);
  fprintf(stderr, "\n");
  va_end(ap);
  fflush(stderr);
  abort();
}

// ---------------------------------------------------------------- device memory
constexpr size_t kArena = size_t(1) << 42;  // address space only (PROT_NONE, no reserve)
struct Alloc {
  size_t size;
  bool live;
};

// ---------------------------------------------------------------- functions and variables
struct Func {
  std::string name;
  int max_dyn_lds = 64 * 1024;
};

// ---------------------------------------------------------------- streams, events, graphs
struct FakeStream {
  int magic = 0x5354;
  bool capturing = false;
};
struct FakeEvent {
  int magic = 0x4556;
  bool recorded = false;
  bool in_capture = false;
  double t = 0.0;
};
struct FakeGraph {
  int magic = 0x4752;
  double cost = 0.0;
};
struct FakeExec {
  int magic = 0x4758;
  double cost = 0.0;
};
// All state lives in one object built on first use: the library's module
// constructors may register their kernels before this file's globals would
// be initialised.
struct State {
  std::mutex mu;
  char *arena = nullptr;
  size_t top = 0;
  std::map<uintptr_t, Alloc> allocs;     // device allocations by start address
  std::map<const void *, Func> funcs;    // registered kernels by host stub
  std::map<const void *, void *> vars;   // registered device variables: host shadow -> device address
  std::set<void *> streams, events, graphs, execs;
  double clock = 0.0;                    // synthetic milliseconds
  bool capturing = false;                // a capture is open (relaxed mode: any stream's work joins it)
  double capture_cost = 0.0;
  uint64_t launches = 0;
  uint64_t seed = 0;
  FILE *trace = nullptr;
};
State &S() {
  static State *s = [] {
    State *n = new State;  // never destroyed: module destructors may still call in
    if (const char *path = getenv("FAKE_HIP_TRACE")) n->trace = fopen(path, "w");
    return n;
  }();
  return *s;
}

void *arena_alloc(size_t size) {
  if (!S().arena) {
    void *p = mmap(nullptr, kArena, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (p == MAP_FAILED) violation("cannot reserve the device address range");
    S().arena = static_cast<char *>(p);
  }
  size_t sz = (size + 255) & ~size_t(255);
  if (sz == 0) sz = 256;
  if (S().top + sz + 4096 > kArena) return nullptr;
  char *p = S().arena + S().top;
  S().top += sz + 4096;  // a gap after every allocation
  S().allocs[(uintptr_t)p] = Alloc{size, true};
  return p;
}

// The live allocation holding [p, p + n), or nullptr.
const Alloc *find_live(const void *p, size_t n) {
  auto it = S().allocs.upper_bound((uintptr_t)p);
  if (it == S().allocs.begin()) return nullptr;
  --it;
  const uintptr_t a = it->first;
  if ((uintptr_t)p < a || (uintptr_t)p + n > a + it->second.size || !it->second.live) return nullptr;
  return &it->second;
}

uint64_t mix(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

void check_stream(hipStream_t s, const char *what) {
  if (s && !S().streams.count((void *)s)) violation("%s: stream %p is not a live stream", what, (void *)s);
}
FakeEvent *check_event(hipEvent_t e, const char *what) {
  if (!S().events.count((void *)e)) violation("%s: event %p is not a live event", what, (void *)e);
  return reinterpret_cast<FakeEvent *>(e);
}

// pending launch configuration (the <<< >>> syntax pushes, the stub pops)
struct CallCfg {
  dim3 grid, block;
  size_t shm;
  hipStream_t st;
};
thread_local CallCfg g_cfg[4];
thread_local int g_cfg_n = 0;

}  // namespace

extern "C" {

// ---------------------------------------------------------------- registration (called by compiler-generated code)
void **__hipRegisterFatBinary(const void *) {
  static void *handle = nullptr;
  return &handle;
}
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *host_fn, char *, const char *device_name, int, void *, void *,
                           void *, void *, int *) {
  std::lock_guard<std::mutex> lk(S().mu);
  S().funcs[host_fn].name = device_name ? device_name : "?";
}
void __hipRegisterVar(void **, char *host_var, char *, const char *, int, size_t size, int, int) {
  std::lock_guard<std::mutex> lk(S().mu);
  S().vars[host_var] = arena_alloc(size);
}
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shm, hipStream_t st) {
  if (g_cfg_n >= 4) violation("launch configuration stack overflow");
  g_cfg[g_cfg_n++] = CallCfg{grid, block, shm, st};
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shm, hipStream_t *st) {
  if (g_cfg_n <= 0) violation("launch configuration stack underflow");
  const CallCfg &c = g_cfg[--g_cfg_n];
  *grid = c.grid;
  *block = c.block;
  *shm = c.shm;
  *st = c.st;
  return hipSuccess;
}

// ---------------------------------------------------------------- launches
hipError_t hipLaunchKernel(const void *fn, dim3 grid, dim3 block, void **args, size_t shm, hipStream_t st) {
  std::lock_guard<std::mutex> lk(S().mu);
  auto it = S().funcs.find(fn);
  if (it == S().funcs.end()) violation("launch of an unregistered function %p", fn);
  const Func &f = it->second;
  check_stream(st, f.name.c_str());
  const uint64_t threads = (uint64_t)block.x * block.y * block.z;
  if (grid.x == 0 || grid.y == 0 || grid.z == 0 || grid.y > 65535 || grid.z > 65535)
    violation("%s: grid %u x %u x %u", f.name.c_str(), grid.x, grid.y, grid.z);
  if (threads == 0 || threads > 1024) violation("%s: block of %llu threads", f.name.c_str(), (unsigned long long)threads);
  if (shm > 160 * 1024) violation("%s: %zu bytes of dynamic LDS", f.name.c_str(), shm);
  if ((int)shm > f.max_dyn_lds)
    violation("%s: %zu bytes of dynamic LDS above the function's limit %d", f.name.c_str(), shm, f.max_dyn_lds);
  if (f.name.find("k_grouped") != std::string::npos) {
    const pj::GroupTab &t = *static_cast<const pj::GroupTab *>(args[0]);
    if (t.n < 1 || t.n > pj::kGroupMax) violation("%s: %d members", f.name.c_str(), t.n);
    if (t.start[0] != 0 || t.start[t.n] != (int)grid.x)
      violation("%s: member ranges [%d, %d) do not tile the grid of %u", f.name.c_str(), t.start[0], t.start[t.n],
                grid.x);
    for (int e = 0; e < t.n; ++e) {
      const int nb = t.start[e + 1] - t.start[e];
      if (nb < 1 || t.gx[e] < 1 || nb % t.gx[e] != 0)
        violation("%s: member %d has %d workgroups on a grid of width %d", f.name.c_str(), e, nb, t.gx[e]);
      if (!find_live(t.args[e], 1)) violation("%s: member %d's argument block %p is not live device memory",
                                              f.name.c_str(), e, t.args[e]);
    }
  }
  if (S().trace) {
    int status = 0;
    char *dm = abi::__cxa_demangle(f.name.c_str(), nullptr, nullptr, &status);
    fprintf(S().trace, "%s grid %u x %u block %llu lds %zu%s\n", status == 0 && dm ? dm : f.name.c_str(), grid.x,
            grid.y, (unsigned long long)threads, shm, S().capturing ? " (captured)" : "");
    free(dm);
  }
  const double cost = ((double)grid.x * grid.y * grid.z * threads) * 1e-7 *
                      (1.0 + (double)(mix(S().seed ^ (uintptr_t)fn) % 1000) / 1000.0);
  ++S().launches;
  if (S().capturing) S().capture_cost += cost;
  else S().clock += cost;
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void *fn, hipFuncAttribute attr, int value) {
  std::lock_guard<std::mutex> lk(S().mu);
  auto it = S().funcs.find(fn);
  if (it == S().funcs.end()) violation("hipFuncSetAttribute on an unregistered function %p", fn);
  if (attr == hipFuncAttributeMaxDynamicSharedMemorySize) {
    if (value < 0 || value > 160 * 1024) return hipErrorInvalidValue;
    it->second.max_dyn_lds = value;
  }
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipPeekAtLastError(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }

// ---------------------------------------------------------------- memory
hipError_t hipMalloc(void **p, size_t size) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!p) return hipErrorInvalidValue;
  *p = arena_alloc(size);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!p) return hipSuccess;
  if (S().capturing) violation("hipFree during graph capture");
  auto it = S().allocs.find((uintptr_t)p);
  if (it == S().allocs.end()) violation("hipFree(%p): not the start of a device allocation", p);
  if (!it->second.live) violation("hipFree(%p): freed twice", p);
  it->second.live = false;
  return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind kind) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (S().capturing) violation("synchronous hipMemcpy during graph capture");
  if (kind != hipMemcpyHostToDevice) violation("hipMemcpy kind %d is not modelled", (int)kind);
  if (n == 0) return hipSuccess;
  if (!find_live(dst, n)) violation("hipMemcpy of %zu bytes to %p: outside live device memory", n, dst);
  volatile unsigned char sink = 0;  // the host source must be readable (AddressSanitizer checks it)
  for (size_t i = 0; i < n; ++i) sink ^= static_cast<const unsigned char *>(src)[i];
  (void)sink;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
  std::lock_guard<std::mutex> lk(S().mu);
  auto it = S().vars.find(symbol);
  if (it == S().vars.end()) return hipErrorInvalidSymbol;
  *p = it->second;
  return hipSuccess;
}

// ---------------------------------------------------------------- device
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *prop, int dev) {
  if (dev != 0) return hipErrorInvalidDevice;
  memset(prop, 0, sizeof *prop);
  snprintf(prop->name, sizeof prop->name, "fake gfx950");
  snprintf(prop->gcnArchName, sizeof prop->gcnArchName, "gfx950:sramecc+:xnack-");
  prop->multiProcessorCount = 256;
  prop->warpSize = 64;
  prop->sharedMemPerBlock = 160 * 1024;
  prop->maxThreadsPerBlock = 1024;
  return hipSuccess;
}

// ---------------------------------------------------------------- streams
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  FakeStream *f = new FakeStream;
  S().streams.insert(f);
  *s = reinterpret_cast<hipStream_t>(f);
  return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t *s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!S().streams.erase((void *)s)) violation("hipStreamDestroy(%p): not a live stream", (void *)s);
  delete reinterpret_cast<FakeStream *>(s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  check_stream(s, "hipStreamSynchronize");
  if (S().capturing) violation("hipStreamSynchronize during graph capture");
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  check_stream(s, "hipStreamWaitEvent");
  check_event(e, "hipStreamWaitEvent");
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  std::lock_guard<std::mutex> lk(S().mu);
  check_stream(s, "hipStreamBeginCapture");
  if (!s) violation("capture on the null stream");
  if (S().capturing) violation("nested graph capture");
  S().capturing = true;
  S().capture_cost = 0.0;
  reinterpret_cast<FakeStream *>(s)->capturing = true;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
  std::lock_guard<std::mutex> lk(S().mu);
  check_stream(s, "hipStreamEndCapture");
  if (!s || !reinterpret_cast<FakeStream *>(s)->capturing) violation("hipStreamEndCapture without a capture");
  reinterpret_cast<FakeStream *>(s)->capturing = false;
  S().capturing = false;
  FakeGraph *f = new FakeGraph;
  f->cost = S().capture_cost;
  S().graphs.insert(f);
  *g = reinterpret_cast<hipGraph_t>(f);
  return hipSuccess;
}

// ---------------------------------------------------------------- events
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  FakeEvent *f = new FakeEvent;
  S().events.insert(f);
  *e = reinterpret_cast<hipEvent_t>(f);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!S().events.erase((void *)e)) violation("hipEventDestroy(%p): not a live event", (void *)e);
  delete reinterpret_cast<FakeEvent *>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  FakeEvent *f = check_event(e, "hipEventRecord");
  check_stream(s, "hipEventRecord");
  f->recorded = true;
  f->in_capture = S().capturing;
  f->t = S().clock;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(S().mu);
  FakeEvent *f = check_event(e, "hipEventSynchronize");
  if (S().capturing) violation("hipEventSynchronize during graph capture");
  if (f->in_capture) violation("hipEventSynchronize on an event recorded inside a capture");
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lk(S().mu);
  FakeEvent *fa = check_event(a, "hipEventElapsedTime");
  FakeEvent *fb = check_event(b, "hipEventElapsedTime");
  if (!fa->recorded || !fb->recorded) return hipErrorInvalidHandle;
  if (fa->in_capture || fb->in_capture) violation("hipEventElapsedTime on events recorded inside a capture");
  *ms = (float)(fb->t - fa->t);
  return hipSuccess;
}

// ---------------------------------------------------------------- graphs
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!S().graphs.count((void *)g)) violation("hipGraphInstantiate: %p is not a live graph", (void *)g);
  FakeExec *f = new FakeExec;
  f->cost = reinterpret_cast<FakeGraph *>(g)->cost;
  S().execs.insert(f);
  *x = reinterpret_cast<hipGraphExec_t>(f);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!S().graphs.erase((void *)g)) violation("hipGraphDestroy(%p): not a live graph", (void *)g);
  delete reinterpret_cast<FakeGraph *>(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!S().execs.erase((void *)x)) violation("hipGraphExecDestroy(%p): not a live executable graph", (void *)x);
  delete reinterpret_cast<FakeExec *>(x);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!S().execs.count((void *)x)) violation("hipGraphLaunch(%p): not a live executable graph", (void *)x);
  check_stream(s, "hipGraphLaunch");
  if (S().capturing) violation("hipGraphLaunch during a capture is not modelled");
  S().clock += reinterpret_cast<FakeExec *>(x)->cost;
  return hipSuccess;
}

// ---------------------------------------------------------------- for the driver
void fake_hip_set_seed(uint64_t seed) {
  std::lock_guard<std::mutex> lk(S().mu);
  S().seed = seed;
}
uint64_t fake_hip_launches(void) {
  std::lock_guard<std::mutex> lk(S().mu);
  return S().launches;
}
// Live streams, events, graphs and executable graphs, and live allocations.
void fake_hip_live(size_t *streams, size_t *events, size_t *graphs, size_t *execs, size_t *allocs) {
  std::lock_guard<std::mutex> lk(S().mu);
  *streams = S().streams.size();
  *events = S().events.size();
  *graphs = S().graphs.size();
  *execs = S().execs.size();
  size_t n = 0;
  for (const auto &kv : S().allocs) n += kv.second.live;
  *allocs = n;
}
int fake_hip_capturing(void) { return S().capturing; }

}  // extern "C"
