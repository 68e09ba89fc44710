// One Adam step (Kingma & Ba, Algorithm 1) over all parameter tensors of a
// network in one launch: the optimizer of the paper's training runs (full-batch
// Adam, Sec. 3.1).  FP32 parameters, gradients and moments.
#include "dev_common.hpp"
#include "group.hpp"
#include "kernels.hpp"

namespace pj {

// The y index of the (virtual) grid picks the tensor (segment); x strides over it.
// The step count comes by value or, for graph replays, from device memory; the
// bias corrections 1 - beta^step are formed here in either case.
struct KAdam {
  static constexpr int NT = 256;
  struct Args {
    AdamArgs a;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    const AdamArgs &a = a_.a;
    const int64_t t = a.step_dev ? *a.step_dev + 1 : a.step;
    const float c1 = 1.f - powf(a.b1, (float)t), c2 = 1.f - powf(a.b2, (float)t);
    const int s = vb.y;
    const int64_t n = a.n[s];
    float *__restrict__ p = a.p[s];
    const float *__restrict__ g = a.g[s];
    float *__restrict__ m = a.m[s];
    float *__restrict__ v = a.v[s];
    for (int64_t i = (int64_t)vb.x * 256 + threadIdx.x; i < n; i += (int64_t)vb.gx * 256) {
      const float gi = g[i];
      const float mi = a.b1 * m[i] + (1.f - a.b1) * gi;
      const float vi = a.b2 * v[i] + (1.f - a.b2) * gi * gi;
      m[i] = mi;
      v[i] = vi;
      p[i] -= a.lr * (mi / c1) / (sqrtf(vi / c2) + a.eps);
    }
  }
};

// Advances a device step counter after a graph's Adam update.
struct KStepCount {
  static constexpr int NT = 64;
  struct Args {
    int64_t * step;
  };
  static __device__ __forceinline__ void run(const Args &a_, VBlock vb) {
    int64_t * step = a_.step;
    if (threadIdx.x == 0) *step += 1;
  }
};

hipError_t launch_step_count(int64_t *step, hipStream_t st) {
  return launch_body<KStepCount>({step}, dim3(1), 0, st);
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t st) {
  int64_t nmax = 0;
  for (int s = 0; s < a.nseg; ++s) nmax = a.n[s] > nmax ? a.n[s] : nmax;
  const int64_t blocks = (nmax + 255) / 256;
  const dim3 grid((unsigned)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024), (unsigned)a.nseg);
  return launch_body<KAdam>({a}, grid, 0, st);
}

}  // namespace pj
