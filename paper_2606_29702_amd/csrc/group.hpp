// Kernel bodies on virtual grids, launched either directly or grouped.
//
// Every kernel of the library is a body B with
//   B::NT          threads per workgroup
//   B::Args        its argument block (plain data: pointers and scalars)
//   B::run(a, vb)  the work of one workgroup, given its place vb in a virtual
//                  grid of vb.gx x vb.gy workgroups (the body never reads
//                  blockIdx or gridDim).
// A direct launch runs one virtual grid as the physical grid.  A grouped
// launch runs the virtual grids of several members (the same body with one
// argument block per network of an ensemble) as one physical grid: member e
// owns the consecutive workgroups start[e] .. start[e+1]-1.  Each member keeps
// its own grid shape, tile order and partial-sum slots, so a grouped launch
// computes bit for bit what the members' direct launches compute.
//
// While a Recorder is installed on the host thread, launch_body appends a
// record (body, argument bytes, grid, dynamic LDS) instead of launching; the
// ensemble step replays the records of all its networks as grouped launches.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

namespace pj {

struct VBlock {
  int x, y, gx, gy;
  int p0;  // physical index of the virtual grid's first workgroup
};

// Workgroups of one launch are dealt round-robin to the 8 XCDs (physical
// index i runs on XCD i % 8), and each XCD has its own L2.  xcd_order maps the
// virtual block to a logical index in [0, gx * gy) such that consecutive
// logical indices run on the same XCD: a kernel that gives consecutive logical
// indices work on the same data (the neuron tiles of one point tile, the
// weight tiles of one split) then reads that data into one L2 instead of
// several.  The map is a bijection; blocks before the first and after the last
// whole round of 8 keep their index.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_order(const VBlock &vb) {
  const int G = vb.gx * vb.gy, v = vb.x + vb.y * vb.gx;
  const int h = (kXcds - vb.p0 % kXcds) % kXcds;  // head blocks before the first whole round
  const int R = G > h ? (G - h) / kXcds : 0;      // whole rounds
  const int u = v - h;
  if (u < 0 || u >= kXcds * R) return v;
  return h + (u % kXcds) * R + u / kXcds;
}

constexpr int kGroupMax = 64;  // members per grouped launch

struct GroupTab {
  int n;                        // members
  int start[kGroupMax + 1];     // physical workgroup ranges, start[0] = 0
  int gx[kGroupMax];            // virtual grid width of each member
  const void *args[kGroupMax];  // argument block of each member (device memory)
};

template <class B>
__global__ __launch_bounds__(B::NT) void k_direct(typename B::Args a) {
  B::run(a, VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y, 0});
}

template <class B>
__global__ __launch_bounds__(B::NT) void k_grouped(GroupTab t) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = t.n - 1;  // the member whose range holds b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t.start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int v = b - t.start[lo], gx = t.gx[lo];
  const int gy = (t.start[lo + 1] - t.start[lo]) / gx;
  B::run(*static_cast<const typename B::Args *>(t.args[lo]), VBlock{v % gx, v / gx, gx, gy, t.start[lo]});
}

// One recorded launch.
struct LaunchRecord {
  const void *key;  // the body: address of its grouped kernel
  int cls = 0;      // kernel class (PINN_K_*) of the launch site, for timing
  hipError_t (*launch_group)(const GroupTab &t, int blocks, size_t lds, hipStream_t st);
  std::vector<unsigned char> args;
  int gx = 0, gy = 0;
  size_t lds = 0;
};

struct Recorder {
  std::vector<LaunchRecord> recs;
};

// The recorder of the calling host thread (null: launches run), and the
// kernel class the host code is launching (stored in each record).
Recorder *&current_recorder();
int &current_record_class();

template <class B>
hipError_t launch_group_of(const GroupTab &t, int blocks, size_t lds, hipStream_t st) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)k_grouped<B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_grouped<B>, dim3((unsigned)blocks), dim3(B::NT), lds, st, t);
  return hipGetLastError();
}

// Launches (or records) body B over a virtual grid.
template <class B>
hipError_t launch_body(const typename B::Args &a, dim3 grid, size_t lds, hipStream_t st) {
  if (grid.x == 0 || grid.y == 0) return hipSuccess;
  if (Recorder *r = current_recorder()) {
    LaunchRecord rec;
    rec.key = (const void *)k_grouped<B>;
    rec.cls = current_record_class();
    rec.launch_group = launch_group_of<B>;
    rec.args.resize(sizeof(typename B::Args));
    std::memcpy(rec.args.data(), &a, sizeof(typename B::Args));
    rec.gx = (int)grid.x;
    rec.gy = (int)grid.y;
    rec.lds = lds;
    r->recs.push_back(std::move(rec));
    return hipSuccess;
  }
  if (lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute((const void *)k_direct<B>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_direct<B>, grid, dim3(B::NT), lds, st, a);
  return hipGetLastError();
}

}  // namespace pj
