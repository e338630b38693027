// Work list of the persistent pair kernels (Alg. 1 CallQuadratic over all
// cells of uneven occupancy in one launch): one item per chunk of at most ti
// consecutive slots of a cell, in cell order. The items are split into 8
// contiguous ranges (queues), one per XCD, so neighbouring cells tend to be
// processed on the same XCD and share its L2; idle workgroups steal from the
// other queues. Each item writes only its own particles' outputs, so the
// results do not depend on which workgroup takes which item.
//
// Buffer layout: [0, kWorkHeader) counters[8] and meta (item count, queue
// boundaries[9]); then per-cell item offsets [C + 1] and scan partials; then
// the items (int2: cell, first slot).
#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct WlLayout {
  int32_t* pos;       // [C + 1]
  int32_t* partials;
  int2* items;
};

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

WlLayout wl_layout(void* buf, int C, int capacity) {
  char* p = static_cast<char*>(buf) + kWorkHeader;
  WlLayout L;
  L.pos = reinterpret_cast<int32_t*>(p);
  p += al256(sizeof(int32_t) * ((size_t)C + 1));
  L.partials = reinterpret_cast<int32_t*>(p);
  p += al256(sizeof(int32_t) * scan_partials_count(C + 1));
  L.items = reinterpret_cast<int2*>(p);
  (void)capacity;
  return L;
}

__global__ __launch_bounds__(kThreads) void k_wl_count(const int32_t* __restrict__ start, int C,
                                                        int n, int ti, int32_t* __restrict__ pos) {
  int c = blockIdx.x * kThreads + threadIdx.x;
  if (c > C) return;
  if (c == C) {
    pos[C] = 0;
    return;
  }
  const int a = min(max(start[c], 0), n), b = min(max(start[c + 1], a), n);
  pos[c] = (b - a + ti - 1) / ti;
}

__global__ __launch_bounds__(kThreads) void k_wl_fill(const int32_t* __restrict__ start, int C,
                                                       int n, int ti, int capacity,
                                                       const int32_t* __restrict__ pos,
                                                       int2* __restrict__ items) {
  int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= C) return;
  const int a = min(max(start[c], 0), n), b = min(max(start[c + 1], a), n);
  int o = pos[c];
  for (int f = a; f < b && o < capacity; f += ti, ++o) items[o] = make_int2(c, f);
}

__global__ void k_wl_meta(const int32_t* __restrict__ pos, int C, int capacity,
                          int32_t* __restrict__ counters, int32_t* __restrict__ meta) {
  if (threadIdx.x == 0) {
    const int total = min(pos[C], capacity);
    meta[0] = total;
    for (int q = 0; q <= kQueues; ++q) meta[1 + q] = (int)(((int64_t)total * q) / kQueues);
    for (int q = 0; q < kQueues; ++q) counters[q] = meta[1 + q];
  }
}

}  // namespace

int worklist_capacity(int n, int n_c, int ti) {
  const int64_t C = (int64_t)n_c * n_c * n_c;
  const int64_t cap = C + (int64_t)n / (ti > 0 ? ti : 1) + 1;
  return (int)(cap < (1LL << 30) ? cap : (1LL << 30));
}

size_t worklist_bytes(int n, int n_c, int ti) {
  const int C = n_c * n_c * n_c;
  const int cap = worklist_capacity(n, n_c, ti);
  return kWorkHeader + al256(sizeof(int32_t) * ((size_t)C + 1)) +
         al256(sizeof(int32_t) * scan_partials_count(C + 1)) + sizeof(int2) * (size_t)cap;
}

hipError_t launch_worklist(const CellsDev& c, const WorkDev& w, hipStream_t s) {
  const int C = c.n_c * c.n_c * c.n_c;
  WlLayout L = wl_layout(reinterpret_cast<char*>(w.counters), C, w.capacity);
  k_wl_count<<<cdiv(C + 1, kThreads), kThreads, 0, s>>>(c.start, C, c.n, w.ti, L.pos);
  hipError_t e = scan_i32(L.pos, C + 1, L.partials, s);
  if (e != hipSuccess) return e;
  k_wl_fill<<<cdiv(C, kThreads), kThreads, 0, s>>>(c.start, C, c.n, w.ti, w.capacity, L.pos,
                                                    w.items);
  k_wl_meta<<<1, 64, 0, s>>>(L.pos, C, w.capacity, w.counters, w.meta);
  return hipGetLastError();
}

WorkDev work_view(const sph_work& w, int n, int n_c) {
  WorkDev d;
  d.ti = w.ti;
  d.capacity = worklist_capacity(n, n_c, w.ti);
  char* base = static_cast<char*>(w.buf);
  d.counters = reinterpret_cast<int32_t*>(base);
  d.meta = reinterpret_cast<int32_t*>(base + 64);
  const int C = n_c * n_c * n_c;
  d.items = wl_layout(base, C, d.capacity).items;
  return d;
}

}  // namespace sph
