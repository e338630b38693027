// Work list of the pair kernels for one launch over all cells of uneven
// occupancy (Alg. 1 CallQuadratic): one item per chunk of at most ti
// consecutive slots of a cell, the cells in brick order (brick_cell). The
// items are split into 8 contiguous ranges, one per XCD, so neighbouring
// cells are processed on the same XCD and share its L2. The ranges balance
// an estimated cost rather than the item count: a chunk of a cell costs
// about (its particle count) x (the particle count of the 27 cells around
// it, capped at 27 x 64) candidate tests, so a few crowded cells weigh as
// much as many sparse ones. Each item writes only its own particles'
// outputs, so no result depends on the split, the order or the schedule.
//
// Buffer layout: [0, kWorkHeader) queue counters[8] and meta (item count,
// range boundaries[9]); then the item offsets [C + 1] and the cost prefix
// [C + 1] of the cells in brick order, one set of scan partials, and the
// items (int2: cell, first slot).
#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;
constexpr int kCostShift = 12;   // cost unit: 4096 candidate tests
constexpr int kNbCap = 27 * 64;  // neighbour-count cap of the cost estimate

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct WlLayout {
  int32_t* pos;       // [C + 1] first item of each cell (brick order)
  int32_t* cost;      // [C + 1] exclusive prefix of the cell costs (brick order)
  int32_t* partials;
  int2* items;
};

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

WlLayout wl_layout(void* buf, int C) {
  char* p = static_cast<char*>(buf) + kWorkHeader;
  WlLayout L;
  L.pos = reinterpret_cast<int32_t*>(p);
  p += al256(sizeof(int32_t) * ((size_t)C + 1));
  L.cost = reinterpret_cast<int32_t*>(p);
  p += al256(sizeof(int32_t) * ((size_t)C + 1));
  L.partials = reinterpret_cast<int32_t*>(p);
  p += al256(sizeof(int32_t) * scan_partials_count(C + 1));
  L.items = reinterpret_cast<int2*>(p);
  return L;
}

__device__ __forceinline__ int cell_count(const int32_t* __restrict__ start, int c, int n) {
  const int a = min(max(start[c], 0), n);
  return max(min(max(start[c + 1], 0), n) - a, 0);
}

// Merged items: in a launch over an occupancy class, consecutive non-empty
// cells of the class along x within one row of a brick (bricks are 4 cells
// wide) are grouped greedily from the row's first cell, up to `merge` cells
// whose particles fit one tile; a cell outside the class, an empty cell or
// a cell with more than ti particles ends a group and is not merged. The
// group's first cell carries one item for all of its slots (a contiguous
// slot range: cells of a row are consecutive in id order); the others carry
// none. Returns the group size m of cell c's group if c starts one (1 for an
// unmerged cell), 0 if c is inside a group started by another cell.
__device__ __forceinline__ int merge_group(const int32_t* __restrict__ start, int n, int n_c,
                                           int ti, int merge, int occ_lo, int occ_hi, int c) {
  int cx, cy, cz;
  cell_coords(c, n_c, cx, cy, cz);
  const int x0 = cx - cx % kBrick, tx = min(kBrick, n_c - x0);
  int rc[kBrick];
#pragma unroll
  for (int l = 0; l < kBrick; ++l) {
    int k = -1;
    if (l < tx) {
      k = cell_count(start, (x0 + l) + n_c * (cy + n_c * cz), n);
      if (k <= 0 || k < occ_lo || k >= occ_hi || k > ti) k = -1;   // not mergeable
    }
    rc[l] = k;
  }
  int l = 0;
  while (l < tx) {
    int m = 1;
    if (rc[l] > 0) {
      int sum = rc[l];
      while (l + m < tx && m < merge && rc[l + m] > 0 && sum + rc[l + m] <= ti) sum += rc[l + m++];
    }
    if (cx - x0 == l) return m;
    if (cx - x0 < l + m) return 0;
    l += m;
  }
  return 1;
}

// Items per cell and the cell's cost estimate, clamped so that the sum over
// all cells fits in int32.
__global__ __launch_bounds__(kThreads) void k_wl_count(const int32_t* __restrict__ start, int n_c,
                                                        int n, int ti, int cost_cap,
                                                        const uint8_t* __restrict__ active,
                                                        int occ_lo, int occ_hi, int merge,
                                                        int32_t* __restrict__ pos,
                                                        int32_t* __restrict__ cost,
                                                        const int32_t* gate) {
  if (gate && *gate == 0) return;             // the cell list was kept: so is this list
  const int C = n_c * n_c * n_c;
  const int j = blockIdx.x * kThreads + threadIdx.x;   // position in brick order
  if (j > C) return;
  if (j == C) {
    pos[C] = 0;
    cost[C] = 0;
    return;
  }
  const int c = brick_cell(j, n_c);
  int cnt = cell_count(start, c, n);
  if (cnt < occ_lo || cnt >= occ_hi) cnt = 0;   // only cells of this occupancy class
  if (active && cnt > 0) {   // only cells that hold an active slot
    const int a = min(max(start[c], 0), n);
    bool any = false;
    for (int k = a; k < a + cnt && !any; ++k) any = active[k] != 0;
    if (!any) cnt = 0;
  }
  if (merge > 1 && cnt > 0 && cnt <= ti) {
    const int m = merge_group(start, n, n_c, ti, merge, occ_lo, occ_hi, c);
    pos[j] = m > 0 ? 1 : 0;          // the group's first cell holds its one item
  } else {
    pos[j] = (cnt + ti - 1) / ti;
  }
  int cx, cy, cz;
  cell_coords(c, n_c, cx, cy, cz);
  int64_t nb = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = (cz + dz + n_c) % n_c;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = (cy + dy + n_c) % n_c;
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = (cx + dx + n_c) % n_c;
        nb += cell_count(start, x + n_c * (y + n_c * z), n);
      }
    }
  }
  // a chunk stages about the particles within a support radius of it; with
  // h following the density that is a bounded number even next to crowded
  // cells, so the neighbour count is capped at that of a 64-per-cell lattice
  const int64_t raw = (int64_t)cnt * min(nb, (int64_t)kNbCap);
  const int64_t units = (raw + (1 << kCostShift) - 1) >> kCostShift;
  cost[j] = (int32_t)min(units, (int64_t)cost_cap);
}

__global__ __launch_bounds__(kThreads) void k_wl_fill(const int32_t* __restrict__ start, int n_c,
                                                       int n, int ti, int capacity, int merge,
                                                       int occ_lo, int occ_hi,
                                                       const int32_t* __restrict__ pos,
                                                       int2* __restrict__ items,
                                                       const int32_t* gate) {
  if (gate && *gate == 0) return;
  const int C = n_c * n_c * n_c;
  const int j = blockIdx.x * kThreads + threadIdx.x;   // position in brick order
  if (j >= C) return;
  const int c = brick_cell(j, n_c);
  const int a = min(max(start[c], 0), n), b = min(max(start[c + 1], a), n);
  int o = pos[j];
  const int end = min(pos[j + 1], capacity);   // this cell's items (none if filtered out)
  if (merge > 1 && o < end && b - a <= ti) {   // one item: the cell or its merged group
    const int m = max(merge_group(start, n, n_c, ti, merge, occ_lo, occ_hi, c), 1);
    items[o] = make_int2(c | ((m - 1) << kMergeShift), a);
    return;
  }
  for (int f = a; f < b && o < end; f += ti, ++o) items[o] = make_int2(c, f);
}

// Range boundaries: range q starts at the first item of the first cell (in
// brick order) whose cost prefix reaches q/8 of the total.
__global__ void k_wl_meta(const int32_t* __restrict__ pos, const int32_t* __restrict__ cost,
                          int C, int capacity, int32_t* __restrict__ counters,
                          int32_t* __restrict__ meta, const int32_t* gate) {
  if (gate && *gate == 0) return;
  const int q = threadIdx.x;
  const int total = min(pos[C], capacity);
  if (q == 0) meta[0] = total;
  if (q > kQueues) return;
  int b;
  if (q == 0) {
    b = 0;
  } else if (q == kQueues) {
    b = total;
  } else {
    const int64_t target = ((int64_t)cost[C] * q + kQueues - 1) / kQueues;
    int lo = 0, hi = C;   // smallest c with cost[c] >= target
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cost[mid] >= target) hi = mid;
      else lo = mid + 1;
    }
    b = min(pos[lo], total);
  }
  meta[1 + q] = b;
  if (q < kQueues) counters[q] = b;
}

}  // namespace

int worklist_capacity(int n, int n_c, int ti) {
  const int64_t C = (int64_t)n_c * n_c * n_c;
  const int64_t t = ti > 0 ? ti : 1;
  const int64_t occupied = C < n ? C : n;
  const int64_t cap = (n + (t - 1) * occupied) / t + 1;
  return (int)(cap < (1LL << 30) ? cap : (1LL << 30));
}

size_t worklist_bytes(int n, int n_c, int ti) {
  const int C = n_c * n_c * n_c;
  const int cap = worklist_capacity(n, n_c, ti);
  return kWorkHeader + 2 * al256(sizeof(int32_t) * ((size_t)C + 1)) +
         al256(sizeof(int32_t) * scan_partials_count(C + 1)) + sizeof(int2) * (size_t)cap;
}

hipError_t launch_worklist(const CellsDev& c, const WorkDev& w, hipStream_t s) {
  return launch_worklist_active(c, w, nullptr, s);
}

hipError_t launch_worklist_active(const CellsDev& c, const WorkDev& w, const uint8_t* active,
                                  hipStream_t s) {
  return launch_worklist_range(c, w, active, 0, 0x7fffffff, s);
}

hipError_t launch_worklist_range(const CellsDev& c, const WorkDev& w, const uint8_t* active,
                                 int occ_lo, int occ_hi, hipStream_t s, const int32_t* gate) {
  const int C = c.n_c * c.n_c * c.n_c;
  WlLayout L = wl_layout(reinterpret_cast<char*>(w.counters), C);
  const int cost_cap = (int)((((int64_t)1 << 31) - 1) / ((int64_t)C + 1));
  // merged items only for plain lists (the h iteration's lists filter cells)
  const int merge = active ? 1 : w.merge;
  k_wl_count<<<cdiv(C + 1, kThreads), kThreads, 0, s>>>(c.start, c.n_c, c.n, w.ti, cost_cap,
                                                         active, occ_lo, occ_hi, merge, L.pos,
                                                         L.cost, gate);
  hipError_t e = scan_i32(L.pos, C + 1, L.partials, s, gate);
  if (e != hipSuccess) return e;
  e = scan_i32(L.cost, C + 1, L.partials, s, gate);
  if (e != hipSuccess) return e;
  k_wl_fill<<<cdiv(C, kThreads), kThreads, 0, s>>>(c.start, c.n_c, c.n, w.ti, w.capacity, merge,
                                                    occ_lo, occ_hi, L.pos, w.items, gate);
  k_wl_meta<<<1, 64, 0, s>>>(L.pos, L.cost, C, w.capacity, w.counters, w.meta, gate);
  return hipGetLastError();
}

WorkDev work_view(const sph_work& w, int n, int n_c) {
  WorkDev d;
  d.ti = w.ti;
  d.sched = w.sched;
  d.capacity = worklist_capacity(n, n_c, w.ti);
  d.merge = w.max_cells > 1 ? min(w.max_cells, kMaxMerge) : 1;
  char* base = static_cast<char*>(w.buf);
  d.counters = reinterpret_cast<int32_t*>(base);
  d.meta = reinterpret_cast<int32_t*>(base + 64);
  const int C = n_c * n_c * n_c;
  d.items = wl_layout(base, C).items;
  return d;
}

}  // namespace sph
