// Cell binning: FP64 cell ids, a stable LSD radix sort by cell id, and the
// CSR cell_start table. The order is stable by (cell id, input index), so
// the permutation is identical on every run and on every device.
#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 8;
constexpr int kTile = kThreads * kRounds;     // keys per radix block
constexpr int kScanPer = 16;                  // elements per thread in scans
constexpr int kScanTile = kThreads * kScanPer;
constexpr int kMaxBuckets = 512;             // radix buckets of the widest digit (9 bits)

// A gated launch does nothing when *gate == 0 (the cell list is kept: no
// particle changed its cell or sub-cell since it was built). The word is
// read at the start of each kernel; only the last kernel of the binning
// changes it.
__device__ __forceinline__ bool gated_off(const int32_t* gate) { return gate && *gate == 0; }

// Morton code of a sub-cell (bit b of sx at 3b, sy at 3b+1, sz at 3b+2)
__device__ __forceinline__ int morton3(int sx, int sy, int sz, int bits) {
  int m = 0;
  for (int b = 0; b < bits; ++b)
    m |= (((sx >> b) & 1) << (3 * b)) | (((sy >> b) & 1) << (3 * b + 1)) |
         (((sz >> b) & 1) << (3 * b + 2));
  return m;
}

// Largest record span staged through LDS by k_bin_keys (8-byte words)
constexpr int kSpanWords = 16;

// key = cell * R^3 + Morton(sub-cell); also h of each record for the
// per-cell maximum.
// nw > 0: the block first copies bytes [lo, lo + 8 nw) of each of its
// records into LDS with consecutive threads on consecutive words (x and h
// read from there), so every record line is fetched once and the loads
// coalesce; nw = 0: each thread reads its record's fields directly.
__global__ __launch_bounds__(kThreads) void k_bin_keys(const char* __restrict__ aos,
                                                        uint32_t stride, uint32_t offx,
                                                        uint32_t offh, int dth, uint32_t lo,
                                                        int nw, int n, int n_c, int sub_bits,
                                                        int32_t* __restrict__ keys,
                                                        int32_t* __restrict__ vals,
                                                        float* __restrict__ hin,
                                                        int32_t* status, const int32_t* gate) {
  __shared__ uint2 span[kThreads * kSpanWords];
  if (gated_off(gate)) return;                 // uniform over the grid
  const int i0 = blockIdx.x * kThreads;
  const int i = i0 + threadIdx.x;
  const bool valid = i < n;   // no early exit: the whole block stages the records
  const char* rec;            // record bytes as seen at offsets offx, offh
  uint32_t rx = offx, rh = offh;
  if (nw > 0) {
    // every word of the block's spans: a thread's loads (at most
    // kSpanWords) are all issued before the first is stored to LDS
    const int nrec = min(kThreads, n - i0);
    const int nwords = nrec * nw;
    uint2 buf[kSpanWords];
#pragma unroll
    for (int q = 0; q < kSpanWords; ++q) {
      const int w = threadIdx.x + q * kThreads;
      buf[q] = make_uint2(0u, 0u);
      if (w < nwords) {
        const int r = w / nw, j = w - r * nw;
        buf[q] = *reinterpret_cast<const uint2*>(aos + (size_t)(i0 + r) * stride + lo + 8 * j);
      }
    }
#pragma unroll
    for (int q = 0; q < kSpanWords; ++q) {
      const int w = threadIdx.x + q * kThreads;
      if (w < nwords) span[w] = buf[q];
    }
    __syncthreads();
    rec = reinterpret_cast<const char*>(span + (valid ? threadIdx.x : 0) * nw);
    rx = offx - lo;
    rh = offh - lo;
  } else {
    rec = aos + (size_t)(valid ? i : 0) * stride;
  }
  const double* x = reinterpret_cast<const double*>(rec + rx);
  const int R = 1 << sub_bits;
  bool bad = false;
  int c[3], sc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double xv = x[k];
    bad |= !isfinite(xv);
    const double xw = wrap01(xv);
    c[k] = cell_axis(xw, n_c);
    const double t = floor(xw * (double)(n_c * R));
    int sa = (t == t) ? (int)fmin(fmax(t - (double)c[k] * R, 0.0), (double)(R - 1)) : 0;
    sc[k] = sa;
  }
  const int cell = c[0] + n_c * (c[1] + n_c * c[2]);
  if (valid) {
    keys[i] = (cell << (3 * sub_bits)) + morton3(sc[0], sc[1], sc[2], sub_bits);
    vals[i] = i;
  }
  // h of each input slot (0 where not positive): the per-cell maximum is
  // taken after the sort, without atomics on the words of crowded cells
  if (hin && valid) {
    const float h = rec_load32(rec, rh, dth);
    hin[i] = h > 0.0f ? h : 0.0f;
  }
  if (valid && bad && status) atomicOr(status, SPH_FLAG_BAD_POSITION);
}

__global__ __launch_bounds__(kThreads) void k_fill_f32(float* __restrict__ p, int n, float v,
                                                        const int32_t* gate) {
  if (gated_off(gate)) return;
  int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per-block digit counts of one pass (D-bit digits, 2^D buckets), stored
// digit-major so that one exclusive scan gives every block's base offsets.
template <int D>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const int32_t* __restrict__ kin,
                                                          int32_t* __restrict__ hist, int n,
                                                          int nblk, int shift, const int32_t* gate) {
  constexpr int NB = 1 << D;
  __shared__ int h[NB];
  if (gated_off(gate)) return;
  const int tid = threadIdx.x;
  for (int d = tid; d < NB; d += kThreads) h[d] = 0;
  __syncthreads();
  const int b = blockIdx.x;
  for (int r = 0; r < kRounds; ++r) {
    int idx = b * kTile + r * kThreads + tid;
    if (idx < n) atomicAdd(&h[(kin[idx] >> shift) & (NB - 1)], 1);
  }
  __syncthreads();
  for (int d = tid; d < NB; d += kThreads) hist[d * nblk + b] = h[d];
}

// --- exclusive scan of int32 (three kernels: tile scan, partials, add) ---
__device__ __forceinline__ int block_exclusive_scan(int v, int* lds, int& total) {
  // Hillis-Steele over 256 threads in LDS
  int tid = threadIdx.x;
  lds[tid] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int t = tid >= off ? lds[tid - off] : 0;
    __syncthreads();
    lds[tid] += t;
    __syncthreads();
  }
  int incl = lds[tid];
  total = lds[kThreads - 1];
  __syncthreads();
  return incl - v;
}

// Stable scatter straight to global memory (9-bit digits: with 512 buckets a
// tile's digit runs are too short for the local reorder below to pay): in
// round r the block ranks keys b*kTile + r*256 + tid in index order. Lanes
// with equal digits are found with D ballots; earlier waves and earlier
// rounds are counted in LDS.
template <int D>
__global__ __launch_bounds__(kThreads) void k_radix_scatter_direct(
    const int32_t* __restrict__ kin, const int32_t* __restrict__ vin, int32_t* __restrict__ kout,
    int32_t* __restrict__ vout, const int32_t* __restrict__ offsets, int n, int nblk, int shift,
    const int32_t* gate) {
  constexpr int NB = 1 << D;
  __shared__ int wcnt[kThreads / 64][NB];
  if (gated_off(gate)) return;
  __shared__ int run[NB];
  __shared__ int base[NB];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int b = blockIdx.x;
  for (int d = tid; d < NB; d += kThreads) {
    base[d] = offsets[d * nblk + b];
    run[d] = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) wcnt[w][d] = 0;
  }
  __syncthreads();
  for (int r = 0; r < kRounds; ++r) {
    int idx = b * kTile + r * kThreads + tid;
    if (b * kTile + r * kThreads >= n) break;     // uniform over the block
    bool valid = idx < n;
    int key = valid ? kin[idx] : 0;
    int val = valid ? vin[idx] : 0;
    int d = (key >> shift) & (NB - 1);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < D; ++bit) {
      uint64_t bl = __ballot((d >> bit) & 1);
      m &= ((d >> bit) & 1) ? bl : ~bl;
    }
    int rank = __popcll(m & lanemask_lt());
    if (valid && rank == 0) wcnt[wave][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      int pre = run[d];
      for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
      int pos = base[d] + pre + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    for (int dd = tid; dd < NB; dd += kThreads) {
      int tot = 0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) {
        tot += wcnt[w][dd];
        wcnt[w][dd] = 0;
      }
      run[dd] += tot;
    }
    __syncthreads();
  }
}

// Stable scatter of one block's tile of kTile keys: the keys are ranked in
// index order (round r holds keys b*kTile + r*256 + tid; lanes with equal
// digits are found with D ballots, earlier waves and rounds are counted in
// LDS) into a block-local order sorted by digit in LDS, and then written out
// digit run by digit run, so consecutive threads store consecutive
// addresses. The block's count of each digit is the difference of two
// consecutive entries of the scanned digit-major histogram.
template <int D>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const int32_t* __restrict__ kin, const int32_t* __restrict__ vin, int32_t* __restrict__ kout,
    int32_t* __restrict__ vout, const int32_t* __restrict__ offsets, int n, int nblk, int shift,
    const int32_t* gate) {
  constexpr int NB = 1 << D;
  constexpr int PER = NB / kThreads;           // digits per thread in the local scan
  static_assert(NB % kThreads == 0, "whole digits per thread");
  __shared__ int wcnt[kThreads / 64][NB];
  __shared__ int run[NB];
  __shared__ int lstart[NB];                   // first local position of each digit
  __shared__ int gbase[NB];                    // global position of the block's first key of each digit
  __shared__ int2 tile[kTile];                 // (key, value) in local digit order
  __shared__ int scan_lds[kThreads];
  if (gated_off(gate)) return;
  const int tid = threadIdx.x, wave = tid >> 6;
  const int b = blockIdx.x;
  const int t0 = b * kTile;
  const int ntile = min(kTile, n - t0);
  // every load of the tile in flight before the ranking
  int key[kRounds], val[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int idx = t0 + r * kThreads + tid;
    key[r] = idx < n ? kin[idx] : 0;
    val[r] = idx < n ? vin[idx] : 0;
  }
  int cnt[PER];
  int csum = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int d = tid * PER + q;
    const int e = d * nblk + b;
    const int o = offsets[e];
    const int o1 = e + 1 < NB * nblk ? offsets[e + 1] : n;
    gbase[d] = o;
    cnt[q] = o1 - o;
    csum += cnt[q];
    run[d] = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) wcnt[w][d] = 0;
  }
  int total;
  int ex = block_exclusive_scan(csum, scan_lds, total);   // barriers inside
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    lstart[tid * PER + q] = ex;
    ex += cnt[q];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (t0 + r * kThreads >= n) break;         // uniform over the block
    const int idx = t0 + r * kThreads + tid;
    const bool valid = idx < n;
    const int d = (key[r] >> shift) & (NB - 1);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < D; ++bit) {
      const uint64_t bl = __ballot((d >> bit) & 1);
      m &= ((d >> bit) & 1) ? bl : ~bl;
    }
    const int rank = __popcll(m & lanemask_lt());
    if (valid && rank == 0) wcnt[wave][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      int pre = run[d];
      for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
      const int lp = min(max(lstart[d] + pre + rank, 0), kTile - 1);
      tile[lp] = make_int2(key[r], val[r]);
    }
    __syncthreads();
    for (int dd = tid; dd < NB; dd += kThreads) {
      int tot = 0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) {
        tot += wcnt[w][dd];
        wcnt[w][dd] = 0;
      }
      run[dd] += tot;
    }
    __syncthreads();
  }
  for (int t = tid; t < ntile; t += kThreads) {
    const int2 kv = tile[t];
    const int d = (kv.x >> shift) & (NB - 1);
    const int pos = min(max(gbase[d] + (t - lstart[d]), 0), n - 1);
    kout[pos] = kv.x;
    vout[pos] = kv.y;
  }
}

__global__ __launch_bounds__(kThreads) void k_scan_tiles(int32_t* __restrict__ data, int len,
                                                          int32_t* __restrict__ partials,
                                                          const int32_t* gate) {
  __shared__ int lds[kThreads];
  if (gated_off(gate)) return;
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
  int v[kScanPer];
  int s = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    v[e] = (base + e < len) ? data[base + e] : 0;
    s += v[e];
  }
  int total;
  int run = block_exclusive_scan(s, lds, total);
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    if (base + e < len) data[base + e] = run;
    run += v[e];
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_partials(int32_t* __restrict__ partials,
                                                             int np, const int32_t* gate) {
  __shared__ int lds[kThreads];
  if (gated_off(gate)) return;
  int carry = 0;
  for (int base = 0; base < np; base += kThreads) {
    int i = base + threadIdx.x;
    int v = i < np ? partials[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, lds, total);
    if (i < np) partials[i] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kThreads) void k_scan_add(int32_t* __restrict__ data, int len,
                                                        const int32_t* __restrict__ partials,
                                                        const int32_t* gate) {
  if (gated_off(gate)) return;
  int add = partials[blockIdx.x];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e)
    if (base + e < len) data[base + e] += add;
}

// CSR starts of the sorted keys: start[c] = first slot whose key is >= c,
// for c = 0 .. C (start[C] = n). Slot k writes the starts of the keys
// between its predecessor's key and its own.
__device__ __forceinline__ void fill_starts(int prev, int cur, int k, int32_t* __restrict__ start) {
  for (int c = prev + 1; c <= cur; ++c) start[c] = k;
}

// Cell ids of the sorted slots (key >> 3 sub_bits) and the CSR tables of
// cells and, with sub_bits > 0, of sub-cells, in one pass over the keys.
__global__ __launch_bounds__(kThreads) void k_cell_tables(const int32_t* __restrict__ skeys,
                                                           int n, int sub_bits, int C,
                                                           int32_t* __restrict__ cell,
                                                           int32_t* __restrict__ cell_start,
                                                           int32_t* __restrict__ sub_start,
                                                           const int32_t* gate) {
  if (gated_off(gate)) return;
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k > n) return;
  const int sh = 3 * sub_bits;
  const int key = k < n ? skeys[k] : (C << sh);
  const int pkey = k > 0 ? skeys[k - 1] : -1;
  const int cur = key >> sh, prev = k > 0 ? (pkey >> sh) : -1;
  if (k < n && sub_bits) cell[k] = cur;
  fill_starts(prev, cur, k, cell_start);
  if (sub_bits) fill_starts(pkey, key, k, sub_start);
}

// Largest h of each cell over its sorted slots: one wave per cell, the
// lanes striding over the cell's slots (h read through perm), then a wave
// maximum; empty cells get 0.
__global__ __launch_bounds__(kThreads) void k_cell_hmax_sorted(const int32_t* __restrict__ start,
                                                                const int32_t* __restrict__ perm,
                                                                const float* __restrict__ hin,
                                                                int C, float* __restrict__ hmax,
                                                                const int32_t* gate) {
  if (gated_off(gate)) return;
  const int c = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (c >= C) return;                          // uniform over the wave
  const int lane = threadIdx.x & 63;
  float m = 0.0f;
  for (int k = start[c] + lane; k < start[c + 1]; k += 64) m = fmaxf(m, hin[perm[k]]);
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) hmax[c] = m;
}

// Last kernel of a gated binning: [1] = whether this call rebuilt the list,
// [0] = 0 (the list now matches the records).
__global__ void k_rebin_done(int32_t* gate) {
  if (threadIdx.x == 0) {
    gate[1] = gate[0] != 0 ? 1 : 0;
    gate[0] = 0;
  }
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct BinWs {
  int32_t *ka, *va, *kb, *vb, *hist, *partials;
  float* hin;   // h per input slot
};

BinWs carve(void* ws, int n, int nblk) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* p = static_cast<char*>(ws);
  BinWs w;
  size_t nb = al(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  w.ka = reinterpret_cast<int32_t*>(p); p += nb;
  w.va = reinterpret_cast<int32_t*>(p); p += nb;
  w.kb = reinterpret_cast<int32_t*>(p); p += nb;
  w.vb = reinterpret_cast<int32_t*>(p); p += nb;
  size_t hl = (size_t)kMaxBuckets * (size_t)(nblk > 0 ? nblk : 1);
  w.hist = reinterpret_cast<int32_t*>(p); p += al(sizeof(int32_t) * hl);
  w.hin = reinterpret_cast<float*>(p); p += nb;
  w.partials = reinterpret_cast<int32_t*>(p);
  return w;
}

hipError_t scan_local(int32_t* data, int len, int32_t* partials, hipStream_t s,
                      const int32_t* gate) {
  int nt = cdiv(len, kScanTile);
  if (nt == 0) return hipSuccess;
  k_scan_tiles<<<nt, kThreads, 0, s>>>(data, len, partials, gate);
  k_scan_partials<<<1, kThreads, 0, s>>>(partials, nt, gate);
  k_scan_add<<<nt, kThreads, 0, s>>>(data, len, partials, gate);
  return hipGetLastError();
}

}  // namespace

size_t scan_partials_count(int len) { return (size_t)cdiv(len, kScanTile) + 1; }

hipError_t scan_i32(int32_t* data, int len, int32_t* partials, hipStream_t s,
                    const int32_t* gate) {
  return scan_local(data, len, partials, s, gate);
}

size_t bin_workspace_bytes(int n, int n_c, int sub_bits) {
  (void)n_c;
  (void)sub_bits;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  int nblk = cdiv(n, kTile);
  size_t hl = (size_t)kMaxBuckets * (size_t)(nblk > 0 ? nblk : 1);
  return 5 * al(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)) + al(sizeof(int32_t) * hl) +
         al(sizeof(int32_t) * ((size_t)cdiv((int64_t)hl, kScanTile) + 1));
}

hipError_t launch_bin(const void* aos, const AosLayout& L, const CellsDev& c, int32_t* cell_start,
                      int32_t* perm, int32_t* cell, int32_t* sub_start, float* hmax, void* ws,
                      hipStream_t s) {
  const int n = c.n, n_c = c.n_c, sb = c.sub_bits;
  const int C = n_c * n_c * n_c;
  const int S = C << (3 * sb);
  const int nblk = cdiv(n, kTile);
  BinWs w = carve(ws, n, nblk);
  const int32_t* gate = c.rebin;         // kept when no particle moved (may be null)
  int32_t* skeys = cell;                 // sorted keys (cell ids when sb == 0)
  if (n > 0) {
    // span of the record bytes the keys need: x, and h when hmax is wanted
    const uint32_t ox = L.off[SPH_A_X], oh = L.off[SPH_A_H];
    const bool want_h = hmax && oh != kAbsent;
    const uint32_t hsz = L.dt[SPH_A_H] == DT_F64 ? 8u : 4u;
    const uint32_t lo = (want_h ? min(ox, oh) : ox) & ~7u;
    const uint32_t hi = (max(ox + 24u, want_h ? oh + hsz : 0u) + 7u) & ~7u;
    const int nw = (hi - lo) / 8 <= (uint32_t)kSpanWords ? (int)((hi - lo) / 8) : 0;
    k_bin_keys<<<cdiv(n, kThreads), kThreads, 0, s>>>(
        static_cast<const char*>(aos), L.stride, ox, oh, L.dt[SPH_A_H], lo, nw, n, n_c, sb, w.ka,
        w.va, want_h ? w.hin : nullptr, c.status, gate);
    int bits = 1;
    while ((1 << bits) < S) ++bits;
    // 9-bit digits where they need fewer passes than 8-bit ones (keys of
    // 9, 17-18, 25-27 bits), else 8-bit digits
    const int passes = (bits + 8) / 9 < (bits + 7) / 8 ? (bits + 8) / 9 : (bits + 7) / 8;
    const int D = passes * 8 >= bits ? 8 : 9;
    int32_t *ks = w.ka, *vs = w.va;
    for (int p = 0; p < passes; ++p) {
      int32_t *kd, *vd;
      if (p == passes - 1) {
        kd = sb ? ((ks == w.ka) ? w.kb : w.ka) : cell;
        vd = perm;
      } else {
        kd = (ks == w.ka) ? w.kb : w.ka;
        vd = (vs == w.va) ? w.vb : w.va;
      }
      if (D == 8) {
        k_radix_hist<8><<<nblk, kThreads, 0, s>>>(ks, w.hist, n, nblk, 8 * p, gate);
      } else {
        k_radix_hist<9><<<nblk, kThreads, 0, s>>>(ks, w.hist, n, nblk, 9 * p, gate);
      }
      hipError_t e = scan_local(w.hist, (1 << D) * nblk, w.partials, s, gate);
      if (e != hipSuccess) return e;
      if (D == 8) {
        k_radix_scatter<8><<<nblk, kThreads, 0, s>>>(ks, vs, kd, vd, w.hist, n, nblk, 8 * p, gate);
      } else {
        k_radix_scatter_direct<9><<<nblk, kThreads, 0, s>>>(ks, vs, kd, vd, w.hist, n, nblk, 9 * p,
                                                          gate);
      }
      ks = kd;
      vs = vd;
    }
    skeys = ks;
  }
  k_cell_tables<<<cdiv(n + 1, kThreads), kThreads, 0, s>>>(skeys, n, sb, C, cell, cell_start,
                                                           sub_start, gate);
  if (hmax) {
    if (n > 0 && L.off[SPH_A_H] != kAbsent) {
      k_cell_hmax_sorted<<<cdiv(C, kThreads / 64), kThreads, 0, s>>>(cell_start, perm, w.hin, C,
                                                                      hmax, gate);
    } else {
      k_fill_f32<<<cdiv(C, kThreads), kThreads, 0, s>>>(hmax, C, 0.0f, gate);
    }
  }
  if (c.rebin) k_rebin_done<<<1, 64, 0, s>>>(c.rebin);
  return hipGetLastError();
}

}  // namespace sph
