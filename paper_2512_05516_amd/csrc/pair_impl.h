// Quadratic kernels (implementation header, included by the pair_*.hip
// translation units): the density loop and the force loop over the cell list
// (Alg. 1 CallQuadratic; Eq. density, Eq. momentum, Eq. energy).
//
// One workgroup per (cell, chunk of TI particles): the chunk's particles i
// are held in registers, K lanes per particle (a chunk may also hold the
// particles of up to four sparse cells along x, with the cells around all of
// them as its neighbourhood). The workgroup walks the
// candidates j of the surrounding cells as one flattened index space and
// stages into LDS those whose distance to the chunk's bounding box is below
// the largest support radius (a conservative prune: every operation of the
// box distance is monotone in the same inputs as the pair test, so no
// accepted pair is ever dropped). The global loads of up to kRounds rounds
// are issued before the first one is used, so a chunk pays about one memory
// latency for its gather; the force-only fields of the staged candidates
// are then loaded cooperatively in one more batch.
//
// Each lane then runs two phases over its share of the staged candidates:
// (A) the FP32 support test (kUnroll LDS reads in flight, branch-free append
// of the candidate index to a per-lane list in LDS) and (B) the kernel sums
// over that list only, so the pair arithmetic runs on accepted pairs instead
// of on every candidate. The K partial sums of a particle are combined with
// a fixed shuffle tree: results are bit-identical run to run.
//
// The loaders (SoA views in compile-time or run-time storage formats, or
// AoS records) are the only difference between the SoA kernels and the
// plain-AoS kernels.
#pragma once
#include <cmath>

#include "sph_device.h"

namespace sph {
namespace pairk {

// --------------------------------------------------------------------------
// Data sources
// --------------------------------------------------------------------------
// Element k of a stored array: format DT fixed at compile time, or taken
// from rt when DT < 0.
template <int DT>
__device__ __forceinline__ float load_fmt(const void* p, int rt, int64_t k, float scale) {
  if constexpr (DT == DT_F32) {
    return static_cast<const float*>(p)[k] * scale;
  } else if constexpr (DT == DT_F16) {
    return f16_bits_to_f32(static_cast<const uint16_t*>(p)[k]) * scale;
  } else if constexpr (DT == DT_BF16) {
    return bf16_bits_to_f32(static_cast<const uint16_t*>(p)[k]) * scale;
  } else {
    return load_q(p, rt, k, scale);
  }
}

template <int PT, int VT, int MT>
struct SoaSrc {
  const void* off[3];
  const uint8_t* anc;     // anchor sub-cell codes (anchor >= SPH_ANCHOR_SUB(1))
  float anc_step;         // sub-cell side s 2^-b of the anchors
  int anchor;             // SPH_ANCHOR_CORNER or SPH_ANCHOR_SUB(b)
  const void* vq[3];
  const void* m;
  const void* h;
  const void* u;
  int pos_dt, vel_dt, mhu_dt;
  float lm, lh, lu;
  const float *rho, *f, *P, *c;
  float *o_rho, *o_wcount, *o_rho_dh, *o_f, *o_P, *o_c;
  int32_t* o_nngb;
  float *o_ax, *o_ay, *o_az, *o_du, *o_vsig;
  int32_t* o_nforce;

  // position relative to the cell corner: the stored offset plus its anchor
  __device__ __forceinline__ void pos(int k, int cell, int n_c, float& x, float& y,
                                      float& z) const {
    (void)cell;
    (void)n_c;
    x = load_fmt<PT>(off[0], pos_dt, k, 1.0f);
    y = load_fmt<PT>(off[1], pos_dt, k, 1.0f);
    z = load_fmt<PT>(off[2], pos_dt, k, 1.0f);
    if (anchor != SPH_ANCHOR_CORNER) {          // uniform over the launch
      const uint32_t c = anchor >= SPH_ANCHOR_SUB(1) ? (uint32_t)anc[k] : 0u;
      x = __builtin_fmaf((float)(c & 3u) + 0.5f, anc_step, x);
      y = __builtin_fmaf((float)((c >> 2) & 3u) + 0.5f, anc_step, y);
      z = __builtin_fmaf((float)((c >> 4) & 3u) + 0.5f, anc_step, z);
    }
  }
  __device__ __forceinline__ void vel(int k, float& x, float& y, float& z) const {
    x = load_fmt<VT>(vq[0], vel_dt, k, 1.0f);
    y = load_fmt<VT>(vq[1], vel_dt, k, 1.0f);
    z = load_fmt<VT>(vq[2], vel_dt, k, 1.0f);
  }
  __device__ __forceinline__ float mass(int k) const { return load_fmt<MT>(m, mhu_dt, k, lm); }
  __device__ __forceinline__ float hsml(int k) const { return load_fmt<MT>(h, mhu_dt, k, lh); }
  __device__ __forceinline__ float uint(int k) const { return load_fmt<MT>(u, mhu_dt, k, lu); }
  __device__ __forceinline__ void dens_in(int k, float& r, float& ff, float& p,
                                          float& cs) const {
    r = rho[k];
    ff = f[k];
    p = P[k];
    cs = c[k];
  }
  __device__ __forceinline__ void dens_out(int k, float r, float wc, float dh, float ff, float p,
                                           float cs, int nn) const {
    o_rho[k] = r;
    o_wcount[k] = wc;
    o_rho_dh[k] = dh;
    o_f[k] = ff;
    o_P[k] = p;
    o_c[k] = cs;
    o_nngb[k] = nn;
  }
  __device__ __forceinline__ void force_out(int k, float ax, float ay, float az, float du,
                                            float vs, int nf) const {
    o_ax[k] = ax;
    o_ay[k] = ay;
    o_az[k] = az;
    o_du[k] = du;
    o_vsig[k] = vs;
    if (o_nforce) o_nforce[k] = nf;
  }
};

struct AosSrc {
  char* base;
  AosLayout L;
  const int32_t* perm;

  __device__ __forceinline__ char* rec(int k) const {
    return base + (size_t)perm[k] * L.stride;
  }
  __device__ __forceinline__ void pos(int k, int cell, int n_c, float& x, float& y,
                                      float& z) const {
    const char* r = rec(k);
    int cx, cy, cz;
    cell_coords(cell, n_c, cx, cy, cz);
    const double* xp = reinterpret_cast<const double*>(r + L.off[SPH_A_X]);
    x = cell_offset(wrap01(xp[0]), cx, n_c);
    y = cell_offset(wrap01(xp[1]), cy, n_c);
    z = cell_offset(wrap01(xp[2]), cz, n_c);
  }
  __device__ __forceinline__ void vel(int k, float& x, float& y, float& z) const {
    const char* r = rec(k);
    x = rec_load32(r, L.off[SPH_A_V], L.dt[SPH_A_V], 0);
    y = rec_load32(r, L.off[SPH_A_V], L.dt[SPH_A_V], 1);
    z = rec_load32(r, L.off[SPH_A_V], L.dt[SPH_A_V], 2);
  }
  __device__ __forceinline__ float mass(int k) const {
    return rec_load32(rec(k), L.off[SPH_A_M], L.dt[SPH_A_M]);
  }
  __device__ __forceinline__ float hsml(int k) const {
    return rec_load32(rec(k), L.off[SPH_A_H], L.dt[SPH_A_H]);
  }
  __device__ __forceinline__ float uint(int k) const {
    return rec_load32(rec(k), L.off[SPH_A_U], L.dt[SPH_A_U]);
  }
  __device__ __forceinline__ void dens_in(int k, float& rr, float& ff, float& p,
                                          float& cs) const {
    const char* r = rec(k);
    rr = rec_load32(r, L.off[SPH_A_RHO], L.dt[SPH_A_RHO]);
    ff = rec_load32(r, L.off[SPH_A_F], L.dt[SPH_A_F]);
    p = rec_load32(r, L.off[SPH_A_P], L.dt[SPH_A_P]);
    cs = rec_load32(r, L.off[SPH_A_C], L.dt[SPH_A_C]);
  }
  __device__ __forceinline__ void dens_out(int k, float rr, float wc, float dh, float ff,
                                           float p, float cs, int nn) const {
    char* r = rec(k);
    rec_store32(r, L.off[SPH_A_RHO], L.dt[SPH_A_RHO], rr);
    rec_store32(r, L.off[SPH_A_WCOUNT], L.dt[SPH_A_WCOUNT], wc);
    rec_store32(r, L.off[SPH_A_RHO_DH], L.dt[SPH_A_RHO_DH], dh);
    rec_store32(r, L.off[SPH_A_F], L.dt[SPH_A_F], ff);
    rec_store32(r, L.off[SPH_A_P], L.dt[SPH_A_P], p);
    rec_store32(r, L.off[SPH_A_C], L.dt[SPH_A_C], cs);
    rec_store_i32(r, L.off[SPH_A_NNGB], nn);
  }
  __device__ __forceinline__ void force_out(int k, float ax, float ay, float az, float du,
                                            float vs, int nf) const {
    char* r = rec(k);
    rec_store32(r, L.off[SPH_A_A], L.dt[SPH_A_A], ax, 0);
    rec_store32(r, L.off[SPH_A_A], L.dt[SPH_A_A], ay, 1);
    rec_store32(r, L.off[SPH_A_A], L.dt[SPH_A_A], az, 2);
    rec_store32(r, L.off[SPH_A_DU], L.dt[SPH_A_DU], du);
    rec_store32(r, L.off[SPH_A_VSIG], L.dt[SPH_A_VSIG], vs);
    rec_store_i32(r, L.off[SPH_A_NFORCE], nf);
  }
};

// Slot indices read from the cell table are clamped to [0, n], so a
// corrupted table can never send a load outside the particle arrays.
__device__ __forceinline__ int clamp_slot(int v, int n) { return min(max(v, 0), n); }

// Spread consecutive workgroups over the 8 XCDs in contiguous ranges: block b
// runs on XCD b % 8, so logical work item (b % 8) * per + b / 8 gives each
// XCD a contiguous slab of cells (shared neighbour cells stay in one L2).
__device__ __forceinline__ int xcd_remap(int b, int G) {
  int per = G >> 3;
  if (b >= (per << 3)) return b;
  return (b & 7) * per + (b >> 3);
}

template <int K>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int o = K / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
template <int K>
__device__ __forceinline__ int group_sum_i(int v) {
#pragma unroll
  for (int o = K / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
template <int K>
__device__ __forceinline__ float group_max(float v) {
#pragma unroll
  for (int o = K / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// Position shift of the cell d cells away along an axis, relative to the
// chunk's cell: d * s in FP32 (-s, 0, s exactly), one expression wherever a
// position is shifted by d cells
__device__ __forceinline__ float cell_shift(int d, float s) { return (float)d * s; }

// Neighbour entry nb of a chunk of w - 2 cells along x (w = 3 for a single
// cell): offsets dx in [-1, w - 2], dy, dz in [-1, 1], nb = (dx + 1) +
// w ((dy + 1) + 3 (dz + 1)), and the periodic cell id.
__device__ __forceinline__ int neighbour_cell(int nb, int w, int cx, int cy, int cz, int n_c,
                                              int& dx, int& dy, int& dz) {
  dx = nb % w - 1;
  dy = (nb / w) % 3 - 1;
  dz = nb / (3 * w) - 1;
  int nx = cx + dx, ny = cy + dy, nz = cz + dz;
  nx += (nx < 0) ? n_c : ((nx >= n_c) ? -n_c : 0);
  ny += (ny < 0) ? n_c : ((ny >= n_c) ? -n_c : 0);
  nz += (nz < 0) ? n_c : ((nz >= n_c) ? -n_c : 0);
  return nx + n_c * (ny + n_c * nz);
}

__device__ __forceinline__ float box_dist2(float x, float y, float z, float lox, float loy,
                                           float loz, float hix, float hiy, float hiz) {
#pragma clang fp contract(off)
  float bx = fmaxf(fmaxf(lox - x, x - hix), 0.0f);
  float by = fmaxf(fmaxf(loy - y, y - hiy), 0.0f);
  float bz = fmaxf(fmaxf(loz - z, z - hiz), 0.0f);
  float xx = bx * bx;
  return __builtin_fmaf(bz, bz, __builtin_fmaf(by, by, xx));
}

// --------------------------------------------------------------------------
// Neighbour cells of a chunk's cells (m cells along x from the chunk's first
// cell, m = 1 unless the work list merges sparse cells): ids, the offsets
// (dx, dy, dz) of each from the chunk's first cell (its frame is shifted by
// cell_shift(delta, s) per axis), the support-radius bound of each (gamma_k * max h * (1 + 2^-8), covering
// storage rounding of h; the cell side when no bound table is given), and
// each cell's slot range. build_nbr issues all of its loads at once and
// ends without a barrier: the caller's next barrier (the chunk box's)
// publishes the table, so the chunk's own loads overlap these.
// --------------------------------------------------------------------------
constexpr int kMaxNbr = 9 * (kMaxMerge + 2);   // neighbour cells of a merged chunk
struct NbrCells {
  int cell[kMaxNbr];
  float hb[kMaxNbr];
  int st[kMaxNbr], cnt[kMaxNbr];   // first slot and particle count of each cell
  int d[kMaxNbr];   // offsets: (dx + 1) | (dy + 1) << 8 | (dz + 1) << 16
  float hbmax;      // largest hb over the nq cells
  int nq;           // neighbour cells: 9 (m + 2)
};

__device__ __forceinline__ void nbr_offsets(const NbrCells& T, int q, int& dx, int& dy, int& dz) {
  const int v = T.d[q];
  dx = (v & 0xff) - 1;
  dy = ((v >> 8) & 0xff) - 1;
  dz = (v >> 16) - 1;
}

__device__ __forceinline__ void build_nbr(NbrCells& T, const CellsDev& cd, int cx, int cy,
                                          int cz, int m, float s32, float gk) {
  const int tid = threadIdx.x;
  const int w = m + 2, nq = 9 * w;
  float hbv = 0.0f;
  if (tid == 0) T.nq = nq;
  if (tid < nq) {
    int dx, dy, dz;
    const int cn = neighbour_cell(tid, w, cx, cy, cz, cd.n_c, dx, dy, dz);
    T.d[tid] = (dx + 1) | ((dy + 1) << 8) | ((dz + 1) << 16);
    T.cell[tid] = cn;
    const int a = clamp_slot(cd.start[cn], cd.n);
    const int b = clamp_slot(cd.start[cn + 1], cd.n);
    hbv = cd.hmax ? gk * cd.hmax[cn] * (1.0f + 0x1p-8f) : s32;
    T.hb[tid] = hbv;
    T.st[tid] = a;
    T.cnt[tid] = max(b - a, 0);
  }
  if (tid < 64) {   // first wave (kMaxNbr <= 64): the largest bound
    float mx = hbv;
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (tid == 0) T.hbmax = mx;
  }
}
static_assert(kMaxNbr <= 64, "the neighbour table is reduced by one wave");

// Block-wide exclusive scan of an int in thread order: returns this
// thread's prefix and sets tb to the block total. One barrier: the caller
// must pass another barrier before `lds` (NT / 64 ints) is written again.
template <int NT>
__device__ __forceinline__ int block_scan(int b, int& tb, int* lds) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int ib = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int xb = __shfl_up(ib, o);
    if (lane >= o) ib += xb;
  }
  if (lane == 63) lds[wave] = ib;
  __syncthreads();
  int pb = 0;
  tb = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int wb = lds[w];
    pb += (w < wave) ? wb : 0;
    tb += wb;
  }
  return pb + ib - b;
}

// Block-wide exclusive scan, in thread order, of a flag (0/1) and of an
// int; returns the block totals. One barrier: the caller must pass another
// barrier before `lds` (2 NT / 64 ints) is written again.
template <int NT>
__device__ __forceinline__ void block_scan2(bool flag, int b, int& ea, int& eb, int& ta, int& tb,
                                            int* lds) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t bal = __ballot(flag);
  const int a = flag ? 1 : 0;
  int ia = __popcll(bal & lanemask_lt()) + a, ib = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int xb = __shfl_up(ib, o);
    if (lane >= o) ib += xb;
  }
  if (lane == 63) {
    lds[wave] = ia;
    lds[NW + wave] = ib;
  }
  __syncthreads();
  int pa = 0, pb = 0;
  ta = 0;
  tb = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int wa = lds[w], wb = lds[NW + w];
    pa += (w < wave) ? wa : 0;
    pb += (w < wave) ? wb : 0;
    ta += wa;
    tb += wb;
  }
  ea = pa + ia - a;
  eb = pb + ib - b;
}

// Position of each flagged thread when the flagged threads are ordered by
// class (0..3) and, within a class, by thread. One barrier: the caller must
// pass another barrier before `lds` (2 NT / 64 ints: a wave's four class
// counts, at most 64 each, as 16-bit halves) is written again.
template <int NT>
__device__ __forceinline__ int class_rank(bool flag, int cls, int* lds) {
  constexpr int NW = NT / 64;
  const int wave = threadIdx.x >> 6;
  uint64_t mine = 0;
  int cnt[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint64_t bal = __ballot(flag && cls == c);
    cnt[c] = __popcll(bal);
    mine = (cls == c) ? bal : mine;
  }
  if ((threadIdx.x & 63) == 0) {
    lds[wave] = cnt[0] | (cnt[1] << 16);
    lds[NW + wave] = cnt[2] | (cnt[3] << 16);
  }
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int a = lds[w], b = lds[NW + w];
    const int v[4] = {a & 0xffff, a >> 16, b & 0xffff, b >> 16};
#pragma unroll
    for (int c = 0; c < 4; ++c) off += (c < cls || (c == cls && w < wave)) ? v[c] : 0;
  }
  return off + __popcll(mine & lanemask_lt());
}

constexpr int kRounds = 4;      // gather rounds whose loads are issued together

// Range table of one batch of candidate ranges: slot ranges, prefix of
// counts and the neighbour index q of each; and, per neighbour cell q, its
// entries: the whole cell, or its sub-cells inside the query box. wbits
// marks the ranges that start inside the current gather window (kRounds
// rounds of NT flattened candidates); it is all zero between windows.
template <int NT>
struct RangeTab {
  static constexpr int kWinWords = kRounds * NT / 32;
  unsigned wbits[kWinWords];
  int start[NT];
  int pre[NT + 1];
  unsigned char q[NT];
  int scan[2 * (NT / 64)];
  int ntab, total;
  int qpre[kMaxNbr + 1];        // prefix of the entry counts of the cells
  unsigned char qw[kMaxNbr];    // 1: whole cell, 0: sub-cells qr
  unsigned char qny[kMaxNbr];   // sub-cell range width along y
  alignas(4) unsigned char qr[kMaxNbr][4];   // local sub-cell range: x0, y0, z0, width nx
};

// A neighbour cell is split into its R^3 sub-cells only when it holds more
// than kSplitFactor * R^3 particles: below that, one range for the whole
// cell costs less than the table work of its sub-cells.
constexpr int kSplitFactor = 2;

// The candidate ranges of a chunk: for each of the nq neighbour cells q
// with bound(q) > 0, the sub-cells (R = 2^sub_bits per axis) of q whose
// boxes lie within bound(q) of the chunk box [lo, hi], or the whole of q
// (a superset) when q is sparse. Entries are processed in
// batches of at most NT: for each batch, `batch(tab)` gathers the
// particles of the batch's ranges. The per-cell index ranges are widened by
// 2^-7 of a sub-cell (twice the 2^-8 margin of the per-entry box test, which
// covers the rounding of stored offsets), so every entry that test keeps is
// enumerated.
// When a batch's ranges hold more than `spread` candidates (more than one
// LDS batch of the caller), they are placed class by class. The class of a
// sub-cell at sub-cell coordinates (gx, gy, gz) from the chunk's cell is its
// parity pattern (gx, gy, gz) & 1 taken together with the complementary
// pattern, ((gx ^ gz) & 1) | ((gy ^ gz) & 1) << 1 (a whole cell: the same of
// its cell offsets). Each class is spread evenly over the neighbourhood, so
// when the staged candidates fill several LDS batches every batch holds a
// similar share of each particle's neighbours, and the per-lane lists of a
// batch are of similar length (in enumeration order a batch covers one side
// of the neighbourhood, and particles on that side hold most of its pairs).
template <int NT, class Bound, class Batch>
__device__ __forceinline__ void for_sub_cells(const CellsDev& cd, const NbrCells& T,
                                              RangeTab<NT>& tab, float s32, float lox, float loy,
                                              float loz, float hix, float hiy, float hiz,
                                              int spread, Bound bound, Batch batch) {
  const int sb = cd.sub_bits, R = 1 << sb;
  const float ss = s32 / (float)R;
  const float inv = (float)R / s32;
  const int* sstart = sb ? cd.sub_start : cd.start;
  const int tid = threadIdx.x;
  const int nq = T.nq;
  if (tid < 64) {   // first wave (nq <= 64): entry counts per cell, then their prefix
    int n = 0;
    if (tid < nq) {
      const int q = tid;
      int dx, dy, dz;
      nbr_offsets(T, q, dx, dy, dz);
      const float bq = bound(q);
      const int cnt = T.cnt[q];
      if (bq > 0.0f && cnt > 0) {
        auto lo_i = [&](float v, int d) {
          return max((int)floorf((v - bq) * inv - 0x1p-7f) - d * R, 0);
        };
        auto hi_i = [&](float v, int d) {
          return min((int)floorf((v + bq) * inv + 0x1p-7f) - d * R, R - 1);
        };
        const int x0 = lo_i(lox, dx), x1 = hi_i(hix, dx);
        const int y0 = lo_i(loy, dy), y1 = hi_i(hiy, dy);
        const int z0 = lo_i(loz, dz), z1 = hi_i(hiz, dz);
        if (x0 <= x1 && y0 <= y1 && z0 <= z1) {
          const bool whole = sb == 0 || cnt <= kSplitFactor * R * R * R;
          const int nx = x1 - x0 + 1;
          n = whole ? 1 : nx * (y1 - y0 + 1) * (z1 - z0 + 1);
          tab.qw[q] = whole ? 1 : 0;
          tab.qny[q] = (unsigned char)(y1 - y0 + 1);
          unsigned char* r = tab.qr[q];
          r[0] = (unsigned char)x0;
          r[1] = (unsigned char)y0;
          r[2] = (unsigned char)z0;
          r[3] = (unsigned char)nx;
        }
      }
    }
    int inc = n;   // inclusive wave scan
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int x = __shfl_up(inc, o);
      if (tid >= o) inc += x;
    }
    if (tid <= nq) tab.qpre[tid] = inc - n;   // lane nq holds the total
  }
  __syncthreads();
  const int NQ = tab.qpre[nq];
  for (int b0 = 0; b0 < NQ; b0 += NT) {
    const int t = b0 + tid;
    bool ok = t < NQ;
    int st = 0, cnt = 0, q = 0, cls = 0;
    if (ok) {
      int lo = 0, hi = nq - 1;   // last q with qpre[q] <= t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab.qpre[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
      q = lo;
      const int e = t - tab.qpre[q];
      int dx, dy, dz;
      nbr_offsets(T, q, dx, dy, dz);
      float bx0, bx1, by0, by1, bz0, bz1;
      if (tab.qw[q]) {
        const float mg = s32 * 0x1p-8f;       // rounding margin of stored offsets
        bx0 = dx * s32 - mg, bx1 = (dx + 1) * s32 + mg;
        by0 = dy * s32 - mg, by1 = (dy + 1) * s32 + mg;
        bz0 = dz * s32 - mg, bz1 = (dz + 1) * s32 + mg;
        st = T.st[q];
        cnt = T.cnt[q];
        cls = ((dx ^ dz) & 1) | (((dy ^ dz) & 1) << 1);
      } else {
        const uchar4 r = *reinterpret_cast<const uchar4*>(tab.qr[q]);
        // e = ex + nx (ey + ny ez), split through FP32 reciprocals (v_rcp,
        // 1 ulp): exact, as e < 2^9 and (e + 1/2) / w lies at least
        // 1 / (2 w) >= 2^-7 from an integer
        const int nx = r.w, nxy = nx * tab.qny[q];
        const int ez = (int)(((float)e + 0.5f) * __builtin_amdgcn_rcpf((float)nxy));
        const int rem = e - ez * nxy;
        const int ey = (int)(((float)rem + 0.5f) * __builtin_amdgcn_rcpf((float)nx));
        const int sx = r.x + (rem - ey * nx), sy = r.y + ey, sz = r.z + ez;
        const float mg = ss * 0x1p-8f;
        const int gx = dx * R + sx, gy = dy * R + sy, gz = dz * R + sz;
        cls = ((gx ^ gz) & 1) | (((gy ^ gz) & 1) << 1);
        bx0 = gx * ss - mg, bx1 = (gx + 1) * ss + mg;
        by0 = gy * ss - mg, by1 = (gy + 1) * ss + mg;
        bz0 = gz * ss - mg, bz1 = (gz + 1) * ss + mg;
        int m = 0;
        for (int b = 0; b < sb; ++b)
          m |= (((sx >> b) & 1) << (3 * b)) | (((sy >> b) & 1) << (3 * b + 1)) |
               (((sz >> b) & 1) << (3 * b + 2));
        const int key = (T.cell[q] << (3 * sb)) + m;
        st = clamp_slot(sstart[key], cd.n);
        cnt = max(clamp_slot(sstart[key + 1], cd.n) - st, 0);
      }
      const float ex = fmaxf(fmaxf(bx0 - hix, lox - bx1), 0.0f);
      const float ey = fmaxf(fmaxf(by0 - hiy, loy - by1), 0.0f);
      const float ez = fmaxf(fmaxf(bz0 - hiz, loz - bz1), 0.0f);
      const float bq = bound(q);
      ok = cnt > 0 && ex * ex + ey * ey + ez * ez < bq * bq * (1.0f + 0x1p-10f);
    }
    int e_idx, e_pre, ntab, total;
    block_scan2<NT>(ok, ok ? cnt : 0, e_idx, e_pre, ntab, total, tab.scan);
    if (total > spread) {   // uniform: more than one LDS batch, order by class
      __syncthreads();
      e_idx = class_rank<NT>(ok, cls, tab.scan);
      if (ok) tab.pre[e_idx] = cnt;
      __syncthreads();
      const int c_t = tid < ntab ? tab.pre[tid] : 0;
      e_pre = block_scan<NT>(c_t, total, tab.scan);
      if (tid < ntab) tab.pre[tid] = e_pre;
    } else if (ok) {
      tab.pre[e_idx] = e_pre;
    }
    if (ok) {
      tab.start[e_idx] = st;
      tab.q[e_idx] = (unsigned char)q;
    }
    if (tid == 0) {
      tab.pre[ntab] = total;
      tab.ntab = ntab;
      tab.total = total;
    }
    __syncthreads();
    batch(tab);
    __syncthreads();
  }
}

// Range lookup for a gather window [sbase, sbase + kRounds NT) of the
// flattened candidates: a bit per window position where a range starts
// (ranges are non-empty, so starts are distinct), a prefix of the bit counts
// per 32-bit word, and the number of ranges that start before the window.
// The range of candidate idx is then the number of starts at or before idx,
// minus one: one LDS read and a popcount instead of a search.
struct WinScan {
  int excl;    // lane w < kWinWords: set bits in the words before word w
  int total;   // set bits in the window
};

// Marks the starts inside the window (the bits are zero on entry); ends with
// a barrier, after which every wave may scan.
template <int NT>
__device__ __forceinline__ void mark_window(RangeTab<NT>& tab, int sbase) {
  const int t = threadIdx.x;
  if (t < tab.ntab) {
    const int p = tab.pre[t] - sbase;
    if (p >= 0 && p < kRounds * NT) atomicOr(&tab.wbits[p >> 5], 1u << (p & 31));
  }
  __syncthreads();
}

// Per-word prefix of the window's bit counts, in every wave (uniform
// control flow: all lanes active).
template <int NT>
__device__ __forceinline__ WinScan scan_window(const RangeTab<NT>& tab) {
  constexpr int NWD = RangeTab<NT>::kWinWords;
  static_assert(NWD <= 64, "one wave scans the window words");
  const int lane = threadIdx.x & 63;
  const int pc = lane < NWD ? __popc(tab.wbits[lane]) : 0;
  int inc = pc;
#pragma unroll
  for (int o = 1; o < NWD; o <<= 1) {
    const int x = __shfl_up(inc, o);
    if (lane >= o) inc += x;
  }
  return {inc - pc, __shfl(inc, NWD - 1)};
}

// Table entry holding flattened candidate idx (sbase <= idx < total, or
// clamped into that range by the caller); nbefore = ranges starting before
// sbase. Uniform control flow (the word prefix comes from another lane).
template <int NT>
__device__ __forceinline__ int window_entry(const RangeTab<NT>& tab, const WinScan& ws,
                                            int nbefore, int sbase, int idx) {
  const int x = idx - sbase;
  const int w = x >> 5;
  const unsigned m = tab.wbits[w] & ((2u << (x & 31)) - 1u);   // bits 0..x&31
  const int e = nbefore + __shfl(ws.excl, w) + __popc(m) - 1;
  return min(max(e, 0), tab.ntab - 1);   // a table entry whatever the bits hold
}

// Clears the window's bits once every thread has read them (callers do this
// after the first barrier that follows the lookups).
template <int NT>
__device__ __forceinline__ void clear_window(RangeTab<NT>& tab) {
  if ((int)threadIdx.x < RangeTab<NT>::kWinWords) tab.wbits[threadIdx.x] = 0u;
}

// Deterministic block-wide compaction with one barrier: wave totals are
// double-buffered by round parity, so a buffer is rewritten only after every
// thread has passed the next round's barrier.
// Returns this thread's slot within the round and adds the round's total to nj.
template <int NT>
__device__ __forceinline__ int compact_round(bool ok, int& nj, int* wtot2, int rnd) {
  constexpr int NW = NT / 64;
  int* wtot = wtot2 + (rnd & 1) * NW;
  const int wave = threadIdx.x >> 6;
  const uint64_t bal = __ballot(ok);
  const int wrank = __popcll(bal & lanemask_lt());
  if ((threadIdx.x & 63) == 0) wtot[wave] = __popcll(bal);
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int t = wtot[w];
    pre += (w < wave) ? t : 0;
    tot += t;
  }
  nj += tot;
  return pre + wrank;
}

// Per-lane neighbour lists: entry e of thread tid lives at lst[e * NT + tid]
// (phase B reads are conflict-free). A lane never holds more than LCAP
// entries: the test phase stops for the whole wave once any lane could
// overflow within the next kUnroll candidates.
constexpr int kUnroll = 8;
constexpr int kFillRounds = 4;  // force-only fields: rounds issued together
constexpr float kFlatRatio = 1.02f;   // force: neighbour support bound^2 / chunk's largest H^2

// Chunk bounding box of the valid particles and the largest H^2
struct ChunkBox {
  float lox, loy, loz, hix, hiy, hiz, h2max;
};

template <int NT>
__device__ __forceinline__ ChunkBox chunk_box(bool vi, float xi, float yi, float zi, float H2,
                                              float* red) {
  // the seven block maxima (minima as maxima of negated values) in one pass:
  // per value a wave shuffle tree, then the wave results in wave order; two
  // barriers
  constexpr int NW = NT / 64;
  const float inf = __builtin_inff();
  float v[7] = {vi ? -xi : -inf, vi ? -yi : -inf, vi ? -zi : -inf,
                vi ? xi : -inf,  vi ? yi : -inf,  vi ? zi : -inf, H2};
#pragma unroll
  for (int k = 0; k < 7; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] = fmaxf(v[k], __shfl_xor(v[k], o));
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 7; ++k) red[k * NW + wave] = v[k];
  }
  __syncthreads();
  float r[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    r[k] = red[k * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) r[k] = fmaxf(r[k], red[k * NW + w]);
  }
  __syncthreads();
  ChunkBox b;
  b.lox = -r[0];
  b.loy = -r[1];
  b.loz = -r[2];
  b.hix = r[3];
  b.hiy = r[4];
  b.hiz = r[5];
  b.h2max = r[6];
  return b;
}

// Phase A over the staged candidates [0, nj) (nj a multiple of K * kUnroll,
// padded with entries nobody accepts): lane kk of its particle tests
// candidates kk, kk + K, ... (`accept(q, index)`) and appends the accepted
// ones to its list; `consume(lo)` runs phase B over list entries [tid, lo)
// whenever the lists may fill up and at the end. The list position is kept
// as a byte offset, so appending costs a select and an add.
template <int NT, int K, int LCAP, class Accept, class Consume>
__device__ __forceinline__ void test_and_consume(const float4* cp, uint16_t* lst, int nj, int kk,
                                                 Accept accept, Consume consume) {
  const int tid = threadIdx.x;
  const int nit = nj / K;
  char* const lb = reinterpret_cast<char*>(lst);
  constexpr int kStep = 2 * NT;     // bytes between a lane's consecutive entries
  int it = 0;
  while (it < nit) {
    int lo = 2 * tid;
    const int lim = 2 * tid + (LCAP - kUnroll) * kStep;
    while (it < nit) {
      const float4* cq = cp + kk + K * it;
      float4 qv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) qv[u] = cq[K * u];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int idx = kk + K * (it + u);
        const bool acc = accept(qv[u], idx);
        *reinterpret_cast<uint16_t*>(lb + lo) = (uint16_t)idx;
        lo += acc ? kStep : 0;
      }
      it += kUnroll;
      if (__any(lo > lim)) break;
    }
    consume(lo >> 1);
  }
}

// Candidate prefilter of phase A. With p = x_i and q = x_j relative to the
// chunk's cell, r^2 = |p|^2 - 2 p.q + |q|^2: staging stores n2 = |q|^2 as
// q's fourth component, each lane keeps c = H^2 - |p|^2 + M and -2p, and
// the test is t = n2 - 2 p.q < c, three FMAs and a compare. Phase B takes
// the exact FP32 support test (dist2) again on the accepted pairs, so the
// prefilter only has to accept a superset of it; M bounds the rounding of
// t, of c and of dist2. With |p|^2 <= Bi, |q|^2 <= Bj and H^2 <= Bj those
// errors add up to less than 19 * 2^-24 * (Bi + Bj); M = 2^-16 (Bi + Bj)
// leaves a factor 13. Bi, Bj follow from the chunk box: the candidates
// lie within one cell side s of it (H <= s, else the status flag is set).
__device__ __forceinline__ float prefilter_margin(const ChunkBox& b, float s) {
  const float ex = fmaxf(fabsf(b.lox), fabsf(b.hix));
  const float ey = fmaxf(fabsf(b.loy), fabsf(b.hiy));
  const float ez = fmaxf(fabsf(b.loz), fabsf(b.hiz));
  const float bi = ex * ex + ey * ey + ez * ez;
  const float bj = (ex + s) * (ex + s) + (ey + s) * (ey + s) + (ez + s) * (ez + s);
  return 0x1p-16f * (bi + bj);
}

__device__ __forceinline__ float norm2(float x, float y, float z) {
  return __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
}

// t = n2 - 2 p.q for a staged candidate q = (x, y, z, n2); m2x = -2 p.x ...
__device__ __forceinline__ float prefilter_t(float m2x, float m2y, float m2z, const float4& q) {
  return __builtin_fmaf(m2z, q.z, __builtin_fmaf(m2y, q.y, __builtin_fmaf(m2x, q.x, q.w)));
}

// dist2 with p given as -2p: fma(-2p, -1/2, -q) is p - q rounded once, the
// same value as dist2's subtraction, so the lanes need not keep p itself.
__device__ __forceinline__ float dist2_m2(float m2x, float m2y, float m2z, float qx, float qy,
                                          float qz, float& dx, float& dy, float& dz) {
#pragma clang fp contract(off)
  dx = __builtin_fmaf(m2x, -0.5f, -qx);
  dy = __builtin_fmaf(m2y, -0.5f, -qy);
  dz = __builtin_fmaf(m2z, -0.5f, -qz);
  float xx = dx * dx;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, xx));
}

// Work distribution. No work list: one workgroup per cell, taking the
// cell's chunks of TI in turn. With a work list, items (cell, first slot)
// of XCD range x = blockIdx % 8 (workgroups are dispatched to the 8 XCDs in
// turn):
//   GRID / STATIC: workgroup l of its XCD takes items lo_x + l, + G/8, ...
//     (GRID launches about one workgroup per item, STATIC only as many as
//     stay resident);
//   DYNAMIC: resident workgroups take items from their XCD's queue with an
//     atomic counter and then steal from the other queues; the counter of
//     the next item is bumped while the current one is processed, so the
//     atomic's latency overlaps the work.
// A merged item (the work list's max_cells > 1) packs m - 1 into the bits
// of the cell id from kMergeShift up: its slots are those of the m cells
// cell, cell + 1, ... of one brick row, at most TI of them.
// The chunk callback takes (cell, m, c0, c1, only_q, out, obase): slots
// [c0, c1) of the m cells from `cell` along x, the neighbour cell index q
// (0..26) the j particles are restricted to (-1: all of them; only with
// m = 1), and the task result records (out == nullptr: the full loop's
// outputs) with slot i's record at out[obase + i].
// Position of slot i of a chunk over the m cells from `cell` along x,
// relative to `cell`: the stored offset in i's own cell, shifted by that
// cell's distance from `cell` with the same expression as the candidates'
// shifts, so that i meets its own candidate copy at r = 0 exactly.
template <class Src>
__device__ __forceinline__ void chunk_pos(const Src& src, const CellsDev& cd, int i, int cell,
                                          int m, float s32, float& x, float& y, float& z) {
  int d = 0;
  for (int k = 1; k < m; ++k) d += i >= clamp_slot(cd.start[cell + k], cd.n) ? 1 : 0;
  src.pos(i, cell + d, cd.n_c, x, y, z);
  x = shifted(x, cell_shift(d, s32));
}

struct LoopItems {
  WorkDev wk;

  template <class Chunk>
  __device__ __forceinline__ void run(const CellsDev& cd, int TI, Chunk chunk) const {
  if (!wk.items) {   // one workgroup per cell, cells in brick order
    const int cell = brick_cell(xcd_remap(blockIdx.x, gridDim.x), cd.n_c);
    const int cs = clamp_slot(cd.start[cell], cd.n);
    const int ce = max(clamp_slot(cd.start[cell + 1], cd.n), cs);
    for (int base = cs; base < ce; base += TI)
      chunk(cell, 1, base, min(base + TI, ce), -1, (sph_task_result*)nullptr, 0);
    return;
  }
  const int C = cd.n_c * cd.n_c * cd.n_c;
  auto item = [&](int it) {
    const int2 v = wk.items[it];
    int cell = v.x, m = 1;
    if (wk.merge > 1) {
      cell = v.x & ((1 << kMergeShift) - 1);
      m = (int)((unsigned)v.x >> kMergeShift) + 1;
    }
    cell = min(max(cell, 0), C - 1);
    if (m > 1) {   // stay within the row (the list builder guarantees it)
      int cx, cy, cz;
      cell_coords(cell, cd.n_c, cx, cy, cz);
      m = min(min(m, kMaxMerge), cd.n_c - cx);
    }
    const int ce = max(clamp_slot(cd.start[cell + m], cd.n), 0);
    const int base = clamp_slot(v.y, ce);
    chunk(cell, m, base, min(base + TI, ce), -1, (sph_task_result*)nullptr, 0);
  };
  const int x = blockIdx.x & (kQueues - 1);
  const int total = min(wk.meta[0], wk.capacity);
  if (wk.sched != SPH_SCHED_DYNAMIC) {
    const int nl = gridDim.x / kQueues;
    const int lo = max(wk.meta[1 + x], 0), hi = min(wk.meta[2 + x], total);
    for (int it = lo + (int)(blockIdx.x / kQueues); it < hi; it += nl) item(it);
    return;
  }
  __shared__ int s_item;
  int qi = 0;   // thread 0: queues tried so far (own queue first)
  auto grab = [&]() {
    while (qi < kQueues) {
      const int q = (x + qi) & (kQueues - 1);
      const int idx = atomicAdd(&wk.counters[q], 1);
      if (idx < min(wk.meta[2 + q], total)) return idx;
      ++qi;
    }
    return -1;
  };
  if (threadIdx.x == 0) s_item = grab();
  __syncthreads();
  int it = __builtin_amdgcn_readfirstlane(s_item);
  while (it >= 0) {
    int nxt = -1, nq = 0;
    if (threadIdx.x == 0 && qi < kQueues) {
      nq = (x + qi) & (kQueues - 1);
      nxt = atomicAdd(&wk.counters[nq], 1);
    }
    __syncthreads();   // every thread has read s_item
    item(it);
    if (threadIdx.x == 0) {
      if (qi >= kQueues) {
        nxt = -1;
      } else if (nxt >= min(wk.meta[2 + nq], total)) {
        ++qi;
        nxt = grab();
      }
      s_item = nxt;
    }
    __syncthreads();
    it = __builtin_amdgcn_readfirstlane(s_item);
  }
}
};

// Neighbour index q = (dx+1) + 3 (dy+1) + 9 (dz+1) of cell cj seen from
// cell ci (periodic), or -2 if cj is not one of the 27 cells around ci.
__device__ __forceinline__ int nbr_index(int ci, int cj, int n_c) {
  int ax, ay, az, bx, by, bz;
  cell_coords(ci, n_c, ax, ay, az);
  cell_coords(cj, n_c, bx, by, bz);
  auto wrap = [&](int d) { return d > 1 ? d - n_c : (d < -1 ? d + n_c : d); };
  const int dx = wrap(bx - ax), dy = wrap(by - ay), dz = wrap(bz - az);
  if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return -2;
  return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}

// Work items of a batch of cell-pair tasks: workgroup b takes item b =
// (task, first slot), i.e. up to TI slots of the task's i range against
// the task's neighbour cell only.
struct TaskItems {
  const sph_task* tasks;
  int ntasks;
  const int32_t* out_off;
  const int2* items;
  int nitems;
  sph_task_result* out;
  int n_out;

  template <class Chunk>
  __device__ __forceinline__ void run(const CellsDev& cd, int TI, Chunk chunk) const {
    const int b = blockIdx.x;
    if (b >= nitems) return;
    const int C = cd.n_c * cd.n_c * cd.n_c;
    const int2 it = items[b];
    const int ti_ = min(max(it.x, 0), ntasks - 1);
    const sph_task t = tasks[ti_];
    const int ci = min(max(t.ci, 0), C - 1), cj = min(max(t.cj, 0), C - 1);
    const int cs = clamp_slot(cd.start[ci], cd.n);
    const int ce = max(clamp_slot(cd.start[ci + 1], cd.n), cs);
    const int ib = min(max(t.i_begin, cs), ce), ie = min(max(t.i_end, ib), ce);
    const int c0 = min(max(it.y, ib), ie), c1 = min(c0 + TI, ie);
    const int o = min(max(out_off[ti_], 0), n_out);
    // records past n_out are dropped: clamp the range to what fits
    const int c1o = min(c1, c0 + max(n_out - (o + (c0 - ib)), 0));
    chunk(ci, 1, c0, c1o, nbr_index(ci, cj, cd.n_c), out, o - ib);
  }
};

// --------------------------------------------------------------------------
// Density
// --------------------------------------------------------------------------
// The second launch bound: the compiler reads it as waves per SIMD =
// blocks x ceil(waves per block / 4). Four waves per SIMD (at most 128
// VGPRs, a few spilled) for every density tile, three (168 VGPRs) for every
// force tile.
template <int NT>
constexpr int kDensityBlocks = 4;
template <int NT>
constexpr int kForceBlocks = 3;

template <int TI, int K, class Src, class Items, int KS>
__global__ __launch_bounds__(TI* K, kDensityBlocks<TI * K>) void k_density(Src src, CellsDev cd, Phys ph,
                                                                    float s32, Items items) {
  using Shape = KernelShape<KS>;
  constexpr int NT = TI * K;
  // staged candidates (LDS for four waves per SIMD); with one lane per
  // particle a batch of 2 NT: a chunk of one lattice cell then fills four
  // batches, one per range class, where three batches would cut a class
  constexpr int CAP = (K == 1 ? 2 : 3) * NT;
  constexpr int LCAP = 32;
  constexpr int kPad = K * kUnroll;
  __shared__ float4 cand[CAP];                 // x, y, z relative to this cell, |x|^2
  __shared__ float cmass[CAP];                 // m_j
  __shared__ uint16_t lst[LCAP * NT];
  __shared__ NbrCells T;
  __shared__ RangeTab<NT> tab;
  __shared__ int wtot[2 * (NT / 64)];
  __shared__ float red[7 * (NT / 64)];

  const int n_c = cd.n_c;
  const int tid = threadIdx.x;
  const int gi = tid / K, kk = tid % K;
  const float gk = ph.gamma_k;

  items.run(cd, TI, [&](int cell, int m, int c0, int c1, int only_q, sph_task_result* tout,
                        int tbase) {
    int cx, cy, cz;
    cell_coords(cell, n_c, cx, cy, cz);
    build_nbr(T, cd, cx, cy, cz, m, s32, gk);
    clear_window<NT>(tab);   // published by the chunk box's barriers
    const int i = c0 + gi;
    const bool vi = i < c1;
    float xi = 0.f, yi = 0.f, zi = 0.f, hi = 0.f, ui = 0.f;
    if (vi) {
      chunk_pos(src, cd, i, cell, m, s32, xi, yi, zi);
      hi = src.hsml(i);
      ui = src.uint(i);
    }
    const float H2 = vi ? support2(gk, hi) : 0.0f;
    const float Hinv = vi ? 1.0f / (gk * hi) : 0.0f;
    const ChunkBox bx = chunk_box<NT>(vi, xi, yi, zi, H2, red);
    if (vi && cd.status && H2 > s32 * s32) atomicOr(cd.status, SPH_FLAG_H_TOO_LARGE);
    const float bext = sqrtf(bx.h2max);
    const float m2x = -2.0f * xi, m2y = -2.0f * yi, m2z = -2.0f * zi;
    const float cpre = vi ? H2 - norm2(xi, yi, zi) + prefilter_margin(bx, s32)
                          : -__builtin_inff();

    float rho = 0.f, wsum = 0.f, dh = 0.f;
    int nn = 0;
    int staged = 0, gathered = 0;     // uniform: work counters of the chunk

    auto pair_phase = [&](int nj) {
      staged += nj;
      // pad [nj, roundup(nj, kPad)) with entries no particle accepts
      const int njp = (nj + kPad - 1) / kPad * kPad;
      if (tid < njp - nj) cand[nj + tid] = make_float4(0.f, 0.f, 0.f, 1e30f);
      __syncthreads();
      test_and_consume<NT, K, LCAP>(
          cand, lst, njp, kk,
          [&](const float4& q, int) { return prefilter_t(m2x, m2y, m2z, q) < cpre; },
          [&](int lo) {
            // list entry e + NT is read while entry e is processed
            int tn = tid < lo ? lst[tid] : 0;
            for (int e = tid; e < lo; e += NT) {
              const int t = tn;
              const float4 q = cand[t];
              const float mj = cmass[t];
              tn = lst[e + NT < lo ? e + NT : e];
              float dx, dy, dz;
              const float r2 = dist2_m2(m2x, m2y, m2z, q.x, q.y, q.z, dx, dy, dz);
              const bool in = r2 < H2;       // the exact support test
              const float u = fast_sqrt(r2) * Hinv;
              float w, dw;
              Shape::w_dw(u, w, dw);
              w = in ? w : 0.0f;
              dw = in ? dw : 0.0f;
              rho = fmaf(mj, w, rho);
              wsum += w;
              dh = fmaf(mj, fmaf(u, dw, 3.0f * w), dh);
              nn += in ? 1 : 0;
            }
          });
      __syncthreads();
    };

    int nj = 0, rnd = 0;
    for_sub_cells<NT>(
        cd, T, tab, s32, bx.lox, bx.loy, bx.loz, bx.hix, bx.hiy, bx.hiz, CAP - kPad,
        [&](int q) { return (only_q == -1 || q == only_q) ? bext : 0.0f; },
        [&](RangeTab<NT>& tb) {
          const int total = tb.total;
          gathered += total;
          int nbefore = 0;
          for (int sbase = 0; sbase < total; sbase += kRounds * NT) {
            mark_window<NT>(tb, sbase);
            const WinScan ws = scan_window<NT>(tb);
            float4 c[kRounds];
            int qq[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
              const int idx = sbase + r * NT + tid;
              const int e = window_entry<NT>(tb, ws, nbefore, sbase, min(idx, total - 1));
              c[r] = make_float4(0.f, 0.f, 0.f, 0.f);
              qq[r] = 0;
              if (idx < total) {
                qq[r] = tb.q[e];
                const int j = min(max(tb.start[e] + (idx - tb.pre[e]), 0), cd.n - 1);
                src.pos(j, T.cell[qq[r]], n_c, c[r].x, c[r].y, c[r].z);
                c[r].w = src.mass(j);
              }
            }
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
              if (sbase + r * NT >= total) break;       // uniform
              const int idx = sbase + r * NT + tid;
              bool ok = idx < total;
              if (ok) {
                int ox, oy, oz;
                nbr_offsets(T, qq[r], ox, oy, oz);
                c[r].x = shifted(c[r].x, cell_shift(ox, s32));
                c[r].y = shifted(c[r].y, cell_shift(oy, s32));
                c[r].z = shifted(c[r].z, cell_shift(oz, s32));
                ok = box_dist2(c[r].x, c[r].y, c[r].z, bx.lox, bx.loy, bx.loz, bx.hix, bx.hiy,
                               bx.hiz) < bx.h2max;
              }
              int njn = nj;
              const int slot = compact_round<NT>(ok, njn, wtot, rnd++);
              if (r == 0) clear_window<NT>(tb);       // every lookup is done
              if (njn > CAP - kPad) {                 // uniform: consume the staged ones first
                pair_phase(nj);
                njn -= nj;
                nj = 0;
              }
              if (ok) {
                cand[nj + slot] = make_float4(c[r].x, c[r].y, c[r].z, norm2(c[r].x, c[r].y, c[r].z));
                cmass[nj + slot] = c[r].w;
              }
              nj = njn;
            }
            nbefore += ws.total;
          }
        });
    pair_phase(nj);

    if (cd.tally && tid == 0) {
      atomicAdd(cd.tally, (unsigned long long)(c1 - c0) * (unsigned long long)staged);
      atomicAdd(cd.tally + 1, (unsigned long long)gathered);
    }
    rho = group_sum<K>(rho);
    wsum = group_sum<K>(wsum);
    dh = group_sum<K>(dh);
    nn = group_sum_i<K>(nn);
    if (vi && kk == 0 && tout) {
      const float Hinv3 = Hinv * Hinv * Hinv;
      float4* r = reinterpret_cast<float4*>(tout + (tbase + i));
      r[0] = make_float4(rho * Hinv3, kFourPiThird * wsum, -gk * dh * Hinv3 * Hinv, 0.0f);
      r[1] = make_float4(0.0f, __int_as_float(nn), 0.0f, 0.0f);
    } else if (vi && kk == 0) {
      const float Hinv3 = Hinv * Hinv * Hinv;
      const float rho_i = rho * Hinv3;
      const float rho_dh = -gk * dh * Hinv3 * Hinv;
      const float omega = 1.0f + hi * rho_dh / (3.0f * rho_i);
      const float f = ph.gradh ? 1.0f / omega : 1.0f;
      const float P = (ph.gamma - 1.0f) * rho_i * ui;
      const float c = sqrtf(ph.gamma * (ph.gamma - 1.0f) * ui);
      src.dens_out(i, rho_i, kFourPiThird * wsum, rho_dh, f, P, c, nn);
    }
    __syncthreads();
  });
}

// --------------------------------------------------------------------------
// Force
// --------------------------------------------------------------------------
template <int TI, int K, class Src, class Items, int KS>
__global__ __launch_bounds__(TI* K, kForceBlocks<TI * K>) void k_force(Src src, CellsDev cd, Phys ph,
                                                                 float s32, Items items) {
  using Shape = KernelShape<KS>;
  constexpr int NT = TI * K;
  constexpr int CAP = 2 * NT;
  // one lane per particle: the lists of a batch of 2 NT stay short, and 24
  // entries keep the block's LDS within 1/12 of the CU's (three waves per SIMD)
  constexpr int LCAP = K == 1 ? 24 : 32;
  constexpr int kPad = K * kUnroll;
  __shared__ float4 cp[CAP];      // x, y, z (relative to this cell), |x|^2
  __shared__ float ch2[CAP];      // H_j^2
  __shared__ float4 cv[CAP];      // v_j, m_j
  __shared__ float4 cs4[CAP];     // 1/H_j, A_j, c_j, rho_j
  __shared__ int cid[CAP];        // sorted slot of j
  __shared__ int selfpos[TI];     // batch << 16 | staged index of particle c0 + k, or -1
  __shared__ uint16_t lst[LCAP * NT];
  __shared__ NbrCells T;
  __shared__ RangeTab<NT> tab;
  __shared__ int wtot[2 * (NT / 64)];
  __shared__ float red[7 * (NT / 64)];

  const int n_c = cd.n_c;
  const int tid = threadIdx.x;
  const int gi = tid / K, kk = tid % K;
  const float gk = ph.gamma_k;
  const float alpha = ph.alpha, beta = ph.beta;

  items.run(cd, TI, [&](int cell, int m, int c0, int c1, int only_q, sph_task_result* tout,
                        int tbase) {
    int cx, cy, cz;
    cell_coords(cell, n_c, cx, cy, cz);
    build_nbr(T, cd, cx, cy, cz, m, s32, gk);
    clear_window<NT>(tab);   // published by the chunk box's barriers
    if (tid < TI) selfpos[tid] = -1;
    const int i = c0 + gi;
    const bool vi = i < c1;
    // lanes without a particle sit far outside the box and accept nothing
    float xi = 1e30f, yi = 1e30f, zi = 1e30f, hi = 1.f, vxi = 0.f, vyi = 0.f, vzi = 0.f;
    float rhoi = 1.f, fi = 1.f, Pi_ = 0.f, ci = 0.f;
    if (vi) {
      chunk_pos(src, cd, i, cell, m, s32, xi, yi, zi);
      src.vel(i, vxi, vyi, vzi);
      hi = src.hsml(i);
      src.dens_in(i, rhoi, fi, Pi_, ci);
    }
    const float H2i = vi ? support2(gk, hi) : 0.0f;
    const float Hinvi = 1.0f / (gk * hi);
    const float Hinv2i = Hinvi * Hinvi;
    const float Hinv4i = Hinv2i * Hinv2i;
    const float Ai = (ph.gradh ? fi : 1.0f) * Pi_ / (rhoi * rhoi);
    const ChunkBox bx = chunk_box<NT>(vi, xi, yi, zi, H2i, red);
    if (vi && cd.status && H2i > s32 * s32) atomicOr(cd.status, SPH_FLAG_H_TOO_LARGE);
    const float bi = sqrtf(bx.h2max);
    // prefilter constants: r^2 < max(H_i^2, H_j^2) becomes
    // t < max(H_i^2 - |p|^2 + M, H_j^2 - (|p|^2 - M))
    const float m2x = -2.0f * xi, m2y = -2.0f * yi, m2z = -2.0f * zi;
    const float mrg = prefilter_margin(bx, s32);
    const float pp = norm2(xi, yi, zi);
    const float cpre = vi ? H2i - pp + mrg : -__builtin_inff();
    const float ppm = vi ? pp - mrg : __builtin_inff();
    // Where no neighbour cell's support bound exceeds the chunk's largest
    // support by much, one threshold per lane replaces the per-candidate
    // max: t < max(H_i^2, Hn^2) - |p|^2 + M, with Hn bounding every H_j of
    // the 27 cells, accepts a superset of the pairs at a few extra entries,
    // and the consume phase applies the exact test to each of them.
    const float hn = only_q == -1 ? T.hbmax : T.hb[only_q];
    const float hn2 = hn * hn;
    const bool flat = hn2 <= kFlatRatio * bx.h2max;   // uniform over the block
    const float cflat = vi ? fmaxf(H2i, hn2) - pp + mrg : -__builtin_inff();

    float ax = 0.f, ay = 0.f, az = 0.f, du = 0.f, vsig = 0.f;
    int nf = 0;
    int staged = 0, gathered = 0;     // uniform: work counters of the chunk

    // force-only fields of staged candidates [from, to), loaded cooperatively
    auto fill = [&](int from, int to) {
      __syncthreads();
      for (int s0 = from; s0 < to; s0 += kFillRounds * NT) {
        float4 v4[kFillRounds], d4[kFillRounds];
        float hj[kFillRounds];
#pragma unroll
        for (int r = 0; r < kFillRounds; ++r) {
          const int sl = s0 + r * NT + tid;
          v4[r] = make_float4(0.f, 0.f, 0.f, 0.f);
          d4[r] = make_float4(1.f, 1.f, 0.f, 0.f);
          hj[r] = 1.f;
          if (sl < to) {
            const int j = cid[sl];
            src.vel(j, v4[r].x, v4[r].y, v4[r].z);
            v4[r].w = src.mass(j);
            hj[r] = src.hsml(j);
            src.dens_in(j, d4[r].x, d4[r].y, d4[r].z, d4[r].w);
          }
        }
#pragma unroll
        for (int r = 0; r < kFillRounds; ++r) {
          const int sl = s0 + r * NT + tid;
          if (sl < to) {
            cv[sl] = v4[r];
            // d4 = (rho, f, P, c) -> (1/H, A, c, rho)
            cs4[sl] = make_float4(1.0f / (gk * hj[r]),
                                  (ph.gradh ? d4[r].y : 1.0f) * d4[r].z / (d4[r].x * d4[r].x),
                                  d4[r].w, d4[r].x);
          }
        }
      }
    };

    int nbatch = 0;   // uniform: LDS batches consumed so far in this chunk
    auto pair_phase = [&](int nj) {
      staged += nj;
      const int njp = (nj + kPad - 1) / kPad * kPad;
      if (tid < njp - nj) {
        cp[nj + tid] = make_float4(0.f, 0.f, 0.f, 1e30f);
        ch2[nj + tid] = 0.f;
        cid[nj + tid] = -1;
      }
      __syncthreads();
      // i's own copy in this batch, or -1
      const int sp = selfpos[gi];
      const int tself = (sp >> 16) == nbatch ? (sp & 0xffff) : -1;
      // list entry e + NT is read while entry e is processed, and all fields
      // of an entry are read at once (one LDS round trip per entry)
      auto consume = [&](int lo) {
            int tn = tid < lo ? lst[tid] : 0;
            for (int e = tid; e < lo; e += NT) {
              const int t = tn;
              const float4 q0 = cp[t];
              const float h2j = ch2[t];
              const float4 q1 = cv[t];
              const float4 q2 = cs4[t];
              tn = lst[e + NT < lo ? e + NT : e];
              float dx, dy, dz;
              const float r2 = dist2_m2(m2x, m2y, m2z, q0.x, q0.y, q0.z, dx, dy, dz);
              // the exact support test, r2 < max(H_i^2, H_j^2), and not the
              // self pair; coincident stored positions (r2 = 0, j != i) stay:
              // w'(0) = 0 makes their terms vanish
              // (the empty asm keeps the force-only loads ahead of the branch,
              // where they overlap the position load)
              asm volatile("" ::"v"(q1.x), "v"(q1.y), "v"(q1.z), "v"(q1.w), "v"(q2.x),
                           "v"(q2.y), "v"(q2.z), "v"(q2.w));
              if (!((r2 < H2i) | (r2 < h2j)) | (t == tself)) continue;
              const float r = fast_sqrt(r2);
              const float rinv = r2 > 0.0f ? fast_rcp(r) : 0.0f;
              const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
              const float gi_ = Shape::dw(r * Hinvi) * Hinv4i;
              const float hj2 = q2.x * q2.x;
              const float gj_ = Shape::dw(r * q2.x) * (hj2 * hj2);
              const float w = (vxi - q1.x) * ex + (vyi - q1.y) * ey + (vzi - q1.z) * ez;
              const float mu = fminf(w, 0.0f);
              const float vs = ci + q2.z - beta * mu;
              const float visc = -alpha * vs * mu * fast_rcp(rhoi + q2.w);
              const float gbar = 0.5f * (gi_ + gj_);
              const float kc = q1.w * (Ai * gi_ + q2.y * gj_ + visc * gbar);
              ax = fmaf(-kc, ex, ax);
              ay = fmaf(-kc, ey, ay);
              az = fmaf(-kc, ez, az);
              du = fmaf(q1.w * (Ai * gi_ + 0.5f * visc * gbar), w, du);
              // vs >= 0: the larger float is the larger int
              vsig = __int_as_float(max(__float_as_int(vsig), __float_as_int(vs)));
              ++nf;
            }
          };
      if (flat)
        test_and_consume<NT, K, LCAP>(
            cp, lst, njp, kk,
            [&](const float4& q0, int) { return prefilter_t(m2x, m2y, m2z, q0) < cflat; },
            consume);
      else
        test_and_consume<NT, K, LCAP>(
            cp, lst, njp, kk,
            [&](const float4& q0, int idx) {
              return prefilter_t(m2x, m2y, m2z, q0) < fmaxf(cpre, ch2[idx] - ppm);
            },
            consume);
      __syncthreads();
      ++nbatch;
    };

    int nj = 0, filled = 0, rnd = 0;
    for_sub_cells<NT>(
        cd, T, tab, s32, bx.lox, bx.loy, bx.loz, bx.hix, bx.hiy, bx.hiz, CAP - kPad,
        [&](int q) { return (only_q == -1 || q == only_q) ? fmaxf(bi, T.hb[q]) : 0.0f; },
        [&](RangeTab<NT>& tb) {
          const int total = tb.total;
          gathered += total;
          int nbefore = 0;
          for (int sbase = 0; sbase < total; sbase += kRounds * NT) {
            mark_window<NT>(tb, sbase);
            const WinScan ws = scan_window<NT>(tb);
            float4 c[kRounds];
            int qq[kRounds], jj[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
              const int idx = sbase + r * NT + tid;
              const int e = window_entry<NT>(tb, ws, nbefore, sbase, min(idx, total - 1));
              c[r] = make_float4(0.f, 0.f, 0.f, 1.f);   // w: h_j, then H_j^2
              qq[r] = 0;
              jj[r] = 0;
              if (idx < total) {
                qq[r] = tb.q[e];
                jj[r] = min(max(tb.start[e] + (idx - tb.pre[e]), 0), cd.n - 1);
                src.pos(jj[r], T.cell[qq[r]], n_c, c[r].x, c[r].y, c[r].z);
                c[r].w = src.hsml(jj[r]);
              }
            }
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
              if (sbase + r * NT >= total) break;       // uniform
              const int idx = sbase + r * NT + tid;
              bool ok = idx < total;
              if (ok) {
                int ox, oy, oz;
                nbr_offsets(T, qq[r], ox, oy, oz);
                c[r].x = shifted(c[r].x, cell_shift(ox, s32));
                c[r].y = shifted(c[r].y, cell_shift(oy, s32));
                c[r].z = shifted(c[r].z, cell_shift(oz, s32));
                c[r].w = support2(gk, c[r].w);
                ok = box_dist2(c[r].x, c[r].y, c[r].z, bx.lox, bx.loy, bx.loz, bx.hix, bx.hiy,
                               bx.hiz) < fmaxf(bx.h2max, c[r].w);
              }
              int njn = nj;
              const int slot = compact_round<NT>(ok, njn, wtot, rnd++);
              if (r == 0) clear_window<NT>(tb);       // every lookup is done
              if (njn > CAP - kPad) {                 // uniform: consume the staged ones first
                fill(filled, nj);
                pair_phase(nj);
                njn -= nj;
                nj = 0;
                filled = 0;
              }
              if (ok) {
                cp[nj + slot] = make_float4(c[r].x, c[r].y, c[r].z, norm2(c[r].x, c[r].y, c[r].z));
                ch2[nj + slot] = c[r].w;
                cid[nj + slot] = jj[r];
                if (jj[r] >= c0 && jj[r] < c1) selfpos[jj[r] - c0] = (nbatch << 16) | (nj + slot);
              }
              nj = njn;
            }
            // force-only fields of this super-round's candidates, one batch
            fill(filled, nj);
            filled = nj;
            nbefore += ws.total;
          }
        });
    pair_phase(nj);

    if (cd.tally && tid == 0) {
      atomicAdd(cd.tally, (unsigned long long)(c1 - c0) * (unsigned long long)staged);
      atomicAdd(cd.tally + 1, (unsigned long long)gathered);
    }
    ax = group_sum<K>(ax);
    ay = group_sum<K>(ay);
    az = group_sum<K>(az);
    du = group_sum<K>(du);
    vsig = group_max<K>(vsig);
    nf = group_sum_i<K>(nf);
    if (vi && kk == 0 && tout) {
      float4* r = reinterpret_cast<float4*>(tout + (tbase + i));
      r[0] = make_float4(ax, ay, az, du);
      r[1] = make_float4(vsig, __int_as_float(nf), 0.0f, 0.0f);
    } else if (vi && kk == 0) {
      src.force_out(i, ax, ay, az, du, vsig, nf);
    }
    __syncthreads();
  });
}

template <int PT, int VT, int MT>
SoaSrc<PT, VT, MT> make_soa(const sph_soa& s, const Prec& p, int n_c) {
  SoaSrc<PT, VT, MT> r;
  for (int k = 0; k < 3; ++k) {
    r.off[k] = s.f[SPH_S_OFF_X + k];
    r.vq[k] = s.f[SPH_S_VQ_X + k];
  }
  r.anchor = p.anchor;
  r.anc = static_cast<const uint8_t*>(s.f[SPH_S_ANC]);
  // s 2^-b, exact: the kernels' cell side scaled by a power of two
  r.anc_step = p.anchor == SPH_ANCHOR_CORNER
                   ? 0.0f
                   : std::ldexp((float)(1.0 / (double)n_c), -(p.anchor - SPH_ANCHOR_SUB(0)));
  r.m = s.f[SPH_S_M];
  r.h = s.f[SPH_S_H];
  r.u = s.f[SPH_S_U];
  r.pos_dt = p.pos;
  r.vel_dt = p.vel;
  r.mhu_dt = p.mhu;
  r.lm = p.load_m;
  r.lh = p.load_h;
  r.lu = p.load_u;
  r.rho = static_cast<const float*>(s.f[SPH_S_RHO]);
  r.f = static_cast<const float*>(s.f[SPH_S_F]);
  r.P = static_cast<const float*>(s.f[SPH_S_P]);
  r.c = static_cast<const float*>(s.f[SPH_S_C]);
  r.o_rho = static_cast<float*>(s.f[SPH_S_RHO]);
  r.o_wcount = static_cast<float*>(s.f[SPH_S_WCOUNT]);
  r.o_rho_dh = static_cast<float*>(s.f[SPH_S_RHO_DH]);
  r.o_f = static_cast<float*>(s.f[SPH_S_F]);
  r.o_P = static_cast<float*>(s.f[SPH_S_P]);
  r.o_c = static_cast<float*>(s.f[SPH_S_C]);
  r.o_nngb = static_cast<int32_t*>(s.f[SPH_S_NNGB]);
  r.o_ax = static_cast<float*>(s.f[SPH_S_A_X]);
  r.o_ay = static_cast<float*>(s.f[SPH_S_A_Y]);
  r.o_az = static_cast<float*>(s.f[SPH_S_A_Z]);
  r.o_du = static_cast<float*>(s.f[SPH_S_DU]);
  r.o_vsig = static_cast<float*>(s.f[SPH_S_VSIG]);
  r.o_nforce = static_cast<int32_t*>(s.f[SPH_S_NFORCE]);
  return r;
}

// Resident workgroups (per CU times CUs), a multiple of the 8 XCDs
static int persistent_grid(const void* kernel, int block) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess ||
      per < 1)
    per = 1;
  return max(cus * per / kQueues, 1) * kQueues;
}

// Grid of a pair launch: cells, about one workgroup per item (rounded up to
// the 8 XCDs), or the resident workgroups.
static int pair_grid(const void* kernel, int block, int C, const WorkDev* w) {
  if (!w) return C;
  if (w->sched == SPH_SCHED_GRID) return (w->capacity + kQueues - 1) / kQueues * kQueues;
  return persistent_grid(kernel, block);
}

static __global__ void k_reset_queues(WorkDev w) {
  if (threadIdx.x < kQueues) w.counters[threadIdx.x] = w.meta[1 + threadIdx.x];
}

template <class S>
hipError_t run_density(const S& src, const CellsDev& c, const Phys& ph, int ti, int k,
                       const WorkDev* w, hipStream_t s) {
  WorkDev wv{};
  if (w) wv = *w;
  const int C = c.n_c * c.n_c * c.n_c;
  const float s32 = (float)(1.0 / (double)c.n_c);
  if (w && w->sched == SPH_SCHED_DYNAMIC) k_reset_queues<<<1, 64, 0, s>>>(*w);
#define SPH_DENS_CASE(TI_, K_)                                                        \
  if (ti == TI_ && k == K_) {                                                         \
    auto kern = ph.kernel == SPH_KERNEL_WENDLAND_C2                                   \
                    ? k_density<TI_, K_, S, LoopItems, SPH_KERNEL_WENDLAND_C2>        \
                    : k_density<TI_, K_, S, LoopItems, SPH_KERNEL_M4>;                \
    const int G = pair_grid((const void*)kern, TI_ * K_, C, w);                       \
    kern<<<G, TI_ * K_, 0, s>>>(src, c, ph, s32, LoopItems{wv});                      \
    return hipGetLastError();                                                         \
  }
  SPH_DENS_CASE(64, 4)
  SPH_DENS_CASE(32, 8)
  SPH_DENS_CASE(128, 2)
  SPH_DENS_CASE(64, 2)
  SPH_DENS_CASE(64, 1)
  SPH_DENS_CASE(16, 16)
  SPH_DENS_CASE(16, 4)
  SPH_DENS_CASE(32, 2)
#undef SPH_DENS_CASE
  return hipErrorInvalidValue;
}

template <class S>
hipError_t run_force(const S& src, const CellsDev& c, const Phys& ph, int ti, int k,
                       const WorkDev* w, hipStream_t s) {
  WorkDev wv{};
  if (w) wv = *w;
  const int C = c.n_c * c.n_c * c.n_c;
  const float s32 = (float)(1.0 / (double)c.n_c);
  if (w && w->sched == SPH_SCHED_DYNAMIC) k_reset_queues<<<1, 64, 0, s>>>(*w);
#define SPH_FORCE_CASE(TI_, K_)                                                       \
  if (ti == TI_ && k == K_) {                                                         \
    auto kern = ph.kernel == SPH_KERNEL_WENDLAND_C2                                   \
                    ? k_force<TI_, K_, S, LoopItems, SPH_KERNEL_WENDLAND_C2>          \
                    : k_force<TI_, K_, S, LoopItems, SPH_KERNEL_M4>;                  \
    const int G = pair_grid((const void*)kern, TI_ * K_, C, w);                       \
    kern<<<G, TI_ * K_, 0, s>>>(src, c, ph, s32, LoopItems{wv});                      \
    return hipGetLastError();                                                         \
  }
  SPH_FORCE_CASE(64, 4)
  SPH_FORCE_CASE(32, 8)
  SPH_FORCE_CASE(128, 2)
  SPH_FORCE_CASE(64, 2)
  SPH_FORCE_CASE(64, 1)
  SPH_FORCE_CASE(16, 16)
  SPH_FORCE_CASE(16, 4)
  SPH_FORCE_CASE(32, 2)
#undef SPH_FORCE_CASE
  return hipErrorInvalidValue;
}

// Task batches: one workgroup per item, density and force kernels
template <class S>
hipError_t run_tasks(const S& src, const CellsDev& c, const Phys& ph, int ti, int k,
                     const TaskItems& dens, const TaskItems& force, hipStream_t s) {
  const float s32 = (float)(1.0 / (double)c.n_c);
#define SPH_TASK_CASE(TI_, K_)                                                         \
  if (ti == TI_ && k == K_) {                                                          \
    const bool wc2 = ph.kernel == SPH_KERNEL_WENDLAND_C2;                                \
    auto kd = wc2 ? k_density<TI_, K_, S, TaskItems, SPH_KERNEL_WENDLAND_C2>             \
                  : k_density<TI_, K_, S, TaskItems, SPH_KERNEL_M4>;                     \
    auto kf = wc2 ? k_force<TI_, K_, S, TaskItems, SPH_KERNEL_WENDLAND_C2>               \
                  : k_force<TI_, K_, S, TaskItems, SPH_KERNEL_M4>;                       \
    if (dens.nitems > 0) kd<<<dens.nitems, TI_ * K_, 0, s>>>(src, c, ph, s32, dens);    \
    if (force.nitems > 0) kf<<<force.nitems, TI_ * K_, 0, s>>>(src, c, ph, s32, force); \
    return hipGetLastError();                                                          \
  }
  SPH_TASK_CASE(64, 4)
  SPH_TASK_CASE(32, 8)
  SPH_TASK_CASE(16, 16)
#undef SPH_TASK_CASE
  return hipErrorInvalidValue;
}

// instantiated in pair_*.hip
hipError_t run_density_dens_f32(const SoaSrc<DT_F32, DT_F32, DT_F32>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_density_dens_r(const SoaSrc<DT_F16, DT_BF16, DT_F16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_density_dens_h(const SoaSrc<DT_F16, DT_F16, DT_F16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_density_dens_b(const SoaSrc<DT_BF16, DT_BF16, DT_BF16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_density_dens_gen(const SoaSrc<-1, -1, -1>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_density_dens_aos(const AosSrc& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_force_force_f32(const SoaSrc<DT_F32, DT_F32, DT_F32>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_force_force_r(const SoaSrc<DT_F16, DT_BF16, DT_F16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_force_force_h(const SoaSrc<DT_F16, DT_F16, DT_F16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_force_force_b(const SoaSrc<DT_BF16, DT_BF16, DT_BF16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_force_force_gen(const SoaSrc<-1, -1, -1>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_force_force_aos(const AosSrc& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s);
hipError_t run_tasks_f32(const SoaSrc<DT_F32, DT_F32, DT_F32>& src, const CellsDev& c,
                         const Phys& ph, int ti, int k, const TaskItems& dens,
                         const TaskItems& force, hipStream_t s);
hipError_t run_tasks_r(const SoaSrc<DT_F16, DT_BF16, DT_F16>& src, const CellsDev& c,
                       const Phys& ph, int ti, int k, const TaskItems& dens,
                       const TaskItems& force, hipStream_t s);
hipError_t run_tasks_gen(const SoaSrc<-1, -1, -1>& src, const CellsDev& c, const Phys& ph,
                         int ti, int k, const TaskItems& dens, const TaskItems& force,
                         hipStream_t s);

}  // namespace pairk
}  // namespace sph
