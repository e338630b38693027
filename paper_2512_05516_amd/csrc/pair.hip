// Quadratic kernels: the density loop and the force loop over the cell list
// (Alg. 1 CallQuadratic; Eq. density, Eq. momentum, Eq. energy).
//
// One workgroup per (cell, chunk of TI particles): the chunk's particles i
// are held in registers, K lanes per particle. The workgroup walks the
// candidates j of the 27 surrounding cells as one flattened index space and
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
#include "sph_device.h"

namespace sph {
namespace {

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

  __device__ __forceinline__ void pos(int k, int cell, int n_c, float& x, float& y,
                                      float& z) const {
    (void)cell;
    (void)n_c;
    x = load_fmt<PT>(off[0], pos_dt, k, 1.0f);
    y = load_fmt<PT>(off[1], pos_dt, k, 1.0f);
    z = load_fmt<PT>(off[2], pos_dt, k, 1.0f);
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

template <int NT>
__device__ __forceinline__ float block_max(float v, float* lds) {
  constexpr int NW = NT / 64;
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = lds[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = fmaxf(r, lds[w]);
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ float block_min(float v, float* lds) {
  return -block_max<NT>(-v, lds);
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

__device__ __forceinline__ void neighbour_cell(int nb, int cx, int cy, int cz, int n_c, float s,
                                               int& cn, float& shx, float& shy, float& shz) {
  int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = nb / 9 - 1;
  int nx = cx + dx, ny = cy + dy, nz = cz + dz;
  nx += (nx < 0) ? n_c : ((nx >= n_c) ? -n_c : 0);
  ny += (ny < 0) ? n_c : ((ny >= n_c) ? -n_c : 0);
  nz += (nz < 0) ? n_c : ((nz >= n_c) ? -n_c : 0);
  cn = nx + n_c * (ny + n_c * nz);
  shx = dx < 0 ? -s : (dx > 0 ? s : 0.0f);
  shy = dy < 0 ? -s : (dy > 0 ? s : 0.0f);
  shz = dz < 0 ? -s : (dz > 0 ? s : 0.0f);
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
// Neighbour-cell table of a block: the 27 cells around the block's cell,
// their slot ranges, the prefix of their counts (a flattened candidate index
// space) and the position shift of each cell relative to the block's cell.
// --------------------------------------------------------------------------
struct NbrTab {
  int start[27];
  int cell[27];
  int pre[28];
  float sh[27][3];
};

__device__ __forceinline__ void build_nbr(NbrTab& T, const CellsDev& cd, int cx, int cy, int cz,
                                          float s32) {
  const int tid = threadIdx.x;
  if (tid < 27) {
    int cn;
    float shx, shy, shz;
    neighbour_cell(tid, cx, cy, cz, cd.n_c, s32, cn, shx, shy, shz);
    const int st = clamp_slot(cd.start[cn], cd.n);
    const int en = max(clamp_slot(cd.start[cn + 1], cd.n), st);
    T.start[tid] = st;
    T.cell[tid] = cn;
    T.pre[tid + 1] = en - st;
    T.sh[tid][0] = shx;
    T.sh[tid][1] = shy;
    T.sh[tid][2] = shz;
  }
  __syncthreads();
  if (tid == 0) {
    T.pre[0] = 0;
    for (int q = 0; q < 27; ++q) T.pre[q + 1] += T.pre[q];
  }
  __syncthreads();
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
constexpr int kRounds = 8;      // gather rounds whose loads are issued together
constexpr int kFillRounds = 4;  // force-only fields: rounds issued together

// Chunk bounding box of the valid particles and the largest H^2
struct ChunkBox {
  float lox, loy, loz, hix, hiy, hiz, h2max;
};

template <int NT>
__device__ __forceinline__ ChunkBox chunk_box(bool vi, float xi, float yi, float zi, float H2,
                                              float* red) {
  const float inf = __builtin_inff();
  ChunkBox b;
  b.lox = block_min<NT>(vi ? xi : inf, red);
  b.loy = block_min<NT>(vi ? yi : inf, red);
  b.loz = block_min<NT>(vi ? zi : inf, red);
  b.hix = block_max<NT>(vi ? xi : -inf, red);
  b.hiy = block_max<NT>(vi ? yi : -inf, red);
  b.hiz = block_max<NT>(vi ? zi : -inf, red);
  b.h2max = block_max<NT>(H2, red);
  return b;
}

// Phase A over the staged candidates [0, nj) (nj a multiple of K * kUnroll,
// padded with entries nobody accepts): lane kk of its particle tests
// candidates kk, kk + K, ... and appends the accepted ones to its list;
// `consume(lo)` runs phase B over list entries [tid, lo) whenever the lists
// may fill up and at the end.
template <int NT, int K, int LCAP, class Accept, class Consume>
__device__ __forceinline__ void test_and_consume(const float4* cp, uint16_t* lst, int nj, int kk,
                                                 Accept accept, Consume consume) {
  const int tid = threadIdx.x;
  const int nit = nj / K;
  int it = 0;
  while (it < nit) {
    int lo = tid;
    const int lim = tid + (LCAP - kUnroll) * NT;
    while (it < nit) {
      const float4* cq = cp + kk + K * it;
      float4 qv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) qv[u] = cq[K * u];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const bool acc = accept(qv[u]);
        lst[lo] = (uint16_t)(kk + K * (it + u));
        lo += acc ? NT : 0;
      }
      it += kUnroll;
      if (__any(lo > lim)) break;
    }
    consume(lo);
  }
}

// --------------------------------------------------------------------------
// Density
// --------------------------------------------------------------------------
template <int TI, int K, class Src>
__global__ __launch_bounds__(TI* K) void k_density(Src src, CellsDev cd, Phys ph, float s32) {
  constexpr int NT = TI * K;
  constexpr int CAP = 4 * NT;
  constexpr int LCAP = 40;
  constexpr int kPad = K * kUnroll;
  __shared__ float4 cand[CAP];                 // x, y, z relative to this cell, m_j
  __shared__ uint16_t lst[LCAP * NT];
  __shared__ NbrTab T;
  __shared__ int wtot[2 * (NT / 64)];
  __shared__ float red[NT / 64];

  const int n_c = cd.n_c;
  const int cell = xcd_remap(blockIdx.x, gridDim.x);
  const int cs = clamp_slot(cd.start[cell], cd.n), ce = max(clamp_slot(cd.start[cell + 1], cd.n), cs);
  if (cs == ce) return;                        // uniform: empty cell
  int cx, cy, cz;
  cell_coords(cell, n_c, cx, cy, cz);
  build_nbr(T, cd, cx, cy, cz, s32);
  const int total = T.pre[27];
  const int tid = threadIdx.x;
  const int gi = tid / K, kk = tid % K;
  const float gk = ph.gamma_k;

  for (int base = cs; base < ce; base += TI) {
    const int i = base + gi;
    const bool vi = i < ce;
    float xi = 0.f, yi = 0.f, zi = 0.f, hi = 0.f, ui = 0.f;
    if (vi) {
      src.pos(i, cell, n_c, xi, yi, zi);
      hi = src.hsml(i);
      ui = src.uint(i);
    }
    const float H2 = vi ? support2(gk, hi) : 0.0f;
    const float Hinv = vi ? 1.0f / (gk * hi) : 0.0f;
    const ChunkBox bx = chunk_box<NT>(vi, xi, yi, zi, H2, red);
    if (vi && cd.status && H2 > s32 * s32) atomicOr(cd.status, SPH_FLAG_H_TOO_LARGE);

    float rho = 0.f, wsum = 0.f, dh = 0.f;
    int nn = 0;

    auto pair_phase = [&](int nj) {
      // pad [nj, roundup(nj, kPad)) with entries no particle accepts
      const int njp = (nj + kPad - 1) / kPad * kPad;
      if (tid < njp - nj) cand[nj + tid] = make_float4(1e30f, 1e30f, 1e30f, 0.f);
      __syncthreads();
      test_and_consume<NT, K, LCAP>(
          cand, lst, njp, kk,
          [&](const float4& q) {
            float dx, dy, dz;
            return dist2(xi, yi, zi, q.x, q.y, q.z, dx, dy, dz) < H2;
          },
          [&](int lo) {
            for (int e = tid; e < lo; e += NT) {
              const float4 q = cand[lst[e]];
              float dx, dy, dz;
              const float r2 = dist2(xi, yi, zi, q.x, q.y, q.z, dx, dy, dz);
              const float u = fast_sqrt(r2) * Hinv;
              float w, dw;
              kernel_w_dw(u, w, dw);
              rho = fmaf(q.w, w, rho);
              wsum += w;
              dh = fmaf(q.w, fmaf(u, dw, 3.0f * w), dh);
            }
            nn += (lo - tid) / NT;
          });
      __syncthreads();
    };

    // gather: the 27 cells' candidates as one flattened index space; the
    // loads of kRounds rounds are in flight before the first prune
    int nj = 0, q = 0, rnd = 0;
    for (int sb = 0; sb < total; sb += kRounds * NT) {
      float4 c[kRounds];
      int qq[kRounds];
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const int idx = sb + r * NT + tid;
        c[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        qq[r] = q;
        if (idx < total) {
          while (idx >= T.pre[q + 1]) ++q;
          qq[r] = q;
          const int j = T.start[q] + (idx - T.pre[q]);
          src.pos(j, T.cell[q], n_c, c[r].x, c[r].y, c[r].z);
          c[r].w = src.mass(j);
        }
      }
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        if (sb + r * NT >= total) break;       // uniform
        const int idx = sb + r * NT + tid;
        bool ok = idx < total;
        if (ok) {
          c[r].x = shifted(c[r].x, T.sh[qq[r]][0]);
          c[r].y = shifted(c[r].y, T.sh[qq[r]][1]);
          c[r].z = shifted(c[r].z, T.sh[qq[r]][2]);
          ok = box_dist2(c[r].x, c[r].y, c[r].z, bx.lox, bx.loy, bx.loz, bx.hix, bx.hiy,
                         bx.hiz) < bx.h2max;
        }
        int njn = nj;
        int slot = compact_round<NT>(ok, njn, wtot, rnd++);
        if (njn > CAP - kPad) {                 // uniform: consume the staged ones first
          pair_phase(nj);
          njn -= nj;
          nj = 0;
        }
        if (ok) cand[nj + slot] = c[r];
        nj = njn;
      }
    }
    pair_phase(nj);

    rho = group_sum<K>(rho);
    wsum = group_sum<K>(wsum);
    dh = group_sum<K>(dh);
    nn = group_sum_i<K>(nn);
    if (vi && kk == 0) {
      const float Hinv3 = Hinv * Hinv * Hinv;
      const float rho_i = rho * Hinv3;
      const float rho_dh = -gk * dh * Hinv3 * Hinv;
      const float omega = 1.0f + hi * rho_dh / (3.0f * rho_i);
      const float f = ph.gradh ? 1.0f / omega : 1.0f;
      const float P = (ph.gamma - 1.0f) * rho_i * ui;
      const float c = sqrtf(ph.gamma * (ph.gamma - 1.0f) * ui);
      src.dens_out(i, rho_i, kFourPiThird * wsum, rho_dh, f, P, c, nn);
    }
  }
}

// --------------------------------------------------------------------------
// Force
// --------------------------------------------------------------------------
template <int TI, int K, class Src>
__global__ __launch_bounds__(TI* K) void k_force(Src src, CellsDev cd, Phys ph, float s32) {
  constexpr int NT = TI * K;
  constexpr int CAP = 5 * NT / 2;
  constexpr int LCAP = 32;
  constexpr int kPad = K * kUnroll;
  __shared__ float4 cp[CAP];      // x, y, z (relative to this cell), H_j^2
  __shared__ float4 cv[CAP];      // v_j, m_j
  __shared__ float4 cs4[CAP];     // 1/H_j, A_j, c_j, rho_j
  __shared__ int cid[CAP];        // sorted slot of j
  __shared__ uint16_t lst[LCAP * NT];
  __shared__ NbrTab T;
  __shared__ int wtot[2 * (NT / 64)];
  __shared__ float red[NT / 64];

  const int n_c = cd.n_c;
  const int cell = xcd_remap(blockIdx.x, gridDim.x);
  const int cs = clamp_slot(cd.start[cell], cd.n), ce = max(clamp_slot(cd.start[cell + 1], cd.n), cs);
  if (cs == ce) return;
  int cx, cy, cz;
  cell_coords(cell, n_c, cx, cy, cz);
  build_nbr(T, cd, cx, cy, cz, s32);
  const int total = T.pre[27];
  const int tid = threadIdx.x;
  const int gi = tid / K, kk = tid % K;
  const float gk = ph.gamma_k;
  const float alpha = ph.alpha, beta = ph.beta;

  for (int base = cs; base < ce; base += TI) {
    const int i = base + gi;
    const bool vi = i < ce;
    // lanes without a particle sit far outside the box and accept nothing
    float xi = 1e30f, yi = 1e30f, zi = 1e30f, hi = 1.f, vxi = 0.f, vyi = 0.f, vzi = 0.f;
    float rhoi = 1.f, fi = 1.f, Pi_ = 0.f, ci = 0.f;
    if (vi) {
      src.pos(i, cell, n_c, xi, yi, zi);
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

    float ax = 0.f, ay = 0.f, az = 0.f, du = 0.f, vsig = 0.f;
    int nf = 0;

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

    auto pair_phase = [&](int nj) {
      const int njp = (nj + kPad - 1) / kPad * kPad;
      if (tid < njp - nj) {
        cp[nj + tid] = make_float4(1e30f, 1e30f, 1e30f, 0.f);
        cid[nj + tid] = -1;
      }
      __syncthreads();
      test_and_consume<NT, K, LCAP>(
          cp, lst, njp, kk,
          [&](const float4& q0) {
            float dx, dy, dz;
            return dist2(xi, yi, zi, q0.x, q0.y, q0.z, dx, dy, dz) < fmaxf(H2i, q0.w);
          },
          [&](int lo) {
            for (int e = tid; e < lo; e += NT) {
              const int t = lst[e];
              const float4 q0 = cp[t];
              float dx, dy, dz;
              const float r2 = dist2(xi, yi, zi, q0.x, q0.y, q0.z, dx, dy, dz);
              // the self pair has r2 = 0 exactly; so may coincident stored
              // positions, for which w'(0) = 0 makes the pair's terms vanish
              if (r2 == 0.0f && cid[t] == i) continue;
              const float4 q1 = cv[t];
              const float4 q2 = cs4[t];
              const float r = fast_sqrt(r2);
              const float rinv = r2 > 0.0f ? fast_rcp(r) : 0.0f;
              const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
              const float gi_ = kernel_dw(r * Hinvi) * Hinv4i;
              const float hj2 = q2.x * q2.x;
              const float gj_ = kernel_dw(r * q2.x) * (hj2 * hj2);
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
              vsig = fmaxf(vsig, vs);
              ++nf;
            }
          });
      __syncthreads();
    };

    int nj = 0, filled = 0, q = 0, rnd = 0;
    for (int sb = 0; sb < total; sb += kRounds * NT) {
      float4 c[kRounds];
      int qq[kRounds], jj[kRounds];
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const int idx = sb + r * NT + tid;
        c[r] = make_float4(0.f, 0.f, 0.f, 1.f);
        qq[r] = q;
        jj[r] = 0;
        if (idx < total) {
          while (idx >= T.pre[q + 1]) ++q;
          qq[r] = q;
          jj[r] = T.start[q] + (idx - T.pre[q]);
          src.pos(jj[r], T.cell[q], n_c, c[r].x, c[r].y, c[r].z);
          c[r].w = src.hsml(jj[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        if (sb + r * NT >= total) break;       // uniform
        const int idx = sb + r * NT + tid;
        bool ok = idx < total;
        if (ok) {
          c[r].x = shifted(c[r].x, T.sh[qq[r]][0]);
          c[r].y = shifted(c[r].y, T.sh[qq[r]][1]);
          c[r].z = shifted(c[r].z, T.sh[qq[r]][2]);
          c[r].w = support2(gk, c[r].w);
          ok = box_dist2(c[r].x, c[r].y, c[r].z, bx.lox, bx.loy, bx.loz, bx.hix, bx.hiy,
                         bx.hiz) < fmaxf(bx.h2max, c[r].w);
        }
        int njn = nj;
        int slot = compact_round<NT>(ok, njn, wtot, rnd++);
        if (njn > CAP - kPad) {                 // uniform: consume the staged ones first
          fill(filled, nj);
          pair_phase(nj);
          njn -= nj;
          nj = 0;
          filled = 0;
        }
        if (ok) {
          cp[nj + slot] = c[r];
          cid[nj + slot] = jj[r];
        }
        nj = njn;
      }
      // force-only fields of this super-round's candidates, one batch
      fill(filled, nj);
      filled = nj;
    }
    pair_phase(nj);

    ax = group_sum<K>(ax);
    ay = group_sum<K>(ay);
    az = group_sum<K>(az);
    du = group_sum<K>(du);
    vsig = group_max<K>(vsig);
    nf = group_sum_i<K>(nf);
    if (vi && kk == 0) src.force_out(i, ax, ay, az, du, vsig, nf);
  }
}

template <int PT, int VT, int MT>
SoaSrc<PT, VT, MT> make_soa(const sph_soa& s, const Prec& p) {
  SoaSrc<PT, VT, MT> r;
  for (int k = 0; k < 3; ++k) {
    r.off[k] = s.f[SPH_S_OFF_X + k];
    r.vq[k] = s.f[SPH_S_VQ_X + k];
  }
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

template <class S>
hipError_t run_density(const S& src, const CellsDev& c, const Phys& ph, int ti, int k,
                       hipStream_t s) {
  const int C = c.n_c * c.n_c * c.n_c;
  const float s32 = (float)(1.0 / (double)c.n_c);
#define SPH_DENS_CASE(TI_, K_)                                                   \
  if (ti == TI_ && k == K_) {                                                    \
    k_density<TI_, K_, S><<<C, TI_ * K_, 0, s>>>(src, c, ph, s32);                \
    return hipGetLastError();                                                    \
  }
  SPH_DENS_CASE(64, 4)
  SPH_DENS_CASE(32, 8)
  SPH_DENS_CASE(128, 2)
  SPH_DENS_CASE(64, 2)
  SPH_DENS_CASE(64, 1)
#undef SPH_DENS_CASE
  return hipErrorInvalidValue;
}

template <class S>
hipError_t run_force(const S& src, const CellsDev& c, const Phys& ph, int ti, int k,
                     hipStream_t s) {
  const int C = c.n_c * c.n_c * c.n_c;
  const float s32 = (float)(1.0 / (double)c.n_c);
#define SPH_FORCE_CASE(TI_, K_)                                                  \
  if (ti == TI_ && k == K_) {                                                    \
    k_force<TI_, K_, S><<<C, TI_ * K_, 0, s>>>(src, c, ph, s32);                  \
    return hipGetLastError();                                                    \
  }
  SPH_FORCE_CASE(64, 4)
  SPH_FORCE_CASE(32, 8)
  SPH_FORCE_CASE(128, 2)
  SPH_FORCE_CASE(64, 2)
  SPH_FORCE_CASE(64, 1)
#undef SPH_FORCE_CASE
  return hipErrorInvalidValue;
}

template <class S>
struct RunDensity {
  static hipError_t go(const S& src, const CellsDev& c, const Phys& ph, int ti, int k,
                       hipStream_t s) {
    return run_density(src, c, ph, ti, k, s);
  }
};
template <class S>
struct RunForce {
  static hipError_t go(const S& src, const CellsDev& c, const Phys& ph, int ti, int k,
                       hipStream_t s) {
    return run_force(src, c, ph, ti, k, s);
  }
};

// Storage formats with compiled-in loaders; every other combination uses the
// run-time loader.
template <template <class> class Run>
hipError_t dispatch_soa(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                        int ti, int k, hipStream_t s) {
  if (p.pos == DT_F32 && p.vel == DT_F32 && p.mhu == DT_F32)
    return Run<SoaSrc<DT_F32, DT_F32, DT_F32>>::go(make_soa<DT_F32, DT_F32, DT_F32>(soa, p), c,
                                                    ph, ti, k, s);
  if (p.pos == DT_F16 && p.vel == DT_BF16 && p.mhu == DT_F16)
    return Run<SoaSrc<DT_F16, DT_BF16, DT_F16>>::go(make_soa<DT_F16, DT_BF16, DT_F16>(soa, p), c,
                                                     ph, ti, k, s);
  return Run<SoaSrc<-1, -1, -1>>::go(make_soa<-1, -1, -1>(soa, p), c, ph, ti, k, s);
}

}  // namespace

bool tile_supported(int ti, int k) {
  return (ti == 64 && (k == 4 || k == 2 || k == 1)) || (ti == 32 && k == 8) ||
         (ti == 128 && k == 2);
}

hipError_t launch_density(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                          int ti, int k, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  return dispatch_soa<RunDensity>(soa, p, c, ph, ti, k, s);
}

hipError_t launch_force(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                        int ti, int k, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  return dispatch_soa<RunForce>(soa, p, c, ph, ti, k, s);
}

hipError_t launch_density_aos(void* aos, const AosLayout& L, const CellsDev& c, const Phys& ph,
                              int ti, int k, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  AosSrc src{static_cast<char*>(aos), L, c.perm};
  return run_density(src, c, ph, ti, k, s);
}

hipError_t launch_force_aos(void* aos, const AosLayout& L, const CellsDev& c, const Phys& ph,
                            int ti, int k, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  AosSrc src{static_cast<char*>(aos), L, c.perm};
  return run_force(src, c, ph, ti, k, s);
}

}  // namespace sph
