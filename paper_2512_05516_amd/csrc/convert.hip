// AoS <-> SoA conversion (Sec. 4.1 operators N, C, U and their transposes).
// Sorted slot k reads or writes record perm[k]. Records are moved whole
// through LDS: a workgroup of 256 slots reads its records as consecutive
// 8-byte words (each wave instruction covers whole 128-byte lines), extracts
// or patches the fields per slot from LDS rows of odd word pitch (no bank
// conflicts on same-offset field access), and writes SoA arrays (coalesced)
// or whole records back. Records wider than kMaxStagedStride bytes take the
// per-field kernels.
#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;

struct SoaOut {
  void* off[3];
  uint8_t* anc;
  void* vq[3];
  void* m;
  void* h;
  void* u;
  double* x[3];
  float* v[3];
  float* uk;
};

__global__ __launch_bounds__(kThreads) void k_convert_direct(const char* __restrict__ aos, AosLayout L,
                                                       CellsDev cd, int view, Prec p, SoaOut o) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= cd.n) return;
  const char* rec = aos + (size_t)cd.perm[k] * L.stride;
  const bool pair_view = view != SPH_VIEW_KICK;
  const bool need_v = view == SPH_VIEW_FORCE || view == SPH_VIEW_FULL || view == SPH_VIEW_KICK;
  const bool need_u = view == SPH_VIEW_DENSITY || view == SPH_VIEW_FULL || view == SPH_VIEW_KICK;
  const double* xp = reinterpret_cast<const double*>(rec + L.off[SPH_A_X]);
  double xw[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) xw[a] = wrap01(xp[a]);
  double v[3] = {0.0, 0.0, 0.0};
  if (need_v) {
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = rec_load(rec, L.off[SPH_A_V], L.dt[SPH_A_V], a);
  }
  const double u = need_u ? rec_load(rec, L.off[SPH_A_U], L.dt[SPH_A_U]) : 0.0;
  if (pair_view) {
    int c3[3], code = 0;
    cell_coords(cd.cell[k], cd.n_c, c3[0], c3[1], c3[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int sa;
      store_q32(o.off[a], p.pos, k, anchor_offset(xw[a], c3[a], cd.n_c, p.anchor, sa), 1.0f);
      code |= sa << (2 * a);
    }
    if (p.anchor >= SPH_ANCHOR_SUB(1)) o.anc[k] = (uint8_t)code;
    store_q(o.m, p.mhu, k, rec_load(rec, L.off[SPH_A_M], L.dt[SPH_A_M]), p.store_m);
    store_q(o.h, p.mhu, k, rec_load(rec, L.off[SPH_A_H], L.dt[SPH_A_H]), p.store_h);
    if (view != SPH_VIEW_FORCE) store_q(o.u, p.mhu, k, u, p.store_u);
    if (view != SPH_VIEW_DENSITY) {
#pragma unroll
      for (int a = 0; a < 3; ++a) store_q(o.vq[a], p.vel, k, v[a], 1.0f);
    }
  }
  if (view == SPH_VIEW_KICK || view == SPH_VIEW_FULL) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      o.x[a][k] = xw[a];
      o.v[a][k] = (float)v[a];
    }
    o.uk[k] = (float)u;
  }
}

struct SoaIn {
  const double* x[3];
  const float* v[3];
  const float* uk;
  const float *rho, *wcount, *rho_dh, *f, *P, *c;
  const int32_t* nngb;
  const float *a[3], *du, *vsig;
  const int32_t* nforce;
};

__global__ __launch_bounds__(kThreads) void k_writeback_direct(SoaIn s, CellsDev cd, int view,
                                                         char* __restrict__ aos, AosLayout L) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= cd.n) return;
  char* rec = aos + (size_t)cd.perm[k] * L.stride;
  if (view == SPH_VIEW_KICK || view == SPH_VIEW_FULL) {
    double* xp = reinterpret_cast<double*>(rec + L.off[SPH_A_X]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xp[a] = s.x[a][k];
      rec_store32(rec, L.off[SPH_A_V], L.dt[SPH_A_V], s.v[a][k], a);
    }
    rec_store32(rec, L.off[SPH_A_U], L.dt[SPH_A_U], s.uk[k]);
  }
  if ((view == SPH_VIEW_DENSITY || view == SPH_VIEW_FULL) && s.rho) {
    rec_store32(rec, L.off[SPH_A_RHO], L.dt[SPH_A_RHO], s.rho[k]);
    rec_store32(rec, L.off[SPH_A_WCOUNT], L.dt[SPH_A_WCOUNT], s.wcount[k]);
    rec_store32(rec, L.off[SPH_A_RHO_DH], L.dt[SPH_A_RHO_DH], s.rho_dh[k]);
    rec_store32(rec, L.off[SPH_A_F], L.dt[SPH_A_F], s.f[k]);
    rec_store32(rec, L.off[SPH_A_P], L.dt[SPH_A_P], s.P[k]);
    rec_store32(rec, L.off[SPH_A_C], L.dt[SPH_A_C], s.c[k]);
    rec_store_i32(rec, L.off[SPH_A_NNGB], s.nngb[k]);
  }
  if ((view == SPH_VIEW_FORCE || view == SPH_VIEW_FULL) && s.a[0]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) rec_store32(rec, L.off[SPH_A_A], L.dt[SPH_A_A], s.a[a][k], a);
    rec_store32(rec, L.off[SPH_A_DU], L.dt[SPH_A_DU], s.du[k]);
    rec_store32(rec, L.off[SPH_A_VSIG], L.dt[SPH_A_VSIG], s.vsig[k]);
    if (s.nforce) rec_store_i32(rec, L.off[SPH_A_NFORCE], s.nforce[k]);
  }
  if (view == SPH_VIEW_FULL) rec_store_i32(rec, L.off[SPH_A_CELL], cd.cell[k]);
}


// --- whole-record staging ----------------------------------------------------
constexpr int kTileSlots = 256;                 // slots per workgroup
// kMaxStagedStride (248): (stride/8 + 1) * 8 * 256 <= 64 KiB

// Copy the records of slots [k0, k0 + nk) between global memory and LDS rows
// of W + 1 words. Word e of the tile is (record e / W, word e % W); the
// (record, word) pair advances by (256 / W, 256 % W) per step, so no division
// runs inside the loop. The tile's record indices are staged in LDS first.
// W_ > 0 fixes the record width at compile time (fully unrolled, all loads of
// a thread in flight at once); W_ = 0 takes it from the layout.
template <int W_, bool kToLds>
__device__ __forceinline__ void stage_records(uint64_t* rows, const int* prm, char* aos, int nk,
                                              int Wrt, uint32_t stride) {
  const int W = W_ > 0 ? W_ : Wrt;
  const int pitch = W + 1;
  const int tid = threadIdx.x;
  const int dr = kThreads / W, dof = kThreads - dr * W;
  int r = tid / W, o = tid - r * W;
  const int total = nk * W;
  if (W_ > 0 && nk == kTileSlots) {
#pragma unroll
    for (int it = 0; it < W_; ++it) {       // kTileSlots * W_ / kThreads == W_ steps
      uint64_t* g = reinterpret_cast<uint64_t*>(aos + (size_t)prm[r] * stride) + o;
      if (kToLds) rows[r * pitch + o] = __builtin_nontemporal_load(g);
      else __builtin_nontemporal_store(rows[r * pitch + o], g);
      r += dr;
      o += dof;
      if (o >= W) {
        o -= W;
        ++r;
      }
    }
    return;
  }
  for (int e = tid; e < total; e += kThreads) {
    uint64_t* g = reinterpret_cast<uint64_t*>(aos + (size_t)prm[r] * stride) + o;
    if (kToLds) rows[r * pitch + o] = *g;
    else *g = rows[r * pitch + o];
    r += dr;
    o += dof;
    if (o >= W) {
      o -= W;
      ++r;
    }
  }
}

// Narrowed fields of the pair views, in the order of SoaOut's arrays
enum : int { kF_OFF = 0, kF_VQ = 3, kF_M = 6, kF_H = 7, kF_U = 8, kNarrowed = 9 };

template <int W_, bool PACK>
__global__ __launch_bounds__(kThreads) void k_convert_staged(const char* __restrict__ aos,
                                                              AosLayout L, CellsDev cd, int view,
                                                              Prec p, SoaOut o) {
  extern __shared__ uint64_t rows[];
  __shared__ int prm[kTileSlots];
  // codes of the truncated fields, assembled into whole words at the end
  __shared__ uint32_t codes[PACK ? kNarrowed : 1][PACK ? kTileSlots : 1];
  const int W = W_ > 0 ? W_ : (int)(L.stride >> 3), pitch = W + 1;
  const int k0 = blockIdx.x * kTileSlots;
  const int nk = min(kTileSlots, cd.n - k0);
  if ((int)threadIdx.x < nk) prm[threadIdx.x] = cd.perm[k0 + threadIdx.x];
  __syncthreads();
  stage_records<W_, true>(rows, prm, const_cast<char*>(aos), nk, W, L.stride);
  __syncthreads();
  const int t = threadIdx.x;
  const bool pair_view = view != SPH_VIEW_KICK;
  const bool need_v = view != SPH_VIEW_DENSITY;
  const bool need_u = view != SPH_VIEW_FORCE;
  // narrowed field f of slot k: an IEEE store, or this slot's code
  auto put = [&](int f, void* dst, int dt, int k, float q) {
    if constexpr (PACK) {
      if (dt >= DT_TRUNC) {
        codes[f][t] = trunc_code(q, dt - DT_TRUNC);
        return;
      }
    }
    store_q32(dst, dt, k, q, 1.0f);
  };
  if constexpr (PACK) {
    for (int f = 0; f < kNarrowed; ++f) codes[f][t] = 0u;   // slots past n
  }
  if (t < nk) {
    const int k = k0 + t;
    const char* rec = reinterpret_cast<const char*>(rows + t * pitch);
    const double* xp = reinterpret_cast<const double*>(rec + L.off[SPH_A_X]);
    double xw[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xw[a] = wrap01(xp[a]);
    double v[3] = {0.0, 0.0, 0.0};
    if (need_v) {
#pragma unroll
      for (int a = 0; a < 3; ++a) v[a] = rec_load(rec, L.off[SPH_A_V], L.dt[SPH_A_V], a);
    }
    const double u = need_u ? rec_load(rec, L.off[SPH_A_U], L.dt[SPH_A_U]) : 0.0;
    if (pair_view) {
      int c3[3], code = 0;
      cell_coords(cd.cell[k], cd.n_c, c3[0], c3[1], c3[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        int sa;
        put(kF_OFF + a, o.off[a], p.pos, k, anchor_offset(xw[a], c3[a], cd.n_c, p.anchor, sa));
        code |= sa << (2 * a);
      }
      if (p.anchor >= SPH_ANCHOR_SUB(1)) o.anc[k] = (uint8_t)code;
      put(kF_M, o.m, p.mhu, k, (float)rec_load(rec, L.off[SPH_A_M], L.dt[SPH_A_M]) * p.store_m);
      put(kF_H, o.h, p.mhu, k, (float)rec_load(rec, L.off[SPH_A_H], L.dt[SPH_A_H]) * p.store_h);
      if (view != SPH_VIEW_FORCE) put(kF_U, o.u, p.mhu, k, (float)u * p.store_u);
      if (view != SPH_VIEW_DENSITY) {
#pragma unroll
        for (int a = 0; a < 3; ++a) put(kF_VQ + a, o.vq[a], p.vel, k, (float)v[a]);
      }
    }
    if (view == SPH_VIEW_KICK || view == SPH_VIEW_FULL) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        o.x[a][k] = xw[a];
        o.v[a][k] = (float)v[a];
      }
      o.uk[k] = (float)u;
    }
  }
  if constexpr (!PACK) return;
  if (!pair_view) return;
  __syncthreads();
  // the tile's 256 codes of T bits fill words [8 T b, 8 T (b + 1)) exactly
  for (int f = 0; f < kNarrowed; ++f) {
    const int dt = f < kF_VQ ? p.pos : (f < kF_M ? p.vel : p.mhu);
    void* dst = f < kF_VQ ? o.off[f] : (f < kF_M ? o.vq[f - kF_VQ] : (f == kF_M ? o.m : (f == kF_H ? o.h : o.u)));
    const bool present = (f < kF_VQ || f == kF_M || f == kF_H) ||
                         (f < kF_M ? view != SPH_VIEW_DENSITY : view != SPH_VIEW_FORCE);
    if (dt < DT_TRUNC || !present) continue;     // uniform
    const int T = dt - DT_TRUNC;
    const int nw = 8 * T;
    for (int w = t; w < nw; w += kThreads) {
      const int b0 = 32 * w;
      uint32_t word = 0u;
      for (int j = b0 / T; j <= (b0 + 31) / T && j < kTileSlots; ++j) {
        const int sh = j * T - b0;
        const uint64_t c = codes[f][j];
        word |= sh >= 0 ? (uint32_t)(c << sh) : (uint32_t)(c >> -sh);
      }
      static_cast<uint32_t*>(dst)[(size_t)blockIdx.x * nw + w] = word;
    }
  }
}

template <int W_>
__global__ __launch_bounds__(kThreads) void k_writeback_staged(SoaIn s, CellsDev cd, int view,
                                                                char* __restrict__ aos,
                                                                AosLayout L) {
  extern __shared__ uint64_t rows[];
  __shared__ int prm[kTileSlots];
  const int W = W_ > 0 ? W_ : (int)(L.stride >> 3), pitch = W + 1;
  const int k0 = blockIdx.x * kTileSlots;
  const int nk = min(kTileSlots, cd.n - k0);
  if ((int)threadIdx.x < nk) prm[threadIdx.x] = cd.perm[k0 + threadIdx.x];
  __syncthreads();
  stage_records<W_, true>(rows, prm, aos, nk, W, L.stride);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < nk) {
    const int k = k0 + t;
    char* rec = reinterpret_cast<char*>(rows + t * pitch);
    if (view == SPH_VIEW_KICK || view == SPH_VIEW_FULL) {
      double* xp = reinterpret_cast<double*>(rec + L.off[SPH_A_X]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        xp[a] = s.x[a][k];
        rec_store32(rec, L.off[SPH_A_V], L.dt[SPH_A_V], s.v[a][k], a);
      }
      rec_store32(rec, L.off[SPH_A_U], L.dt[SPH_A_U], s.uk[k]);
    }
    if ((view == SPH_VIEW_DENSITY || view == SPH_VIEW_FULL) && s.rho) {
      rec_store32(rec, L.off[SPH_A_RHO], L.dt[SPH_A_RHO], s.rho[k]);
      rec_store32(rec, L.off[SPH_A_WCOUNT], L.dt[SPH_A_WCOUNT], s.wcount[k]);
      rec_store32(rec, L.off[SPH_A_RHO_DH], L.dt[SPH_A_RHO_DH], s.rho_dh[k]);
      rec_store32(rec, L.off[SPH_A_F], L.dt[SPH_A_F], s.f[k]);
      rec_store32(rec, L.off[SPH_A_P], L.dt[SPH_A_P], s.P[k]);
      rec_store32(rec, L.off[SPH_A_C], L.dt[SPH_A_C], s.c[k]);
      rec_store_i32(rec, L.off[SPH_A_NNGB], s.nngb[k]);
    }
    if ((view == SPH_VIEW_FORCE || view == SPH_VIEW_FULL) && s.a[0]) {
#pragma unroll
      for (int a = 0; a < 3; ++a) rec_store32(rec, L.off[SPH_A_A], L.dt[SPH_A_A], s.a[a][k], a);
      rec_store32(rec, L.off[SPH_A_DU], L.dt[SPH_A_DU], s.du[k]);
      rec_store32(rec, L.off[SPH_A_VSIG], L.dt[SPH_A_VSIG], s.vsig[k]);
      if (s.nforce) rec_store_i32(rec, L.off[SPH_A_NFORCE], s.nforce[k]);
    }
    if (view == SPH_VIEW_FULL) rec_store_i32(rec, L.off[SPH_A_CELL], cd.cell[k]);
  }
  __syncthreads();
  stage_records<W_, false>(rows, prm, aos, nk, W, L.stride);
}

}  // namespace

hipError_t launch_convert(const void* aos, const AosLayout& L, const CellsDev& c, int view,
                          const Prec& p, const sph_soa& out, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  SoaOut o;
  for (int a = 0; a < 3; ++a) {
    o.off[a] = out.f[SPH_S_OFF_X + a];
    o.vq[a] = out.f[SPH_S_VQ_X + a];
    o.x[a] = static_cast<double*>(out.f[SPH_S_X_X + a]);
    o.v[a] = static_cast<float*>(out.f[SPH_S_V_X + a]);
  }
  o.m = out.f[SPH_S_M];
  o.h = out.f[SPH_S_H];
  o.u = out.f[SPH_S_U];
  o.uk = static_cast<float*>(out.f[SPH_S_UK]);
  o.anc = static_cast<uint8_t*>(out.f[SPH_S_ANC]);
  if (L.stride <= kMaxStagedStride) {
    const size_t lds = (size_t)kTileSlots * ((L.stride >> 3) + 1) * 8;
    const int G = (c.n + kTileSlots - 1) / kTileSlots;
    const char* a = static_cast<const char*>(aos);
    const bool pack = p.pos >= DT_TRUNC || p.vel >= DT_TRUNC || p.mhu >= DT_TRUNC;
    if (L.stride == 128 && pack)
      k_convert_staged<16, true><<<G, kThreads, lds, s>>>(a, L, c, view, p, o);
    else if (L.stride == 128)
      k_convert_staged<16, false><<<G, kThreads, lds, s>>>(a, L, c, view, p, o);
    else if (pack)
      k_convert_staged<0, true><<<G, kThreads, lds, s>>>(a, L, c, view, p, o);
    else
      k_convert_staged<0, false><<<G, kThreads, lds, s>>>(a, L, c, view, p, o);
  } else {
    k_convert_direct<<<(c.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(
        static_cast<const char*>(aos), L, c, view, p, o);
  }
  return hipGetLastError();
}

hipError_t launch_writeback(const sph_soa& in, const CellsDev& c, int view, void* aos,
                            const AosLayout& L, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  SoaIn si;
  for (int a = 0; a < 3; ++a) {
    si.x[a] = static_cast<const double*>(in.f[SPH_S_X_X + a]);
    si.v[a] = static_cast<const float*>(in.f[SPH_S_V_X + a]);
    si.a[a] = static_cast<const float*>(in.f[SPH_S_A_X + a]);
  }
  si.uk = static_cast<const float*>(in.f[SPH_S_UK]);
  si.rho = static_cast<const float*>(in.f[SPH_S_RHO]);
  si.wcount = static_cast<const float*>(in.f[SPH_S_WCOUNT]);
  si.rho_dh = static_cast<const float*>(in.f[SPH_S_RHO_DH]);
  si.f = static_cast<const float*>(in.f[SPH_S_F]);
  si.P = static_cast<const float*>(in.f[SPH_S_P]);
  si.c = static_cast<const float*>(in.f[SPH_S_C]);
  si.nngb = static_cast<const int32_t*>(in.f[SPH_S_NNGB]);
  si.du = static_cast<const float*>(in.f[SPH_S_DU]);
  si.vsig = static_cast<const float*>(in.f[SPH_S_VSIG]);
  si.nforce = static_cast<const int32_t*>(in.f[SPH_S_NFORCE]);
  if (L.stride <= kMaxStagedStride) {
    const size_t lds = (size_t)kTileSlots * ((L.stride >> 3) + 1) * 8;
    const int G = (c.n + kTileSlots - 1) / kTileSlots;
    if (L.stride == 128)
      k_writeback_staged<16><<<G, kThreads, lds, s>>>(si, c, view, static_cast<char*>(aos), L);
    else
      k_writeback_staged<0><<<G, kThreads, lds, s>>>(si, c, view, static_cast<char*>(aos), L);
  } else {
    k_writeback_direct<<<(c.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(
        si, c, view, static_cast<char*>(aos), L);
  }
  return hipGetLastError();
}

}  // namespace sph
