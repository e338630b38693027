// AoS <-> SoA conversion (Sec. 4.1 operators N, C, U and their transposes).
// Gather: sorted slot k reads record perm[k]; every write is coalesced
// (consecutive slots, consecutive addresses), the record reads are one
// 128-byte line per particle for the FP32 record.
#include "sph_device.h"

namespace sph {
namespace {

constexpr int kThreads = 256;

struct SoaOut {
  void* off[3];
  void* vq[3];
  void* m;
  void* h;
  void* u;
  double* x[3];
  float* v[3];
  float* uk;
};

__global__ __launch_bounds__(kThreads) void k_convert(const char* __restrict__ aos, AosLayout L,
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
    int c3[3];
    cell_coords(cd.cell[k], cd.n_c, c3[0], c3[1], c3[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) store_q32(o.off[a], p.pos, k, cell_offset(xw[a], c3[a], cd.n_c), 1.0f);
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

__global__ __launch_bounds__(kThreads) void k_writeback(SoaIn s, CellsDev cd, int view,
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
  k_convert<<<(c.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(static_cast<const char*>(aos),
                                                                  L, c, view, p, o);
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
  k_writeback<<<(c.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(si, c, view,
                                                                    static_cast<char*>(aos), L);
  return hipGetLastError();
}

}  // namespace sph
