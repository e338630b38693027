// Host-side data management (Eq. gpu_soa_conversion_cpu_datamanagement; the
// soa_conversion_handler(host) semantics of Sec. 3.1): the host bins the
// AoS, gathers and quantises the view into pinned staging with worker
// threads, and the GPU receives only SoA arrays and the cell list.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "sph_internal.h"

namespace sph {
sph_status host_fail(sph_status code, const char* msg);
}

namespace {

using namespace sph;

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

int esz(int dt) { return (dt == SPH_F32) ? 4 : 2; }

struct Plan {
  size_t off_start, off_perm, off_cell, off_hmax;
  size_t off_pos[3], off_vq[3], off_m, off_h, off_u, off_x[3], off_v[3], off_uk, off_anc;
  size_t off_dens[4], off_acc[4];   // FORCE_IN: rho, f, P, c; KICK_IN: a[3], du
  size_t total;
  bool pair, kick, vq, u, dens_in, acc_in, anc;
};

Plan plan(int n, int n_c, int view, const sph_precision& p) {
  Plan pl;
  size_t C = (size_t)n_c * n_c * n_c;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += al256(bytes);
    return r;
  };
  const bool force = view == SPH_VIEW_FORCE || view == SPH_VIEW_FORCE_IN;
  const bool kick = view == SPH_VIEW_KICK || view == SPH_VIEW_KICK_IN;
  pl.pair = !kick;
  pl.kick = kick || view == SPH_VIEW_FULL;
  pl.vq = force || view == SPH_VIEW_FULL;
  pl.u = view == SPH_VIEW_DENSITY || view == SPH_VIEW_FULL;
  pl.dens_in = view == SPH_VIEW_FORCE_IN;
  pl.acc_in = view == SPH_VIEW_KICK_IN;
  pl.off_start = take(4 * (C + 1));
  pl.off_perm = take(4 * (size_t)n);
  pl.off_cell = take(4 * (size_t)n);
  pl.off_hmax = take(4 * (size_t)C);
  for (int a = 0; a < 3; ++a) {
    pl.off_pos[a] = pl.pair ? take((size_t)n * esz(p.pos)) : 0;
    pl.off_vq[a] = pl.vq ? take((size_t)n * esz(p.vel)) : 0;
    pl.off_x[a] = pl.kick ? take((size_t)n * 8) : 0;
    pl.off_v[a] = pl.kick ? take((size_t)n * 4) : 0;
  }
  pl.anc = pl.pair && p.pos_anchor >= SPH_ANCHOR_SUB(1);
  pl.off_anc = pl.anc ? take((size_t)n) : 0;
  pl.off_m = pl.pair ? take((size_t)n * esz(p.mhu)) : 0;
  pl.off_h = pl.pair ? take((size_t)n * esz(p.mhu)) : 0;
  pl.off_u = pl.u ? take((size_t)n * esz(p.mhu)) : 0;
  pl.off_uk = pl.kick ? take((size_t)n * 4) : 0;
  for (int q = 0; q < 4; ++q) {
    pl.off_dens[q] = pl.dens_in ? take((size_t)n * 4) : 0;
    pl.off_acc[q] = pl.acc_in ? take((size_t)n * 4) : 0;
  }
  pl.total = o;
  return pl;
}

bool known_view(int v) { return v >= SPH_VIEW_DENSITY && v <= SPH_VIEW_KICK_IN; }

// FP32 offset of a wrapped coordinate from its anchor (the definition of
// sph_precision.pos_anchor; the same FP64 expression as the device convert,
// so host and device gathers store identical values) and the sub-cell
// index a along the axis
float anchor_offset(double xw, int c, int n_c, int anchor, int& a) {
  if (anchor == SPH_ANCHOR_CORNER) {
    a = 0;
    return (float)(xw - (double)c / (double)n_c);
  }
  const int R = 1 << (anchor - 1);
  const double t = std::floor(xw * (double)(n_c * R));
  a = (t == t) ? (int)std::fmin(std::fmax(t - (double)c * R, 0.0), (double)(R - 1)) : 0;
  const double o = ((double)c * R + a + 0.5) / ((double)n_c * R);
  return (float)(xw - o);
}

double rec_d(const char* rec, uint32_t off, int dt, int c = 0) {
  if (dt == SPH_F64) {
    double v;
    memcpy(&v, rec + off + 8 * c, 8);
    return v;
  }
  float v;
  memcpy(&v, rec + off + 4 * c, 4);
  return (double)v;
}

// RNE(RNE32(v) * scale) in format dt, written at element k of p
void put(char* p, int dt, size_t k, double v, float scale) {
  float q = (float)v * scale;
  if (dt == SPH_F32) {
    memcpy(p + 4 * k, &q, 4);
  } else if (dt == SPH_F16) {
    _Float16 h = (_Float16)q;
    memcpy(p + 2 * k, &h, 2);
  } else {
    __bf16 b = (__bf16)q;
    memcpy(p + 2 * k, &b, 2);
  }
}

int axis_cell(double xw, int n_c) {
  double t = std::floor(xw * (double)n_c);
  if (!(t == t)) return 0;
  return (int)std::min(std::max(t, 0.0), (double)(n_c - 1));
}

template <class F>
void parallel_for(int nthreads, int64_t n, F&& f) {
  if (nthreads <= 1 || n < 4096) {
    f(0, (int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
    th.emplace_back([&f, t, lo, hi] { f(t, lo, hi); });
  }
  for (auto& x : th) x.join();
}

// Cell list of the host records: FP64 cell ids (same definition as the
// device binning), stable order by (cell, input index), and the largest h
// of each cell (as stored, read as FP32; positive values only, 0 for a cell
// without any) when hmax is non-NULL.
void bin_host(const char* aos, const sph_aos_layout& L, int n, int n_c, int nthreads,
              int32_t* start, int32_t* perm, int32_t* cell, float* hmax) {
  const int C = n_c * n_c * n_c;
  const int T = (n < 4096) ? 1 : nthreads;
  const bool want_hmax = hmax != nullptr && L.offset[SPH_A_H] != SPH_ABSENT;
  std::vector<int32_t> cid((size_t)std::max(n, 1));
  std::vector<int32_t> hist((size_t)T * C, 0);
  std::vector<float> hm(want_hmax ? (size_t)T * C : 0, 0.0f);
  // 1. cell ids and per-thread histograms over contiguous input ranges
  parallel_for(T, n, [&](int t, int64_t lo, int64_t hi) {
    int32_t* h = hist.data() + (size_t)t * C;
    for (int64_t i = lo; i < hi; ++i) {
      const char* rec = aos + (size_t)i * L.stride;
      int c3[3];
      for (int a = 0; a < 3; ++a) {
        double x = rec_d(rec, L.offset[SPH_A_X], SPH_F64, a);
        c3[a] = axis_cell(x - std::floor(x), n_c);
      }
      int c = c3[0] + n_c * (c3[1] + n_c * c3[2]);
      cid[(size_t)i] = c;
      h[c]++;
      if (want_hmax) {
        const float hv = (float)rec_d(rec, L.offset[SPH_A_H], L.dtype[SPH_A_H]);
        float& m = hm[(size_t)t * C + c];
        if (hv > 0.0f && hv > m) m = hv;
      }
    }
  });
  if (hmax && !want_hmax) std::fill(hmax, hmax + C, 0.0f);
  if (want_hmax) {
    for (int c = 0; c < C; ++c) {
      float m = 0.0f;
      for (int t = 0; t < T; ++t) m = std::max(m, hm[(size_t)t * C + c]);
      hmax[c] = m;
    }
  }
  // 2. stable positions: cell-major, then thread (input range) order
  int32_t run = 0;
  for (int c = 0; c < C; ++c) {
    start[c] = run;
    for (int t = 0; t < T; ++t) {
      int32_t v = hist[(size_t)t * C + c];
      hist[(size_t)t * C + c] = run;
      run += v;
    }
  }
  start[C] = run;
  parallel_for(T, n, [&](int t, int64_t lo, int64_t hi) {
    int32_t* h = hist.data() + (size_t)t * C;
    for (int64_t i = lo; i < hi; ++i) {
      int c = cid[(size_t)i];
      int32_t pos = h[c]++;
      perm[pos] = (int32_t)i;
      cell[pos] = c;
    }
  });
}

// Gather and quantise the view's fields in slot order into the staging
// areas of the plan (the FORCE_IN / KICK_IN extras are FP32 copies).
void gather_host(const char* aos, const sph_aos_layout& L, int n, int n_c, const int32_t* perm,
                 const int32_t* cell, const Plan& pl, const sph_precision& prec, char* st,
                 int nthreads) {
  const float sm = std::ldexp(1.0f, prec.scale_m), sh = std::ldexp(1.0f, prec.scale_h),
              su = std::ldexp(1.0f, prec.scale_u);
  const int dens_f[4] = {SPH_A_RHO, SPH_A_F, SPH_A_P, SPH_A_C};
  parallel_for(nthreads, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t k = lo; k < hi; ++k) {
      const char* rec = aos + (size_t)perm[k] * L.stride;
      double xw[3];
      for (int a = 0; a < 3; ++a) {
        double x = rec_d(rec, L.offset[SPH_A_X], SPH_F64, a);
        xw[a] = x - std::floor(x);
      }
      int c = cell[k];
      int c3[3] = {c % n_c, (c / n_c) % n_c, c / (n_c * n_c)};
      if (pl.pair) {
        int code = 0;
        for (int a = 0; a < 3; ++a) {
          int sa;
          float off = anchor_offset(xw[a], c3[a], n_c, prec.pos_anchor, sa);
          put(st + pl.off_pos[a], prec.pos, (size_t)k, (double)off, 1.0f);
          code |= sa << (2 * a);
        }
        if (pl.anc) reinterpret_cast<uint8_t*>(st + pl.off_anc)[k] = (uint8_t)code;
        put(st + pl.off_m, prec.mhu, (size_t)k, rec_d(rec, L.offset[SPH_A_M], L.dtype[SPH_A_M]), sm);
        put(st + pl.off_h, prec.mhu, (size_t)k, rec_d(rec, L.offset[SPH_A_H], L.dtype[SPH_A_H]), sh);
      }
      if (pl.u)
        put(st + pl.off_u, prec.mhu, (size_t)k, rec_d(rec, L.offset[SPH_A_U], L.dtype[SPH_A_U]), su);
      if (pl.vq)
        for (int a = 0; a < 3; ++a)
          put(st + pl.off_vq[a], prec.vel, (size_t)k, rec_d(rec, L.offset[SPH_A_V], L.dtype[SPH_A_V], a),
              1.0f);
      if (pl.kick) {
        for (int a = 0; a < 3; ++a) {
          reinterpret_cast<double*>(st + pl.off_x[a])[k] = xw[a];
          reinterpret_cast<float*>(st + pl.off_v[a])[k] =
              (float)rec_d(rec, L.offset[SPH_A_V], L.dtype[SPH_A_V], a);
        }
        reinterpret_cast<float*>(st + pl.off_uk)[k] = (float)rec_d(rec, L.offset[SPH_A_U], L.dtype[SPH_A_U]);
      }
      if (pl.dens_in)
        for (int q = 0; q < 4; ++q)
          reinterpret_cast<float*>(st + pl.off_dens[q])[k] =
              (float)rec_d(rec, L.offset[dens_f[q]], L.dtype[dens_f[q]]);
      if (pl.acc_in) {
        for (int a = 0; a < 3; ++a)
          reinterpret_cast<float*>(st + pl.off_acc[a])[k] =
              (float)rec_d(rec, L.offset[SPH_A_A], L.dtype[SPH_A_A], a);
        reinterpret_cast<float*>(st + pl.off_acc[3])[k] =
            (float)rec_d(rec, L.offset[SPH_A_DU], L.dtype[SPH_A_DU]);
      }
    }
  });
}

struct Cp {
  void* dev;
  size_t off, bytes;
};

// the view's device arrays and their staging areas
std::vector<Cp> view_copies(const Plan& pl, const sph_soa& out, int n, const sph_precision& prec) {
  std::vector<Cp> cps;
  for (int a = 0; a < 3; ++a) {
    if (pl.pair) cps.push_back({out.f[SPH_S_OFF_X + a], pl.off_pos[a], (size_t)n * esz(prec.pos)});
    if (pl.vq) cps.push_back({out.f[SPH_S_VQ_X + a], pl.off_vq[a], (size_t)n * esz(prec.vel)});
    if (pl.kick) {
      cps.push_back({out.f[SPH_S_X_X + a], pl.off_x[a], (size_t)n * 8});
      cps.push_back({out.f[SPH_S_V_X + a], pl.off_v[a], (size_t)n * 4});
    }
  }
  if (pl.anc) cps.push_back({out.f[SPH_S_ANC], pl.off_anc, (size_t)n});
  if (pl.pair) {
    cps.push_back({out.f[SPH_S_M], pl.off_m, (size_t)n * esz(prec.mhu)});
    cps.push_back({out.f[SPH_S_H], pl.off_h, (size_t)n * esz(prec.mhu)});
  }
  if (pl.u) cps.push_back({out.f[SPH_S_U], pl.off_u, (size_t)n * esz(prec.mhu)});
  if (pl.kick) cps.push_back({out.f[SPH_S_UK], pl.off_uk, (size_t)n * 4});
  const int dens_s[4] = {SPH_S_RHO, SPH_S_F, SPH_S_P, SPH_S_C};
  const int acc_s[4] = {SPH_S_A_X, SPH_S_A_Y, SPH_S_A_Z, SPH_S_DU};
  for (int q = 0; q < 4; ++q) {
    if (pl.dens_in) cps.push_back({out.f[dens_s[q]], pl.off_dens[q], (size_t)n * 4});
    if (pl.acc_in) cps.push_back({out.f[acc_s[q]], pl.off_acc[q], (size_t)n * 4});
  }
  return cps;
}

// argument checks shared by sph_convert_host and sph_gather_host
sph_status check_gather(const char* fn, const void* aos_host, const sph_aos_layout* layout, int n,
                        int n_c, int view, const sph_precision* prec, const sph_soa* out,
                        const void* staging_host) {
  std::string f(fn);
  if (!layout || !prec || !out || !staging_host)
    return host_fail(SPH_E_INVALID, (f + ": NULL argument").c_str());
  if (!known_view(view)) return host_fail(SPH_E_INVALID, (f + ": unknown view").c_str());
  if (n < 0 || n_c < 3 || n_c > 1290) return host_fail(SPH_E_RANGE, (f + ": bad n or n_c").c_str());
  if (n > 0 && !aos_host) return host_fail(SPH_E_INVALID, (f + ": aos_host is NULL").c_str());
  if (prec->pos_anchor < SPH_ANCHOR_CORNER || prec->pos_anchor > SPH_ANCHOR_SUB(2) ||
      prec->reserved != 0)
    return host_fail(SPH_E_INVALID, (f + ": bad precision pos_anchor or reserved").c_str());
  const int fmt[3] = {prec->pos, prec->vel, prec->mhu};
  for (int q : fmt) {
    if (q >= SPH_TRUNC + 9 && q <= SPH_TRUNC + 32)
      return host_fail(SPH_E_UNSUPPORTED,
                       (f + ": truncated storage is written by sph_convert only").c_str());
    if (q != SPH_F32 && q != SPH_F16 && q != SPH_BF16)
      return host_fail(SPH_E_INVALID, (f + ": bad precision format").c_str());
  }
  const sph_aos_layout& L = *layout;
  if (L.stride == 0 || L.offset[SPH_A_X] == SPH_ABSENT || L.dtype[SPH_A_X] != SPH_F64)
    return host_fail(SPH_E_INVALID, (f + ": layout needs an FP64 X field").c_str());
  const Plan pl = plan(n, n_c, view, *prec);
  auto needf = [&](int q) { return L.offset[q] != SPH_ABSENT; };
  if ((pl.pair && (!needf(SPH_A_M) || !needf(SPH_A_H))) || ((pl.vq || pl.kick) && !needf(SPH_A_V)) ||
      ((pl.u || pl.kick) && !needf(SPH_A_U)) ||
      (pl.dens_in && (!needf(SPH_A_RHO) || !needf(SPH_A_F) || !needf(SPH_A_P) || !needf(SPH_A_C))) ||
      (pl.acc_in && (!needf(SPH_A_A) || !needf(SPH_A_DU))))
    return host_fail(SPH_E_INVALID, (f + ": layout lacks a field of the view").c_str());
  for (const Cp& c : view_copies(pl, *out, n, *prec))
    if (!c.dev) return host_fail(SPH_E_INVALID, (f + ": soa view field is NULL").c_str());
  return SPH_OK;
}

sph_status enqueue_h2d(const char* fn, const std::vector<Cp>& cps, const char* st,
                       hipStream_t stream) {
  for (const Cp& c : cps) {
    if (c.bytes == 0) continue;
    hipError_t e = hipMemcpyAsync(c.dev, st + c.off, c.bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
      std::string m = std::string(fn) + ": hipMemcpyAsync failed: " + hipGetErrorString(e);
      return host_fail(SPH_E_HIP, m.c_str());
    }
  }
  return SPH_OK;
}

// Host writeback of a view (the fields of sph_writeback): staging layout
// and the device arrays it comes from.
struct WbField {
  int soa, rec, comp;   // SoA field, record field, component
  int kind;             // 0 FP32 value, 1 int32, 2 FP64 position
};

std::vector<WbField> wb_fields(int view) {
  std::vector<WbField> w;
  if (view == SPH_VIEW_KICK) {
    for (int a = 0; a < 3; ++a) w.push_back({SPH_S_X_X + a, SPH_A_X, a, 2});
    for (int a = 0; a < 3; ++a) w.push_back({SPH_S_V_X + a, SPH_A_V, a, 0});
    w.push_back({SPH_S_UK, SPH_A_U, 0, 0});
  } else if (view == SPH_VIEW_DENSITY) {
    w.push_back({SPH_S_RHO, SPH_A_RHO, 0, 0});
    w.push_back({SPH_S_WCOUNT, SPH_A_WCOUNT, 0, 0});
    w.push_back({SPH_S_RHO_DH, SPH_A_RHO_DH, 0, 0});
    w.push_back({SPH_S_F, SPH_A_F, 0, 0});
    w.push_back({SPH_S_P, SPH_A_P, 0, 0});
    w.push_back({SPH_S_C, SPH_A_C, 0, 0});
    w.push_back({SPH_S_NNGB, SPH_A_NNGB, 0, 1});
  } else if (view == SPH_VIEW_FORCE) {
    for (int a = 0; a < 3; ++a) w.push_back({SPH_S_A_X + a, SPH_A_A, a, 0});
    w.push_back({SPH_S_DU, SPH_A_DU, 0, 0});
    w.push_back({SPH_S_VSIG, SPH_A_VSIG, 0, 0});
    w.push_back({SPH_S_NFORCE, SPH_A_NFORCE, 0, 1});
  }
  return w;
}

size_t wb_bytes(int n, const std::vector<WbField>& w) {
  size_t b = 0;
  for (const WbField& f : w) b += al256((size_t)n * (f.kind == 2 ? 8 : 4));
  return b;
}

}  // namespace

extern "C" {

sph_status sph_host_staging_size(int32_t n, int32_t n_c, int32_t view, const sph_precision* prec,
                                 size_t* bytes) {
  if (!bytes || !prec) return host_fail(SPH_E_INVALID, "sph_host_staging_size: NULL argument");
  if (n < 0) return host_fail(SPH_E_INVALID, "sph_host_staging_size: n is negative");
  if (n_c < 3 || n_c > 1290) return host_fail(SPH_E_RANGE, "sph_host_staging_size: n_c out of range");
  if (!known_view(view)) return host_fail(SPH_E_INVALID, "sph_host_staging_size: unknown view");
  *bytes = plan(n, n_c, view, *prec).total;
  return SPH_OK;
}

sph_status sph_convert_host(const void* aos_host, const sph_aos_layout* layout,
                            const sph_cells* cells, int32_t view, const sph_precision* prec,
                            const sph_soa* out, void* staging_host, size_t staging_bytes,
                            int32_t nthreads, hipStream_t stream) {
  if (!cells) return host_fail(SPH_E_INVALID, "sph_convert_host: NULL argument");
  const int n = cells->n, n_c = cells->n_c;
  if (!cells->cell_start || !cells->perm || !cells->cell)
    return host_fail(SPH_E_INVALID, "sph_convert_host: cell list pointers are NULL");
  if (cells->sub_bits != 0)
    return host_fail(SPH_E_UNSUPPORTED,
                     "sph_convert_host: sub-cell order (sub_bits > 0) is built by sph_bin only");
  sph_status st0 = check_gather("sph_convert_host", aos_host, layout, n, n_c, view, prec, out,
                                staging_host);
  if (st0 != SPH_OK) return st0;
  const Plan pl = plan(n, n_c, view, *prec);
  if (staging_bytes < pl.total) return host_fail(SPH_E_NOMEM, "sph_convert_host: staging too small");
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  char* st = static_cast<char*>(staging_host);
  const char* aos = static_cast<const char*>(aos_host);
  const int C = n_c * n_c * n_c;
  int32_t* start = reinterpret_cast<int32_t*>(st + pl.off_start);
  int32_t* perm = reinterpret_cast<int32_t*>(st + pl.off_perm);
  int32_t* cell = reinterpret_cast<int32_t*>(st + pl.off_cell);
  const bool want_hmax = cells->hmax != nullptr && layout->offset[SPH_A_H] != SPH_ABSENT;
  bin_host(aos, *layout, n, n_c, nthreads, start, perm, cell,
           want_hmax ? reinterpret_cast<float*>(st + pl.off_hmax) : nullptr);
  gather_host(aos, *layout, n, n_c, perm, cell, pl, *prec, st, nthreads);
  // H2D copies on the caller's stream (operator M)
  std::vector<Cp> cps = {{cells->cell_start, pl.off_start, 4 * ((size_t)C + 1)},
                         {cells->perm, pl.off_perm, 4 * (size_t)n},
                         {cells->cell, pl.off_cell, 4 * (size_t)n}};
  if (want_hmax) cps.push_back({cells->hmax, pl.off_hmax, 4 * (size_t)C});
  for (const Cp& c : view_copies(pl, *out, n, *prec)) cps.push_back(c);
  return enqueue_h2d("sph_convert_host", cps, st, stream);
}

sph_status sph_bin_host(const void* aos_host, const sph_aos_layout* layout, int32_t n, int32_t n_c,
                        int32_t* cell_start, int32_t* perm, int32_t* cell, float* hmax,
                        int32_t nthreads) {
  if (!layout || !cell_start || (n > 0 && (!aos_host || !perm || !cell)))
    return host_fail(SPH_E_INVALID, "sph_bin_host: NULL argument");
  if (n < 0 || n_c < 3 || n_c > 1290) return host_fail(SPH_E_RANGE, "sph_bin_host: bad n or n_c");
  if (layout->stride == 0 || layout->offset[SPH_A_X] == SPH_ABSENT ||
      layout->dtype[SPH_A_X] != SPH_F64)
    return host_fail(SPH_E_INVALID, "sph_bin_host: layout needs an FP64 X field");
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  bin_host(static_cast<const char*>(aos_host), *layout, n, n_c, nthreads, cell_start, perm, cell,
           hmax);
  return SPH_OK;
}

sph_status sph_gather_host(const void* aos_host, const sph_aos_layout* layout, int32_t n,
                           int32_t n_c, const int32_t* perm, const int32_t* cell, int32_t view,
                           const sph_precision* prec, const sph_soa* out, void* staging_host,
                           size_t staging_bytes, int32_t nthreads, hipStream_t stream) {
  sph_status st0 = check_gather("sph_gather_host", aos_host, layout, n, n_c, view, prec, out,
                                staging_host);
  if (st0 != SPH_OK) return st0;
  if (n > 0 && (!perm || !cell)) return host_fail(SPH_E_INVALID, "sph_gather_host: NULL cell list");
  const Plan pl = plan(n, n_c, view, *prec);
  if (staging_bytes < pl.total) return host_fail(SPH_E_NOMEM, "sph_gather_host: staging too small");
  const int C = n_c * n_c * n_c;
  for (int32_t k = 0; k < n; ++k)   // the gather indexes records and cells with these
    if (perm[k] < 0 || perm[k] >= n || cell[k] < 0 || cell[k] >= C)
      return host_fail(SPH_E_RANGE, "sph_gather_host: perm or cell entry out of range");
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  char* st = static_cast<char*>(staging_host);
  gather_host(static_cast<const char*>(aos_host), *layout, n, n_c, perm, cell, pl, *prec, st,
              nthreads);
  return enqueue_h2d("sph_gather_host", view_copies(pl, *out, n, *prec), st, stream);
}

sph_status sph_writeback_host_size(int32_t n, int32_t view, size_t* bytes) {
  if (!bytes) return host_fail(SPH_E_INVALID, "sph_writeback_host_size: NULL argument");
  if (n < 0) return host_fail(SPH_E_INVALID, "sph_writeback_host_size: n is negative");
  if (view != SPH_VIEW_DENSITY && view != SPH_VIEW_FORCE && view != SPH_VIEW_KICK)
    return host_fail(SPH_E_INVALID, "sph_writeback_host_size: view must be DENSITY, FORCE or KICK");
  *bytes = wb_bytes(n, wb_fields(view));
  return SPH_OK;
}

sph_status sph_writeback_host(const sph_soa* soa, int32_t n, const int32_t* perm, int32_t view,
                              void* aos_host, const sph_aos_layout* layout, void* staging_host,
                              size_t staging_bytes, int32_t nthreads, hipStream_t stream) {
  if (!soa || !layout || !staging_host || (n > 0 && (!perm || !aos_host)))
    return host_fail(SPH_E_INVALID, "sph_writeback_host: NULL argument");
  if (n < 0) return host_fail(SPH_E_INVALID, "sph_writeback_host: n is negative");
  if (view != SPH_VIEW_DENSITY && view != SPH_VIEW_FORCE && view != SPH_VIEW_KICK)
    return host_fail(SPH_E_INVALID, "sph_writeback_host: view must be DENSITY, FORCE or KICK");
  const sph_aos_layout& L = *layout;
  if (L.stride == 0) return host_fail(SPH_E_INVALID, "sph_writeback_host: layout stride is 0");
  const std::vector<WbField> w = wb_fields(view);
  if (staging_bytes < wb_bytes(n, w)) return host_fail(SPH_E_NOMEM, "sph_writeback_host: staging too small");
  for (const WbField& f : w) {
    if (!soa->f[f.soa]) return host_fail(SPH_E_INVALID, "sph_writeback_host: soa field is NULL");
    if (L.offset[f.rec] == SPH_ABSENT && f.kind == 2)
      return host_fail(SPH_E_INVALID, "sph_writeback_host: layout needs an FP64 X field");
  }
  if (L.offset[SPH_A_X] != SPH_ABSENT && L.dtype[SPH_A_X] != SPH_F64)
    return host_fail(SPH_E_INVALID, "sph_writeback_host: layout needs an FP64 X field");
  for (int32_t k = 0; k < n; ++k)
    if (perm[k] < 0 || perm[k] >= n)
      return host_fail(SPH_E_RANGE, "sph_writeback_host: perm entry out of range");
  // D2H copies into the staging, then the scatter into the records
  char* st = static_cast<char*>(staging_host);
  std::vector<size_t> off;
  size_t o = 0;
  for (const WbField& f : w) {
    off.push_back(o);
    const size_t b = (size_t)n * (f.kind == 2 ? 8 : 4);
    if (b) {
      hipError_t e = hipMemcpyAsync(st + o, soa->f[f.soa], b, hipMemcpyDeviceToHost, stream);
      if (e != hipSuccess)
        return host_fail(SPH_E_HIP, (std::string("sph_writeback_host: hipMemcpyAsync failed: ") +
                                     hipGetErrorString(e)).c_str());
    }
    o += al256(b);
  }
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess)
    return host_fail(SPH_E_HIP, (std::string("sph_writeback_host: stream failed: ") +
                                 hipGetErrorString(e)).c_str());
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  char* aos = static_cast<char*>(aos_host);
  parallel_for(nthreads, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t k = lo; k < hi; ++k) {
      char* rec = aos + (size_t)perm[k] * L.stride;
      for (size_t q = 0; q < w.size(); ++q) {
        const WbField& f = w[q];
        const uint32_t ro = L.offset[f.rec];
        if (ro == SPH_ABSENT) continue;
        const char* src = st + off[q];
        if (f.kind == 2) {
          memcpy(rec + ro + 8 * f.comp, src + 8 * k, 8);
        } else if (f.kind == 1) {
          memcpy(rec + ro, src + 4 * k, 4);
        } else {
          float v;
          memcpy(&v, src + 4 * k, 4);
          if (L.dtype[f.rec] == SPH_F64) {
            double d = (double)v;
            memcpy(rec + ro + 8 * f.comp, &d, 8);
          } else {
            memcpy(rec + ro + 4 * f.comp, &v, 4);
          }
        }
      }
    }
  });
  return SPH_OK;
}

}  // extern "C"
