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
  size_t off_pos[3], off_vq[3], off_m, off_h, off_u, off_x[3], off_v[3], off_uk;
  size_t total;
  bool pair, kick, vq, u;
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
  pl.pair = view != SPH_VIEW_KICK;
  pl.kick = view == SPH_VIEW_KICK || view == SPH_VIEW_FULL;
  pl.vq = view == SPH_VIEW_FORCE || view == SPH_VIEW_FULL;
  pl.u = view == SPH_VIEW_DENSITY || view == SPH_VIEW_FULL;
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
  pl.off_m = pl.pair ? take((size_t)n * esz(p.mhu)) : 0;
  pl.off_h = pl.pair ? take((size_t)n * esz(p.mhu)) : 0;
  pl.off_u = pl.u ? take((size_t)n * esz(p.mhu)) : 0;
  pl.off_uk = pl.kick ? take((size_t)n * 4) : 0;
  pl.total = o;
  return pl;
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

}  // namespace

extern "C" {

sph_status sph_host_staging_size(int32_t n, int32_t n_c, int32_t view, const sph_precision* prec,
                                 size_t* bytes) {
  if (!bytes || !prec) return host_fail(SPH_E_INVALID, "sph_host_staging_size: NULL argument");
  if (n < 0) return host_fail(SPH_E_INVALID, "sph_host_staging_size: n is negative");
  if (n_c < 3 || n_c > 1290) return host_fail(SPH_E_RANGE, "sph_host_staging_size: n_c out of range");
  if (view < SPH_VIEW_DENSITY || view > SPH_VIEW_FULL)
    return host_fail(SPH_E_INVALID, "sph_host_staging_size: unknown view");
  *bytes = plan(n, n_c, view, *prec).total;
  return SPH_OK;
}

sph_status sph_convert_host(const void* aos_host, const sph_aos_layout* layout,
                            const sph_cells* cells, int32_t view, const sph_precision* prec,
                            const sph_soa* out, void* staging_host, size_t staging_bytes,
                            int32_t nthreads, hipStream_t stream) {
  if (!layout || !cells || !prec || !out || !staging_host)
    return host_fail(SPH_E_INVALID, "sph_convert_host: NULL argument");
  if (view < SPH_VIEW_DENSITY || view > SPH_VIEW_FULL)
    return host_fail(SPH_E_INVALID, "sph_convert_host: unknown view");
  const int n = cells->n, n_c = cells->n_c;
  if (n < 0 || n_c < 3 || n_c > 1290) return host_fail(SPH_E_RANGE, "sph_convert_host: bad n or n_c");
  if (n > 0 && !aos_host) return host_fail(SPH_E_INVALID, "sph_convert_host: aos_host is NULL");
  if (!cells->cell_start || !cells->perm || !cells->cell)
    return host_fail(SPH_E_INVALID, "sph_convert_host: cell list pointers are NULL");
  if (cells->sub_bits != 0)
    return host_fail(SPH_E_UNSUPPORTED,
                     "sph_convert_host: sub-cell order (sub_bits > 0) is built by sph_bin only");
  const int fmt[3] = {prec->pos, prec->vel, prec->mhu};
  for (int f : fmt) {
    if (f >= SPH_TRUNC + 9 && f <= SPH_TRUNC + 32)
      return host_fail(SPH_E_UNSUPPORTED,
                       "sph_convert_host: truncated storage is written by sph_convert only");
    if (f != SPH_F32 && f != SPH_F16 && f != SPH_BF16)
      return host_fail(SPH_E_INVALID, "sph_convert_host: bad precision format");
  }
  const sph_aos_layout& L = *layout;
  if (L.stride == 0 || L.offset[SPH_A_X] == SPH_ABSENT || L.dtype[SPH_A_X] != SPH_F64)
    return host_fail(SPH_E_INVALID, "sph_convert_host: layout needs an FP64 X field");
  Plan pl = plan(n, n_c, view, *prec);
  if (staging_bytes < pl.total) return host_fail(SPH_E_NOMEM, "sph_convert_host: staging too small");
  auto needf = [&](int f) { return L.offset[f] != SPH_ABSENT; };
  if ((pl.pair && (!needf(SPH_A_M) || !needf(SPH_A_H))) || ((pl.vq || pl.kick) && !needf(SPH_A_V)) ||
      ((pl.u || pl.kick) && !needf(SPH_A_U)))
    return host_fail(SPH_E_INVALID, "sph_convert_host: layout lacks a field of the view");
  auto req = [&](int f) { return out->f[f] != nullptr; };
  for (int a = 0; a < 3; ++a) {
    if ((pl.pair && !req(SPH_S_OFF_X + a)) || (pl.vq && !req(SPH_S_VQ_X + a)) ||
        (pl.kick && (!req(SPH_S_X_X + a) || !req(SPH_S_V_X + a))))
      return host_fail(SPH_E_INVALID, "sph_convert_host: soa view field is NULL");
  }
  if ((pl.pair && (!req(SPH_S_M) || !req(SPH_S_H))) || (pl.u && !req(SPH_S_U)) ||
      (pl.kick && !req(SPH_S_UK)))
    return host_fail(SPH_E_INVALID, "sph_convert_host: soa view field is NULL");

  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  char* st = static_cast<char*>(staging_host);
  const char* aos = static_cast<const char*>(aos_host);
  const int C = n_c * n_c * n_c;
  int32_t* start = reinterpret_cast<int32_t*>(st + pl.off_start);
  int32_t* perm = reinterpret_cast<int32_t*>(st + pl.off_perm);
  int32_t* cell = reinterpret_cast<int32_t*>(st + pl.off_cell);

  // 1. cell ids (FP64, same definition as the device binning) and
  //    per-thread histograms over contiguous input ranges
  //    and per-thread largest h of each cell (h as stored, read as FP32;
  //    positive values only, 0 for a cell without any)
  const int T = (n < 4096) ? 1 : nthreads;
  const bool want_hmax = cells->hmax != nullptr && L.offset[SPH_A_H] != SPH_ABSENT;
  std::vector<int32_t> cid((size_t)std::max(n, 1));
  std::vector<int32_t> hist((size_t)T * C, 0);
  std::vector<float> hm(want_hmax ? (size_t)T * C : 0, 0.0f);
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
  float* hmax = reinterpret_cast<float*>(st + pl.off_hmax);
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
  // 3. gather and quantise the view in slot order
  const float sm = std::ldexp(1.0f, prec->scale_m), sh = std::ldexp(1.0f, prec->scale_h),
              su = std::ldexp(1.0f, prec->scale_u);
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
        for (int a = 0; a < 3; ++a) {
          float off = (float)(xw[a] - (double)c3[a] / (double)n_c);
          put(st + pl.off_pos[a], prec->pos, (size_t)k, (double)off, 1.0f);
        }
        put(st + pl.off_m, prec->mhu, (size_t)k, rec_d(rec, L.offset[SPH_A_M], L.dtype[SPH_A_M]), sm);
        put(st + pl.off_h, prec->mhu, (size_t)k, rec_d(rec, L.offset[SPH_A_H], L.dtype[SPH_A_H]), sh);
      }
      if (pl.u)
        put(st + pl.off_u, prec->mhu, (size_t)k, rec_d(rec, L.offset[SPH_A_U], L.dtype[SPH_A_U]), su);
      if (pl.vq)
        for (int a = 0; a < 3; ++a)
          put(st + pl.off_vq[a], prec->vel, (size_t)k, rec_d(rec, L.offset[SPH_A_V], L.dtype[SPH_A_V], a),
              1.0f);
      if (pl.kick) {
        for (int a = 0; a < 3; ++a) {
          reinterpret_cast<double*>(st + pl.off_x[a])[k] = xw[a];
          reinterpret_cast<float*>(st + pl.off_v[a])[k] =
              (float)rec_d(rec, L.offset[SPH_A_V], L.dtype[SPH_A_V], a);
        }
        reinterpret_cast<float*>(st + pl.off_uk)[k] = (float)rec_d(rec, L.offset[SPH_A_U], L.dtype[SPH_A_U]);
      }
    }
  });
  // 4. H2D copies on the caller's stream (operator M)
  struct Cp {
    void* dst;
    size_t off, bytes;
  };
  std::vector<Cp> cps = {{cells->cell_start, pl.off_start, 4 * ((size_t)C + 1)},
                         {cells->perm, pl.off_perm, 4 * (size_t)n},
                         {cells->cell, pl.off_cell, 4 * (size_t)n}};
  if (want_hmax) cps.push_back({cells->hmax, pl.off_hmax, 4 * (size_t)C});
  for (int a = 0; a < 3; ++a) {
    if (pl.pair) cps.push_back({out->f[SPH_S_OFF_X + a], pl.off_pos[a], (size_t)n * esz(prec->pos)});
    if (pl.vq) cps.push_back({out->f[SPH_S_VQ_X + a], pl.off_vq[a], (size_t)n * esz(prec->vel)});
    if (pl.kick) {
      cps.push_back({out->f[SPH_S_X_X + a], pl.off_x[a], (size_t)n * 8});
      cps.push_back({out->f[SPH_S_V_X + a], pl.off_v[a], (size_t)n * 4});
    }
  }
  if (pl.pair) {
    cps.push_back({out->f[SPH_S_M], pl.off_m, (size_t)n * esz(prec->mhu)});
    cps.push_back({out->f[SPH_S_H], pl.off_h, (size_t)n * esz(prec->mhu)});
  }
  if (pl.u) cps.push_back({out->f[SPH_S_U], pl.off_u, (size_t)n * esz(prec->mhu)});
  if (pl.kick) cps.push_back({out->f[SPH_S_UK], pl.off_uk, (size_t)n * 4});
  for (const Cp& c : cps) {
    if (c.bytes == 0) continue;
    hipError_t e = hipMemcpyAsync(c.dst, st + c.off, c.bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
      std::string m = std::string("sph_convert_host: hipMemcpyAsync failed: ") + hipGetErrorString(e);
      return host_fail(SPH_E_HIP, m.c_str());
    }
  }
  return SPH_OK;
}

}  // extern "C"
