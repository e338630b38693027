// Host entry points of libsphmi: argument validation, conversion of the ABI
// structs to the kernels' parameter blocks, HIP error mapping and the
// thread-local last-error message. Nothing here allocates device memory.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "sph_internal.h"

using namespace sph;

namespace {

thread_local std::string g_err;

sph_status fail(sph_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
sph_status fail(sph_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

sph_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return SPH_OK;
  return fail(SPH_E_HIP, "%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
}

bool is_float_dt(int dt) { return dt == SPH_F32 || dt == SPH_F64; }
bool is_store_dt(int dt) {
  return dt == SPH_F32 || dt == SPH_F16 || dt == SPH_BF16 || is_trunc(dt);
}

int elem_size(int dt) {
  switch (dt) {
    case SPH_F64: return 8;
    case SPH_F32: return 4;
    case SPH_F16:
    case SPH_BF16: return 2;
    case SPH_I32: return 4;
    default: return 0;
  }
}

int field_comps(int f) { return (f == SPH_A_X || f == SPH_A_V || f == SPH_A_A) ? 3 : 1; }
bool field_is_int(int f) { return f == SPH_A_NNGB || f == SPH_A_NFORCE || f == SPH_A_CELL; }

const char* aos_field_name(int f) {
  static const char* names[SPH_A_NFIELDS] = {"X", "V", "A", "M", "H", "U", "RHO", "P", "C",
                                             "DU", "RHO_DH", "WCOUNT", "F", "VSIG", "NNGB",
                                             "NFORCE", "CELL"};
  return (f >= 0 && f < SPH_A_NFIELDS) ? names[f] : "?";
}

// Validate the layout; `need` is a bitmask of fields that must be present.
sph_status check_layout(const sph_aos_layout* l, uint32_t need, AosLayout& out) {
  if (!l) return fail(SPH_E_INVALID, "layout is NULL");
  if (l->stride == 0 || l->stride % 8 != 0)
    return fail(SPH_E_INVALID, "layout stride %u must be a positive multiple of 8", l->stride);
  out.stride = l->stride;
  for (int f = 0; f < SPH_A_NFIELDS; ++f) {
    out.off[f] = l->offset[f];
    out.dt[f] = l->dtype[f];
    if (l->offset[f] == SPH_ABSENT) {
      if (need & (1u << f)) return fail(SPH_E_INVALID, "layout lacks field %s", aos_field_name(f));
      continue;
    }
    int dt = l->dtype[f];
    if (f == SPH_A_X && dt != SPH_F64)
      return fail(SPH_E_INVALID, "layout field X must be SPH_F64");
    if (field_is_int(f) ? dt != SPH_I32 : !is_float_dt(dt))
      return fail(SPH_E_INVALID, "layout field %s has unsupported dtype %d", aos_field_name(f), dt);
    uint64_t size = (uint64_t)elem_size(dt) * (uint64_t)field_comps(f);
    if ((uint64_t)l->offset[f] + size > l->stride)
      return fail(SPH_E_INVALID, "layout field %s exceeds the stride", aos_field_name(f));
    if (l->offset[f] % (uint32_t)elem_size(dt) != 0)
      return fail(SPH_E_INVALID, "layout field %s is misaligned", aos_field_name(f));
  }
  return SPH_OK;
}

constexpr uint32_t bit(int f) { return 1u << f; }

// AoS base pointers must be 8-byte aligned (records are moved as 8-byte words)
sph_status check_aos_ptr(const void* aos, int n) {
  if (n > 0 && !aos) return fail(SPH_E_INVALID, "aos is NULL");
  if (reinterpret_cast<uintptr_t>(aos) % 8 != 0) return fail(SPH_E_INVALID, "aos is not 8-byte aligned");
  return SPH_OK;
}

sph_status check_cells(const sph_cells* c, bool need_lists, CellsDev& out) {
  if (!c) return fail(SPH_E_INVALID, "cells is NULL");
  if (c->n < 0) return fail(SPH_E_INVALID, "cells->n = %d is negative", c->n);
  if (c->n_c < 3) return fail(SPH_E_RANGE, "cells->n_c = %d must be >= 3", c->n_c);
  if (c->n_c > 1290) return fail(SPH_E_RANGE, "cells->n_c = %d: n_c^3 overflows int32", c->n_c);
  if (c->sub_bits < 0 || c->sub_bits > 3)
    return fail(SPH_E_RANGE, "cells->sub_bits = %d must be in [0, 3]", c->sub_bits);
  if (c->reserved != 0) return fail(SPH_E_INVALID, "cells->reserved must be 0");
  const int64_t C = (int64_t)c->n_c * c->n_c * c->n_c;
  if ((C << (3 * c->sub_bits)) >= (1LL << 31))
    return fail(SPH_E_RANGE, "n_c^3 * 8^sub_bits must be < 2^31");
  if (need_lists && (!c->cell_start || !c->perm || !c->cell))
    return fail(SPH_E_INVALID, "cells->cell_start, perm and cell must be device pointers");
  if (need_lists && c->sub_bits > 0 && !c->sub_start)
    return fail(SPH_E_INVALID, "cells->sub_start is required when sub_bits > 0");
  out.n = c->n;
  out.n_c = c->n_c;
  out.sub_bits = c->sub_bits;
  out.start = c->cell_start;
  out.perm = c->perm;
  out.cell = c->cell;
  out.sub_start = c->sub_bits > 0 ? c->sub_start : c->cell_start;
  out.hmax = c->hmax;
  out.status = c->status;
  out.tally = reinterpret_cast<unsigned long long*>(c->tally);
  out.rebin = c->rebin;
  return SPH_OK;
}

// Merged work items (several sparse cells per item) need the cell ids to fit
// below the item's cell-count bits
sph_status check_merge(const sph_work* w, const CellsDev& c) {
  if (w->reserved != 0) return fail(SPH_E_INVALID, "work->reserved must be 0");
  if (w->max_cells < 0 || w->max_cells > kMaxMerge)
    return fail(SPH_E_INVALID, "work->max_cells = %d must be in [0, %d]", w->max_cells, kMaxMerge);
  if (w->max_cells > 1 && (int64_t)c.n_c * c.n_c * c.n_c >= ((int64_t)1 << kMergeShift))
    return fail(SPH_E_RANGE, "work->max_cells > 1 needs n_c^3 < 2^%d", kMergeShift);
  return SPH_OK;
}

// Work list of a launch over items with tile ti (NULL: one workgroup per cell)
sph_status check_work(const sph_work* w, const CellsDev& c, int ti, WorkDev& out, bool& use) {
  use = w != nullptr;
  if (!w) return SPH_OK;
  if (!w->buf) return fail(SPH_E_INVALID, "work->buf is NULL");
  if (w->ti != ti) return fail(SPH_E_INVALID, "work->ti = %d differs from the tile's ti = %d", w->ti, ti);
  if (w->sched < SPH_SCHED_GRID || w->sched > SPH_SCHED_DYNAMIC)
    return fail(SPH_E_INVALID, "work->sched = %d is not an SPH_SCHED_* value", w->sched);
  if (w->bytes < worklist_bytes(c.n, c.n_c, w->ti))
    return fail(SPH_E_NOMEM, "work->bytes %zu < %zu", w->bytes, worklist_bytes(c.n, c.n_c, w->ti));
  const sph_status st = check_merge(w, c);
  if (st != SPH_OK) return st;
  out = work_view(*w, c.n, c.n_c);
  return SPH_OK;
}

sph_status check_prec(const sph_precision* p, Prec& out) {
  if (!p) return fail(SPH_E_INVALID, "precision is NULL");
  if (!is_store_dt(p->pos) || !is_store_dt(p->vel) || !is_store_dt(p->mhu))
    return fail(SPH_E_INVALID,
                "precision formats must be SPH_F32, SPH_F16, SPH_BF16 or SPH_TRUNC_BITS(9..32)");
  const int32_t sc[3] = {p->scale_m, p->scale_h, p->scale_u};
  for (int q = 0; q < 3; ++q)
    if (sc[q] < -64 || sc[q] > 64) return fail(SPH_E_INVALID, "precision scale %d out of range", sc[q]);
  if (p->pos_anchor < SPH_ANCHOR_CORNER || p->pos_anchor > SPH_ANCHOR_SUB(2))
    return fail(SPH_E_INVALID, "precision pos_anchor %d is not SPH_ANCHOR_CORNER or SPH_ANCHOR_SUB(0..2)",
                p->pos_anchor);
  if (p->reserved != 0) return fail(SPH_E_INVALID, "precision reserved must be 0");
  out.pos = p->pos;
  out.vel = p->vel;
  out.mhu = p->mhu;
  out.anchor = p->pos_anchor;
  out.store_m = std::ldexp(1.0f, p->scale_m);
  out.store_h = std::ldexp(1.0f, p->scale_h);
  out.store_u = std::ldexp(1.0f, p->scale_u);
  out.load_m = std::ldexp(1.0f, -p->scale_m);
  out.load_h = std::ldexp(1.0f, -p->scale_h);
  out.load_u = std::ldexp(1.0f, -p->scale_u);
  return SPH_OK;
}

sph_status check_params(const sph_params* p, Phys& out) {
  if (!p) return fail(SPH_E_INVALID, "params is NULL");
  const double v[4] = {p->gamma_k, p->gamma, p->alpha, p->beta};
  for (double x : v)
    if (!std::isfinite(x)) return fail(SPH_E_INVALID, "params must be finite");
  if (!(p->gamma_k > 0.0)) return fail(SPH_E_INVALID, "params->gamma_k must be positive");
  out.gamma_k = (float)p->gamma_k;
  out.gamma = (float)p->gamma;
  out.alpha = (float)p->alpha;
  out.beta = (float)p->beta;
  out.gradh = p->gradh ? 1 : 0;
  if (p->kernel != SPH_KERNEL_M4 && p->kernel != SPH_KERNEL_WENDLAND_C2)
    return fail(SPH_E_INVALID, "params->kernel = %d is not a known kernel", p->kernel);
  out.kernel = p->kernel;
  return SPH_OK;
}

sph_status check_soa(const sph_soa* s, const int* fields, int nf, const char* what) {
  if (!s) return fail(SPH_E_INVALID, "%s: soa is NULL", what);
  for (int q = 0; q < nf; ++q)
    if (!s->f[fields[q]]) return fail(SPH_E_INVALID, "%s: soa field %d is NULL", what, fields[q]);
  return SPH_OK;
}

// Positions anchored at sub-cell centres of depth b >= 1 need the ANC codes
sph_status check_anchor(const sph_soa* s, const Prec& p, const char* what) {
  if (p.anchor >= SPH_ANCHOR_SUB(1) && !s->f[SPH_S_ANC])
    return fail(SPH_E_INVALID, "%s: soa field ANC is NULL (pos_anchor %d needs it)", what, p.anchor);
  return SPH_OK;
}

sph_status resolve_tile(sph_tile t, int& ti, int& k) {
  ti = t.ti;
  k = t.k;
  if (ti == 0 && k == 0) {
    ti = 64;
    k = 4;
  }
  if (!tile_supported(ti, k)) return fail(SPH_E_UNSUPPORTED, "tile {%d, %d} is not compiled in", ti, k);
  return SPH_OK;
}

#define SPH_TRY(x)                  \
  do {                              \
    sph_status _st = (x);           \
    if (_st != SPH_OK) return _st;  \
  } while (0)

const int kDensIn[] = {SPH_S_OFF_X, SPH_S_OFF_Y, SPH_S_OFF_Z, SPH_S_M, SPH_S_H, SPH_S_U,
                       SPH_S_RHO, SPH_S_WCOUNT, SPH_S_RHO_DH, SPH_S_F, SPH_S_P, SPH_S_C,
                       SPH_S_NNGB};
const int kForceIn[] = {SPH_S_OFF_X, SPH_S_OFF_Y, SPH_S_OFF_Z, SPH_S_VQ_X, SPH_S_VQ_Y, SPH_S_VQ_Z,
                        SPH_S_M, SPH_S_H, SPH_S_RHO, SPH_S_F, SPH_S_P, SPH_S_C, SPH_S_A_X,
                        SPH_S_A_Y, SPH_S_A_Z, SPH_S_DU, SPH_S_VSIG};
const int kKickIn[] = {SPH_S_X_X, SPH_S_X_Y, SPH_S_X_Z, SPH_S_V_X, SPH_S_V_Y, SPH_S_V_Z, SPH_S_UK,
                       SPH_S_A_X, SPH_S_A_Y, SPH_S_A_Z, SPH_S_DU};
const int kReduceIn[] = {SPH_S_VQ_X, SPH_S_VQ_Y, SPH_S_VQ_Z, SPH_S_A_X, SPH_S_A_Y, SPH_S_A_Z,
                         SPH_S_DU};
const int kViewDens[] = {SPH_S_OFF_X, SPH_S_OFF_Y, SPH_S_OFF_Z, SPH_S_M, SPH_S_H, SPH_S_U};
const int kViewForce[] = {SPH_S_OFF_X, SPH_S_OFF_Y, SPH_S_OFF_Z, SPH_S_VQ_X, SPH_S_VQ_Y,
                          SPH_S_VQ_Z, SPH_S_M, SPH_S_H};
const int kViewKick[] = {SPH_S_X_X, SPH_S_X_Y, SPH_S_X_Z, SPH_S_V_X, SPH_S_V_Y, SPH_S_V_Z,
                         SPH_S_UK};

template <size_t N>
constexpr int len(const int (&)[N]) { return (int)N; }

sph_status check_view_soa(const sph_soa* s, int view, const char* what) {
  switch (view) {
    case SPH_VIEW_DENSITY: return check_soa(s, kViewDens, len(kViewDens), what);
    case SPH_VIEW_FORCE: return check_soa(s, kViewForce, len(kViewForce), what);
    case SPH_VIEW_KICK: return check_soa(s, kViewKick, len(kViewKick), what);
    case SPH_VIEW_FULL:
      SPH_TRY(check_soa(s, kViewDens, len(kViewDens), what));
      SPH_TRY(check_soa(s, kViewForce, len(kViewForce), what));
      return check_soa(s, kViewKick, len(kViewKick), what);
    default: return fail(SPH_E_INVALID, "%s: unknown view %d", what, view);
  }
}

uint32_t view_aos_fields(int view) {
  uint32_t need = bit(SPH_A_X);
  if (view == SPH_VIEW_DENSITY || view == SPH_VIEW_FULL)
    need |= bit(SPH_A_M) | bit(SPH_A_H) | bit(SPH_A_U);
  if (view == SPH_VIEW_FORCE || view == SPH_VIEW_FULL)
    need |= bit(SPH_A_V) | bit(SPH_A_M) | bit(SPH_A_H);
  if (view == SPH_VIEW_KICK || view == SPH_VIEW_FULL) need |= bit(SPH_A_V) | bit(SPH_A_U);
  return need;
}

}  // namespace

namespace sph {
sph_status host_fail(sph_status code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace sph

extern "C" {

int32_t sph_abi_version(void) { return SPH_ABI_VERSION; }

sph_status sph_storage_bytes(int32_t n, int32_t dtype, size_t* bytes) {
  if (!bytes || n < 0) return fail(SPH_E_INVALID, "sph_storage_bytes: bad arguments");
  if (!is_store_dt(dtype))
    return fail(SPH_E_INVALID, "sph_storage_bytes: dtype %d is not a storage format", dtype);
  *bytes = storage_bytes(n, dtype);
  return SPH_OK;
}

const char* sph_last_error(void) { return g_err.c_str(); }

int32_t sph_tile_supported(sph_tile tile) { return tile_supported(tile.ti, tile.k) ? 1 : 0; }

sph_status sph_bin_workspace_size(int32_t n, int32_t n_c, size_t* bytes) {
  if (!bytes) return fail(SPH_E_INVALID, "bytes is NULL");
  if (n < 0) return fail(SPH_E_INVALID, "n = %d is negative", n);
  if (n_c < 3 || n_c > 1290) return fail(SPH_E_RANGE, "n_c = %d out of range [3, 1290]", n_c);
  *bytes = bin_workspace_bytes(n, n_c, 0);
  return SPH_OK;
}

sph_status sph_worklist_size(int32_t n, int32_t n_c, int32_t ti, size_t* bytes) {
  if (!bytes) return fail(SPH_E_INVALID, "bytes is NULL");
  if (n < 0) return fail(SPH_E_INVALID, "n = %d is negative", n);
  if (n_c < 3 || n_c > 1290) return fail(SPH_E_RANGE, "n_c = %d out of range [3, 1290]", n_c);
  if (ti < 1 || ti > 4096) return fail(SPH_E_INVALID, "ti = %d out of range [1, 4096]", ti);
  *bytes = worklist_bytes(n, n_c, ti);
  return SPH_OK;
}

sph_status sph_worklist(const sph_cells* cells, sph_work* work, hipStream_t stream) {
  return sph_worklist_occupancy(cells, work, 0, 0x7fffffff, stream);
}

sph_status sph_worklist_occupancy(const sph_cells* cells, sph_work* work, int32_t occ_lo,
                                  int32_t occ_hi, hipStream_t stream) {
  CellsDev c;
  SPH_TRY(check_cells(cells, true, c));
  if (!work || !work->buf) return fail(SPH_E_INVALID, "work or work->buf is NULL");
  if (work->ti < 1 || work->ti > 4096) return fail(SPH_E_INVALID, "work->ti = %d out of range", work->ti);
  if (work->sched < SPH_SCHED_GRID || work->sched > SPH_SCHED_DYNAMIC)
    return fail(SPH_E_INVALID, "work->sched = %d is not an SPH_SCHED_* value", work->sched);
  if (work->bytes < worklist_bytes(c.n, c.n_c, work->ti))
    return fail(SPH_E_NOMEM, "work->bytes %zu < %zu", work->bytes,
                worklist_bytes(c.n, c.n_c, work->ti));
  if (occ_lo < 0 || occ_hi <= occ_lo)
    return fail(SPH_E_INVALID, "occupancy range [%d, %d) is empty or negative", occ_lo, occ_hi);
  SPH_TRY(check_merge(work, c));
  WorkDev w = work_view(*work, c.n, c.n_c);
  return hip_status(launch_worklist_range(c, w, nullptr, occ_lo, occ_hi, stream,
                                          c.rebin ? c.rebin + 1 : nullptr),
                    "sph_worklist");
}

sph_status sph_bin(const void* aos, const sph_aos_layout* layout, const sph_cells* cells,
                   void* workspace, size_t workspace_bytes, hipStream_t stream) {
  AosLayout L;
  CellsDev c;
  SPH_TRY(check_layout(layout, bit(SPH_A_X), L));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_aos_ptr(aos, c.n));
  size_t need = bin_workspace_bytes(c.n, c.n_c, c.sub_bits);
  if (!workspace) return fail(SPH_E_INVALID, "workspace is NULL");
  if (workspace_bytes < need)
    return fail(SPH_E_NOMEM, "workspace has %zu bytes, sph_bin needs %zu", workspace_bytes, need);
  return hip_status(launch_bin(aos, L, c, cells->cell_start, cells->perm, cells->cell,
                               cells->sub_bits > 0 ? cells->sub_start : nullptr, cells->hmax,
                               workspace, stream),
                    "sph_bin");
}

sph_status sph_convert(const void* aos, const sph_aos_layout* layout, const sph_cells* cells,
                       int32_t view, const sph_precision* prec, const sph_soa* out,
                       hipStream_t stream) {
  AosLayout L;
  CellsDev c;
  Prec p;
  SPH_TRY(check_view_soa(out, view, "sph_convert"));
  SPH_TRY(check_layout(layout, view_aos_fields(view), L));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_prec(prec, p));
  if (view != SPH_VIEW_KICK) SPH_TRY(check_anchor(out, p, "sph_convert"));
  SPH_TRY(check_aos_ptr(aos, c.n));
  if ((is_trunc(p.pos) || is_trunc(p.vel) || is_trunc(p.mhu)) && L.stride > kMaxPackedStride)
    return fail(SPH_E_UNSUPPORTED,
                "sph_convert: truncated storage needs records of at most %u bytes",
                kMaxPackedStride);
  return hip_status(launch_convert(aos, L, c, view, p, *out, stream), "sph_convert");
}

sph_status sph_writeback(const sph_soa* soa, const sph_cells* cells, int32_t view, void* aos,
                         const sph_aos_layout* layout, hipStream_t stream) {
  AosLayout L;
  CellsDev c;
  if (!soa) return fail(SPH_E_INVALID, "sph_writeback: soa is NULL");
  if (view < SPH_VIEW_DENSITY || view > SPH_VIEW_FULL)
    return fail(SPH_E_INVALID, "sph_writeback: unknown view %d", view);
  uint32_t need = bit(SPH_A_X);
  if (view == SPH_VIEW_KICK || view == SPH_VIEW_FULL) {
    SPH_TRY(check_view_soa(soa, SPH_VIEW_KICK, "sph_writeback"));
    need |= bit(SPH_A_V) | bit(SPH_A_U);
  }
  bool dens = (view == SPH_VIEW_DENSITY || view == SPH_VIEW_FULL) && soa->f[SPH_S_RHO];
  bool force = (view == SPH_VIEW_FORCE || view == SPH_VIEW_FULL) && soa->f[SPH_S_A_X];
  if (dens) {
    const int f[] = {SPH_S_RHO, SPH_S_WCOUNT, SPH_S_RHO_DH, SPH_S_F, SPH_S_P, SPH_S_C, SPH_S_NNGB};
    SPH_TRY(check_soa(soa, f, len(f), "sph_writeback"));
  }
  if (force) {
    const int f[] = {SPH_S_A_X, SPH_S_A_Y, SPH_S_A_Z, SPH_S_DU, SPH_S_VSIG};
    SPH_TRY(check_soa(soa, f, len(f), "sph_writeback"));
  }
  SPH_TRY(check_layout(layout, need, L));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_aos_ptr(aos, c.n));
  return hip_status(launch_writeback(*soa, c, view, aos, L, stream), "sph_writeback");
}

sph_status sph_density(const sph_soa* soa, const sph_precision* prec, const sph_cells* cells,
                       const sph_params* params, sph_tile tile, const sph_work* work,
                       hipStream_t stream) {
  CellsDev c;
  Prec p;
  Phys ph;
  WorkDev w;
  bool use_w;
  int ti, k;
  SPH_TRY(check_soa(soa, kDensIn, len(kDensIn), "sph_density"));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_prec(prec, p));
  SPH_TRY(check_anchor(soa, p, "sph_density"));
  SPH_TRY(check_params(params, ph));
  SPH_TRY(resolve_tile(tile, ti, k));
  SPH_TRY(check_work(work, c, ti, w, use_w));
  return hip_status(launch_density(*soa, p, c, ph, ti, k, use_w ? &w : nullptr, stream),
                    "sph_density");
}

sph_status sph_force(const sph_soa* soa, const sph_precision* prec, const sph_cells* cells,
                     const sph_params* params, sph_tile tile, const sph_work* work,
                     hipStream_t stream) {
  CellsDev c;
  Prec p;
  Phys ph;
  WorkDev w;
  bool use_w;
  int ti, k;
  SPH_TRY(check_soa(soa, kForceIn, len(kForceIn), "sph_force"));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_prec(prec, p));
  SPH_TRY(check_anchor(soa, p, "sph_force"));
  SPH_TRY(check_params(params, ph));
  SPH_TRY(resolve_tile(tile, ti, k));
  SPH_TRY(check_work(work, c, ti, w, use_w));
  return hip_status(launch_force(*soa, p, c, ph, ti, k, use_w ? &w : nullptr, stream),
                    "sph_force");
}

int32_t sph_task_tile_supported(sph_tile tile) {
  return task_tile_supported(tile.ti, tile.k) ? 1 : 0;
}

sph_status sph_tasks_run(const sph_soa* soa, const sph_precision* prec, const sph_cells* cells,
                         const sph_params* params, sph_tile tile, const sph_task* tasks,
                         int32_t n_tasks, const int32_t* out_off, const int32_t* items,
                         int32_t n_dens, int32_t n_force, sph_task_result* out, int32_t n_out,
                         hipStream_t stream) {
  CellsDev c;
  Prec p;
  Phys ph;
  if (n_dens < 0 || n_force < 0 || n_out < 0 || n_tasks < 0)
    return fail(SPH_E_INVALID, "sph_tasks_run: negative count");
  if (n_dens > 0) SPH_TRY(check_soa(soa, kDensIn, len(kDensIn), "sph_tasks_run"));
  if (n_force > 0) SPH_TRY(check_soa(soa, kForceIn, len(kForceIn), "sph_tasks_run"));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_prec(prec, p));
  if (n_dens + n_force > 0) SPH_TRY(check_anchor(soa, p, "sph_tasks_run"));
  SPH_TRY(check_params(params, ph));
  const int ti = tile.ti ? tile.ti : 64, k = tile.k ? tile.k : 4;
  if (!task_tile_supported(ti, k))
    return fail(SPH_E_UNSUPPORTED, "sph_tasks_run: tile %dx%d not supported", ti, k);
  if (n_dens + n_force == 0) return SPH_OK;
  if (n_tasks == 0) return fail(SPH_E_INVALID, "sph_tasks_run: items but no tasks");
  if (!tasks || !out_off || !items || !out)
    return fail(SPH_E_INVALID, "sph_tasks_run: NULL task array");
  if ((reinterpret_cast<uintptr_t>(out) & 15) || (reinterpret_cast<uintptr_t>(items) & 7))
    return fail(SPH_E_INVALID, "sph_tasks_run: out must be 16-byte and items 8-byte aligned");
  return hip_status(launch_tasks(*soa, p, c, ph, ti, k, tasks, n_tasks, out_off, items, n_dens,
                                 n_force, out, n_out, stream),
                    "sph_tasks_run");
}

sph_status sph_smoothing_length_workspace_size(int32_t n, size_t* bytes) {
  if (!bytes || n < 0) return fail(SPH_E_INVALID, "sph_smoothing_length_workspace_size: bad arguments");
  *bytes = hiter_workspace_bytes(n);
  return SPH_OK;
}

sph_status sph_smoothing_length(const sph_soa* soa, const sph_precision* prec,
                                const sph_cells* cells, const sph_params* params, double eta,
                                double tol, int32_t max_iter, sph_tile tile,
                                const sph_work* work, void* workspace, size_t workspace_bytes,
                                void* aos, const sph_aos_layout* layout, int32_t* iterations,
                                int32_t* unconverged, hipStream_t stream) {
  CellsDev c;
  Prec p;
  Phys ph;
  WorkDev w;
  bool use_w;
  int ti, k;
  SPH_TRY(check_soa(soa, kDensIn, len(kDensIn), "sph_smoothing_length"));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_prec(prec, p));
  SPH_TRY(check_anchor(soa, p, "sph_smoothing_length"));
  SPH_TRY(check_params(params, ph));
  SPH_TRY(resolve_tile(tile, ti, k));
  SPH_TRY(check_work(work, c, ti, w, use_w));
  if (p.mhu != SPH_F32)
    return fail(SPH_E_UNSUPPORTED, "sph_smoothing_length: H must be stored in SPH_F32");
  if (!(eta > 0.0) || !std::isfinite(eta) || !(tol > 0.0) || !std::isfinite(tol))
    return fail(SPH_E_INVALID, "sph_smoothing_length: eta and tol must be positive");
  if (max_iter < 1 || max_iter > 1000)
    return fail(SPH_E_INVALID, "sph_smoothing_length: max_iter must be 1..1000");
  if (!iterations || !unconverged)
    return fail(SPH_E_INVALID, "sph_smoothing_length: NULL result pointer");
  if (!workspace || workspace_bytes < hiter_workspace_bytes(c.n))
    return fail(SPH_E_NOMEM, "sph_smoothing_length: workspace too small");
  AosLayout L{};
  if (aos) {
    SPH_TRY(check_layout(layout, bit(SPH_A_H), L));
    SPH_TRY(check_aos_ptr(aos, c.n));
  }
  // largest FP32 h whose support fits a cell both in the kernels' FP32 test,
  // (gamma_k h)^2 <= (1 / n_c)^2, and exactly, gamma_k h <= 1 / n_c
  const float s32 = (float)(1.0 / (double)c.n_c);
  float h_max = s32 / ph.gamma_k;
  while (h_max > 0.0f) {
    const float H = ph.gamma_k * h_max;
    if (H * H <= s32 * s32 && params->gamma_k * (double)h_max <= 1.0 / (double)c.n_c) break;
    h_max = std::nextafter(h_max, 0.0f);
  }
  *iterations = 0;
  *unconverged = c.n;
  if (c.n == 0) {
    *unconverged = 0;
    return SPH_OK;
  }
  hipError_t e = launch_hiter_init(*soa, p, c.n, h_max, workspace, stream);
  if (e != hipSuccess) return hip_status(e, "sph_smoothing_length");
  int32_t left = c.n;
  int it = 0;
  while (it < max_iter) {
    if (use_w) e = launch_worklist_active(c, w, hiter_active(workspace, c.n), stream);
    if (e == hipSuccess) e = launch_density(*soa, p, c, ph, ti, k, use_w ? &w : nullptr, stream);
    if (e == hipSuccess)
      e = launch_hiter_update(*soa, p, c.n, (float)eta, (float)tol, h_max, workspace, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&left, hiter_left(workspace, c.n), sizeof(int32_t),
                         hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_status(e, "sph_smoothing_length");
    ++it;
    if (left == 0) break;
  }
  *iterations = it;
  *unconverged = left;
  if (c.hmax) e = launch_cell_hmax(*soa, p, c, const_cast<float*>(c.hmax), stream);
  if (e == hipSuccess && aos) e = launch_write_h(*soa, p, c, aos, L, stream);
  return hip_status(e, "sph_smoothing_length");
}

sph_status sph_kick_drift(const sph_soa* soa, const sph_cells* cells, double dt_kick,
                          double dt_drift, int32_t* moved, hipStream_t stream) {
  CellsDev c;
  SPH_TRY(check_soa(soa, kKickIn, len(kKickIn), "sph_kick_drift"));
  SPH_TRY(check_cells(cells, false, c));
  if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift))
    return fail(SPH_E_INVALID, "time steps must be finite");
  return hip_status(launch_kick_drift(*soa, c, dt_kick, dt_drift, moved, stream), "sph_kick_drift");
}

sph_status sph_reduce_workspace_size(int32_t n, size_t* bytes) {
  if (!bytes) return fail(SPH_E_INVALID, "bytes is NULL");
  if (n < 0) return fail(SPH_E_INVALID, "n = %d is negative", n);
  *bytes = reduce_workspace_bytes(n);
  return SPH_OK;
}

sph_status sph_reduce(const sph_soa* soa, const sph_precision* prec, const sph_cells* cells,
                      double* out, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  CellsDev c;
  Prec p;
  SPH_TRY(check_soa(soa, kReduceIn, len(kReduceIn), "sph_reduce"));
  SPH_TRY(check_cells(cells, false, c));
  SPH_TRY(check_prec(prec, p));
  if (!out) return fail(SPH_E_INVALID, "sph_reduce: out is NULL");
  if (!workspace) return fail(SPH_E_INVALID, "sph_reduce: workspace is NULL");
  if (workspace_bytes < reduce_workspace_bytes(c.n))
    return fail(SPH_E_NOMEM, "sph_reduce: workspace has %zu bytes, needs %zu", workspace_bytes,
                reduce_workspace_bytes(c.n));
  return hip_status(launch_reduce(*soa, p, c.n, out, workspace, stream), "sph_reduce");
}

sph_status sph_reduce_static(const sph_soa* soa, const sph_precision* prec,
                             const sph_cells* cells, double* out, hipStream_t stream) {
  CellsDev c;
  Prec p;
  SPH_TRY(check_soa(soa, kReduceIn, len(kReduceIn), "sph_reduce_static"));
  SPH_TRY(check_cells(cells, false, c));
  SPH_TRY(check_prec(prec, p));
  if (!out) return fail(SPH_E_INVALID, "sph_reduce_static: out is NULL");
  if (reduce_workspace_bytes(c.n) > reduce_scratch_bytes())
    return fail(SPH_E_NOMEM, "sph_reduce_static: %d slots need %zu scratch bytes, the library "
                "holds %zu", c.n, reduce_workspace_bytes(c.n), reduce_scratch_bytes());
  void* ws = nullptr;
  SPH_TRY(hip_status(reduce_scratch(&ws), "sph_reduce_static: scratch address"));
  return hip_status(launch_reduce(*soa, p, c.n, out, ws, stream), "sph_reduce_static");
}

sph_status sph_reduce_aos(const void* aos, const sph_aos_layout* layout, const sph_cells* cells,
                          double* out, void* workspace, size_t workspace_bytes,
                          hipStream_t stream) {
  CellsDev c;
  AosLayout L;
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_layout(layout, bit(SPH_A_V) | bit(SPH_A_A) | bit(SPH_A_DU), L));
  SPH_TRY(check_aos_ptr(aos, c.n));
  if (!out) return fail(SPH_E_INVALID, "sph_reduce_aos: out is NULL");
  if (!workspace) return fail(SPH_E_INVALID, "sph_reduce_aos: workspace is NULL");
  if (workspace_bytes < reduce_workspace_bytes(c.n))
    return fail(SPH_E_NOMEM, "sph_reduce_aos: workspace has %zu bytes, needs %zu",
                workspace_bytes, reduce_workspace_bytes(c.n));
  return hip_status(launch_reduce_aos(aos, L, c, out, workspace, stream), "sph_reduce_aos");
}

sph_status sph_predict(const sph_soa* soa, const sph_precision* prec, const sph_cells* cells,
                       const void* aos, const sph_aos_layout* layout, double dt_half,
                       hipStream_t stream) {
  static const int kPredIn[] = {SPH_S_V_X, SPH_S_V_Y, SPH_S_V_Z, SPH_S_UK,
                                SPH_S_VQ_X, SPH_S_VQ_Y, SPH_S_VQ_Z, SPH_S_U};
  CellsDev c;
  Prec p;
  AosLayout L;
  SPH_TRY(check_soa(soa, kPredIn, len(kPredIn), "sph_predict"));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_prec(prec, p));
  SPH_TRY(check_layout(layout, bit(SPH_A_A) | bit(SPH_A_DU), L));
  SPH_TRY(check_aos_ptr(aos, c.n));
  if (is_trunc(p.vel) || is_trunc(p.mhu))
    return fail(SPH_E_UNSUPPORTED, "sph_predict: truncated storage is written by sph_convert only");
  if (!std::isfinite(dt_half)) return fail(SPH_E_INVALID, "sph_predict: dt_half must be finite");
  return hip_status(launch_predict(*soa, p, c, aos, L, dt_half, stream), "sph_predict");
}

sph_status sph_step_totals(const sph_soa* soa, const sph_precision* prec, const sph_cells* cells,
                           const sph_params* params, double c_cfl, double* out, void* workspace,
                           size_t workspace_bytes, hipStream_t stream) {
  static const int kTotIn[] = {SPH_S_M, SPH_S_H, SPH_S_V_X, SPH_S_V_Y, SPH_S_V_Z, SPH_S_UK,
                               SPH_S_VSIG};
  CellsDev c;
  Prec p;
  Phys ph;
  SPH_TRY(check_soa(soa, kTotIn, len(kTotIn), "sph_step_totals"));
  SPH_TRY(check_cells(cells, false, c));
  SPH_TRY(check_prec(prec, p));
  SPH_TRY(check_params(params, ph));
  if (!(c_cfl > 0.0) || !std::isfinite(c_cfl))
    return fail(SPH_E_INVALID, "sph_step_totals: c_cfl must be positive and finite");
  if (!out) return fail(SPH_E_INVALID, "sph_step_totals: out is NULL");
  if (!workspace) return fail(SPH_E_INVALID, "sph_step_totals: workspace is NULL");
  if (workspace_bytes < reduce_workspace_bytes(c.n))
    return fail(SPH_E_NOMEM, "sph_step_totals: workspace has %zu bytes, needs %zu",
                workspace_bytes, reduce_workspace_bytes(c.n));
  return hip_status(launch_step_totals(*soa, p, c.n, params->gamma_k, c_cfl, out, workspace,
                                       stream),
                    "sph_step_totals");
}

sph_status sph_density_aos(void* aos, const sph_aos_layout* layout, const sph_cells* cells,
                           const sph_params* params, sph_tile tile, const sph_work* work,
                           hipStream_t stream) {
  AosLayout L;
  CellsDev c;
  Phys ph;
  WorkDev w;
  bool use_w;
  int ti, k;
  SPH_TRY(check_layout(layout,
                       bit(SPH_A_X) | bit(SPH_A_M) | bit(SPH_A_H) | bit(SPH_A_U) | bit(SPH_A_RHO) |
                           bit(SPH_A_WCOUNT) | bit(SPH_A_RHO_DH) | bit(SPH_A_F) | bit(SPH_A_P) |
                           bit(SPH_A_C),
                       L));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_params(params, ph));
  SPH_TRY(resolve_tile(tile, ti, k));
  SPH_TRY(check_aos_ptr(aos, c.n));
  SPH_TRY(check_work(work, c, ti, w, use_w));
  return hip_status(launch_density_aos(aos, L, c, ph, ti, k, use_w ? &w : nullptr, stream),
                    "sph_density_aos");
}

sph_status sph_force_aos(void* aos, const sph_aos_layout* layout, const sph_cells* cells,
                         const sph_params* params, sph_tile tile, const sph_work* work,
                         hipStream_t stream) {
  AosLayout L;
  CellsDev c;
  Phys ph;
  WorkDev w;
  bool use_w;
  int ti, k;
  SPH_TRY(check_layout(layout,
                       bit(SPH_A_X) | bit(SPH_A_V) | bit(SPH_A_A) | bit(SPH_A_M) | bit(SPH_A_H) |
                           bit(SPH_A_RHO) | bit(SPH_A_F) | bit(SPH_A_P) | bit(SPH_A_C) |
                           bit(SPH_A_DU) | bit(SPH_A_VSIG),
                       L));
  SPH_TRY(check_cells(cells, true, c));
  SPH_TRY(check_params(params, ph));
  SPH_TRY(resolve_tile(tile, ti, k));
  SPH_TRY(check_aos_ptr(aos, c.n));
  SPH_TRY(check_work(work, c, ti, w, use_w));
  return hip_status(launch_force_aos(aos, L, c, ph, ti, k, use_w ? &w : nullptr, stream),
                    "sph_force_aos");
}

sph_status sph_kick_drift_aos(void* aos, const sph_aos_layout* layout, const sph_cells* cells,
                              double dt_kick, double dt_drift, int32_t* moved,
                              hipStream_t stream) {
  AosLayout L;
  CellsDev c;
  SPH_TRY(check_layout(layout,
                       bit(SPH_A_X) | bit(SPH_A_V) | bit(SPH_A_A) | bit(SPH_A_U) | bit(SPH_A_DU), L));
  SPH_TRY(check_cells(cells, false, c));
  if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift))
    return fail(SPH_E_INVALID, "time steps must be finite");
  SPH_TRY(check_aos_ptr(aos, c.n));
  return hip_status(launch_kick_drift_aos(aos, L, c.n, c.n_c, c.sub_bits, dt_kick, dt_drift, moved, stream),
                    "sph_kick_drift_aos");
}

sph_status sph_hbm_probe(int32_t mode, const void* src, void* dst, size_t bytes,
                         hipStream_t stream) {
  if (mode != SPH_PROBE_COPY && mode != SPH_PROBE_READ && mode != SPH_PROBE_WRITE)
    return fail(SPH_E_INVALID, "sph_hbm_probe: unknown mode %d", mode);
  if (bytes % 16 != 0) return fail(SPH_E_INVALID, "sph_hbm_probe: bytes must be a multiple of 16");
  if (bytes == 0) return SPH_OK;
  const bool need_src = mode != SPH_PROBE_WRITE;
  if ((need_src && !src) || !dst) return fail(SPH_E_INVALID, "sph_hbm_probe: NULL buffer");
  if ((need_src && (reinterpret_cast<uintptr_t>(src) & 15)) ||
      (mode != SPH_PROBE_READ && (reinterpret_cast<uintptr_t>(dst) & 15)))
    return fail(SPH_E_INVALID, "sph_hbm_probe: buffers must be 16-byte aligned");
  if (bytes / 16 >= (size_t)1 << 38) return fail(SPH_E_RANGE, "sph_hbm_probe: too many bytes");
  return hip_status(launch_hbm_probe(mode, src, dst, bytes, stream), "sph_hbm_probe");
}

sph_status sph_sync(hipStream_t stream) {
  return hip_status(hipStreamSynchronize(stream), "sph_sync");
}

}  // extern "C"
