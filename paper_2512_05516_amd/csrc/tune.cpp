// Autotuner of the pair loops: times candidate (tile, schedule) pairs through
// the public entry points, so every candidate is validated exactly as a
// caller's launch would be.
#include <hip/hip_runtime_api.h>

#include <vector>

#include "sph_internal.h"

namespace sph {
sph_status host_fail(sph_status code, const char* msg);
}

namespace {

// Tiles in the order they are tried (ti, k)
const int kTiles[][2] = {{64, 4}, {32, 8}, {128, 2}, {64, 2}, {64, 1}, {16, 16}, {16, 4}, {32, 2}};
const int kScheds[] = {-1, SPH_SCHED_GRID, SPH_SCHED_STATIC, SPH_SCHED_DYNAMIC};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" {

sph_status sph_tune_candidates(sph_tune_entry* out, int32_t max, int32_t* count) {
  if (!count) return sph::host_fail(SPH_E_INVALID, "sph_tune_candidates: count is NULL");
  if (max < 0 || (max > 0 && !out))
    return sph::host_fail(SPH_E_INVALID, "sph_tune_candidates: bad output buffer");
  int n = 0;
  for (const auto& t : kTiles) {
    if (!sph_tile_supported(sph_tile{t[0], t[1]})) continue;
    for (int s : kScheds) {
      if (n < max) out[n] = sph_tune_entry{sph_tile{t[0], t[1]}, s, -1.0f};
      ++n;
    }
  }
  *count = n;
  return SPH_OK;
}

sph_status sph_autotune(int32_t loop, const sph_soa* soa, const sph_precision* prec,
                        const sph_cells* cells, const sph_params* params,
                        sph_tune_entry* cand, int32_t ncand, int32_t reps, void* work_buf,
                        size_t work_bytes, int32_t* best, hipStream_t stream) {
  if (loop != 0 && loop != 1) return sph::host_fail(SPH_E_INVALID, "sph_autotune: loop must be 0 or 1");
  if (!cand || ncand < 1 || !best || !cells)
    return sph::host_fail(SPH_E_INVALID, "sph_autotune: NULL or empty argument");
  if (reps < 1 || reps > 1000) return sph::host_fail(SPH_E_INVALID, "sph_autotune: reps out of range");
  for (int i = 0; i < ncand; ++i) {
    if (cand[i].sched < -1 || cand[i].sched > SPH_SCHED_DYNAMIC)
      return sph::host_fail(SPH_E_INVALID, "sph_autotune: candidate schedule out of range");
    if (!sph_tile_supported(cand[i].tile))
      return sph::host_fail(SPH_E_UNSUPPORTED, "sph_autotune: candidate tile not supported");
  }
  auto run = [&](const sph_tune_entry& e, const sph_work* w) {
    return loop == 0 ? sph_density(soa, prec, cells, params, e.tile, w, stream)
                     : sph_force(soa, prec, cells, params, e.tile, w, stream);
  };
  Events ev;
  if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
    return sph::host_fail(SPH_E_HIP, "sph_autotune: hipEventCreate failed");
  int bi = -1;
  for (int i = 0; i < ncand; ++i) {
    sph_tune_entry& e = cand[i];
    e.ms = -1.0f;
    sph_work w{e.tile.ti, e.sched < 0 ? 0 : e.sched, work_buf, work_bytes};
    const sph_work* wp = nullptr;
    if (e.sched >= 0) {
      size_t need = 0;
      sph_status st = sph_worklist_size(cells->n, cells->n_c, e.tile.ti, &need);
      if (st != SPH_OK) return st;
      if (!work_buf || need > work_bytes) continue;
      st = sph_worklist(cells, &w, stream);
      if (st != SPH_OK) return st;
      wp = &w;
    }
    sph_status st = run(e, wp);
    if (st != SPH_OK) return st;
    if (hipEventRecord(ev.a, stream) != hipSuccess)
      return sph::host_fail(SPH_E_HIP, "sph_autotune: hipEventRecord failed");
    for (int r = 0; r < reps; ++r) {
      st = run(e, wp);
      if (st != SPH_OK) return st;
    }
    float ms = 0.0f;
    if (hipEventRecord(ev.b, stream) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess ||
        hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess)
      return sph::host_fail(SPH_E_HIP, "sph_autotune: timing with HIP events failed");
    e.ms = ms / (float)reps;
    if (bi < 0 || e.ms < cand[bi].ms) bi = i;
  }
  if (bi < 0) return sph::host_fail(SPH_E_NOMEM, "sph_autotune: no candidate fits work_bytes");
  *best = bi;
  return SPH_OK;
}

}  // extern "C"
