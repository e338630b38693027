// Internal declarations of libsphmi shared by the host entry points
// (abi.cpp) and the HIP translation units that launch the kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sphmi.h"

namespace sph {

enum : int { DT_F64 = SPH_F64, DT_F32 = SPH_F32, DT_F16 = SPH_F16, DT_BF16 = SPH_BF16,
             DT_I32 = SPH_I32, DT_TRUNC = SPH_TRUNC };
constexpr int kTruncTile = 256;   // slots whose codes fill whole words (256 T bits)
constexpr uint32_t kMaxStagedStride = 248;   // largest record staged through LDS by convert
constexpr uint32_t kMaxPackedStride = 208;   // ... when it also packs truncated codes (9 KiB)
inline bool is_trunc(int dt) { return dt >= DT_TRUNC + 9 && dt <= DT_TRUNC + 32; }
// bytes of a field of n values stored in dt (packed codes: whole tiles of
// 256 values plus two words read past the last value's word)
inline size_t storage_bytes(int64_t n, int dt) {
  if (is_trunc(dt))
    return (size_t)(((n + kTruncTile - 1) / kTruncTile) * 8 * (dt - DT_TRUNC) + 2) * 4;
  return (size_t)n * (dt == DT_F32 ? 4 : 2);
}
constexpr uint32_t kAbsent = SPH_ABSENT;

// AoS layout as passed to kernels (by value)
struct AosLayout {
  uint32_t stride;
  uint32_t off[SPH_A_NFIELDS];
  int32_t dt[SPH_A_NFIELDS];
};

// Precision as passed to kernels: formats and exact power-of-two factors
struct Prec {
  int pos, vel, mhu;
  int anchor;                        // SPH_ANCHOR_CORNER or SPH_ANCHOR_SUB(b)
  float store_m, store_h, store_u;   // 2^scale (applied before storing)
  float load_m, load_h, load_u;      // 2^-scale (applied after loading)
};

struct Phys {
  float gamma_k, gamma, alpha, beta;
  int gradh;
  int kernel;   // SPH_KERNEL_*
};

struct CellsDev {
  int n, n_c;
  int sub_bits;
  const int32_t* start;
  const int32_t* perm;
  const int32_t* cell;
  const int32_t* sub_start;
  const float* hmax;
  int32_t* status;
  unsigned long long* tally;   // [0] candidate tests, [1] gathered (may be null)
  int32_t* rebin;              // [0] moved since the list was built, [1] rebuilt flag
};

// Work list of the pair kernels (device buffer layout): 8 queue counters,
// the item count and the 8 XCD range boundaries, then items (cell, first
// slot). sched: SPH_SCHED_GRID / _STATIC / _DYNAMIC.
struct WorkDev {
  int ti;
  int sched;
  int capacity;
  int merge;           // > 1: items may span that many cells (cell | (m - 1) << 29)
  int32_t* counters;   // [8] next item index of each queue
  int32_t* meta;       // [0] item count, [1..9] range boundaries
  int2* items;         // [capacity]
};
constexpr int kQueues = 8;
constexpr size_t kWorkHeader = 256;   // bytes before the items
constexpr int kMaxMerge = 4;          // cells per merged work item
constexpr int kMergeShift = 29;       // item.x = cell | (cells - 1) << kMergeShift

// --- launchers (return hipError_t of the launch) ---
size_t bin_workspace_bytes(int n, int n_c, int sub_bits);
hipError_t launch_bin(const void* aos, const AosLayout& L, const CellsDev& c, int32_t* cell_start,
                      int32_t* perm, int32_t* cell, int32_t* sub_start, float* hmax, void* ws,
                      hipStream_t s);

// exclusive scan of int32 in place; partials: scan_partials_count(len) ints;
// with gate non-null the kernels do nothing when *gate == 0
size_t scan_partials_count(int len);
hipError_t scan_i32(int32_t* data, int len, int32_t* partials, hipStream_t s,
                    const int32_t* gate = nullptr);

size_t worklist_bytes(int n, int n_c, int ti);
int worklist_capacity(int n, int n_c, int ti);
hipError_t launch_worklist(const CellsDev& c, const WorkDev& w, hipStream_t s);
// gate non-null: the kernels do nothing when *gate == 0
hipError_t launch_worklist_range(const CellsDev& c, const WorkDev& w, const uint8_t* active,
                                 int occ_lo, int occ_hi, hipStream_t s,
                                 const int32_t* gate = nullptr);
// work list of the cells that hold at least one slot with active[k] != 0
hipError_t launch_worklist_active(const CellsDev& c, const WorkDev& w, const uint8_t* active,
                                  hipStream_t s);

// smoothing-length iteration: workspace, init, one update step, cell bounds
size_t hiter_workspace_bytes(int n);
hipError_t launch_hiter_init(const sph_soa& soa, const Prec& p, int n, float h_max, void* ws,
                             hipStream_t s);
hipError_t launch_hiter_update(const sph_soa& soa, const Prec& p, int n, float eta, float tol,
                               float h_max, void* ws, hipStream_t s);
const uint8_t* hiter_active(void* ws, int n);
const int32_t* hiter_left(void* ws, int n);
hipError_t launch_cell_hmax(const sph_soa& soa, const Prec& p, const CellsDev& c, float* hmax,
                            hipStream_t s);
hipError_t launch_write_h(const sph_soa& soa, const Prec& p, const CellsDev& c, void* aos,
                          const AosLayout& L, hipStream_t s);
WorkDev work_view(const sph_work& w, int n, int n_c);

hipError_t launch_convert(const void* aos, const AosLayout& L, const CellsDev& c, int view,
                          const Prec& p, const sph_soa& out, hipStream_t s);
hipError_t launch_writeback(const sph_soa& in, const CellsDev& c, int view, void* aos,
                            const AosLayout& L, hipStream_t s);

bool tile_supported(int ti, int k);
hipError_t launch_density(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                          int ti, int k, const WorkDev* w, hipStream_t s);
hipError_t launch_force(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                        int ti, int k, const WorkDev* w, hipStream_t s);
hipError_t launch_density_aos(void* aos, const AosLayout& L, const CellsDev& c, const Phys& ph,
                              int ti, int k, const WorkDev* w, hipStream_t s);
hipError_t launch_force_aos(void* aos, const AosLayout& L, const CellsDev& c, const Phys& ph,
                            int ti, int k, const WorkDev* w, hipStream_t s);

bool task_tile_supported(int ti, int k);
hipError_t launch_tasks(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                        int ti, int k, const sph_task* tasks, int n_tasks,
                        const int32_t* out_off, const int32_t* items, int n_dens, int n_force,
                        sph_task_result* out, int n_out, hipStream_t s);

hipError_t launch_kick_drift(const sph_soa& soa, const CellsDev& c, double dtk, double dtd,
                             int32_t* moved, hipStream_t s);
hipError_t launch_kick_drift_aos(void* aos, const AosLayout& L, int n, int n_c, int sub_bits,
                                 double dtk, double dtd, int32_t* moved, hipStream_t s);

size_t reduce_workspace_bytes(int n);
hipError_t launch_predict(const sph_soa& soa, const Prec& p, const CellsDev& c, const void* aos,
                          const AosLayout& L, double dth, hipStream_t s);
hipError_t launch_step_totals(const sph_soa& soa, const Prec& p, int n, double gamma_k,
                              double c_cfl, double* out, void* ws, hipStream_t s);
hipError_t launch_reduce(const sph_soa& soa, const Prec& p, int n, double* out, void* ws,
                         hipStream_t s);
hipError_t launch_reduce_aos(const void* aos, const AosLayout& L, const CellsDev& c, double* out,
                             void* ws, hipStream_t s);
hipError_t launch_hbm_probe(int mode, const void* src, void* dst, size_t bytes, hipStream_t s);
// the reduction's device-resident scratch on the current device (address
// resolved once per device) and its size
hipError_t reduce_scratch(void** ptr);
size_t reduce_scratch_bytes();

}  // namespace sph
