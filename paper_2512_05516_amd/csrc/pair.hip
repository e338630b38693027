// Dispatch of the quadratic kernels: storage format and data source to the
// instantiation units (pair_*.hip), tile checks.
#include "pair_impl.h"

namespace sph {
using namespace pairk;

bool tile_supported(int ti, int k) {
  return (ti == 64 && (k == 4 || k == 2 || k == 1)) || (ti == 32 && (k == 8 || k == 2)) ||
         (ti == 128 && k == 2) || (ti == 16 && (k == 16 || k == 4));
}

// Storage formats with compiled-in loaders (FP32; FP16 positions and m/h/u
// with BF16 velocities; all FP16; all BF16); every other combination uses
// the run-time loader.
hipError_t launch_density(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                          int ti, int k, const WorkDev* w, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  if (p.pos == DT_F32 && p.vel == DT_F32 && p.mhu == DT_F32)
    return run_density_dens_f32(make_soa<DT_F32, DT_F32, DT_F32>(soa, p, c.n_c), c, ph, ti, k, w, s);
  if (p.pos == DT_F16 && p.vel == DT_BF16 && p.mhu == DT_F16)
    return run_density_dens_r(make_soa<DT_F16, DT_BF16, DT_F16>(soa, p, c.n_c), c, ph, ti, k, w, s);
  if (p.pos == DT_F16 && p.vel == DT_F16 && p.mhu == DT_F16)
    return run_density_dens_h(make_soa<DT_F16, DT_F16, DT_F16>(soa, p, c.n_c), c, ph, ti, k, w, s);
  if (p.pos == DT_BF16 && p.vel == DT_BF16 && p.mhu == DT_BF16)
    return run_density_dens_b(make_soa<DT_BF16, DT_BF16, DT_BF16>(soa, p, c.n_c), c, ph, ti, k, w, s);
  return run_density_dens_gen(make_soa<-1, -1, -1>(soa, p, c.n_c), c, ph, ti, k, w, s);
}

hipError_t launch_force(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                        int ti, int k, const WorkDev* w, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  if (p.pos == DT_F32 && p.vel == DT_F32 && p.mhu == DT_F32)
    return run_force_force_f32(make_soa<DT_F32, DT_F32, DT_F32>(soa, p, c.n_c), c, ph, ti, k, w, s);
  if (p.pos == DT_F16 && p.vel == DT_BF16 && p.mhu == DT_F16)
    return run_force_force_r(make_soa<DT_F16, DT_BF16, DT_F16>(soa, p, c.n_c), c, ph, ti, k, w, s);
  if (p.pos == DT_F16 && p.vel == DT_F16 && p.mhu == DT_F16)
    return run_force_force_h(make_soa<DT_F16, DT_F16, DT_F16>(soa, p, c.n_c), c, ph, ti, k, w, s);
  if (p.pos == DT_BF16 && p.vel == DT_BF16 && p.mhu == DT_BF16)
    return run_force_force_b(make_soa<DT_BF16, DT_BF16, DT_BF16>(soa, p, c.n_c), c, ph, ti, k, w, s);
  return run_force_force_gen(make_soa<-1, -1, -1>(soa, p, c.n_c), c, ph, ti, k, w, s);
}

hipError_t launch_density_aos(void* aos, const AosLayout& L, const CellsDev& c, const Phys& ph,
                              int ti, int k, const WorkDev* w, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  AosSrc src{static_cast<char*>(aos), L, c.perm};
  return run_density_dens_aos(src, c, ph, ti, k, w, s);
}

hipError_t launch_force_aos(void* aos, const AosLayout& L, const CellsDev& c, const Phys& ph,
                            int ti, int k, const WorkDev* w, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  AosSrc src{static_cast<char*>(aos), L, c.perm};
  return run_force_force_aos(src, c, ph, ti, k, w, s);
}

bool task_tile_supported(int ti, int k) {
  return (ti == 64 && k == 4) || (ti == 32 && k == 8) || (ti == 16 && k == 16);
}

hipError_t launch_tasks(const sph_soa& soa, const Prec& p, const CellsDev& c, const Phys& ph,
                        int ti, int k, const sph_task* tasks, int n_tasks,
                        const int32_t* out_off, const int32_t* items, int n_dens, int n_force,
                        sph_task_result* out, int n_out, hipStream_t s) {
  if (c.n == 0 || n_dens + n_force == 0) return hipSuccess;
  const int2* it = reinterpret_cast<const int2*>(items);
  const TaskItems d{tasks, n_tasks, out_off, it, n_dens, out, n_out};
  const TaskItems f{tasks, n_tasks, out_off, it + n_dens, n_force, out, n_out};
  if (p.pos == DT_F32 && p.vel == DT_F32 && p.mhu == DT_F32)
    return run_tasks_f32(make_soa<DT_F32, DT_F32, DT_F32>(soa, p, c.n_c), c, ph, ti, k, d, f, s);
  if (p.pos == DT_F16 && p.vel == DT_BF16 && p.mhu == DT_F16)
    return run_tasks_r(make_soa<DT_F16, DT_BF16, DT_F16>(soa, p, c.n_c), c, ph, ti, k, d, f, s);
  return run_tasks_gen(make_soa<-1, -1, -1>(soa, p, c.n_c), c, ph, ti, k, d, f, s);
}

}  // namespace sph
