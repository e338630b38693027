// Instantiation of the cell-pair task kernels for one data source (SoaSrc<DT_F16, DT_BF16, DT_F16>).
#include "pair_impl.h"

namespace sph {
namespace pairk {

hipError_t run_tasks_r(const SoaSrc<DT_F16, DT_BF16, DT_F16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                       const TaskItems& dens, const TaskItems& force, hipStream_t s) {
  return run_tasks(src, c, ph, ti, k, dens, force, s);
}

}  // namespace pairk
}  // namespace sph
