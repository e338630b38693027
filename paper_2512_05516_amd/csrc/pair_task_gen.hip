// Instantiation of the cell-pair task kernels for one data source (SoaSrc<-1, -1, -1>).
#include "pair_impl.h"

namespace sph {
namespace pairk {

hipError_t run_tasks_gen(const SoaSrc<-1, -1, -1>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                       const TaskItems& dens, const TaskItems& force, hipStream_t s) {
  return run_tasks(src, c, ph, ti, k, dens, force, s);
}

}  // namespace pairk
}  // namespace sph
