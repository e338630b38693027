// Instantiation of the force kernel for one data source (SoaSrc<DT_F16, DT_F16, DT_F16>).
#include "pair_impl.h"

namespace sph {
namespace pairk {

hipError_t run_force_force_h(const SoaSrc<DT_F16, DT_F16, DT_F16>& src, const CellsDev& c, const Phys& ph, int ti, int k,
                  const WorkDev* w, hipStream_t s) {
  return run_force(src, c, ph, ti, k, w, s);
}

}  // namespace pairk
}  // namespace sph
