// Column-kernel instantiations for MODE_EPS (eps_build).
#include "sg_column.h"

namespace sg {

template hipError_t launch_mode<MODE_EPS>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace sg
