// Column-kernel instantiations for MODE_VJP_GEPS (eps_grad_vjp_geps).
#include "sg_column.h"

namespace sg {

template hipError_t launch_mode<MODE_VJP_GEPS>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace sg
