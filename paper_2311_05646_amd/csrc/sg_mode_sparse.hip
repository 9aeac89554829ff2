// Column-kernel instantiations for MODE_VJP_SPARSE (eps_grad_vjp_sparse).
#include "sg_column.h"

namespace sg {

template hipError_t launch_mode<MODE_VJP_SPARSE>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace sg
