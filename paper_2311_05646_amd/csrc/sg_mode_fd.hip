// Column-kernel instantiations for MODE_FD (eps_grad_fd).
#include "sg_column.h"

namespace sg {

template hipError_t launch_mode<MODE_FD>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace sg
