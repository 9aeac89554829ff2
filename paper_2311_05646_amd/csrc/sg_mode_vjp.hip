// Column-kernel instantiations for MODE_VJP_FIELDS (eps_grad_vjp and the serving loop's batched launches).
#include "sg_column.h"

namespace sg {

template hipError_t launch_mode<MODE_VJP_FIELDS>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);

hipError_t launch_column_batch(int tree, int variant, const KParams* plist, const int* first, int nreq,
                               int64_t blocks, hipStream_t st) {
    switch (variant) {
        case VAR_BOX_LIN: return launch_batch_variant<MODE_VJP_FIELDS, T_BOX, S_LIN>(tree, plist, first, nreq, blocks, st);
        case VAR_GCART_LIN:
            return launch_batch_variant<MODE_VJP_FIELDS, T_BOX | T_GCART, S_LIN>(tree, plist, first, nreq, blocks, st);
        case VAR_ELL_SIGMOID:
            return launch_batch_variant<MODE_VJP_FIELDS, T_BOX | T_ELL, S_LIN | S_SIGMOID>(tree, plist, first, nreq, blocks,
                                                                                          st);
        case VAR_SERIES_LIN:
            return launch_batch_variant<MODE_VJP_FIELDS, T_BOX | T_SERIES, S_LIN>(tree, plist, first, nreq, blocks, st);
        case VAR_POLAR_SIGMOID:
            return launch_batch_variant<MODE_VJP_FIELDS, T_BOX | T_POLAR, S_LIN | S_SIGMOID>(tree, plist, first, nreq,
                                                                                            blocks, st);
        default: return launch_batch_variant<MODE_VJP_FIELDS, T_ALL, S_ALL>(tree, plist, first, nreq, blocks, st);
    }
}

}  // namespace sg
