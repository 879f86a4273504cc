// shapes.hpp -- the launch-shape table of the register-resident distance
// kernels (definition of for_shapes_p).  Included only by the shapes_*.hip
// translation units, each of which instantiates it for one precision and one
// selection width, so that the kernels of the table compile in parallel.
#pragma once
#include "knn_impl.hpp"

namespace sg {
namespace knn {

template <int PR, class M>
bool for_shapes_p(int d, M& m) {
    const int need = nstep_for(PR, padded_d(PR, d));
#define SG_ONE(PR, NS, W0) m.template add<PR, NS, W0, 1, CB, 0>()
#define SG_THREE(PR, NS, W0)                     \
    do {                                         \
        m.template add<PR, NS, W0, 1, CB, 0>();  \
        m.template add<PR, NS, 4, 1, CB, 64>();  \
        m.template add<PR, NS, 4, 1, CB, 32>();  \
    } while (0)
// ... and, for short rows, 32-row tiles with buffers short enough for four
// workgroups per CU
#define SG_FOUR(PR, NS, W0)                                         \
    do {                                                            \
        SG_THREE(PR, NS, W0);                                       \
        m.template add<PR, NS, 4, 1, cbq_four_wgs<PR, NS>(), 32>(); \
    } while (0)
    if constexpr (PR == SG_PREC_FP32) {
        if (need <= 16) SG_THREE(SG_PREC_FP32, 16, TWAVES);
        else if (need <= 32) SG_THREE(SG_PREC_FP32, 32, TWAVES);
        else if (need <= 48) SG_ONE(SG_PREC_FP32, 48, TWAVES);
        else if (need <= 64) SG_ONE(SG_PREC_FP32, 64, TWAVES);
        else return false;
    } else if constexpr (PR == SG_PREC_F16 || PR == SG_PREC_BF16) {
        if (need <= 2) SG_ONE(PR, 2, TWAVES);
        else if (need <= 4) SG_FOUR(PR, 4, TWAVES);
        else if (need <= 6) SG_FOUR(PR, 6, TWAVES);
        else if (need <= 8) SG_FOUR(PR, 8, TWAVES);
        else if (need <= 12) SG_ONE(PR, 12, TWAVES);
        else if (need <= 16) SG_ONE(PR, 16, TWAVES);
        else if (need <= 24) SG_ONE(PR, 24, 4);
        else if (need <= 32) SG_ONE(PR, 32, 4);
        else if (need <= 48) SG_ONE(PR, 48, 4);
        else return false;
    } else if constexpr (PR == SG_PREC_I8) {
        if (need <= 1) SG_FOUR(SG_PREC_I8, 1, TWAVES);
        else if (need <= 2) SG_FOUR(SG_PREC_I8, 2, TWAVES);
        else if (need <= 4) SG_FOUR(SG_PREC_I8, 4, TWAVES);
        else if (need <= 8) SG_FOUR(SG_PREC_I8, 8, TWAVES);
        else return false;
    } else {
        if (need <= 1) SG_FOUR(SG_PREC_FP8, 1, TWAVES);
        else if (need <= 2) SG_FOUR(SG_PREC_FP8, 2, TWAVES);
        else if (need <= 4) SG_ONE(SG_PREC_FP8, 4, TWAVES);
        else if (need <= 8) SG_ONE(SG_PREC_FP8, 8, 4);
        else if (need <= 16) SG_ONE(SG_PREC_FP8, 16, 4);
        else return false;
    }
    return true;
#undef SG_ONE
#undef SG_THREE
#undef SG_FOUR
}

}  // namespace knn
}  // namespace sg
