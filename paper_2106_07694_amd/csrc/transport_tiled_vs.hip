// transport_tiled_vs.hip -- the tiled RK3 stage kernels for runs whose
// settling speed is set by S (eq. 13), built apart so that the two forms
// compile in parallel.
#include "transport_tiled.h"

namespace lbw {

hipError_t launch_transport_tiled_vs(int dim, int precision, const RunDev &r, const lbw_launch &l,
                                     hipStream_t st, const BatchArgs *b) {
    return tiled_any<true>(dim, precision, r, l, st, b);
}

}  // namespace lbw
