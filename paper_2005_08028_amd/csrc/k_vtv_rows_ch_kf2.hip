// Row-pipelined VTV passes of Chambolle's (2004) semi-implicit step, 2 frames per wavefront,
// float32 duals.
#include "k_vtv_rows.h"

namespace sci {

int launch_vtv_rows_ch_kf2(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                            float lam, hipStream_t s)
{
    return launch_vtv_kf<2, 1>(m, nx, ny, B, fpw, ng, x, tp, lam, s);
}

} // namespace sci
