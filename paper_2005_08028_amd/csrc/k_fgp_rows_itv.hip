// Row-pipelined fused-schedule FGP passes for ITV2D with float32 dual storage.
#include "k_fgp_rows.h"

namespace sci {

int launch_rows_itv_f32(int H, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                         hipStream_t s)
{
    return launch_rows<TV_ITV2D, DT_F32>(H, m, nx, ny, B, x, tp, lam, s);
}

} // namespace sci
