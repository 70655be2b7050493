// Row-pipelined passes of Chambolle's (2004) semi-implicit step for ATV and
// ITV2D with float32 dual storage.
#include "k_fgp_rows.h"

namespace sci {

int launch_rows_ch_f32(int tv, int H, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                       hipStream_t s)
{
    if (tv == TV_ATV) return launch_rows<TV_ATV, DT_F32, 1>(H, m, nx, ny, B, x, tp, lam, s);
    if (tv == TV_ITV2D) return launch_rows<TV_ITV2D, DT_F32, 1>(H, m, nx, ny, B, x, tp, lam, s);
    return SCI_ERR_UNSUPPORTED;
}

} // namespace sci
