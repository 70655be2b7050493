// Row-pipelined VTV passes, 3 frame(s) per wavefront, 16-bit dual storage
// (bf16 or f16) between passes.
#include "k_vtv_rows.h"

namespace sci {

int launch_vtv_rows16_kf3(int dual_dtype, int m, int nx, int ny, int B, int fpw, int ng, const float *x,
                           const TilePass &tp, float lam, hipStream_t s)
{
    if (dual_dtype == DT_BF16) return launch_vtv_kf<3, 0, DT_BF16>(m, nx, ny, B, fpw, ng, x, tp, lam, s);
    if (dual_dtype == DT_F16) return launch_vtv_kf<3, 0, DT_F16>(m, nx, ny, B, fpw, ng, x, tp, lam, s);
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
