// Fused-schedule FGP passes for ATV with float32 dual storage, every tile shape.
#include "k_fgp_tile.h"
#include "k_fgp_tile_shapes.h"

namespace sci {

int launch_tile_atv_f32(int shape, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                         hipStream_t s)
{
    switch (shape) {
#define SCI_CASE(id, R, NW, C, WPE)                                                                                 \
    case id: return launch_tile_shape<TV_ATV, DT_F32, R, NW, C, WPE>(m, nx, ny, B, x, tp, lam, s);
        SCI_TILE_SHAPES(SCI_CASE)
#undef SCI_CASE
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
