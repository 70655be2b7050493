// Fused-schedule FGP passes with 16-bit dual storage (bf16, f16), default tile
// shape, and the dispatcher over TV kind, storage type and shape (tiled or
// row-pipelined).
#include "k_fgp_tile.h"
#include "k_fgp_tile_shapes.h"

namespace sci {

int launch_tile_atv_f32(int shape, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                        hipStream_t s);
int launch_tile_itv_f32(int shape, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                        hipStream_t s);
int launch_rows_atv_f32(int H, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                        hipStream_t s);
int launch_rows_itv_f32(int H, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                        hipStream_t s);
int launch_rows_ch_f32(int tv, int H, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam,
                       hipStream_t s);

bool tile_supported(int tv) { return tv == TV_ATV || tv == TV_ITV2D; }

int tile_shape_count() { return kTileShapes + kRowShapes; }

bool tile_shape_info(int shape, int *rows, int *waves, int *cols)
{
    switch (shape) {
#define SCI_CASE(id, R, NW, C, WPE)                                                                                 \
    case id: *rows = R; *waves = NW; *cols = C; return true;
        SCI_TILE_SHAPES(SCI_CASE)
#undef SCI_CASE
#define SCI_CASE(id, H)                                                                                             \
    case id: *rows = H; *waves = 1; *cols = kRowCols; return true;
        SCI_ROW_SHAPES(SCI_CASE)
#undef SCI_CASE
    }
    return false;
}

bool tile_shape_pipelined(int shape) { return shape >= kTileShapes && shape < kTileShapes + kRowShapes; }

int launch_fgp_tile(int tv, int dual_dtype, int m, int shape, int nx, int ny, int B, const float *x,
                    const TilePass &tp, float lam, hipStream_t s, bool chambolle04)
{
    if (m < 1 || m > kTileMaxM || shape < 0 || shape >= tile_shape_count()) return SCI_ERR_INVALID_ARG;
    // A cold pass that neither returns nor keeps the dual never stores it, so
    // its storage type does not matter: 16-bit requests take the float32 row
    // kernels too (same bits as a float32 pass; registers are float32).
    const bool no_dual_io = tp.mode == 0 && !tp.pn_out && !tp.pp_out;
    if (tv == TV_VTV) // one row-pipelined kernel, whatever the shape
        return launch_vtv_rows(m, nx, ny, B, x, tp, lam, s, chambolle04, no_dual_io ? DT_F32 : dual_dtype);
    if (chambolle04) { // row-pipelined shapes, float32 duals, ATV and ITV2D
        int H = 0, w = 0, c = 0;
        if (dual_dtype != DT_F32 || !tile_supported(tv) || !tile_shape_pipelined(shape)) return SCI_ERR_UNSUPPORTED;
        tile_shape_info(shape, &H, &w, &c);
        return launch_rows_ch_f32(tv, H, m, nx, ny, B, x, tp, lam, s);
    }
    if (!tile_supported(tv)) return SCI_ERR_UNSUPPORTED;
    if ((dual_dtype == DT_F32 || no_dual_io) && tile_shape_pipelined(shape)) {
        int H = 0, w = 0, c = 0;
        tile_shape_info(shape, &H, &w, &c);
        return tv == TV_ATV ? launch_rows_atv_f32(H, m, nx, ny, B, x, tp, lam, s)
                            : launch_rows_itv_f32(H, m, nx, ny, B, x, tp, lam, s);
    }
    if (dual_dtype == DT_F32)
        return tv == TV_ATV ? launch_tile_atv_f32(shape, m, nx, ny, B, x, tp, lam, s)
                            : launch_tile_itv_f32(shape, m, nx, ny, B, x, tp, lam, s);
    // 16-bit storage: the default shape only
    if (dual_dtype == DT_BF16)
        return tv == TV_ATV ? launch_tile_shape<TV_ATV, DT_BF16, 4, 16, 1, 8>(m, nx, ny, B, x, tp, lam, s)
                            : launch_tile_shape<TV_ITV2D, DT_BF16, 4, 16, 1, 8>(m, nx, ny, B, x, tp, lam, s);
    if (dual_dtype == DT_F16)
        return tv == TV_ATV ? launch_tile_shape<TV_ATV, DT_F16, 4, 16, 1, 8>(m, nx, ny, B, x, tp, lam, s)
                            : launch_tile_shape<TV_ITV2D, DT_F16, 4, 16, 1, 8>(m, nx, ny, B, x, tp, lam, s);
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
