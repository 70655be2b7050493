// Tile shapes of the fused-schedule kernel, as (rows per wavefront R,
// wavefronts per workgroup NW, columns per lane C, occupancy hint WPE).
// Tile = (64*C) x (NW*R) pixels including the recomputed halo.
#pragma once

#define SCI_TILE_SHAPES(X)                                                                                          \
    X(0, 4, 16, 1, 8) /* 64 x 64,   1024 threads */                                                                 \
    X(1, 8, 16, 1, 4) /* 64 x 128,  1024 threads */                                                                 \
    X(2, 8, 8, 1, 4)  /* 64 x 64,   512 threads  */                                                                 \
    X(3, 4, 8, 1, 8)  /* 64 x 32,   512 threads  */                                                                 \
    X(4, 4, 16, 2, 4) /* 128 x 64,  1024 threads */                                                                 \
    X(5, 8, 8, 2, 2)  /* 128 x 64,  512 threads  */                                                                 \
    X(6, 7, 16, 2, 4) /* 128 x 112, 1024 threads */                                                                 \
    X(7, 6, 16, 2, 4) /* 128 x 96,  1024 threads */                                                                 \
    X(8, 6, 12, 3, 3) /* 192 x 72,  768 threads  */

// Row-pipelined shapes (k_fgp_rows.h), numbered after the tiled ones: one
// wavefront walks a segment of H rows of a strip of 64 * kRowCols columns.
#define SCI_ROW_SHAPES(X) X(9, 32) X(10, 64) X(11, 96) X(12, 128) X(13, 192) X(14, 256)

namespace sci {
constexpr int kTileShapes = 9; // tiled shapes (ids 0 .. kTileShapes-1)
constexpr int kRowShapes = 6;  // row-pipelined shapes (ids kTileShapes ..)
constexpr int kRowCols = 2;    // columns per lane of the row-pipelined kernel
}
