// Device-side problem table of the batched GAP-TV solve, and its launchers.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "sci_internal.h"

namespace sci {

struct BatchProb {
    int nx, ny, B;
    int outer_iters; // this problem's outer iteration count
    int ntx, ntiles; // tiles per frame of the denoise launch's (shape, pass length)
    int wg_base;     // first workgroup of this problem in a denoise launch
    int pb_base;     // first 256-pixel block of this problem in setup launches
    int pj_base;     // first block of this problem in projection launches
    int pairs;       // 1: the projection takes two adjacent pixels per thread (even nx*ny, 8-byte aligned)
    const float *Y, *C;
    float *Sinv, *x, *theta;
    uint32_t *cbits; // masks packed one bit per frame (valid when *cflag != 0)
    int *cflag;      // 1: every mask entry is 0 or 1 and B <= 32
};

// Interior extent of a tile of `shape` for pass length m.
void batch_tile_extent(int shape, int m, int *tile_w, int *tile_h);
// theta^(0) = Phi^T y, Sinv and the packed masks for the first n problems
// (x = theta^(0) where outer_iters == 0).
void launch_batch_setup(int n, int nblocks, const BatchProb *tab, hipStream_t s);
// GAP projection of the first n problems (nblocks: their projection blocks).
int launch_batch_project(int n, int nblocks, int maxB, const BatchProb *tab, hipStream_t s);
// Cold-start fused denoise (m iterations, theta output) of the first n problems.
int launch_batch_denoise(int tv, int shape, int m, int n, int nwg, const BatchProb *tab, const TileBeta &bt,
                         float lam, hipStream_t s);

} // namespace sci
