// Row-pipelined VTV passes, 1 frame per wavefront, float32 duals.
#include "k_vtv_rows.h"

namespace sci {

int launch_vtv_rows_kf1(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                        float lam, hipStream_t s);
int launch_vtv_rows_kf2(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                        float lam, hipStream_t s);
int launch_vtv_rows_kf3(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                        float lam, hipStream_t s);
int launch_vtv_rows_kf4(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                        float lam, hipStream_t s);

int launch_vtv_rows_ch_kf1(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                            float lam, hipStream_t s);
int launch_vtv_rows_ch_kf2(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                            float lam, hipStream_t s);
int launch_vtv_rows_ch_kf3(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                            float lam, hipStream_t s);
int launch_vtv_rows_ch_kf4(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                            float lam, hipStream_t s);

int launch_vtv_rows16_kf1(int dual_dtype, int m, int nx, int ny, int B, int fpw, int ng, const float *x,
                          const TilePass &tp, float lam, hipStream_t s);
int launch_vtv_rows16_kf2(int dual_dtype, int m, int nx, int ny, int B, int fpw, int ng, const float *x,
                          const TilePass &tp, float lam, hipStream_t s);
int launch_vtv_rows16_kf3(int dual_dtype, int m, int nx, int ny, int B, int fpw, int ng, const float *x,
                          const TilePass &tp, float lam, hipStream_t s);
int launch_vtv_rows16_kf4(int dual_dtype, int m, int nx, int ny, int B, int fpw, int ng, const float *x,
                          const TilePass &tp, float lam, hipStream_t s);

// Frames per wavefront and wavefronts per workgroup: the split of the
// streaming VTV pass (at most kVtvMaxWaves wavefronts).
static int vtv_fpw(int B) { return (B + kVtvMaxWaves - 1) / kVtvMaxWaves; }

int vtv_rows_max_pass(int B) { return B >= 1 ? vtv_rows_max_m(vtv_fpw(B)) : 0; }

int launch_vtv_rows(int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam, hipStream_t s,
                    bool chambolle04, int dual_dtype)
{
    if (B < 1 || m < 1 || m > vtv_rows_max_pass(B)) return SCI_ERR_UNSUPPORTED;
    const int fpw = vtv_fpw(B), ng = (B + fpw - 1) / fpw;
    if (dual_dtype != DT_F32) { // 16-bit storage between passes (projection step only)
        if (chambolle04) return SCI_ERR_UNSUPPORTED;
        switch (fpw) {
        case 1: return launch_vtv_rows16_kf1(dual_dtype, m, nx, ny, B, fpw, ng, x, tp, lam, s);
        case 2: return launch_vtv_rows16_kf2(dual_dtype, m, nx, ny, B, fpw, ng, x, tp, lam, s);
        case 3: return launch_vtv_rows16_kf3(dual_dtype, m, nx, ny, B, fpw, ng, x, tp, lam, s);
        case 4: return launch_vtv_rows16_kf4(dual_dtype, m, nx, ny, B, fpw, ng, x, tp, lam, s);
        }
        return SCI_ERR_UNSUPPORTED;
    }
    if (chambolle04) {
        switch (fpw) {
        case 1: return launch_vtv_rows_ch_kf1(m, nx, ny, B, fpw, ng, x, tp, lam, s);
        case 2: return launch_vtv_rows_ch_kf2(m, nx, ny, B, fpw, ng, x, tp, lam, s);
        case 3: return launch_vtv_rows_ch_kf3(m, nx, ny, B, fpw, ng, x, tp, lam, s);
        case 4: return launch_vtv_rows_ch_kf4(m, nx, ny, B, fpw, ng, x, tp, lam, s);
        }
        return SCI_ERR_UNSUPPORTED;
    }
    switch (fpw) {
    case 1: return launch_vtv_rows_kf1(m, nx, ny, B, fpw, ng, x, tp, lam, s);
    case 2: return launch_vtv_rows_kf2(m, nx, ny, B, fpw, ng, x, tp, lam, s);
    case 3: return launch_vtv_rows_kf3(m, nx, ny, B, fpw, ng, x, tp, lam, s);
    case 4: return launch_vtv_rows_kf4(m, nx, ny, B, fpw, ng, x, tp, lam, s);
    }
    return SCI_ERR_UNSUPPORTED;
}

int launch_vtv_rows_kf1(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp,
                         float lam, hipStream_t s)
{
    return launch_vtv_kf<1, 0>(m, nx, ny, B, fpw, ng, x, tp, lam, s);
}

} // namespace sci
