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

bool vtv_rows_quad(int B, int m) { return B >= 1 && vtv_quad_inst(vtv_fpw(B), m, 0, DT_F32); } // same for every type

// With 2 frames per wavefront, passes longer than 8 need registers that cost
// co-resident workgroups. With the dual records between passes two passes of
// 5 beat one of 10 for every B (measured at 1024x1024, 10 iterations: B = 9,
// 10, 12, 14, 16 one pass 214, 212, 242, 271, 276 us against two 198, 207,
// 231, 235, 261); without them only below 7 wavefronts (B = 9, 10, 12: one
// pass 252, 252, 257 against two 218, 219, 248; B = 14, 16: 272, 276 against
// 284, 310). At 3 frames per wavefront one pass of 7 beats two (7 iterations,
// B = 17-24: 213-226 against 268-319 us with records).
int vtv_rows_auto_pass(int B, bool records)
{
    if (B < 1) return 0;
    const int fpw = vtv_fpw(B), ng = (B + fpw - 1) / fpw;
    if (fpw == 2 && (records || ng < 7)) return std::min(8, vtv_rows_max_m(fpw));
    return vtv_rows_max_m(fpw);
}

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
