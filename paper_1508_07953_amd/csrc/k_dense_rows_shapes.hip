// k_dense_rows_shapes.hip -- the row-layout dense search at block shapes
// other than each patch width's default (kernels in k_dense_rows.h), for the
// autotuner: wavefronts per block and 32-query column blocks per wavefront.
// The candidates are the ones the hand sweep at D = 64 found within ~10 % of
// the best (six and two column blocks, eight wavefronts) and, for wide
// patches, three column blocks (fewer registers per wavefront).
#include "k_dense_rows.h"

namespace riann {

namespace {

struct Shape {
    int dp, waves, cols;
};

// the default of each width first (launched by k_dense_rows.hip)
constexpr Shape kShapes[] = {
    {32, 4, 4},  {32, 4, 6},  {32, 8, 4},  {32, 4, 2},
    {64, 4, 4},  {64, 4, 6},  {64, 8, 4},  {64, 4, 2},
    {96, 4, 4},  {96, 4, 6},  {96, 8, 4},  {96, 4, 2},
    {128, 4, 4}, {128, 8, 4}, {128, 4, 2}, {128, 4, 3},
    {160, 4, 4}, {160, 8, 4}, {160, 4, 2}, {160, 4, 3},
    {192, 4, 4}, {192, 8, 4}, {192, 4, 2}, {192, 4, 3},
    {224, 4, 2}, {224, 8, 2},
    {256, 4, 2}, {256, 8, 2},
};

template <int DP>
hipError_t launch_shape_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                          hipStream_t st) {
    const int wv = ix.row_waves, qb = ix.row_cols;
    if constexpr (DP <= 96) {
        if (wv == 4 && qb == 6) return launch_rows_t<DP, 4, 6>(ix, fb, w, st);
        if (wv == 8 && qb == 4) return launch_rows_t<DP, 8, 4>(ix, fb, w, st);
        if (wv == 4 && qb == 2) return launch_rows_t<DP, 4, 2>(ix, fb, w, st);
    } else if constexpr (DP <= 192) {
        if (wv == 8 && qb == 4) return launch_rows_t<DP, 8, 4>(ix, fb, w, st);
        if (wv == 4 && qb == 2) return launch_rows_t<DP, 4, 2>(ix, fb, w, st);
        if (wv == 4 && qb == 3) return launch_rows_t<DP, 4, 3>(ix, fb, w, st);
    } else {
        if (wv == 8 && qb == 2) return launch_rows_t<DP, 8, 2>(ix, fb, w, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int dense_rows_shapes(int Dp, int *waves, int *cols, int max) {
    int n = 0;
    for (const Shape &s : kShapes) {
        if (s.dp != Dp) continue;
        if (n < max) {
            if (waves) waves[n] = s.waves;
            if (cols) cols[n] = s.cols;
        }
        ++n;
    }
    return n;
}

hipError_t launch_dense_rows_shape(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                                   hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_shape_t<32>(ix, fb, w, st);
    case 64: return launch_shape_t<64>(ix, fb, w, st);
    case 96: return launch_shape_t<96>(ix, fb, w, st);
    case 128: return launch_shape_t<128>(ix, fb, w, st);
    case 160: return launch_shape_t<160>(ix, fb, w, st);
    case 192: return launch_shape_t<192>(ix, fb, w, st);
    case 224: return launch_shape_t<224>(ix, fb, w, st);
    case 256: return launch_shape_t<256>(ix, fb, w, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace riann
