// Cone filter of element fields (the sensitivity filtering of Section 4,
// radius rf of Table 2): launcher shared by the C ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace mtomg {

enum FilterMode { FILTER_DENSITY = 0, FILTER_DENSITY_ADJOINT = 1, FILTER_SENSITIVITY = 2 };

// Largest supported radius in elements (weights reach offsets ceil(rf) - 1).
constexpr double FILTER_MAX_RF = 16.0;
// Doubles of the largest weight table (31 x 31 weights + 32 x 32 prefix sums).
constexpr int FILTER_TAB_MAX = 31 * 31 + 32 * 32;

// Stencil half-width R = ceil(rf) - 1 (0 for rf <= 1).
int filter_radius_cells(double rf);

// Host: the weight table the kernel reads, W = 2R + 1: weights
// max(0, rf - |(di, dj)|) by columns (tab[(di + R) W + dj + R]), then the
// prefix sums P[a][b] over stencil rows < a and columns < b ((W+1)^2,
// row-major).
void filter_table(double rf, double* tab);

// Device address of this GPU's statically allocated weight table
// (FILTER_TAB_MAX doubles, shared by every call on the GPU until the process
// ends); looked up on the first call per device, with that device current.
hipError_t filter_static_table(double** tab);

// filter_table(rf) written into tab (device) by a kernel on st.
void launch_filter_table(hipStream_t st, double rf, double* tab);

// in, x, out: device [ny][nx][m] FP64; x is read by FILTER_SENSITIVITY only;
// tab: device copy of filter_table(rf).  Asynchronous on st.
void launch_cone_filter(hipStream_t st, int nx, int ny, int m, double rf, int mode, double gmin, const double* tab,
                        const double* x, const double* in, double* out);

}  // namespace mtomg
