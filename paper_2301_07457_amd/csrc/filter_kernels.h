// Cone filter of element fields (the sensitivity filtering of Section 4,
// radius rf of Table 2): launcher shared by the C ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace mtomg {

enum FilterMode { FILTER_DENSITY = 0, FILTER_DENSITY_ADJOINT = 1, FILTER_SENSITIVITY = 2 };

// Largest supported radius in elements (weights reach offsets ceil(rf) - 1).
constexpr double FILTER_MAX_RF = 16.0;

// in, x, out: device [ny][nx][m] FP64; x is read by FILTER_SENSITIVITY only.
// Asynchronous on st.
void launch_cone_filter(hipStream_t st, int nx, int ny, int m, double rf, int mode, double gmin, const double* x,
                        const double* in, double* out);

}  // namespace mtomg
