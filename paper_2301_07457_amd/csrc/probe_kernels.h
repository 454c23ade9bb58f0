// Streaming kernels for the practical HBM ceiling (see probe_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mtomg {

enum ProbeKind { PROBE_READ = 0, PROBE_COPY = 1, PROBE_TRIAD = 2 };

// Workgroups of a probe launch: 8 per compute unit of the current device.
int probe_blocks();

// One pass over n doubles (n even, arrays 16-byte aligned):
//   READ:  sum of a, one double per workgroup written to b[0 .. blocks-1];
//   COPY:  b = a;
//   TRIAD: a = b + 3 c.
void launch_probe(hipStream_t st, int kind, double* a, double* b, double* c, size_t n, int blocks);

}  // namespace mtomg
