// Streaming kernels that measure the practical HBM ceiling of this GPU, for
// the roofline the solver's bandwidth-bound kernels are held against: a
// read-only pass (a sum, one value written per workgroup), a copy and a
// triad (a = b + s c).  16-byte loads and stores, four per thread and step
// in flight, a grid of 8 workgroups of 256 threads per compute unit walking
// the arrays with a grid stride.
#include <hip/hip_runtime.h>

#include "probe_kernels.h"

namespace mtomg {

namespace {

constexpr int PT = 256, UNROLL = 4;

__global__ __launch_bounds__(PT) void k_read(const double2* __restrict__ a, size_t n2, double* __restrict__ out) {
    double s = 0.0;
    const size_t stride = (size_t)gridDim.x * PT * UNROLL;
    for (size_t base = (size_t)blockIdx.x * PT * UNROLL + threadIdx.x; base < n2; base += stride) {
        double2 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const size_t k = base + (size_t)u * PT;
            v[u] = k < n2 ? a[k] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) s += v[u].x + v[u].y;
    }
    // one value per workgroup keeps the loads alive
    __shared__ double red[PT];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < PT; ++k) t += red[k];
        out[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(PT) void k_copy(const double2* __restrict__ a, double2* __restrict__ b, size_t n2) {
    const size_t stride = (size_t)gridDim.x * PT * UNROLL;
    for (size_t base = (size_t)blockIdx.x * PT * UNROLL + threadIdx.x; base < n2; base += stride) {
        double2 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const size_t k = base + (size_t)u * PT;
            if (k < n2) v[u] = a[k];
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const size_t k = base + (size_t)u * PT;
            if (k < n2) b[k] = v[u];
        }
    }
}

__global__ __launch_bounds__(PT) void k_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                              const double2* __restrict__ c, double s, size_t n2) {
    const size_t stride = (size_t)gridDim.x * PT * UNROLL;
    for (size_t base = (size_t)blockIdx.x * PT * UNROLL + threadIdx.x; base < n2; base += stride) {
        double2 vb[UNROLL], vc[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const size_t k = base + (size_t)u * PT;
            if (k < n2) {
                vb[u] = b[k];
                vc[u] = c[k];
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const size_t k = base + (size_t)u * PT;
            if (k < n2) a[k] = make_double2(vb[u].x + s * vc[u].x, vb[u].y + s * vc[u].y);
        }
    }
}

}  // namespace

int probe_blocks() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return 8 * cus;
}

void launch_probe(hipStream_t st, int kind, double* a, double* b, double* c, size_t n, int blocks) {
    const size_t n2 = n / 2;
    const double2* ca = reinterpret_cast<const double2*>(a);
    switch (kind) {
        case PROBE_READ:
            hipLaunchKernelGGL(k_read, dim3(blocks), dim3(PT), 0, st, ca, n2, b);
            break;
        case PROBE_COPY:
            hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(PT), 0, st, ca, reinterpret_cast<double2*>(b), n2);
            break;
        default:
            hipLaunchKernelGGL(k_triad, dim3(blocks), dim3(PT), 0, st, reinterpret_cast<double2*>(a),
                               reinterpret_cast<const double2*>(b), reinterpret_cast<const double2*>(c), 3.0, n2);
            break;
    }
}

}  // namespace mtomg
