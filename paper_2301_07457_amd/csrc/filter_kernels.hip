// Cone filter of element fields, per phase:
//   H_ef = max(0, rf - |c_e - c_f|)  (centres e, f; distances in element widths),
//   truncated at the grid edge, with S_e = sum_f H_ef:
//   density           out_e = sum_f H_ef in_f / S_e
//   density adjoint   out_e = sum_f H_ef (in_f / S_f)      (H is symmetric)
//   sensitivity       out_e = sum_f H_ef x_f in_f / (max(gmin, x_e) S_e)
//
// A stencil gather that is bound by vector FP64 arithmetic and LDS reads,
// not by HBM: each output reads (2R+1)^2 neighbours, R = ceil(rf) - 1.
// A workgroup of four waves owns a 64 x 32 tile of one phase; the tile and
// its R-wide halo are staged once in LDS (values outside the grid are 0).
// Lane l of wave w forms the 8 outputs of column l, rows 8w .. 8w+7: for
// each column offset di it takes the weight column w[.][di] from a small
// table in device memory through scalar loads (the weights are the same
// for every lane) and walks the 8 + 2R tile rows once, each value feeding
// up to 8 accumulators (R is a template parameter, so these loops
// unroll).  S_e, the sum of the weights over the part of the stencil
// inside the grid, is a rectangle sum of a 2-D prefix table of the weights
// stored after them (four reads).  The phases of a tile are consecutive
// workgroups, so the interleaved phase values of a row are fetched from
// HBM once.
#include "filter_kernels.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace mtomg {

namespace {

constexpr int FT_X = 64, FT_RY = 8, FT_WAVES = 4, FT_Y = FT_RY * FT_WAVES, FT_THREADS = 64 * FT_WAVES;

// S_e of element (i, j) from the prefix table P[(2R+2)^2], where
// P[a][b] sums the weights of stencil rows dj < a - R and columns
// di < b - R.
template <int R>
__device__ __forceinline__ double weight_sum(const double* P, int i, int j, int nx, int ny) {
    constexpr int W1 = 2 * R + 2;
    const int a0 = R - min(j, R), a1 = R + 1 + min(ny - 1 - j, R);
    const int b0 = R - min(i, R), b1 = R + 1 + min(nx - 1 - i, R);
    return (P[a1 * W1 + b1] - P[a0 * W1 + b1]) - (P[a1 * W1 + b0] - P[a0 * W1 + b0]);
}

template <int R>
__global__ __launch_bounds__(FT_THREADS) void k_cone_filter(int nx, int ny, int m, int mode, double gmin,
                                                            const double* __restrict__ tab,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ in,
                                                            double* __restrict__ out) {
    constexpr int W = 2 * R + 1;
    constexpr int TW = FT_X + 2 * R, TH = FT_Y + 2 * R;
    extern __shared__ double tile[];   // [TH][TW]
    // the weights are read through the constant address space, so the
    // uniform loads of the main loop become scalar loads
    typedef const __attribute__((address_space(4))) double cdouble;
    cdouble* wcol = (cdouble*)tab;     // [W][W] weights, column di at wcol[di * W]
    const double* P = tab + W * W;     // [W + 1][W + 1] prefix sums
    const int k = blockIdx.x;
    const int bx = blockIdx.y * FT_X, by = blockIdx.z * FT_Y;
    // every load of the tile is issued before the first is used (one
    // memory round trip per workgroup, not one per element)
    constexpr int NL = (TW * TH + FT_THREADS - 1) / FT_THREADS;
    double v[NL], xv[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int t = threadIdx.x + q * FT_THREADS;
        const int gx = bx - R + t % TW, gy = by - R + t / TW;
        const bool ok = t < TW * TH && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        const size_t e = ok ? ((size_t)gy * nx + gx) * m + k : 0;
        v[q] = ok ? in[e] : 0.0;
        xv[q] = (ok && mode == FILTER_SENSITIVITY) ? x[e] : 1.0;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int t = threadIdx.x + q * FT_THREADS;
        if (t >= TW * TH) break;
        double val = v[q] * xv[q];
        if (mode == FILTER_DENSITY_ADJOINT && val != 0.0) {
            const int gx = bx - R + t % TW, gy = by - R + t / TW;
            val /= weight_sum<R>(P, gx, gy, nx, ny);
        }
        tile[t] = val;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[FT_RY];
#pragma unroll
    for (int r = 0; r < FT_RY; ++r) acc[r] = 0.0;
    const double* trow = tile + wave * FT_RY * TW + lane;
#pragma unroll 1
    for (int di = 0; di < W; ++di) {
        double wc[W];
#pragma unroll
        for (int dj = 0; dj < W; ++dj) wc[dj] = wcol[di * W + dj];
#pragma unroll
        for (int jj = 0; jj < FT_RY + 2 * R; ++jj) {
            const double v = trow[jj * TW + di];
#pragma unroll
            for (int r = 0; r < FT_RY; ++r) {
                const int dj = jj - r;
                if (dj >= 0 && dj < W) acc[r] = fma(wc[dj], v, acc[r]);
            }
        }
    }

    const int i = bx + lane;
    if (i >= nx) return;
    double xe[FT_RY];
#pragma unroll
    for (int r = 0; r < FT_RY; ++r) {
        const int j = by + wave * FT_RY + r;
        xe[r] = (mode == FILTER_SENSITIVITY && j < ny) ? x[((size_t)j * nx + i) * m + k] : 1.0;
    }
#pragma unroll
    for (int r = 0; r < FT_RY; ++r) {
        const int j = by + wave * FT_RY + r;
        if (j >= ny) break;
        double o = acc[r];
        if (mode == FILTER_DENSITY) o /= weight_sum<R>(P, i, j, nx, ny);
        else if (mode == FILTER_SENSITIVITY) o /= fmax(gmin, xe[r]) * weight_sum<R>(P, i, j, nx, ny);
        out[((size_t)j * nx + i) * m + k] = o;
    }
}

template <int R>
void launch_r(hipStream_t st, int nx, int ny, int m, int mode, double gmin, const double* tab, const double* x,
              const double* in, double* out) {
    const size_t lds = sizeof(double) * (FT_X + 2 * R) * (FT_Y + 2 * R);
    const dim3 grid(m, (nx + FT_X - 1) / FT_X, (ny + FT_Y - 1) / FT_Y);
    hipLaunchKernelGGL(k_cone_filter<R>, grid, dim3(FT_THREADS), lds, st, nx, ny, m, mode, gmin, tab, x, in, out);
}

}  // namespace

int filter_radius_cells(double rf) { return rf <= 1.0 ? 0 : (int)ceil(rf) - 1; }

void filter_table(double rf, double* tab) {
    const int R = filter_radius_cells(rf), W = 2 * R + 1, W1 = W + 1;
    double* w = tab;
    double* P = tab + W * W;
    for (int di = -R; di <= R; ++di)
        for (int dj = -R; dj <= R; ++dj)
            w[(di + R) * W + dj + R] = std::max(0.0, rf - std::sqrt((double)(di * di + dj * dj)));
    // running sums along each stencil row (dj), then down the columns
    for (int a = 0; a < W1; ++a) {
        double s = 0.0;
        P[a * W1] = 0.0;
        for (int b = 0; b < W; ++b) {
            if (a > 0) s += w[b * W + (a - 1)];
            P[a * W1 + b + 1] = s;
        }
    }
    for (int a = 1; a < W1; ++a)
        for (int b = 0; b < W1; ++b) P[a * W1 + b] += P[(a - 1) * W1 + b];
}

// ---------------------------------------------------------------------------
// The weight table in static device memory, for callers that cannot allocate
// ---------------------------------------------------------------------------
namespace {

// One table of the largest radius per GPU, held until the process ends.
// Host code must not pass this name to a kernel (on the host it is a
// stand-in, not a device address): filter_static_table() returns the
// device address of this GPU's copy.
static __device__ __align__(256) double scratch[FILTER_TAB_MAX];

constexpr int MAX_DEVICES = 64;
double* scratch_ptr[MAX_DEVICES] = {};
std::mutex scratch_mu;

// filter_table(rf) built on the device, in the host's operation order
// (same weights, same running sums), by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_filter_table(double rf, int R, double* __restrict__ tab) {
    const int W = 2 * R + 1, W1 = W + 1;
    double* w = tab;
    double* P = tab + W * W;
    const int t = threadIdx.x;
    if (t < W * W) {
        const int di = t / W - R, dj = t % W - R;
        w[t] = fmax(0.0, rf - sqrt((double)(di * di + dj * dj)));
    }
    __syncthreads();
    if (t < W1) {   // running sums along stencil row a = t
        double s = 0.0;
        P[t * W1] = 0.0;
        for (int b = 0; b < W; ++b) {
            if (t > 0) s += w[b * W + (t - 1)];
            P[t * W1 + b + 1] = s;
        }
    }
    __syncthreads();
    if (t < W1)     // then down column b = t
        for (int a = 1; a < W1; ++a) P[a * W1 + t] += P[(a - 1) * W1 + t];
}

}  // namespace

hipError_t filter_static_table(double** tab) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        // this device's copy of the array, looked up once with the device current
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *tab = scratch_ptr[dev];
    return hipSuccess;
}

void launch_filter_table(hipStream_t st, double rf, double* tab) {
    hipLaunchKernelGGL(k_filter_table, dim3(1), dim3(1024), 0, st, rf, filter_radius_cells(rf), tab);
}

void launch_cone_filter(hipStream_t st, int nx, int ny, int m, double rf, int mode, double gmin, const double* tab,
                        const double* x, const double* in, double* out) {
    switch (filter_radius_cells(rf)) {
#define MTOMG_FILTER_CASE(r) \
    case r: launch_r<r>(st, nx, ny, m, mode, gmin, tab, x, in, out); break;
        MTOMG_FILTER_CASE(0) MTOMG_FILTER_CASE(1) MTOMG_FILTER_CASE(2) MTOMG_FILTER_CASE(3)
        MTOMG_FILTER_CASE(4) MTOMG_FILTER_CASE(5) MTOMG_FILTER_CASE(6) MTOMG_FILTER_CASE(7)
        MTOMG_FILTER_CASE(8) MTOMG_FILTER_CASE(9) MTOMG_FILTER_CASE(10) MTOMG_FILTER_CASE(11)
        MTOMG_FILTER_CASE(12) MTOMG_FILTER_CASE(13) MTOMG_FILTER_CASE(14) MTOMG_FILTER_CASE(15)
#undef MTOMG_FILTER_CASE
        default: break;
    }
}

}  // namespace mtomg
