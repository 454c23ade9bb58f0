// Device-side building blocks shared by the solver kernels (gfx950, wave64).
//
// Element operator.  Every level of the hierarchy is a grid of square
// elements whose stiffness is the integral of E(xi, eta) B^T D B over the
// element (Eq. 7), with bilinear B (Eq. 9) and the plane-stress D (Eq. 8),
// in local coordinates xi, eta in [0, 1] (the 2D result does not depend on
// the element size).  On the finest grid E is constant per element (Eq. 5);
// on a coarse grid the Galerkin product P^T K P of the finer operator is,
// element by element, the same integral with the coarse bilinear basis and
// the fine modulus field E underneath it.  Because the strains of a bilinear
// field are linear in xi and eta, that integral only sees the six moments
//   M00 = int E, M10 = int E xi, M01 = int E eta,
//   M20 = int E xi^2, M11 = int E xi eta, M02 = int E eta^2,
// so one coarse element is stored as 6 numbers instead of an 8x8 matrix.
// A fine element of modulus E has moments E * (1, 1/2, 1/2, 1/3, 1/4, 1/3).
//
// Local element nodes are 0 (0,0), 1 (1,0), 2 (1,1), 3 (0,1); element (i,j)
// has nodes (i,j), (i+1,j), (i+1,j+1), (i,j+1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mtomg {

constexpr int WAVE = 64;
constexpr int WAVES_PER_WG = 4;
constexpr int WG_THREADS = WAVE * WAVES_PER_WG;

template <typename T> struct V2 { T x, y; };

template <typename T> struct Mom { T m00, m10, m01, m20, m11, m02; };

// Material constants of Eq. (8) for unit modulus: c = 1/(1-nu^2),
// cnu = c*nu, g = c*(1-nu)/2 (shear).
template <typename T> struct Mat { T c, cnu, g, omega; };

template <typename T>
__device__ __forceinline__ Mom<T> mom_zero() { return Mom<T>{T(0), T(0), T(0), T(0), T(0), T(0)}; }

template <typename T>
__device__ __forceinline__ Mom<T> mom_const(T E) {
    return Mom<T>{E, E * T(0.5), E * T(0.5), E * (T(1) / T(3)), E * T(0.25), E * (T(1) / T(3))};
}

// Nodal forces f = K_e u_e of one element from its moments.
// The bilinear displacement has du_x/dxi = Ax + Bx eta, du_x/deta = Cx + Bx xi
// (same for y); stresses sigma_xx, sigma_yy, tau are linear in (1, xi, eta)
// and each nodal force integrates E * (linear shape derivative) * stress.
// With UNIFORM (moments of a constant modulus E = m.m00, the finest grid)
// E is folded into the material constants and the moments of the unit
// modulus (1, 1/2, 1/2, 1/3, 1/4, 1/3) become literals.
template <bool UNIFORM = false, typename T>
__device__ __forceinline__ void elem_force(const Mom<T>& m, const Mat<T>& k,
                                           const V2<T>& u0, const V2<T>& u1,
                                           const V2<T>& u2, const V2<T>& u3,
                                           V2<T>& f0, V2<T>& f1, V2<T>& f2, V2<T>& f3) {
    const T Ax = u1.x - u0.x, Cx = u3.x - u0.x, Bx = (u0.x - u1.x) + (u2.x - u3.x);
    const T Ay = u1.y - u0.y, Cy = u3.y - u0.y, By = (u0.y - u1.y) + (u2.y - u3.y);
    if constexpr (UNIFORM) {
        const T h = T(0.5), q = T(0.25), r = T(1) / T(3);
        const T cE = k.c * m.m00, nE = k.cnu * m.m00, gE = k.g * m.m00;
        const T s0 = cE * Ax + nE * Cy, s1 = nE * By, s2 = cE * Bx;
        const T w0 = nE * Ax + cE * Cy, w1 = cE * By, w2 = nE * Bx;
        const T t0 = gE * (Cx + Ay), t1 = gE * Bx, t2 = gE * By;
        const T Sxx = s0 + h * (s1 + s2);
        const T Sxe = h * s0 + q * s1 + r * s2;
        const T Syy = w0 + h * (w1 + w2);
        const T Syx = h * w0 + r * w1 + q * w2;
        const T Tt = t0 + h * (t1 + t2);
        const T Ttx = h * t0 + r * t1 + q * t2;
        const T Tte = h * t0 + q * t1 + r * t2;
        const T a = Sxx - Sxe, b = Tt - Ttx, c = Syy - Syx, d = Tt - Tte;
        f0.x = -a - b;   f1.x = a - Ttx;  f2.x = Sxe + Ttx; f3.x = b - Sxe;
        f0.y = -c - d;   f1.y = d - Syx;  f2.y = Syx + Tte; f3.y = c - Tte;
        return;
    }
    // sigma_xx = s0 + s1 xi + s2 eta; sigma_yy = w0 + w1 xi + w2 eta; tau = t0 + t1 xi + t2 eta
    const T s0 = k.c * Ax + k.cnu * Cy, s1 = k.cnu * By, s2 = k.c * Bx;
    const T w0 = k.cnu * Ax + k.c * Cy, w1 = k.c * By, w2 = k.cnu * Bx;
    const T t0 = k.g * (Cx + Ay), t1 = k.g * Bx, t2 = k.g * By;
    const T Sxx = s0 * m.m00 + s1 * m.m10 + s2 * m.m01;   // int E sxx
    const T Sxe = s0 * m.m01 + s1 * m.m11 + s2 * m.m02;   // int E sxx eta
    const T Syy = w0 * m.m00 + w1 * m.m10 + w2 * m.m01;   // int E syy
    const T Syx = w0 * m.m10 + w1 * m.m20 + w2 * m.m11;   // int E syy xi
    const T Tt = t0 * m.m00 + t1 * m.m10 + t2 * m.m01;    // int E tau
    const T Ttx = t0 * m.m10 + t1 * m.m20 + t2 * m.m11;   // int E tau xi
    const T Tte = t0 * m.m01 + t1 * m.m11 + t2 * m.m02;   // int E tau eta
    const T a = Sxx - Sxe, b = Tt - Ttx, c = Syy - Syx, d = Tt - Tte;
    f0.x = -a - b;   f1.x = a - Ttx;  f2.x = Sxe + Ttx; f3.x = b - Sxe;
    f0.y = -c - d;   f1.y = d - Syx;  f2.y = Syx + Tte; f3.y = c - Tte;
}

// Diagonal of K_e at the 8 local DOFs:
// K[ax][ax] = int E (c (dN_a/dxi)^2 + g (dN_a/deta)^2), K[ay][ay] with c and g swapped.
// With UNIFORM (moments of a constant modulus E = m.m00, the finest grid)
// every integral of a squared shape derivative is E/3, so all eight
// entries are E (c + g) / 3.
template <bool UNIFORM = false, typename T>
__device__ __forceinline__ void elem_diag(const Mom<T>& m, const Mat<T>& k,
                                          V2<T>& d0, V2<T>& d1, V2<T>& d2, V2<T>& d3) {
    if constexpr (UNIFORM) {
        const T v = m.m00 * ((k.c + k.g) * (T(1) / T(3)));
        d0 = d1 = d2 = d3 = V2<T>{v, v};
        return;
    }
    const T P0 = m.m00 - T(2) * m.m01 + m.m02;  // int E (1-eta)^2
    const T P1 = m.m02;                          // int E eta^2
    const T Q0 = m.m00 - T(2) * m.m10 + m.m20;  // int E (1-xi)^2
    const T Q1 = m.m20;                          // int E xi^2
    d0.x = k.c * P0 + k.g * Q0; d0.y = k.c * Q0 + k.g * P0;
    d1.x = k.c * P0 + k.g * Q1; d1.y = k.c * Q1 + k.g * P0;
    d2.x = k.c * P1 + k.g * Q1; d2.y = k.c * Q1 + k.g * P1;
    d3.x = k.c * P1 + k.g * Q0; d3.y = k.c * Q0 + k.g * P1;
}

// Moments of a parent element from its four children (s, t) in {0,1}^2,
// each given in its own local coordinates: xi = (s + xi')/2, eta = (t + eta')/2,
// d xi d eta = d xi' d eta' / 4.
template <typename T>
__device__ __forceinline__ void mom_accumulate_child(Mom<T>& P, const Mom<T>& c, int s, int t) {
    const T S = T(s), U = T(t);
    P.m00 += T(0.25) * c.m00;
    P.m10 += T(0.125) * (S * c.m00 + c.m10);
    P.m01 += T(0.125) * (U * c.m00 + c.m01);
    P.m20 += T(0.0625) * (S * c.m00 + T(2) * S * c.m10 + c.m20);
    P.m11 += T(0.0625) * (S * U * c.m00 + S * c.m01 + U * c.m10 + c.m11);
    P.m02 += T(0.0625) * (U * c.m00 + T(2) * U * c.m01 + c.m02);
}

// omega / d, the damped-Jacobi weight of a node.  In FP32 (the multigrid
// cycle's precision there) by the hardware reciprocal (1 ulp) instead of the
// correctly rounded division sequence (about ten instructions); in FP64 the
// division itself.
__device__ __forceinline__ float w_over(float omega, float d) { return omega * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double w_over(double omega, double d) { return omega / d; }

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
// the same for every lane of a wave: readfirstlane lets the compiler keep
// row indices, masks and addresses derived from it in scalar registers
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Neighbour lanes by whole-wave DPP shifts (a VALU operand modifier, no
// LDS round trip): from_left gives lane l the value of lane l-1 (lane 0
// gets 0), from_right the value of lane l+1 (lane 63 gets 0).  Edge lanes
// are halo lanes in every kernel, so their values are never used.
constexpr int DPP_WAVE_SHR1 = 0x138, DPP_WAVE_SHL1 = 0x130;
template <int CTRL> __device__ __forceinline__ int dpp_shift(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL> __device__ __forceinline__ float dpp_shift(float v) {
    return __int_as_float(dpp_shift<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_shift(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_shift<CTRL>((int)(b & 0xffffffff));
    const int hi = dpp_shift<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T> __device__ __forceinline__ T from_left(T v) { return dpp_shift<DPP_WAVE_SHR1>(v); }
template <typename T> __device__ __forceinline__ T from_right(T v) { return dpp_shift<DPP_WAVE_SHL1>(v); }

template <typename T> __device__ __forceinline__ V2<T> from_left(V2<T> v) {
    return V2<T>{from_left(v.x), from_left(v.y)};
}
template <typename T> __device__ __forceinline__ V2<T> from_right(V2<T> v) {
    return V2<T>{from_right(v.x), from_right(v.y)};
}

template <typename T> __device__ __forceinline__ V2<T> operator+(V2<T> a, V2<T> b) { return V2<T>{a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ V2<T> operator-(V2<T> a, V2<T> b) { return V2<T>{a.x - b.x, a.y - b.y}; }

// Fixed-order wave sum (tree over lane distance 32, 16, ..., 1); the result
// is valid in lane 0.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, WAVE);
    return v;
}

// Fixed-order workgroup sum of one double per thread (WG_THREADS threads);
// every thread gets the result.  Requires all threads of the block to call.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[WAVES_PER_WG];
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES_PER_WG; ++w) s += red[w];
    return s;
}

// Two block_sums sharing one barrier pair (each sum in block_sum's order).
__device__ __forceinline__ void block_sum2(double& a, double& b) {
    __shared__ double red[2][WAVES_PER_WG];
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if (lane_id() == 0) {
        red[0][wave_id()] = a;
        red[1][wave_id()] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES_PER_WG; ++w) {
        sa += red[0][w];
        sb += red[1][w];
    }
    a = sa;
    b = sb;
}

// Sums of K partial arrays (p[q] holds n[q] >= 1 entries, n[q] used) in a
// fixed order, identical in every block that computes them: thread t adds
// entries t, t + WG_THREADS, ... in increasing order, then the wave and
// workgroup trees of block_sum.  Loads go out eight per thread and array at
// a time, all before the first add (out-of-range slots load a valid entry
// and are not added), and the K reductions share one barrier pair.
// issue() sends the first eight loads per thread and array; a kernel calls
// it before its own tile loads, so the two latencies overlap, and finish()
// later (all threads of the block).
template <int K>
struct PartialSums {
    static constexpr int U = 8;
    const double* p[K];
    int n[K];
    double v[K][U];

    __device__ __forceinline__ void load_chunk(int base) {
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = base + threadIdx.x + u * WG_THREADS;
                v[q][u] = p[q][max(min(k, n[q] - 1), 0)];
            }
    }

    __device__ __forceinline__ void issue(const double* const (&ps)[K], const int (&ns)[K]) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            p[q] = ps[q];
            n[q] = ns[q];
        }
        load_chunk(0);
    }

    __device__ __forceinline__ void add_chunk(int base, double (&s)[K]) const {
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = base + threadIdx.x + u * WG_THREADS;
                s[q] = (k < n[q]) ? s[q] + v[q][u] : s[q];
            }
    }

    __device__ __forceinline__ void finish(double (&out)[K]) {
        double s[K];
        int nmax = 0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            s[q] = 0.0;
            nmax = max(nmax, n[q]);
        }
        // the values issue() loaded enter here and no earlier: without this
        // the compiler may hoist the first adds (and their wait for the
        // loads) above the caller's tile loads, serialising the two
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) asm volatile("" : "+v"(v[q][u]) : : "memory");
        add_chunk(0, s);   // the chunk issue() loaded, outside the loop
        for (int base = U * WG_THREADS; base < nmax; base += U * WG_THREADS) {
            load_chunk(base);
            add_chunk(base, s);
        }
        __shared__ double red[K][WAVES_PER_WG];
#pragma unroll
        for (int q = 0; q < K; ++q) s[q] = wave_sum(s[q]);
        __syncthreads();
        if (lane_id() == 0) {
#pragma unroll
            for (int q = 0; q < K; ++q) red[q][wave_id()] = s[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES_PER_WG; ++w) t += red[q][w];
            out[q] = t;
        }
    }
};

// The sums of PartialSums in one call.  Requires all threads of the block.
template <int K>
__device__ __forceinline__ void sum_partials_k(const double* const (&p)[K], const int (&n)[K], double (&out)[K]) {
    PartialSums<K> ps;
    ps.issue(p, n);
    ps.finish(out);
}

// Sum of n >= 1 partials in a fixed order; identical in every block that calls it.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n) {
    const double* ps[1] = {p};
    const int ns[1] = {n};
    double out[1];
    sum_partials_k<1>(ps, ns, out);
    return out[0];
}


// ---------------------------------------------------------------------------
// tile mapping: consecutive tiles land on the same XCD (workgroups are
// dispatched round-robin over the 8 XCDs), so vertical and horizontal halo
// reads of neighbouring tiles hit the same L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int n_tiles) {
    const int per = (n_tiles + 7) >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// State word of a system (0 = running; a null pointer reads 0).  The load is
// unconditional, so a latency-bound kernel can issue it together with its
// data loads and test it once they are in flight.
static __device__ int g_state_running = 0;   // never written
__device__ __forceinline__ int load_state(const int* w) { return *(w ? w : &g_state_running); }

// Nodal vector access with the clamped row (j = 0) and out-of-grid nodes read
// as 0.  The index is clamped into the grid and the load is always issued,
// then masked: no branch, so the loads of consecutive rows can be batched.
// use = false reads 0 (v must still point at a nodal vector of the level).
template <typename T>
__device__ __forceinline__ V2<T> load_node(const T* __restrict__ v, int nx, int ny, int i, int j,
                                           bool use = true) {
    const bool ok = use & (i >= 0) & (i <= nx) & (j >= 1) & (j <= ny);
    const int ic = min(max(i, 0), nx), jc = min(max(j, 1), ny);
    const size_t n = (size_t)jc * (nx + 1) + ic;
    // the clamped address always holds finite data, so multiplying by the
    // 0/1 mask zeroes it exactly; the value is used unconditionally, which
    // keeps the load out of any branch
    const T msk = ok ? T(1) : T(0);
    if constexpr (sizeof(T) == 4) {
        const float2 w = reinterpret_cast<const float2*>(v)[n];
        return V2<T>{w.x * msk, w.y * msk};
    } else {
        const double2 w = reinterpret_cast<const double2*>(v)[n];
        return V2<T>{w.x * msk, w.y * msk};
    }
}

// The same load without the mask: the value at the clamped address, for
// callers that select every use of it by the node's own validity anyway.
template <typename T>
__device__ __forceinline__ V2<T> load_node_clamped(const T* __restrict__ v, int nx, int ny, int i, int j) {
    const int ic = min(max(i, 0), nx), jc = min(max(j, 1), ny);
    const size_t n = (size_t)jc * (nx + 1) + ic;
    if constexpr (sizeof(T) == 4) {
        const float2 w = reinterpret_cast<const float2*>(v)[n];
        return V2<T>{w.x, w.y};
    } else {
        const double2 w = reinterpret_cast<const double2*>(v)[n];
        return V2<T>{w.x, w.y};
    }
}

template <typename T>
__device__ __forceinline__ void store_node(T* __restrict__ v, int nx, int i, int j, V2<T> a) {
    const size_t n = (size_t)j * (nx + 1) + i;
    if constexpr (sizeof(T) == 4) {
        reinterpret_cast<float2*>(v)[n] = make_float2(a.x, a.y);
    } else {
        reinterpret_cast<double2*>(v)[n] = make_double2(a.x, a.y);
    }
}

// Operator data of one level: the finest grid stores E per element, a
// coarse grid stores 6 moment planes (plane stride nx*ny).
template <typename T> struct LevelOp {
    int nx, ny;
    const T* __restrict__ data;
};

template <typename T, bool FINE>
__device__ __forceinline__ Mom<T> load_elem(const LevelOp<T>& L, int i, int j) {
    const bool ok = (i >= 0) & (i < L.nx) & (j >= 0) & (j < L.ny);
    const int ic = min(max(i, 0), L.nx - 1), jc = min(max(j, 0), L.ny - 1);
    const size_t e = (size_t)jc * L.nx + ic;
    const T msk = ok ? T(1) : T(0);   // see load_node
    if constexpr (FINE) {
        return mom_const<T>(L.data[e] * msk);
    } else {
        const size_t ps = (size_t)L.nx * L.ny;
        return Mom<T>{L.data[e] * msk, L.data[ps + e] * msk, L.data[2 * ps + e] * msk,
                      L.data[3 * ps + e] * msk, L.data[4 * ps + e] * msk, L.data[5 * ps + e] * msk};
    }
}

}  // namespace mtomg
