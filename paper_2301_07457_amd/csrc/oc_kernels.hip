// Optimality-criteria pair update of the alternating active-phase loop
// (Section 4); the arithmetic is described in oc_kernels.h.
//
// Passes.  k_oc_prep forms q, lo, hi per element and per-workgroup partial
// records for the bracket of t; k_oc_bracket (one workgroup) reduces them
// and sets the first candidate.  Each Newton pass is k_oc_eval (S(t) and
// its slope sum_{lo < q t < hi} q, per-workgroup records) and k_oc_next
// (one workgroup: reduce, new bracket and candidate); k_oc_apply writes the
// pair and k_oc_finish records the largest change and lambda.  Each of the
// OC_BLOCKS workgroups owns a fixed, strided set of elements and the
// one-workgroup kernels sum the records in block order, so every pass is
// deterministic; the records cross workgroups only at kernel boundaries.
#include <math.h>

#include <algorithm>

#include "device_common.h"
#include "oc_kernels.h"

namespace mtomg {

namespace {

constexpr int REC = 8;   // doubles per partial record

// Fixed-order sums (or min / max) of the records' fields, by the whole block.
__device__ __forceinline__ double block_min(double v) {
    __shared__ double red[OC_THREADS / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < OC_THREADS / 64; ++w) r = fmin(r, red[w]);
    return r;
}
__device__ __forceinline__ double block_max(double v) { return -block_min(-v); }

// Sum over records 0 .. nrec-1 of field f: thread t adds records t, t + 256, ...
__device__ __forceinline__ double records_sum(const double* part, int nrec, int f) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nrec; k += OC_THREADS) v += part[(size_t)k * REC + f];
    return block_sum(v);
}
__device__ __forceinline__ double records_min(const double* part, int nrec, int f) {
    double v = INFINITY;
    for (int k = threadIdx.x; k < nrec; k += OC_THREADS) v = fmin(v, part[(size_t)k * REC + f]);
    return block_min(v);
}
__device__ __forceinline__ double records_max(const double* part, int nrec, int f) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nrec; k += OC_THREADS) v = fmax(v, part[(size_t)k * REC + f]);
    return block_max(v);
}

__device__ __forceinline__ double eta_pow(double v, double eta) { return eta == 0.5 ? sqrt(v) : pow(v, eta); }

// q, lo, hi per element; records: min lo/q, max hi/q (q > 0), sum lo,
// sum (q > 0 ? hi : lo), sum q.
__global__ __launch_bounds__(OC_THREADS) void k_oc_prep(OcPair op, const double* __restrict__ g,
                                                        const double* __restrict__ x, double* __restrict__ q,
                                                        double* __restrict__ lo, double* __restrict__ hi,
                                                        double* __restrict__ part) {
    double tmin = INFINITY, tmax = 0.0, slo = 0.0, shi = 0.0, sq = 0.0;
    for (int e = blockIdx.x * OC_THREADS + threadIdx.x; e < op.n_e; e += gridDim.x * OC_THREADS) {
        const double* xe = x + (size_t)e * op.m;
        const double ya = xe[op.a];
        double yb;
        if (op.b < op.m) {
            yb = xe[op.b];
        } else {
            double sum = 0.0;
            for (int i = 0; i < op.m; ++i) sum += xe[i];
            yb = 1.0 - sum;
        }
        const double gb = op.b < op.m ? g[(size_t)e * op.m + op.b] : 0.0;
        const double d = g[(size_t)e * op.m + op.a] - gb;
        const double sp = ya + yb;
        const double l = fmax(op.eps, ya - op.move);
        const double h = fmin(fmin(1.0, sp - op.eps), ya + op.move);
        const double qe = ya * eta_pow(fmax(0.0, -d), op.eta);
        q[e] = qe;
        lo[e] = l;
        hi[e] = h;
        slo += l;
        sq += qe;
        if (qe > 0.0) {
            tmin = fmin(tmin, l / qe);
            tmax = fmax(tmax, h / qe);
            shi += h;
        } else {
            shi += l;
        }
    }
    tmin = block_min(tmin);
    tmax = block_max(tmax);
    slo = block_sum(slo);
    shi = block_sum(shi);
    sq = block_sum(sq);
    if (threadIdx.x == 0) {
        double* rec = part + (size_t)blockIdx.x * REC;
        rec[0] = tmin;
        rec[1] = tmax;
        rec[2] = slo;
        rec[3] = shi;
        rec[4] = sq;
    }
}

// One workgroup: the bracket and the first candidate, or the answer at once
// when the target lies outside [S(0), S(inf)].
__global__ __launch_bounds__(OC_THREADS) void k_oc_bracket(OcPair op, const double* __restrict__ part, int nrec,
                                                           OcState* s) {
    const double tl = records_min(part, nrec, 0);
    const double thv = records_max(part, nrec, 1);
    const double Slo = records_sum(part, nrec, 2);
    const double Shi = records_sum(part, nrec, 3);
    const double Sq = records_sum(part, nrec, 4);
    if (threadIdx.x == 0) {
        double t = 0.0;
        int done = 0;
        if (!(thv > 0.0) || op.target <= Slo) {   // every element at lo (t = 0: lambda = inf)
            done = 1;
        } else if (op.target >= Shi) {              // every element with q > 0 at hi:
            t = 2.0 * thv;                          // q t >= 2 hi > hi, whatever the rounding of hi / q
            done = 1;
        } else {
            t = op.target / Sq;     // the root when no bound is active
            if (!(t > tl && t < thv)) t = sqrt(tl * thv);
        }
        s->tl = tl;
        s->th = thv;
        s->t = t;
        s->S = 0.0;
        s->change = 0.0;
        s->lambda = 0.0;
        s->done = done;
        s->passes = 0;
        s->count = 0u;
        s->pad = 0;
    }
}

// One Newton pass: S(t) and the slope per workgroup ...
__global__ __launch_bounds__(OC_THREADS) void k_oc_eval(OcPair op, const double* __restrict__ q,
                                                        const double* __restrict__ lo,
                                                        const double* __restrict__ hi,
                                                        double* __restrict__ part, const OcState* s) {
    if (s->done) return;
    const double t = s->t;
    double S = 0.0, D = 0.0;
    for (int e = blockIdx.x * OC_THREADS + threadIdx.x; e < op.n_e; e += gridDim.x * OC_THREADS) {
        const double qe = q[e], v = qe * t, l = lo[e], h = hi[e];
        S += fmin(fmax(v, l), h);
        if (v > l && v < h) D += qe;
    }
    S = block_sum(S);
    D = block_sum(D);
    if (threadIdx.x == 0) {
        double* rec = part + (size_t)blockIdx.x * REC;
        rec[0] = S;
        rec[1] = D;
    }
}

// ... and one workgroup reduces them and picks the next candidate: the
// Newton step if it stays strictly inside the bracket, else the geometric
// middle of the bracket.
__global__ __launch_bounds__(OC_THREADS) void k_oc_next(OcPair op, const double* __restrict__ part, int nrec,
                                                        OcState* s) {
    if (s->done) return;
    const double t = s->t;
    const double S = records_sum(part, nrec, 0);
    const double D = records_sum(part, nrec, 1);
    if (threadIdx.x == 0) {
        double tl = s->tl, th = s->th;
        s->S = S;
        s->passes += 1;
        if (S < op.target) tl = t;
        else th = t;
        int done = 0;
        double tn = t;
        if (fabs(S - op.target) <= 1e-14 * op.target || th - tl <= 1e-15 * th) {
            done = 1;
        } else {
            tn = D > 0.0 ? t + (op.target - S) / D : -1.0;
            if (!(tn > tl && tn < th)) tn = sqrt(tl * th);
        }
        s->tl = tl;
        s->th = th;
        s->t = tn;
        s->done = done;
    }
}

// y = clamp(q t, lo, hi) into phase a, s - y into phase b; per-workgroup
// largest change ...
__global__ __launch_bounds__(OC_THREADS) void k_oc_apply(OcPair op, const double* __restrict__ q,
                                                         const double* __restrict__ lo,
                                                         const double* __restrict__ hi, double* __restrict__ x,
                                                         double* __restrict__ part, const OcState* s) {
    const double t = s->t;
    double ch = 0.0;
    for (int e = blockIdx.x * OC_THREADS + threadIdx.x; e < op.n_e; e += gridDim.x * OC_THREADS) {
        double* xe = x + (size_t)e * op.m;
        const double ya = xe[op.a];
        const double y = fmin(fmax(q[e] * t, lo[e]), hi[e]);
        if (op.b < op.m) xe[op.b] = (ya + xe[op.b]) - y;
        xe[op.a] = y;
        ch = fmax(ch, fabs(y - ya));
    }
    ch = block_max(ch);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * REC] = ch;
}

// ... and one workgroup records the largest change and lambda = t^(-1/eta).
__global__ __launch_bounds__(OC_THREADS) void k_oc_finish(OcPair op, const double* __restrict__ part, int nrec,
                                                          OcState* s) {
    const double v = records_max(part, nrec, 0);
    if (threadIdx.x == 0) {
        const double t = s->t;
        s->change = v;
        s->lambda = t > 0.0 ? pow(t, -1.0 / op.eta) : INFINITY;
    }
}

__global__ void k_sum_cases(const double* __restrict__ in, int n_cases, size_t n, double* __restrict__ out) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int k = 0; k < n_cases; ++k) v += in[(size_t)k * n + e];
        out[e] = v;
    }
}

// Largest change of any phase (void included) per block, then one block
// takes the maximum of the block values.
__global__ __launch_bounds__(OC_THREADS) void k_oc_change(const double* __restrict__ x0,
                                                          const double* __restrict__ x, int n_e, int m,
                                                          double* __restrict__ part) {
    double ch = 0.0;
    for (int e = blockIdx.x * OC_THREADS + threadIdx.x; e < n_e; e += OC_BLOCKS * OC_THREADS) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i < m; ++i) {
            const double a = x0[(size_t)e * m + i], b = x[(size_t)e * m + i];
            ch = fmax(ch, fabs(b - a));
            s0 += a;
            s1 += b;
        }
        ch = fmax(ch, fabs((1.0 - s1) - (1.0 - s0)));
    }
    ch = block_max(ch);
    if (threadIdx.x == 0) part[blockIdx.x] = ch;
}

__global__ __launch_bounds__(OC_THREADS) void k_max_of(const double* __restrict__ part, int n, double* out) {
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += OC_THREADS) v = fmax(v, part[k]);
    v = block_max(v);
    if (threadIdx.x == 0) *out = v;
}

int blocks_for(int n_e) { return std::min(OC_BLOCKS, std::max(1, (n_e + OC_THREADS - 1) / OC_THREADS)); }

}  // namespace

size_t oc_scratch_doubles(int n_e) { return 3 * (size_t)n_e + (size_t)OC_BLOCKS * REC; }

void launch_oc_pair(hipStream_t st, const OcPair& op, const double* g, double* x, double* scratch, OcState* state) {
    double* q = scratch;
    double* lo = q + op.n_e;
    double* hi = lo + op.n_e;
    double* part = hi + op.n_e;
    const int nb = blocks_for(op.n_e);
    hipLaunchKernelGGL(k_oc_prep, dim3(nb), dim3(OC_THREADS), 0, st, op, g, x, q, lo, hi, part);
    hipLaunchKernelGGL(k_oc_bracket, dim3(1), dim3(OC_THREADS), 0, st, op, part, nb, state);
    for (int k = 0; k < OC_MAX_PASSES; ++k) {
        hipLaunchKernelGGL(k_oc_eval, dim3(nb), dim3(OC_THREADS), 0, st, op, q, lo, hi, part, state);
        hipLaunchKernelGGL(k_oc_next, dim3(1), dim3(OC_THREADS), 0, st, op, part, nb, state);
    }
    hipLaunchKernelGGL(k_oc_apply, dim3(nb), dim3(OC_THREADS), 0, st, op, q, lo, hi, x, part, state);
    hipLaunchKernelGGL(k_oc_finish, dim3(1), dim3(OC_THREADS), 0, st, op, part, nb, state);
}

void launch_sum_cases(hipStream_t st, const double* in, int n_cases, size_t n, double* out) {
    const unsigned nb = (unsigned)std::min<size_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_sum_cases, dim3(std::max(1u, nb)), dim3(256), 0, st, in, n_cases, n, out);
}

void launch_oc_change(hipStream_t st, const double* x0, const double* x, int n_e, int m, double* partials,
                      double* out) {
    const int nb = blocks_for(n_e);
    hipLaunchKernelGGL(k_oc_change, dim3(nb), dim3(OC_THREADS), 0, st, x0, x, n_e, m, partials);
    hipLaunchKernelGGL(k_max_of, dim3(1), dim3(OC_THREADS), 0, st, partials, nb, out);
}

}  // namespace mtomg
