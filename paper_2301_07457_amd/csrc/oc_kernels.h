// Optimality-criteria update of the alternating active-phase loop
// (Section 4): one binary sub-problem on a pair of phases (a, b), a < b,
// of the densities x [n_e][m] (b == m is the void, whose share
// 1 - sum_i x_i is implicit).  With s_e = alpha_a + alpha_b held fixed per
// element and the pair sensitivity d_e = g_a - g_b (g of the void is 0):
//   lo_e = max(eps, alpha_a - move),  hi_e = min(1, s_e - eps, alpha_a + move),
//   y_e(lambda) = clamp(alpha_a (max(0, -d_e) / lambda)^eta, lo_e, hi_e),
// with the multiplier lambda > 0 such that sum_e y_e = target (the volume of
// phase a); then alpha_a = y, alpha_b = s - y.
//
// On the device the candidate is written y_e(t) = clamp(q_e t, lo_e, hi_e),
// q_e = alpha_a max(0, -d_e)^eta and t = lambda^(-eta): S(t) = sum_e y_e(t)
// is continuous, piecewise linear and non-decreasing in t, so the root is
// found by Newton steps on S, kept inside a shrinking bracket (a geometric
// bisection step wherever Newton would leave it).  Every pass reads q, lo,
// hi once (24 B per element) and sums in a fixed order; a one-workgroup
// kernel after it reduces the per-workgroup sums and sets the next
// candidate, so the host only queues passes (those after convergence exit
// at once).
#pragma once

#include <hip/hip_runtime.h>

namespace mtomg {

// Workgroups of every OC pass (a grid-stride loop covers larger grids).
constexpr int OC_BLOCKS = 1024;
constexpr int OC_THREADS = 256;
// Newton passes queued per pair update; a converged state makes the rest
// return at once (3 to 6 passes are typical).
constexpr int OC_MAX_PASSES = 24;

// Device state of one pair update.
struct OcState {
    double t, tl, th;       // candidate and bracket in t = lambda^(-eta)
    double S;               // S(t) of the last pass
    double change;          // largest |alpha_a new - old| (set by the apply pass)
    double lambda;          // final multiplier
    int done, passes;       // converged; passes run
    unsigned int count;     // unused (keeps the layout of 64 bytes)
    int pad;
};

struct OcPair {
    int n_e, m, a, b;
    double eta, move, eps, target;
};

// Doubles of scratch per pair update: q, lo, hi [n_e] + partials [OC_BLOCKS][4].
size_t oc_scratch_doubles(int n_e);

// Queue one pair update on st: prep (q, lo, hi and the bracket), Newton
// passes, then the update of x in place.  g: the filtered gradient [n_e][m];
// scratch: oc_scratch_doubles(n_e) doubles; state: device OcState.
void launch_oc_pair(hipStream_t st, const OcPair& op, const double* g, double* x, double* scratch, OcState* state);

// out[e] = sum_k in[k * n + e] over k = 0 .. n_cases - 1, in that order.
void launch_sum_cases(hipStream_t st, const double* in, int n_cases, size_t n, double* out);

// Largest change of any phase, void included, between x0 and x [n_e][m],
// written to *out (device); partials: OC_BLOCKS doubles.
void launch_oc_change(hipStream_t st, const double* x0, const double* x, int n_e, int m, double* partials,
                      double* out);

}  // namespace mtomg
