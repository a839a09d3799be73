// Scalar rules shared by the factorization kernels and by the host-side
// checks of the CPU test suite (this header needs no HIP: compiled by hipcc
// the functions are __host__ __device__, by a host compiler plain inline).
#pragma once

#include <cmath>

#include "seemps_hip.h"

#if defined(__HIPCC__)
#define SMPS_HD __host__ __device__
#else
#define SMPS_HD
#endif

namespace smps {

// Numerical rank floor: a vector whose squared norm is at most
// (u * max(nvec, len))^2 * ||X||_F^2, with u the unit roundoff of the
// arithmetic that produced X, is rounding noise of a rank-deficient matrix and
// counts as a zero singular value.
SMPS_HD inline double zero_floor2(double total2, int nv, int len, double u) {
    const double f = u * (double)(nv > len ? nv : len);
    return f * f * total2;
}

struct TruncResult {
    int r;         // kept rank
    double delta;  // discarded weight, tail summed from the smallest value up
    double kept;   // kept weight, summed from the smallest kept value up
};

// Truncation rule of the split (Sec. 2.3) on the descending values s[0..nv)
// of a matrix with vectors of length len:
//   REL_NORM2: the smallest r >= 1 whose tail sum_{j>=r} s_j^2 (accumulated
//              from the smallest value up) is at most tol * total;
//   REL_SV:    r = #{ s_j > tol * s_0 }, at least 1;
// then r <- min(r, max_rank, nv, len).  total is sum_j s_j^2 (same order), or
// *total_ext when given, in which case the weight the values miss,
// max(0, *total_ext - sum_j s_j^2), is counted in every tail.
SMPS_HD inline TruncResult trunc_rule(const double* s, int nv, int len, int mode, double tol, int max_rank,
                                      const double* total_ext) {
    double all = 0.0;
    for (int j = nv - 1; j >= 0; --j) all += s[j] * s[j];
    const double total = total_ext ? *total_ext : all;
    const double missed = total_ext ? fmax(0.0, total - all) : 0.0;
    int r;
    if (mode == SMPS_TRUNC_REL_SV) {
        r = 0;
        const double thr = tol * (nv > 0 ? s[0] : 0.0);
        for (int j = 0; j < nv; ++j) r += s[j] > thr;
    } else {
        const double thr = tol * total;
        double t = missed;
        int cand = nv;
        if (t <= thr) {
            while (cand > 1) {
                const double tn = t + s[cand - 1] * s[cand - 1];
                if (tn <= thr) {
                    t = tn;
                    --cand;
                } else {
                    break;
                }
            }
        }
        r = cand;
    }
    if (r < 1) r = 1;
    if (r > max_rank) r = max_rank;
    if (r > nv) r = nv;
    if (r > len) r = len;
    TruncResult out{r, 0.0, 0.0};
    for (int j = nv - 1; j >= r; --j) out.delta += s[j] * s[j];
    out.delta += missed;
    for (int j = r - 1; j >= 0; --j) out.kept += s[j] * s[j];
    return out;
}

// A one-sided Jacobi run that used its whole sweep budget and rotated in its
// last sweep has not converged (reported as status bit 2).
SMPS_HD inline bool jacobi_unconverged(int rotating_sweeps, int max_sweeps) { return rotating_sweeps >= max_sweeps; }

}  // namespace smps
