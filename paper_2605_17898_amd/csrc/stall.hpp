// Stagnation rule and precision fallback of the CG driver (host code only; no
// HIP, so that it can be compiled and checked on its own).
//
// CG on an inexact product (the BF16 forms, or any form on a very
// ill-conditioned system) can stop reducing its recurrence residual well above
// the tolerance: inexact Krylov methods reach a residual gap of about
// (product error) x (condition number), after which the iteration only
// wanders.  Nothing in the plain method ends such a cycle before the
// iteration cap.  The driver therefore
//   * ends a column's cycle when its recurrence residual has stagnated: it
//     has made no new minimum (a fall below kStallGain of the best squared
//     norm so far) for a window of max(kStallMin, a quarter of the cycle's
//     length) iterations, after having fallen tenfold below the cycle's start
//     (kStallArm on the squared norm) and while it is not above that start.
//     The residual norm of CG is not monotone: on ill-conditioned systems it
//     can first rise by an order of magnitude and stay there for hundreds of
//     iterations while the energy-norm error falls, so a rule without those
//     two conditions would end healthy cycles;
//   * takes the next more accurate product form (x1 -> x2 -> x3 -> FP32
//     direct differences, the operator of the recomputed residual itself) for
//     every column from the next cycle on when a cycle stagnated, when it
//     left the true residual above kNoProgress of its value at the cycle's
//     start, or when two further cycles with the same reduction would still
//     end above the tolerance (the form's error floor is far above it, so
//     refinement on that form would take several more full solves);
//   * ends a cycle early, with the same fallback, when a residual replacement
//     finds that the recurrence has left the true residual while that true
//     residual is still that far above the tolerance (the floor is reached:
//     the rest of the cycle could only lower the recurrence);
//   * gives a column up (MFGP_NOT_CONVERGED, its iterate kept) when a cycle
//     on the last form left its true residual no smaller than before.
#pragma once

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "../../include/mfgp.h"

namespace mfgp {

constexpr int kStallMin = 100;         // shortest stagnation window (iterations)
constexpr double kStallGain = 0.9;     // a new minimum: rr < 0.9 * best rr
constexpr double kStallArm = 1e-2;     // the rule applies once rr <= 1e-2 rr at the cycle's start
constexpr double kNoProgress = 0.7;    // cycle factor above which a more accurate form is taken

struct StallTracker {
    double start_rr = 0.0;
    double best = std::numeric_limits<double>::infinity();
    int best_it = 0;
    int start = 0;
    bool armed = false;

    // A new cycle starts at iteration `it` with squared residual norm `rr`.
    void begin(int it, double rr) {
        start_rr = rr;
        best = rr;
        best_it = it;
        start = it;
        armed = false;
    }
    // The recurrence's squared residual norm seen at iteration `it` (at the
    // host's checks, in increasing `it`); true when the cycle has stagnated.
    bool update(int it, double rr) {
        if (rr < kStallGain * best) {
            best = rr;
            best_it = it;
        }
        if (best <= kStallArm * start_rr) armed = true;
        if (!armed || !(rr <= start_rr)) return false;
        const int window = std::max(kStallMin, (it - start) / 4);
        return it - best_it >= window;
    }
};

// The next more accurate product form, or -1 when there is none.
inline int more_accurate_precision(int precision) {
    switch (precision) {
        case MFGP_BF16X1: return MFGP_BF16X2;
        case MFGP_BF16X2: return MFGP_BF16X3;
        case MFGP_BF16X3: return MFGP_FP32_DIRECT;
        case MFGP_FP32: return MFGP_FP32_DIRECT;
        case MFGP_FP32_GRAM: return MFGP_FP32_DIRECT;
        default: return -1;   // FP32 direct differences and the VALU form are the residual's operator
    }
}

// True when a finished cycle (true relative residual relt_start -> relt_end,
// ended by stagnation or not) should move the solve to a more accurate form:
// it stagnated, it cut the true residual by less than 1 / kNoProgress, or two
// more cycles with the same reduction would still end above tol.
inline bool cycle_wants_fallback(bool stalled, double relt_start, double relt_end, double tol) {
    const double f = relt_end / relt_start;
    return stalled || !(relt_end <= kNoProgress * relt_start) || !(relt_end * f * f <= tol);
}

// Largest ||r|| / ||b|| of the recurrence over the columns still iterating,
// or over every column when none is (what a progress report shows: a column
// that has stopped keeps its last norm, which says nothing of the others).
inline double worst_recurrence(const std::vector<int>& active, const std::vector<double>& rr,
                               const std::vector<double>& b2) {
    double live = -1.0, all = 0.0;
    for (size_t c = 0; c < rr.size(); ++c) {
        if (!(b2[c] > 0.0)) continue;
        const double v = std::sqrt(rr[c] / b2[c]);
        all = std::max(all, v);
        if (active[c]) live = std::max(live, v);
    }
    return live >= 0.0 ? live : all;
}

// True when a cycle on the last form left the true residual no smaller.
inline bool cycle_gave_nothing(double relt_start, double relt_end) { return !(relt_end < relt_start); }

}  // namespace mfgp
