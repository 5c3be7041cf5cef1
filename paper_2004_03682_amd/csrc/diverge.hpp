// diverge.hpp -- the rule by which an amplitude iteration is declared
// divergent (plain host code, no HIP).
//
// Intruder states (model-space energies close to, or above, those of
// states outside it) make the Jacobi iteration of the amplitude equations
// diverge: the largest step grows geometrically.  The rule watches the
// largest step of every iteration of one sector:
//   * best = the smallest max|step| since the watch (re)started, floored at
//     kFloor so that rounding-level steps near convergence are not mistaken
//     for growth;
//   * a step larger than kGrowth * best is growth: the first time, the DIIS
//     subspace is cleared (its extrapolation may be what drives the growth)
//     and the watch restarts from this step; a second time, the iteration is
//     given up.
#pragma once

#include <cmath>

namespace fscc {

struct DivergenceWatch {
    static constexpr double kGrowth = 1e3;
    static constexpr double kFloor = 1e-8;
    enum Action { CONTINUE = 0, RESET_DIIS = 1, GIVE_UP = 2 };

    double best = INFINITY;
    int resets = 0;

    void restart() {
        best = INFINITY;
        resets = 0;
    }

    // One iteration's max|step|; non-finite steps give up at once.
    Action observe(double step) {
        if (!std::isfinite(step)) return GIVE_UP;
        if (std::isfinite(best) && step > kGrowth * std::fmax(best, kFloor)) {
            if (resets > 0) return GIVE_UP;
            ++resets;
            best = step;
            return RESET_DIIS;
        }
        if (step < best) best = step;
        return CONTINUE;
    }
};

}  // namespace fscc
