// Host-side check of the divergence rule (no GPU): feeds a sequence of
// max|step| values to fscc::DivergenceWatch and returns its actions.
#include "diverge.hpp"

extern "C" void diverge_actions(const double* steps, int n, int* actions) {
    fscc::DivergenceWatch w;
    for (int k = 0; k < n; ++k) actions[k] = (int)w.observe(steps[k]);
}

extern "C" int diverge_constants(double* growth, double* floor_) {
    *growth = fscc::DivergenceWatch::kGrowth;
    *floor_ = fscc::DivergenceWatch::kFloor;
    return 0;
}
