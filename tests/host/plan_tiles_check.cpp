// Host-side check of the planner's gather tile tables (no GPU): for every
// gather of every operation list, the 16 x 16 destination tiles must stay
// inside the destination, cover no element twice, and cover every element
// except those an accumulating gather leaves unchanged (all maps zero).
#include <cstdio>
#include <vector>

#include "plan.hpp"

using namespace fscc;

extern "C" int plan_tiles_check(int nocc, int nvirt, int G, const int* irrep, const double* eps, int nact,
                                const int* act, int* ops_checked) {
    System S;
    S.nocc = nocc;
    S.nvirt = nvirt;
    S.G = G;
    S.irrep.assign(irrep, irrep + nocc + nvirt);
    S.eps.assign(eps, eps + nocc + nvirt);
    S.active.assign(act, act + nact);
    Plan P;
    build_plan_ccsd(S, P);
    int bad = 0, nops = 0;
    for (auto* L : {&P.ops, &P.ops01_prep, &P.ops01, &P.ops02_prep, &P.ops02})
        for (auto& o : *L) {
            if (o.kind != OP_GATHER || o.gtiles.empty()) continue;
            ++nops;
            std::vector<unsigned char> seen((size_t)o.n, 0);
            for (auto& t : o.gtiles) {
                if (t.nr < 1 || t.nr > 16 || t.nc < 1 || t.nc > 16 || t.nc > t.ld) {
                    ++bad;
                    continue;
                }
                for (int r = 0; r < t.nr; ++r)
                    for (int c = 0; c < t.nc; ++c) {
                        const long long k = t.k0 + (long long)r * t.ld + c;
                        if (k < 0 || k >= o.n) {
                            ++bad;
                            continue;
                        }
                        if (seen[(size_t)k]++) ++bad;
                    }
            }
            // an element no tile covers must be one an accumulating gather leaves
            // unchanged: every term's map a structural zero there
            for (long long k = 0; k < o.n; ++k)
                if (!seen[(size_t)k]) {
                    bool zero = o.beta == 1;
                    for (size_t q = 0; q < o.mapsA.size() && zero; ++q) zero = P.maps[o.mapsA[q]][(size_t)k] == MAP_ZERO;
                    if (!zero) {
                        ++bad;
                        break;
                    }
                }
        }
    *ops_checked = nops;
    return bad;
}
