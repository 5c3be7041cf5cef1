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
    // affine tiles: inside the destination, no element twice, every element an
    // accumulating gather changes covered, and every affine term equal to the
    // term's map on its tile (offset, stride and sign), every zero term a
    // structural zero there
    for (auto* L : {&P.ops, &P.ops01_prep, &P.ops01, &P.ops02_prep, &P.ops02})
        for (auto& o : *L) {
            if (o.kind != OP_GATHER || o.rtiles.empty()) continue;
            ++nops;
            const size_t NT = o.mapsA.size();
            if (o.rterms.size() != o.rtiles.size() * NT) {
                ++bad;
                continue;
            }
            std::vector<unsigned char> seen((size_t)o.n, 0);
            for (size_t i = 0; i < o.rtiles.size(); ++i) {
                const GTile& t = o.rtiles[i];
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
                        for (size_t q = 0; q < NT; ++q) {
                            const RTerm& rt = o.rterms[i * NT + q];
                            const uint32_t m = P.maps[o.mapsA[q]][(size_t)k];
                            if (rt.s0 == RTERM_MAPPED) continue;
                            if (rt.s0 == RTERM_ZERO) {
                                if (m != MAP_ZERO) ++bad;
                                continue;
                            }
                            const long long off = (rt.s0 & ~RTERM_NEG) + (long long)r * rt.sa + (long long)c * rt.sb;
                            const uint32_t want = (uint32_t)off | ((rt.s0 & RTERM_NEG) ? MAP_NEG : 0u);
                            if (off < 0 || off > 0x7FFFFFFFLL || m != want) ++bad;
                        }
                    }
            }
            for (long long k = 0; k < o.n; ++k)
                if (!seen[(size_t)k]) {
                    bool zero = o.beta == 1;
                    for (size_t q = 0; q < NT && zero; ++q) zero = P.maps[o.mapsA[q]][(size_t)k] == MAP_ZERO;
                    if (!zero) {
                        ++bad;
                        break;
                    }
                }
        }
    *ops_checked = nops;
    return bad;
}
