// layout.hpp -- symmetry-blocked (DPD) tensor layouts and reorder maps.
//
// Host-only C++.  A tensor is stored as a list of dense blocks, one per
// value of a "pair irrep" kappa (the partition of tensors into blocks by
// spinor subsets of the symmetry-handling section, generalised to rank-4
// tensors seen as supermatrices as in the TTGT decomposition of the
// algorithm-design section).  Each block is a row-major matrix whose rows
// enumerate the tuples of a row *group* of indices and whose columns
// enumerate the tuples of a column group.
//
// Spinors are addressed by their position in an irrep-sorted order of their
// space (occupied or virtual): all spinors of irrep 0 in ascending global
// index, then irrep 1, ...  A group holds 0..3 slots; one adjacent pair of
// slots of the same space may be "packed" (only p < q stored; the tensor is
// antisymmetric in that pair).  The irrep of a group is
// kappa = sum_s sg_s * g_s (mod G) with per-slot signs sg = +-1.  Within a
// kappa, sub-blocks are ordered lexicographically by the slot irreps and are
// dense in the local indices (packed pairs: strict upper triangle, row-major).
//
// A layout pairs row block kappa with column tuples of irrep colsign*kappa.
// Reorders (the transpositions of TTGT) are gather maps built here once per
// plan: for every destination element, the source offset and a sign bit.
#pragma once

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <exception>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

namespace fscc {

struct Space {
    int G = 1;
    int n = 0;
    std::vector<int> cnt, off;   // per irrep
    std::vector<int> irr, loc;   // per sorted position
    std::vector<int> glob;       // sorted position -> global spinor index

    // members: global spinor indices (ascending) with their irrep labels
    static Space make(int G, const std::vector<int>& global_idx, const std::vector<int>& labels) {
        Space s;
        s.G = G;
        s.n = (int)global_idx.size();
        s.cnt.assign(G, 0);
        for (int k = 0; k < s.n; ++k) {
            if (labels[k] < 0 || labels[k] >= G) throw std::invalid_argument("irrep label out of range");
            s.cnt[labels[k]]++;
        }
        s.off.assign(G + 1, 0);
        for (int g = 0; g < G; ++g) s.off[g + 1] = s.off[g] + s.cnt[g];
        s.irr.resize(s.n);
        s.loc.resize(s.n);
        s.glob.resize(s.n);
        std::vector<int> fill(G, 0);
        // global_idx ascending => within-irrep order ascending
        for (int k = 0; k < s.n; ++k) {
            int g = labels[k];
            int p = s.off[g] + fill[g]++;
            s.irr[p] = g;
            s.loc[p] = p - s.off[g];
            s.glob[p] = global_idx[k];
        }
        return s;
    }
};

inline int modG(int x, int G) { return ((x % G) + G) % G; }
inline int64_t tri(int64_t n) { return n * (n - 1) / 2; }
inline int64_t pairidx(int64_t a, int64_t b, int64_t n) { return a * (2 * n - a - 1) / 2 + (b - a - 1); }

constexpr uint32_t MAP_ZERO = 0xFFFFFFFFu;
constexpr uint32_t MAP_NEG = 0x80000000u;
constexpr int64_t MAP_MAX_OFF = 0x7FFFFFFELL;

struct Slot {
    int logical;        // index of the tensor's logical slot
    const Space* sp;
    int sg;             // +1 / -1 in the group irrep
};

// One index group (row or column side of a layout).
struct Group {
    int ns = 0;
    Slot s[3] = {};
    int packed = -1;     // -1 none, 0: slots (0,1) packed, 1: slots (1,2) packed
    int G = 1;
    std::vector<int64_t> size;   // per kappa
    std::vector<int64_t> tab;    // [kappa][g0][g1] -> offset within kappa (-1 absent)

    int64_t& T(int k, int g0, int g1) { return tab[((int64_t)k * G + g0) * G + g1]; }
    int64_t T(int k, int g0, int g1) const { return tab[((int64_t)k * G + g0) * G + g1]; }

    int n_(int k, int g) const { return s[k].sp->cnt[g]; }

    int64_t subcount(const int* g) const {
        if (ns == 0) return 1;
        if (ns == 1) return n_(0, g[0]);
        if (ns == 2) {
            if (packed == 0 && g[0] == g[1]) return tri(n_(0, g[0]));
            return (int64_t)n_(0, g[0]) * n_(1, g[1]);
        }
        if (packed == 0 && g[0] == g[1]) return tri(n_(0, g[0])) * n_(2, g[2]);
        if (packed == 1 && g[1] == g[2]) return n_(0, g[0]) * tri(n_(1, g[1]));
        return (int64_t)n_(0, g[0]) * n_(1, g[1]) * n_(2, g[2]);
    }

    bool allowed(const int* g) const {
        if (packed == 0 && g[0] > g[1]) return false;
        if (packed == 1 && g[1] > g[2]) return false;
        return true;
    }

    // enumerate the sub-block irrep tuples of kappa k in storage order
    template <class F>
    void for_sub(int k, F f) const {
        int g[3] = {0, 0, 0};
        if (ns == 0) {
            if (k == 0) f(g);
            return;
        }
        if (ns == 1) {
            g[0] = modG(s[0].sg * k, G);
            f(g);
            return;
        }
        if (ns == 2) {
            for (g[0] = 0; g[0] < G; ++g[0]) {
                g[1] = modG(s[1].sg * (k - s[0].sg * g[0]), G);
                if (allowed(g)) f(g);
            }
            return;
        }
        for (g[0] = 0; g[0] < G; ++g[0])
            for (g[1] = 0; g[1] < G; ++g[1]) {
                g[2] = modG(s[2].sg * (k - s[0].sg * g[0] - s[1].sg * g[1]), G);
                if (allowed(g)) f(g);
            }
    }

    void init(int G_) {
        G = G_;
        for (int k = 0; k < ns; ++k)
            if (!s[k].sp || s[k].sp->G != G) throw std::logic_error("group space/irrep mismatch");
        if (packed == 0 && !(ns >= 2 && s[0].sp == s[1].sp && s[0].sg == s[1].sg))
            throw std::logic_error("bad packing (0,1)");
        if (packed == 1 && !(ns == 3 && s[1].sp == s[2].sp && s[1].sg == s[2].sg))
            throw std::logic_error("bad packing (1,2)");
        size.assign(G, 0);
        tab.assign((size_t)G * G * G, -1);
        for (int k = 0; k < G; ++k) {
            int64_t o = 0;
            for_sub(k, [&](const int* g) {
                T(k, g[0], g[1]) = o;
                o += subcount(g);
            });
            size[k] = o;
        }
    }

    int kappa_of(const int* g) const {
        int x = 0;
        for (int k = 0; k < ns; ++k) x += s[k].sg * g[k];
        return modG(x, G);
    }

    // offset within its kappa of the tuple of positions p (already canonical)
    int64_t local(const int* p, int* kap) const {
        int g[3] = {0, 0, 0}, l[3] = {0, 0, 0};
        for (int k = 0; k < ns; ++k) {
            g[k] = s[k].sp->irr[p[k]];
            l[k] = s[k].sp->loc[p[k]];
        }
        int k = kappa_of(g);
        *kap = k;
        int64_t base = T(k, g[0], g[1]);
        if (base < 0) return -1;
        if (ns == 0) return 0;
        if (ns == 1) return base + l[0];
        if (ns == 2) {
            if (packed == 0 && g[0] == g[1]) return base + pairidx(l[0], l[1], n_(0, g[0]));
            return base + (int64_t)l[0] * n_(1, g[1]) + l[1];
        }
        if (packed == 0 && g[0] == g[1]) return base + pairidx(l[0], l[1], n_(0, g[0])) * n_(2, g[2]) + l[2];
        if (packed == 1 && g[1] == g[2]) return base + (int64_t)l[0] * tri(n_(1, g[1])) + pairidx(l[1], l[2], n_(1, g[1]));
        return base + ((int64_t)l[0] * n_(1, g[1]) + l[1]) * n_(2, g[2]) + l[2];
    }

    // canonicalise a packed pair in place: returns 0 if the element is zero by
    // antisymmetry, else the sign (+1/-1) picked up by ordering the pair.
    int canon(int* p) const {
        if (packed < 0) return 1;
        int a = packed, b = packed + 1;
        if (p[a] == p[b]) return 0;
        if (p[a] > p[b]) {
            std::swap(p[a], p[b]);
            return -1;
        }
        return 1;
    }

    // positions of all tuples of kappa k, in storage order (flattened, ns per tuple)
    std::vector<int> tuples(int k) const {
        std::vector<int> out;
        out.reserve((size_t)size[k] * std::max(ns, 1));
        for_sub(k, [&](const int* g) {
            int n0 = ns > 0 ? n_(0, g[0]) : 1, n1 = ns > 1 ? n_(1, g[1]) : 1, n2 = ns > 2 ? n_(2, g[2]) : 1;
            int o0 = ns > 0 ? s[0].sp->off[g[0]] : 0, o1 = ns > 1 ? s[1].sp->off[g[1]] : 0,
                o2 = ns > 2 ? s[2].sp->off[g[2]] : 0;
            if (ns == 0) {
                out.push_back(0);
                return;
            }
            for (int a = 0; a < n0; ++a)
                for (int b = 0; b < n1; ++b) {
                    if (ns >= 2 && packed == 0 && g[0] == g[1] && b <= a) continue;
                    for (int c = 0; c < n2; ++c) {
                        if (ns == 3 && packed == 1 && g[1] == g[2] && c <= b) continue;
                        out.push_back(o0 + a);
                        if (ns >= 2) out.push_back(o1 + b);
                        if (ns >= 3) out.push_back(o2 + c);
                    }
                }
        });
        return out;
    }
};

// Host threads for building one plan's maps: at most 16 (and at most
// OMP_NUM_THREADS when that is set); 1 inside a worker thread (plans of a
// batch are themselves built in parallel).
inline int& plan_thread_depth() {
    static thread_local int depth = 0;
    return depth;
}
inline int plan_threads() {
    if (plan_thread_depth() > 0) return 1;
    int n = (int)std::max(1u, std::thread::hardware_concurrency());
    if (const char* e = std::getenv("OMP_NUM_THREADS")) {
        const int m = std::atoi(e);
        if (m > 0) n = std::min(n, m);
    }
    return std::min(n, 16);
}

// Run body(i) for i in [0, n) on up to plan_threads() threads (the first
// exception is rethrown after all threads have finished).
template <class F>
void parallel_for(size_t n, F body) {
    const int nt = (int)std::min<size_t>(n, (size_t)plan_threads());
    if (nt <= 1) {
        for (size_t i = 0; i < n; ++i) body(i);
        return;
    }
    std::atomic<size_t> next{0};
    std::vector<std::exception_ptr> errs(nt);
    std::vector<std::thread> pool;
    for (int w = 0; w < nt; ++w)
        pool.emplace_back([&, w]() {
            plan_thread_depth()++;
            try {
                for (size_t i; (i = next.fetch_add(1)) < n;) body(i);
            } catch (...) {
                errs[w] = std::current_exception();
            }
            plan_thread_depth()--;
        });
    for (auto& t : pool) t.join();
    for (auto& e : errs)
        if (e) std::rethrow_exception(e);
}

struct Layout {
    int G = 1;
    int rank = 0;              // number of logical slots
    Group R, C;
    int colsign = 1;
    std::vector<char> kmask;   // materialised row kappas
    std::vector<int64_t> boff, nrow, ncol;
    int64_t total = 0;
    std::string name;

    int col_kappa(int k) const { return modG(colsign * k, G); }

    // pos[] indexed by logical slot.  Returns offset or -1 (structural zero);
    // *sign receives +-1 from packed-pair ordering.
    int64_t find(const int* pos, int* sign) const {
        int pr[3] = {0, 0, 0}, pc[3] = {0, 0, 0};
        for (int k = 0; k < R.ns; ++k) pr[k] = pos[R.s[k].logical];
        for (int k = 0; k < C.ns; ++k) pc[k] = pos[C.s[k].logical];
        int s1 = R.canon(pr), s2 = C.canon(pc);
        if (s1 == 0 || s2 == 0) return -1;
        int kr, kc;
        int64_t lr = R.local(pr, &kr), lc = C.local(pc, &kc);
        if (lr < 0 || lc < 0) return -1;
        if (kc != col_kappa(kr)) return -1;
        if (!kmask[kr]) throw std::logic_error("lookup into a non-materialised block of " + name);
        *sign = s1 * s2;
        return boff[kr] + lr * ncol[kr] + lc;
    }

    // visit every stored element, in chunks of rows on several host threads:
    // f(offset, pos[logical]) must only write state owned by `offset`
    template <class F>
    void for_each_par(F f) const {
        if (total < (int64_t)1 << 20 || plan_threads() <= 1) {
            for_each(f);
            return;
        }
        std::vector<std::vector<int>> rt(G), ct(G);
        struct Chunk {
            int k;
            int64_t r0, r1;
        };
        std::vector<Chunk> work;
        for (int k = 0; k < G; ++k) {
            if (!kmask[k] || nrow[k] == 0 || ncol[k] == 0) continue;
            rt[k] = R.tuples(k);
            ct[k] = C.tuples(col_kappa(k));
            const int64_t step = std::max<int64_t>(1, ((int64_t)1 << 16) / ncol[k]);
            for (int64_t r = 0; r < nrow[k]; r += step) work.push_back(Chunk{k, r, std::min(nrow[k], r + step)});
        }
        const int rs = std::max(R.ns, 1), cs = std::max(C.ns, 1);
        parallel_for(work.size(), [&](size_t i) {
            const Chunk& w = work[i];
            int pos[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int64_t o = boff[w.k] + w.r0 * ncol[w.k];
            for (int64_t r = w.r0; r < w.r1; ++r) {
                for (int q = 0; q < R.ns; ++q) pos[R.s[q].logical] = rt[w.k][r * rs + q];
                for (int64_t c = 0; c < ncol[w.k]; ++c) {
                    for (int q = 0; q < C.ns; ++q) pos[C.s[q].logical] = ct[w.k][c * cs + q];
                    f(o, pos);
                    ++o;
                }
            }
        });
    }

    // visit every stored element in storage order: f(offset, pos[logical])
    template <class F>
    void for_each(F f) const {
        for (int k = 0; k < G; ++k) {
            if (!kmask[k] || nrow[k] == 0 || ncol[k] == 0) continue;
            std::vector<int> rt = R.tuples(k), ct = C.tuples(col_kappa(k));
            int rs = std::max(R.ns, 1), cs = std::max(C.ns, 1);
            int pos[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int64_t o = boff[k];
            for (int64_t r = 0; r < nrow[k]; ++r) {
                for (int q = 0; q < R.ns; ++q) pos[R.s[q].logical] = rt[r * rs + q];
                for (int64_t c = 0; c < ncol[k]; ++c) {
                    for (int q = 0; q < C.ns; ++q) pos[C.s[q].logical] = ct[c * cs + q];
                    f(o, pos);
                    ++o;
                }
            }
        }
    }
};

// Build a layout.  rows/cols: slots; packR/packC: packing of each group.
inline Layout make_layout(const std::string& name, int G, std::vector<Slot> rows, int packR, std::vector<Slot> cols,
                          int packC, int colsign, int only_kappa = -1) {
    Layout L;
    L.name = name;
    L.G = G;
    L.R.ns = (int)rows.size();
    L.C.ns = (int)cols.size();
    int rank = 0;
    for (size_t k = 0; k < rows.size(); ++k) {
        L.R.s[k] = rows[k];
        rank = std::max(rank, rows[k].logical + 1);
    }
    for (size_t k = 0; k < cols.size(); ++k) {
        L.C.s[k] = cols[k];
        rank = std::max(rank, cols[k].logical + 1);
    }
    L.rank = rank;
    L.R.packed = packR;
    L.C.packed = packC;
    L.R.init(G);
    L.C.init(G);
    L.colsign = colsign;
    L.kmask.assign(G, 1);
    if (only_kappa >= 0)
        for (int k = 0; k < G; ++k) L.kmask[k] = (k == only_kappa);
    L.boff.assign(G + 1, 0);
    L.nrow.assign(G, 0);
    L.ncol.assign(G, 0);
    for (int k = 0; k < G; ++k) {
        L.nrow[k] = L.kmask[k] ? L.R.size[k] : 0;
        L.ncol[k] = L.kmask[k] ? L.C.size[L.col_kappa(k)] : 0;
        L.boff[k + 1] = L.boff[k] + L.nrow[k] * L.ncol[k];
    }
    L.total = L.boff[G];
    return L;
}

// The boundary format of an integral class: allowed (g1,g2,g3) tuples in
// lexicographic order (g4 = g1+g2-g3), dense [n1][n2][n3][n4] blocks.
struct FullBlocks {
    int G = 1;
    const Space* sp[4] = {};
    std::vector<int64_t> boff;   // [g1][g2][g3]
    int64_t total = 0;

    static FullBlocks make(int G, const Space* a, const Space* b, const Space* c, const Space* d) {
        FullBlocks F;
        F.G = G;
        F.sp[0] = a;
        F.sp[1] = b;
        F.sp[2] = c;
        F.sp[3] = d;
        F.boff.assign((size_t)G * G * G, 0);
        int64_t o = 0;
        for (int g1 = 0; g1 < G; ++g1)
            for (int g2 = 0; g2 < G; ++g2)
                for (int g3 = 0; g3 < G; ++g3) {
                    int g4 = modG(g1 + g2 - g3, G);
                    F.boff[((size_t)g1 * G + g2) * G + g3] = o;
                    o += (int64_t)a->cnt[g1] * b->cnt[g2] * c->cnt[g3] * d->cnt[g4];
                }
        F.total = o;
        return F;
    }

    int64_t find(const int* pos, int* sign) const {
        int g[4], l[4];
        for (int k = 0; k < 4; ++k) {
            g[k] = sp[k]->irr[pos[k]];
            l[k] = sp[k]->loc[pos[k]];
        }
        if (modG(g[0] + g[1] - g[2] - g[3], G) != 0) return -1;
        *sign = 1;
        int64_t o = boff[((size_t)g[0] * G + g[1]) * G + g[2]];
        return o + (((int64_t)l[0] * sp[1]->cnt[g[1]] + l[1]) * sp[2]->cnt[g[2]] + l[2]) * sp[3]->cnt[g[3]] + l[3];
    }
};

// Gather map dst <- src: dst logical slot tuple x, src logical slot j takes
// x[perm[j]]; entry = src offset | sign bit, or MAP_ZERO.  `sign` multiplies all.
template <class Src>
std::vector<uint32_t> build_map(const Layout& dst, const Src& src, const std::vector<int>& perm, int sign) {
    std::vector<uint32_t> m((size_t)dst.total, MAP_ZERO);
    dst.for_each_par([&](int64_t o, const int* x) {
        int y[8];
        for (size_t j = 0; j < perm.size(); ++j) y[j] = x[perm[j]];
        int s = 1;
        int64_t so = src.find(y, &s);
        if (so < 0) return;
        if (so > MAP_MAX_OFF) throw std::length_error("gather source too large for 31-bit maps");
        m[(size_t)o] = (uint32_t)so | ((s * sign) < 0 ? MAP_NEG : 0u);
    });
    return m;
}

}  // namespace fscc
