// plan_ccsd.cpp -- the (0h,0p) CCSD residual as TTGT operations.
//
// Equations: spin-orbital CCSD (Stanton-Gauss intermediates) for a diagonal
// Fock matrix and complex antisymmetrised integrals, with the W_abef term
// never materialised: its bare-integral part is the particle-particle ladder
//   L_ij^ab = sum_{c<d} <ab||cd> tau_ij^cd               (one GEMM per pair irrep)
// its T1 part is -P(ab) sum_m t_m^b Z_ij^am with Z_ij^am = sum_{e<f} <am||ef> tau_ij^ef,
// and its tau*tau part is folded into the hole-hole ladder through
//   W'_mnij = <mn||ij> + P(ij) sum_e t_j^e <mn||ie> + 1/2 sum_ef tau_ij^ef <mn||ef>.
// Residual R = RHS - D*t with D_i^a = e_i - e_a, D_ij^ab = e_i + e_j - e_a - e_b
// (Eq. (3)-(4): D is the negative of the H0 eigenvalue differences).
//
// Integral views used below (<pq||rs> antisymmetric in (pq), (rs); Hermitian):
//   <mb||ej> = -<mb||je>            (OVOV)
//   <mn||ej> = -<mn||je>            (OOOV)
//   <ab||ej> = -conj <je||ab>       (OVVV)
//   <mb||ij> =  conj <ij||mb>       (OOOV)
//   <ab||ij> =  conj <ij||ab>       (OOVV)   -- the T2 driver
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "plan.hpp"

namespace fscc {
namespace {

bool same_group(const Group& a, const Group& b) {
    if (a.ns != b.ns || a.packed != b.packed) return false;
    for (int k = 0; k < a.ns; ++k)
        if (a.s[k].sp != b.s[k].sp || a.s[k].sg != b.s[k].sg) return false;
    return true;
}

struct Builder {
    Plan& P;
    int G;
    const Space* o;
    const Space* v;
    std::vector<Op>* out;   // op list being built

    Builder(Plan& p) : P(p), G(p.G), o(&p.O), v(&p.V), out(&p.ops) {}

    Slot s(int l, const Space* sp, int sg) const { return Slot{l, sp, sg}; }

    // dst (+)= alpha * sum_t sign_t * cj(src[map_t]) [* src2[map2_t]]
    struct Term {
        std::vector<int> perm;
        int sign;
        std::vector<int> perm2;   // for the second operand (bilinear); empty if none
    };

    // 16 x 16 tiles of the destination blocks (row-major, leading dimension = columns)
    static std::vector<GTile> dest_tiles(const Layout& Ld) {
        std::vector<GTile> t;
        if (Ld.total < 256) return t;
        for (int k = 0; k < Ld.G; ++k) {
            if (!Ld.kmask[k] || Ld.nrow[k] == 0 || Ld.ncol[k] == 0) continue;
            for (int64_t r = 0; r < Ld.nrow[k]; r += 16)
                for (int64_t c = 0; c < Ld.ncol[k]; c += 16)
                    t.push_back(GTile{Ld.boff[k] + r * Ld.ncol[k] + c, (int32_t)Ld.ncol[k],
                                      (int16_t)std::min<int64_t>(16, Ld.nrow[k] - r),
                                      (int16_t)std::min<int64_t>(16, Ld.ncol[k] - c)});
        }
        return t;
    }

    // An accumulating gather (beta = 1) leaves a destination tile unchanged
    // when every term's map is a structural zero on it: such tiles are
    // dropped from the tiled traversal (e.g. the t1 x t1 part of tau and U
    // touches a few irrep blocks only).
    void prune_zero_tiles(Op& op) const {
        if (op.beta != 1) return;
        std::vector<char> any(op.gtiles.size(), 0);
        parallel_for(op.gtiles.size(), [&](size_t i) {
            const GTile& t = op.gtiles[i];
            bool a = false;
            for (size_t q = 0; q < op.mapsA.size() && !a; ++q) {
                const std::vector<uint32_t>& m = P.maps[op.mapsA[q]];
                for (int r = 0; r < t.nr && !a; ++r)
                    for (int c = 0; c < t.nc && !a; ++c) a = m[(size_t)(t.k0 + (int64_t)r * t.ld + c)] != MAP_ZERO;
            }
            any[i] = a;
        });
        std::vector<GTile> keep;
        for (size_t i = 0; i < op.gtiles.size(); ++i)
            if (any[i]) keep.push_back(op.gtiles[i]);
        op.gtiles.swap(keep);
    }

    // Affine traversal of a reorder without a second operand.  Each 16 x 16
    // destination tile is cut into rectangles on which every term's map is
    // affine: rows are cut where the first column of some term stops
    // continuing the step of the strip's first two rows (or changes sign or
    // zero status), columns likewise along the strip's first row.  Each
    // rectangle is then checked element by element; a term that is not
    // affine on it keeps its map there (RTERM_MAPPED).  Rectangles of an
    // accumulating gather on which every term is zero are dropped.
    void affine_tiles(Op& op) const {
        op.rtiles.clear();
        op.rterms.clear();
        op.runits.clear();
        if (op.src2 >= 0 || op.gtiles.empty()) return;
        const int NT = (int)op.mapsA.size();
        std::vector<const std::vector<uint32_t>*> M;
        for (int m : op.mapsA) M.push_back(&P.maps[m]);
        auto at = [&](int t, const GTile& g, int r, int c) { return (*M[t])[(size_t)(g.k0 + (int64_t)r * g.ld + c)]; };
        auto kind = [](uint32_t v) { return v == MAP_ZERO ? 0 : (v & MAP_NEG) ? 2 : 1; };
        auto off = [](uint32_t v) { return (int64_t)(v & ~MAP_NEG); };
        // does element (r1 | c1) continue the affine run started at (r0, c0) along rows (dr) or columns?
        auto continues = [&](const GTile& g, int r0, int c0, int r1, int c1) {
            for (int t = 0; t < NT; ++t) {
                const uint32_t a = at(t, g, r0, c0), b = at(t, g, r1, c1);
                if (kind(a) != kind(b)) return false;
                const int d = (r1 - r0) + (c1 - c0);
                if (kind(a) && d >= 2) {
                    const uint32_t n1 = r1 > r0 ? at(t, g, r0 + 1, c0) : at(t, g, r0, c0 + 1);
                    if (off(b) != off(a) + (int64_t)d * (off(n1) - off(a))) return false;
                }
            }
            return true;
        };
        // each 16 x 16 tile on its own (host threads), then concatenated in order
        std::vector<std::vector<GTile>> part_t(op.gtiles.size());
        std::vector<std::vector<RTerm>> part_q(op.gtiles.size());
        parallel_for(op.gtiles.size(), [&](size_t gi) {
            const GTile& g = op.gtiles[gi];
            for (int r0 = 0; r0 < g.nr;) {
                int r1 = r0 + 1;
                while (r1 < g.nr && continues(g, r0, 0, r1, 0)) ++r1;
                for (int c0 = 0; c0 < g.nc;) {
                    int c1 = c0 + 1;
                    while (c1 < g.nc && continues(g, r0, c0, r0, c1)) ++c1;
                    GTile rt{g.k0 + (int64_t)r0 * g.ld + c0, g.ld, (int16_t)(r1 - r0), (int16_t)(c1 - c0)};
                    std::vector<RTerm> tt(NT);
                    bool any = false;
                    for (int t = 0; t < NT; ++t) {
                        const uint32_t a = at(t, g, r0, c0);
                        const int64_t sa = r1 - r0 > 1 ? off(at(t, g, r0 + 1, c0)) - off(a) : 0;
                        const int64_t sb = c1 - c0 > 1 ? off(at(t, g, r0, c0 + 1)) - off(a) : 0;
                        bool ok = sa >= INT32_MIN && sa <= INT32_MAX && sb >= INT32_MIN && sb <= INT32_MAX;
                        for (int r = r0; r < r1 && ok; ++r)
                            for (int c = c0; c < c1 && ok; ++c) {
                                const uint32_t v = at(t, g, r, c);
                                ok = kind(v) == kind(a) &&
                                     (kind(v) == 0 || off(v) == off(a) + (r - r0) * sa + (c - c0) * sb);
                            }
                        if (!ok)
                            tt[t] = RTerm{RTERM_MAPPED, 0, 0};
                        else if (kind(a) == 0)
                            tt[t] = RTerm{RTERM_ZERO, 0, 0};
                        else
                            tt[t] = RTerm{off(a) | (kind(a) == 2 ? RTERM_NEG : 0), (int32_t)sa, (int32_t)sb};
                        any |= tt[t].s0 != RTERM_ZERO;
                    }
                    if (any || op.beta != 1) {
                        part_t[gi].push_back(rt);
                        part_q[gi].insert(part_q[gi].end(), tt.begin(), tt.end());
                    }
                    c0 = c1;
                }
                r0 = r1;
            }
        });
        for (size_t gi = 0; gi < op.gtiles.size(); ++gi) {
            op.rtiles.insert(op.rtiles.end(), part_t[gi].begin(), part_t[gi].end());
            op.rterms.insert(op.rterms.end(), part_q[gi].begin(), part_q[gi].end());
        }
        // work units: consecutive tiles up to RUNIT_MAX_ELEMS elements / RUNIT_MAX_RECTS tiles
        op.runits.clear();
        for (size_t i = 0; i < op.rtiles.size();) {
            RUnit u{(int32_t)i, 0};
            int el = 0;
            while (i < op.rtiles.size() && u.count < RUNIT_MAX_RECTS &&
                   el + op.rtiles[i].nr * op.rtiles[i].nc <= RUNIT_MAX_ELEMS) {
                el += op.rtiles[i].nr * op.rtiles[i].nc;
                ++u.count;
                ++i;
            }
            op.runits.push_back(u);
        }
    }

    void gather(const std::string& name, int dst, const Layout& Ld, int src, const Layout& Ls,
                const std::vector<Term>& terms, cplx alpha, int beta, bool conj = false, int src2 = -1,
                const Layout* Ls2 = nullptr) {
        Op op;
        op.kind = OP_GATHER;
        op.name = name;
        op.dst = dst;
        op.src = src;
        op.src2 = src2;
        op.alpha = alpha;
        op.beta = beta;
        op.conj = conj;
        op.n = Ld.total;
        if (P.bufs[dst].n != Ld.total) throw std::logic_error("gather dst size mismatch: " + name);
        if (P.bufs[src].n != Ls.total) throw std::logic_error("gather src size mismatch: " + name);
        op.gtiles = dest_tiles(Ld);
        for (size_t t = 0; t < terms.size(); ++t) {
            op.mapsA.push_back(P.map(name + "/A" + std::to_string(t), build_map(Ld, Ls, terms[t].perm, terms[t].sign)));
            if (src2 >= 0)
                op.mapsB.push_back(P.map(name + "/B" + std::to_string(t), build_map(Ld, *Ls2, terms[t].perm2, 1)));
        }
        affine_tiles(op);
        prune_zero_tiles(op);
        out->push_back(std::move(op));
    }

    // dst = beta*dst + alpha * sum_t s_t src_t[perm_t]: reorders of several
    // buffers summed into one destination in a single pass (term order kept)
    void gather_sum(const std::string& name, int dst, const Layout& Ld,
                    const std::vector<std::pair<int, const Layout*>>& srcs, const std::vector<Term>& terms,
                    cplx alpha, int beta) {
        if (srcs.size() != terms.size() || terms.empty() || terms.size() > 4)
            throw std::logic_error("gather_sum: one source per term, 1..4 terms: " + name);
        Op op;
        op.kind = OP_GATHER;
        op.name = name;
        op.dst = dst;
        op.src = srcs[0].first;
        op.alpha = alpha;
        op.beta = beta;
        op.n = Ld.total;
        if (P.bufs[dst].n != Ld.total) throw std::logic_error("gather dst size mismatch: " + name);
        op.gtiles = dest_tiles(Ld);
        for (size_t t = 0; t < terms.size(); ++t) {
            if (P.bufs[srcs[t].first].n != srcs[t].second->total)
                throw std::logic_error("gather src size mismatch: " + name);
            op.srcT.push_back(srcs[t].first);
            op.mapsA.push_back(P.map(name + "/A" + std::to_string(t),
                                     build_map(Ld, *srcs[t].second, terms[t].perm, terms[t].sign)));
        }
        affine_tiles(op);
        prune_zero_tiles(op);
        out->push_back(std::move(op));
    }

    void gemm(const std::string& name, int bA, const Layout& A, bool tA, bool cA, int bB, const Layout& B, bool tB,
              bool cB, int bC, const Layout& C, cplx alpha, int beta) {
        const Group& AM = tA ? A.C : A.R;
        const Group& AK = tA ? A.R : A.C;
        const Group& BK = tB ? B.C : B.R;
        const Group& BN = tB ? B.R : B.C;
        if (!same_group(AM, C.R)) throw std::logic_error("gemm " + name + ": A/M group != C rows");
        if (!same_group(AK, BK)) throw std::logic_error("gemm " + name + ": K groups differ");
        if (!same_group(BN, C.C)) throw std::logic_error("gemm " + name + ": B/N group != C cols");
        if (P.bufs[bA].n != A.total || P.bufs[bB].n != B.total || P.bufs[bC].n != C.total)
            throw std::logic_error("gemm " + name + ": buffer size mismatch");
        Op op;
        op.kind = OP_GEMM;
        op.name = name;
        op.src = bA;
        op.src2 = bB;
        op.dst = bC;
        op.tA = tA;
        op.tB = tB;
        op.cA = cA;
        op.cB = cB;
        op.alpha = alpha;
        op.beta = beta;
        for (int r = 0; r < G; ++r) {
            if (!C.kmask[r] || C.nrow[r] == 0 || C.ncol[r] == 0) continue;
            int a = tA ? modG(A.colsign * r, G) : r;
            int kK = tA ? a : A.col_kappa(a);
            int b = tB ? modG(B.colsign * kK, G) : kK;
            int nK = tB ? b : B.col_kappa(b);
            if (nK != C.col_kappa(r)) throw std::logic_error("gemm " + name + ": kappa mismatch");
            int64_t M = C.nrow[r], N = C.ncol[r], K = AK.size[kK];
            if (K == 0 && beta) continue;
            GemmProblem pr{0, 0, C.boff[r], (int)M, (int)N, (int)K, 1, 1, (int)C.ncol[r]};
            if (K > 0) {
                if (!A.kmask[a] || !B.kmask[b]) throw std::logic_error("gemm " + name + ": operand block not stored");
                int64_t ar = tA ? K : M, ac = tA ? M : K, br = tB ? N : K, bc = tB ? K : N;
                if (A.nrow[a] != ar || A.ncol[a] != ac) throw std::logic_error("gemm " + name + ": A block shape");
                if (B.nrow[b] != br || B.ncol[b] != bc) throw std::logic_error("gemm " + name + ": B block shape");
                pr.a_off = A.boff[a];
                pr.lda = (int)A.ncol[a];
                pr.b_off = B.boff[b];
                pr.ldb = (int)B.ncol[b];
            }
            op.flops += 8.0 * (double)M * (double)N * (double)K;
            op.probs.push_back(pr);
        }
        out->push_back(std::move(op));
    }

    void axpby(const std::string& name, int dst, int src, int64_t n, cplx alpha, int beta, bool conj) {
        Op op;
        op.kind = OP_AXPBY;
        op.name = name;
        op.dst = dst;
        op.src = src;
        op.n = n;
        op.alpha = alpha;
        op.beta = beta;
        op.conj = conj;
        out->push_back(std::move(op));
    }

    void mul(const std::string& name, int dst, int d, int64_t n) {
        Op op;
        op.kind = OP_MUL;
        op.name = name;
        op.dst = dst;
        op.src2 = d;
        op.n = n;
        out->push_back(std::move(op));
    }

    void diag(const std::string& name, int dst, int d, int src, int64_t n) {
        Op op;
        op.kind = OP_DIAG;
        op.name = name;
        op.dst = dst;
        op.src2 = d;
        op.src = src;
        op.n = n;
        out->push_back(std::move(op));
    }

    // constant derived from integral class `cls` (boundary full blocks)
    int derived(const std::string& name, int cls, const Layout& L, const std::vector<int>& perm, int sign, bool conj) {
        int b = P.buf(name, L.total, BUF_CONST);
        int m = P.map(name + "/pack", build_map(L, P.full[cls], perm, sign));
        P.setup.push_back({cls, b, m, conj, name});
        return b;
    }
};

}  // namespace

void build_plan_ccsd(const System& S, Plan& P) {
    const int G = S.G;
    P.G = G;
    if (G < 1 || S.nocc < 0 || S.nvirt < 0) throw std::invalid_argument("bad system sizes");
    {
        std::vector<int> gi, li, ga, la;
        for (int p = 0; p < S.nocc; ++p) {
            gi.push_back(p);
            li.push_back(S.irrep[p]);
        }
        for (int p = S.nocc; p < S.nocc + S.nvirt; ++p) {
            ga.push_back(p);
            la.push_back(S.irrep[p]);
        }
        P.O = Space::make(G, gi, li);
        P.V = Space::make(G, ga, la);
    }
    Builder B(P);
    const Space* o = &P.O;
    const Space* v = &P.V;
    auto s = [&](int l, const Space* sp, int sg) { return Slot{l, sp, sg}; };
    using T = Builder::Term;

    P.full[IC_OOOO] = FullBlocks::make(G, o, o, o, o);
    P.full[IC_OOOV] = FullBlocks::make(G, o, o, o, v);
    P.full[IC_OOVV] = FullBlocks::make(G, o, o, v, v);
    P.full[IC_OVOV] = FullBlocks::make(G, o, v, o, v);
    P.full[IC_OVVV] = FullBlocks::make(G, o, v, v, v);
    P.full[IC_VVVV] = FullBlocks::make(G, v, v, v, v);

    // ---------------------------------------------------------------- layouts
    // amplitudes: T1 (i,a) = [g][o_g][v_g];  T2 (i,j,a,b) = [G][ij<][ab<]
    P.L_T1 = make_layout("T1", G, {s(0, o, 1)}, -1, {s(1, v, 1)}, -1, 1);
    P.L_T2 = make_layout("T2", G, {s(0, o, 1), s(1, o, 1)}, 0, {s(2, v, 1), s(3, v, 1)}, 0, 1);
    const Layout& L_T1 = P.L_T1;
    const Layout& L_T2 = P.L_T2;
    // rank-2 quantities seen as vectors over (p,q) pairs of pair irrep 0 (same memory as [g][n_g][m_g])
    Layout L_T1v = make_layout("T1v", G, {s(0, o, -1), s(1, v, 1)}, -1, {}, -1, 1, 0);
    Layout L_T1w = make_layout("T1w", G, {s(0, o, 1), s(1, v, -1)}, -1, {}, -1, 1, 0);

    P.b_t1 = P.buf("t1", L_T1.total, BUF_IN_T1);
    P.b_t2 = P.buf("t2", L_T2.total, BUF_IN_T2);
    P.b_r1 = P.buf("r1", L_T1.total, BUF_OUT_R1);
    P.b_r2 = P.buf("r2", L_T2.total, BUF_OUT_R2);

    // denominators
    {
        P.D1.assign(L_T1.total, 0.0);
        L_T1.for_each([&](int64_t k, const int* x) { P.D1[k] = S.eps[o->glob[x[0]]] - S.eps[v->glob[x[1]]]; });
        P.D2.assign(L_T2.total, 0.0);
        L_T2.for_each([&](int64_t k, const int* x) {
            P.D2[k] = S.eps[o->glob[x[0]]] + S.eps[o->glob[x[1]]] - S.eps[v->glob[x[2]]] - S.eps[v->glob[x[3]]];
        });
        P.b_D1 = P.buf("D1", L_T1.total, BUF_REAL);
        P.b_D2 = P.buf("D2", L_T2.total, BUF_REAL);
        P.eps_o.assign(o->n, 0.0);
        P.eps_v.assign(v->n, 0.0);
        for (int i = 0; i < o->n; ++i) P.eps_o[i] = S.eps[o->glob[i]];
        for (int a = 0; a < v->n; ++a) P.eps_v[a] = S.eps[v->glob[a]];
    }

    // ------------------------------------------------------- stored integrals
    // OOOO <ij||kl> [ij<|kl<]
    Layout L_OOOO = make_layout("OOOO", G, {s(0, o, 1), s(1, o, 1)}, 0, {s(2, o, 1), s(3, o, 1)}, 0, 1);
    int b_oooo = B.derived("V_oooo", IC_OOOO, L_OOOO, {0, 1, 2, 3}, 1, false);
    // OOVV <ij||ab> [ij<|ab<]
    Layout L_OOVV = make_layout("OOVV", G, {s(0, o, 1), s(1, o, 1)}, 0, {s(2, v, 1), s(3, v, 1)}, 0, 1);
    int b_oovv = B.derived("V_oovv", IC_OOVV, L_OOVV, {0, 1, 2, 3}, 1, false);
    P.b_oovv = b_oovv;
    // VVVV <ab||cd> [ab<|cd<]
    Layout L_VVVV = make_layout("VVVV", G, {s(0, v, 1), s(1, v, 1)}, 0, {s(2, v, 1), s(3, v, 1)}, 0, 1);
    int b_vvvv = B.derived("V_vvvv", IC_VVVV, L_VVVV, {0, 1, 2, 3}, 1, false);
    // OVVV <ma||ef> [(m,a)|ef<]
    Layout L_OVVV = make_layout("OVVV", G, {s(0, o, 1), s(1, v, 1)}, -1, {s(2, v, 1), s(3, v, 1)}, 0, 1);
    int b_ovvv = B.derived("V_ovvv", IC_OVVV, L_OVVV, {0, 1, 2, 3}, 1, false);

    // <mn||ef> as [(m,e)|(n,f)] (ph supermatrix): logical (m,n,e,f)
    Layout L_oovv_ph = make_layout("oovv_ph", G, {s(0, o, -1), s(2, v, 1)}, -1, {s(1, o, 1), s(3, v, -1)}, -1, 1);
    int b_oovv_ph = B.derived("V_oovv_ph", IC_OOVV, L_oovv_ph, {0, 1, 2, 3}, 1, false);
    // <mn||ef> as [(m,n<,f)|(e)]
    Layout L_oovv_2b = make_layout("oovv_2b", G, {s(0, o, 1), s(1, o, 1), s(3, v, -1)}, 0, {s(2, v, 1)}, -1, 1);
    int b_oovv_2b = B.derived("V_oovv_2b", IC_OOVV, L_oovv_2b, {0, 1, 2, 3}, 1, false);
    // <mn||ef> as [(m)|(n,ef<)]
    Layout L_oovv_3b = make_layout("oovv_3b", G, {s(0, o, 1)}, -1, {s(1, o, 1), s(2, v, -1), s(3, v, -1)}, 1, -1);
    int b_oovv_3b = B.derived("V_oovv_3b", IC_OOVV, L_oovv_3b, {0, 1, 2, 3}, 1, false);
    // <mn||ie> as [(m,i)|(n,e)], pair irrep 0 only: logical (m,n,i,e)
    Layout L_ooov_3a = make_layout("ooov_3a", G, {s(0, o, -1), s(2, o, 1)}, -1, {s(1, o, -1), s(3, v, 1)}, -1, -1, 0);
    int b_ooov_3a = B.derived("V_ooov_3a", IC_OOOV, L_ooov_3a, {0, 1, 2, 3}, 1, false);
    // <mn||ie> as [(m,n<,i)|(e)]
    Layout L_ooov_5b = make_layout("ooov_5b", G, {s(0, o, 1), s(1, o, 1), s(2, o, -1)}, 0, {s(3, v, 1)}, -1, 1);
    int b_ooov_5b = B.derived("V_ooov_5b", IC_OOOV, L_ooov_5b, {0, 1, 2, 3}, 1, false);
    // <mn||ej> = -<mn||je> as [(m,e,j)|(n)]: logical (m,n,e,j)
    Layout L_oovo_9c = make_layout("oovo_9c", G, {s(0, o, -1), s(2, v, 1), s(3, o, 1)}, -1, {s(1, o, 1)}, -1, 1);
    int b_oovo_9c = B.derived("V_oovo_9c", IC_OOOV, L_oovo_9c, {0, 1, 3, 2}, -1, false);
    // <mb||ij> = conj <ij||mb> as [(i,j<,b)|(m)]: logical (m,b,i,j)
    Layout L_ovoo_12 = make_layout("ovoo_12", G, {s(2, o, 1), s(3, o, 1), s(1, v, -1)}, 0, {s(0, o, 1)}, -1, 1);
    int b_ovoo_12 = B.derived("V_ovoo_12", IC_OOOV, L_ovoo_12, {2, 3, 0, 1}, 1, true);
    // <mn||ie> as [(i)|(m,n<,e)]: logical (m,n,i,e)
    Layout L_ooov_14f = make_layout("ooov_14f", G, {s(2, o, 1)}, -1, {s(0, o, 1), s(1, o, 1), s(3, v, -1)}, 0, 1);
    int b_ooov_14f = B.derived("V_ooov_14f", IC_OOOV, L_ooov_14f, {0, 1, 2, 3}, 1, false);
    // <mb||ej> = -<mb||je> as [(m,e)|(j,b)] (the ring W layout): logical (m,b,e,j)
    Layout L_W = make_layout("W", G, {s(0, o, -1), s(2, v, 1)}, -1, {s(3, o, -1), s(1, v, 1)}, -1, 1);
    int b_ring0 = B.derived("V_ovvo_ring", IC_OVOV, L_W, {0, 1, 3, 2}, -1, false);
    // <mb||ej> as [(m,b,j)|(e)]
    Layout L_ovvo_9f = make_layout("ovvo_9f", G, {s(0, o, 1), s(1, v, 1), s(3, o, -1)}, -1, {s(2, v, 1)}, -1, 1);
    int b_ovvo_9f = B.derived("V_ovvo_9f", IC_OVOV, L_ovvo_9f, {0, 1, 3, 2}, -1, false);
    // <na||if> as [(i,a)|(n,f)], pair irrep 0: logical (n,a,i,f)
    Layout L_ovov_14d = make_layout("ovov_14d", G, {s(2, o, -1), s(1, v, 1)}, -1, {s(0, o, -1), s(3, v, 1)}, -1, 1, 0);
    int b_ovov_14d = B.derived("V_ovov_14d", IC_OVOV, L_ovov_14d, {0, 1, 2, 3}, 1, false);
    // <ma||fe> as [(a,e)|(m,f)], pair irrep 0: logical (m,a,f,e)
    Layout L_ovvv_2a = make_layout("ovvv_2a", G, {s(1, v, -1), s(3, v, 1)}, -1, {s(0, o, -1), s(2, v, 1)}, -1, -1, 0);
    int b_ovvv_2a = B.derived("V_ovvv_2a", IC_OVVV, L_ovvv_2a, {0, 1, 2, 3}, 1, false);
    // <mb||ef> as [(m,e,b)|(f)]: logical (m,b,e,f)
    Layout L_ovvv_9b = make_layout("ovvv_9b", G, {s(0, o, 1), s(2, v, -1), s(1, v, 1)}, -1, {s(3, v, 1)}, -1, 1);
    int b_ovvv_9b = B.derived("V_ovvv_9b", IC_OVVV, L_ovvv_9b, {0, 1, 2, 3}, 1, false);
    // <ab||ej> = -conj <je||ab> as [(a,b<,j)|(e)]: logical (a,b,e,j)
    Layout L_vvvo_11 = make_layout("vvvo_11", G, {s(0, v, 1), s(1, v, 1), s(3, o, -1)}, 0, {s(2, v, 1)}, -1, 1);
    int b_vvvo_11 = B.derived("V_vvvo_11", IC_OVVV, L_vvvo_11, {3, 2, 0, 1}, -1, true);
    // <ma||ef> as [(m,ef<)|(a)]: logical (m,a,e,f)
    Layout L_ovvv_14e = make_layout("ovvv_14e", G, {s(0, o, 1), s(2, v, -1), s(3, v, -1)}, 1, {s(1, v, 1)}, -1, -1);
    int b_ovvv_14e = B.derived("V_ovvv_14e", IC_OVVV, L_ovvv_14e, {0, 1, 2, 3}, 1, false);

    // ------------------------------------------------------------------ tau
    int b_tau = P.buf("tau", L_T2.total, BUF_SCRATCH);
    int b_taut = P.buf("tau~", L_T2.total, BUF_SCRATCH);
    P.b_tau = b_tau;
    Layout L_Fme_v = make_layout("Fme_v", G, {s(0, o, -1), s(1, v, 1)}, -1, {}, -1, 1, 0);
    Layout L_Fme_m = make_layout("Fme_m", G, {s(0, o, 1)}, -1, {s(1, v, 1)}, -1, 1);
    int b_Fme = P.buf("Fme", L_T1.total, BUF_SCRATCH);
    Layout L_Fae_v = make_layout("Fae_v", G, {s(0, v, -1), s(1, v, 1)}, -1, {}, -1, 1, 0);
    Layout L_Fae_m = make_layout("Fae_m", G, {s(0, v, 1)}, -1, {s(1, v, 1)}, -1, 1);
    int nvv0 = (int)L_Fae_m.total;
    int b_Fae = P.buf("Fae", nvv0, BUF_SCRATCH);
    Layout L_tt_2b = make_layout("tau~_2b", G, {s(2, v, 1)}, -1, {s(0, o, 1), s(1, o, 1), s(3, v, -1)}, 0, 1);
    int b_tt2b = P.buf("tau~_2b", L_tt_2b.total, BUF_SCRATCH);
    Layout L_Fmi_v = make_layout("Fmi_v", G, {s(0, o, -1), s(1, o, 1)}, -1, {}, -1, 1, 0);
    Layout L_Fmi_m = make_layout("Fmi_m", G, {s(0, o, 1)}, -1, {s(1, o, 1)}, -1, 1);
    int b_Fmi = P.buf("Fmi", L_Fmi_m.total, BUF_SCRATCH);
    Layout L_tt_3b = make_layout("tau~_3b", G, {s(1, o, 1), s(2, v, -1), s(3, v, -1)}, 1, {s(0, o, 1)}, -1, -1);
    int b_tt3b = P.buf("tau~_3b", L_tt_3b.total, BUF_SCRATCH);
    // tau = t2 + t_i^a t_j^b - t_i^b t_j^a   (T1 logical (i,a); T2 logical (i,j,a,b))
    std::vector<T> tt = {T{{0, 2}, 1, {1, 3}}, T{{0, 3}, -1, {1, 2}}};
    auto emit_tau_F = [&]() {
        B.axpby("tau=t2", b_tau, P.b_t2, L_T2.total, 1.0, 0, false);
        B.gather("tau+=t1t1", b_tau, L_T2, P.b_t1, L_T1, tt, 1.0, 1, false, P.b_t1, &L_T1);
        B.axpby("tau~=t2", b_taut, P.b_t2, L_T2.total, 1.0, 0, false);
        B.gather("tau~+=t1t1/2", b_taut, L_T2, P.b_t1, L_T1, tt, 0.5, 1, false, P.b_t1, &L_T1);
        // F_me = sum_nf <mn||ef> t_n^f
        B.gemm("Fme", b_oovv_ph, L_oovv_ph, false, false, P.b_t1, L_T1w, false, false, b_Fme, L_Fme_v, 1.0, 0);
        // F_ae = sum_mf t_m^f <ma||fe> - sum_{m<n,f} tau~_mn^af <mn||ef>
        B.gemm("Fae.1", b_ovvv_2a, L_ovvv_2a, false, false, P.b_t1, L_T1v, false, false, b_Fae, L_Fae_v, 1.0, 0);
        B.gather("tau~->2b", b_tt2b, L_tt_2b, b_taut, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        B.gemm("Fae.2", b_tt2b, L_tt_2b, false, false, b_oovv_2b, L_oovv_2b, false, false, b_Fae, L_Fae_m, -1.0, 1);
        // F_mi = sum_ne t_n^e <mn||ie> + sum_{n,e<f} tau~_in^ef <mn||ef>
        B.gemm("Fmi.1", b_ooov_3a, L_ooov_3a, false, false, P.b_t1, L_T1v, false, false, b_Fmi, L_Fmi_v, 1.0, 0);
        B.gather("tau~->3b", b_tt3b, L_tt_3b, b_taut, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        B.gemm("Fmi.2", b_oovv_3b, L_oovv_3b, false, false, b_tt3b, L_tt_3b, false, false, b_Fmi, L_Fmi_m, 1.0, 1);
    };
    emit_tau_F();

    // ------------------------------------------------------------ W'_mnij
    Layout L_Wp = make_layout("W'", G, {s(0, o, 1), s(1, o, 1)}, 0, {s(2, o, 1), s(3, o, 1)}, 0, 1);
    int b_Wp = P.buf("W'", L_Wp.total, BUF_SCRATCH);
    B.axpby("W'=<mn||ij>", b_Wp, b_oooo, L_Wp.total, 1.0, 0, false);
    Layout L_X5 = make_layout("X5", G, {s(0, o, 1), s(1, o, 1), s(2, o, -1)}, 0, {s(3, o, 1)}, -1, 1);
    int b_X5 = P.buf("X5", L_X5.total, BUF_SCRATCH);
    B.gemm("W'.t1", b_ooov_5b, L_ooov_5b, false, false, P.b_t1, L_T1, true, false, b_X5, L_X5, 1.0, 0);
    B.gather("W'+=P(ij)X5", b_Wp, L_Wp, b_X5, L_X5, {T{{0, 1, 2, 3}, 1, {}}, T{{0, 1, 3, 2}, -1, {}}}, 1.0, 1);
    B.gemm("W'.tau", b_oovv, L_OOVV, false, false, b_tau, L_T2, true, false, b_Wp, L_Wp, 1.0, 1);

    // --------------------------------------------------------- T2 residual
    B.axpby("r2=<ab||ij>", P.b_r2, b_oovv, L_T2.total, 1.0, 0, true);
    B.gemm("hh-ladder", b_Wp, L_Wp, true, false, b_tau, L_T2, false, false, P.b_r2, L_T2, 1.0, 1);
    B.gemm("pp-ladder", b_tau, L_T2, false, false, b_vvvv, L_VVVV, true, false, P.b_r2, L_T2, 1.0, 1);
    // Z_ij^am = -sum_{e<f} <ma||ef> tau_ij^ef ;  r2 += -P(ab) sum_m t_m^b Z_ij^am
    Layout L_Z1 = make_layout("Z1", G, {s(0, o, 1), s(1, v, 1)}, -1, {s(2, o, 1), s(3, o, 1)}, 0, 1);
    int b_Z1 = P.buf("Z1", L_Z1.total, BUF_SCRATCH);
    B.gemm("Z", b_ovvv, L_OVVV, false, false, b_tau, L_T2, true, false, b_Z1, L_Z1, -1.0, 0);
    Layout L_Z2 = make_layout("Z2", G, {s(2, o, 1), s(3, o, 1), s(1, v, -1)}, 0, {s(0, o, 1)}, -1, 1);
    int b_Z2 = P.buf("Z2", L_Z2.total, BUF_SCRATCH);
    B.gather("Z1->Z2", b_Z2, L_Z2, b_Z1, L_Z1, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
    Layout L_Y8 = make_layout("Y8", G, {s(0, o, 1), s(1, o, 1), s(2, v, -1)}, 0, {s(3, v, 1)}, -1, 1);
    int b_Y8 = P.buf("Y8", L_Y8.total, BUF_SCRATCH);
    B.gemm("Z.t1", b_Z2, L_Z2, false, false, P.b_t1, L_T1, false, false, b_Y8, L_Y8, 1.0, 0);
    // Y8 also collects -Y10a and -Y12 below (the same layout; their
    // antisymmetrisers are the negative of Y8's), then one pass adds
    // -P(ab) Y8 to r2

    // ---------------------------------------------------------------- ring
    int b_W = P.buf("W", L_W.total, BUF_SCRATCH);
    Layout L_X9b = make_layout("X9b", G, {s(0, o, 1), s(1, v, -1), s(2, v, 1)}, -1, {s(3, o, 1)}, -1, 1);
    int b_X9b = P.buf("X9b", L_X9b.total, BUF_SCRATCH);
    B.gemm("W.t1.ovvv", b_ovvv_9b, L_ovvv_9b, false, false, P.b_t1, L_T1, true, false, b_X9b, L_X9b, 1.0, 0);
    Layout L_X9c = make_layout("X9c", G, {s(0, o, -1), s(1, v, 1), s(2, o, 1)}, -1, {s(3, v, 1)}, -1, 1);
    int b_X9c = P.buf("X9c", L_X9c.total, BUF_SCRATCH);
    B.gemm("W.t1.ooov", b_oovo_9c, L_oovo_9c, false, false, P.b_t1, L_T1, false, false, b_X9c, L_X9c, -1.0, 0);
    // W = <mb||ej> + X9b + X9c in one pass
    B.gather_sum("W=V+X9b+X9c", b_W, L_W, {{b_ring0, &L_W}, {b_X9b, &L_X9b}, {b_X9c, &L_X9c}},
                 {T{{0, 1, 2, 3}, 1, {}}, T{{0, 2, 1, 3}, 1, {}}, T{{0, 2, 3, 1}, 1, {}}}, 1.0, 0);
    // U_(n,f),(j,b) = 1/2 t_jn^fb + t_j^f t_n^b  : logical (n,f,j,b)
    Layout L_U = make_layout("U", G, {s(0, o, 1), s(1, v, -1)}, -1, {s(2, o, -1), s(3, v, 1)}, -1, 1);
    int b_U = P.buf("U", L_U.total, BUF_SCRATCH);
    B.gather("U=t2/2", b_U, L_U, P.b_t2, L_T2, {T{{2, 0, 1, 3}, 1, {}}}, 0.5, 0);
    B.gather("U+=t1t1", b_U, L_U, P.b_t1, L_T1, {T{{2, 1}, 1, {0, 3}}}, 1.0, 1, false, P.b_t1, &L_T1);
    B.gemm("W.U", b_oovv_ph, L_oovv_ph, false, false, b_U, L_U, false, false, b_W, L_W, -1.0, 1);
    // ring: X_(i,a),(j,b) = sum_(m,e) t_im^ae W_mbej
    Layout L_Tr = make_layout("Tring", G, {s(0, o, -1), s(2, v, 1)}, -1, {s(1, o, -1), s(3, v, 1)}, -1, -1);
    int b_Tr = P.buf("Tring", L_Tr.total, BUF_SCRATCH);
    B.gather("t2->ring", b_Tr, L_Tr, P.b_t2, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
    Layout L_X = make_layout("Xring", G, {s(0, o, -1), s(1, v, 1)}, -1, {s(2, o, -1), s(3, v, 1)}, -1, -1);
    int b_X = P.buf("Xring", L_X.total, BUF_SCRATCH);
    B.gemm("ring", b_Tr, L_Tr, false, false, b_W, L_W, false, false, b_X, L_X, 1.0, 0);
    // Y9_ijab = sum_me t_i^e t_m^a <mb||ej>
    Layout L_Q = make_layout("Q", G, {s(0, o, 1), s(1, v, 1), s(2, o, -1)}, -1, {s(3, o, 1)}, -1, 1);
    int b_Q = P.buf("Q", L_Q.total, BUF_SCRATCH);
    B.gemm("Q", b_ovvo_9f, L_ovvo_9f, false, false, P.b_t1, L_T1, true, false, b_Q, L_Q, 1.0, 0);
    Layout L_Q2 = make_layout("Q2", G, {s(3, o, 1), s(2, o, 1), s(1, v, -1)}, -1, {s(0, o, 1)}, -1, 1);
    int b_Q2 = P.buf("Q2", L_Q2.total, BUF_SCRATCH);
    B.gather("Q->Q2", b_Q2, L_Q2, b_Q, L_Q, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
    Layout L_Y9 = make_layout("Y9", G, {s(0, o, 1), s(1, o, 1), s(2, v, -1)}, -1, {s(3, v, 1)}, -1, 1);
    int b_Y9 = P.buf("Y9", L_Y9.total, BUF_SCRATCH);
    B.gemm("Y9", b_Q2, L_Q2, false, false, P.b_t1, L_T1, false, false, b_Y9, L_Y9, 1.0, 0);
    B.gather("r2+=PP X", P.b_r2, L_T2, b_X, L_X,
             {T{{0, 2, 1, 3}, 1, {}}, T{{1, 2, 0, 3}, -1, {}}, T{{0, 3, 1, 2}, -1, {}}, T{{1, 3, 0, 2}, 1, {}}}, 1.0, 1);
    B.gather("r2+=-PP Y9", P.b_r2, L_T2, b_Y9, L_Y9,
             {T{{0, 1, 3, 2}, -1, {}}, T{{1, 0, 3, 2}, 1, {}}, T{{0, 1, 2, 3}, 1, {}}, T{{1, 0, 2, 3}, -1, {}}}, 1.0, 1);

    // ------------------------------------------------------------ F terms
    // F'_be = F_be - 1/2 sum_m t_m^b F_me
    Layout L_Fbe = make_layout("Fbe", G, {s(0, v, 1)}, -1, {s(1, v, 1)}, -1, 1);
    int b_Fbe = P.buf("Fbe", L_Fbe.total, BUF_SCRATCH);
    B.axpby("Fbe=Fae", b_Fbe, b_Fae, L_Fbe.total, 1.0, 0, false);
    B.gemm("Fbe.t1", P.b_t1, L_T1, true, false, b_Fme, L_Fme_m, false, false, b_Fbe, L_Fbe, -0.5, 1);
    Layout L_T10a = make_layout("T10a", G, {s(0, o, 1), s(1, o, 1), s(2, v, -1)}, 0, {s(3, v, 1)}, -1, 1);
    int b_T10a = P.buf("T10a", L_T10a.total, BUF_SCRATCH);
    B.gather("t2->10a", b_T10a, L_T10a, P.b_t2, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
    // Y10a = sum_e t_ij^ae F'_be enters r2 as P(ab) Y10a: collected into Y8 as -Y10a
    B.gemm("t2.Fbe", b_T10a, L_T10a, false, false, b_Fbe, L_Fbe, true, false, b_Y8, L_Y8, -1.0, 1);
    // F'_mj = F_mj + 1/2 sum_e t_j^e F_me
    Layout L_Fmj = make_layout("Fmj", G, {s(0, o, 1)}, -1, {s(1, o, 1)}, -1, 1);
    int b_Fmj = P.buf("Fmj", L_Fmj.total, BUF_SCRATCH);
    B.axpby("Fmj=Fmi", b_Fmj, b_Fmi, L_Fmj.total, 1.0, 0, false);
    B.gemm("Fmj.t1", b_Fme, L_Fme_m, false, false, P.b_t1, L_T1, true, false, b_Fmj, L_Fmj, 0.5, 1);
    P.b_Fbe = b_Fbe;
    P.b_Fmj = b_Fmj;
    P.fbe_diag.assign(v->n, -1);
    P.fmj_diag.assign(o->n, -1);
    L_Fbe.for_each([&](int64_t k, const int* p) { if (p[0] == p[1]) P.fbe_diag[p[0]] = k; });
    L_Fmj.for_each([&](int64_t k, const int* p) { if (p[0] == p[1]) P.fmj_diag[p[0]] = k; });
    Layout L_T10b = make_layout("T10b", G, {s(2, v, 1), s(3, v, 1), s(0, o, -1)}, 0, {s(1, o, 1)}, -1, 1);
    int b_T10b = P.buf("T10b", L_T10b.total, BUF_SCRATCH);
    B.gather("t2->10b", b_T10b, L_T10b, P.b_t2, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
    Layout L_Y10b = make_layout("Y10b", G, {s(0, v, 1), s(1, v, 1), s(2, o, -1)}, 0, {s(3, o, 1)}, -1, 1);
    int b_Y10b = P.buf("Y10b", L_Y10b.total, BUF_SCRATCH);
    B.gemm("t2.Fmj", b_T10b, L_T10b, false, false, b_Fmj, L_Fmj, false, false, b_Y10b, L_Y10b, 1.0, 0);
    // P(ij) sum_e t_i^e <ab||ej> (Y11): the same layout and antisymmetriser as
    // -P(ij) Y10b, so it accumulates into Y10b and one pass adds both to r2
    B.gemm("t1.vvvo", b_vvvo_11, L_vvvo_11, false, false, P.b_t1, L_T1, true, false, b_Y10b, L_Y10b, 1.0, 1);
    B.gather("r2+=-P(ij)Y10b", P.b_r2, L_T2, b_Y10b, L_Y10b, {T{{2, 3, 0, 1}, -1, {}}, T{{2, 3, 1, 0}, 1, {}}}, 1.0, 1);
    // -P(ab) sum_m t_m^a <mb||ij> (Y12): collected into Y8 as -Y12
    B.gemm("t1.ovoo", b_ovoo_12, L_ovoo_12, false, false, P.b_t1, L_T1, false, false, b_Y8, L_Y8, -1.0, 1);
    B.gather("r2+=-P(ab)Y8", P.b_r2, L_T2, b_Y8, L_Y8, {T{{0, 1, 2, 3}, -1, {}}, T{{0, 1, 3, 2}, 1, {}}}, 1.0, 1);
    B.diag("r2-=D2*t2", P.b_r2, P.b_D2, P.b_t2, L_T2.total);

    // --------------------------------------------------------- T1 residual
    Layout L_R1v = make_layout("R1v", G, {s(0, o, -1), s(1, v, 1)}, -1, {}, -1, 1, 0);
    B.gemm("t1.Fae", P.b_t1, L_T1, false, false, b_Fae, L_Fae_m, true, false, P.b_r1, L_T1, 1.0, 0);
    B.gemm("Fmi.t1", b_Fmi, L_Fmi_m, true, false, P.b_t1, L_T1, false, false, P.b_r1, L_T1, -1.0, 1);
    B.gemm("t2.Fme", b_Tr, L_Tr, false, false, b_Fme, L_Fme_v, false, false, P.b_r1, L_R1v, 1.0, 1);
    B.gemm("t1.ovov", b_ovov_14d, L_ovov_14d, false, false, P.b_t1, L_T1v, false, false, P.b_r1, L_R1v, -1.0, 1);
    Layout L_T14e = make_layout("T14e", G, {s(0, o, 1)}, -1, {s(1, o, 1), s(2, v, -1), s(3, v, -1)}, 1, -1);
    int b_T14e = P.buf("T14e", L_T14e.total, BUF_SCRATCH);
    B.gather("t2->14e", b_T14e, L_T14e, P.b_t2, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
    B.gemm("t2.ovvv", b_T14e, L_T14e, false, false, b_ovvv_14e, L_ovvv_14e, false, false, P.b_r1, L_T1, -1.0, 1);
    Layout L_T14f = make_layout("T14f", G, {s(0, o, 1), s(1, o, 1), s(3, v, -1)}, 0, {s(2, v, 1)}, -1, 1);
    int b_T14f = P.buf("T14f", L_T14f.total, BUF_SCRATCH);
    B.gather("t2->14f", b_T14f, L_T14f, P.b_t2, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
    B.gemm("ooov.t2", b_ooov_14f, L_ooov_14f, false, false, b_T14f, L_T14f, false, false, P.b_r1, L_T1, -1.0, 1);
    B.diag("r1-=D1*t1", P.b_r1, P.b_D1, P.b_t1, L_T1.total);


    // =====================================================================
    // (0h,1p) sector: Bloch equation Q Hbar_N (P + S) = S H_eff on the
    // {1p, 2p1h} space, sigma(x) = Hbar_N r(x), r(x) = e_x + s_x.
    if (!S.active.empty()) {
        P.has01 = true;
        std::vector<int> act(S.active);
        std::sort(act.begin(), act.end());
        for (size_t k = 1; k < act.size(); ++k)
            if (act[k] == act[k - 1]) throw std::invalid_argument("duplicate active spinor");
        std::vector<int> xl;
        for (int gidx : act) {
            if (gidx < S.nocc || gidx >= S.nocc + S.nvirt) throw std::invalid_argument("active spinor is not virtual");
            xl.push_back(S.irrep[gidx]);
        }
        P.X = Space::make(G, act, xl);
        const Space* x = &P.X;
        P.x_vpos.assign(x->n, 0);
        P.x_order.assign(x->n, 0);
        for (int q = 0; q < x->n; ++q) {
            int gidx = x->glob[q];
            for (int a = 0; a < v->n; ++a)
                if (v->glob[a] == gidx) P.x_vpos[q] = a;
            for (size_t k = 0; k < S.active.size(); ++k)
                if (S.active[k] == gidx) P.x_order[q] = (int)k;
        }
        // amplitudes: S1 (x,a) = [g][x_g][v_g] (all virtuals a; active a are model-space entries),
        //             S2 (x,j,a,b) = [G][(x,j)][ab<]
        P.L_S1 = make_layout("S1", G, {s(0, x, 1)}, -1, {s(1, v, 1)}, -1, 1);
        P.L_S2 = make_layout("S2", G, {s(0, x, 1), s(1, o, 1)}, -1, {s(2, v, 1), s(3, v, 1)}, 0, 1);
        P.L_Heff = make_layout("Heff", G, {s(0, x, 1)}, -1, {s(1, x, 1)}, -1, 1);
        const Layout& L_S1 = P.L_S1;
        const Layout& L_S2 = P.L_S2;
        const Layout& L_Heff = P.L_Heff;
        Layout L_S1v = make_layout("S1v", G, {s(0, x, -1), s(1, v, 1)}, -1, {}, -1, 1, 0);
        P.b_s1 = P.buf("s1", L_S1.total, BUF_IN_S1);
        P.b_s2 = P.buf("s2", L_S2.total, BUF_IN_S2);
        P.b_rs1 = P.buf("rs1", L_S1.total, BUF_OUT_RS1);
        P.b_rs2 = P.buf("rs2", L_S2.total, BUF_OUT_RS2);
        // denominators D_x^a = e_x - e_a, D_xj^ab = e_x + e_j - e_a - e_b; model-space entries masked
        P.D1x.assign(L_S1.total, -1.0);   // masked entries: any negative value keeps D + Delta away from 0
        P.mask1.assign(L_S1.total, 0.0);
        std::vector<cplx> eid(L_S1.total, 0.0);
        L_S1.for_each([&](int64_t k, const int* p) {
            bool model = false;
            for (int q = 0; q < x->n; ++q)
                if (P.x_vpos[q] == p[1]) model = true;
            if (!model) {
                P.D1x[k] = S.eps[x->glob[p[0]]] - S.eps[v->glob[p[1]]];
                P.mask1[k] = 1.0;
            }
            if (P.x_vpos[p[0]] == p[1]) eid[k] = 1.0;
        });
        P.D2x.assign(L_S2.total, 0.0);
        L_S2.for_each([&](int64_t k, const int* p) {
            P.D2x[k] = S.eps[x->glob[p[0]]] + S.eps[o->glob[p[1]]] - S.eps[v->glob[p[2]]] - S.eps[v->glob[p[3]]];
        });
        P.b_D1x = P.buf("D1x", L_S1.total, BUF_REAL);
        P.b_D2x = P.buf("D2x", L_S2.total, BUF_REAL);
        P.b_mask1 = P.buf("mask1", L_S1.total, BUF_REAL);
        int b_eid = P.buf("Eid", L_S1.total, BUF_CONST);
        P.const_host.push_back({b_eid, std::move(eid)});

        // ---------------------------------------------------- Hbar (prepare)
        B.out = &P.ops01_prep;
        emit_tau_F();
        int b_t1c = P.buf("t1(01)", L_T1.total, BUF_SCRATCH);
        B.axpby("t1 copy", b_t1c, P.b_t1, L_T1.total, 1.0, 0, false);
        int b_tauc = P.buf("tau(01)", L_T2.total, BUF_SCRATCH);
        B.axpby("tau copy", b_tauc, b_tau, L_T2.total, 1.0, 0, false);
        int b_Fov = P.buf("Fbar_ov", L_T1.total, BUF_SCRATCH);
        B.axpby("Fbar_ov=Fme", b_Fov, b_Fme, L_T1.total, 1.0, 0, false);
        // Fbar_vv = F_ae + diag(e_v) - 1/2 sum_m t_m^a F_me
        std::vector<cplx> dv(L_Fae_m.total, 0.0), dov(L_Fmi_m.total, 0.0);
        L_Fae_m.for_each([&](int64_t k, const int* p) { if (p[0] == p[1]) dv[k] = S.eps[v->glob[p[0]]]; });
        L_Fmi_m.for_each([&](int64_t k, const int* p) { if (p[0] == p[1]) dov[k] = S.eps[o->glob[p[0]]]; });
        int b_dv = P.buf("diag e_v", L_Fae_m.total, BUF_CONST);
        int b_do = P.buf("diag e_o", L_Fmi_m.total, BUF_CONST);
        P.const_host.push_back({b_dv, std::move(dv)});
        P.const_host.push_back({b_do, std::move(dov)});
        int b_Fvv = P.buf("Fbar_vv", L_Fae_m.total, BUF_SCRATCH);
        B.axpby("Fbar_vv=Fae", b_Fvv, b_Fae, L_Fae_m.total, 1.0, 0, false);
        B.axpby("Fbar_vv+=e", b_Fvv, b_dv, L_Fae_m.total, 1.0, 1, false);
        B.gemm("Fbar_vv.t1", P.b_t1, L_T1, true, false, b_Fme, L_Fme_m, false, false, b_Fvv, L_Fae_m, -0.5, 1);
        // Fbar_oo = F_mi + diag(e_o) + 1/2 sum_e F_me t_i^e
        int b_Foo = P.buf("Fbar_oo", L_Fmi_m.total, BUF_SCRATCH);
        P.b_Fvv01 = b_Fvv;
        P.b_Foo01 = b_Foo;
        P.fvv_diag.assign(v->n, 0);
        P.foo_diag.assign(o->n, 0);
        L_Fae_m.for_each([&](int64_t k, const int* p) { if (p[0] == p[1]) P.fvv_diag[p[0]] = k; });
        L_Fmi_m.for_each([&](int64_t k, const int* p) { if (p[0] == p[1]) P.foo_diag[p[0]] = k; });
        B.axpby("Fbar_oo=Fmi", b_Foo, b_Fmi, L_Fmi_m.total, 1.0, 0, false);
        B.axpby("Fbar_oo+=e", b_Foo, b_do, L_Fmi_m.total, 1.0, 1, false);
        B.gemm("Fbar_oo.t1", b_Fme, L_Fme_m, false, false, P.b_t1, L_T1, true, false, b_Foo, L_Fmi_m, 0.5, 1);
        // Wbar_amef = <am||ef> - sum_n t_n^a <nm||ef>, layout [(m,ef<)|(a)]
        int b_Wam = P.buf("Wbar_amef", L_ovvv_14e.total, BUF_SCRATCH);
        B.axpby("Wbar_amef=-<ma||ef>", b_Wam, b_ovvv_14e, L_ovvv_14e.total, -1.0, 0, false);
        B.gemm("Wbar_amef.t1", b_oovv_3b, L_oovv_3b, true, false, P.b_t1, L_T1, false, false, b_Wam, L_ovvv_14e, -1.0, 1);
        // Wbar_mbej (ring layout) = <mb||ej> + sum_f t_j^f <mb||ef> - sum_n t_n^b <mn||ej>
        //                           - sum_nf (t_jn^fb + t_j^f t_n^b) <mn||ef>
        int b_Wb = P.buf("Wbar_mbej", L_W.total, BUF_SCRATCH);
        int b_X9b01 = P.buf("X9b(01)", L_X9b.total, BUF_SCRATCH);
        int b_X9c01 = P.buf("X9c(01)", L_X9c.total, BUF_SCRATCH);
        int b_U01 = P.buf("U(01)", L_U.total, BUF_SCRATCH);
        B.axpby("Wbar=<mb||ej>", b_Wb, b_ring0, L_W.total, 1.0, 0, false);
        B.gemm("Wbar.t1.ovvv", b_ovvv_9b, L_ovvv_9b, false, false, P.b_t1, L_T1, true, false, b_X9b01, L_X9b, 1.0, 0);
        B.gather("Wbar+=X9b", b_Wb, L_W, b_X9b01, L_X9b, {T{{0, 2, 1, 3}, 1, {}}}, 1.0, 1);
        B.gemm("Wbar.t1.ooov", b_oovo_9c, L_oovo_9c, false, false, P.b_t1, L_T1, false, false, b_X9c01, L_X9c, -1.0, 0);
        B.gather("Wbar+=X9c", b_Wb, L_W, b_X9c01, L_X9c, {T{{0, 2, 3, 1}, 1, {}}}, 1.0, 1);
        B.gather("U'=t2", b_U01, L_U, P.b_t2, L_T2, {T{{2, 0, 1, 3}, 1, {}}}, 1.0, 0);
        B.gather("U'+=t1t1", b_U01, L_U, P.b_t1, L_T1, {T{{2, 1}, 1, {0, 3}}}, 1.0, 1, false, P.b_t1, &L_T1);
        B.gemm("Wbar.U'", b_oovv_ph, L_oovv_ph, false, false, b_U01, L_U, false, false, b_Wb, L_W, -1.0, 1);
        // Xc_mbej = <mb||ej> - sum_nf t_nj^bf <mn||ef>  (ring layout, then [(m,b,j)|(e)])
        int b_Xc = P.buf("Xc ring", L_W.total, BUF_SCRATCH);
        int b_Tnf = P.buf("t_nj^bf", L_U.total, BUF_SCRATCH);
        B.axpby("Xc=<mb||ej>", b_Xc, b_ring0, L_W.total, 1.0, 0, false);
        B.gather("t2->(n,f|j,b)", b_Tnf, L_U, P.b_t2, L_T2, {T{{0, 2, 3, 1}, 1, {}}}, 1.0, 0);
        B.gemm("Xc.t2", b_oovv_ph, L_oovv_ph, false, false, b_Tnf, L_U, false, false, b_Xc, L_W, -1.0, 1);
        int b_Xc9f = P.buf("Xc", L_ovvo_9f.total, BUF_SCRATCH);
        B.gather("Xc->(m,b,j|e)", b_Xc9f, L_ovvo_9f, b_Xc, L_W, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        // t2 as [(m)|(j,ab<)] and in the ring layout
        Layout L_Tm = make_layout("T2(m|j,ab<)", G, {s(0, o, 1)}, -1, {s(1, o, 1), s(2, v, -1), s(3, v, -1)}, 1, -1);
        int b_Tm = P.buf("T2(m|j,ab<)", L_Tm.total, BUF_SCRATCH);
        B.gather("t2->(m|j,ab<)", b_Tm, L_Tm, P.b_t2, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        int b_Tr01 = P.buf("Tring(01)", L_Tr.total, BUF_SCRATCH);
        B.gather("t2->ring(01)", b_Tr01, L_Tr, P.b_t2, L_T2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);

        // ------------------------------------------------ sigma + residual
        B.out = &P.ops01;
        int b_r1x = P.buf("r1(x)", L_S1.total, BUF_SCRATCH);
        B.axpby("r1=s1", b_r1x, P.b_s1, L_S1.total, 1.0, 0, false);
        B.mul("r1*=mask", b_r1x, P.b_mask1, L_S1.total);
        B.axpby("r1+=e_x", b_r1x, b_eid, L_S1.total, 1.0, 1, false);
        // rho_xj^ef = s_xj^ef + r(x)^e t_j^f - r(x)^f t_j^e
        int b_rho = P.buf("rho", L_S2.total, BUF_SCRATCH);
        B.axpby("rho=s2", b_rho, P.b_s2, L_S2.total, 1.0, 0, false);
        B.gather("rho+=r1t1", b_rho, L_S2, b_r1x, L_S1, {T{{0, 2}, 1, {1, 3}}, T{{0, 3}, -1, {1, 2}}}, 1.0, 1, false,
                 b_t1c, &L_T1);
        // S2 ladder: sigma2 = sum_{e<f} <ab||ef> rho_xj^ef
        B.gemm("S2-ladder", b_rho, L_S2, false, false, b_vvvv, L_VVVV, true, false, P.b_rs2, L_S2, 1.0, 0);
        // -P(ab) sum_m t_m^b Z_xj^am,  Z_xj^am = -sum_{e<f} <ma||ef> rho_xj^ef
        Layout L_Z1x = make_layout("Z1x", G, {s(0, o, 1), s(1, v, 1)}, -1, {s(2, x, 1), s(3, o, 1)}, -1, 1);
        int b_Z1x = P.buf("Z1x", L_Z1x.total, BUF_SCRATCH);
        B.gemm("S2.Z", b_ovvv, L_OVVV, false, false, b_rho, L_S2, true, false, b_Z1x, L_Z1x, -1.0, 0);
        Layout L_Z2x = make_layout("Z2x", G, {s(2, x, 1), s(3, o, 1), s(1, v, -1)}, -1, {s(0, o, 1)}, -1, 1);
        int b_Z2x = P.buf("Z2x", L_Z2x.total, BUF_SCRATCH);
        B.gather("Z1x->Z2x", b_Z2x, L_Z2x, b_Z1x, L_Z1x, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        Layout L_Y4 = make_layout("Y4x", G, {s(0, x, 1), s(1, o, 1), s(2, v, -1)}, -1, {s(3, v, 1)}, -1, 1);
        int b_Y4 = P.buf("Y4x", L_Y4.total, BUF_SCRATCH);
        B.gemm("S2.Z.t1", b_Z2x, L_Z2x, false, false, b_t1c, L_T1, false, false, b_Y4, L_Y4, 1.0, 0);
        B.gather("rs2+=-P(ab)Y4", P.b_rs2, L_S2, b_Y4, L_Y4, {T{{0, 1, 2, 3}, -1, {}}, T{{0, 1, 3, 2}, 1, {}}}, 1.0, 1);
        // hole-hole part: sum_{m<n} tau_mn^ab (X_mn,xj + w_mn,xj)
        Layout L_Xpp = make_layout("X''", G, {s(0, o, 1), s(1, o, 1)}, 0, {s(2, x, 1), s(3, o, 1)}, -1, 1);
        int b_Xpp = P.buf("X''", L_Xpp.total, BUF_SCRATCH);
        B.gemm("S2.X", b_oovv, L_OOVV, false, false, b_rho, L_S2, true, false, b_Xpp, L_Xpp, 1.0, 0);
        Layout L_w = make_layout("w", G, {s(0, o, 1), s(1, o, 1), s(2, o, -1)}, 0, {s(3, x, 1)}, -1, 1);
        int b_w = P.buf("w", L_w.total, BUF_SCRATCH);
        B.gemm("S2.w", b_ooov_5b, L_ooov_5b, false, false, b_r1x, L_S1, true, false, b_w, L_w, -1.0, 0);
        B.gather("X''+=w", b_Xpp, L_Xpp, b_w, L_w, {T{{0, 1, 3, 2}, 1, {}}}, 1.0, 1);
        B.gemm("S2.hh", b_Xpp, L_Xpp, true, false, b_tauc, L_T2, false, false, P.b_rs2, L_S2, 1.0, 1);
        // sum_e <ab||ej> r(x)^e
        Layout L_Y6 = make_layout("Y6x", G, {s(0, v, 1), s(1, v, 1), s(2, o, -1)}, 0, {s(3, x, 1)}, -1, 1);
        int b_Y6 = P.buf("Y6x", L_Y6.total, BUF_SCRATCH);
        B.gemm("S2.vvvo", b_vvvo_11, L_vvvo_11, false, false, b_r1x, L_S1, true, false, b_Y6, L_Y6, 1.0, 0);
        B.gather("rs2+=Y6", P.b_rs2, L_S2, b_Y6, L_Y6, {T{{2, 3, 1, 0}, 1, {}}}, 1.0, 1);
        // P(ab) sum_e Fbar_be s_xj^ae
        Layout L_S7 = make_layout("S2(x,j,a|e)", G, {s(0, x, 1), s(1, o, 1), s(2, v, -1)}, -1, {s(3, v, 1)}, -1, 1);
        int b_S7 = P.buf("S2(x,j,a|e)", L_S7.total, BUF_SCRATCH);
        B.gather("s2->(x,j,a|e)", b_S7, L_S7, P.b_s2, L_S2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        int b_Y7 = P.buf("Y7x", L_S7.total, BUF_SCRATCH);
        B.gemm("S2.Fvv", b_S7, L_S7, false, false, b_Fvv, L_Fae_m, true, false, b_Y7, L_S7, 1.0, 0);
        B.gather("rs2+=P(ab)Y7", P.b_rs2, L_S2, b_Y7, L_S7, {T{{0, 1, 2, 3}, 1, {}}, T{{0, 1, 3, 2}, -1, {}}}, 1.0, 1);
        // -sum_m Fbar_mj s_xm^ab
        Layout L_S8 = make_layout("S2(x,ab<|m)", G, {s(0, x, 1), s(2, v, -1), s(3, v, -1)}, 1, {s(1, o, 1)}, -1, -1);
        int b_S8 = P.buf("S2(x,ab<|m)", L_S8.total, BUF_SCRATCH);
        B.gather("s2->(x,ab<|m)", b_S8, L_S8, P.b_s2, L_S2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        int b_Y8 = P.buf("Y8x", L_S8.total, BUF_SCRATCH);
        B.gemm("S2.Foo", b_S8, L_S8, false, false, b_Foo, L_Fmi_m, false, false, b_Y8, L_S8, 1.0, 0);
        B.gather("rs2+=-Y8", P.b_rs2, L_S2, b_Y8, L_S8, {T{{0, 1, 2, 3}, -1, {}}}, 1.0, 1);
        // P(ab) sum_me Wbar_mbej s_xm^ae  (ring)
        Layout L_S9 = make_layout("S2 ring", G, {s(0, x, -1), s(2, v, 1)}, -1, {s(1, o, -1), s(3, v, 1)}, -1, -1);
        int b_S9 = P.buf("S2 ring", L_S9.total, BUF_SCRATCH);
        B.gather("s2->ring", b_S9, L_S9, P.b_s2, L_S2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        Layout L_Y9x = make_layout("Y9x", G, {s(0, x, -1), s(1, v, 1)}, -1, {s(2, o, -1), s(3, v, 1)}, -1, -1);
        int b_Y9x = P.buf("Y9x", L_Y9x.total, BUF_SCRATCH);
        B.gemm("S2.ring", b_S9, L_S9, false, false, b_Wb, L_W, false, false, b_Y9x, L_Y9x, 1.0, 0);
        B.gather("rs2+=P(ab)Y9", P.b_rs2, L_S2, b_Y9x, L_Y9x, {T{{0, 2, 1, 3}, 1, {}}, T{{0, 3, 1, 2}, -1, {}}}, 1.0, 1);
        // -P(ab) sum_mf t_mj^af v_mbf^x,  v_mbf^x = sum_e <mb||ef> r(x)^e
        Layout L_Yv = make_layout("Yv", G, {s(0, o, 1), s(1, v, -1), s(2, v, 1)}, -1, {s(3, x, 1)}, -1, 1);
        int b_Yv = P.buf("Yv", L_Yv.total, BUF_SCRATCH);
        B.gemm("S2.v", b_ovvv_9b, L_ovvv_9b, false, false, b_r1x, L_S1, true, false, b_Yv, L_Yv, 1.0, 0);
        Layout L_vp = make_layout("v'", G, {s(0, o, -1), s(1, v, 1)}, -1, {s(2, x, -1), s(3, v, 1)}, -1, 1);
        int b_vp = P.buf("v'", L_vp.total, BUF_SCRATCH);
        // v'(m,f,x,b) = -Yv(m,f,b,x)
        B.gather("Yv->v'", b_vp, L_vp, b_Yv, L_Yv, {T{{0, 1, 3, 2}, -1, {}}}, 1.0, 0);
        Layout L_Cv = make_layout("Cv", G, {s(0, o, -1), s(1, v, 1)}, -1, {s(2, x, -1), s(3, v, 1)}, -1, -1);
        int b_Cv = P.buf("Cv", L_Cv.total, BUF_SCRATCH);
        B.gemm("S2.t2.v", b_Tr01, L_Tr, false, false, b_vp, L_vp, false, false, b_Cv, L_Cv, 1.0, 0);
        B.gather("rs2+=P(ab)Cv", P.b_rs2, L_S2, b_Cv, L_Cv, {T{{1, 2, 0, 3}, 1, {}}, T{{1, 3, 0, 2}, -1, {}}}, 1.0, 1);
        // -P(ab) sum_m t_m^a y_mbj^x,  y_mbj^x = sum_e Xc_mbej r(x)^e
        Layout L_Yy = make_layout("Yy", G, {s(0, o, 1), s(1, v, 1), s(2, o, -1)}, -1, {s(3, x, 1)}, -1, 1);
        int b_Yy = P.buf("Yy", L_Yy.total, BUF_SCRATCH);
        B.gemm("S2.y", b_Xc9f, L_ovvo_9f, false, false, b_r1x, L_S1, true, false, b_Yy, L_Yy, 1.0, 0);
        Layout L_Yy2 = make_layout("Yy2", G, {s(3, x, 1), s(2, o, 1), s(1, v, -1)}, -1, {s(0, o, 1)}, -1, 1);
        int b_Yy2 = P.buf("Yy2", L_Yy2.total, BUF_SCRATCH);
        B.gather("Yy->Yy2", b_Yy2, L_Yy2, b_Yy, L_Yy, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        Layout L_Yy3 = make_layout("Yy3", G, {s(0, x, 1), s(1, o, 1), s(2, v, -1)}, -1, {s(3, v, 1)}, -1, 1);
        int b_Yy3 = P.buf("Yy3", L_Yy3.total, BUF_SCRATCH);
        B.gemm("S2.y.t1", b_Yy2, L_Yy2, false, false, b_t1c, L_T1, false, false, b_Yy3, L_Yy3, 1.0, 0);
        B.gather("rs2+=-P(ab)Yy3", P.b_rs2, L_S2, b_Yy3, L_Yy3, {T{{0, 1, 3, 2}, -1, {}}, T{{0, 1, 2, 3}, 1, {}}}, 1.0, 1);
        // sigma1 = sum_e Fbar_ae r^e + sum_me Fbar_me s_xm^ae + sum_{m,e<f} Wbar_amef s_xm^ef
        B.gemm("S1.Fvv", b_r1x, L_S1, false, false, b_Fvv, L_Fae_m, true, false, P.b_rs1, L_S1, 1.0, 0);
        B.gemm("S1.Fov", b_S9, L_S9, false, false, b_Fov, L_Fme_v, false, false, P.b_rs1, L_S1v, 1.0, 1);
        Layout L_S12 = make_layout("S2(x|m,ef<)", G, {s(0, x, 1)}, -1, {s(1, o, 1), s(2, v, -1), s(3, v, -1)}, 1, -1);
        int b_S12 = P.buf("S2(x|m,ef<)", L_S12.total, BUF_SCRATCH);
        B.gather("s2->(x|m,ef<)", b_S12, L_S12, P.b_s2, L_S2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
        B.gemm("S1.Wamef", b_S12, L_S12, false, false, b_Wam, L_ovvv_14e, false, false, P.b_rs1, L_S1, 1.0, 1);
        // -sum_m (q_xm + u_xm) t_mj^ab,  q_xm = sum_{n,e<f} <mn||ef> s_xn^ef,  u_xm = sum_e Fbar_me r(x)^e
        Layout L_q = make_layout("q", G, {s(0, x, 1)}, -1, {s(1, o, 1)}, -1, 1);
        int b_q = P.buf("q", L_q.total, BUF_SCRATCH);
        B.gemm("S2.q", b_S12, L_S12, false, false, b_oovv_3b, L_oovv_3b, true, false, b_q, L_q, 1.0, 0);
        B.gemm("S2.u", b_r1x, L_S1, false, false, b_Fov, L_Fme_m, true, false, b_q, L_q, 1.0, 1);
        int b_C9 = P.buf("C9", L_S12.total, BUF_SCRATCH);
        B.gemm("S2.q.t2", b_q, L_q, false, false, b_Tm, L_Tm, false, false, b_C9, L_S12, -1.0, 0);
        // H_eff[y][x] = sigma(x)^y  (block diagonal)
        P.b_heff = P.buf("Heff", L_Heff.total, BUF_SCRATCH);
        {
            Op op;
            op.kind = OP_GATHER;
            op.name = "Heff=sigma1";
            op.dst = P.b_heff;
            op.src = P.b_rs1;
            op.alpha = 1.0;
            op.beta = 0;
            op.n = L_Heff.total;
            std::vector<uint32_t> m((size_t)L_Heff.total, MAP_ZERO);
            L_Heff.for_each([&](int64_t k, const int* p) {
                int pos[2] = {p[1], P.x_vpos[p[0]]};    // sigma(x)^y: S1 logical (x, a = y)
                int sg = 1;
                int64_t so = L_S1.find(pos, &sg);
                if (so >= 0) m[(size_t)k] = (uint32_t)so;
            });
            op.mapsA.push_back(P.map("Heff/A0", std::move(m)));
            B.out->push_back(std::move(op));
        }
        // Bloch residual: R1 = sigma1 - sum_y s_y^a Heff_yx (masked);  R2 = sigma2 + C9 - sum_y s_yj^ab Heff_yx
        B.gemm("R1.Heff", P.b_heff, L_Heff, true, false, P.b_s1, L_S1, false, false, P.b_rs1, L_S1, -1.0, 1);
        B.mul("R1*=mask", P.b_rs1, P.b_mask1, L_S1.total);
        B.gemm("R2.Heff", P.b_heff, L_Heff, true, false, b_S12, L_S12, false, false, b_C9, L_S12, -1.0, 1);
        B.gather("rs2+=C9", P.b_rs2, L_S2, b_C9, L_S12, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 1);

        // =================================================================
        // (0h,2p) sector over the active pairs x < y, at fixed T and (0h,1p)
        // amplitudes.  Omega|xy> = R_x R_y |Phi> + S_xy |Phi> (R_x the dressed
        // one-particle attachment r(x) = e_x + s_x); projected on the 2p space:
        //   sigma2 = K + sum_{e<f} Wbar_abef omega^ef + P(ab) sum_e Fbar_be s^ae
        //   omega  = A_ab[r1(x)^a r1(y)^b] + s_xy^ab
        //   K      = A_ab[sigma1(x)^a r1(y)^b + r1(x)^a sigma1(y)^b]
        //            + sum_m [g(x)_m s_ym^ab - g(y)_m s_xm^ab]
        //            + P(ab) { sum_me (Y - v)(x)_a,me s_ym^be + v(y)_a,me s_xm^be }
        //   g(x)_m = sum_e Fbar_me r1(x)^e + sum_{n,e<f} <mn||ef> s_xn^ef
        //   v(x)_a,me = sum_f Wbar_amef r1(x)^f,  Y(x)_a,me = sum_{m'e'} s_xm'^ae' <m'm||e'e>
        //   H_eff[zw, xy] = sigma2(xy)^zw;  R = sigma2 - sum_{z<w} omega(zw) H_eff[zw, xy]
        if (x->n >= 2) {
            P.has02 = true;
            P.L_S02 = make_layout("S02", G, {s(0, x, 1), s(1, x, 1)}, 0, {s(2, v, 1), s(3, v, 1)}, 0, 1);
            P.L_Heff02 = make_layout("Heff02", G, {s(0, x, 1), s(1, x, 1)}, 0, {s(2, x, 1), s(3, x, 1)}, 0, 1);
            const Layout& L_S02 = P.L_S02;
            const Layout& L_H2 = P.L_Heff02;
            P.b_s02 = P.buf("s02", L_S02.total, BUF_IN_P2);
            P.b_rs02 = P.buf("rs02", L_S02.total, BUF_OUT_RP2);
            // D_xy^ab = e_x + e_y - e_a - e_b; model pairs (a, b both active) are not amplitudes
            std::vector<char> isact(v->n, 0);
            for (int q = 0; q < x->n; ++q) isact[P.x_vpos[q]] = 1;
            P.D02.assign(L_S02.total, -1.0);   // masked entries: negative, so D + Delta never vanishes
            P.mask02.assign(L_S02.total, 0.0);
            L_S02.for_each([&](int64_t k, const int* p) {
                if (isact[p[2]] && isact[p[3]]) return;
                P.D02[k] = S.eps[x->glob[p[0]]] + S.eps[x->glob[p[1]]] - S.eps[v->glob[p[2]]] - S.eps[v->glob[p[3]]];
                P.mask02[k] = 1.0;
            });
            P.b_D02 = P.buf("D02", L_S02.total, BUF_REAL);
            P.b_mask02 = P.buf("mask02", L_S02.total, BUF_REAL);

            // ------------------------------------------ fixed part (prepare)
            B.out = &P.ops02_prep;
            B.axpby("r1=s1 (02)", b_r1x, P.b_s1, L_S1.total, 1.0, 0, false);
            B.mul("r1*=mask (02)", b_r1x, P.b_mask1, L_S1.total);
            B.axpby("r1+=e_x (02)", b_r1x, b_eid, L_S1.total, 1.0, 1, false);
            B.gather("s2->ring (02)", b_S9, L_S9, P.b_s2, L_S2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
            B.gather("s2->(x|m,ef<) (02)", b_S12, L_S12, P.b_s2, L_S2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
            // sigma1(x) (the (0h,1p) sigma vector, 1p part)
            int b_sg1 = P.buf("sigma1(02)", L_S1.total, BUF_SCRATCH);
            B.gemm("P2.sigma1.Fvv", b_r1x, L_S1, false, false, b_Fvv, L_Fae_m, true, false, b_sg1, L_S1, 1.0, 0);
            B.gemm("P2.sigma1.Fov", b_S9, L_S9, false, false, b_Fov, L_Fme_v, false, false, b_sg1, L_S1v, 1.0, 1);
            B.gemm("P2.sigma1.Wamef", b_S12, L_S12, false, false, b_Wam, L_ovvv_14e, false, false, b_sg1, L_S1, 1.0, 1);
            // g(x)_m
            int b_g = P.buf("g(02)", L_q.total, BUF_SCRATCH);
            B.gemm("P2.g.oovv", b_S12, L_S12, false, false, b_oovv_3b, L_oovv_3b, true, false, b_g, L_q, 1.0, 0);
            B.gemm("P2.g.Fov", b_r1x, L_S1, false, false, b_Fov, L_Fme_m, true, false, b_g, L_q, 1.0, 1);
            // omega_pp = A_ab[r1(x)^a r1(y)^b]
            int b_wpp = P.buf("omega_pp", L_S02.total, BUF_SCRATCH);
            B.gather("omega_pp", b_wpp, L_S02, b_r1x, L_S1, {T{{0, 2}, 1, {1, 3}}, T{{0, 3}, -1, {1, 2}}}, 1.0, 0,
                     false, b_r1x, &L_S1);
            // K: legs on one line
            int b_K = P.buf("K02", L_S02.total, BUF_SCRATCH);
            B.gather("K=sigma1 r1", b_K, L_S02, b_sg1, L_S1, {T{{0, 2}, 1, {1, 3}}, T{{0, 3}, -1, {1, 2}}}, 1.0, 0,
                     false, b_r1x, &L_S1);
            B.gather("K+=r1 sigma1", b_K, L_S02, b_r1x, L_S1, {T{{0, 2}, 1, {1, 3}}, T{{0, 3}, -1, {1, 2}}}, 1.0, 1,
                     false, b_sg1, &L_S1);
            // K += sum_m g(x)_m s_ym^ab - (x <-> y)
            Layout L_S2m = make_layout("S2(m|y,ab<)", G, {s(1, o, 1)}, -1, {s(0, x, -1), s(2, v, 1), s(3, v, 1)}, 1, 1);
            int b_S2m = P.buf("S2(m|y,ab<)", L_S2m.total, BUF_SCRATCH);
            B.gather("s2->(m|y,ab<)", b_S2m, L_S2m, P.b_s2, L_S2, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
            Layout L_Hg = make_layout("Hg02", G, {s(0, x, 1)}, -1, {s(1, x, -1), s(2, v, 1), s(3, v, 1)}, 1, 1);
            int b_Hg = P.buf("Hg02", L_Hg.total, BUF_SCRATCH);
            B.gemm("P2.g.s2", b_g, L_q, false, false, b_S2m, L_S2m, false, false, b_Hg, L_Hg, 1.0, 0);
            B.gather("K+=Hg", b_K, L_S02, b_Hg, L_Hg, {T{{0, 1, 2, 3}, 1, {}}, T{{1, 0, 2, 3}, -1, {}}}, 1.0, 1);
            // v(x)_a,me = sum_f Wbar_amef r1(x)^f
            Layout L_Wp = make_layout("Wbar(a,m,e|f)", G, {s(1, v, 1), s(0, o, 1), s(2, v, -1)}, -1, {s(3, v, 1)}, -1, 1);
            int b_Wp = P.buf("Wbar(a,m,e|f)", L_Wp.total, BUF_SCRATCH);
            B.gather("Wbar->(a,m,e|f)", b_Wp, L_Wp, b_Wam, L_ovvv_14e, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
            Layout L_vt = make_layout("v(a,m,e|x)", G, {s(1, v, 1), s(0, o, 1), s(2, v, -1)}, -1, {s(3, x, 1)}, -1, 1);
            int b_vt = P.buf("v(a,m,e|x)", L_vt.total, BUF_SCRATCH);
            B.gemm("P2.v", b_Wp, L_Wp, false, false, b_r1x, L_S1, true, false, b_vt, L_vt, 1.0, 0);
            Layout L_v3 = make_layout("v(x,a|m,e)", G, {s(0, x, -1), s(2, v, 1)}, -1, {s(1, o, -1), s(3, v, 1)}, -1, 1);
            int b_v3 = P.buf("v(x,a|m,e)", L_v3.total, BUF_SCRATCH);
            B.gather("v->(x,a|m,e)", b_v3, L_v3, b_vt, L_vt, {T{{1, 2, 3, 0}, 1, {}}}, 1.0, 0);
            // Y(x)_a,me = sum_{m'e'} s_xm'^ae' <m'm||e'e>, then U = Y - v in the same layout
            Layout L_Yr = make_layout("Y(x,a|n,f)", G, {s(0, x, -1), s(2, v, 1)}, -1, {s(1, o, 1), s(3, v, -1)}, -1, -1);
            int b_Yr = P.buf("Y(x,a|n,f)", L_Yr.total, BUF_SCRATCH);
            B.gemm("P2.Y", b_S9, L_S9, false, false, b_oovv_ph, L_oovv_ph, false, false, b_Yr, L_Yr, 1.0, 0);
            int b_U3 = P.buf("U(x,a|m,e)", L_v3.total, BUF_SCRATCH);
            B.gather("U=Y", b_U3, L_v3, b_Yr, L_Yr, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
            B.axpby("U-=v", b_U3, b_v3, L_v3.total, -1.0, 1, false);
            // C[(x,a),(y,b)] = sum_me U s_ym^be,  C'[(x,a),(y,b)] = sum_me v s_ym^be
            Layout L_C3 = make_layout("C(x,a|y,b)", G, {s(0, x, -1), s(2, v, 1)}, -1, {s(1, x, -1), s(3, v, 1)}, -1, -1);
            int b_C3 = P.buf("C(x,a|y,b)", L_C3.total, BUF_SCRATCH);
            int b_C3p = P.buf("C'(x,a|y,b)", L_C3.total, BUF_SCRATCH);
            B.gemm("P2.U.s2", b_U3, L_v3, false, false, b_S9, L_S9, true, false, b_C3, L_C3, 1.0, 0);
            B.gemm("P2.v.s2", b_v3, L_v3, false, false, b_S9, L_S9, true, false, b_C3p, L_C3, 1.0, 0);
            B.gather("K+=P(ab)C", b_K, L_S02, b_C3, L_C3, {T{{0, 1, 2, 3}, 1, {}}, T{{0, 1, 3, 2}, -1, {}}}, 1.0, 1);
            B.gather("K+=P(ab)C'", b_K, L_S02, b_C3p, L_C3, {T{{1, 0, 2, 3}, 1, {}}, T{{1, 0, 3, 2}, -1, {}}}, 1.0, 1);

            // ---------------------------------------- per iteration: sigma2 + residual
            B.out = &P.ops02;
            int b_om = P.buf("omega", L_S02.total, BUF_SCRATCH);
            B.axpby("omega=omega_pp", b_om, b_wpp, L_S02.total, 1.0, 0, false);
            B.axpby("omega+=s", b_om, P.b_s02, L_S02.total, 1.0, 1, false);
            B.axpby("sigma2=K", P.b_rs02, b_K, L_S02.total, 1.0, 0, false);
            // sum_{e<f} Wbar_abef omega^ef: bare ladder, T1 part, tau part
            B.gemm("P2-ladder", b_om, L_S02, false, false, b_vvvv, L_VVVV, true, false, P.b_rs02, L_S02, 1.0, 1);
            Layout L_Z02 = make_layout("Z02", G, {s(0, o, 1), s(1, v, 1)}, -1, {s(2, x, 1), s(3, x, 1)}, 0, 1);
            int b_Z02 = P.buf("Z02", L_Z02.total, BUF_SCRATCH);
            B.gemm("P2.Z", b_ovvv, L_OVVV, false, false, b_om, L_S02, true, false, b_Z02, L_Z02, -1.0, 0);
            Layout L_Z2b = make_layout("Z02'", G, {s(2, x, 1), s(3, x, 1), s(1, v, -1)}, 0, {s(0, o, 1)}, -1, 1);
            int b_Z2b = P.buf("Z02'", L_Z2b.total, BUF_SCRATCH);
            B.gather("Z02->Z02'", b_Z2b, L_Z2b, b_Z02, L_Z02, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
            Layout L_Y4b = make_layout("Y4(02)", G, {s(0, x, 1), s(1, x, 1), s(2, v, -1)}, 0, {s(3, v, 1)}, -1, 1);
            int b_Y4b = P.buf("Y4(02)", L_Y4b.total, BUF_SCRATCH);
            B.gemm("P2.Z.t1", b_Z2b, L_Z2b, false, false, b_t1c, L_T1, false, false, b_Y4b, L_Y4b, 1.0, 0);
            B.gather("sigma2+=-P(ab)Y4", P.b_rs02, L_S02, b_Y4b, L_Y4b,
                     {T{{0, 1, 2, 3}, -1, {}}, T{{0, 1, 3, 2}, 1, {}}}, 1.0, 1);
            Layout L_X02 = make_layout("X02", G, {s(0, o, 1), s(1, o, 1)}, 0, {s(2, x, 1), s(3, x, 1)}, 0, 1);
            int b_X02 = P.buf("X02", L_X02.total, BUF_SCRATCH);
            B.gemm("P2.X", b_oovv, L_OOVV, false, false, b_om, L_S02, true, false, b_X02, L_X02, 1.0, 0);
            B.gemm("P2.hh", b_X02, L_X02, true, false, b_tauc, L_T2, false, false, P.b_rs02, L_S02, 1.0, 1);
            // P(ab) sum_e Fbar_be s^ae
            Layout L_S7b = make_layout("S02(x,y,a|e)", G, {s(0, x, 1), s(1, x, 1), s(2, v, -1)}, 0, {s(3, v, 1)}, -1, 1);
            int b_S7b = P.buf("S02(x,y,a|e)", L_S7b.total, BUF_SCRATCH);
            B.gather("s02->(x,y,a|e)", b_S7b, L_S7b, P.b_s02, L_S02, {T{{0, 1, 2, 3}, 1, {}}}, 1.0, 0);
            int b_Y7b = P.buf("Y7(02)", L_S7b.total, BUF_SCRATCH);
            B.gemm("P2.Fvv", b_S7b, L_S7b, false, false, b_Fvv, L_Fae_m, true, false, b_Y7b, L_S7b, 1.0, 0);
            B.gather("sigma2+=P(ab)Y7", P.b_rs02, L_S02, b_Y7b, L_S7b, {T{{0, 1, 2, 3}, 1, {}}, T{{0, 1, 3, 2}, -1, {}}},
                     1.0, 1);
            // H_eff[zw, xy] = sigma2(xy)^zw
            P.b_heff02 = P.buf("Heff02", L_H2.total, BUF_SCRATCH);
            {
                Op op;
                op.kind = OP_GATHER;
                op.name = "Heff02=sigma2";
                op.dst = P.b_heff02;
                op.src = P.b_rs02;
                op.alpha = 1.0;
                op.beta = 0;
                op.n = L_H2.total;
                std::vector<uint32_t> m((size_t)L_H2.total, MAP_ZERO);
                L_H2.for_each([&](int64_t k, const int* p) {
                    int pos[4] = {p[2], p[3], P.x_vpos[p[0]], P.x_vpos[p[1]]};   // sigma2(xy)^zw
                    int sg = 1;
                    int64_t so = L_S02.find(pos, &sg);
                    if (so >= 0) m[(size_t)k] = (uint32_t)so | (sg < 0 ? MAP_NEG : 0u);
                });
                op.mapsA.push_back(P.map("Heff02/A0", std::move(m)));
                B.out->push_back(std::move(op));
            }
            // Bloch residual R = sigma2 - sum_{z<w} omega(zw) H_eff[zw, xy], model pairs masked
            B.gemm("P2.R.Heff", P.b_heff02, L_H2, true, false, b_om, L_S02, false, false, P.b_rs02, L_S02, -1.0, 1);
            B.mul("R02*=mask", P.b_rs02, P.b_mask02, L_S02.total);
        }
        B.out = &P.ops;
    }
}

}  // namespace fscc
