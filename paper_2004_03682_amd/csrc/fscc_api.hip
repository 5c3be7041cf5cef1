// fscc_api.hip -- C ABI of the library (include/fscc.h): context, device
// memory, execution of the (0h,0p) and (0h,1p) residual plans on a HIP
// stream, Jacobi + DIIS update, correlation energy and H_eff.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include <unistd.h>

#include "runtime.hpp"

namespace fscc {
namespace rt {

// Default tile shape from a cost model: padded MFMA work at a per-shape
// efficiency, against operand re-reads (A once per column tile, B once per
// row tile) at HBM speed.  fscc_autotune() replaces it by measurement.
// Shape limits of the vector-ALU forms (the MFMA tiles and the skinny form
// take any shape).
bool cfg_ok(const Op& o, int cfg, bool real) {
    if (cfg < 0 || cfg >= ZCFG_N) return false;
    if (real && (cfg == ZCFG_SKINNY || cfg == ZCFG_DOT)) return false;   // no real form of these kernels
    if (cfg == ZCFG_TALL) {
        if (o.tA) return false;
        for (auto& p : o.probs)
            if (p.K > ZTALL_MAX_K || p.N > ZTALL_MAX_KN || (long long)p.K * p.N > ZTALL_MAX_KN) return false;
    }
    if (cfg == ZCFG_RED) {
        if (o.tB) return false;
        for (auto& p : o.probs)
            if (p.M > ZRED_MAX_M || p.N > ZRED_MAX_N) return false;
    }
    if (cfg == ZCFG_DOT) {
        if (o.tA || !o.tB) return false;
        for (auto& p : o.probs)
            if (p.M > ZDOT_MAX_M) return false;
    }
    return true;
}

double cfg_cost(const Op& o, int cfg) {
    static const double eff[ZCFG_N] = {1.0, 1.4, 1.4, 1.6, 1.8, 1.8, 1.0, 1.0, 1.0, 1.3, 1.3, 1.0, 1.3, 1.3};
    if (cfg == ZCFG_TALL || cfg == ZCFG_RED || cfg == ZCFG_DOT) {
        // streaming forms: every operand element read once, exact work on the
        // vector ALUs
        double fl = 0.0, by = 0.0;
        for (auto& p : o.probs) {
            fl += 8.0 * p.M * p.N * (double)std::max(p.K, 1);
            by += 16.0 * ((double)p.M * p.K + (double)p.K * p.N + (1.0 + o.beta) * p.M * p.N);
        }
        return std::max(fl / 20e12, by / 6e12) + (cfg == ZCFG_RED ? 4e-6 : 0.0);
    }
    if (cfg == ZCFG_SKINNY) {
        // exact work on the vector ALUs (~20 TFLOP/s from LDS); A re-read once
        // per 32-column block, B once per 64-row block
        double fl = 0.0, by = 0.0;
        for (auto& p : o.probs) {
            const double tm = (p.M + ZSKINNY_BM - 1) / ZSKINNY_BM, tn = (p.N + ZSKINNY_BN - 1) / ZSKINNY_BN;
            fl += 8.0 * p.M * p.N * (double)std::max(p.K, 1);
            by += 16.0 * ((double)p.M * p.K * tn + (double)p.N * p.K * tm + 2.0 * p.M * p.N);
        }
        return std::max(fl / 20e12, by / 4e12) + 4e-6;
    }
    int bm, bn;
    zcfg_tile(cfg, &bm, &bn);
    double fl = 0.0, by = 0.0;
    for (auto& p : o.probs) {
        double tm = (p.M + bm - 1) / bm, tn = (p.N + bn - 1) / bn;
        fl += 8.0 * tm * bm * tn * bn * (double)std::max(p.K, 1);
        by += 16.0 * ((double)p.M * p.K * tn + (double)p.K * p.N * tm) + 16.0 * (double)p.M * p.N;
    }
    return std::max(fl * eff[cfg] / 60e12, by / 5e12);
}

int pick_cfg(const Op& o, bool real) {
    int best = ZCFG_64x64;
    double bc = cfg_cost(o, best);
    for (int c = 0; c < ZCFG_N; ++c) {
        if (!cfg_ok(o, c, real)) continue;
        double x = cfg_cost(o, c);
        if (x < bc * 0.95) {
            best = c;
            bc = x;
        }
    }
    return best;
}

// Workgroups of one launch are handed to the 8 XCDs round-robin (block b runs on
// XCD b % 8) and each XCD has its own L2.  Permute the logical tile sequence so
// that 8 consecutive logical tiles (which share operand panels) land on one XCD
// in consecutive dispatch slots: block 64u + 8v + x takes logical tile
// 64u + 8x + v.  A trailing partial round keeps the identity order.
std::vector<ZTile> xcd_order(const std::vector<ZTile>& logical) {
    const size_t n = logical.size(), full = n / 64 * 64;
    std::vector<ZTile> out(logical);
    for (size_t b = 0; b < full; ++b) {
        const size_t u = b / 64, v = (b / 8) % 8, x = b % 8;
        out[b] = logical[64 * u + 8 * x + v];
    }
    return out;
}

void free_gemm(GemmDev& g) {
    if (g.probs) (void)hipFree(g.probs);
    if (g.tiles) (void)hipFree(g.tiles);
    if (g.reds) (void)hipFree(g.reds);
    if (g.work) (void)hipFree(g.work);
    fscc_ctx::free_mixed(g.mx);
    g = GemmDev();
}

// The contractions that run in split precision: the particle-particle ladder
// and the two ring GEMM sets (W_mbej's T2 part and the ring itself); in the
// bf16 form also the ladder's T1 part Z_ij^am = sum_{e<f} <am||ef> tau_ij^ef
// (its split-FP32 form is slower than FP64) and the (0h,1p) sector's ladder
// over all virtual pairs (HBM-bound: 12 instead of 16 bytes per <ab||cd>).
bool mixed_eligible(const Op& o, int prec) {
    if (o.kind != OP_GEMM) return false;
    if (o.name == "Z" || o.name == "S2-ladder") return prec == FSCC_SPLIT_BF16;
    return o.name == "pp-ladder" || o.name == "W.U" || o.name == "ring";
}

long long round_up(long long x, long long m) { return (x + m - 1) / m * m; }

// Split-precision plan of one GEMM op: piece-plane descriptors of both
// operands (A rows = M; B rows = N, both with the contraction index as the
// panel depth) and the tile list of the split kernel.
MixedDev* plan_mixed(fscc_ctx* c, const Op& o, int prec, int cfg) {
    MixedDev* m = new MixedDev();
    try {
        m->prec = prec;
        m->cfg = cfg;
        const int es = prec == FSCC_SPLIT_BF16 ? 2 : 4, npl = prec == FSCC_SPLIT_BF16 ? 6 : 4;
        std::vector<SplitProb> sa, sb;
        std::vector<MProb> pr;
        long long oa = 0, ob = 0, cha = 0, chb = 0;
        for (auto& p : o.probs) {
            const int kp = (int)round_up(p.K, 32);
            const int ra = (int)round_up(std::max(p.M, 1), 64), rb = (int)round_up(std::max(p.N, 1), 64);
            sa.push_back(SplitProb{p.a_off, oa, p.M, p.K, p.lda, o.tA ? 1 : 0, ra, kp});
            sb.push_back(SplitProb{p.b_off, ob, p.N, p.K, p.ldb, o.tB ? 0 : 1, rb, kp});
            pr.push_back(MProb{oa, ob, p.c_off, p.M, p.N, kp, p.ldc, ra, rb});
            cha = std::max(cha, (long long)ra * kp / 8);
            chb = std::max(chb, (long long)rb * kp / 8);
            oa += (long long)ra * kp;
            ob += (long long)rb * kp;
        }
        int bm, bn;
        mcfg_tile(cfg, &bm, &bn);
        std::vector<ZTile> tl;
        for (size_t q = 0; q < pr.size(); ++q) {
            const int mt = (pr[q].M + bm - 1) / bm, nt = (pr[q].N + bn - 1) / bn;
            for (int mg = 0; mg < mt; mg += 8)
                for (int n = 0; n < nt; ++n)
                    for (int mm = mg; mm < std::min(mt, mg + 8); ++mm)
                        tl.push_back(ZTile{(int)q, mm * bm, n * bn, o.probs[q].sys});
        }
        std::stable_sort(tl.begin(), tl.end(), [&](const ZTile& x, const ZTile& y) { return pr[x.prob].Kp > pr[y.prob].Kp; });
        tl = xcd_order(tl);
        m->ntiles = (int)tl.size();
        auto up = [&](const void* h, size_t bytes) {
            void* d = c->dalloc(std::max<size_t>(bytes, 16));
            if (bytes) hip_check(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice), "mixed plan upload");
            return d;
        };
        m->probs = (MProb*)up(pr.data(), pr.size() * sizeof(MProb));
        m->tiles = (ZTile*)up(tl.data(), tl.size() * sizeof(ZTile));
        m->a.sp = (SplitProb*)up(sa.data(), sa.size() * sizeof(SplitProb));
        m->b.sp = (SplitProb*)up(sb.data(), sb.size() * sizeof(SplitProb));
        m->a.nsp = (int)sa.size();
        m->b.nsp = (int)sb.size();
        m->a.max_chunks = cha;
        m->b.max_chunks = chb;
        m->a.plane = round_up(std::max(oa, 1LL), 64);
        m->b.plane = round_up(std::max(ob, 1LL), 64);
        m->a.planes = c->dalloc((size_t)m->a.plane * npl * es);
        m->b.planes = c->dalloc((size_t)m->b.plane * npl * es);
        m->a.conj = o.cA;
        m->b.conj = o.cB;
        m->a.constant = c->plan.bufs[o.src].kind == BUF_CONST;
        m->b.constant = c->plan.bufs[o.src2].kind == BUF_CONST;
    } catch (...) {
        fscc_ctx::free_mixed(m);
        throw;
    }
    return m;
}

// Default split-kernel tile: the largest one that still gives the launch
// enough workgroups to cover the chip.
int pick_mcfg(const Op& o) {
    for (int cfg : {MCFG_64x64, MCFG_64x32, MCFG_32x64, MCFG_32x32}) {
        int bm, bn;
        mcfg_tile(cfg, &bm, &bn);
        long long t = 0;
        for (auto& p : o.probs) t += (long long)((p.M + bm - 1) / bm) * ((p.N + bn - 1) / bn);
        if (t >= 512) return cfg;
    }
    return MCFG_32x32;
}

// Switch the eligible GEMM ops of the (0h,0p) and (0h,1p) residuals to
// precision `prec` (planning their split form on first use); FP64 keeps the
// plans.
void apply_precision(fscc_ctx* c, int prec) {
    if (prec != FSCC_FP64)
        for (OpList* L : {&c->L00, &c->L01}) {
            if (!L->ops) continue;
            std::vector<Op>& ops = *L->ops;
            for (size_t k = 0; k < ops.size(); ++k) {
                if (!mixed_eligible(ops[k], prec)) continue;
                GemmDev& g = L->g[k];
                if (g.mx && g.mx->prec == prec) continue;
                fscc_ctx::free_mixed(g.mx);
                g.mx = plan_mixed(c, ops[k], prec, pick_mcfg(ops[k]));
            }
        }
    c->prec = prec;
}

// Algorithmic bytes of one call of an operation: every destination element
// written once (and read once when accumulating), every distinct source
// element read once, for the GEMMs each operand element read once.
// Structural zeros of a gather map read nothing, an accumulating gather
// leaves the elements whose terms are all structural zeros untouched, and
// index maps are not counted.
double op_bytes(const Plan& P, const Op& o, const std::vector<int64_t>& nnz, size_t es) {
    const double e = (double)es;
    switch (o.kind) {
        case OP_GEMM: {
            double b = 0.0;
            for (auto& q : o.probs)
                b += e * ((double)q.M * q.K + (double)q.K * q.N + (1.0 + o.beta) * (double)q.M * q.N);
            return b;
        }
        case OP_AXPBY: return e * (double)o.n * (2.0 + o.beta);
        case OP_DIAG: return e * (double)o.n * 3.0 + 8.0 * (double)o.n;
        case OP_MUL: return e * (double)o.n * 2.0 + 8.0 * (double)o.n;
        case OP_GATHER: {
            int64_t written = o.n;
            if (o.beta) {
                bool host_maps = true;
                for (int m : o.mapsA) host_maps = host_maps && (int64_t)P.maps[m].size() == o.n;
                for (int m : o.mapsB) host_maps = host_maps && (int64_t)P.maps[m].size() == o.n;
                if (host_maps) {
                    written = 0;
                    for (int64_t k = 0; k < o.n; ++k) {
                        bool any = false;
                        for (size_t t = 0; t < o.mapsA.size() && !any; ++t)
                            any = P.maps[o.mapsA[t]][k] != MAP_ZERO &&
                                  (t >= o.mapsB.size() || P.maps[o.mapsB[t]][k] != MAP_ZERO);
                        written += any;
                    }
                }
            }
            double b = e * (double)written * (1.0 + o.beta);
            // distinct source buffers: at most their size, at most the entries that read them
            std::vector<std::pair<int, int64_t>> reads;
            for (size_t t = 0; t < o.mapsA.size(); ++t) {
                const int src = o.srcT.empty() ? o.src : o.srcT[t];
                auto it = std::find_if(reads.begin(), reads.end(), [&](const auto& r) { return r.first == src; });
                if (it == reads.end()) reads.push_back({src, nnz[o.mapsA[t]]});
                else it->second += nnz[o.mapsA[t]];
            }
            for (auto& r : reads) b += e * (double)std::min<int64_t>(r.second, P.bufs[r.first].n);
            if (o.src2 >= 0) b += e * (double)P.bufs[o.src2].n;
            return b;
        }
    }
    return 0.0;
}

std::string& free_call_error() {
    static thread_local std::string msg;
    return msg;
}

void plan_gemm_host(bool real, const Op& o, int cfg, int bk, bool allow_split, bool m3, GemmHost& h) {
    h = GemmHost();
    GemmDev& g = h.g;
    g.cfg = cfg;
    g.bk = bk;
    g.m3 = m3 && !real && cfg != ZCFG_SKINNY && cfg != ZCFG_TALL && cfg != ZCFG_RED && cfg != ZCFG_DOT;
    g.role = o.name == "pp-ladder" ? 1 : (o.name == "ring" || o.name == "W.U") ? 2 : 0;
    int bm, bn;
    zcfg_tile(g.cfg, &bm, &bn);
    long long tiles0 = 0;
    int maxK = 0;
    g.maxM = 0;
    for (auto& p : o.probs) {
        tiles0 += (long long)((p.M + bm - 1) / bm) * ((p.N + bn - 1) / bn);
        maxK = std::max(maxK, p.K);
        g.maxM = std::max(g.maxM, p.M);
    }
    const long long target = 2048;
    int S = tiles0 > 0 ? (int)std::min<long long>(512, (target + tiles0 - 1) / tiles0) : 1;
    std::vector<int> Sq(o.probs.size(), 1);
    bool split = false;
    if (cfg == ZCFG_SKINNY) {
        // the skinny kernel always writes partial blocks: K chunks of >= 64
        split = true;
        for (size_t q = 0; q < o.probs.size(); ++q)
            Sq[q] = allow_split ? std::max(1, std::min(S, (o.probs[q].K + 63) / 64)) : 1;
    } else if (cfg == ZCFG_RED) {
        // the reduction form always writes partial blocks: K chunks of at most
        // ZRED_LDS / M (the chunk of A is staged in LDS) and, when splitting
        // for parallelism is allowed, of >= 128
        split = true;
        for (size_t q = 0; q < o.probs.size(); ++q) {
            const GemmProblem& p = o.probs[q];
            const int cap = ZRED_LDS / std::max(1, p.M);
            const int need = (p.K + cap - 1) / cap;
            Sq[q] = std::max(1, std::max(need, allow_split ? std::min(S, (p.K + 127) / 128) : 1));
        }
    } else if (cfg != ZCFG_TALL && cfg != ZCFG_DOT && allow_split && S > 1 && maxK >= 512)
        for (size_t q = 0; q < o.probs.size(); ++q) {
            Sq[q] = std::max(1, std::min(S, (o.probs[q].K + 255) / 256));
            split |= Sq[q] > 1;
        }
    std::vector<ZProb>& pr = h.pr;
    std::vector<int> psys;
    std::vector<ZTile> tl;
    std::vector<ZRed>& rd = h.rd;
    long long woff = 0;
    int maxMN = 0;
    for (size_t q = 0; q < o.probs.size(); ++q) {
        const GemmProblem& p = o.probs[q];
        if (!split) {
            pr.push_back(ZProb{p.a_off, p.b_off, p.c_off, p.M, p.N, p.K, p.lda, p.ldb, p.ldc});
            psys.push_back(p.sys);
        } else {
            int chunk = (p.K + Sq[q] - 1) / std::max(Sq[q], 1);
            int ns = 0;
            for (int k0 = 0; k0 < std::max(p.K, 1); k0 += std::max(chunk, 1)) {
                int len = std::max(0, std::min(chunk, p.K - k0));
                long long ao = p.a_off + (o.tA ? (long long)k0 * p.lda : k0);
                long long bo = p.b_off + (o.tB ? k0 : (long long)k0 * p.ldb);
                pr.push_back(ZProb{ao, bo, woff + (long long)ns * p.M * p.N, p.M, p.N, len, p.lda, p.ldb, p.N});
                psys.push_back(p.sys);
                ++ns;
                if (p.K == 0) break;
            }
            rd.push_back(ZRed{p.c_off, woff, p.M, p.N, p.ldc, ns, p.sys, 0});
            g.maxS = std::max(g.maxS, ns);
            woff += (long long)ns * p.M * p.N;
            if ((long long)p.M * p.N > 0x7FFFFFFFLL) throw std::length_error("split-K problem exceeds 2^31 outputs");
            maxMN = std::max(maxMN, p.M * p.N);
        }
    }
    // Logical tile order inside a problem: bands of up to 8 row tiles, the band's
    // row tiles innermost, so neighbouring tiles share one column panel of B.
    for (size_t q = 0; q < pr.size(); ++q) {
        const int mt = (pr[q].M + bm - 1) / bm, nt = (pr[q].N + bn - 1) / bn;
        for (int mg = 0; mg < mt; mg += 8)
            for (int n = 0; n < nt; ++n)
                for (int m = mg; m < std::min(mt, mg + 8); ++m) tl.push_back(ZTile{(int)q, m * bm, n * bn, psys[q]});
    }
    // longest-K tiles first (uneven symmetry blocks)
    std::stable_sort(tl.begin(), tl.end(), [&](const ZTile& a, const ZTile& b) { return pr[a.prob].K > pr[b.prob].K; });
    h.tl = xcd_order(tl);
    g.ntiles = (int)h.tl.size();
    g.split = split;
    if (split) {
        g.nred = (int)rd.size();
        g.maxMN = maxMN;
    }
    h.work_elems = split ? std::max<long long>(1, woff) : 0;
}

void plan_gemm(fscc_ctx* c, const Op& o, GemmDev& g, int cfg, int bk, bool allow_split, bool m3) {
    GemmHost h;
    plan_gemm_host(c->real, o, cfg, bk, allow_split, m3, h);
    g = h.g;
    g.probs = (ZProb*)c->dalloc(std::max<size_t>(1, h.pr.size()) * sizeof(ZProb));
    g.tiles = (ZTile*)c->dalloc(std::max<size_t>(1, h.tl.size()) * sizeof(ZTile));
    if (!h.pr.empty()) hip_check(hipMemcpy(g.probs, h.pr.data(), h.pr.size() * sizeof(ZProb), hipMemcpyHostToDevice), "probs");
    if (!h.tl.empty()) hip_check(hipMemcpy(g.tiles, h.tl.data(), h.tl.size() * sizeof(ZTile), hipMemcpyHostToDevice), "tiles");
    if (g.split) {
        g.reds = (ZRed*)c->dalloc(h.rd.size() * sizeof(ZRed));
        hip_check(hipMemcpy(g.reds, h.rd.data(), h.rd.size() * sizeof(ZRed), hipMemcpyHostToDevice), "reds");
        g.work = (double2*)c->dalloc((size_t)h.work_elems * c->esz());
    }
}


// Cost-model default of a GEMM operation before (or without) autotuning:
// pick_cfg's tile with 16-deep K slices and split-K allowed, in the
// direct-to-LDS form wherever that tile has one (the form the autotuner
// keeps for the large contractions).
void plan_gemm_default(fscc_ctx* c, const Op& o, GemmDev& g) {
    const int cfg = pick_cfg(o, c->real);
    plan_gemm(c, o, g, cfg, 16, true);
    if (zcfg_has_dl(cfg)) g.lds = LDS_DIRECT;
}

void setup_list(fscc_ctx* c, OpList& L, std::vector<Op>& ops) {
    L.ops = &ops;
    for (auto& o : ops) {
        if (o.kind == OP_GATHER && !o.gtiles.empty()) {
            GTile* d = (GTile*)c->dalloc(o.gtiles.size() * sizeof(GTile));
            hip_check(hipMemcpy(d, o.gtiles.data(), o.gtiles.size() * sizeof(GTile), hipMemcpyHostToDevice), "tiles");
            o.d_gtiles = d;
        }
        if (o.kind == OP_GATHER && !o.rtiles.empty() && !c->real) {
            GTile* d = (GTile*)c->dalloc(o.rtiles.size() * sizeof(GTile));
            hip_check(hipMemcpy(d, o.rtiles.data(), o.rtiles.size() * sizeof(GTile), hipMemcpyHostToDevice), "rtiles");
            o.d_rtiles = d;
            RTerm* q = (RTerm*)c->dalloc(o.rterms.size() * sizeof(RTerm));
            hip_check(hipMemcpy(q, o.rterms.data(), o.rterms.size() * sizeof(RTerm), hipMemcpyHostToDevice), "rterms");
            o.d_rterms = q;
            RUnit* un = (RUnit*)c->dalloc(o.runits.size() * sizeof(RUnit));
            hip_check(hipMemcpy(un, o.runits.data(), o.runits.size() * sizeof(RUnit), hipMemcpyHostToDevice), "runits");
            o.d_runits = un;
        }
    }
    L.g.assign(ops.size(), GemmDev());
    L.ms.assign(ops.size(), 0.0);
    L.calls.assign(ops.size(), 0);
    for (size_t k = 0; k < ops.size(); ++k)
        if (ops[k].kind == OP_GEMM) plan_gemm_default(c, ops[k], L.g[k]);
}

void setup_diis(fscc_ctx* c, Diis& d, int64_t n1, int64_t n2, int bD1, int bD2) {
    d.n1 = n1;
    d.n2 = n2;
    d.b_D1 = bD1;
    d.b_D2 = bD2;
    int64_t n = std::max<int64_t>(1, n1 + n2);
    d.ht = (double2*)c->dalloc((size_t)kMaxDiis * n * c->esz());   // doubles in a real context
    d.he = (double2*)c->dalloc((size_t)kMaxDiis * n * c->esz());
    d.dB = (double*)c->dalloc(kMaxDiis * kMaxDiis * sizeof(double));
}

void bind_io(fscc_ctx* c, const fscc_c128* t1, const fscc_c128* t2, fscc_c128* r1, fscc_c128* r2) {
    Plan& P = c->plan;
    c->dbuf[P.b_t1] = (void*)t1;
    c->dbuf[P.b_t2] = (void*)t2;
    c->dbuf[P.b_r1] = (void*)r1;
    c->dbuf[P.b_r2] = (void*)r2;
}

void bind_io01(fscc_ctx* c, const fscc_c128* s1, const fscc_c128* s2, fscc_c128* r1, fscc_c128* r2) {
    Plan& P = c->plan;
    c->dbuf[P.b_s1] = (void*)s1;
    c->dbuf[P.b_s2] = (void*)s2;
    c->dbuf[P.b_rs1] = (void*)r1;
    c->dbuf[P.b_rs2] = (void*)r2;
}

void bind_io02(fscc_ctx* c, const fscc_c128* s, fscc_c128* r) {
    Plan& P = c->plan;
    c->dbuf[P.b_s02] = (void*)s;
    c->dbuf[P.b_rs02] = (void*)r;
}

bool all_integrals(const fscc_ctx* c) {
    for (int k = 0; k < IC_N; ++k)
        if (!c->have_cls[k]) return false;
    return true;
}

// Device buffers, uploads of the host constants and per-iteration maps, GEMM
// plans of the op lists, DIIS state and reduction scratch of a context whose
// plan is built (setup maps stay on the host until their class is imported).
void ctx_allocate(fscc_ctx* c, bool diis) {
    Plan& P = c->plan;
    // buffers
    c->dbuf.assign(P.bufs.size(), nullptr);
    for (size_t k = 0; k < P.bufs.size(); ++k) {
        const BufDesc& b = P.bufs[k];
        if (caller_buffer(b.kind)) continue;
        size_t bytes = (size_t)b.n * (b.kind == BUF_REAL ? sizeof(double) : c->esz());
        c->dbuf[k] = c->dalloc(bytes);
    }
    auto up_real = [&](int b, const std::vector<double>& v) {
        if (b >= 0 && !v.empty())
            hip_check(hipMemcpy(c->dbuf[b], v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
    };
    up_real(P.b_D1, P.D1);
    up_real(P.b_D2, P.D2);
    up_real(P.b_D1x, P.D1x);
    up_real(P.b_D2x, P.D2x);
    up_real(P.b_mask1, P.mask1);
    up_real(P.b_D02, P.D02);
    up_real(P.b_mask02, P.mask02);
    for (auto& hc : P.const_host) {
        if (hc.data.empty()) continue;
        if (c->real) {   // these constants are real (unit entries, orbital energies)
            std::vector<double> re(hc.data.size());
            for (size_t k = 0; k < re.size(); ++k) re[k] = hc.data[k].real();
            hip_check(hipMemcpy(c->dbuf[hc.buf], re.data(), re.size() * sizeof(double), hipMemcpyHostToDevice),
                      "const upload");
        } else {
            hip_check(hipMemcpy(c->dbuf[hc.buf], hc.data.data(), hc.data.size() * sizeof(double2),
                                hipMemcpyHostToDevice), "const upload");
        }
    }
    // maps of the per-iteration gathers (setup maps are uploaded at set_integrals)
    c->dmap.assign(P.maps.size(), nullptr);
    std::vector<char> is_setup(P.maps.size(), 0);
    for (auto& sg : P.setup) is_setup[sg.map] = 1;
    std::vector<int64_t> nnz(P.maps.size(), 0);
    for (size_t k = 0; k < P.maps.size(); ++k)
        if (!is_setup[k])
            for (uint32_t e : P.maps[k]) nnz[k] += e != MAP_ZERO;
    for (auto* L : {&P.ops, &P.ops01_prep, &P.ops01, &P.ops02_prep, &P.ops02})
        for (auto& o : *L) o.bytes = op_bytes(P, o, nnz, c->esz());
    for (size_t k = 0; k < P.maps.size(); ++k) {
        if (is_setup[k]) continue;
        c->dmap[k] = (uint32_t*)c->dalloc(P.maps[k].size() * sizeof(uint32_t));
        hip_check(hipMemcpy(c->dmap[k], P.maps[k].data(), P.maps[k].size() * sizeof(uint32_t), hipMemcpyHostToDevice),
                  "map upload");
        std::vector<uint32_t>().swap(P.maps[k]);
    }
    setup_list(c, c->L00, P.ops);
    setup_list(c, c->L01p, P.ops01_prep);
    setup_list(c, c->L01, P.ops01);
    setup_list(c, c->L02p, P.ops02_prep);
    setup_list(c, c->L02, P.ops02);
    c->L01.base = (int)P.ops.size();
    c->L02.base = (int)(P.ops.size() + P.ops01.size());
    if (diis) setup_diis(c, c->diis[0], c->n1(), c->n2(), P.b_D1, P.b_D2);
    if (P.has01) {
        setup_diis(c, c->diis[1], P.L_S1.total, P.L_S2.total, P.b_D1x, P.b_D2x);
        int64_t ntmp = std::max<int64_t>(P.L_S1.total + P.L_S2.total, P.has02 ? P.L_S02.total : 0);
        c->rs_tmp = (double2*)c->dalloc((size_t)std::max<int64_t>(1, ntmp) * sizeof(double2));
    }
    if (P.has02) setup_diis(c, c->diis[2], 0, P.L_S02.total, -1, P.b_D02);
    c->part = (double*)c->dalloc(1024 * kDiisMax * sizeof(double));
    c->part_max = (double*)c->dalloc(2048 * sizeof(double));
    c->coef = (double*)c->dalloc((kMaxDiis + 1) * sizeof(double));
    c->scal = (double*)c->dalloc(4 * sizeof(double));
    c->epart = (double*)c->dalloc(2048 * sizeof(double));
    c->eout = (double*)c->dalloc(4 * sizeof(double));
    hip_check(hipHostMalloc((void**)&c->hscal, 8 * sizeof(double), hipHostMallocDefault), "hipHostMalloc");
}

}  // namespace rt
}  // namespace fscc


// Chunk lists of the GEMMs that read buffer b as a transposed B operand (rows
// of K contiguous elements): problems are cut along N so that every piece's
// rows span at most `half` elements, and consecutive pieces are packed into
// chunks whose rows lie in one window of `half` elements.
static std::vector<std::vector<StreamChunk>> stream_plan(fscc_ctx* c, OpList& L, int b, long long half) {
    std::vector<std::vector<StreamChunk>> out(L.ops->size());
    for (size_t k = 0; k < L.ops->size(); ++k) {
        const Op& o = (*L.ops)[k];
        if (o.kind != OP_GEMM || o.src2 != b) continue;
        std::vector<GemmProblem> pieces;
        for (const GemmProblem& p : o.probs) {
            if (p.M <= 0 || p.N <= 0) continue;
            if (p.K <= 0) {
                GemmProblem q = p;
                pieces.push_back(q);
                continue;
            }
            if ((long long)p.ldb > half) throw std::invalid_argument("staging buffer smaller than one operand row");
            const int rows = (int)std::max<long long>(1, half / p.ldb);
            for (int n0 = 0; n0 < p.N; n0 += rows) {
                GemmProblem q = p;
                q.N = std::min(rows, p.N - n0);
                q.b_off = p.b_off + (int64_t)n0 * p.ldb;
                q.c_off = p.c_off + n0;
                pieces.push_back(q);
            }
        }
        std::stable_sort(pieces.begin(), pieces.end(),
                         [](const GemmProblem& a, const GemmProblem& b2) { return a.b_off < b2.b_off; });
        const GemmDev& g0 = L.g[k];
        std::vector<std::vector<GemmProblem>> groups;
        std::vector<std::pair<long long, long long>> span;
        for (const GemmProblem& q : pieces) {
            const long long lo = q.b_off, hi = q.K > 0 ? q.b_off + (long long)(q.N - 1) * q.ldb + q.K : q.b_off;
            if (groups.empty() || hi - span.back().first > half) {
                groups.push_back({});
                span.push_back({lo, hi});
            }
            groups.back().push_back(q);
            span.back().second = std::max(span.back().second, hi);
        }
        for (size_t j = 0; j < groups.size(); ++j) {
            Op sub = o;
            sub.probs = groups[j];
            StreamChunk ch;
            ch.lo = span[j].first;
            ch.hi = span[j].second;
            plan_gemm(c, sub, ch.g, g0.cfg, g0.bk, true, g0.m3);
            hip_check(hipEventCreateWithFlags(&ch.copied, hipEventDisableTiming), "event");
            out[k].push_back(ch);
        }
    }
    return out;
}

extern "C" {

const char* fscc_last_error(const fscc_ctx* ctx) {
    if (ctx) return ctx->err.c_str();
    const std::string& e = free_call_error();
    return e.empty() ? "null context" : e.c_str();
}

fscc_status fscc_create(const fscc_system* sys, fscc_precision prec, void* hip_stream, fscc_ctx** out) {
    if (!sys || !out) return FSCC_EINVAL;
    *out = nullptr;
    if (prec != FSCC_FP64 && prec != FSCC_SPLIT_FP32 && prec != FSCC_SPLIT_BF16 && prec != FSCC_REAL_FP64)
        return FSCC_EINVAL;
    if (sys->nocc < 0 || sys->nvirt < 0 || sys->nirrep < 1 || !sys->irrep || !sys->eps) return FSCC_EINVAL;
    if (sys->nact < 0 || (sys->nact > 0 && !sys->active)) return FSCC_EINVAL;
    fscc_ctx* c = new (std::nothrow) fscc_ctx();
    if (!c) return FSCC_ENOMEM;
    fscc_status s = guarded(c, [&]() -> fscc_status {
        hip_check(hipGetDevice(&c->device), "hipGetDevice");
        c->st = (hipStream_t)hip_stream;
        System S;
        S.nocc = sys->nocc;
        S.nvirt = sys->nvirt;
        S.G = sys->nirrep;
        int n = sys->nocc + sys->nvirt;
        S.irrep.assign(sys->irrep, sys->irrep + n);
        S.eps.assign(sys->eps, sys->eps + n);
        if (sys->nact > 0) S.active.assign(sys->active, sys->active + sys->nact);
        for (int p = 0; p < n; ++p) {
            if (S.irrep[p] < 0 || S.irrep[p] >= S.G) throw std::invalid_argument("irrep label out of range");
            if (!std::isfinite(S.eps[p])) throw std::invalid_argument("non-finite orbital energy");
        }
        build_plan_ccsd(S, c->plan);
        c->real = prec == FSCC_REAL_FP64;
        ctx_allocate(c, true);
        apply_precision(c, c->real ? FSCC_FP64 : prec);
        return FSCC_OK;
    });
    if (s != FSCC_OK) {
        delete c;
        return s;
    }
    *out = c;
    return FSCC_OK;
}

void fscc_destroy(fscc_ctx* ctx) {
    if (!ctx) return;
    if (ctx->st) (void)hipStreamSynchronize(ctx->st);
    else (void)hipDeviceSynchronize();
    delete ctx;
}

fscc_status fscc_layout(const fscc_ctx* ctx, fscc_sector sector, size_t* n1, size_t* n2) {
    if (!ctx || !n1 || !n2) return FSCC_EINVAL;
    if (sector == FSCC_S00) {
        *n1 = (size_t)ctx->n1();
        *n2 = (size_t)ctx->n2();
        return FSCC_OK;
    }
    if (sector == FSCC_S01 && ctx->plan.has01) {
        *n1 = (size_t)ctx->plan.L_S1.total;
        *n2 = (size_t)ctx->plan.L_S2.total;
        return FSCC_OK;
    }
    if (sector == FSCC_S02 && ctx->plan.has02) {
        *n1 = 0;
        *n2 = (size_t)ctx->plan.L_S02.total;
        return FSCC_OK;
    }
    return FSCC_EINVAL;
}

namespace {

uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Input checks of one boundary class buffer before it is packed: every value
// finite (a full scan), and at `nsample` sampled elements the symmetries that
// relate two elements of the same class -- antisymmetry <pq||rs> = -<qp||rs>
// and <pq||rs> = -<pq||sr> where both indices of a pair lie in one space, and
// Hermiticity <pq||rs> = conj <rs||pq> where (pq) and (rs) span the same
// spaces (plain symmetry in a real context).  Returns FSCC_OK, FSCC_EINVAL
// (non-finite values) or FSCC_ESYMM with a message naming the element.
fscc_status check_class(fscc_ctx* ctx, int cls, const void* dev, int64_t n) {
    const int64_t ndbl = ctx->real ? n : 2 * n;
    unsigned long long* cnt = (unsigned long long*)ctx->dalloc(sizeof(unsigned long long));
    unsigned long long bad = 0;
    hipError_t e = launch_count_nonfinite((const double*)dev, ndbl, cnt, ctx->st);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, cnt, sizeof(bad), hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    (void)hipFree(cnt);
    hip_check(e, "non-finite scan");
    static const char* names[IC_N] = {"OOOO", "OOOV", "OOVV", "OVOV", "OVVV", "VVVV"};
    if (bad) return fail(ctx, FSCC_EINVAL, std::to_string(bad) + " non-finite values in integral class " + names[cls]);
    const FullBlocks& F = ctx->plan.full[cls];
    const bool swap12 = F.sp[0] == F.sp[1], swap34 = F.sp[2] == F.sp[3];
    const bool herm = F.sp[0] == F.sp[2] && F.sp[1] == F.sp[3];
    if (ctx->validate_n <= 0 || n == 0 || !(swap12 || swap34 || herm)) return FSCC_OK;
    for (int k = 0; k < 4; ++k)
        if (F.sp[k]->n == 0) return FSCC_OK;
    // sampled elements: (offset, partner offset, kind) with kind 0: partner = -x, 1: partner = conj(x)
    struct Pick {
        int64_t self, other;
        int kind;
        int pos[4];
    };
    std::vector<Pick> picks;
    uint64_t rng = 0x5EEDull + (uint64_t)cls;
    const int G = F.G;
    for (int tries = 0; (int)picks.size() < ctx->validate_n && tries < 8 * ctx->validate_n; ++tries) {
        int pos[4];
        for (int k = 0; k < 3; ++k) pos[k] = (int)(splitmix64(rng) % (uint64_t)F.sp[k]->n);
        const int g3 = modG(F.sp[0]->irr[pos[0]] + F.sp[1]->irr[pos[1]] - F.sp[2]->irr[pos[2]], G);
        const int c3 = F.sp[3]->cnt[g3];
        if (c3 == 0) continue;
        pos[3] = F.sp[3]->off[g3] + (int)(splitmix64(rng) % (uint64_t)c3);
        int sg;
        const int64_t self = F.find(pos, &sg);
        if (self < 0) continue;
        auto partner = [&](int a, int b, int c, int d, int kind) {
            const int q[4] = {pos[a], pos[b], pos[c], pos[d]};
            int s2;
            const int64_t o = F.find(q, &s2);
            if (o >= 0) picks.push_back(Pick{self, o, kind, {pos[0], pos[1], pos[2], pos[3]}});
        };
        if (swap12) partner(1, 0, 2, 3, 0);
        if (swap34) partner(0, 1, 3, 2, 0);
        if (herm) partner(2, 3, 0, 1, 1);
    }
    if (picks.empty()) return FSCC_OK;
    std::vector<int64_t> idx;
    for (auto& p : picks) {
        idx.push_back(p.self);
        idx.push_back(p.other);
    }
    const size_t es = ctx->esz();
    int64_t* didx = (int64_t*)ctx->dalloc(idx.size() * sizeof(int64_t));
    void* dval = ctx->dalloc(idx.size() * es);
    std::vector<double2> val(idx.size());
    e = hipMemcpyAsync(didx, idx.data(), idx.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->st);
    if (e == hipSuccess && fscc_ws_gather(dev, es, didx, idx.size(), dval, ctx->st) != FSCC_OK) e = hipErrorLaunchFailure;
    if (ctx->real) {
        std::vector<double> rv(idx.size());
        if (e == hipSuccess) e = hipMemcpyAsync(rv.data(), dval, idx.size() * es, hipMemcpyDeviceToHost, ctx->st);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
        for (size_t k = 0; k < rv.size(); ++k) val[k] = make_double2(rv[k], 0.0);
    } else {
        if (e == hipSuccess) e = hipMemcpyAsync(val.data(), dval, idx.size() * es, hipMemcpyDeviceToHost, ctx->st);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    }
    (void)hipFree(didx);
    (void)hipFree(dval);
    hip_check(e, "symmetry sample");
    double scale = 0.0;
    for (auto& v : val) scale = std::max(scale, std::hypot(v.x, v.y));
    const double tol = 1e-10 * scale;
    for (size_t k = 0; k < picks.size(); ++k) {
        const double2 x = val[2 * k], y = val[2 * k + 1];
        const double dev_ = picks[k].kind == 0 ? std::hypot(x.x + y.x, x.y + y.y) : std::hypot(x.x - y.x, x.y + y.y);
        if (dev_ > tol) {
            const Pick& p = picks[k];
            std::string at = "<" + std::to_string(F.sp[0]->glob[p.pos[0]]) + " " + std::to_string(F.sp[1]->glob[p.pos[1]]) +
                             "||" + std::to_string(F.sp[2]->glob[p.pos[2]]) + " " +
                             std::to_string(F.sp[3]->glob[p.pos[3]]) + ">";
            return fail(ctx, FSCC_ESYMM,
                        std::string("integral class ") + names[cls] + ": " + at +
                            (p.kind == 0 ? " violates antisymmetry" : " violates Hermiticity") + " by " +
                            std::to_string(dev_) + " (tolerance " + std::to_string(tol) + ")");
        }
    }
    return FSCC_OK;
}

}  // namespace

fscc_status fscc_set_integrals(fscc_ctx* ctx, fscc_iclass cls, const fscc_c128* dev_blocks, size_t n) {
    if (!ctx) return FSCC_EINVAL;
    if ((int)cls < 0 || (int)cls >= IC_N) return fail(ctx, FSCC_EINVAL, "bad integral class");
    Plan& P = ctx->plan;
    if ((int64_t)n != P.full[cls].total)
        return fail(ctx, FSCC_EINVAL, "integral class size " + std::to_string(n) + " != expected " +
                                          std::to_string(P.full[cls].total));
    if (n > 0 && !dev_blocks) return fail(ctx, FSCC_EINVAL, "null integral buffer");
    if (ctx->have_cls[cls]) return fail(ctx, FSCC_ESTATE, "integral class already set");
    return guarded(ctx, [&]() -> fscc_status {
        const fscc_status chk = check_class(ctx, (int)cls, dev_blocks, (int64_t)n);
        if (chk != FSCC_OK) return chk;
        for (auto& sg : P.setup) {
            if (sg.cls != (int)cls) continue;
            std::vector<uint32_t>& m = P.maps[sg.map];
            int64_t cnt = P.bufs[sg.dst].n;
            if (cnt > 0) {
                if ((int64_t)m.size() != cnt) throw std::logic_error("setup map already consumed: " + sg.name);
                uint32_t* dm = (uint32_t*)ctx->dalloc(m.size() * sizeof(uint32_t));
                hip_check(hipMemcpyAsync(dm, m.data(), m.size() * sizeof(uint32_t), hipMemcpyHostToDevice, ctx->st),
                          "pack map upload");
                GatherMaps gm{};
                gm.a[0] = dm;
                if (ctx->real)
                    hip_check(launch_dgather(ctx->D(sg.dst), (const double*)dev_blocks, nullptr, gm, 1, cnt, 1.0, 0,
                                             ctx->st),
                              "integral pack");
                else
                    hip_check(launch_gather(ctx->B(sg.dst), (const double2*)dev_blocks, nullptr, gm, 1, cnt, 1.0, 0.0,
                                            0, sg.conj ? 1 : 0, ctx->st),
                              "integral pack");
                hip_check(hipStreamSynchronize(ctx->st), "pack sync");
                (void)hipFree(dm);
            }
            std::vector<uint32_t>().swap(m);
        }
        ctx->have_cls[cls] = true;
        return FSCC_OK;
    });
}

fscc_status fscc_set_validation(fscc_ctx* ctx, int nsample) {
    if (!ctx) return FSCC_EINVAL;
    if (nsample < 0 || nsample > (1 << 20)) return fail(ctx, FSCC_EINVAL, "validation sample count out of range");
    ctx->validate_n = nsample;
    return FSCC_OK;
}

fscc_status fscc_set_streams(fscc_ctx* ctx, int n) {
    if (!ctx) return FSCC_EINVAL;
    if (n != 1 && n != 2) return fail(ctx, FSCC_EINVAL, "stream count must be 1 or 2");
    return guarded(ctx, [&]() -> fscc_status {
        hip_check(hipStreamSynchronize(ctx->st), "sync");
        ctx->streams = n;
        return FSCC_OK;
    });
}

fscc_status fscc_build_residual(fscc_ctx* ctx, fscc_sector sector, const fscc_c128* t1, const fscc_c128* t2,
                                fscc_c128* r1, fscc_c128* r2) {
    if (!ctx) return FSCC_EINVAL;
    if (!all_integrals(ctx)) return fail(ctx, FSCC_ESTATE, "integrals not set");
    int64_t n1, n2;
    if (sector == FSCC_S00) {
        n1 = ctx->n1();
        n2 = ctx->n2();
    } else if (sector == FSCC_S01 && ctx->plan.has01) {
        if (!ctx->ready01) return fail(ctx, FSCC_ESTATE, "(0h,1p) sector not prepared (fscc_prepare_sector)");
        n1 = ctx->plan.L_S1.total;
        n2 = ctx->plan.L_S2.total;
    } else if (sector == FSCC_S02 && ctx->plan.has02) {
        if (!ctx->ready02) return fail(ctx, FSCC_ESTATE, "(0h,2p) sector not prepared (fscc_prepare_sector)");
        n1 = 0;
        n2 = ctx->plan.L_S02.total;
    } else {
        return fail(ctx, FSCC_EINVAL, "sector not available for this system");
    }
    if ((n1 && (!t1 || !r1)) || (n2 && (!t2 || !r2))) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
    if ((n1 && (const void*)r1 == (const void*)t1) || (n2 && (const void*)r2 == (const void*)t2))
        return fail(ctx, FSCC_EINVAL, "residual aliases amplitudes");
    return guarded(ctx, [&]() -> fscc_status {
        if (sector == FSCC_S00) {
            bind_io(ctx, t1, t2, r1, r2);
            ctx->run_list(ctx->L00, ctx->prof);
            ctx->resid00 = true;
        } else if (sector == FSCC_S01) {
            bind_io01(ctx, t1, t2, r1, r2);
            ctx->run_list(ctx->L01, ctx->prof);
        } else {
            bind_io02(ctx, t2, r2);
            ctx->run_list(ctx->L02, ctx->prof);
        }
        return FSCC_OK;
    });
}

fscc_status fscc_prepare_sector(fscc_ctx* ctx, fscc_sector sector, const fscc_c128* t1, const fscc_c128* t2) {
    if (!ctx) return FSCC_EINVAL;
    if (sector == FSCC_S02) {
        Plan& P = ctx->plan;
        if (!P.has02) return fail(ctx, FSCC_EINVAL, "no (0h,2p) sector for this system (needs two active spinors)");
        if (!ctx->ready01) return fail(ctx, FSCC_ESTATE, "(0h,1p) sector not prepared (fscc_prepare_sector)");
        if ((P.L_S1.total && !t1) || (P.L_S2.total && !t2)) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
        return guarded(ctx, [&]() -> fscc_status {
            bind_io01(ctx, t1, t2, nullptr, nullptr);
            ctx->run_list(ctx->L02p, false);
            hip_check(hipStreamSynchronize(ctx->st), "prepare sync");
            ctx->ready02 = true;
            ctx->diis[2].order.clear();
            ctx->diis[2].watch.restart();
            return FSCC_OK;
        });
    }
    if (sector != FSCC_S01 || !ctx->plan.has01) return fail(ctx, FSCC_EINVAL, "no (0h,1p) sector for this system");
    if (!all_integrals(ctx)) return fail(ctx, FSCC_ESTATE, "integrals not set");
    if ((ctx->n1() && !t1) || (ctx->n2() && !t2)) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
    return guarded(ctx, [&]() -> fscc_status {
        bind_io(ctx, t1, t2, nullptr, nullptr);
        ctx->run_list(ctx->L01p, false);
        hip_check(hipStreamSynchronize(ctx->st), "prepare sync");
        ctx->ready01 = true;
        ctx->ready02 = false;   // the (0h,2p) fixed part depends on T through the (0h,1p) Hbar
        ctx->diis[1].order.clear();
        ctx->diis[1].watch.restart();
        return FSCC_OK;
    });
}

// Copy n elements of device buffer b to the host as complex values (a real
// context's buffers hold doubles: imaginary parts 0).  Synchronises.
static std::vector<double2> read_elements(fscc_ctx* ctx, int b, int64_t n) {
    std::vector<double2> h((size_t)n);
    if (n == 0) return h;
    if (ctx->real) {
        std::vector<double> d((size_t)n);
        hip_check(hipMemcpyAsync(d.data(), ctx->dbuf[b], d.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->st),
                  "d2h");
        hip_check(hipStreamSynchronize(ctx->st), "d2h sync");
        for (size_t k = 0; k < d.size(); ++k) h[k] = make_double2(d[k], 0.0);
    } else {
        hip_check(hipMemcpyAsync(h.data(), ctx->dbuf[b], h.size() * sizeof(double2), hipMemcpyDeviceToHost, ctx->st),
                  "d2h");
        hip_check(hipStreamSynchronize(ctx->st), "d2h sync");
    }
    return h;
}

fscc_status fscc_heff(fscc_ctx* ctx, const fscc_c128* s1, const fscc_c128* s2, fscc_c128* heff_host) {
    if (!ctx || !heff_host) return FSCC_EINVAL;
    Plan& P = ctx->plan;
    if (!P.has01) return fail(ctx, FSCC_EINVAL, "no (0h,1p) sector for this system");
    if (!ctx->ready01) return fail(ctx, FSCC_ESTATE, "(0h,1p) sector not prepared (fscc_prepare_sector)");
    if ((P.L_S1.total && !s1) || (P.L_S2.total && !s2)) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
    return guarded(ctx, [&]() -> fscc_status {
        // residual scratch: complex elements, or doubles at the same offsets in a real context
        fscc_c128* rs1 = (fscc_c128*)ctx->rs_tmp;
        fscc_c128* rs2 = ctx->real ? (fscc_c128*)((double*)ctx->rs_tmp + P.L_S1.total)
                                   : (fscc_c128*)(ctx->rs_tmp + P.L_S1.total);
        bind_io01(ctx, s1, s2, rs1, rs2);
        ctx->run_list(ctx->L01, false);
        std::vector<double2> h = read_elements(ctx, P.b_heff, P.L_Heff.total);
        const int nact = P.X.n;
        for (int k = 0; k < nact * nact; ++k) heff_host[k] = fscc_c128{0.0, 0.0};
        // block-diagonal [g][y_g][x_g] in irrep-sorted active order -> dense [y][x] in the caller's order
        int64_t off = 0;
        for (int g = 0; g < P.G; ++g) {
            int ng = P.X.cnt[g], o0 = P.X.off[g];
            for (int a = 0; a < ng; ++a)
                for (int b = 0; b < ng; ++b) {
                    double2 v = h[(size_t)(off + (int64_t)a * ng + b)];
                    heff_host[P.x_order[o0 + a] * nact + P.x_order[o0 + b]] = fscc_c128{v.x, v.y};
                }
            off += (int64_t)ng * ng;
        }
        return FSCC_OK;
    });
}

fscc_status fscc_heff2(fscc_ctx* ctx, const fscc_c128* s, fscc_c128* heff_host) {
    if (!ctx || !heff_host) return FSCC_EINVAL;
    Plan& P = ctx->plan;
    if (!P.has02) return fail(ctx, FSCC_EINVAL, "no (0h,2p) sector for this system");
    if (!ctx->ready02) return fail(ctx, FSCC_ESTATE, "(0h,2p) sector not prepared (fscc_prepare_sector)");
    if (P.L_S02.total && !s) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
    return guarded(ctx, [&]() -> fscc_status {
        bind_io02(ctx, s, (fscc_c128*)ctx->rs_tmp);
        ctx->run_list(ctx->L02, false);
        std::vector<double2> h = read_elements(ctx, P.b_heff02, P.L_Heff02.total);
        // [G][zw<][xy<] over irrep-sorted active pairs -> dense [pair(zw)][pair(xy)] over the pairs
        // i < j of the caller's active list (row-major upper triangle); a pair whose irrep-sorted
        // order is the reverse of the caller's order contributes with a minus sign
        const int nact = P.X.n, np = nact * (nact - 1) / 2;
        for (int k = 0; k < np * np; ++k) heff_host[k] = fscc_c128{0.0, 0.0};
        auto pidx = [&](int p, int q, int* sg) {
            int i = P.x_order[p], j = P.x_order[q];
            *sg = 1;
            if (i > j) {
                std::swap(i, j);
                *sg = -1;
            }
            return i * (2 * nact - i - 1) / 2 + (j - i - 1);
        };
        P.L_Heff02.for_each([&](int64_t k, const int* p) {
            int s1, s2;
            int r = pidx(p[0], p[1], &s1), c = pidx(p[2], p[3], &s2);
            double2 v = h[(size_t)k];
            heff_host[r * np + c] = fscc_c128{s1 * s2 * v.x, s1 * s2 * v.y};
        });
        return FSCC_OK;
    });
}

// Dressed (0h,0p) Jacobi denominators: the part of the T2 residual that is
// diagonal in the amplitude is -(f_i + f_j - f_a - f_b) t_ij^ab with
// f_p = eps_p + F'_pp (F'_be, F'_mj of the last residual evaluation: the
// one-body intermediates that multiply t2), and likewise f_i - f_a for T1;
// dividing the residual by these instead of the bare orbital-energy
// differences leaves the solution (R = 0) unchanged.  Capped at -floor.
static fscc_status precondition00(fscc_ctx* ctx, int mode, double floor) {
    Plan& P = ctx->plan;
    Diis& D = ctx->diis[FSCC_S00];
    if (mode == 0) {
        D.b_D1 = P.b_D1;
        D.b_D2 = P.b_D2;
    } else {
        std::vector<double2> fbe = read_elements(ctx, P.b_Fbe, P.bufs[P.b_Fbe].n);
        std::vector<double2> fmj = read_elements(ctx, P.b_Fmj, P.bufs[P.b_Fmj].n);
        const size_t no = P.eps_o.size(), nv = P.eps_v.size();
        if (no > 65535 || nv > 65535) throw std::invalid_argument("dressed denominators support up to 65535 spinors per space");
        std::vector<double> f(no + nv);
        for (size_t i = 0; i < no; ++i)
            f[i] = P.eps_o[i] + (P.fmj_diag[i] >= 0 ? fmj[(size_t)P.fmj_diag[i]].x : 0.0);
        for (size_t a = 0; a < nv; ++a)
            f[no + a] = P.eps_v[a] + (P.fbe_diag[a] >= 0 ? fbe[(size_t)P.fbe_diag[a]].x : 0.0);
        const int64_t n1 = P.L_T1.total, n2 = P.L_T2.total;
        if (ctx->b_pre1 < 0) {
            // first use: the orbital positions of every amplitude, kept on the device
            std::vector<uint16_t> i1((size_t)n1 * 2), i2((size_t)n2 * 4);
            P.L_T1.for_each([&](int64_t k, const int* x) {
                i1[2 * k] = (uint16_t)x[0];
                i1[2 * k + 1] = (uint16_t)x[1];
            });
            P.L_T2.for_each_par([&](int64_t k, const int* x) {
                for (int q = 0; q < 4; ++q) i2[4 * k + q] = (uint16_t)x[q];
            });
            ctx->d_idx1 = (uint16_t*)ctx->dalloc(std::max<size_t>(i1.size(), 1) * sizeof(uint16_t));
            ctx->d_idx2 = (uint16_t*)ctx->dalloc(std::max<size_t>(i2.size(), 1) * sizeof(uint16_t));
            ctx->d_fov = (double*)ctx->dalloc(std::max<size_t>(f.size(), 1) * sizeof(double));
            if (!i1.empty())
                hip_check(hipMemcpy(ctx->d_idx1, i1.data(), i1.size() * sizeof(uint16_t), hipMemcpyHostToDevice), "idx1");
            if (!i2.empty())
                hip_check(hipMemcpy(ctx->d_idx2, i2.data(), i2.size() * sizeof(uint16_t), hipMemcpyHostToDevice), "idx2");
            ctx->b_pre1 = (int)P.bufs.size();
            P.bufs.push_back(BufDesc{"D1 dressed", n1, BUF_REAL});
            ctx->dbuf.push_back(ctx->dalloc(std::max<size_t>((size_t)n1, 1) * sizeof(double)));
            ctx->b_pre2 = (int)P.bufs.size();
            P.bufs.push_back(BufDesc{"D2 dressed", n2, BUF_REAL});
            ctx->dbuf.push_back(ctx->dalloc(std::max<size_t>((size_t)n2, 1) * sizeof(double)));
        }
        if (!f.empty())
            hip_check(hipMemcpyAsync(ctx->d_fov, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice, ctx->st),
                      "f upload");
        hip_check(launch_dressed_denoms(ctx->d_idx1, 2, ctx->d_fov, (int)no, floor, ctx->D(ctx->b_pre1), n1, ctx->st),
                  "D1 dressed");
        hip_check(launch_dressed_denoms(ctx->d_idx2, 4, ctx->d_fov, (int)no, floor, ctx->D(ctx->b_pre2), n2, ctx->st),
                  "D2 dressed");
        // the host vector f is read by the copy above before it goes out of scope
        hip_check(hipStreamSynchronize(ctx->st), "dressed sync");
        D.b_D1 = ctx->b_pre1;
        D.b_D2 = ctx->b_pre2;
    }
    D.order.clear();
    D.watch.restart();
    return FSCC_OK;
}

fscc_status fscc_denominators(fscc_ctx* ctx, fscc_sector sector, double* D1, double* D2) {
    if (!ctx) return FSCC_EINVAL;
    if (sector != FSCC_S00) return fail(ctx, FSCC_EINVAL, "denominators of the (0h,0p) sector only");
    if ((ctx->n1() && !D1) || (ctx->n2() && !D2)) return fail(ctx, FSCC_EINVAL, "null denominator buffer");
    return guarded(ctx, [&]() -> fscc_status {
        const Diis& D = ctx->diis[FSCC_S00];
        if (ctx->n1())
            hip_check(hipMemcpyAsync(D1, ctx->dbuf[D.b_D1], sizeof(double) * ctx->n1(), hipMemcpyDeviceToDevice, ctx->st),
                      "D1 copy");
        if (ctx->n2())
            hip_check(hipMemcpyAsync(D2, ctx->dbuf[D.b_D2], sizeof(double) * ctx->n2(), hipMemcpyDeviceToDevice, ctx->st),
                      "D2 copy");
        return FSCC_OK;
    });
}

fscc_status fscc_precondition(fscc_ctx* ctx, fscc_sector sector, int mode, double floor) {
    if (!ctx) return FSCC_EINVAL;
    Plan& P = ctx->plan;
    if (sector == FSCC_S00) {
        if (mode < 0 || mode > 1 || !(floor > 0.0)) return fail(ctx, FSCC_EINVAL, "bad preconditioner mode or floor");
        if (mode == 1 && !ctx->resid00)
            return fail(ctx, FSCC_ESTATE, "evaluate a (0h,0p) residual before the dressed preconditioner");
        return guarded(ctx, [&]() -> fscc_status { return precondition00(ctx, mode, floor); });
    }
    if (sector != FSCC_S01 || !P.has01) return fail(ctx, FSCC_EINVAL, "no preconditioner modes for this sector");
    if (mode < 0 || mode > 1 || !(floor > 0.0)) return fail(ctx, FSCC_EINVAL, "bad preconditioner mode or floor");
    if (mode == 1 && !ctx->ready01) return fail(ctx, FSCC_ESTATE, "(0h,1p) sector not prepared (fscc_prepare_sector)");
    return guarded(ctx, [&]() -> fscc_status {
        std::vector<double> d1 = P.D1x, d2 = P.D2x;
        if (mode == 1) {
            std::vector<double2> fv = read_elements(ctx, P.b_Fvv01, P.bufs[P.b_Fvv01].n);
            std::vector<double2> fo = read_elements(ctx, P.b_Foo01, P.bufs[P.b_Foo01].n);
            auto fvd = [&](int p) { return fv[(size_t)P.fvv_diag[p]].x; };
            auto fod = [&](int i) { return fo[(size_t)P.foo_diag[i]].x; };
            P.L_S1.for_each([&](int64_t k, const int* p) {
                if (P.mask1[k] != 0.0) d1[k] = std::min(fvd(P.x_vpos[p[0]]) - fvd(p[1]), -floor);
            });
            P.L_S2.for_each([&](int64_t k, const int* p) {
                d2[k] = std::min(fvd(P.x_vpos[p[0]]) + fod(p[1]) - fvd(p[2]) - fvd(p[3]), -floor);
            });
        }
        if (!d1.empty())
            hip_check(hipMemcpy(ctx->dbuf[P.b_D1x], d1.data(), d1.size() * sizeof(double), hipMemcpyHostToDevice), "D1x");
        if (!d2.empty())
            hip_check(hipMemcpy(ctx->dbuf[P.b_D2x], d2.data(), d2.size() * sizeof(double), hipMemcpyHostToDevice), "D2x");
        ctx->diis[1].order.clear();
        ctx->diis[1].watch.restart();
        return FSCC_OK;
    });
}

fscc_status fscc_ladder(fscc_ctx* ctx, const fscc_c128* tau, fscc_c128* out) {
    if (!ctx || !tau || !out) return FSCC_EINVAL;
    if (!ctx->have_cls[IC_VVVV]) return fail(ctx, FSCC_ESTATE, "VVVV integrals not set");
    return guarded(ctx, [&]() -> fscc_status {
        Plan& P = ctx->plan;
        for (size_t k = 0; k < P.ops.size(); ++k)
            if (P.ops[k].name == "pp-ladder") {
                if (ctx->sp.buf >= 0 && !ctx->sp.ch00[k].empty())
                    ctx->run_streamed(P.ops[k], ctx->sp.ch00[k], 0, tau, out);
                else
                    ctx->run_op(P.ops[k], &ctx->L00.g[k], 0, (const double2*)tau, (double2*)out);
                return FSCC_OK;
            }
        throw std::logic_error("no ladder op");
    });
}

fscc_status fscc_diis_reset(fscc_ctx* ctx, fscc_sector sector, int ndiis) {
    if (!ctx) return FSCC_EINVAL;
    if (!(sector == FSCC_S00 || (sector == FSCC_S01 && ctx->plan.has01) || (sector == FSCC_S02 && ctx->plan.has02)))
        return fail(ctx, FSCC_EINVAL, "sector not available for this system");
    if (ndiis < 0 || ndiis > kMaxDiis) return fail(ctx, FSCC_EINVAL, "DIIS depth out of range");
    ctx->diis[sector].ndiis = ndiis;
    ctx->diis[sector].order.clear();
    ctx->diis[sector].watch.restart();
    return FSCC_OK;
}

namespace {

// The update of one sector up to the device work: Jacobi step, DIIS dots,
// bordered solve and extrapolation enqueued on the stream, the subspace's
// slot bookkeeping done, and max|step| / dropped vectors copied to pinned
// host memory (hscal[0..1]); update_finish reads them after a sync.
void update_enqueue(fscc_ctx* ctx, fscc_sector sector, fscc_c128* t1, fscc_c128* t2, const fscc_c128* r1,
                    const fscc_c128* r2) {
    Diis& D = ctx->diis[sector];
    const int64_t n1 = D.n1, n2 = D.n2, n = n1 + n2;
    const int depth = std::max(1, D.ndiis);
    std::vector<int>& ord = D.order;
    int slot;
    if ((int)ord.size() < depth) {
        std::vector<char> used(kMaxDiis, 0);
        for (int s : ord) used[s] = 1;
        slot = 0;
        while (used[slot]) ++slot;
    } else {
        slot = ord.front();
        ord.erase(ord.begin());
    }
    ord.push_back(slot);
    double2* ht = D.ht + (size_t)slot * n;
    double2* he = D.he + (size_t)slot * n;
    int nb1 = n1 > 0 ? reduce_blocks(n1) : 0, nb2 = n2 > 0 ? reduce_blocks(n2) : 0;
    if (ctx->real) {
        // the same sequence on doubles (history slots hold n doubles)
        double* dht = (double*)D.ht + (size_t)slot * n;
        double* dhe = (double*)D.he + (size_t)slot * n;
        if (n1 > 0)
            hip_check(launch_djacobi((const double*)t1, (const double*)r1, (const double*)ctx->dbuf[D.b_D1], dht, dhe, n1,
                                     ctx->part_max, nb1, ctx->st, D.shift, D.dyn_S, D.dyn_n),
                      "jacobi 1");
        if (n2 > 0)
            hip_check(launch_djacobi((const double*)t2, (const double*)r2, (const double*)ctx->dbuf[D.b_D2], dht + n1,
                                     dhe + n1, n2, ctx->part_max + nb1, nb2, ctx->st, D.shift, D.dyn_S, D.dyn_n),
                      "jacobi 2");
        int m = (int)ord.size();
        std::vector<const double*> ev(m);
        for (int j = 0; j < m; ++j) ev[j] = (const double*)D.he + (size_t)ord[j] * n;
        int nbd = reduce_blocks(n);
        hip_check(launch_ddots(ev.data(), m, dhe, n, ctx->part, nbd, ctx->st), "diis dots");
        DiisOrder dord{};
        for (int j = 0; j < m; ++j) dord.v[j] = ord[j];
        hip_check(launch_finish_diis(ctx->part, nbd, m, ctx->part_max, nb1 + nb2, D.dB, kMaxDiis, slot, dord,
                                     ctx->coef, ctx->scal, ctx->st),
                  "diis solve");
        std::vector<const double*> xs(kMaxDiis);
        for (int q = 0; q < kMaxDiis; ++q) xs[q] = (const double*)D.ht + (size_t)q * n;
        if (n1 > 0) hip_check(launch_dlincomb((double*)t1, xs.data(), ctx->coef, kMaxDiis, n1, ctx->st), "lincomb 1");
        if (n2 > 0) {
            for (int q = 0; q < kMaxDiis; ++q) xs[q] = (const double*)D.ht + (size_t)q * n + n1;
            hip_check(launch_dlincomb((double*)t2, xs.data(), ctx->coef, kMaxDiis, n2, ctx->st), "lincomb 2");
        }
    } else {
        if (n1 > 0)
            hip_check(launch_jacobi((const double2*)t1, (const double2*)r1, (const double*)ctx->dbuf[D.b_D1], ht, he, n1,
                                    ctx->part_max, nb1, ctx->st, D.shift, D.dyn_S, D.dyn_n),
                      "jacobi 1");
        if (n2 > 0)
            hip_check(launch_jacobi((const double2*)t2, (const double2*)r2, (const double*)ctx->dbuf[D.b_D2], ht + n1,
                                    he + n1, n2, ctx->part_max + nb1, nb2, ctx->st, D.shift, D.dyn_S, D.dyn_n),
                      "jacobi 2");
        int m = (int)ord.size();
        std::vector<const double2*> ev(m);
        for (int j = 0; j < m; ++j) ev[j] = D.he + (size_t)ord[j] * n;
        int nbd = reduce_blocks(n);
        hip_check(launch_dots(ev.data(), m, he, n, ctx->part, nbd, ctx->st), "diis dots");
        DiisOrder dord{};
        for (int j = 0; j < m; ++j) dord.v[j] = ord[j];
        hip_check(launch_finish_diis(ctx->part, nbd, m, ctx->part_max, nb1 + nb2, D.dB, kMaxDiis, slot, dord,
                                     ctx->coef, ctx->scal, ctx->st),
                  "diis solve");
        std::vector<const double2*> xs(kMaxDiis);
        for (int s = 0; s < kMaxDiis; ++s) xs[s] = D.ht + (size_t)s * n;
        if (n1 > 0) hip_check(launch_lincomb((double2*)t1, xs.data(), ctx->coef, kMaxDiis, n1, ctx->st), "lincomb 1");
        if (n2 > 0) {
            for (int s = 0; s < kMaxDiis; ++s) xs[s] = D.ht + (size_t)s * n + n1;
            hip_check(launch_lincomb((double2*)t2, xs.data(), ctx->coef, kMaxDiis, n2, ctx->st), "lincomb 2");
        }
    }
    hip_check(hipMemcpyAsync(ctx->hscal, ctx->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->st), "scal");
}

// After the stream has synchronised: subspace bookkeeping from the device's
// solve and the divergence watch.
fscc_status update_finish(fscc_ctx* ctx, fscc_sector sector, double* max_step) {
    Diis& D = ctx->diis[sector];
    std::vector<int>& ord = D.order;
    int dropped = (int)ctx->hscal[1];
    if (dropped > 0) ord.erase(ord.begin(), ord.begin() + std::min(dropped, (int)ord.size() - 1));
    if (D.ndiis <= 1) ord.clear();
    double mx = ctx->hscal[0];
    switch (D.watch.observe(mx)) {
        case DivergenceWatch::CONTINUE:
            break;
        case DivergenceWatch::RESET_DIIS:
            ord.clear();   // the next step starts a fresh subspace
            break;
        case DivergenceWatch::GIVE_UP:
            ord.clear();
            D.watch.restart();
            if (!std::isfinite(mx))
                return fail(ctx, FSCC_ENOCONV, "non-finite amplitude step (amplitudes left at their input values)");
            *max_step = mx;
            return fail(ctx, FSCC_ENOCONV,
                        "max|step| = " + std::to_string(mx) + " grew more than " +
                            std::to_string(DivergenceWatch::kGrowth) +
                            "x above its smallest value again after a DIIS reset: the iteration diverges "
                            "(amplitudes hold the last, finite, iterate)");
    }
    *max_step = mx;
    return FSCC_OK;
}

// (0h,0p) energy of t1, t2: tau = t2 + t1 t1 (the first two operations of
// the plan), sum <ij||ab> tau, result copied to hscal[4..5].
void energy_enqueue(fscc_ctx* ctx, const fscc_c128* t1, const fscc_c128* t2) {
    Plan& P = ctx->plan;
    bind_io(ctx, t1, t2, nullptr, nullptr);
    for (size_t k = 0; k < 2; ++k) ctx->run_op(P.ops[k], &ctx->L00.g[k]);
    int nb = reduce_blocks(ctx->n2());
    if (ctx->real)
        hip_check(launch_ddot(ctx->D(P.b_oovv), ctx->D(P.b_tau), ctx->n2(), ctx->epart, nb, ctx->eout, ctx->st), "energy");
    else
        hip_check(launch_zdotu(ctx->B(P.b_oovv), ctx->B(P.b_tau), ctx->n2(), ctx->epart, nb, ctx->eout, ctx->st), "energy");
    hip_check(hipMemcpyAsync(ctx->hscal + 4, ctx->eout, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->st), "e d2h");
}

}  // namespace

fscc_status fscc_update_amplitudes(fscc_ctx* ctx, fscc_sector sector, fscc_c128* t1, fscc_c128* t2,
                                   const fscc_c128* r1, const fscc_c128* r2, double* max_step) {
    if (!ctx || !max_step) return FSCC_EINVAL;
    if (!(sector == FSCC_S00 || (sector == FSCC_S01 && ctx->plan.has01) || (sector == FSCC_S02 && ctx->plan.has02)))
        return fail(ctx, FSCC_EINVAL, "sector not available for this system");
    Diis& D = ctx->diis[sector];
    if ((D.n1 && (!t1 || !r1)) || (D.n2 && (!t2 || !r2))) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
    return guarded(ctx, [&]() -> fscc_status {
        update_enqueue(ctx, sector, t1, t2, r1, r2);
        hip_check(hipStreamSynchronize(ctx->st), "update sync");
        return update_finish(ctx, sector, max_step);
    });
}

fscc_status fscc_iterate(fscc_ctx* ctx, fscc_c128* t1, fscc_c128* t2, fscc_c128* r1, fscc_c128* r2, double* max_step,
                         double* e_re, double* e_im) {
    if (!ctx || !max_step || !e_re || !e_im) return FSCC_EINVAL;
    if (!all_integrals(ctx)) return fail(ctx, FSCC_ESTATE, "integrals not set");
    const int64_t n1 = ctx->n1(), n2 = ctx->n2();
    if ((n1 && (!t1 || !r1)) || (n2 && (!t2 || !r2))) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
    if ((n1 && (const void*)r1 == (const void*)t1) || (n2 && (const void*)r2 == (const void*)t2))
        return fail(ctx, FSCC_EINVAL, "residual aliases amplitudes");
    return guarded(ctx, [&]() -> fscc_status {
        bind_io(ctx, t1, t2, r1, r2);
        ctx->run_list(ctx->L00, ctx->prof);
        ctx->resid00 = true;
        update_enqueue(ctx, FSCC_S00, t1, t2, r1, r2);
        energy_enqueue(ctx, t1, t2);
        hip_check(hipStreamSynchronize(ctx->st), "iteration sync");
        *e_re = ctx->hscal[4];
        *e_im = ctx->hscal[5];
        return update_finish(ctx, FSCC_S00, max_step);
    });
}

fscc_status fscc_energy(fscc_ctx* ctx, const fscc_c128* t1, const fscc_c128* t2, double* e_re, double* e_im) {
    if (!ctx || !e_re || !e_im) return FSCC_EINVAL;
    if (!ctx->have_cls[IC_OOVV]) return fail(ctx, FSCC_ESTATE, "OOVV integrals not set");
    if ((ctx->n1() && !t1) || (ctx->n2() && !t2)) return fail(ctx, FSCC_EINVAL, "null amplitude buffer");
    return guarded(ctx, [&]() -> fscc_status {
        energy_enqueue(ctx, t1, t2);
        hip_check(hipStreamSynchronize(ctx->st), "energy sync");
        *e_re = ctx->hscal[4];
        *e_im = ctx->hscal[5];
        return FSCC_OK;
    });
}

fscc_status fscc_work(const fscc_ctx* ctx, double* gemm_flops, double* ladder_flops, double* ladder_bytes) {
    if (!ctx || !gemm_flops || !ladder_flops || !ladder_bytes) return FSCC_EINVAL;
    const Plan& P = ctx->plan;
    double f = 0, lf = 0, lb = 0;
    for (auto& o : P.ops) {
        if (o.kind != OP_GEMM) continue;
        f += o.flops;
        if (o.name == "pp-ladder") {
            lf = o.flops;
            lb = 16.0 * (double)P.bufs[o.src2].n;
        }
    }
    *gemm_flops = f;
    *ladder_flops = lf;
    *ladder_bytes = lb;
    return FSCC_OK;
}

fscc_status fscc_profile(fscc_ctx* ctx, int enable) {
    if (!ctx) return FSCC_EINVAL;
    return guarded(ctx, [&]() -> fscc_status {
        ctx->prof = enable != 0;
        for (OpList* L : {&ctx->L00, &ctx->L01, &ctx->L02}) {
            ctx->collect(*L);   // finish outstanding timings before clearing
            std::fill(L->ms.begin(), L->ms.end(), 0.0);
            std::fill(L->calls.begin(), L->calls.end(), 0);
        }
        return FSCC_OK;
    });
}

fscc_status fscc_profile_select(fscc_ctx* ctx, int k) {
    if (!ctx) return FSCC_EINVAL;
    int n = 0;
    if (fscc_op_count(ctx, &n) != FSCC_OK || k < -1 || k >= n) return fail(ctx, FSCC_EINVAL, "no such operation");
    ctx->prof_sel = k;
    return FSCC_OK;
}

// operations are numbered: (0h,0p) residual first, then the (0h,1p) and (0h,2p) residuals
static bool op_ref(fscc_ctx* ctx, int k, OpList** L, int* j) {
    int n0 = (int)ctx->plan.ops.size(), n1 = (int)ctx->plan.ops01.size(), n2 = (int)ctx->plan.ops02.size();
    if (k < 0 || k >= n0 + n1 + n2) return false;
    if (k < n0) {
        *L = &ctx->L00;
        *j = k;
    } else if (k < n0 + n1) {
        *L = &ctx->L01;
        *j = k - n0;
    } else {
        *L = &ctx->L02;
        *j = k - n0 - n1;
    }
    return true;
}

fscc_status fscc_op_count(const fscc_ctx* ctx, int* count) {
    if (!ctx || !count) return FSCC_EINVAL;
    *count = (int)(ctx->plan.ops.size() + ctx->plan.ops01.size() + ctx->plan.ops02.size());
    return FSCC_OK;
}

fscc_status fscc_op_traffic(const fscc_ctx* ctx, int k, int* kind, double* bytes) {
    if (!ctx || !kind || !bytes) return FSCC_EINVAL;
    OpList* L;
    int j;
    if (!op_ref(const_cast<fscc_ctx*>(ctx), k, &L, &j)) return FSCC_EINVAL;
    const Op& o = (*L->ops)[j];
    *kind = o.kind == OP_GATHER ? 0 : o.kind == OP_GEMM ? 1 : 2;
    *bytes = o.bytes;
    return FSCC_OK;
}

fscc_status fscc_op_run(fscc_ctx* ctx, int k, int reps) {
    if (!ctx || reps < 1 || reps > 1000) return FSCC_EINVAL;
    OpList* L;
    int j;
    if (!op_ref(ctx, k, &L, &j)) return fail(ctx, FSCC_EINVAL, "op index out of range");
    const Plan& P = ctx->plan;
    auto bound = [&](std::initializer_list<int> ids) {
        for (int b : ids)
            if (b >= 0 && P.bufs[b].n > 0 && !ctx->dbuf[b]) return false;
        return true;
    };
    const bool ok = L == &ctx->L00   ? bound({P.b_t1, P.b_t2, P.b_r1, P.b_r2}) && all_integrals(ctx)
                    : L == &ctx->L01 ? ctx->ready01 && bound({P.b_s1, P.b_s2, P.b_rs1, P.b_rs2})
                                     : ctx->ready02 && bound({P.b_s02, P.b_rs02});
    if (!ok) return fail(ctx, FSCC_ESTATE, "evaluate the operation's residual once first");
    return guarded(ctx, [&]() -> fscc_status {
        const Op& o = (*L->ops)[j];
        for (int r = 0; r < reps; ++r) ctx->run_op(o, o.kind == OP_GEMM ? &L->g[j] : nullptr);
        return FSCC_OK;
    });
}

fscc_status fscc_op_info(fscc_ctx* ctx, int k, const char** name, double* ms, int* calls, double* flops) {
    if (!ctx || !name || !ms || !calls || !flops) return FSCC_EINVAL;
    OpList* L;
    int j;
    if (!op_ref(ctx, k, &L, &j)) return fail(ctx, FSCC_EINVAL, "op index out of range");
    return guarded(ctx, [&]() -> fscc_status {
        ctx->collect(*L);
        const Op& o = (*L->ops)[j];
        *name = o.name.c_str();
        *ms = L->ms[j];
        *calls = L->calls[j];
        *flops = o.flops;
        return FSCC_OK;
    });
}

// Measure every candidate (tile shape x K depth x split) of each GEMM op on
// the device and keep the fastest.  Timing is data independent, so the
// context's own buffers and zeroed temporary amplitude buffers are used.
namespace {

// ---- autotune result cache ------------------------------------------------
// One JSON file holds entries keyed by the GPU architecture, the precision,
// the tuning level, a version of the kernel set and a hash of every operation
// of the context's plans (kind, name, sizes, GEMM problem shapes); an entry
// lists per operation the chosen form: GEMM [1, tile, bk, split, 3M, DB,
// split-precision tile or -1], reorder [0, traversal], other [2].
constexpr int kTuneVersion = 6;

std::vector<OpList*> tune_lists(fscc_ctx* c) { return {&c->L00, &c->L01, &c->L02}; }

std::string tune_key(fscc_ctx* c, int level) {
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, c->device), "hipGetDeviceProperties");
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xFF;
            h *= 1099511628211ull;
        }
    };
    for (OpList* L : tune_lists(c)) {
        if (!L->ops) continue;
        mix(L->ops->size());
        for (const Op& o : *L->ops) {
            mix((uint64_t)o.kind);
            for (char ch : o.name) mix((uint64_t)(unsigned char)ch);
            mix((uint64_t)o.n);
            mix(o.mapsA.size());
            mix(o.gtiles.size());
            mix(o.rtiles.size());
            mix((uint64_t)o.tA | ((uint64_t)o.tB << 1));
            for (const GemmProblem& q : o.probs) {
                mix((uint64_t)q.M);
                mix((uint64_t)q.N);
                mix((uint64_t)q.K);
                mix(((uint64_t)q.lda << 40) ^ ((uint64_t)q.ldb << 20) ^ (uint64_t)q.ldc);
            }
        }
    }
    char hex[32];
    std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)h);
    std::string arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == '"' || ch == '\\') ch = '_';
    return arch + "|p" + std::to_string(c->prec) + "|L" + std::to_string(level) + "|v" + std::to_string(kTuneVersion) +
           (c->real ? "|real" : "|complex") + "|" + hex;
}

std::vector<std::array<int, 7>> tune_collect(fscc_ctx* c) {
    std::vector<std::array<int, 7>> out;
    for (OpList* L : tune_lists(c)) {
        if (!L->ops) continue;
        for (size_t k = 0; k < L->ops->size(); ++k) {
            const Op& o = (*L->ops)[k];
            if (o.kind == OP_GEMM) {
                const GemmDev& g = L->g[k];
                out.push_back({1, g.cfg, g.bk, g.split ? 1 : 0, g.m3 ? 1 : 0, g.lds, g.mx ? g.mx->cfg : -1});
            } else if (o.kind == OP_GATHER) {
                out.push_back({0, o.use_rtiles ? 2 : o.use_gtiles ? 1 : 0, 0, 0, 0, 0, -1});
            } else {
                out.push_back({2, 0, 0, 0, 0, 0, -1});
            }
        }
    }
    return out;
}

// Read the entry for key; false if the file or the entry is absent or malformed.
bool tune_load(const std::string& path, const std::string& key, std::vector<std::array<int, 7>>& ops) {
    std::FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    std::string text;
    char buf[65536];
    for (size_t r; (r = std::fread(buf, 1, sizeof buf, f)) > 0;) text.append(buf, r);
    std::fclose(f);
    const std::string tag = "{\"key\": \"" + key + "\", \"ops\": [";
    size_t p = text.find(tag);
    if (p == std::string::npos) return false;
    p += tag.size();
    ops.clear();
    while (p < text.size()) {
        while (p < text.size() && (text[p] == ' ' || text[p] == ',')) ++p;
        if (p < text.size() && text[p] == ']') return true;
        if (p >= text.size() || text[p] != '[') return false;
        ++p;
        std::array<int, 7> a;
        for (int j = 0; j < 7; ++j) {
            while (p < text.size() && (text[p] == ' ' || text[p] == ',')) ++p;
            char* end = nullptr;
            const long v = std::strtol(text.c_str() + p, &end, 10);
            if (end == text.c_str() + p) return false;
            a[j] = (int)v;
            p = (size_t)(end - text.c_str());
        }
        while (p < text.size() && text[p] == ' ') ++p;
        if (p >= text.size() || text[p] != ']') return false;
        ++p;
        ops.push_back(a);
    }
    return false;
}

// Add (or replace) the entry for key; the file is rewritten through a
// temporary file and a rename, so a reader never sees half an entry.
void tune_store(const std::string& path, const std::string& key, const std::vector<std::array<int, 7>>& ops) {
    const std::string head = "{\"key\": \"";
    std::vector<std::string> keep;
    if (std::FILE* f = std::fopen(path.c_str(), "r")) {
        std::string text;
        char buf[65536];
        for (size_t r; (r = std::fread(buf, 1, sizeof buf, f)) > 0;) text.append(buf, r);
        std::fclose(f);
        // one entry per line; keep the other keys' entries
        for (size_t a = 0; a < text.size();) {
            size_t b = text.find('\n', a);
            if (b == std::string::npos) b = text.size();
            std::string line = text.substr(a, b - a);
            while (!line.empty() && (line.back() == ',' || line.back() == '\r')) line.pop_back();
            if (line.rfind(head, 0) == 0 && line.rfind(head + key + "\"", 0) != 0) keep.push_back(line);
            a = b + 1;
        }
    }
    std::string e = head + key + "\", \"ops\": [";
    for (size_t i = 0; i < ops.size(); ++i) {
        e += i ? ", [" : "[";
        for (int j = 0; j < 7; ++j) e += (j ? ", " : "") + std::to_string(ops[i][j]);
        e += "]";
    }
    e += "]}";
    keep.push_back(e);
    const std::string tmp = path + ".tmp." + std::to_string((long long)getpid());
    std::FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;   // an unwritable cache only costs the next run its tuning
    std::fputs("{\"fscc_autotune_cache\": 1, \"entries\": [\n", f);
    for (size_t i = 0; i < keep.size(); ++i) {
        std::fputs(keep[i].c_str(), f);
        std::fputs(i + 1 < keep.size() ? ",\n" : "\n", f);
    }
    std::fputs("]}\n", f);
    if (std::fclose(f) == 0) {
        if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
    } else {
        std::remove(tmp.c_str());
    }
}

// Apply cached choices; false (nothing changed) if they do not fit this plan.
bool tune_apply(fscc_ctx* c, const std::vector<std::array<int, 7>>& ops) {
    size_t i = 0;
    for (OpList* L : tune_lists(c)) {
        if (!L->ops) continue;
        for (size_t k = 0; k < L->ops->size(); ++k, ++i) {
            if (i >= ops.size()) return false;
            const Op& o = (*L->ops)[k];
            const auto& a = ops[i];
            const int kind = o.kind == OP_GEMM ? 1 : o.kind == OP_GATHER ? 0 : 2;
            if (a[0] != kind) return false;
            if (kind == 1) {
                if (!cfg_ok(o, a[1], c->real) || (a[2] != 16 && a[2] != 32)) return false;
                if (a[5] < LDS_STAGED || a[5] > LDS_DIRECT) return false;
                if (a[5] != LDS_STAGED && a[2] != 16) return false;
                if (a[5] == LDS_DOUBLE && c->real) return false;
                if ((a[5] == LDS_DOUBLE && !zcfg_has_db(a[1])) || (a[5] == LDS_DIRECT && !zcfg_has_dl(a[1]))) return false;
                if (a[6] >= MCFG_N) return false;
            } else if (kind == 0) {
                if (a[1] < 0 || a[1] > 2 || (a[1] == 2 && !o.d_rtiles) || (a[1] == 1 && !o.d_gtiles)) return false;
            }
        }
    }
    if (i != ops.size()) return false;
    i = 0;
    for (OpList* L : tune_lists(c)) {
        if (!L->ops) continue;
        for (size_t k = 0; k < L->ops->size(); ++k, ++i) {
            Op& o = (*L->ops)[k];
            const auto& a = ops[i];
            if (a[0] == 0) {
                o.use_rtiles = a[1] == 2;
                o.use_gtiles = a[1] == 1;
            } else if (a[0] == 1) {
                GemmDev& g = L->g[k];
                MixedDev* keep = g.mx;
                g.mx = nullptr;
                free_gemm(g);
                plan_gemm(c, o, g, a[1], a[2], a[3] != 0, a[4] != 0);
                g.lds = a[5];
                g.mx = keep;
                if (a[6] >= 0 && g.mx && g.mx->cfg != a[6]) {
                    const int prec = g.mx->prec;
                    fscc_ctx::free_mixed(g.mx);
                    g.mx = plan_mixed(c, o, prec, a[6]);
                }
            }
        }
    }
    return true;
}

}  // namespace

fscc_status fscc_tune_cache(fscc_ctx* ctx, const char* path) {
    if (!ctx) return FSCC_EINVAL;
    ctx->tune_path = path ? path : "";
    return FSCC_OK;
}

fscc_status fscc_autotune_cached(const fscc_ctx* ctx, int* from_cache) {
    if (!ctx || !from_cache) return FSCC_EINVAL;
    *from_cache = ctx->tune_from_cache ? 1 : 0;
    return FSCC_OK;
}

fscc_status fscc_autotune(fscc_ctx* ctx, int level) {
    if (!ctx) return FSCC_EINVAL;
    if (ctx->sp.buf >= 0) return fail(ctx, FSCC_ESTATE, "autotune before moving VVVV out of device memory");
    if (level < 0 || level > 2) return fail(ctx, FSCC_EINVAL, "autotune level must be 0, 1 or 2");
    return guarded(ctx, [&]() -> fscc_status {
        Plan& P = ctx->plan;
        std::vector<OpList*> lists = {&ctx->L00, &ctx->L01, &ctx->L02};
        if (level == 0) {
            for (OpList* L : lists)
                for (size_t k = 0; k < L->ops->size(); ++k) {
                    const Op& o = (*L->ops)[k];
                    (*L->ops)[k].use_gtiles = false;
                    (*L->ops)[k].use_rtiles = false;
                    if (o.kind != OP_GEMM) continue;
                    MixedDev* keep = L->g[k].mx;
                    L->g[k].mx = nullptr;
                    free_gemm(L->g[k]);
                    plan_gemm_default(ctx, o, L->g[k]);
                    L->g[k].mx = keep;
                }
            return FSCC_OK;
        }
        ctx->tune_from_cache = false;
        std::string key;
        if (!ctx->tune_path.empty()) {
            key = tune_key(ctx, level);
            std::vector<std::array<int, 7>> cached;
            if (tune_load(ctx->tune_path, key, cached) && tune_apply(ctx, cached)) {
                ctx->tune_from_cache = true;
                return FSCC_OK;
            }
        }
        int64_t nio = 2 * std::max<int64_t>(1, ctx->n1()) + 2 * std::max<int64_t>(1, ctx->n2());
        if (P.has01) nio += 2 * std::max<int64_t>(1, P.L_S1.total) + 2 * std::max<int64_t>(1, P.L_S2.total);
        if (P.has02) nio += 2 * std::max<int64_t>(1, P.L_S02.total);
        double2* tmp = (double2*)ctx->dalloc((size_t)nio * sizeof(double2));   // large enough for either element type
        hip_check(hipMemsetAsync(tmp, 0, (size_t)nio * sizeof(double2), ctx->st), "memset");
        {
            double2* q = tmp;
            auto take = [&](int64_t cnt) {
                double2* r = q;
                q += std::max<int64_t>(1, cnt);
                return (fscc_c128*)r;
            };
            fscc_c128* a = take(ctx->n1());
            fscc_c128* b = take(ctx->n2());
            fscc_c128* c = take(ctx->n1());
            fscc_c128* d = take(ctx->n2());
            bind_io(ctx, a, b, c, d);
            if (P.has01) {
                fscc_c128* e = take(P.L_S1.total);
                fscc_c128* f = take(P.L_S2.total);
                fscc_c128* g = take(P.L_S1.total);
                fscc_c128* h = take(P.L_S2.total);
                bind_io01(ctx, e, f, g, h);
            }
            if (P.has02) {
                fscc_c128* e = take(P.L_S02.total);
                fscc_c128* f = take(P.L_S02.total);
                bind_io02(ctx, e, f);
            }
        }
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        // FSCC_AUTOTUNE_LOG=1: every measured candidate on stderr
        const bool tlog = std::getenv("FSCC_AUTOTUNE_LOG") != nullptr;
        auto note = [&](const Op& o, const GemmDev& g, float ms) {
            if (tlog)
                std::fprintf(stderr, "autotune %-16s cfg %2d bk %d split %d m3 %d lds %d: %.4f ms\n", o.name.c_str(), g.cfg,
                             g.bk, g.split ? 1 : 0, g.m3 ? 1 : 0, g.lds, ms);
        };
        auto time_op = [&](const Op& o, const GemmDev* g) -> float {
            ctx->run_op(o, g);
            float best = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                hip_check(hipEventRecord(e0, ctx->st), "event");
                ctx->run_op(o, g);
                hip_check(hipEventRecord(e1, ctx->st), "event");
                hip_check(hipEventSynchronize(e1), "event sync");
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
                best = std::min(best, ms);
            }
            return best;
        };
        for (OpList* L : lists)
            for (size_t k = 0; k < L->ops->size() && level == 1; ++k) {
                const Op& o = (*L->ops)[k];
                if (o.kind == OP_GATHER && o.d_gtiles && !ctx->real) {
                    // destination order, 16 x 16 tiles or affine tiles, whichever is fastest
                    Op& m = (*L->ops)[k];
                    m.use_gtiles = false;
                    m.use_rtiles = false;
                    const float rows = time_op(m, nullptr);
                    m.use_gtiles = true;
                    const float tiles = time_op(m, nullptr);
                    float aff = 1e30f;
                    if (m.d_rtiles) {
                        m.use_rtiles = true;
                        aff = time_op(m, nullptr);
                    }
                    m.use_rtiles = aff < std::min(rows, tiles);
                    m.use_gtiles = !m.use_rtiles && tiles < rows;
                    if (tlog)
                        std::fprintf(stderr, "autotune %-16s reorder rows %.4f tiles %.4f affine %.4f ms\n", m.name.c_str(),
                                     rows, tiles, aff);
                    continue;
                }
                if (o.kind != OP_GEMM || o.flops < 1e5) continue;
                MixedDev* keep = L->g[k].mx;   // the FP64 candidates are timed without it
                L->g[k].mx = nullptr;
                GemmDev best = L->g[k];
                float best_ms = time_op(o, &best);
                for (int cfg = 0; cfg < ZCFG_N; ++cfg)
                    for (int bk : {16, 32})
                        for (int sp = 1; sp >= 0; --sp) {
                            if ((cfg == ZCFG_SKINNY || cfg == ZCFG_TALL || cfg == ZCFG_RED || cfg == ZCFG_DOT) && bk != 16)
                                continue;
                            if (((cfg == ZCFG_TALL || cfg == ZCFG_DOT) && sp == 1) || (cfg == ZCFG_RED && sp == 0)) continue;
                            if (!cfg_ok(o, cfg, ctx->real)) continue;
                            GemmDev cand;
                            plan_gemm(ctx, o, cand, cfg, bk, sp == 1);
                            // a plan without a split that the sp = 1 pass already timed
                            const bool timed_split_pass = !(cfg == ZCFG_TALL || cfg == ZCFG_DOT);
                            if (sp == 0 && !cand.split && timed_split_pass) {
                                GemmDev probe;
                                plan_gemm(ctx, o, probe, cfg, bk, true);
                                bool same = !probe.split;
                                free_gemm(probe);
                                if (same) {
                                    free_gemm(cand);
                                    continue;
                                }
                            }
                            // the LDS staging forms of the same plan: through registers,
                            // double-buffered, direct-to-LDS ring
                            for (int lds = LDS_STAGED; lds <= LDS_DIRECT; ++lds) {
                                if (lds != LDS_STAGED &&
                                    (bk != 16 || (lds == LDS_DOUBLE && (ctx->real || !zcfg_has_db(cfg))) ||
                                     (lds == LDS_DIRECT && !zcfg_has_dl(cfg))))
                                    continue;
                                cand.lds = lds;
                                float ms = time_op(o, &cand);
                                note(o, cand, ms);
                                if (ms < best_ms) {
                                    if (best.probs != cand.probs) free_gemm(best);
                                    best = cand;
                                    best_ms = ms;
                                }
                            }
                            if (best.probs != cand.probs) free_gemm(cand);
                        }
                if (best.m3) {   // the winner's tile with the four-product complex form
                    GemmDev alt;
                    plan_gemm(ctx, o, alt, best.cfg, best.bk, best.split, false);
                    alt.lds = best.lds;
                    float ms = time_op(o, &alt);
                    note(o, alt, ms);
                    if (ms < best_ms) {
                        free_gemm(best);
                        best = alt;
                        best_ms = ms;
                    } else {
                        free_gemm(alt);
                    }
                }
                L->g[k] = best;
                L->g[k].mx = keep;
            }
        if (ctx->prec != FSCC_FP64)
            for (OpList* ML : {&ctx->L00, &ctx->L01})
            for (size_t k = 0; ML->ops && k < ML->ops->size(); ++k) {
                const Op& o = (*ML->ops)[k];
                GemmDev& g = ML->g[k];
                if (!mixed_eligible(o, ctx->prec) || !g.mx) continue;
                float best_ms = time_op(o, &g);
                for (int cfg = 0; cfg < MCFG_N; ++cfg) {
                    if (cfg == g.mx->cfg) continue;
                    MixedDev* old = g.mx;
                    g.mx = plan_mixed(ctx, o, ctx->prec, cfg);
                    float ms = time_op(o, &g);
                    if (ms < best_ms) {
                        best_ms = ms;
                        fscc_ctx::free_mixed(old);
                    } else {
                        fscc_ctx::free_mixed(g.mx);
                        g.mx = old;
                    }
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        hip_check(hipStreamSynchronize(ctx->st), "autotune sync");
        (void)hipFree(tmp);
        // the caller-buffer slots pointed into tmp: unbound until the next residual
        for (size_t b = 0; b < P.bufs.size(); ++b)
            if (caller_buffer(P.bufs[b].kind)) ctx->dbuf[b] = nullptr;
        if (!key.empty()) tune_store(ctx->tune_path, key, tune_collect(ctx));
        return FSCC_OK;
    });
}

fscc_status fscc_dynamic_shift(fscc_ctx* ctx, fscc_sector sector, double S, int n) {
    if (!ctx) return FSCC_EINVAL;
    if (sector != FSCC_S00 && sector != FSCC_S01 && sector != FSCC_S02) return fail(ctx, FSCC_EINVAL, "unknown sector");
    if (sector == FSCC_S01 && !ctx->plan.has01) return fail(ctx, FSCC_EINVAL, "context has no (0h,1p) sector");
    if (sector == FSCC_S02 && !ctx->plan.has02) return fail(ctx, FSCC_EINVAL, "context has no (0h,2p) sector");
    if (!(S <= 0.0 && S > -1e6) || (S < 0.0 && (n < 1 || n > 16)))
        return fail(ctx, FSCC_EINVAL, "dynamic shift needs -1e6 < S <= 0 and 1 <= n <= 16");
    Diis& D = ctx->diis[sector];
    D.dyn_S = S;
    D.dyn_n = S < 0.0 ? n : 0;
    D.order.clear();   // iterates of other equations are no DIIS history
    D.watch.restart();
    return FSCC_OK;
}

// Linearised least-squares Pade fit: modified Gram-Schmidt QR of the
// augmented complex system [A | y] (Bjorck's least-squares form), then back
// substitution; at most 17 unknowns.
fscc_status fscc_pade(int npts, const double* x, const fscc_c128* y, int L, int M, double x0, fscc_c128* out) {
    if (!x || !y || !out || L < 0 || M < 0 || L + M + 1 > 17 || npts < L + M + 1 || npts > 4096) return FSCC_EINVAL;
    typedef std::complex<double> cd;
    const int nu = L + M + 1, nc = nu + 1;
    // column j of the augmented matrix: Q[j * npts + i]
    //   rows: sum_j a_j x^j - y sum_{j>=1} b_j x^j = y
    std::vector<cd> Q((size_t)nc * npts);
    for (int i = 0; i < npts; ++i) {
        const cd yi(y[i].re, y[i].im);
        if (!std::isfinite(x[i]) || !std::isfinite(yi.real()) || !std::isfinite(yi.imag())) return FSCC_EINVAL;
        double p = 1.0;
        for (int j = 0; j <= L; ++j, p *= x[i]) Q[(size_t)j * npts + i] = p;
        p = x[i];
        for (int j = 1; j <= M; ++j, p *= x[i]) Q[(size_t)(L + j) * npts + i] = -yi * p;
        Q[(size_t)nu * npts + i] = yi;
    }
    std::vector<cd> R((size_t)nu * nc, cd(0.0));
    std::vector<double> n0(nu, 0.0);
    for (int j = 0; j < nu; ++j) {
        for (int i = 0; i < npts; ++i) n0[j] += std::norm(Q[(size_t)j * npts + i]);
        n0[j] = std::sqrt(n0[j]);
    }
    for (int j = 0; j < nu; ++j) {
        double nrm = 0.0;
        for (int i = 0; i < npts; ++i) nrm += std::norm(Q[(size_t)j * npts + i]);
        nrm = std::sqrt(nrm);
        if (!(nrm > 1e-12 * n0[j])) return FSCC_EINVAL;   // numerically rank deficient
        R[(size_t)j * nc + j] = nrm;
        for (int i = 0; i < npts; ++i) Q[(size_t)j * npts + i] /= nrm;
        for (int k = j + 1; k < nc; ++k) {
            cd d = 0.0;
            for (int i = 0; i < npts; ++i) d += std::conj(Q[(size_t)j * npts + i]) * Q[(size_t)k * npts + i];
            R[(size_t)j * nc + k] = d;
            for (int i = 0; i < npts; ++i) Q[(size_t)k * npts + i] -= d * Q[(size_t)j * npts + i];
        }
    }
    std::vector<cd> coef(nu);
    for (int r = nu - 1; r >= 0; --r) {
        cd acc = R[(size_t)r * nc + nu];
        for (int k = r + 1; k < nu; ++k) acc -= R[(size_t)r * nc + k] * coef[k];
        coef[r] = acc / R[(size_t)r * nc + r];
    }
    cd num = 0.0, den = 1.0;
    double p = 1.0;
    for (int j = 0; j <= L; ++j, p *= x0) num += coef[j] * p;
    p = x0;
    for (int j = 1; j <= M; ++j, p *= x0) den += coef[L + j] * p;
    const cd v = num / den;
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return FSCC_EINVAL;
    out->re = v.real();
    out->im = v.imag();
    return FSCC_OK;
}

fscc_status fscc_vvvv_out_of_core(fscc_ctx* ctx, size_t staging_bytes) {
    if (!ctx) return FSCC_EINVAL;
    if (!all_integrals(ctx)) return fail(ctx, FSCC_ESTATE, "integrals not set");
    return guarded(ctx, [&]() -> fscc_status {
        Plan& P = ctx->plan;
        int b = -1;
        for (auto& o : P.ops)
            if (o.name == "pp-ladder") b = o.src2;
        if (b < 0) throw std::logic_error("no ladder op");
        const size_t es = ctx->esz();
        const size_t bytes = (size_t)P.bufs[b].n * es;
        if (staging_bytes == 0) {   // back to device memory
            if (ctx->sp.buf < 0) return FSCC_OK;
            hip_check(hipStreamSynchronize(ctx->st), "sync");
            hip_check(hipStreamSynchronize(ctx->sp.cs), "sync");
            void* d = ctx->dalloc(bytes);
            hip_check(hipMemcpy(d, ctx->sp.host, bytes, hipMemcpyHostToDevice), "operand to device");
            ctx->dbuf[b] = d;
            ctx->free_stream();
            return FSCC_OK;
        }
        if (ctx->sp.buf >= 0) return fail(ctx, FSCC_ESTATE, "VVVV is already out of device memory");
        if (ctx->prec != FSCC_FP64) return fail(ctx, FSCC_ESTATE, "out-of-core VVVV needs FP64 precision");
        // every reader of the buffer must be a GEMM taking it as a transposed B
        for (OpList* L : {&ctx->L00, &ctx->L01p, &ctx->L01, &ctx->L02p, &ctx->L02})
            for (auto& o : *L->ops) {
                const bool reads = o.src == b || o.dst == b || o.src2 == b ||
                                   std::find(o.srcT.begin(), o.srcT.end(), b) != o.srcT.end();
                if (reads && !(o.kind == OP_GEMM && o.src2 == b && o.tB && L != &ctx->L01p && L != &ctx->L02p))
                    return fail(ctx, FSCC_EINVAL, "operation " + o.name + " cannot stream VVVV");
            }
        StreamPlan& sp = ctx->sp;
        try {
            sp.half = (long long)(staging_bytes / 2 / es);
            if (sp.half < 1) throw std::invalid_argument("staging buffer too small");
            hip_check(hipHostMalloc(&sp.host, std::max<size_t>(bytes, 16), hipHostMallocDefault), "hipHostMalloc");
            hip_check(hipStreamSynchronize(ctx->st), "sync");
            if (bytes) hip_check(hipMemcpy(sp.host, ctx->dbuf[b], bytes, hipMemcpyDeviceToHost), "operand to host");
            sp.bytes = bytes;
            for (int s = 0; s < 2; ++s) {
                sp.stage[s] = ctx->dalloc((size_t)sp.half * es);
                hip_check(hipEventCreateWithFlags(&sp.free_ev[s], hipEventDisableTiming), "event");
                hip_check(hipEventRecord(sp.free_ev[s], ctx->st), "event");
            }
            hip_check(hipStreamCreateWithFlags(&sp.cs, hipStreamNonBlocking), "copy stream");
            sp.ch00 = stream_plan(ctx, ctx->L00, b, sp.half);
            sp.ch01 = stream_plan(ctx, ctx->L01, b, sp.half);
            sp.ch02 = stream_plan(ctx, ctx->L02, b, sp.half);
            sp.buf = b;
        } catch (...) {
            ctx->free_stream();
            throw;
        }
        (void)hipFree(ctx->dbuf[b]);
        ctx->dbuf[b] = nullptr;
        return FSCC_OK;
    });
}

fscc_status fscc_gather_order(fscc_ctx* ctx, int tiled) {
    if (!ctx) return FSCC_EINVAL;
    if (tiled < 0 || tiled > 2) return fail(ctx, FSCC_EINVAL, "gather order must be 0, 1 or 2");
    for (OpList* L : {&ctx->L00, &ctx->L01p, &ctx->L01, &ctx->L02p, &ctx->L02})
        if (L->ops)
            for (auto& o : *L->ops) {
                // affine tiles where the gather has them, 16 x 16 tiles otherwise
                o.use_rtiles = tiled == 2 && o.d_rtiles != nullptr;
                o.use_gtiles = !o.use_rtiles && tiled >= 1 && o.d_gtiles != nullptr;
            }
    return FSCC_OK;
}

fscc_status fscc_level_shift(fscc_ctx* ctx, fscc_sector sector, double shift) {
    if (!ctx) return FSCC_EINVAL;
    if (sector != FSCC_S00) return fail(ctx, FSCC_EINVAL, "level shift applies to the (0h,0p) sector");
    if (!(shift >= 0.0 && shift < 1e6)) return fail(ctx, FSCC_EINVAL, "level shift must be in [0, 1e6)");
    ctx->diis[sector].shift = shift;
    return FSCC_OK;
}

fscc_status fscc_set_precision(fscc_ctx* ctx, fscc_precision prec) {
    if (!ctx) return FSCC_EINVAL;
    if (prec != FSCC_FP64 && prec != FSCC_SPLIT_FP32 && prec != FSCC_SPLIT_BF16)
        return fail(ctx, FSCC_EINVAL, "unknown precision");
    if (ctx->real && prec != FSCC_FP64) return fail(ctx, FSCC_EINVAL, "a real context computes in FP64 only");
    if (ctx->sp.buf >= 0 && prec != FSCC_FP64)
        return fail(ctx, FSCC_ESTATE, "split precision needs VVVV in device memory");
    return guarded(ctx, [&]() -> fscc_status {
        apply_precision(ctx, prec);
        return FSCC_OK;
    });
}

fscc_status fscc_get_precision(const fscc_ctx* ctx, int* prec) {
    if (!ctx || !prec) return FSCC_EINVAL;
    *prec = ctx->real ? FSCC_REAL_FP64 : ctx->prec;
    return FSCC_OK;
}

fscc_status fscc_mixed_config(const fscc_ctx* ctx, int k, int* cfg) {
    if (!ctx || !cfg) return FSCC_EINVAL;
    OpList* L;
    int j;
    if (!op_ref(const_cast<fscc_ctx*>(ctx), k, &L, &j)) return FSCC_EINVAL;
    const GemmDev& g = L->g[j];
    *cfg = (g.mx && g.mx->prec == ctx->prec && ctx->prec != FSCC_FP64) ? g.mx->cfg : -1;
    return FSCC_OK;
}

fscc_status fscc_zgemm_split(int prec, int cfg, int tA, int tB, int cA, int cB, int M, int N, int K,
                             const fscc_c128* A, int lda, const fscc_c128* B, int ldb, fscc_c128* C, int ldc,
                             double alpha_re, double alpha_im, int beta, void* hip_stream) {
    if (prec != FSCC_SPLIT_FP32 && prec != FSCC_SPLIT_BF16) return FSCC_EINVAL;
    if (M < 0 || N < 0 || K < 0 || cfg < 0 || cfg >= MCFG_N) return FSCC_EINVAL;
    if ((M > 0 && N > 0) && (!C || (K > 0 && (!A || !B)))) return FSCC_EINVAL;
    if (ldc < N || lda < (tA ? M : K) || ldb < (tB ? K : N)) return FSCC_EINVAL;
    if (M == 0 || N == 0) return FSCC_OK;
    fscc_ctx* c = new (std::nothrow) fscc_ctx();
    if (!c) return FSCC_ENOMEM;
    c->st = (hipStream_t)hip_stream;
    fscc_status s = guarded(c, [&]() -> fscc_status {
        // a one-op plan with two caller buffers (ids 0 and 1), neither constant
        c->plan.bufs.push_back(BufDesc{"A", 0, BUF_SCRATCH});
        c->plan.bufs.push_back(BufDesc{"B", 0, BUF_SCRATCH});
        Op o;
        o.kind = OP_GEMM;
        o.name = "zgemm";
        o.src = 0;
        o.src2 = 1;
        o.tA = tA != 0;
        o.tB = tB != 0;
        o.cA = cA != 0;
        o.cB = cB != 0;
        o.alpha = cplx(alpha_re, alpha_im);
        o.beta = beta ? 1 : 0;
        o.probs.push_back(GemmProblem{0, 0, 0, M, N, K, std::max(lda, 1), std::max(ldb, 1), ldc});
        MixedDev* m = plan_mixed(c, o, prec, cfg);
        c->prec = prec;
        hipError_t e = c->run_mixed(o, *m, (const double2*)A, (const double2*)B, (double2*)C, o.beta);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        fscc_ctx::free_mixed(m);
        hip_check(e, "zgemm_split");
        return FSCC_OK;
    });
    delete c;
    return s;
}

fscc_status fscc_gemm_config(const fscc_ctx* ctx, int k, int* cfg, int* bk, int* split) {
    if (!ctx || !cfg || !bk || !split) return FSCC_EINVAL;
    OpList* L;
    int j;
    if (!op_ref(const_cast<fscc_ctx*>(ctx), k, &L, &j)) return FSCC_EINVAL;
    const GemmDev& g = L->g[j];
    *cfg = (*L->ops)[j].kind == OP_GEMM ? (g.cfg | (g.m3 ? FSCC_CFG_3M : 0) | (g.lds == LDS_DOUBLE ? FSCC_CFG_DB : 0) |
                                           (g.lds == LDS_DIRECT ? FSCC_CFG_DL : 0))
                                        : -1;
    *bk = g.bk;
    *split = g.split ? 1 : 0;
    return FSCC_OK;
}

fscc_status fscc_zgemm(int cfg, int bk, int tA, int tB, int cA, int cB, int M, int N, int K, const fscc_c128* A, int lda,
                       const fscc_c128* B, int ldb, fscc_c128* C, int ldc, double alpha_re, double alpha_im, int beta,
                       int allow_split, void* hip_stream) {
    const bool m3 = cfg >= 0 && (cfg & FSCC_CFG_3M);
    const bool db = cfg >= 0 && (cfg & FSCC_CFG_DB);
    const bool dl = cfg >= 0 && (cfg & FSCC_CFG_DL);
    if (cfg >= 0) cfg &= ~(FSCC_CFG_3M | FSCC_CFG_DB | FSCC_CFG_DL);
    if (M < 0 || N < 0 || K < 0 || cfg >= ZCFG_N || (bk != 16 && bk != 32)) return FSCC_EINVAL;
    if (db && (dl || bk != 16 || !zcfg_has_db(cfg))) return FSCC_EINVAL;
    if (dl && (bk != 16 || !zcfg_has_dl(cfg))) return FSCC_EINVAL;
    if ((M > 0 && N > 0) && (!C || (K > 0 && (!A || !B)))) return FSCC_EINVAL;
    if (ldc < N || lda < (tA ? M : K) || ldb < (tB ? K : N)) return FSCC_EINVAL;
    fscc_ctx* c = new (std::nothrow) fscc_ctx();
    if (!c) return FSCC_ENOMEM;
    c->st = (hipStream_t)hip_stream;
    fscc_status s = guarded(c, [&]() -> fscc_status {
        Op o;
        o.kind = OP_GEMM;
        o.name = "zgemm";
        o.tA = tA != 0;
        o.tB = tB != 0;
        o.cA = cA != 0;
        o.cB = cB != 0;
        o.alpha = cplx(alpha_re, alpha_im);
        o.beta = beta ? 1 : 0;
        if (M > 0 && N > 0) o.probs.push_back(GemmProblem{0, 0, 0, M, N, K, std::max(lda, 1), std::max(ldb, 1), ldc});
        if (cfg >= 0 && !cfg_ok(o, cfg)) return FSCC_EINVAL;
        GemmDev g;
        plan_gemm(c, o, g, cfg < 0 ? pick_cfg(o) : cfg, bk, allow_split != 0, cfg < 0 || m3);
        g.lds = dl ? LDS_DIRECT : db ? LDS_DOUBLE : LDS_STAGED;
        hipError_t e;
        if (!g.split) {
            e = launch_zgemm(g.cfg, g.bk, o.tA, o.tB, (const double2*)A, (const double2*)B, (double2*)C, g.probs, g.tiles,
                             g.ntiles, alpha_re, alpha_im, o.beta, o.cA, o.cB, c->st, 0, nullptr, g.maxM, g.m3, g.lds);
        } else {
            e = launch_zgemm(g.cfg, g.bk, o.tA, o.tB, (const double2*)A, (const double2*)B, g.work, g.probs, g.tiles,
                             g.ntiles, 1.0, 0.0, 0, o.cA, o.cB, c->st, 0, nullptr, g.maxM, g.m3, g.lds);
            if (e == hipSuccess)
                e = launch_splitk_reduce((double2*)C, g.work, g.reds, g.nred, g.maxMN, g.maxS, alpha_re, alpha_im, o.beta, c->st);
        }
        hip_check(e, "zgemm");
        hip_check(hipStreamSynchronize(c->st), "zgemm sync");
        free_gemm(g);
        return FSCC_OK;
    });
    if (s != FSCC_OK) free_call_error() = c->err;
    delete c;
    return s;
}


fscc_status fscc_dgemm(int cfg, int bk, int tA, int tB, int M, int N, int K, const double* A, int lda, const double* B,
                       int ldb, double* C, int ldc, double alpha, int beta, int allow_split, void* hip_stream) {
    const bool dl = cfg >= 0 && (cfg & FSCC_CFG_DL);
    if (cfg >= 0) cfg &= ~FSCC_CFG_DL;
    if (M < 0 || N < 0 || K < 0 || cfg >= ZCFG_N || (bk != 16 && bk != 32)) return FSCC_EINVAL;
    if (dl && (bk != 16 || !zcfg_has_dl(cfg))) return FSCC_EINVAL;
    if ((M > 0 && N > 0) && (!C || (K > 0 && (!A || !B)))) return FSCC_EINVAL;
    if (ldc < N || lda < (tA ? M : K) || ldb < (tB ? K : N)) return FSCC_EINVAL;
    fscc_ctx* c = new (std::nothrow) fscc_ctx();
    if (!c) return FSCC_ENOMEM;
    c->st = (hipStream_t)hip_stream;
    c->real = true;
    fscc_status s = guarded(c, [&]() -> fscc_status {
        Op o;
        o.kind = OP_GEMM;
        o.name = "dgemm";
        o.tA = tA != 0;
        o.tB = tB != 0;
        o.alpha = cplx(alpha, 0.0);
        o.beta = beta ? 1 : 0;
        if (M > 0 && N > 0) o.probs.push_back(GemmProblem{0, 0, 0, M, N, K, std::max(lda, 1), std::max(ldb, 1), ldc});
        if (cfg >= 0 && !cfg_ok(o, cfg, true)) return FSCC_EINVAL;
        GemmDev g;
        plan_gemm(c, o, g, cfg < 0 ? pick_cfg(o, true) : cfg, bk, allow_split != 0);
        g.lds = dl ? LDS_DIRECT : LDS_STAGED;
        hipError_t e;
        if (!g.split) {
            e = launch_dgemm(g.cfg, g.bk, o.tA, o.tB, A, B, C, g.probs, g.tiles, g.ntiles, alpha, o.beta, c->st, 0,
                             nullptr, g.maxM, g.lds);
        } else {
            e = launch_dgemm(g.cfg, g.bk, o.tA, o.tB, A, B, (double*)g.work, g.probs, g.tiles, g.ntiles, 1.0, 0, c->st,
                             0, nullptr, g.maxM, g.lds);
            if (e == hipSuccess)
                e = launch_dsplitk_reduce(C, (const double*)g.work, g.reds, g.nred, g.maxMN, g.maxS, alpha, o.beta, c->st);
        }
        hip_check(e, "dgemm");
        hip_check(hipStreamSynchronize(c->st), "dgemm sync");
        free_gemm(g);
        return FSCC_OK;
    });
    delete c;
    return s;
}
}  // extern "C"
