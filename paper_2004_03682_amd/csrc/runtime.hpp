// runtime.hpp -- host runtime shared by the single-system and batched C ABI:
// device GEMM plans, op lists, DIIS state and the context that executes a
// residual plan on a HIP stream.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fscc.h"
#include "diverge.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace fscc {
namespace rt {


// one operand of a split-precision GEMM: its piece planes and how to fill them
struct SplitDev {
    SplitProb* sp = nullptr;
    int nsp = 0;
    long long max_chunks = 0;
    void* planes = nullptr;
    long long plane = 0;      // elements per plane
    bool conj = false;
    bool constant = false;    // integral-derived: split once, then reused
    bool valid = false;
};

// split-precision form of one GEMM op (FSCC_SPLIT_BF16 / FSCC_SPLIT_FP32)
struct MixedDev {
    int prec = 0;
    int cfg = 0;
    MProb* probs = nullptr;
    ZTile* tiles = nullptr;
    int ntiles = 0;
    SplitDev a, b;
};

struct GemmDev {
    ZProb* probs = nullptr;
    ZTile* tiles = nullptr;
    int ntiles = 0;
    int cfg = 0;
    int bk = 16;
    // split-K: the tiles write partial products into `work`, a second pass reduces
    bool split = false;
    int role = 0;   // 1: pp-ladder, 2: ring GEMMs (distinct kernel symbols in profiles)
    ZRed* reds = nullptr;
    int nred = 0;
    int maxMN = 0;
    int maxS = 0;    // largest number of K chunks of a problem (split)
    int maxM = 0;   // largest M over the problems (ZCFG_RED picks its register tile by it)
    bool m3 = false;   // MFMA tiles: complex product from three real products
    int lds = LDS_STAGED;   // MFMA tiles: how K slices are staged in LDS (launch_zgemm)
    double2* work = nullptr;
    MixedDev* mx = nullptr;   // present for the ops that may run in split precision
};

struct HipError : std::runtime_error {
    explicit HipError(const std::string& s) : std::runtime_error(s) {}
};

inline void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int kMaxDiis = kDiisMax;

// one executable op list with its device GEMM lists and timing slots
// One chunk of a GEMM whose B operand streams from pinned host memory: the
// problem pieces whose B rows lie in [lo, hi) (elements of the host copy)
struct StreamChunk {
    long long lo = 0, hi = 0;
    GemmDev g;
    hipEvent_t copied = nullptr;
};

// Out-of-core operand (the packed <ab||cd> integrals): host copy, two device
// staging buffers used alternately, a copy stream, and the chunk lists of the
// GEMMs that read it (indexed like the op list; empty = not streamed).
struct StreamPlan {
    int buf = -1;
    void* host = nullptr;
    size_t bytes = 0;
    void* stage[2] = {nullptr, nullptr};
    long long half = 0;   // elements per staging buffer
    hipStream_t cs = nullptr;
    hipEvent_t free_ev[2] = {nullptr, nullptr};
    int next = 0;         // staging buffer of the next chunk
    std::vector<std::vector<StreamChunk>> ch00, ch01, ch02;
};

struct OpList {
    std::vector<Op>* ops = nullptr;
    std::vector<GemmDev> g;
    std::vector<hipEvent_t> ev;
    std::vector<char> pend;   // events recorded, elapsed time not yet added
    std::vector<double> ms;
    std::vector<int> calls;
    int base = 0;             // number of the first operation (fscc_op_info numbering)
    // Two-stream schedule (fscc_ctx::streams == 2): operations that are bound
    // by the matrix cores run on the context's stream, the others (reorders,
    // elementwise and memory-bound GEMMs) on a second stream, so that the two
    // kinds overlap where the operations' buffers allow.  on2[k]: operation k
    // runs on the second stream; wait[k]: the latest operation of the other
    // stream that k depends on (-1: none); rec[k]: an event is recorded after
    // k for such a wait.
    std::vector<char> on2, rec;
    std::vector<int> wait;
    std::vector<hipEvent_t> xev;
    hipEvent_t fork = nullptr, join = nullptr;
};

// Dependencies of an operation list through its buffers: operation k reads
// src, src2, every term source and, when it accumulates (beta = 1, diagonal
// and multiply forms), dst; it writes dst.  k depends on the last writer of
// every buffer it reads or writes (read after write, write after write) and
// on every reader of dst since that writer (write after read).  Buffers are
// separate allocations, so distinct ids never overlap.
inline std::vector<std::vector<int>> op_dependencies(const std::vector<Op>& ops) {
    std::vector<std::vector<int>> deps(ops.size());
    std::vector<int> last_w;
    std::vector<std::vector<int>> readers;
    auto grow = [&](int b) {
        if (b >= (int)last_w.size()) {
            last_w.resize(b + 1, -1);
            readers.resize(b + 1);
        }
    };
    for (size_t k = 0; k < ops.size(); ++k) {
        const Op& o = ops[k];
        std::vector<int> rd;
        for (int b : {o.src, o.src2})
            if (b >= 0) rd.push_back(b);
        for (int b : o.srcT)
            if (b >= 0) rd.push_back(b);
        if (o.beta || o.kind == OP_DIAG || o.kind == OP_MUL) rd.push_back(o.dst);
        std::vector<int>& d = deps[k];
        for (int b : rd) {
            grow(b);
            if (last_w[b] >= 0) d.push_back(last_w[b]);
        }
        if (o.dst >= 0) {
            grow(o.dst);
            if (last_w[o.dst] >= 0) d.push_back(last_w[o.dst]);
            for (int r : readers[o.dst]) d.push_back(r);
        }
        std::sort(d.begin(), d.end());
        d.erase(std::unique(d.begin(), d.end()), d.end());
        d.erase(std::remove(d.begin(), d.end(), (int)k), d.end());
        for (int b : rd) readers[b].push_back((int)k);
        if (o.dst >= 0) {
            last_w[o.dst] = (int)k;
            readers[o.dst].clear();
        }
    }
    return deps;
}

// The two-stream schedule of a list (see OpList): GEMMs with more than
// 8 flops per algorithmic byte on the first stream, everything else on the
// second.
inline void build_two_stream(OpList& L) {
    const std::vector<Op>& ops = *L.ops;
    const size_t n = ops.size();
    L.on2.assign(n, 0);
    L.rec.assign(n, 0);
    L.wait.assign(n, -1);
    for (size_t k = 0; k < n; ++k) {
        const Op& o = ops[k];
        L.on2[k] = !(o.kind == OP_GEMM && o.flops > 8.0 * std::max(o.bytes, 1.0));
    }
    const std::vector<std::vector<int>> deps = op_dependencies(ops);
    for (size_t k = 0; k < n; ++k) {
        int w = -1;
        for (int j : deps[k])
            if (L.on2[j] != L.on2[k]) w = std::max(w, j);
        L.wait[k] = w;
        if (w >= 0) L.rec[w] = 1;
    }
}

// DIIS state of one sector
struct Diis {
    int ndiis = 6;
    std::vector<int> order;   // live slots, oldest first
    double2* ht = nullptr;
    double2* he = nullptr;
    double* dB = nullptr;
    int64_t n1 = 0, n2 = 0;
    int b_D1 = -1, b_D2 = -1;
    double shift = 0.0;   // level shift of the Jacobi denominators
    double dyn_S = 0.0;   // dynamic denominator shift (changes the solved equations)
    int dyn_n = 0;
    DivergenceWatch watch;   // growth of max|step| (reset of the subspace, then give up)
};


}  // namespace rt
}  // namespace fscc

using namespace fscc;
using namespace fscc::rt;

struct fscc_ctx {
    int device = 0;
    hipStream_t st = nullptr;
    Plan plan;
    std::vector<void*> dbuf;
    std::vector<uint32_t*> dmap;
    OpList L00, L01p, L01, L02p, L02;
    StreamPlan sp;   // out-of-core VVVV (fscc_vvvv_out_of_core)
    bool have_cls[IC_N] = {false, false, false, false, false, false};
    bool ready01 = false;
    bool ready02 = false;
    bool resid00 = false;   // a (0h,0p) residual has been evaluated (its F'_be, F'_mj are current)
    int b_pre1 = -1, b_pre2 = -1;   // dressed (0h,0p) denominators (fscc_precondition)
    uint16_t *d_idx1 = nullptr, *d_idx2 = nullptr;   // per amplitude: its (i, a) / (i, j, a, b) positions
    double* d_fov = nullptr;                          // f_p of the occupied, then the virtual positions
    Diis diis[3];
    double* part = nullptr;
    double* part_max = nullptr;
    double* coef = nullptr;
    double* scal = nullptr;
    double* hscal = nullptr;   // pinned host
    double* epart = nullptr;
    double* eout = nullptr;
    double2* rs_tmp = nullptr; // residual scratch for fscc_heff
    bool prof = false;
    int prof_sel = -1;   // with prof: time only this operation (-1: all)
    // operation lists on one stream or two (see OpList); the second stream is
    // created on first use, with the default priority
    int streams = 1;
    hipStream_t st2 = nullptr;
    // real arithmetic (real double groups): every amplitude, integral and
    // intermediate buffer holds doubles instead of complex doubles
    bool real = false;
    size_t esz() const { return real ? sizeof(double) : sizeof(double2); }
    double* D(int id) const { return (double*)dbuf[id]; }
    int prec = FSCC_FP64;
    const int* d_active = nullptr;   // batched plans: per-system flags, GEMM tiles of 0-systems are skipped
    int validate_n = 4096;           // sampled symmetry checks per integral class (fscc_set_validation)
    std::string tune_path;           // autotune result cache (fscc_tune_cache); empty = none
    bool tune_from_cache = false;    // the last fscc_autotune applied cached choices
    std::string err;

    int64_t n1() const { return plan.L_T1.total; }
    int64_t n2() const { return plan.L_T2.total; }

    void* dalloc(size_t bytes) {
        void* p = nullptr;
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) throw std::bad_alloc();
        return p;
    }

    static void free_mixed(MixedDev*& m) {
        if (!m) return;
        void* ps[] = {m->probs, m->tiles, m->a.sp, m->a.planes, m->b.sp, m->b.planes};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        delete m;
        m = nullptr;
    }

    static void free_gemm_dev(GemmDev& g) {
        if (g.probs) (void)hipFree(g.probs);
        if (g.tiles) (void)hipFree(g.tiles);
        if (g.reds) (void)hipFree(g.reds);
        if (g.work) (void)hipFree(g.work);
        g.probs = nullptr;
        g.tiles = nullptr;
        g.reds = nullptr;
        g.work = nullptr;
    }

    void free_stream() {
        for (auto* L : {&sp.ch00, &sp.ch01, &sp.ch02})
            for (auto& v : *L)
                for (auto& c : v) {
                    free_gemm_dev(c.g);
                    if (c.copied) (void)hipEventDestroy(c.copied);
                }
        for (int s = 0; s < 2; ++s) {
            if (sp.stage[s]) (void)hipFree(sp.stage[s]);
            if (sp.free_ev[s]) (void)hipEventDestroy(sp.free_ev[s]);
        }
        if (sp.cs) (void)hipStreamDestroy(sp.cs);
        if (sp.host) (void)hipHostFree(sp.host);
        sp = StreamPlan();
    }

    static void free_list(OpList& L) {
        if (L.ops)
            for (auto& o : *L.ops)
                if (o.d_gtiles) {
                    (void)hipFree((void*)o.d_gtiles);
                    o.d_gtiles = nullptr;
                }
        for (auto& g : L.g) {
            if (g.probs) (void)hipFree(g.probs);
            if (g.tiles) (void)hipFree(g.tiles);
            if (g.reds) (void)hipFree(g.reds);
            if (g.work) (void)hipFree(g.work);
            free_mixed(g.mx);
        }
        for (auto& e : L.ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : L.xev)
            if (e) (void)hipEventDestroy(e);
        if (L.fork) (void)hipEventDestroy(L.fork);
        if (L.join) (void)hipEventDestroy(L.join);
    }

    ~fscc_ctx() {
        if (sp.cs) (void)hipStreamSynchronize(sp.cs);
        free_stream();
        for (size_t k = 0; k < dbuf.size(); ++k)
            if (!caller_buffer(plan.bufs[k].kind) && dbuf[k]) (void)hipFree(dbuf[k]);
        for (auto* m : dmap)
            if (m) (void)hipFree(m);
        free_list(L00);
        free_list(L01p);
        free_list(L01);
        free_list(L02p);
        free_list(L02);
        for (auto& d : diis) {
            if (d.ht) (void)hipFree(d.ht);
            if (d.he) (void)hipFree(d.he);
            if (d.dB) (void)hipFree(d.dB);
        }
        for (void* p : seg_mem)
            if (p) (void)hipFree(p);
        void* ps[] = {part, part_max, coef, scal, epart, eout, rs_tmp, d_idx1, d_idx2, d_fov};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        if (hscal) (void)hipHostFree(hscal);
        if (st2) {
            (void)hipStreamSynchronize(st2);
            (void)hipStreamDestroy(st2);
        }
    }

    double2* B(int id) const { return (double2*)dbuf[id]; }

    // batched plans: block tables of the segmented elementwise launches, per buffer
    std::vector<SegBlocks> segb;
    std::vector<void*> seg_mem;

    SegBlocks seg_of(int buf, const int* flags) const {
        if (!d_active || buf < 0 || buf >= (int)segb.size() || !segb[buf].sys) return SegBlocks();
        SegBlocks sb = segb[buf];
        sb.active = flags ? flags : d_active;
        return sb;
    }

    // the real-arithmetic form of run_op (real alpha, no conjugation)
    hipError_t run_op_real(const Op& o, const GemmDev* gd, int beta_override, const double* A_override,
                           double* C_override) {
        switch (o.kind) {
            case OP_AXPBY:
                return launch_daxpby(D(o.dst), D(o.src), o.n, o.alpha.real(), o.beta, st);
            case OP_DIAG:
                return launch_ddiag(D(o.dst), (const double*)dbuf[o.src2], D(o.src), o.n, st);
            case OP_MUL:
                return launch_dmul(D(o.dst), (const double*)dbuf[o.src2], o.n, st);
            case OP_GATHER: {
                GatherMaps gm;
                for (int t = 0; t < 4; ++t) {
                    gm.a[t] = t < (int)o.mapsA.size() ? dmap[o.mapsA[t]] : nullptr;
                    gm.b[t] = t < (int)o.mapsB.size() ? dmap[o.mapsB[t]] : nullptr;
                    gm.src[t] = t < (int)o.srcT.size() ? (const void*)D(o.srcT[t]) : nullptr;
                }
                return launch_dgather(D(o.dst), D(o.src), o.src2 >= 0 ? D(o.src2) : nullptr, gm, (int)o.mapsA.size(),
                                      o.n, o.alpha.real(), o.beta, st);
            }
            case OP_GEMM: {
                const GemmDev& g = *gd;
                const int beta = beta_override >= 0 ? beta_override : o.beta;
                const double* Ap = A_override ? A_override : D(o.src);
                double* Cp = C_override ? C_override : D(o.dst);
                if (!g.split)
                    return launch_dgemm(g.cfg, g.bk, o.tA, o.tB, Ap, D(o.src2), Cp, g.probs, g.tiles, g.ntiles,
                                        o.alpha.real(), beta, st, g.role, nullptr, g.maxM, g.lds);
                hipError_t e = launch_dgemm(g.cfg, g.bk, o.tA, o.tB, Ap, D(o.src2), (double*)g.work, g.probs, g.tiles,
                                            g.ntiles, 1.0, 0, st, g.role, nullptr, g.maxM, g.lds);
                if (e == hipSuccess)
                    e = launch_dsplitk_reduce(Cp, (const double*)g.work, g.reds, g.nred, g.maxMN, g.maxS, o.alpha.real(), beta,
                                              st);
                return e;
            }
        }
        return hipSuccess;
    }

    // seg_flags (batched plans only): per-system flags used instead of d_active
    // for the elementwise and gather launches of this call
    void run_op(const Op& o, const GemmDev* gd, int beta_override = -1, const double2* A_override = nullptr,
                double2* C_override = nullptr, const int* seg_flags = nullptr) {
        hipError_t e = hipSuccess;
        if (real) {
            hip_check(run_op_real(o, gd, beta_override, (const double*)A_override, (double*)C_override), o.name.c_str());
            return;
        }
        const SegBlocks sb = seg_of(o.dst, seg_flags);
        switch (o.kind) {
            case OP_AXPBY:
                e = launch_axpby(B(o.dst), B(o.src), o.n, o.alpha.real(), o.alpha.imag(), o.beta, o.conj, st, sb);
                break;
            case OP_DIAG:
                e = launch_diag(B(o.dst), (const double*)dbuf[o.src2], B(o.src), o.n, st, sb);
                break;
            case OP_MUL:
                e = launch_mul(B(o.dst), (const double*)dbuf[o.src2], o.n, st, sb);
                break;
            case OP_GATHER: {
                GatherMaps gm;
                for (int t = 0; t < 4; ++t) {
                    gm.a[t] = t < (int)o.mapsA.size() ? dmap[o.mapsA[t]] : nullptr;
                    gm.b[t] = t < (int)o.mapsB.size() ? dmap[o.mapsB[t]] : nullptr;
                    gm.src[t] = t < (int)o.srcT.size() ? (const void*)B(o.srcT[t]) : nullptr;
                }
                if (o.use_rtiles && o.d_rtiles && !sb.sys)
                    e = launch_reorder(B(o.dst), B(o.src), gm, (int)o.mapsA.size(), o.d_runits, (int)o.runits.size(),
                                       o.d_rtiles, o.d_rterms, o.alpha.real(), o.alpha.imag(), o.beta, o.conj, st);
                else if (o.use_gtiles && o.d_gtiles && !sb.sys)
                    e = launch_gather_tiled(B(o.dst), B(o.src), o.src2 >= 0 ? B(o.src2) : nullptr, gm,
                                            (int)o.mapsA.size(), o.d_gtiles, (int)o.gtiles.size(), o.alpha.real(),
                                            o.alpha.imag(), o.beta, o.conj, st);
                else
                    e = launch_gather(B(o.dst), B(o.src), o.src2 >= 0 ? B(o.src2) : nullptr, gm, (int)o.mapsA.size(),
                                      o.n, o.alpha.real(), o.alpha.imag(), o.beta, o.conj, st, sb);
                break;
            }
            case OP_GEMM: {
                const GemmDev& g = *gd;
                int beta = beta_override >= 0 ? beta_override : o.beta;
                const double2* Ap = A_override ? A_override : B(o.src);
                double2* Cp = C_override ? C_override : B(o.dst);
                if (prec != FSCC_FP64 && g.mx && g.mx->prec == prec && !(A_override && g.mx->a.constant)) {
                    e = run_mixed(o, *g.mx, Ap, B(o.src2), Cp, beta);
                } else if (!g.split) {
                    e = launch_zgemm(g.cfg, g.bk, o.tA, o.tB, Ap, B(o.src2), Cp, g.probs, g.tiles, g.ntiles,
                                     o.alpha.real(), o.alpha.imag(), beta, o.cA, o.cB, st, g.role, d_active, g.maxM, g.m3, g.lds);
                } else {
                    e = launch_zgemm(g.cfg, g.bk, o.tA, o.tB, Ap, B(o.src2), g.work, g.probs, g.tiles, g.ntiles, 1.0,
                                     0.0, 0, o.cA, o.cB, st, g.role, d_active, g.maxM, g.m3, g.lds);
                    if (e == hipSuccess)
                        e = launch_splitk_reduce(Cp, g.work, g.reds, g.nred, g.maxMN, g.maxS, o.alpha.real(), o.alpha.imag(),
                                                 beta, st, d_active);
                }
                break;
            }
        }
        hip_check(e, o.name.c_str());
    }

    hipError_t split_operand(SplitDev& d, const double2* src, bool bf16) {
        if (d.constant && d.valid) return hipSuccess;
        hipError_t e = launch_split(bf16, src, d.planes, d.plane, d.sp, d.nsp, d.max_chunks, d.conj ? 1 : 0, st);
        if (e == hipSuccess && d.constant) d.valid = true;
        return e;
    }

    hipError_t run_mixed(const Op& o, MixedDev& m, const double2* A, const double2* Bm, double2* C, int beta) {
        const bool bf = m.prec == FSCC_SPLIT_BF16;
        hipError_t e = split_operand(m.a, A, bf);
        if (e == hipSuccess) e = split_operand(m.b, Bm, bf);
        if (e == hipSuccess)
            e = launch_zgemm_split(bf, m.cfg, m.a.planes, m.a.plane, m.b.planes, m.b.plane, C, m.probs, m.tiles,
                                   m.ntiles, o.alpha.real(), o.alpha.imag(), beta, st,
                                   o.name == "pp-ladder" ? 1 : 2);
        return e;
    }

    std::vector<std::vector<StreamChunk>>* stream_chunks(OpList& L) {
        if (sp.buf < 0) return nullptr;
        if (&L == &L00) return &sp.ch00;
        if (&L == &L01) return &sp.ch01;
        if (&L == &L02) return &sp.ch02;
        return nullptr;
    }

    // A GEMM whose B operand is streamed: per chunk, the copy stream brings its
    // rows into the staging buffer not in use (after the GEMM that last read
    // it), and the GEMM of the chunk runs on the context's stream once the copy
    // has landed, so copies and matrix-core work overlap.  B is addressed as
    // stage - lo, so the problems keep their offsets into the full operand.
    void run_streamed(const Op& o, std::vector<StreamChunk>& chunks, int beta_override = -1,
                      const void* A_override = nullptr, void* C_override = nullptr) {
        const size_t es = esz();
        int s = sp.next;
        for (auto& c : chunks) {
            hip_check(hipStreamWaitEvent(sp.cs, sp.free_ev[s], 0), "stream wait");
            if (c.hi > c.lo)
                hip_check(hipMemcpyAsync(sp.stage[s], (const char*)sp.host + (size_t)c.lo * es,
                                         (size_t)(c.hi - c.lo) * es, hipMemcpyHostToDevice, sp.cs),
                          "operand stream copy");
            hip_check(hipEventRecord(c.copied, sp.cs), "event");
            hip_check(hipStreamWaitEvent(st, c.copied, 0), "stream wait");
            const void* Bp = (const char*)sp.stage[s] - (ptrdiff_t)((size_t)c.lo * es);
            if (real) {
                hip_check(gemm_real(o, c.g, beta_override, (const double*)A_override, (double*)C_override,
                                    (const double*)Bp),
                          o.name.c_str());
            } else {
                hip_check(gemm_complex(o, c.g, beta_override, (const double2*)A_override, (double2*)C_override,
                                       (const double2*)Bp),
                          o.name.c_str());
            }
            hip_check(hipEventRecord(sp.free_ev[s], st), "event");
            s ^= 1;
        }
        sp.next = s;
    }

    hipError_t gemm_complex(const Op& o, const GemmDev& g, int beta_override, const double2* A_override,
                            double2* C_override, const double2* Bp) {
        const int beta = beta_override >= 0 ? beta_override : o.beta;
        const double2* Ap = A_override ? A_override : B(o.src);
        double2* Cp = C_override ? C_override : B(o.dst);
        if (!g.split)
            return launch_zgemm(g.cfg, g.bk, o.tA, o.tB, Ap, Bp, Cp, g.probs, g.tiles, g.ntiles, o.alpha.real(),
                                o.alpha.imag(), beta, o.cA, o.cB, st, g.role, nullptr, g.maxM, g.m3, g.lds);
        hipError_t e = launch_zgemm(g.cfg, g.bk, o.tA, o.tB, Ap, Bp, g.work, g.probs, g.tiles, g.ntiles, 1.0, 0.0, 0,
                                    o.cA, o.cB, st, g.role, nullptr, g.maxM, g.m3, g.lds);
        if (e == hipSuccess)
            e = launch_splitk_reduce(Cp, g.work, g.reds, g.nred, g.maxMN, g.maxS, o.alpha.real(), o.alpha.imag(), beta, st);
        return e;
    }

    hipError_t gemm_real(const Op& o, const GemmDev& g, int beta_override, const double* A_override,
                         double* C_override, const double* Bp) {
        const int beta = beta_override >= 0 ? beta_override : o.beta;
        const double* Ap = A_override ? A_override : D(o.src);
        double* Cp = C_override ? C_override : D(o.dst);
        if (!g.split)
            return launch_dgemm(g.cfg, g.bk, o.tA, o.tB, Ap, Bp, Cp, g.probs, g.tiles, g.ntiles, o.alpha.real(), beta,
                                st, g.role, nullptr, g.maxM, g.lds);
        hipError_t e = launch_dgemm(g.cfg, g.bk, o.tA, o.tB, Ap, Bp, (double*)g.work, g.probs, g.tiles, g.ntiles, 1.0,
                                    0, st, g.role, nullptr, g.maxM, g.lds);
        if (e == hipSuccess)
            e = launch_dsplitk_reduce(Cp, (const double*)g.work, g.reds, g.nred, g.maxMN, g.maxS, o.alpha.real(), beta, st);
        return e;
    }

    // add the elapsed times of operations timed earlier (waits for their end events)
    void collect(OpList& L) {
        for (size_t k = 0; k < L.pend.size(); ++k) {
            if (!L.pend[k]) continue;
            hip_check(hipEventSynchronize(L.ev[2 * k + 1]), "event sync");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, L.ev[2 * k], L.ev[2 * k + 1]), "elapsed");
            L.ms[k] += ms;
            L.calls[k] += 1;
            L.pend[k] = 0;
        }
    }

    // timed: HIP events around every operation (or only operation prof_sel),
    // read back lazily, so timing adds no synchronisation to the stream
    void run_list(OpList& L, bool timed) {
        std::vector<Op>& ops = *L.ops;
        if (timed && L.ev.size() != 2 * ops.size()) {
            L.ev.assign(2 * ops.size(), nullptr);
            for (auto& e : L.ev) hip_check(hipEventCreate(&e), "hipEventCreate");
            L.pend.assign(ops.size(), 0);
        }
        if (timed) collect(L);
        std::vector<std::vector<StreamChunk>>* sc = stream_chunks(L);
        if (streams == 2 && !sc && !d_active) {
            run_list_two(L, timed);
            return;
        }
        for (size_t k = 0; k < ops.size(); ++k) {
            const bool tk = timed && (prof_sel < 0 || prof_sel == L.base + (int)k);
            if (tk) hip_check(hipEventRecord(L.ev[2 * k], st), "event");
            if (sc && k < sc->size() && !(*sc)[k].empty()) run_streamed(ops[k], (*sc)[k]);
            else run_op(ops[k], &L.g[k]);
            if (tk) {
                hip_check(hipEventRecord(L.ev[2 * k + 1], st), "event");
                L.pend[k] = 1;
            }
        }
    }

    // run_list on two streams: the second stream first waits for the work
    // already on the context's stream, every cross-stream dependency is an
    // event wait, and the context's stream finally waits for the second, so
    // that callers see one stream.  Operations launch on the member stream st,
    // which is switched per operation (and restored on every exit).
    void run_list_two(OpList& L, bool timed) {
        std::vector<Op>& ops = *L.ops;
        if (!st2) hip_check(hipStreamCreateWithFlags(&st2, hipStreamNonBlocking), "second stream");
        if (L.on2.size() != ops.size()) {
            build_two_stream(L);
            L.xev.assign(ops.size(), nullptr);
            for (size_t k = 0; k < ops.size(); ++k)
                if (L.rec[k]) hip_check(hipEventCreateWithFlags(&L.xev[k], hipEventDisableTiming), "event");
            hip_check(hipEventCreateWithFlags(&L.fork, hipEventDisableTiming), "event");
            hip_check(hipEventCreateWithFlags(&L.join, hipEventDisableTiming), "event");
        }
        const hipStream_t s0 = st;
        struct Restore {
            hipStream_t& s;
            hipStream_t v;
            ~Restore() { s = v; }
        } restore{st, s0};
        hip_check(hipEventRecord(L.fork, s0), "event");
        hip_check(hipStreamWaitEvent(st2, L.fork, 0), "stream wait");
        for (size_t k = 0; k < ops.size(); ++k) {
            const hipStream_t s = L.on2[k] ? st2 : s0;
            if (L.wait[k] >= 0) hip_check(hipStreamWaitEvent(s, L.xev[L.wait[k]], 0), "stream wait");
            const bool tk = timed && (prof_sel < 0 || prof_sel == L.base + (int)k);
            if (tk) hip_check(hipEventRecord(L.ev[2 * k], s), "event");
            st = s;
            run_op(ops[k], &L.g[k]);
            st = s0;
            if (tk) {
                hip_check(hipEventRecord(L.ev[2 * k + 1], s), "event");
                L.pend[k] = 1;
            }
            if (L.rec[k]) hip_check(hipEventRecord(L.xev[k], s), "event");
        }
        hip_check(hipEventRecord(L.join, st2), "event");
        hip_check(hipStreamWaitEvent(s0, L.join, 0), "stream wait");
    }
};


namespace fscc {
namespace rt {

inline fscc_status fail(fscc_ctx* c, fscc_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

// Last error message of the context-free calls (fscc_zgemm, fscc_zgemm_noalloc)
// on the calling thread; fscc_last_error(NULL) returns it.
std::string& free_call_error();
inline fscc_status free_call_fail(fscc_status s, const std::string& msg) {
    free_call_error() = msg;
    return s;
}

template <class F>
fscc_status guarded(fscc_ctx* c, F f) {
    try {
        return f();
    } catch (const HipError& e) {
        return fail(c, FSCC_EHIP, e.what());
    } catch (const std::bad_alloc&) {
        return fail(c, FSCC_ENOMEM, "device or host allocation failed");
    } catch (const std::invalid_argument& e) {
        return fail(c, FSCC_EINVAL, e.what());
    } catch (const std::exception& e) {
        return fail(c, FSCC_EINVAL, e.what());
    } catch (...) {
        return fail(c, FSCC_EINVAL, "unknown error");
    }
}

bool cfg_ok(const Op& o, int cfg, bool real = false);
double cfg_cost(const Op& o, int cfg);
int pick_cfg(const Op& o, bool real = false);
std::vector<ZTile> xcd_order(const std::vector<ZTile>& logical);
void free_gemm(GemmDev& g);
bool mixed_eligible(const Op& o, int prec);
MixedDev* plan_mixed(fscc_ctx* c, const Op& o, int prec, int cfg);
int pick_mcfg(const Op& o);
void apply_precision(fscc_ctx* c, int prec);
void plan_gemm(fscc_ctx* c, const Op& o, GemmDev& g, int cfg, int bk, bool allow_split, bool m3 = true);
// The host half of plan_gemm: problem, tile and split-K reduction tables of one
// GEMM op, and the split-K workspace size (complex or real elements).  h.g
// holds the launch parameters with null device pointers.
struct GemmHost {
    GemmDev g;
    std::vector<ZProb> pr;
    std::vector<ZTile> tl;
    std::vector<ZRed> rd;
    long long work_elems = 0;
};
void plan_gemm_host(bool real, const Op& o, int cfg, int bk, bool allow_split, bool m3, GemmHost& h);
double op_bytes(const Plan& P, const Op& o, const std::vector<int64_t>& nnz, size_t es);
void setup_list(fscc_ctx* c, OpList& L, std::vector<Op>& ops);
void setup_diis(fscc_ctx* c, Diis& d, int64_t n1, int64_t n2, int bD1, int bD2);
void bind_io(fscc_ctx* c, const fscc_c128* t1, const fscc_c128* t2, fscc_c128* r1, fscc_c128* r2);
void bind_io01(fscc_ctx* c, const fscc_c128* s1, const fscc_c128* s2, fscc_c128* r1, fscc_c128* r2);
void bind_io02(fscc_ctx* c, const fscc_c128* s, fscc_c128* r);
bool all_integrals(const fscc_ctx* c);
void ctx_allocate(fscc_ctx* c, bool diis);

}  // namespace rt
}  // namespace fscc
