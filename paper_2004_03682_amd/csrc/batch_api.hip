// batch_api.hip -- many independent systems in one set of grouped launches.
//
// The residual plans of all systems are concatenated buffer by buffer: every
// buffer of the merged plan holds system 0's part, then system 1's, ...; the
// GEMM problem lists (one problem per pair irrep and system) are merged into
// one grouped launch per contraction, the gather maps are rebased, and the
// elementwise operations run over the concatenation.  The uneven symmetry
// blocks of all systems thus share each launch, and the tile list is ordered
// and tuned as for one system.  The Jacobi + DIIS update keeps a separate
// subspace per system on the device (batched kernels), freezes a system once
// its step falls below the tolerance (its GEMM tiles are then skipped), and
// one whole iteration can be captured as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <array>
#include <memory>
#include <thread>

#include "runtime.hpp"

namespace fscc {
namespace rt {

namespace {

void merge_plans(const std::vector<std::unique_ptr<Plan>>& sub, Plan& M, std::vector<std::vector<int64_t>>& base) {
    const Plan& P0 = *sub[0];
    const size_t nb = P0.bufs.size(), nsys = sub.size();
    for (auto& sp : sub) {
        const Plan& P = *sp;
        if (P.bufs.size() != nb || P.ops.size() != P0.ops.size()) throw std::logic_error("batched plans differ in shape");
        for (size_t b = 0; b < nb; ++b)
            if (P.bufs[b].name != P0.bufs[b].name || P.bufs[b].kind != P0.bufs[b].kind)
                throw std::logic_error("batched plans differ in buffer " + P0.bufs[b].name);
        if (P.has01) throw std::invalid_argument("batched systems carry the (0h,0p) sector only (nact must be 0)");
    }
    base.assign(nsys, std::vector<int64_t>(nb, 0));
    M.bufs = P0.bufs;
    for (size_t b = 0; b < nb; ++b) {
        int64_t off = 0;
        for (size_t s = 0; s < nsys; ++s) {
            base[s][b] = off;
            off += sub[s]->bufs[b].n;
        }
        M.bufs[b].n = off;
    }
    M.b_t1 = P0.b_t1;
    M.b_t2 = P0.b_t2;
    M.b_r1 = P0.b_r1;
    M.b_r2 = P0.b_r2;
    M.b_D1 = P0.b_D1;
    M.b_D2 = P0.b_D2;
    M.b_oovv = P0.b_oovv;
    M.b_tau = P0.b_tau;
    M.L_T1.total = M.bufs[P0.b_t1].n;
    M.L_T2.total = M.bufs[P0.b_t2].n;
    for (auto& sp : sub) {
        M.D1.insert(M.D1.end(), sp->D1.begin(), sp->D1.end());
        M.D2.insert(M.D2.end(), sp->D2.begin(), sp->D2.end());
    }
    auto whole = [&](size_t k, int buf, int64_t n_s, size_t s) {
        if (buf >= 0 && n_s != sub[s]->bufs[buf].n)
            throw std::logic_error("operation " + P0.ops[k].name + " covers part of a buffer; cannot batch");
    };
    for (size_t k = 0; k < P0.ops.size(); ++k) {
        const Op& o0 = P0.ops[k];
        Op o = o0;
        o.probs.clear();
        o.gtiles.clear();   // batched gathers run over segments in destination order
        o.d_gtiles = nullptr;
        o.use_gtiles = false;
        o.rtiles.clear();
        o.rterms.clear();
        o.runits.clear();
        o.d_rtiles = nullptr;
        o.d_rterms = nullptr;
        o.d_runits = nullptr;
        o.use_rtiles = false;
        o.mapsA.clear();
        o.mapsB.clear();
        o.flops = 0;
        o.n = 0;
        for (size_t s = 0; s < nsys; ++s) {
            const Op& os = sub[s]->ops[k];
            if (os.kind != o0.kind || os.name != o0.name) throw std::logic_error("batched plans differ in operations");
            o.flops += os.flops;
        }
        switch (o0.kind) {
            case OP_GEMM:
                for (size_t s = 0; s < nsys; ++s)
                    for (GemmProblem p : sub[s]->ops[k].probs) {
                        p.a_off += base[s][o0.src];
                        p.b_off += base[s][o0.src2];
                        p.c_off += base[s][o0.dst];
                        p.sys = (int)s;
                        o.probs.push_back(p);
                    }
                break;
            case OP_GATHER: {
                for (size_t s = 0; s < nsys; ++s) {
                    whole(k, o0.dst, sub[s]->ops[k].n, s);
                    o.n += sub[s]->ops[k].n;
                }
                auto rebase = [&](const std::vector<int>& ids_of_sys0, bool second) {
                    std::vector<int> out;
                    for (size_t t = 0; t < ids_of_sys0.size(); ++t) {
                        std::vector<uint32_t> m;
                        m.reserve((size_t)o.n);
                        for (size_t s = 0; s < nsys; ++s) {
                            const Op& os = sub[s]->ops[k];
                            const std::vector<uint32_t>& ms = sub[s]->maps[second ? os.mapsB[t] : os.mapsA[t]];
                            const int src_t = second ? o0.src2 : (t < o0.srcT.size() ? o0.srcT[t] : o0.src);
                            const int64_t sh = base[s][src_t];
                            for (uint32_t e : ms) {
                                if (e == MAP_ZERO) {
                                    m.push_back(e);
                                    continue;
                                }
                                const int64_t off = (int64_t)(e & ~MAP_NEG) + sh;
                                if (off >= (int64_t)0x7FFFFFFF) throw std::length_error("batched gather source exceeds 2^31 elements");
                                m.push_back((uint32_t)off | (e & MAP_NEG));
                            }
                        }
                        out.push_back(M.map(P0.map_names[ids_of_sys0[t]], std::move(m)));
                    }
                    return out;
                };
                o.mapsA = rebase(o0.mapsA, false);
                o.mapsB = rebase(o0.mapsB, true);
                break;
            }
            case OP_AXPBY:
            case OP_DIAG:
            case OP_MUL:
                for (size_t s = 0; s < nsys; ++s) {
                    whole(k, o0.dst, sub[s]->ops[k].n, s);
                    o.n += sub[s]->ops[k].n;
                }
                break;
        }
        M.ops.push_back(std::move(o));
    }
}

}  // namespace
}  // namespace rt
}  // namespace fscc

struct fscc_batch {
    fscc_ctx c;
    int nsys = 0;
    std::vector<std::unique_ptr<Plan>> sub;
    std::vector<std::vector<int64_t>> base;
    std::vector<std::array<char, IC_N>> have;
    std::vector<BSeg> seg;
    int nblk = 32;
    int ndiis = 6;
    double tol = 1e-10;
    double shift = 0.0;
    BSeg* dseg = nullptr;
    BState* dstate = nullptr;
    int* dactive = nullptr;
    int* dupd = nullptr;   // systems updated in the current iteration
    double2 *ht = nullptr, *he = nullptr;
    double *Bm = nullptr, *coef = nullptr, *maxstep = nullptr, *part = nullptr, *part_max = nullptr, *epart = nullptr,
           *report = nullptr;
    double* hreport = nullptr;   // pinned host copy of the report rows
    double *pre1 = nullptr, *pre2 = nullptr;   // dressed Jacobi denominators (fscc_batch_precondition)
    bool dressed = false;
    bool iterated = false;   // a residual has been evaluated (the F' intermediates are current)

    const double* jD1() { return dressed ? pre1 : (const double*)c.dbuf[c.plan.b_D1]; }
    const double* jD2() { return dressed ? pre2 : (const double*)c.dbuf[c.plan.b_D2]; }
    hipStream_t gst = nullptr;   // stream used for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void* gkey[4] = {nullptr, nullptr, nullptr, nullptr};

    double* maxstep_tmp() { return epart; }   // nsys doubles of scratch outside an iteration

    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    }
    ~fscc_batch() {
        if (c.st) (void)hipStreamSynchronize(c.st);
        else (void)hipDeviceSynchronize();
        drop_graph();
        if (gst) (void)hipStreamDestroy(gst);
        void* ps[] = {dseg, dstate, dactive, dupd, ht, he, Bm, coef, maxstep, part, part_max, epart, report, pre1, pre2};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        if (hreport) (void)hipHostFree(hreport);
    }
};

namespace {

fscc_status bfail(fscc_batch* b, fscc_status s, const std::string& msg) { return fail(b ? &b->c : nullptr, s, msg); }

bool batch_ready(const fscc_batch* b) {
    for (auto& h : b->have)
        for (int k = 0; k < IC_N; ++k)
            if (!h[k]) return false;
    return true;
}

// residual -> update -> energy -> report rows to pinned host memory
void enqueue_iteration(fscc_batch* b, hipStream_t st, const fscc_c128* t1, const fscc_c128* t2, fscc_c128* r1,
                       fscc_c128* r2) {
    fscc_ctx& c = b->c;
    hipStream_t keep = c.st;
    c.st = st;
    try {
        Plan& P = c.plan;
        bind_io(&c, t1, t2, r1, r2);
        c.run_list(c.L00, false);
        hip_check(launch_batch_update((const double2*)t1, (const double2*)t2, (const double2*)r1, (const double2*)r2,
                                      (double2*)t1, (double2*)t2, b->jD1(), b->jD2(), b->dseg, b->dstate, b->ht,
                                      b->he, b->part_max,
                                      b->part, b->Bm, b->coef, b->maxstep, b->tol, b->shift, b->dactive, b->dupd, b->nsys, b->nblk, st),
                  "batch update");
        // tau of the updated amplitudes (the systems updated in this iteration)
        for (size_t k = 0; k < 2; ++k) c.run_op(P.ops[k], &c.L00.g[k], -1, nullptr, nullptr, b->dupd);
        hip_check(launch_batch_energy(c.B(P.b_oovv), c.B(P.b_tau), b->dseg, b->dstate, b->maxstep, b->epart, b->report,
                                      b->nsys, b->nblk, st),
                  "batch energy");
        hip_check(hipMemcpyAsync(b->hreport, b->report, (size_t)b->nsys * 6 * sizeof(double), hipMemcpyDeviceToHost, st),
                  "report d2h");
    } catch (...) {
        c.st = keep;
        throw;
    }
    c.st = keep;
}

}  // namespace

extern "C" {

fscc_status fscc_batch_create(const fscc_system* sys, int nsys, fscc_precision prec, void* hip_stream,
                              fscc_batch** out) {
    if (!sys || !out || nsys < 1) return FSCC_EINVAL;
    *out = nullptr;
    if (prec != FSCC_FP64 && prec != FSCC_SPLIT_FP32 && prec != FSCC_SPLIT_BF16) return FSCC_EINVAL;
    for (int s = 0; s < nsys; ++s) {
        const fscc_system& y = sys[s];
        if (y.nocc < 0 || y.nvirt < 0 || y.nirrep < 1 || !y.irrep || !y.eps || y.nact != 0) return FSCC_EINVAL;
    }
    fscc_batch* b = new (std::nothrow) fscc_batch();
    if (!b) return FSCC_ENOMEM;
    fscc_status st = guarded(&b->c, [&]() -> fscc_status {
        fscc_ctx& c = b->c;
        hip_check(hipGetDevice(&c.device), "hipGetDevice");
        c.st = (hipStream_t)hip_stream;
        b->nsys = nsys;
        b->sub.resize(nsys);
        std::vector<System> S(nsys);
        for (int s = 0; s < nsys; ++s) {
            const fscc_system& y = sys[s];
            S[s].nocc = y.nocc;
            S[s].nvirt = y.nvirt;
            S[s].G = y.nirrep;
            const int n = y.nocc + y.nvirt;
            S[s].irrep.assign(y.irrep, y.irrep + n);
            S[s].eps.assign(y.eps, y.eps + n);
            for (int p = 0; p < n; ++p) {
                if (S[s].irrep[p] < 0 || S[s].irrep[p] >= S[s].G) throw std::invalid_argument("irrep label out of range");
                if (!std::isfinite(S[s].eps[p])) throw std::invalid_argument("non-finite orbital energy");
            }
            b->sub[s].reset(new Plan());
        }
        // independent plans, built in parallel
        const int nw = std::max(1, std::min<int>(nsys, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
        std::vector<std::exception_ptr> errs(nw);
        std::vector<std::thread> pool;
        for (int w = 0; w < nw; ++w)
            pool.emplace_back([&, w]() {
                plan_thread_depth()++;   // no nested threads inside one system's plan
                try {
                    for (int s = w; s < nsys; s += nw) build_plan_ccsd(S[s], *b->sub[s]);
                } catch (...) {
                    errs[w] = std::current_exception();
                }
                plan_thread_depth()--;
            });
        for (auto& t : pool) t.join();
        for (auto& e : errs)
            if (e) std::rethrow_exception(e);
        merge_plans(b->sub, c.plan, b->base);
        ctx_allocate(&c, false);
        // per-iteration maps of the systems' own plans are no longer needed
        for (auto& sp : b->sub) {
            std::vector<char> keep(sp->maps.size(), 0);
            for (auto& sg : sp->setup) keep[sg.map] = 1;
            for (size_t k = 0; k < sp->maps.size(); ++k)
                if (!keep[k]) std::vector<uint32_t>().swap(sp->maps[k]);
            sp->ops.clear();
        }
        b->have.assign(nsys, std::array<char, IC_N>{0, 0, 0, 0, 0, 0});
        // segments and per-system DIIS history
        b->seg.resize(nsys);
        int64_t o1 = 0, o2 = 0, ho = 0;
        for (int s = 0; s < nsys; ++s) {
            const int64_t n1 = b->sub[s]->bufs[c.plan.b_t1].n, n2 = b->sub[s]->bufs[c.plan.b_t2].n;
            b->seg[s] = BSeg{o1, n1, o2, n2, ho};
            o1 += n1;
            o2 += n2;
            ho += 8 * (n1 + n2);
        }
        b->nblk = std::max(8, std::min(128, 4096 / nsys));
        b->dseg = (BSeg*)c.dalloc(sizeof(BSeg) * nsys);
        hip_check(hipMemcpy(b->dseg, b->seg.data(), sizeof(BSeg) * nsys, hipMemcpyHostToDevice), "segments");
        b->dstate = (BState*)c.dalloc(sizeof(BState) * nsys);
        b->dactive = (int*)c.dalloc(sizeof(int) * nsys);
        b->ht = (double2*)c.dalloc(sizeof(double2) * (size_t)std::max<int64_t>(1, ho));
        b->he = (double2*)c.dalloc(sizeof(double2) * (size_t)std::max<int64_t>(1, ho));
        b->Bm = (double*)c.dalloc(sizeof(double) * 64 * nsys);
        b->coef = (double*)c.dalloc(sizeof(double) * 8 * nsys);
        b->maxstep = (double*)c.dalloc(sizeof(double) * nsys);
        b->part = (double*)c.dalloc(sizeof(double) * 8 * nsys * b->nblk);
        b->part_max = (double*)c.dalloc(sizeof(double) * nsys * b->nblk);
        b->epart = (double*)c.dalloc(sizeof(double) * 2 * nsys * b->nblk);
        b->report = (double*)c.dalloc(sizeof(double) * 6 * nsys);
        hip_check(hipHostMalloc((void**)&b->hreport, sizeof(double) * 6 * nsys, hipHostMallocDefault), "hipHostMalloc");
        hip_check(hipStreamCreateWithFlags(&b->gst, hipStreamNonBlocking), "capture stream");
        c.d_active = b->dactive;
        b->dupd = (int*)c.dalloc(sizeof(int) * nsys);
        // block tables of the segmented elementwise launches: one per destination buffer
        c.segb.assign(c.plan.bufs.size(), SegBlocks());
        for (const Op& o : c.plan.ops) {
            if (o.kind == OP_GEMM || o.dst < 0 || c.segb[o.dst].sys) continue;
            std::vector<int> bs;
            std::vector<long long> b0, b1;
            for (int s = 0; s < nsys; ++s) {
                const long long base = b->base[s][o.dst], n = b->sub[s]->bufs[o.dst].n;
                for (long long k = 0; k < n; k += 256) {
                    bs.push_back(s);
                    b0.push_back(base + k);
                    b1.push_back(base + n);
                }
            }
            SegBlocks sb;
            sb.nblk = (int)bs.size();
            int* ds = (int*)c.dalloc(sizeof(int) * std::max<size_t>(1, bs.size()));
            long long* d0 = (long long*)c.dalloc(sizeof(long long) * std::max<size_t>(1, bs.size()));
            long long* d1 = (long long*)c.dalloc(sizeof(long long) * std::max<size_t>(1, bs.size()));
            c.seg_mem.push_back(ds);
            c.seg_mem.push_back(d0);
            c.seg_mem.push_back(d1);
            if (!bs.empty()) {
                hip_check(hipMemcpy(ds, bs.data(), sizeof(int) * bs.size(), hipMemcpyHostToDevice), "seg tables");
                hip_check(hipMemcpy(d0, b0.data(), sizeof(long long) * bs.size(), hipMemcpyHostToDevice), "seg tables");
                hip_check(hipMemcpy(d1, b1.data(), sizeof(long long) * bs.size(), hipMemcpyHostToDevice), "seg tables");
            }
            sb.sys = ds;
            sb.start = d0;
            sb.end = d1;
            c.segb[o.dst] = sb;
        }
        apply_precision(&c, prec);
        return FSCC_OK;
    });
    if (st != FSCC_OK) {
        delete b;
        return st;
    }
    fscc_status r = fscc_batch_reset(b, 6, 1e-10, 0.0);
    if (r != FSCC_OK) {
        delete b;
        return r;
    }
    *out = b;
    return FSCC_OK;
}

void fscc_batch_destroy(fscc_batch* b) { delete b; }

const char* fscc_batch_last_error(const fscc_batch* b) { return b ? b->c.err.c_str() : "null batch"; }

fscc_ctx* fscc_batch_context(fscc_batch* b) { return b ? &b->c : nullptr; }

fscc_status fscc_batch_sizes(const fscc_batch* b, size_t* n1, size_t* n2) {
    if (!b || !n1 || !n2) return FSCC_EINVAL;
    *n1 = (size_t)b->c.n1();
    *n2 = (size_t)b->c.n2();
    return FSCC_OK;
}

fscc_status fscc_batch_segment(const fscc_batch* b, int s, size_t* off1, size_t* n1, size_t* off2, size_t* n2) {
    if (!b || !off1 || !n1 || !off2 || !n2 || s < 0 || s >= b->nsys) return FSCC_EINVAL;
    const BSeg& g = b->seg[s];
    *off1 = (size_t)g.off1;
    *n1 = (size_t)g.n1;
    *off2 = (size_t)g.off2;
    *n2 = (size_t)g.n2;
    return FSCC_OK;
}

fscc_status fscc_batch_set_integrals(fscc_batch* b, int s, fscc_iclass cls, const fscc_c128* dev_blocks, size_t n) {
    if (!b) return FSCC_EINVAL;
    if (s < 0 || s >= b->nsys) return bfail(b, FSCC_EINVAL, "system index out of range");
    if ((int)cls < 0 || (int)cls >= IC_N) return bfail(b, FSCC_EINVAL, "bad integral class");
    Plan& P = *b->sub[s];
    if ((int64_t)n != P.full[cls].total)
        return bfail(b, FSCC_EINVAL, "integral class size " + std::to_string(n) + " != expected " +
                                         std::to_string(P.full[cls].total));
    if (n > 0 && !dev_blocks) return bfail(b, FSCC_EINVAL, "null integral buffer");
    if (b->have[s][cls]) return bfail(b, FSCC_ESTATE, "integral class already set");
    return guarded(&b->c, [&]() -> fscc_status {
        fscc_ctx& c = b->c;
        for (auto& sg : P.setup) {
            if (sg.cls != (int)cls) continue;
            std::vector<uint32_t>& m = P.maps[sg.map];
            const int64_t cnt = P.bufs[sg.dst].n;
            if (cnt > 0) {
                if ((int64_t)m.size() != cnt) throw std::logic_error("setup map already consumed: " + sg.name);
                uint32_t* dm = (uint32_t*)c.dalloc(m.size() * sizeof(uint32_t));
                hip_check(hipMemcpyAsync(dm, m.data(), m.size() * sizeof(uint32_t), hipMemcpyHostToDevice, c.st),
                          "pack map upload");
                GatherMaps gm{};
                gm.a[0] = dm;
                hip_check(launch_gather(c.B(sg.dst) + b->base[s][sg.dst], (const double2*)dev_blocks, nullptr, gm, 1,
                                        cnt, 1.0, 0.0, 0, sg.conj ? 1 : 0, c.st),
                          "integral pack");
                hip_check(hipStreamSynchronize(c.st), "pack sync");
                (void)hipFree(dm);
            }
            std::vector<uint32_t>().swap(m);
        }
        b->have[s][cls] = 1;
        return FSCC_OK;
    });
}

fscc_status fscc_batch_reset(fscc_batch* b, int ndiis, double tol, double shift) {
    if (!b) return FSCC_EINVAL;
    if (ndiis < 1 || ndiis > 8 || !(tol > 0.0) || !(shift >= 0.0 && shift < 1e6))
        return bfail(b, FSCC_EINVAL, "ndiis must be 1..8, tol > 0 and 0 <= shift < 1e6");
    return guarded(&b->c, [&]() -> fscc_status {
        b->ndiis = ndiis;
        b->tol = tol;
        b->shift = shift;
        std::vector<BState> h(b->nsys, BState{0, ndiis - 1, 1, 0, 0, 0, ndiis, 0});
        std::vector<int> a(b->nsys, 1);
        hip_check(hipMemcpy(b->dstate, h.data(), sizeof(BState) * b->nsys, hipMemcpyHostToDevice), "state");
        hip_check(hipMemcpy(b->dactive, a.data(), sizeof(int) * b->nsys, hipMemcpyHostToDevice), "active");
        if (b->dupd) hip_check(hipMemcpy(b->dupd, a.data(), sizeof(int) * b->nsys, hipMemcpyHostToDevice), "upd");
        b->drop_graph();   // the tolerance is a kernel argument of the captured update
        return FSCC_OK;
    });
}

fscc_status fscc_batch_build_residual(fscc_batch* b, const fscc_c128* t1, const fscc_c128* t2, fscc_c128* r1,
                                      fscc_c128* r2) {
    if (!b) return FSCC_EINVAL;
    if (!batch_ready(b)) return bfail(b, FSCC_ESTATE, "integrals not set for every system");
    const int64_t n1 = b->c.n1(), n2 = b->c.n2();
    if ((n1 && (!t1 || !r1)) || (n2 && (!t2 || !r2))) return bfail(b, FSCC_EINVAL, "null amplitude buffer");
    if ((n1 && (const void*)r1 == (const void*)t1) || (n2 && (const void*)r2 == (const void*)t2))
        return bfail(b, FSCC_EINVAL, "residual aliases amplitudes");
    return guarded(&b->c, [&]() -> fscc_status {
        bind_io(&b->c, t1, t2, r1, r2);
        b->c.run_list(b->c.L00, b->c.prof);
        b->iterated = true;
        return FSCC_OK;
    });
}

fscc_status fscc_batch_step(fscc_batch* b, fscc_c128* t1, fscc_c128* t2, fscc_c128* r1, fscc_c128* r2, int use_graph,
                            double* report) {
    if (!b || !report) return FSCC_EINVAL;
    if (!batch_ready(b)) return bfail(b, FSCC_ESTATE, "integrals not set for every system");
    const int64_t n1 = b->c.n1(), n2 = b->c.n2();
    if ((n1 && (!t1 || !r1)) || (n2 && (!t2 || !r2))) return bfail(b, FSCC_EINVAL, "null amplitude buffer");
    if ((n1 && (const void*)r1 == (const void*)t1) || (n2 && (const void*)r2 == (const void*)t2))
        return bfail(b, FSCC_EINVAL, "residual aliases amplitudes");
    return guarded(&b->c, [&]() -> fscc_status {
        fscc_ctx& c = b->c;
        if (!use_graph) {
            if (c.prof) {
                bind_io(&c, t1, t2, r1, r2);
                c.run_list(c.L00, true);
                hip_check(launch_batch_update((const double2*)t1, (const double2*)t2, (const double2*)r1,
                                              (const double2*)r2, (double2*)t1, (double2*)t2, b->jD1(), b->jD2(),
                                              b->dseg, b->dstate, b->ht, b->he, b->part_max, b->part, b->Bm, b->coef,
                                              b->maxstep, b->tol, b->shift, b->dactive, b->dupd, b->nsys, b->nblk, c.st),
                          "batch update");
                for (size_t k = 0; k < 2; ++k) c.run_op(c.plan.ops[k], &c.L00.g[k], -1, nullptr, nullptr, b->dupd);
                hip_check(launch_batch_energy(c.B(c.plan.b_oovv), c.B(c.plan.b_tau), b->dseg, b->dstate, b->maxstep,
                                              b->epart, b->report, b->nsys, b->nblk, c.st),
                          "batch energy");
                hip_check(hipMemcpyAsync(b->hreport, b->report, (size_t)b->nsys * 6 * sizeof(double),
                                         hipMemcpyDeviceToHost, c.st),
                          "report d2h");
            } else {
                enqueue_iteration(b, c.st, t1, t2, r1, r2);
            }
        } else {
            const void* key[4] = {t1, t2, r1, r2};
            if (!b->gexec || !std::equal(key, key + 4, b->gkey)) {
                b->drop_graph();
                hip_check(hipStreamSynchronize(c.st), "pre-capture sync");
                hip_check(hipStreamBeginCapture(b->gst, hipStreamCaptureModeThreadLocal), "begin capture");
                try {
                    enqueue_iteration(b, b->gst, t1, t2, r1, r2);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(b->gst, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                hip_check(hipStreamEndCapture(b->gst, &b->graph), "end capture");
                hip_check(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "graph instantiate");
                std::copy(key, key + 4, b->gkey);
            }
            hip_check(hipGraphLaunch(b->gexec, c.st), "graph launch");
        }
        hip_check(hipStreamSynchronize(c.st), "step sync");
        b->iterated = true;
        std::memcpy(report, b->hreport, sizeof(double) * 6 * b->nsys);
        return FSCC_OK;
    });
}

fscc_status fscc_batch_denominators(fscc_batch* b, double* D1, double* D2) {
    if (!b || (b->c.n1() && !D1) || (b->c.n2() && !D2)) return FSCC_EINVAL;
    return guarded(&b->c, [&]() -> fscc_status {
        fscc_ctx& c = b->c;
        if (c.n1())
            hip_check(hipMemcpyAsync(D1, c.dbuf[c.plan.b_D1], sizeof(double) * c.n1(), hipMemcpyDeviceToDevice, c.st),
                      "D1 copy");
        if (c.n2())
            hip_check(hipMemcpyAsync(D2, c.dbuf[c.plan.b_D2], sizeof(double) * c.n2(), hipMemcpyDeviceToDevice, c.st),
                      "D2 copy");
        return FSCC_OK;
    });
}

fscc_status fscc_batch_maxnorm(fscc_batch* b, const fscc_c128* r1, const fscc_c128* r2, double* out) {
    if (!b || !out || (b->c.n1() && !r1) || (b->c.n2() && !r2)) return FSCC_EINVAL;
    return guarded(&b->c, [&]() -> fscc_status {
        fscc_ctx& c = b->c;
        hip_check(launch_batch_maxnorm((const double2*)r1, (const double2*)r2, (const double*)c.dbuf[c.plan.b_D1],
                                       (const double*)c.dbuf[c.plan.b_D2], b->dseg, b->part_max, b->maxstep_tmp(),
                                       b->nsys, b->nblk, c.st),
                  "batch maxnorm");
        hip_check(hipMemcpyAsync(b->hreport, b->maxstep_tmp(), sizeof(double) * b->nsys, hipMemcpyDeviceToHost, c.st),
                  "maxnorm d2h");
        hip_check(hipStreamSynchronize(c.st), "maxnorm sync");
        std::memcpy(out, b->hreport, sizeof(double) * b->nsys);
        return FSCC_OK;
    });
}

fscc_status fscc_batch_restart(fscc_batch* b, const int* mask) {
    if (!b || !mask) return FSCC_EINVAL;
    return guarded(&b->c, [&]() -> fscc_status {
        fscc_ctx& c = b->c;
        std::vector<BState> h(b->nsys);
        std::vector<int> a(b->nsys);
        hip_check(hipStreamSynchronize(c.st), "restart sync");
        hip_check(hipMemcpy(h.data(), b->dstate, sizeof(BState) * b->nsys, hipMemcpyDeviceToHost), "state d2h");
        hip_check(hipMemcpy(a.data(), b->dactive, sizeof(int) * b->nsys, hipMemcpyDeviceToHost), "active d2h");
        for (int s = 0; s < b->nsys; ++s) {
            if (!mask[s]) continue;
            h[s].count = 0;
            h[s].newest = h[s].nd - 1;
            h[s].active = 1;
            h[s].upd = 0;
            h[s].failed = 0;
            a[s] = 1;
        }
        hip_check(hipMemcpy(b->dstate, h.data(), sizeof(BState) * b->nsys, hipMemcpyHostToDevice), "state h2d");
        hip_check(hipMemcpy(b->dactive, a.data(), sizeof(int) * b->nsys, hipMemcpyHostToDevice), "active h2d");
        return FSCC_OK;
    });
}

// Dressed Jacobi denominators per system (the single-system rule of
// fscc_precondition, sector (0h,0p)): f_p = e_p + Re F'_pp from each system's
// F'_be, F'_mj segments of the last residual, written at the system's T1/T2
// segment offsets; the DIIS subspaces restart (iteration counts and the
// active flags are kept).
fscc_status fscc_batch_precondition(fscc_batch* b, int mode, double floor) {
    if (!b) return FSCC_EINVAL;
    if (mode < 0 || mode > 1 || !(floor > 0.0)) return bfail(b, FSCC_EINVAL, "bad preconditioner mode or floor");
    if (mode == 1 && !b->iterated)
        return bfail(b, FSCC_ESTATE, "evaluate a residual (or step) before the dressed preconditioner");
    return guarded(&b->c, [&]() -> fscc_status {
        fscc_ctx& c = b->c;
        Plan& M = c.plan;
        hip_check(hipStreamSynchronize(c.st), "precondition sync");
        if (mode == 0) {
            if (b->dressed) b->drop_graph();
            b->dressed = false;
        } else {
            const int bf = b->sub[0]->b_Fbe, bm = b->sub[0]->b_Fmj;
            std::vector<double2> fbe((size_t)M.bufs[bf].n), fmj((size_t)M.bufs[bm].n);
            hip_check(hipMemcpy(fbe.data(), c.dbuf[bf], fbe.size() * sizeof(double2), hipMemcpyDeviceToHost), "F'be d2h");
            hip_check(hipMemcpy(fmj.data(), c.dbuf[bm], fmj.size() * sizeof(double2), hipMemcpyDeviceToHost), "F'mj d2h");
            std::vector<double> d1((size_t)c.n1()), d2((size_t)c.n2());
            parallel_for((size_t)b->nsys, [&](size_t s) {
                const Plan& P = *b->sub[s];
                std::vector<double> fo(P.eps_o), fv(P.eps_v);
                for (size_t i = 0; i < fo.size(); ++i)
                    if (P.fmj_diag[i] >= 0) fo[i] += fmj[(size_t)(b->base[s][bm] + P.fmj_diag[i])].x;
                for (size_t a = 0; a < fv.size(); ++a)
                    if (P.fbe_diag[a] >= 0) fv[a] += fbe[(size_t)(b->base[s][bf] + P.fbe_diag[a])].x;
                const int64_t o1 = b->seg[s].off1, o2 = b->seg[s].off2;
                P.L_T1.for_each([&](int64_t k, const int* x) { d1[o1 + k] = std::min(fo[x[0]] - fv[x[1]], -floor); });
                P.L_T2.for_each([&](int64_t k, const int* x) {
                    d2[o2 + k] = std::min(fo[x[0]] + fo[x[1]] - fv[x[2]] - fv[x[3]], -floor);
                });
            });
            if (!b->pre1) {
                b->pre1 = (double*)c.dalloc(std::max<size_t>(d1.size(), 1) * sizeof(double));
                b->pre2 = (double*)c.dalloc(std::max<size_t>(d2.size(), 1) * sizeof(double));
            }
            if (!d1.empty())
                hip_check(hipMemcpy(b->pre1, d1.data(), d1.size() * sizeof(double), hipMemcpyHostToDevice), "D1 dressed");
            if (!d2.empty())
                hip_check(hipMemcpy(b->pre2, d2.data(), d2.size() * sizeof(double), hipMemcpyHostToDevice), "D2 dressed");
            if (!b->dressed) b->drop_graph();   // the captured update reads the bare denominators
            b->dressed = true;
        }
        std::vector<BState> h(b->nsys);
        hip_check(hipMemcpy(h.data(), b->dstate, sizeof(BState) * b->nsys, hipMemcpyDeviceToHost), "state d2h");
        for (auto& x : h) {
            x.count = 0;
            x.newest = x.nd - 1;
        }
        hip_check(hipMemcpy(b->dstate, h.data(), sizeof(BState) * b->nsys, hipMemcpyHostToDevice), "state h2d");
        return FSCC_OK;
    });
}

}  // extern "C"
