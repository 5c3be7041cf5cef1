// noalloc_api.hip -- fscc_zgemm_noalloc: the grouped complex GEMM of
// fscc_zgemm for callers that must not allocate device memory.  Its problem,
// tile and split-K reduction tables and the split-K partial sums live in one
// static device array (`scratch`) instead of buffers allocated per call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.hpp"

namespace {

// Largest plan the entry point takes: tables plus split-K partial sums.
constexpr size_t kScratchBytes = FSCC_NOALLOC_SCRATCH_BYTES;

// One copy per GPU the library runs on, held until the process ends.  Host
// code never uses this name as a device address: it takes the per-device
// address returned by hipGetSymbolAddress (scratch_address below).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, looked up once per device with
// that device current (the previous current device is restored).
hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of the scratch a plan needs: the three tables and the partial sums.
size_t plan_bytes(const GemmHost& h) {
    return align256(h.pr.size() * sizeof(ZProb)) + align256(h.tl.size() * sizeof(ZTile)) +
           align256(h.rd.size() * sizeof(ZRed)) + (size_t)h.work_elems * sizeof(double2);
}

}  // namespace

extern "C" {

fscc_status fscc_zgemm_noalloc(int cfg, int bk, int tA, int tB, int cA, int cB, int M, int N, int K,
                               const fscc_c128* A, int lda, const fscc_c128* B, int ldb, fscc_c128* C, int ldc,
                               double alpha_re, double alpha_im, int beta, int allow_split, void* hip_stream) {
    const bool m3 = cfg >= 0 && (cfg & FSCC_CFG_3M);
    const bool db = cfg >= 0 && (cfg & FSCC_CFG_DB);
    const bool dl = cfg >= 0 && (cfg & FSCC_CFG_DL);
    if (cfg >= 0) cfg &= ~(FSCC_CFG_3M | FSCC_CFG_DB | FSCC_CFG_DL);
    if (M < 0 || N < 0 || K < 0 || cfg >= ZCFG_N || (bk != 16 && bk != 32) ||
        (db && (dl || bk != 16 || !zcfg_has_db(cfg))) || (dl && (bk != 16 || !zcfg_has_dl(cfg))))
        return free_call_fail(FSCC_EINVAL, "fscc_zgemm_noalloc: bad size, tile id or K depth");
    if ((M > 0 && N > 0) && (!C || (K > 0 && (!A || !B))))
        return free_call_fail(FSCC_EINVAL, "fscc_zgemm_noalloc: null operand");
    if (ldc < N || lda < (tA ? M : K) || ldb < (tB ? K : N))
        return free_call_fail(FSCC_EINVAL, "fscc_zgemm_noalloc: leading dimension too small");
    hipStream_t st = (hipStream_t)hip_stream;
    try {
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
        if (cfg >= 0 && !cfg_ok(o, cfg)) return free_call_fail(FSCC_EINVAL, "fscc_zgemm_noalloc: shape does not fit the tile form");
        const int form = cfg < 0 ? pick_cfg(o) : cfg;
        GemmHost h;
        plan_gemm_host(false, o, form, bk, allow_split != 0, cfg < 0 || m3, h);
        // an optional K split whose partial sums do not fit runs unsplit
        // (same kernel, one K chunk per tile)
        if (plan_bytes(h) > kScratchBytes && h.g.split && allow_split)
            plan_gemm_host(false, o, form, bk, false, cfg < 0 || m3, h);
        if (plan_bytes(h) > kScratchBytes)
            return free_call_fail(FSCC_EINVAL, "fscc_zgemm_noalloc: plan needs " + std::to_string(plan_bytes(h)) +
                                                   " bytes of scratch, more than the static " +
                                                   std::to_string(kScratchBytes));
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        if (st) hip_check(hipStreamGetDevice(st, &dev), "hipStreamGetDevice");
        if (dev < 0 || dev >= kMaxDevices) return free_call_fail(FSCC_EINVAL, "fscc_zgemm_noalloc: device id out of range");
        void* base = nullptr;
        hip_check(scratch_address(dev, &base), "hipGetSymbolAddress(scratch)");
        unsigned char* p = (unsigned char*)base;
        GemmDev g = h.g;
        g.lds = dl ? LDS_DIRECT : db ? LDS_DOUBLE : LDS_STAGED;
        g.probs = (ZProb*)p;
        p += align256(h.pr.size() * sizeof(ZProb));
        g.tiles = (ZTile*)p;
        p += align256(h.tl.size() * sizeof(ZTile));
        g.reds = (ZRed*)p;
        p += align256(h.rd.size() * sizeof(ZRed));
        g.work = g.split ? (double2*)p : nullptr;
        // the tables are copied in on the stream; every partial-sum element is
        // written by the GEMM before the reduction reads it, so nothing is cleared
        if (!h.pr.empty())
            hip_check(hipMemcpyAsync(g.probs, h.pr.data(), h.pr.size() * sizeof(ZProb), hipMemcpyHostToDevice, st), "probs");
        if (!h.tl.empty())
            hip_check(hipMemcpyAsync(g.tiles, h.tl.data(), h.tl.size() * sizeof(ZTile), hipMemcpyHostToDevice, st), "tiles");
        if (!h.rd.empty())
            hip_check(hipMemcpyAsync(g.reds, h.rd.data(), h.rd.size() * sizeof(ZRed), hipMemcpyHostToDevice, st), "reds");
        hipError_t e = hipSuccess;
        if (g.ntiles > 0) {
            if (!g.split) {
                e = launch_zgemm(g.cfg, g.bk, o.tA, o.tB, (const double2*)A, (const double2*)B, (double2*)C, g.probs,
                                 g.tiles, g.ntiles, alpha_re, alpha_im, o.beta, o.cA, o.cB, st, 0, nullptr, g.maxM, g.m3, g.lds);
            } else {
                e = launch_zgemm(g.cfg, g.bk, o.tA, o.tB, (const double2*)A, (const double2*)B, g.work, g.probs, g.tiles,
                                 g.ntiles, 1.0, 0.0, 0, o.cA, o.cB, st, 0, nullptr, g.maxM, g.m3, g.lds);
                if (e == hipSuccess)
                    e = launch_splitk_reduce((double2*)C, g.work, g.reds, g.nred, g.maxMN, g.maxS, alpha_re, alpha_im,
                                             o.beta, st);
            }
        }
        hip_check(e, "zgemm_noalloc");
        // the host tables must outlive the copies; the scratch is reused by the next call
        hip_check(hipStreamSynchronize(st), "zgemm_noalloc sync");
        return FSCC_OK;
    } catch (const HipError& e) {
        return free_call_fail(FSCC_EHIP, e.what());
    } catch (const std::bad_alloc&) {
        return free_call_fail(FSCC_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return free_call_fail(FSCC_EINVAL, e.what());
    } catch (...) {
        return free_call_fail(FSCC_EINVAL, "unknown error");
    }
}

}  // extern "C"
