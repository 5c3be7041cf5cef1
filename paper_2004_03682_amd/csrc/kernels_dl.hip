// kernels_dl.hip -- grouped complex FP64 GEMM with direct-to-LDS loads.
//
// The same contraction as k_zgemm (one workgroup per output tile of a flat
// tile list, v_mfma_f64_16x16x4_f64, three- or four-product complex form),
// but the K slices travel from device memory straight into LDS
// (global_load_lds_dwordx4: one complex element per lane, no register
// staging) through a ring of S stages: slice k + S - 1 is in flight while
// the matrix cores work on slice k.  Without register staging the tiles need
// fewer registers and, with two stages, little LDS, so more workgroups share
// a CU and cover each other's waits.
//
// LDS layout of one stage: the A slice, then the B slice, complex elements
// (re, im interleaved, 16 bytes).  An operand whose K index is contiguous in
// device memory keeps rows of 16 elements with the columns XOR-swizzled by
// the row (element k of row r sits in column k ^ (r & 15)), so that the 16
// lanes reading one fragment column hit 16 different 16-byte bank groups;
// an operand whose M (or N) index is contiguous keeps K rows of BM (BN)
// elements and needs no swizzle.  Edge handling: rows past M (columns past
// N) and k past K load a clamped in-range element; garbage rows and columns
// only reach outputs that are not stored, and the A fragment elements of
// k past K are replaced by zero in the last slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace fscc {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kThreads = 256;
constexpr int kBK = 16;   // K depth of one stage

template <int N>
__device__ __forceinline__ void wait_vmem() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// this wave's LDS reads done, then the workgroup barrier; the memory clobber
// keeps the compiler from moving LDS accesses across it
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ void dma16(const double2* g, double2* l) {
    __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)l, 16, 0, 0);
}

typedef double dbl2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t lds_addr(const double2* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// The fragment reads of one 4-deep step: NF 16-byte LDS reads and the wait
// for them in one asm block.  Written out because the compiler, which cannot
// tell the stages apart, would otherwise make every LDS read wait for all
// direct-to-LDS loads in flight, including those of the next slice (the
// pipeline would drain every slice).  Their order against the loads and
// barriers is kept by the explicit waits and the memory clobbers.
template <int NF>
__device__ __forceinline__ void lds_frags(dbl2 (&v)[NF], const uint32_t (&a)[NF]) {
    static_assert(NF >= 2 && NF <= 5, "fragment count");
    if constexpr (NF == 2) {
        asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %3\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1])
                     : "v"(a[0]), "v"(a[1])
                     : "memory");
    } else if constexpr (NF == 3) {
        asm volatile("ds_read_b128 %0, %3\n\tds_read_b128 %1, %4\n\tds_read_b128 %2, %5\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2])
                     : "v"(a[0]), "v"(a[1]), "v"(a[2])
                     : "memory");
    } else if constexpr (NF == 4) {
        asm volatile("ds_read_b128 %0, %4\n\tds_read_b128 %1, %5\n\tds_read_b128 %2, %6\n\tds_read_b128 %3, %7\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])
                     : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3])
                     : "memory");
    } else {
        asm volatile("ds_read_b128 %0, %5\n\tds_read_b128 %1, %6\n\tds_read_b128 %2, %7\n\tds_read_b128 %3, %8\n\t"
                     "ds_read_b128 %4, %9\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4])
                     : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4])
                     : "memory");
    }
}

// Stage I of the ring as an LDS variable of its own; the ring is unrolled so
// that every stage is named at compile time (no run-time stage arithmetic in
// the load and fragment addresses).
template <int SE, int I>
__device__ __forceinline__ double2* lds_stage() {
    __shared__ double2 buf[SE];
    return buf;
}

// f(integral_constant<I>, kb + I) for I = 0..S-1 while kb + I < n
template <int I, int S, class F>
__device__ __forceinline__ void unroll_ring(F& f, int kb, int n) {
    if constexpr (I < S) {
        if (kb + I < n) {
            f(std::integral_constant<int, I>{}, kb + I);
            unroll_ring<I + 1, S>(f, kb, n);
        }
    }
}

template <int BM, int BN, int WM, int WN, int S, bool TA, bool TB, int ROLE, bool M3>
__global__ __launch_bounds__(256) void k_zgemm_dl(const double2* __restrict__ A, const double2* __restrict__ B,
                                                  double2* __restrict__ C, const ZProb* __restrict__ probs,
                                                  const ZTile* __restrict__ tiles, double ar, double ai, int beta,
                                                  int cA, int cB, const int* __restrict__ active) {
    constexpr int BK = kBK;
    constexpr int FM = BM / (16 * WM);
    constexpr int FN = BN / (16 * WN);
    constexpr int AE = BM * BK, BE = BN * BK, SE = AE + BE;   // elements per stage
    constexpr int AI = AE / kThreads, BI = BE / kThreads;     // loads per thread per slice
    static_assert(WM * WN == 4, "four waves");
    static_assert(FM >= 1 && FN >= 1, "tile too small");
    static_assert(AE % kThreads == 0 && BE % kThreads == 0, "whole load instructions");
    static_assert((S - 2) * (AI + BI) <= 63, "vmcnt range");
    static_assert(S >= 2 && S <= 4, "ring depth");

    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;   // whole workgroup: a converged system of a batch
    const ZProb pr = probs[tl.prob];
    const int M = pr.M, N = pr.N, K = pr.K;
    const double2* Ap = A + pr.a_off;
    const double2* Bp = B + pr.b_off;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int m0 = tl.m0, n0 = tl.n0;
    const double sA = cA ? -1.0 : 1.0;
    const double sB = cB ? -1.0 : 1.0;

    dbl4 accr[FM][FN], acci[FM][FN], accs[M3 ? FM : 1][M3 ? FN : 1];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            accr[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (M3) accs[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
        }

    // Per load instruction u of this thread: the LDS slot q = (4u + wave)*64 +
    // lane of the stage, and the device element it receives, written as
    // base[u] + min(k0 + kq[u], K - 1) * kstride.
    const double2* abase[AI];
    const double2* bbase[BI];
    int akq[AI], bkq[BI];
    const long long askk = TA ? pr.lda : 1, bskk = TB ? 1 : pr.ldb;
#pragma unroll
    for (int u = 0; u < AI; ++u) {
        const int q = (4 * u + wave) * 64 + lane;
        if (!TA) {   // rows of BK: (m, k) with the columns swizzled by the row
            const int r = q / BK, c = q % BK;
            const int m = min(m0 + r, M - 1);
            abase[u] = Ap + (long long)m * pr.lda;
            akq[u] = c ^ (r & 15);
        } else {     // K rows of BM
            const int kr = q / BM, c = q % BM;
            abase[u] = Ap + min(m0 + c, M - 1);
            akq[u] = kr;
        }
    }
#pragma unroll
    for (int u = 0; u < BI; ++u) {
        const int q = (4 * u + wave) * 64 + lane;
        if (TB) {    // rows of BK: (n, k), swizzled
            const int r = q / BK, c = q % BK;
            const int n = min(n0 + r, N - 1);
            bbase[u] = Bp + (long long)n * pr.ldb;
            bkq[u] = c ^ (r & 15);
        } else {     // K rows of BN
            const int kr = q / BN, c = q % BN;
            bbase[u] = Bp + min(n0 + c, N - 1);
            bkq[u] = kr;
        }
    }

    auto issue = [&](auto stage, int kt) {
        const int k0 = kt * BK;
        double2* st = lds_stage<SE, decltype(stage)::value>();
#pragma unroll
        for (int u = 0; u < AI; ++u)
            dma16(abase[u] + (long long)min(k0 + akq[u], K - 1) * askk, st + (4 * u + wave) * 64);
#pragma unroll
        for (int u = 0; u < BI; ++u)
            dma16(bbase[u] + (long long)min(k0 + bkq[u], K - 1) * bskk, st + AE + (4 * u + wave) * 64);
    };

    const int lr = lane & 15;        // row (A) / column (B) inside a 16-wide fragment
    const int lk = lane >> 4;        // k inside a 4-deep step
    const int wm0 = wm * FM * 16, wn0 = wn * FN * 16;
    const bool wave_live = m0 + wm0 < M && n0 + wn0 < N;

    // one slice of matrix-core work on stage s; krem < BK in the last slice
    // of a K that is not a multiple of BK
    constexpr int NF = FM + FN;
    auto compute = [&](auto stage, int krem) {
        const double2* As = lds_stage<SE, decltype(stage)::value>();
        const double2* Bs = As + AE;
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int k = ks * 4 + lk;
            uint32_t addr[NF];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int r = wm0 + i * 16 + lr;
                addr[i] = lds_addr(TA ? As + k * BM + r : As + r * BK + (k ^ (r & 15)));
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int c = wn0 + j * 16 + lr;
                addr[FM + j] = lds_addr(TB ? Bs + c * BK + (k ^ (c & 15)) : Bs + k * BN + c);
            }
            dbl2 v[NF];
            lds_frags<NF>(v, addr);
            // 0 for the k past K of a last slice (their clamped elements are
            // finite), else 1
            const double kf = k < krem ? 1.0 : 0.0;
            double a_r[FM], a_i[FM], b_r[FN], b_i[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                a_r[i] = kf * v[i].x;
                a_i[i] = (kf * sA) * v[i].y;
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                b_r[j] = v[FM + j].x;
                b_i[j] = sB * v[FM + j].y;
            }
            if constexpr (M3) {
                double a_s[FM], b_s[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) a_s[i] = a_r[i] + a_i[i];
#pragma unroll
                for (int j = 0; j < FN; ++j) b_s[j] = b_r[j] + b_i[j];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[i], b_r[j], accr[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i[i], b_i[j], acci[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        accs[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_s[i], b_s[j], accs[i][j], 0, 0, 0);
            } else {
                double a_n[FM];
#pragma unroll
                for (int i = 0; i < FM; ++i) a_n[i] = -a_i[i];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[i], b_r[j], accr[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[i], b_i[j], acci[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_n[i], b_i[j], accr[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i[i], b_r[j], acci[i][j], 0, 0, 0);
            }
        }
    };

    // Ring of S stages: slices 0..S-2 go out first; at slice kt this thread
    // waits until its own loads of slice kt have landed (the loads of the
    // S - 2 later slices may still be in flight), the barrier makes every
    // thread's loads visible and frees the stage read at kt - 1, which then
    // receives slice kt + S - 1.  Every thread issues the same number of
    // loads per slice, so the counts are exact.
    const int nk = K > 0 ? (K + BK - 1) / BK : 0;
    // Slices past the last one are issued as copies of the last slice (into
    // stages that are never read again), so that every step waits for the
    // same count; the ring drains before the epilogue.
    auto prologue = [&](auto stage, int) {
        if constexpr (decltype(stage)::value < S - 1) issue(stage, min((int)decltype(stage)::value, nk - 1));
    };
    if (nk > 0) unroll_ring<0, S>(prologue, 0, S);
    // slice kt lives in stage kt % S; the ring is unrolled by S so that
    // every stage index is a compile-time constant
    auto step = [&](auto stage, int kt) {
        constexpr int I = decltype(stage)::value;
        wait_vmem<(S - 2) * (AI + BI)>();
        lds_barrier();
        issue(std::integral_constant<int, (I + S - 1) % S>{}, min(kt + S - 1, nk - 1));
        if (wave_live) compute(stage, K - kt * BK);
    };
    for (int kb = 0; kb < nk; kb += S) unroll_ring<0, S>(step, kb, nk);
    wait_vmem<0>();

    // epilogue: accumulator element q of a lane is row 4*q + lane/16,
    // column lane%16 of the fragment
    double2* Cp = C + pr.c_off;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            int col = n0 + wn0 + j * 16 + lr;
            if (col >= N) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int row = m0 + wm0 + i * 16 + q * 4 + lk;
                if (row >= M) continue;
                double xr, xi;
                if constexpr (M3) {
                    xr = accr[i][j][q] - acci[i][j][q];
                    xi = accs[i][j][q] - accr[i][j][q] - acci[i][j][q];
                } else {
                    xr = accr[i][j][q];
                    xi = acci[i][j][q];
                }
                double2 out = make_double2(ar * xr - ai * xi, ar * xi + ai * xr);
                double2* c = Cp + (long long)row * pr.ldc + col;
                if (beta) {
                    double2 old = *c;
                    out.x += old.x;
                    out.y += old.y;
                }
                *c = out;
            }
        }
}

template <int BM, int BN, int WM, int WN, int S, bool M3>
hipError_t launch_dl_cfg(bool tA, bool tB, const double2* A, const double2* B, double2* C, const ZProb* probs,
                         const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA, int cB,
                         hipStream_t st, int role, const int* active) {
    dim3 grid(ntiles), block(kThreads);
    if (!tA && !tB) {
        if (role == 2) k_zgemm_dl<BM, BN, WM, WN, S, false, false, 2, M3><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else k_zgemm_dl<BM, BN, WM, WN, S, false, false, 0, M3><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    } else if (!tA && tB) {
        if (role == 1) k_zgemm_dl<BM, BN, WM, WN, S, false, true, 1, M3><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else k_zgemm_dl<BM, BN, WM, WN, S, false, true, 0, M3><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    } else if (tA && !tB) {
        k_zgemm_dl<BM, BN, WM, WN, S, true, false, 0, M3><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    } else {
        k_zgemm_dl<BM, BN, WM, WN, S, true, true, 0, M3><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    }
    return hipGetLastError();
}

template <bool M3>
hipError_t launch_dl_m3(int cfg, bool tA, bool tB, const double2* A, const double2* B, double2* C, const ZProb* probs,
                        const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA, int cB,
                        hipStream_t st, int role, const int* active) {
    // two stages: three workgroups of the 32- and 16-row tiles per CU (at most
    // 48 KB of LDS each), two of the 64x64 tiles; measured faster than three
    // stages at two workgroups per CU (more waves to cover each other's LDS
    // and barrier waits)
    switch (cfg) {
        case ZCFG_32x32: return launch_dl_cfg<32, 32, 2, 2, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x16: return launch_dl_cfg<64, 16, 4, 1, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_16x64: return launch_dl_cfg<16, 64, 1, 4, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_32x64: return launch_dl_cfg<32, 64, 2, 2, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x32: return launch_dl_cfg<64, 32, 2, 2, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x32R: return launch_dl_cfg<64, 32, 4, 1, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x64: return launch_dl_cfg<64, 64, 2, 2, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x64R: return launch_dl_cfg<64, 64, 4, 1, 2, M3>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        default: return hipErrorInvalidValue;
    }
}


// ---------------------------------------------------------------------------
// Real form (real-arithmetic contexts): the same ring with one double per LDS
// slot.  A double travels as two 4-byte direct-to-LDS loads of neighbouring
// lanes (global_load_lds_dword; 4-byte alignment is all a real operand
// guarantees), so one wave instruction moves 32 elements.  Rows of an operand
// whose K index is contiguous are XOR-swizzled as in the complex form (the 16
// lanes of an 8-byte fragment column read 16 different bank pairs); one real
// MFMA chain per fragment.

__device__ __forceinline__ void dma4(const void* g, double* l) {
    __builtin_amdgcn_global_load_lds(g, (lds_void*)l, 4, 0, 0);
}

template <int SE, int I>
__device__ __forceinline__ double* lds_stage_d() {
    __shared__ double buf[SE];
    return buf;
}

__device__ __forceinline__ uint32_t lds_addr_d(const double* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// NF 8-byte LDS reads and their wait in one asm block (see lds_frags)
#define DSR64(o, i) "ds_read_b64 %" #o ", %" #i "\n\t"
template <int NF>
__device__ __forceinline__ void lds_frags64(double (&v)[NF], const uint32_t (&a)[NF]) {
    static_assert(NF >= 2 && NF <= 5, "fragment count");
    if constexpr (NF == 2) {
        asm volatile(DSR64(0, 2) DSR64(1, 3) "s_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1])
                     : "v"(a[0]), "v"(a[1])
                     : "memory");
    } else if constexpr (NF == 3) {
        asm volatile(DSR64(0, 3) DSR64(1, 4) DSR64(2, 5) "s_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2])
                     : "v"(a[0]), "v"(a[1]), "v"(a[2])
                     : "memory");
    } else if constexpr (NF == 4) {
        asm volatile(DSR64(0, 4) DSR64(1, 5) DSR64(2, 6) DSR64(3, 7) "s_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])
                     : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3])
                     : "memory");
    } else {
        asm volatile(DSR64(0, 5) DSR64(1, 6) DSR64(2, 7) DSR64(3, 8) DSR64(4, 9) "s_waitcnt lgkmcnt(0)"
                     : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4])
                     : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4])
                     : "memory");
    }
}
#undef DSR64

template <int BM, int BN, int WM, int WN, int S, bool TA, bool TB, int ROLE>
__global__ __launch_bounds__(256) void k_dgemm_dl(const double* __restrict__ A, const double* __restrict__ B,
                                                  double* __restrict__ C, const ZProb* __restrict__ probs,
                                                  const ZTile* __restrict__ tiles, double alpha, int beta,
                                                  const int* __restrict__ active) {
    constexpr int BK = kBK;
    constexpr int FM = BM / (16 * WM);
    constexpr int FN = BN / (16 * WN);
    constexpr int AE = BM * BK, BE = BN * BK, SE = AE + BE;   // doubles per stage
    constexpr int AI = AE / (4 * 32), BI = BE / (4 * 32);     // loads per thread per slice (4 waves x 32 doubles)
    static_assert(WM * WN == 4, "four waves");
    static_assert(FM >= 1 && FN >= 1, "tile too small");
    static_assert(AE % 128 == 0 && BE % 128 == 0, "whole load instructions");
    static_assert((S - 2) * (AI + BI) <= 63, "vmcnt range");
    static_assert(S >= 2 && S <= 4, "ring depth");

    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;
    const ZProb pr = probs[tl.prob];
    const int M = pr.M, N = pr.N, K = pr.K;
    const double* Ap = A + pr.a_off;
    const double* Bp = B + pr.b_off;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int m0 = tl.m0, n0 = tl.n0;

    dbl4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    // load instruction u of this thread: element slot q = (4u + wave)*32 +
    // lane/2 of the stage, word lane&1 of that double
    const int word = lane & 1;
    const double* abase[AI];
    const double* bbase[BI];
    int akq[AI], bkq[BI];
    const long long askk = TA ? pr.lda : 1, bskk = TB ? 1 : pr.ldb;
#pragma unroll
    for (int u = 0; u < AI; ++u) {
        const int q = (4 * u + wave) * 32 + (lane >> 1);
        if (!TA) {
            const int r = q / BK, c = q % BK;
            abase[u] = Ap + (long long)min(m0 + r, M - 1) * pr.lda;
            akq[u] = c ^ (r & 15);
        } else {
            const int kr = q / BM, c = q % BM;
            abase[u] = Ap + min(m0 + c, M - 1);
            akq[u] = kr;
        }
    }
#pragma unroll
    for (int u = 0; u < BI; ++u) {
        const int q = (4 * u + wave) * 32 + (lane >> 1);
        if (TB) {
            const int r = q / BK, c = q % BK;
            bbase[u] = Bp + (long long)min(n0 + r, N - 1) * pr.ldb;
            bkq[u] = c ^ (r & 15);
        } else {
            const int kr = q / BN, c = q % BN;
            bbase[u] = Bp + min(n0 + c, N - 1);
            bkq[u] = kr;
        }
    }

    auto issue = [&](auto stage, int kt) {
        const int k0 = kt * BK;
        double* st = lds_stage_d<SE, decltype(stage)::value>();
#pragma unroll
        for (int u = 0; u < AI; ++u)
            dma4((const char*)(abase[u] + (long long)min(k0 + akq[u], K - 1) * askk) + 4 * word,
                 st + (4 * u + wave) * 32);
#pragma unroll
        for (int u = 0; u < BI; ++u)
            dma4((const char*)(bbase[u] + (long long)min(k0 + bkq[u], K - 1) * bskk) + 4 * word,
                 st + AE + (4 * u + wave) * 32);
    };

    const int lr = lane & 15;
    const int lk = lane >> 4;
    const int wm0 = wm * FM * 16, wn0 = wn * FN * 16;
    const bool wave_live = m0 + wm0 < M && n0 + wn0 < N;

    constexpr int NF = FM + FN;
    auto compute = [&](auto stage, int krem) {
        const double* As = lds_stage_d<SE, decltype(stage)::value>();
        const double* Bs = As + AE;
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int k = ks * 4 + lk;
            uint32_t addr[NF];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int r = wm0 + i * 16 + lr;
                addr[i] = lds_addr_d(TA ? As + k * BM + r : As + r * BK + (k ^ (r & 15)));
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int c = wn0 + j * 16 + lr;
                addr[FM + j] = lds_addr_d(TB ? Bs + c * BK + (k ^ (c & 15)) : Bs + k * BN + c);
            }
            double v[NF];
            lds_frags64<NF>(v, addr);
            const double kf = k < krem ? 1.0 : 0.0;   // zero for k past K (clamped, finite elements)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(kf * v[i], v[FM + j], acc[i][j], 0, 0, 0);
        }
    };

    const int nk = K > 0 ? (K + BK - 1) / BK : 0;
    auto prologue = [&](auto stage, int) {
        if constexpr (decltype(stage)::value < S - 1) issue(stage, min((int)decltype(stage)::value, nk - 1));
    };
    if (nk > 0) unroll_ring<0, S>(prologue, 0, S);
    auto step = [&](auto stage, int kt) {
        constexpr int I = decltype(stage)::value;
        wait_vmem<(S - 2) * (AI + BI)>();
        lds_barrier();
        issue(std::integral_constant<int, (I + S - 1) % S>{}, min(kt + S - 1, nk - 1));
        if (wave_live) compute(stage, K - kt * BK);
    };
    for (int kb = 0; kb < nk; kb += S) unroll_ring<0, S>(step, kb, nk);
    wait_vmem<0>();

    double* Cp = C + pr.c_off;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn0 + j * 16 + lr;
            if (col >= N) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm0 + i * 16 + q * 4 + lk;
                if (row >= M) continue;
                double out = alpha * acc[i][j][q];
                double* c = Cp + (long long)row * pr.ldc + col;
                if (beta) out += *c;
                *c = out;
            }
        }
}

template <int BM, int BN, int WM, int WN, int S>
hipError_t launch_ddl_cfg(bool tA, bool tB, const double* A, const double* B, double* C, const ZProb* probs,
                          const ZTile* tiles, int ntiles, double alpha, int beta, hipStream_t st, int role,
                          const int* active) {
    dim3 grid(ntiles), block(kThreads);
    if (!tA && !tB) {
        if (role == 2) k_dgemm_dl<BM, BN, WM, WN, S, false, false, 2><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        else k_dgemm_dl<BM, BN, WM, WN, S, false, false, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    } else if (!tA && tB) {
        if (role == 1) k_dgemm_dl<BM, BN, WM, WN, S, false, true, 1><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        else k_dgemm_dl<BM, BN, WM, WN, S, false, true, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    } else if (tA && !tB) {
        k_dgemm_dl<BM, BN, WM, WN, S, true, false, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    } else {
        k_dgemm_dl<BM, BN, WM, WN, S, true, true, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    }
    return hipGetLastError();
}

}  // namespace

bool zcfg_has_dl(int cfg) {
    return cfg == ZCFG_32x32 || cfg == ZCFG_64x16 || cfg == ZCFG_16x64 || cfg == ZCFG_32x64 || cfg == ZCFG_64x32 ||
           cfg == ZCFG_64x32R || cfg == ZCFG_64x64 || cfg == ZCFG_64x64R;
}

hipError_t launch_zgemm_dl(int cfg, bool tA, bool tB, const double2* A, const double2* B, double2* C,
                           const ZProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA,
                           int cB, hipStream_t st, int role, const int* active, bool m3) {
    if (ntiles <= 0) return hipSuccess;
    return m3 ? launch_dl_m3<true>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active)
              : launch_dl_m3<false>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
}

}  // namespace fscc

namespace fscc {

hipError_t launch_dgemm_dl(int cfg, bool tA, bool tB, const double* A, const double* B, double* C,
                           const ZProb* probs, const ZTile* tiles, int ntiles, double alpha, int beta, hipStream_t st,
                           int role, const int* active) {
    if (ntiles <= 0) return hipSuccess;
    switch (cfg) {
        case ZCFG_32x32: return launch_ddl_cfg<32, 32, 2, 2, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x16: return launch_ddl_cfg<64, 16, 4, 1, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_16x64: return launch_ddl_cfg<16, 64, 1, 4, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_32x64: return launch_ddl_cfg<32, 64, 2, 2, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x32: return launch_ddl_cfg<64, 32, 2, 2, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x32R: return launch_ddl_cfg<64, 32, 4, 1, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x64: return launch_ddl_cfg<64, 64, 2, 2, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x64R: return launch_ddl_cfg<64, 64, 4, 1, 2>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fscc
