// kernels.hip -- gfx950 kernels of the FS-RCCSD hot path.
//
//  * k_zgemm   grouped complex GEMM on FP64 matrix cores
//              (v_mfma_f64_16x16x4_f64), LDS-staged tiles, one workgroup per
//              output tile of a flat tile list covering every (problem = pair
//              irrep block) of one contraction.  Complex products use four
//              real MFMA chains: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
//  * k_gather  reorders / antisymmetrisers of the TTGT scheme: a gather through
//              precomputed 32-bit maps (offset + sign bit), up to four terms,
//              optionally multiplied by a second gathered operand (t1 x t1).
//  * elementwise / reduction kernels of the Jacobi + DIIS update and the energy.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace fscc {

typedef double dbl4 __attribute__((ext_vector_type(4)));

static constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// grouped complex GEMM

// ROLE only distinguishes kernel symbols in profiles (0 generic, 1 pp-ladder, 2 ring).
// M3: the complex product with three real matrix products, P1 = Ar Br,
// P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), Re = P1 - P2, Im = P3 - P1 - P2 (the
// sums formed in registers from the LDS fragments); otherwise four products
// (Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br).
// Waves with a single 16x16 fragment on 16-deep slices fit in 96 registers:
// they ask for five waves per SIMD (more global-load latency hidden); the
// larger fragment grids keep three, which they reach without spills.
constexpr int zgemm_min_waves(int BM, int BN, int BK) { return (BK == 16 && BM * BN == 1024) ? 5 : 3; }

// DB: two LDS buffers per operand (double buffering): slice k+1 is stored
// into one buffer while the matrix cores work on slice k from the other, with
// one barrier per slice (otherwise one buffer pair and two barriers).
template <int BM, int BN, int WM, int WN, int BK, bool TA, bool TB, int ROLE, bool M3, bool DB>
__global__ __launch_bounds__(256, zgemm_min_waves(BM, BN, BK)) void k_zgemm(const double2* __restrict__ A, const double2* __restrict__ B,
                                               double2* __restrict__ C, const ZProb* __restrict__ probs,
                                               const ZTile* __restrict__ tiles, double ar, double ai, int beta,
                                               int cA, int cB, const int* __restrict__ active) {
    // odd row padding: the transposed slice stores (4 k rows x 16 columns per
    // wave) and the fragment reads (4 k rows x 16 columns) spread over the
    // LDS banks
    constexpr int PAD = 1;
    constexpr int FM = BM / (16 * WM);
    constexpr int FN = BN / (16 * WN);
    constexpr int KS_UNROLL = FM * FN >= 4 ? 1 : BK / 4;   // 4-deep steps unrolled per slice
    static_assert(WM * WN == 4, "four waves");
    static_assert(FM >= 1 && FN >= 1, "tile too small");
    __shared__ double As[DB ? 4 : 2][BK][BM + PAD];
    __shared__ double Bs[DB ? 4 : 2][BK][BN + PAD];

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

    // 4M: accr = Re, acci = Im.  3M: accr = P1, acci = P2, accs = P3.
    dbl4 accr[FM][FN], acci[FM][FN], accs[M3 ? FM : 1][M3 ? FN : 1];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            accr[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (M3) accs[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
        }

    // register staging of one BK slice: vectors of 4 consecutive complex along
    // the contiguous dimension of each operand
    constexpr int AV = BM * BK / 4;   // vec4 per A slice
    constexpr int BV = BN * BK / 4;
    constexpr int AVT = (AV + kThreads - 1) / kThreads;
    constexpr int BVT = (BV + kThreads - 1) / kThreads;
    double2 ra[AVT][4], rb[BVT][4];

    auto load_slice = [&](int k0) {
#pragma unroll
        for (int u = 0; u < AVT; ++u) {
            int v = tid + u * kThreads;
#pragma unroll
            for (int e = 0; e < 4; ++e) ra[u][e] = make_double2(0.0, 0.0);
            if (v < AV) {
                if (!TA) {   // A row-major [M][lda], k contiguous
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
                    int m = m0 + r;
                    if (m < M) {
                        const double2* p = Ap + (long long)m * pr.lda + k0 + kk;
                        if (k0 + kk + 3 < K) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) ra[u][e] = p[e];
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (k0 + kk + e < K) ra[u][e] = p[e];
                        }
                    }
                } else {     // A stored [K][lda], m contiguous
                    int kr = v / (BM / 4), mm = (v % (BM / 4)) * 4;
                    int k = k0 + kr;
                    if (k < K) {
                        const double2* p = Ap + (long long)k * pr.lda + m0 + mm;
                        if (m0 + mm + 3 < M) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) ra[u][e] = p[e];
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (m0 + mm + e < M) ra[u][e] = p[e];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < BVT; ++u) {
            int v = tid + u * kThreads;
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[u][e] = make_double2(0.0, 0.0);
            if (v < BV) {
                if (!TB) {   // B row-major [K][ldb], n contiguous
                    int kr = v / (BN / 4), nn = (v % (BN / 4)) * 4;
                    int k = k0 + kr;
                    if (k < K) {
                        const double2* p = Bp + (long long)k * pr.ldb + n0 + nn;
                        if (n0 + nn + 3 < N) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) rb[u][e] = p[e];
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (n0 + nn + e < N) rb[u][e] = p[e];
                        }
                    }
                } else {     // B stored [N][ldb], k contiguous
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
                    int n = n0 + r;
                    if (n < N) {
                        const double2* p = Bp + (long long)n * pr.ldb + k0 + kk;
                        if (k0 + kk + 3 < K) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) rb[u][e] = p[e];
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (k0 + kk + e < K) rb[u][e] = p[e];
                        }
                    }
                }
            }
        }
    };

    auto store_slice = [&](int buf) {
#pragma unroll
        for (int u = 0; u < AVT; ++u) {
            int v = tid + u * kThreads;
            if (v < AV) {
                if (!TA) {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        As[buf][kk + e][r] = ra[u][e].x;
                    }
                } else {
                    int kr = v / (BM / 4), mm = (v % (BM / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) As[buf][kr][mm + e] = ra[u][e].x;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < BVT; ++u) {
            int v = tid + u * kThreads;
            if (v < BV) {
                if (!TB) {
                    int kr = v / (BN / 4), nn = (v % (BN / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) Bs[buf][kr][nn + e] = rb[u][e].x;
                } else {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) Bs[buf][kk + e][r] = rb[u][e].x;
                }
            }
        }
    };
    // imaginary planes share the same LDS arrays in a second pass (see below)
    auto store_slice_im = [&](int buf) {
#pragma unroll
        for (int u = 0; u < AVT; ++u) {
            int v = tid + u * kThreads;
            if (v < AV) {
                if (!TA) {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) As[buf][kk + e][r] = sA * ra[u][e].y;
                } else {
                    int kr = v / (BM / 4), mm = (v % (BM / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) As[buf][kr][mm + e] = sA * ra[u][e].y;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < BVT; ++u) {
            int v = tid + u * kThreads;
            if (v < BV) {
                if (!TB) {
                    int kr = v / (BN / 4), nn = (v % (BN / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) Bs[buf][kr][nn + e] = sB * rb[u][e].y;
                } else {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) Bs[buf][kk + e][r] = sB * rb[u][e].y;
                }
            }
        }
    };

    const int lr = lane & 15;        // row (A) / column (B) inside a 16-wide fragment
    const int lk = lane >> 4;        // k inside a 4-deep step
    const int wm0 = wm * FM * 16, wn0 = wn * FN * 16;
    // a wave whose whole fragment block lies outside the problem (edge tiles)
    // issues no MFMA
    const bool wave_live = m0 + wm0 < M && n0 + wn0 < N;

    // one K slice of matrix-core work on the LDS planes As/Bs[pb] (real) and
    // [pb + 1] (imaginary)
    auto compute = [&](int pb) {
        // large fragment grids: one 4-deep step at a time keeps the register
        // count (and so the occupancy) of the 64x64 tile in check
#pragma unroll KS_UNROLL
        for (int ks = 0; ks < BK / 4; ++ks) {
            if (!wave_live) break;
            double a_r[FM], a_i[FM], a_n[FM], b_r[FN], b_i[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                a_r[i] = As[pb][ks * 4 + lk][wm0 + i * 16 + lr];
                a_i[i] = As[pb + 1][ks * 4 + lk][wm0 + i * 16 + lr];
                a_n[i] = -a_i[i];
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                b_r[j] = Bs[pb][ks * 4 + lk][wn0 + j * 16 + lr];
                b_i[j] = Bs[pb + 1][ks * 4 + lk][wn0 + j * 16 + lr];
            }
            if constexpr (M3) {
                double a_s[FM], b_s[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) a_s[i] = a_r[i] + a_i[i];
#pragma unroll
                for (int j = 0; j < FN; ++j) b_s[j] = b_r[j] + b_i[j];
                // three passes over the fragment grid, one per real product
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
                // four passes over the fragment grid so that consecutive MFMAs
                // update different accumulators
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

    if constexpr (!DB) {
        // LDS buffer 0 holds the real planes, buffer 1 the imaginary planes; the
        // global loads of slice k+1 are in flight while slice k is multiplied
        if (K > 0) load_slice(0);
        for (int k0 = 0; k0 < K; k0 += BK) {
            __syncthreads();
            store_slice(0);
            store_slice_im(1);
            __syncthreads();
            if (k0 + BK < K) load_slice(k0 + BK);
            compute(0);
        }
    } else {
        // planes 0/1 and 2/3 alternate: slice k+1 is written into one pair
        // (its global loads were issued one slice earlier) and the loads of
        // slice k+2 are issued before the matrix cores start on slice k in the
        // other pair; the barrier after the slice separates the reads of a
        // pair from its next writes
        if (K > 0) {
            load_slice(0);
            store_slice(0);
            store_slice_im(1);
            if (BK < K) load_slice(BK);
        }
        __syncthreads();
        int cur = 0;
        for (int k0 = 0; k0 < K; k0 += BK) {
            if (k0 + BK < K) {
                store_slice(2 * (cur ^ 1));
                store_slice_im(2 * (cur ^ 1) + 1);
                if (k0 + 2 * BK < K) load_slice(k0 + 2 * BK);
            }
            compute(2 * cur);
            __syncthreads();
            cur ^= 1;
        }
    }

    // epilogue: for the FP64 16x16x4 MFMA, accumulator element q of a lane is
    // row 4*q + lane/16, column lane%16 of the fragment
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

// Skinny products (a small M or N, or a short K): each workgroup takes a
// block of at most 64 x 32 outputs of one K chunk, stages the A rows and B
// columns of a K slice in LDS, and every thread accumulates up to 8 outputs on
// the vector ALUs (small blocks: several threads per output, summed in a
// fixed order), so no MFMA work is wasted on padding.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_zskinny(const double2* __restrict__ A, const double2* __restrict__ B,
                                                 double2* __restrict__ C, const ZProb* __restrict__ probs,
                                                 const ZTile* __restrict__ tiles, double ar, double ai, int beta,
                                                 int cA, int cB, const int* __restrict__ active) {
    constexpr int LDS = 4096;                       // staged complex elements (64 KB)
    constexpr int MAXO = ZSKINNY_MAX_MN / kThreads;  // outputs per thread
    __shared__ double2 sm[LDS];
    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;
    const ZProb pr = probs[tl.prob];
    // this workgroup's block: rows m0.., columns n0.. of at most ZSKINNY_BM x ZSKINNY_BN
    const int M = min(ZSKINNY_BM, pr.M - tl.m0), N = min(ZSKINNY_BN, pr.N - tl.n0), K = pr.K, MN = M * N;
    const int tid = threadIdx.x;
    // K slice: the largest power of two <= min(256, LDS / (M + N))
    int kss = 0;
    while ((2 << kss) <= LDS / max(1, M + N) && (2 << kss) <= 256) ++kss;
    const int KS = 1 << kss;
    // G threads per output when the block is small: thread (o, g) sums k = g, g+G, ...
    const int G = (MN > 0 && MN <= kThreads / 2) ? kThreads / MN : 1;
    double2* As = sm;            // [M][KS]
    double2* Bs = sm + M * KS;   // [KS][N]
    const double sA = cA ? -1.0 : 1.0, sB = cB ? -1.0 : 1.0;
    const double2* Ap = A + pr.a_off + (TA ? (long long)tl.m0 : (long long)tl.m0 * pr.lda);
    const double2* Bp = B + pr.b_off + (TB ? (long long)tl.n0 * pr.ldb : (long long)tl.n0);
    double accr[MAXO], acci[MAXO];
#pragma unroll
    for (int j = 0; j < MAXO; ++j) accr[j] = acci[j] = 0.0;
    const int nA = M * KS, nAB = (M + N) * KS;   // staged elements (<= LDS)
    for (int k0 = 0; k0 < K; k0 += KS) {
        const int kl = min(KS, K - k0);
        __syncthreads();
        // batches of 4 elements per thread: the 4 global loads are in flight together
        for (int base = 0; base < nAB; base += 4 * kThreads) {
            double2 v[4];
            int dst[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = base + tid + j * kThreads;
                v[j] = make_double2(0.0, 0.0);
                dst[j] = -1;
                if (e < nA) {
                    int m, k;
                    if (!TA) {
                        m = e >> kss;
                        k = e & (KS - 1);
                    } else {
                        k = e / M;
                        m = e - k * M;
                    }
                    if (k < kl) v[j] = TA ? Ap[(long long)(k0 + k) * pr.lda + m] : Ap[(long long)m * pr.lda + k0 + k];
                    v[j].y *= sA;
                    dst[j] = m * KS + k;
                } else if (e < nAB) {
                    const int f = e - nA;
                    int n, k;
                    if (!TB) {
                        k = f / N;
                        n = f - k * N;
                    } else {
                        n = f >> kss;
                        k = f & (KS - 1);
                    }
                    if (k < kl) v[j] = TB ? Bp[(long long)n * pr.ldb + k0 + k] : Bp[(long long)(k0 + k) * pr.ldb + n];
                    v[j].y *= sB;
                    dst[j] = nA + k * N + n;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (dst[j] >= 0) sm[dst[j]] = v[j];
        }
        __syncthreads();
        if (G > 1) {
            const int o = tid % MN, g = tid / MN;
            if (g < G) {
                const int m = o / N, n = o % N;
                double sr = accr[0], si = acci[0];
                const double2* a = As + m * KS;
#pragma unroll 2
                for (int k = g; k < kl; k += G) {
                    const double2 x = a[k], y = Bs[k * N + n];
                    sr += x.x * y.x - x.y * y.y;
                    si += x.x * y.y + x.y * y.x;
                }
                accr[0] = sr;
                acci[0] = si;
            }
        } else {
#pragma unroll
            for (int j = 0; j < MAXO; ++j) {
                const int o = tid + j * kThreads;
                if (o < MN) {
                    const int m = o / N, n = o % N;
                    double sr = accr[j], si = acci[j];
                    const double2* a = As + m * KS;
#pragma unroll 2
                    for (int k = 0; k < kl; ++k) {
                        const double2 x = a[k], y = Bs[k * N + n];
                        sr += x.x * y.x - x.y * y.y;
                        si += x.x * y.y + x.y * y.x;
                    }
                    accr[j] = sr;
                    acci[j] = si;
                }
            }
        }
    }
    if (G > 1) {   // combine the G partial sums of each output (fixed order)
        __syncthreads();
        const int o = tid % MN, g = tid / MN;
        if (g < G) sm[g * MN + o] = make_double2(accr[0], acci[0]);
        __syncthreads();
        if (tid < MN) {
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < G; ++q) {
                sr += sm[q * MN + tid].x;
                si += sm[q * MN + tid].y;
            }
            accr[0] = sr;
            acci[0] = si;
        }
    }
    double2* Cp = C + pr.c_off + (long long)tl.m0 * pr.ldc + tl.n0;
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
        const int o = tid + j * kThreads;
        if (o < MN && (G == 1 || j == 0)) {
            const int m = o / N, n = o % N;
            double2 out = make_double2(ar * accr[j] - ai * acci[j], ar * acci[j] + ai * accr[j]);
            double2* c = Cp + (long long)m * pr.ldc + n;
            if (beta) {
                const double2 old = *c;
                out.x += old.x;
                out.y += old.y;
            }
            *c = out;
        }
    }
}

// Tall products (many rows, K <= ZTALL_MAX_K, K*N <= ZTALL_MAX_KN, A stored
// with k contiguous): B is staged in LDS once per workgroup and every thread
// streams one row of A with eight independent loads in flight, so the large
// operand is read once at full width and nothing is padded to a 16-wide
// matrix-core fragment.
template <bool TB>
__global__ __launch_bounds__(256) void k_ztall(const double2* __restrict__ A, const double2* __restrict__ B,
                                               double2* __restrict__ C, const ZProb* __restrict__ probs,
                                               const ZTile* __restrict__ tiles, double ar, double ai, int beta,
                                               int cA, int cB, const int* __restrict__ active) {
    __shared__ double2 Bs[ZTALL_MAX_KN];   // [k][n]
    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;
    const ZProb pr = probs[tl.prob];
    const int N = pr.N, K = pr.K;
    const double sA = cA ? -1.0 : 1.0, sB = cB ? -1.0 : 1.0;
    const double2* Bp = B + pr.b_off;
    for (int e = threadIdx.x; e < K * N; e += kThreads) {
        const int k = e / N, n = e - k * N;
        double2 v = TB ? Bp[(long long)n * pr.ldb + k] : Bp[(long long)k * pr.ldb + n];
        v.y *= sB;
        Bs[e] = v;
    }
    __syncthreads();
    const int m = tl.m0 + (int)threadIdx.x;
    if (m >= pr.M) return;
    const double2* a = A + pr.a_off + (long long)m * pr.lda;
    double2* c = C + pr.c_off + (long long)m * pr.ldc;
    for (int n0 = 0; n0 < N; n0 += 8) {
        double xr[8], xi[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) xr[q] = xi[q] = 0.0;
        for (int k0 = 0; k0 < K; k0 += 8) {
            double2 av[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) av[j] = k0 + j < K ? a[k0 + j] : make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (k0 + j < K) {
                    const double pr_ = av[j].x, pi_ = sA * av[j].y;
                    const double2* b = Bs + (k0 + j) * N + n0;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (n0 + q < N) {
                            const double2 y = b[q];
                            xr[q] += pr_ * y.x - pi_ * y.y;
                            xi[q] += pr_ * y.y + pi_ * y.x;
                        }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (n0 + q < N) {
                double2 out = make_double2(ar * xr[q] - ai * xi[q], ar * xi[q] + ai * xr[q]);
                if (beta) {
                    const double2 old = c[n0 + q];
                    out.x += old.x;
                    out.y += old.y;
                }
                c[n0 + q] = out;
            }
    }
}

// Reduction-shaped products (M <= MAXM, N <= 256, long K, B stored with n
// contiguous): one workgroup per K chunk (M * chunk <= ZRED_LDS).  The chunk
// of A is staged in LDS; thread t then takes column n = t % N and every P-th
// k from t / N (P = 256 / N), so each step of the workgroup reads P
// consecutive rows of B as one contiguous span, and the B rows of the next U
// steps are in flight while the current ones are used (only B loads occupy
// the memory queue).  The P partial sums of an output are combined in LDS in
// a fixed order.
template <bool TA, int MAXM, int U>
__global__ __launch_bounds__(256) void k_zred(const double2* __restrict__ A, const double2* __restrict__ B,
                                              double2* __restrict__ C, const ZProb* __restrict__ probs,
                                              const ZTile* __restrict__ tiles, double ar, double ai, int beta,
                                              int cA, int cB, const int* __restrict__ active) {
    __shared__ double2 As[ZRED_LDS];   // [m][k] of the chunk
    __shared__ double2 red[kThreads];
    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;
    const ZProb pr = probs[tl.prob];
    const int M = pr.M, N = pr.N, K = pr.K;
    if (M <= 0 || N <= 0) return;
    const int P = kThreads / N;
    const int tid = threadIdx.x, n = tid % N, kl = tid / N;
    const bool live = kl < P;
    const double sA = cA ? -1.0 : 1.0, sB = cB ? -1.0 : 1.0;
    const double2* Ap = A + pr.a_off;
    const double2* Bp = B + pr.b_off + n;
    for (int e = tid; e < M * K; e += kThreads) {
        int i, k;
        if (TA) {   // A(i, k) at Ap[k * lda + i]: i fastest for coalescing
            k = e / M;
            i = e - k * M;
        } else {
            i = e / K;
            k = e - i * K;
        }
        double2 v = TA ? Ap[(long long)k * pr.lda + i] : Ap[(long long)i * pr.lda + k];
        v.y *= sA;
        As[i * K + k] = v;
    }
    __syncthreads();
    double xr[MAXM], xi[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) xr[i] = xi[i] = 0.0;
    auto fma_k = [&](const double2 b, int k) {
        const double br = b.x, bi = sB * b.y;
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
            if (i < M) {
                const double2 x = As[i * K + k];
                xr[i] += x.x * br - x.y * bi;
                xi[i] += x.x * bi + x.y * br;
            }
    };
    if (live) {
        const int step = U * P;
        int k = kl;
        double2 nb[U];
        if (k + (U - 1) * P < K) {
#pragma unroll
            for (int u = 0; u < U; ++u) nb[u] = Bp[(long long)(k + u * P) * pr.ldb];
        }
        for (; k + (U - 1) * P < K; k += step) {
            double2 cb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) cb[u] = nb[u];
            if (k + step + (U - 1) * P < K) {
#pragma unroll
                for (int u = 0; u < U; ++u) nb[u] = Bp[(long long)(k + step + u * P) * pr.ldb];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) fma_k(cb[u], k + u * P);
        }
        for (; k < K; k += P) fma_k(Bp[(long long)k * pr.ldb], k);
    }
    double2* Cp = C + pr.c_off;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        if (i >= M) break;
        __syncthreads();
        if (live) red[kl * N + n] = make_double2(xr[i], xi[i]);
        __syncthreads();
        if (tid < N) {
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < P; ++q) {
                sr += red[q * N + tid].x;
                si += red[q * N + tid].y;
            }
            double2 out = make_double2(ar * sr - ai * si, ar * si + ai * sr);
            double2* c = Cp + (long long)i * pr.ldc + tid;
            if (beta) {
                const double2 old = *c;
                out.x += old.x;
                out.y += old.y;
            }
            *c = out;
        }
    }
}

// Dot-product-shaped products (M <= MAXM rows of A, B stored transposed so
// that every output C(m, n) is the dot product of the contiguous K-vectors
// A(m, :) and B(n, :)): one workgroup per ZDOT_ROWS rows of B, each of its
// four waves streaming four rows.  A is staged in LDS in chunks of ZDOT_KC;
// lane l takes k = l, l + 64, ... of the chunk, so every load instruction of
// a wave reads 1 KB of one B row contiguously and the four rows x four
// k-steps of a chunk (16 loads per lane) are issued before they are used.
// Each B element is read once; the 64 lane partial sums of an output are
// combined by a fixed butterfly.
template <int MAXM>
__global__ __launch_bounds__(256) void k_zdot(const double2* __restrict__ A, const double2* __restrict__ B,
                                              double2* __restrict__ C, const ZProb* __restrict__ probs,
                                              const ZTile* __restrict__ tiles, double ar, double ai, int beta,
                                              int cA, int cB, const int* __restrict__ active) {
    constexpr int RW = ZDOT_ROWS / 4, KS = ZDOT_KC / 64;
    __shared__ double2 As[MAXM * ZDOT_KC];
    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;
    const ZProb pr = probs[tl.prob];
    const int M = pr.M, N = pr.N, K = pr.K;
    if (M <= 0 || N <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nb = tl.n0 + wave * RW;
    const double sA = cA ? -1.0 : 1.0, sB = cB ? -1.0 : 1.0;
    const double2* Ap = A + pr.a_off;
    const double2* Bp = B + pr.b_off;
    double xr[RW][MAXM], xi[RW][MAXM];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int i = 0; i < MAXM; ++i) xr[r][i] = xi[r][i] = 0.0;
    for (int k0 = 0; k0 < K; k0 += ZDOT_KC) {
        const int kc = min(ZDOT_KC, K - k0);
        __syncthreads();
        for (int e = tid; e < M * ZDOT_KC; e += kThreads) {
            const int i = e / ZDOT_KC, k = e - i * ZDOT_KC;
            double2 v = make_double2(0.0, 0.0);
            if (k < kc) {
                v = Ap[(long long)i * pr.lda + k0 + k];
                v.y *= sA;
            }
            As[e] = v;
        }
        __syncthreads();
        double2 b[KS][RW];
#pragma unroll
        for (int q = 0; q < KS; ++q)
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int k = q * 64 + lane, n = nb + r;
                b[q][r] = (k < kc && n < N) ? Bp[(long long)n * pr.ldb + k0 + k] : make_double2(0.0, 0.0);
            }
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const int k = q * 64 + lane;
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                if (i >= M) break;
                const double2 a = As[i * ZDOT_KC + k];
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const double br = b[q][r].x, bi = sB * b[q][r].y;
                    xr[r][i] += a.x * br - a.y * bi;
                    xi[r][i] += a.x * bi + a.y * br;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            if (i >= M) break;
            double sr = xr[r][i], si = xi[r][i];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                sr += __shfl_xor(sr, off, 64);
                si += __shfl_xor(si, off, 64);
            }
            const int n = nb + r;
            if (lane == 0 && n < N) {
                double2 out = make_double2(ar * sr - ai * si, ar * si + ai * sr);
                double2* c = C + pr.c_off + (long long)i * pr.ldc + n;
                if (beta) {
                    const double2 old = *c;
                    out.x += old.x;
                    out.y += old.y;
                }
                *c = out;
            }
        }
}

void zcfg_tile(int cfg, int* bm, int* bn) {
    switch (cfg) {
        case ZCFG_SKINNY: *bm = ZSKINNY_BM; *bn = ZSKINNY_BN; break;
        case ZCFG_TALL: *bm = ZTALL_ROWS; *bn = ZTALL_MAX_KN; break;
        case ZCFG_RED: *bm = ZRED_MAX_M; *bn = ZRED_MAX_N; break;
        case ZCFG_DOT: *bm = ZDOT_MAX_M; *bn = ZDOT_ROWS; break;
        case ZCFG_128x16: *bm = 128; *bn = 16; break;
        case ZCFG_16x128: *bm = 16; *bn = 128; break;
        case ZCFG_32x32: *bm = 32; *bn = 32; break;
        case ZCFG_64x16: *bm = 64; *bn = 16; break;
        case ZCFG_16x64: *bm = 16; *bn = 64; break;
        case ZCFG_32x64: *bm = 32; *bn = 64; break;
        case ZCFG_64x32: *bm = 64; *bn = 32; break;
        case ZCFG_64x64R: *bm = 64; *bn = 64; break;
        case ZCFG_64x32R: *bm = 64; *bn = 32; break;
        default: *bm = 64; *bn = 64; break;
    }
}

template <int BM, int BN, int WM, int WN, int BK, bool M3, bool DB>
static hipError_t launch_cfg(bool tA, bool tB, const double2* A, const double2* B, double2* C, const ZProb* probs,
                             const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA, int cB,
                             hipStream_t st, int role, const int* active) {
    dim3 grid(ntiles), block(kThreads);
    if (!tA && !tB) {
        if (role == 2) k_zgemm<BM, BN, WM, WN, BK, false, false, 2, M3, DB><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else k_zgemm<BM, BN, WM, WN, BK, false, false, 0, M3, DB><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    } else if (!tA && tB) {
        if (role == 1) k_zgemm<BM, BN, WM, WN, BK, false, true, 1, M3, DB><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else k_zgemm<BM, BN, WM, WN, BK, false, true, 0, M3, DB><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    } else if (tA && !tB) {
        k_zgemm<BM, BN, WM, WN, BK, true, false, 0, M3, DB><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    } else {
        k_zgemm<BM, BN, WM, WN, BK, true, true, 0, M3, DB><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
    }
    return hipGetLastError();
}

template <int BK, bool M3>
static hipError_t launch_bk(int cfg, bool tA, bool tB, const double2* A, const double2* B, double2* C,
                            const ZProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA,
                            int cB, hipStream_t st, int role, const int* active) {
    switch (cfg) {
        case ZCFG_128x16: return launch_cfg<128, 16, 4, 1, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_16x128: return launch_cfg<16, 128, 1, 4, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_32x32: return launch_cfg<32, 32, 2, 2, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x16: return launch_cfg<64, 16, 4, 1, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_16x64: return launch_cfg<16, 64, 1, 4, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x64: return launch_cfg<64, 64, 2, 2, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_32x64: return launch_cfg<32, 64, 2, 2, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x32: return launch_cfg<64, 32, 2, 2, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x64R: return launch_cfg<64, 64, 4, 1, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x32R: return launch_cfg<64, 32, 4, 1, BK, M3, false>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        default: return hipErrorInvalidValue;
    }
}

// double-buffered forms: 16-deep slices, tiles whose two LDS buffer pairs
// stay within 64 KB per workgroup
template <bool M3>
static hipError_t launch_db(int cfg, bool tA, bool tB, const double2* A, const double2* B, double2* C,
                            const ZProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA,
                            int cB, hipStream_t st, int role, const int* active) {
    switch (cfg) {
        case ZCFG_32x32: return launch_cfg<32, 32, 2, 2, 16, M3, true>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x16: return launch_cfg<64, 16, 4, 1, 16, M3, true>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_16x64: return launch_cfg<16, 64, 1, 4, 16, M3, true>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_32x64: return launch_cfg<32, 64, 2, 2, 16, M3, true>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x32: return launch_cfg<64, 32, 2, 2, 16, M3, true>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        case ZCFG_64x32R: return launch_cfg<64, 32, 4, 1, 16, M3, true>(tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        default: return hipErrorInvalidValue;
    }
}

bool zcfg_has_db(int cfg) {
    return cfg == ZCFG_32x32 || cfg == ZCFG_64x16 || cfg == ZCFG_16x64 || cfg == ZCFG_32x64 || cfg == ZCFG_64x32 ||
           cfg == ZCFG_64x32R;
}

hipError_t launch_zgemm(int cfg, int bk, bool tA, bool tB, const double2* A, const double2* B, double2* C,
                        const ZProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA,
                        int cB, hipStream_t st, int role, const int* active, int max_m, bool m3, int lds) {
    if (ntiles <= 0) return hipSuccess;
    if (lds == LDS_DIRECT) {
        if (bk != 16 || !zcfg_has_dl(cfg)) return hipErrorInvalidValue;
        return launch_zgemm_dl(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active, m3);
    }
    if (lds == LDS_DOUBLE) {
        if (bk != 16 || !zcfg_has_db(cfg)) return hipErrorInvalidValue;
        return m3 ? launch_db<true>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active)
                  : launch_db<false>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
    }
    if (cfg == ZCFG_TALL) {
        if (tA) return hipErrorInvalidValue;
        dim3 grid(ntiles), block(kThreads);
        if (tB) k_ztall<true><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else k_ztall<false><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        return hipGetLastError();
    }
    if (cfg == ZCFG_RED) {
        if (tB || max_m < 1 || max_m > ZRED_MAX_M) return hipErrorInvalidValue;
        dim3 grid(ntiles), block(kThreads);
        if (max_m <= 2) {
            if (tA) k_zred<true, 2, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
            else k_zred<false, 2, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        } else if (max_m <= 4) {
            if (tA) k_zred<true, 4, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
            else k_zred<false, 4, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        } else {
            if (tA) k_zred<true, 8, 4><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
            else k_zred<false, 8, 4><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        }
        return hipGetLastError();
    }
    if (cfg == ZCFG_DOT) {
        if (tA || !tB || max_m < 1 || max_m > ZDOT_MAX_M) return hipErrorInvalidValue;
        dim3 grid(ntiles), block(kThreads);
        if (max_m <= 2) k_zdot<2><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else if (max_m <= 4) k_zdot<4><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else k_zdot<8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        return hipGetLastError();
    }
    if (cfg == ZCFG_SKINNY) {
        dim3 grid(ntiles), block(kThreads);
        if (!tA && !tB) k_zskinny<false, false><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else if (!tA && tB) k_zskinny<false, true><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else if (tA && !tB) k_zskinny<true, false><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        else k_zskinny<true, true><<<grid, block, 0, st>>>(A, B, C, probs, tiles, ar, ai, beta, cA, cB, active);
        return hipGetLastError();
    }
    if (m3) {
        if (bk == 32) return launch_bk<32, true>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        if (bk == 16) return launch_bk<16, true>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
    } else {
        if (bk == 32) return launch_bk<32, false>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
        if (bk == 16) return launch_bk<16, false>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, ar, ai, beta, cA, cB, st, role, active);
    }
    return hipErrorInvalidValue;
}

// Split-K second pass: each workgroup takes 16 consecutive outputs of one
// problem; 16 threads per output sum every 16th partial block (four loads in
// flight), and the 16 partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_splitk_reduce(double2* __restrict__ C, const double2* __restrict__ W,
                                                       const ZRed* __restrict__ reds, double ar, double ai, int beta,
                                                       const int* __restrict__ active) {
    __shared__ double2 part[kThreads];
    const ZRed r = reds[blockIdx.y];
    if (active && !active[r.sys]) return;
    const long long mn = (long long)r.M * r.N;
    const int o = threadIdx.x & 15, g = threadIdx.x >> 4;
    const long long e = (long long)blockIdx.x * 16 + o;
    double sr = 0.0, si = 0.0;
    if (e < mn) {
        const double2* w = W + r.w_off + e;
        int s = g;
        for (; s + 48 < r.S; s += 64) {
            const double2 x0 = w[(long long)s * mn], x1 = w[(long long)(s + 16) * mn];
            const double2 x2 = w[(long long)(s + 32) * mn], x3 = w[(long long)(s + 48) * mn];
            sr += x0.x;
            si += x0.y;
            sr += x1.x;
            si += x1.y;
            sr += x2.x;
            si += x2.y;
            sr += x3.x;
            si += x3.y;
        }
        for (; s < r.S; s += 16) {
            const double2 x = w[(long long)s * mn];
            sr += x.x;
            si += x.y;
        }
    }
    part[threadIdx.x] = make_double2(sr, si);
    __syncthreads();
    if (g == 0 && e < mn) {
        sr = 0.0;
        si = 0.0;
        for (int q = 0; q < 16; ++q) {
            sr += part[q * 16 + o].x;
            si += part[q * 16 + o].y;
        }
        const int m = (int)(e / r.N), n = (int)(e % r.N);
        double2* c = C + r.c_off + (long long)m * r.ldc + n;
        double2 out = make_double2(ar * sr - ai * si, ar * si + ai * sr);
        if (beta) {
            const double2 old = *c;
            out.x += old.x;
            out.y += old.y;
        }
        *c = out;
    }
}

// The same pass for few K chunks (S <= ZRED_FEW_S, the MFMA tiles' split):
// one output per thread, its S partial values read in chunk order (the
// summation order of the kernel above), every load coalesced.
__global__ __launch_bounds__(256) void k_splitk_reduce_few(double2* __restrict__ C, const double2* __restrict__ W,
                                                           const ZRed* __restrict__ reds, double ar, double ai,
                                                           int beta, const int* __restrict__ active) {
    const ZRed r = reds[blockIdx.y];
    if (active && !active[r.sys]) return;
    const long long mn = (long long)r.M * r.N;
    if ((long long)blockIdx.x * blockDim.x >= mn) return;   // whole workgroup past this problem
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mn) return;
    const double2* w = W + r.w_off + e;
    double sr = 0.0, si = 0.0;
    int s = 0;
    for (; s + 4 <= r.S; s += 4) {
        const double2 x0 = w[(long long)s * mn], x1 = w[(long long)(s + 1) * mn];
        const double2 x2 = w[(long long)(s + 2) * mn], x3 = w[(long long)(s + 3) * mn];
        sr += x0.x;
        si += x0.y;
        sr += x1.x;
        si += x1.y;
        sr += x2.x;
        si += x2.y;
        sr += x3.x;
        si += x3.y;
    }
    for (; s < r.S; ++s) {
        const double2 x = w[(long long)s * mn];
        sr += x.x;
        si += x.y;
    }
    // C rows contiguous (ldc == N): the output index is e itself; otherwise
    // split it with 32-bit arithmetic (M*N < 2^31, checked by the planner)
    long long ci = e;
    if (r.ldc != r.N) {
        const unsigned ue = (unsigned)e, un = (unsigned)r.N;
        ci = (long long)(ue / un) * r.ldc + (ue % un);
    }
    double2* c = C + r.c_off + ci;
    double2 out = make_double2(ar * sr - ai * si, ar * si + ai * sr);
    if (beta) {
        const double2 old = *c;
        out.x += old.x;
        out.y += old.y;
    }
    *c = out;
}

hipError_t launch_splitk_reduce(double2* C, const double2* W, const ZRed* reds, int nred, int maxMN, int maxS,
                                double ar, double ai, int beta, hipStream_t st, const int* active) {
    if (nred <= 0 || maxMN <= 0) return hipSuccess;
    if (maxS <= ZRED_FEW_S) {
        dim3 grid((unsigned)((maxMN + kThreads - 1) / kThreads), (unsigned)nred);
        k_splitk_reduce_few<<<grid, kThreads, 0, st>>>(C, W, reds, ar, ai, beta, active);
    } else {
        dim3 grid((unsigned)((maxMN + 15) / 16), (unsigned)nred);
        k_splitk_reduce<<<grid, kThreads, 0, st>>>(C, W, reds, ar, ai, beta, active);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gather / reorder

__device__ __forceinline__ double2 map_load(const double2* __restrict__ s, uint32_t m) {
    if (m == 0xFFFFFFFFu) return make_double2(0.0, 0.0);
    double2 x = s[m & 0x7FFFFFFFu];
    if (m & 0x80000000u) {
        x.x = -x.x;
        x.y = -x.y;
    }
    return x;
}

// Workgroup b of a launch of G runs on XCD b % 8, and each XCD has its own L2.
// The reorders number their work so that XCD x takes one contiguous run of
// about G / 8 logical blocks (x < G % 8 take one more): neighbouring
// destination blocks, which read neighbouring source elements (the same cache
// lines, for a transposition), then share one L2 instead of fetching those
// lines once per XCD.  A bijection of [0, G).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned G) {
    const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + i;
}

// element of this thread in a plain or segmented launch; false if none
__device__ __forceinline__ bool elem_index(const SegBlocks& sb, long long n, long long* k) {
    if (sb.sys) {
        const int b = blockIdx.x;
        if (!sb.active[sb.sys[b]]) return false;
        *k = sb.start[b] + threadIdx.x;
        return *k < sb.end[b];
    }
    *k = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    return *k < n;
}

__host__ inline unsigned elem_grid(const SegBlocks& sb, long long n) {
    return sb.sys ? (unsigned)sb.nblk : (unsigned)((n + kThreads - 1) / kThreads);
}

// one destination element: dst[k] = beta*dst[k] + alpha * sum_t s_t cj(src[mA_t[k]]) (* src2[mB_t[k]])
template <int NT, bool BIL>
__device__ __forceinline__ void gather_elem(double2* __restrict__ dst, const double2* __restrict__ src,
                                            const double2* __restrict__ src2, const GatherMaps& maps, long long k,
                                            double ar, double ai, int beta, int conj) {
    double sr = 0.0, si = 0.0;
    bool any = false;   // some term is not a structural zero
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const uint32_t ma = maps.a[t][k];
        double2 x = map_load(maps.src[t] ? (const double2*)maps.src[t] : src, ma);
        if (conj) x.y = -x.y;
        if (!BIL) any = any || ma != 0xFFFFFFFFu;
        if (BIL) {
            const uint32_t mb = maps.b[t][k];
            any = any || (ma != 0xFFFFFFFFu && mb != 0xFFFFFFFFu);
            double2 y = map_load(src2, mb);
            double xr = x.x * y.x - x.y * y.y, xi = x.x * y.y + x.y * y.x;
            x.x = xr;
            x.y = xi;
        }
        sr += x.x;
        si += x.y;
    }
    // an accumulating gather leaves an element whose terms are all structural
    // zeros as it is (no read, no write)
    if (beta && !any) return;
    double2 out = make_double2(ar * sr - ai * si, ar * si + ai * sr);
    if (beta) {
        double2 o = dst[k];
        out.x += o.x;
        out.y += o.y;
    }
    dst[k] = out;
}

template <int NT, bool BIL>
__global__ __launch_bounds__(256) void k_gather(double2* __restrict__ dst, const double2* __restrict__ src,
                                                const double2* __restrict__ src2, GatherMaps maps, long long n,
                                                double ar, double ai, int beta, int conj, SegBlocks sb) {
    long long k;
    if (!elem_index(sb, n, &k)) return;
    gather_elem<NT, BIL>(dst, src, src2, maps, k, ar, ai, beta, conj);
}

// The same gather traversing the destination in 16 x 16 tiles of its blocks
// (one workgroup per tile, an 8 x 8 quarter per wave): where the maps follow
// a transposition, the 64 source elements of a wave then lie in fewer cache
// lines than along one destination row.
template <int NT, bool BIL>
__global__ __launch_bounds__(256) void k_gather_tiled(double2* __restrict__ dst, const double2* __restrict__ src,
                                                      const double2* __restrict__ src2, GatherMaps maps,
                                                      const GTile* __restrict__ tiles, double ar, double ai, int beta,
                                                      int conj) {
    const GTile t = tiles[xcd_block(blockIdx.x, gridDim.x)];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r = (w >> 1) * 8 + (l >> 3), c = (w & 1) * 8 + (l & 7);
    if (r >= t.nr || c >= t.nc) return;
    gather_elem<NT, BIL>(dst, src, src2, maps, t.k0 + (long long)r * t.ld + c, ar, ai, beta, conj);
}

hipError_t launch_gather_tiled(double2* dst, const double2* src, const double2* src2, GatherMaps maps, int nt,
                               const GTile* tiles, int ntiles, double ar, double ai, int beta, int conj,
                               hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid((unsigned)ntiles), block(kThreads);
    bool bil = src2 != nullptr;
#define FSCC_GT(NT)                                                                                                \
    if (bil) k_gather_tiled<NT, true><<<grid, block, 0, st>>>(dst, src, src2, maps, tiles, ar, ai, beta, conj);   \
    else k_gather_tiled<NT, false><<<grid, block, 0, st>>>(dst, src, src2, maps, tiles, ar, ai, beta, conj);
    switch (nt) {
        case 1: FSCC_GT(1); break;
        case 2: FSCC_GT(2); break;
        case 3: FSCC_GT(3); break;
        case 4: FSCC_GT(4); break;
        default: return hipErrorInvalidValue;
    }
#undef FSCC_GT
    return hipGetLastError();
}

// The same gather traversing its affine tiles (at most 16 x 16 destination
// elements each), grouped into work units of at most 256 elements and 8 tiles:
// one single-wave workgroup per unit, element e of the unit (tiles
// concatenated, row-major inside each) on lane e % 64, so a lane handles up
// to four elements and keeps up to 4 x NT independent loads in flight (every
// term's loads are issued before any is used).  A term is read with
// consecutive lanes on consecutive source elements: along the destination
// rows when its column stride is 1 (or it has no affine form), down the
// columns when its row stride is 1 -- a transposition, staged through LDS so
// that the destination is written along its rows.  Affine terms read no map;
// the others use their maps.
template <int NT>
__global__ __launch_bounds__(64) void k_reorder(double2* __restrict__ dst, const double2* __restrict__ src,
                                                GatherMaps maps, const RUnit* __restrict__ units,
                                                const GTile* __restrict__ tiles, const RTerm* __restrict__ terms,
                                                double ar, double ai, int beta, int conj) {
    __shared__ double2 tr[NT][RUNIT_MAX_ELEMS];
    const int lane = threadIdx.x;
    const RUnit u = units[xcd_block(blockIdx.x, gridDim.x)];
    // tile of each of the lane's elements: element offsets of the unit's tiles
    int start[RUNIT_MAX_RECTS + 1];
    GTile tl[RUNIT_MAX_RECTS];
    start[0] = 0;
#pragma unroll
    for (int j = 0; j < RUNIT_MAX_RECTS; ++j) {
        tl[j] = j < u.count ? tiles[u.first + j] : GTile{0, 0, 0, 0};
        start[j + 1] = start[j] + (int)tl[j].nr * tl[j].nc;
    }
    const int n = start[RUNIT_MAX_RECTS];
    // per element: its tile (selected without dynamic register indexing)
    int jt[4], st[4];
    GTile te[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = lane + 64 * k;
        jt[k] = 0;
        st[k] = 0;
        te[k] = tl[0];
#pragma unroll
        for (int i = 1; i < RUNIT_MAX_RECTS; ++i)
            if (i < u.count && e >= start[i]) {
                jt[k] = i;
                st[k] = start[i];
                te[k] = tl[i];
            }
    }
    double2 x[NT][4];
    bool cmk[NT][4];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const double2* __restrict__ s = maps.src[q] ? (const double2*)maps.src[q] : src;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = lane + 64 * k;
            x[q][k] = make_double2(0.0, 0.0);
            cmk[q][k] = false;
            if (e >= n) continue;
            const GTile t = te[k];
            const RTerm rt = terms[(long long)(u.first + jt[k]) * NT + q];
            const int nr = t.nr, nc = t.nc, el = e - st[k];
            const bool cm = rt.s0 >= 0 && rt.sa == 1 && rt.sb != 1 && nr > 1;
            const int r = cm ? el % nr : el / nc, c = cm ? el / nr : el % nc;
            if (rt.s0 == RTERM_MAPPED) {
                x[q][k] = map_load(s, maps.a[q][t.k0 + (long long)r * t.ld + c]);
            } else if (rt.s0 != RTERM_ZERO) {
                x[q][k] = s[(rt.s0 & ~RTERM_NEG) + (long long)r * rt.sa + (long long)c * rt.sb];
                if (rt.s0 & RTERM_NEG) {
                    x[q][k].x = -x[q][k].x;
                    x[q][k].y = -x[q][k].y;
                }
            }
            if (conj) x[q][k].y = -x[q][k].y;
            cmk[q][k] = cm;
            // a transposed read: element (r, c) of the tile is unit element st + r * nc + c
            if (cm) tr[q][st[k] + r * nc + c] = x[q][k];
        }
    }
    // a single wave: the barrier orders the LDS writes before the reads
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = lane + 64 * k;
        if (e >= n) continue;
        const GTile t = te[k];
        const int el = e - st[k], r = el / t.nc, c = el % t.nc;
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            // the term's orientation is that of the tile, the same for all its elements: the
            // row-major read of element e, or the LDS copy of a transposed read
            const double2 y = cmk[q][k] ? tr[q][e] : x[q][k];
            sr += y.x;
            si += y.y;
        }
        double2* d = dst + t.k0 + (long long)r * t.ld + c;
        double2 out = make_double2(ar * sr - ai * si, ar * si + ai * sr);
        if (beta) {
            const double2 o = *d;
            out.x += o.x;
            out.y += o.y;
        }
        *d = out;
    }
}

hipError_t launch_reorder(double2* dst, const double2* src, GatherMaps maps, int nt, const RUnit* units, int nunits,
                          const GTile* tiles, const RTerm* terms, double ar, double ai, int beta, int conj,
                          hipStream_t st) {
    if (nunits <= 0) return hipSuccess;
    dim3 grid((unsigned)nunits), block(64);
    switch (nt) {
        case 1: k_reorder<1><<<grid, block, 0, st>>>(dst, src, maps, units, tiles, terms, ar, ai, beta, conj); break;
        case 2: k_reorder<2><<<grid, block, 0, st>>>(dst, src, maps, units, tiles, terms, ar, ai, beta, conj); break;
        case 3: k_reorder<3><<<grid, block, 0, st>>>(dst, src, maps, units, tiles, terms, ar, ai, beta, conj); break;
        case 4: k_reorder<4><<<grid, block, 0, st>>>(dst, src, maps, units, tiles, terms, ar, ai, beta, conj); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gather(double2* dst, const double2* src, const double2* src2, GatherMaps maps, int nt,
                         long long n, double ar, double ai, int beta, int conj, hipStream_t st, SegBlocks sb) {
    if (n <= 0 || (sb.sys && sb.nblk <= 0)) return hipSuccess;
    dim3 grid(elem_grid(sb, n)), block(kThreads);
    bool bil = src2 != nullptr;
#define FSCC_G(NT)                                                                                               \
    if (bil) k_gather<NT, true><<<grid, block, 0, st>>>(dst, src, src2, maps, n, ar, ai, beta, conj, sb);      \
    else k_gather<NT, false><<<grid, block, 0, st>>>(dst, src, src2, maps, n, ar, ai, beta, conj, sb);
    switch (nt) {
        case 1: FSCC_G(1); break;
        case 2: FSCC_G(2); break;
        case 3: FSCC_G(3); break;
        case 4: FSCC_G(4); break;
        default: return hipErrorInvalidValue;
    }
#undef FSCC_G
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise

__global__ __launch_bounds__(256) void k_axpby(double2* __restrict__ dst, const double2* __restrict__ src, long long n,
                                               double ar, double ai, int beta, int conj, SegBlocks sb) {
    long long k;
    if (!elem_index(sb, n, &k)) return;
    double2 x = src[k];
    if (conj) x.y = -x.y;
    double2 out = make_double2(ar * x.x - ai * x.y, ar * x.y + ai * x.x);
    if (beta) {
        double2 o = dst[k];
        out.x += o.x;
        out.y += o.y;
    }
    dst[k] = out;
}

hipError_t launch_axpby(double2* dst, const double2* src, long long n, double ar, double ai, int beta, int conj,
                        hipStream_t st, SegBlocks sb) {
    if (n <= 0 || (sb.sys && sb.nblk <= 0)) return hipSuccess;
    k_axpby<<<elem_grid(sb, n), kThreads, 0, st>>>(dst, src, n, ar, ai, beta, conj, sb);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_diag(double2* __restrict__ dst, const double* __restrict__ d,
                                              const double2* __restrict__ src, long long n, SegBlocks sb) {
    long long k;
    if (!elem_index(sb, n, &k)) return;
    double2 o = dst[k], x = src[k];
    double dd = d[k];
    o.x -= dd * x.x;
    o.y -= dd * x.y;
    dst[k] = o;
}

hipError_t launch_diag(double2* dst, const double* d, const double2* src, long long n, hipStream_t st, SegBlocks sb) {
    if (n <= 0 || (sb.sys && sb.nblk <= 0)) return hipSuccess;
    k_diag<<<elem_grid(sb, n), kThreads, 0, st>>>(dst, d, src, n, sb);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mul(double2* __restrict__ dst, const double* __restrict__ d, long long n,
                                             SegBlocks sb) {
    long long k;
    if (!elem_index(sb, n, &k)) return;
    double2 o = dst[k];
    double dd = d[k];
    dst[k] = make_double2(dd * o.x, dd * o.y);
}

hipError_t launch_mul(double2* dst, const double* d, long long n, hipStream_t st, SegBlocks sb) {
    if (n <= 0 || (sb.sys && sb.nblk <= 0)) return hipSuccess;
    k_mul<<<elem_grid(sb, n), kThreads, 0, st>>>(dst, d, n, sb);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero(double2* __restrict__ dst, long long n) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = make_double2(0.0, 0.0);
}

hipError_t launch_zero(double2* dst, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_zero<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(dst, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reductions (deterministic: fixed grid, per-block partials, one final block)

int reduce_blocks(long long n) {
    long long b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
            sh[threadIdx.x] = (a > b || a != a) ? a : b;   // NaN propagates
        }
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Dynamic denominator shift of one amplitude (sector shift S < 0, exponent
// n >= 1): Delta = S (S / (min(D, 0) + S))^n; the shifted equations are
// R = Delta t, solved by the step (R - Delta t) / (D + Delta).
__device__ __forceinline__ double dyn_delta(double d, double S, int n) {
    const double q = S / (fmin(d, 0.0) + S);
    double p = q;
    for (int i = 1; i < n; ++i) p *= q;
    return S * p;
}

__global__ __launch_bounds__(256) void k_jacobi(const double2* __restrict__ t, const double2* __restrict__ r,
                                                const double* __restrict__ D, double2* __restrict__ ht,
                                                double2* __restrict__ he, long long n, double* part_max,
                                                double shift, double dS, int dn) {
    __shared__ double sh[kThreads];
    double mx = 0.0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads) {
        double2 rr = r[k], tt = t[k];
        double d = D[k];
        if (dS != 0.0) {
            const double dl = dyn_delta(d, dS, dn);
            rr.x -= dl * tt.x;
            rr.y -= dl * tt.y;
            d += dl;
        }
        d -= shift;
        double2 s = make_double2(rr.x / d, rr.y / d);
        he[k] = s;
        ht[k] = make_double2(tt.x + s.x, tt.y + s.y);
        double a = sqrt(s.x * s.x + s.y * s.y);
        mx = (a > mx || a != a) ? a : mx;
    }
    double b = block_max(mx, sh);
    if (threadIdx.x == 0) part_max[blockIdx.x] = b;
}

hipError_t launch_jacobi(const double2* t, const double2* r, const double* D, double2* hist_t, double2* hist_e,
                         long long n, double* part_max, int nblk, hipStream_t st, double shift, double dyn_S,
                         int dyn_n) {
    if (dyn_S != 0.0 && !(dyn_S < 0.0 && dyn_n >= 1)) return hipErrorInvalidValue;
    k_jacobi<<<nblk, kThreads, 0, st>>>(t, r, D, hist_t, hist_e, n, part_max, shift, dyn_S, dyn_n);
    return hipGetLastError();
}

// part[b*kDiisMax + j] = Re sum conj(e_j) enew over block b's share
struct PtrList {
    const double2* p[kDiisMax];
};

__global__ __launch_bounds__(256) void k_dots(PtrList e, int m, const double2* __restrict__ enew, long long n,
                                              double* part) {
    __shared__ double sh[kThreads];
    double acc[kDiisMax];
#pragma unroll
    for (int j = 0; j < kDiisMax; ++j) acc[j] = 0.0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads) {
        double2 y = enew[k];
#pragma unroll
        for (int j = 0; j < kDiisMax; ++j)
            if (j < m) {
                double2 x = e.p[j][k];
                acc[j] += x.x * y.x + x.y * y.y;
            }
    }
#pragma unroll
    for (int j = 0; j < kDiisMax; ++j)
        if (j < m) {
            double b = block_sum(acc[j], sh);
            if (threadIdx.x == 0) part[blockIdx.x * kDiisMax + j] = b;
        }
}

hipError_t launch_dots(const double2* const* e, int m, const double2* enew, long long n, double* part, int nblk,
                       hipStream_t st) {
    if (m < 0 || m > kDiisMax) return hipErrorInvalidValue;
    PtrList pl;
    for (int j = 0; j < kDiisMax; ++j) pl.p[j] = j < m ? e[j] : nullptr;
    k_dots<<<nblk, kThreads, 0, st>>>(pl, m, enew, n, part);
    return hipGetLastError();
}

// Bordered Pulay system over the slots order[0..m) (oldest first) of the
// symmetric matrix B (leading dimension ldb): Gaussian elimination with
// partial pivoting in FP64; a pivot below 1e-14 * max|A| drops the oldest
// slot and the solve is repeated.  coef[slot] receives the coefficients (0 for
// slots not used).  Single-thread code; the working matrix wa ((MAXM + 1) x
// (MAXM + 2)) and x (MAXM + 1) live in LDS (as private arrays they would be
// scratch memory, which made the solve 20x slower).  Returns the number of
// dropped slots.
template <int MAXM>
__device__ int diis_solve(const double* B, int ldb, const int* order, int m, double* coef, double* __restrict__ wa,
                          double* __restrict__ x) {
    auto A = [wa](int i, int j) -> double& { return wa[i * (MAXM + 2) + j]; };
    for (int j = 0; j < ldb; ++j) coef[j] = 0.0;
    int first = 0, dropped = 0;
    while (true) {
        int k = m - first;
        if (k <= 1) {
            coef[order[m - 1]] = 1.0;
            break;
        }
        double scale = 0.0;
        for (int i = 0; i < k; ++i) scale = fmax(scale, fabs(B[order[first + i] * ldb + order[first + i]]));
        if (!(scale > 0.0)) scale = 1.0;
        for (int i = 0; i < k; ++i) {
            for (int j = 0; j < k; ++j) A(i, j) = B[order[first + i] * ldb + order[first + j]] / scale;
            A(i, k) = -1.0;
            A(i, k + 1) = 0.0;
        }
        for (int j = 0; j < k; ++j) A(k, j) = -1.0;
        A(k, k) = 0.0;
        A(k, k + 1) = -1.0;
        int nn = k + 1;
        double amax = 0.0;
        for (int i = 0; i < nn; ++i)
            for (int j = 0; j < nn; ++j) amax = fmax(amax, fabs(A(i, j)));
        bool singular = false;
        for (int c = 0; c < nn && !singular; ++c) {
            int p = c;
            for (int i = c + 1; i < nn; ++i)
                if (fabs(A(i, c)) > fabs(A(p, c))) p = i;
            if (!(fabs(A(p, c)) >= 1e-14 * amax)) {
                singular = true;
                break;
            }
            if (p != c)
                for (int j = 0; j <= nn; ++j) {
                    double t = A(c, j);
                    A(c, j) = A(p, j);
                    A(p, j) = t;
                }
            for (int i = c + 1; i < nn; ++i) {
                double f = A(i, c) / A(c, c);
                for (int j = c; j <= nn; ++j) A(i, j) -= f * A(c, j);
            }
        }
        if (singular) {
            ++first;
            ++dropped;
            continue;
        }
        for (int i = nn - 1; i >= 0; --i) {
            double s = A(i, nn);
            for (int j = i + 1; j < nn; ++j) s -= A(i, j) * x[j];
            x[i] = s / A(i, i);
        }
        for (int i = 0; i < k; ++i) coef[order[first + i]] = x[i];
        break;
    }
    return dropped;
}

// One workgroup: reduce the dot partials into row/column `newslot` of B,
// then solve the bordered Pulay system over the slots listed in `order`
// (oldest first) by Gaussian elimination with partial pivoting in FP64;
// if a pivot is below 1e-14 * max|A| the oldest slot is dropped and the solve
// repeated.  coef[slot] receives the coefficient (0 for unused slots);
// scal[0] = max |step|, scal[1] = number of dropped slots.  A step that is
// not finite sets coef[ldb] = 1 (the extrapolation then leaves the
// amplitudes at their input values) and leaves B untouched; otherwise
// coef[ldb] = 0.
__global__ __launch_bounds__(256) void k_finish_diis(const double* __restrict__ part, int nblk, int m,
                                                     const double* __restrict__ part_max, int nblk_max,
                                                     double* __restrict__ B, int ldb, int newslot,
                                                     DiisOrder ord, double* __restrict__ coef,
                                                     double* __restrict__ scal) {
    __shared__ double sh[kThreads];
    __shared__ double row[kDiisMax];
    __shared__ int order[kDiisMax];
    __shared__ double wa[(kDiisMax + 1) * (kDiisMax + 2)], wx[kDiisMax + 1];
    if (threadIdx.x < kDiisMax) order[threadIdx.x] = (int)threadIdx.x < m ? ord.v[threadIdx.x] : 0;
    for (int j = 0; j < m; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kThreads) v += part[b * kDiisMax + j];
        double s = block_sum(v, sh);
        if (threadIdx.x == 0) row[j] = s;
    }
    double mx = 0.0;
    for (int b = threadIdx.x; b < nblk_max; b += kThreads) {
        double a = part_max[b];
        mx = (a > mx || a != a) ? a : mx;
    }
    mx = block_max(mx, sh);
    __syncthreads();
    if (threadIdx.x != 0) return;
    scal[0] = mx;
    if (!isfinite(mx)) {
        for (int j = 0; j < ldb; ++j) coef[j] = 0.0;
        coef[ldb] = 1.0;
        scal[1] = 0.0;
        return;
    }
    coef[ldb] = 0.0;
    // row[j] pairs the new vector with the slot order[j]
    for (int j = 0; j < m; ++j) {
        B[newslot * ldb + order[j]] = row[j];
        B[order[j] * ldb + newslot] = row[j];
    }
    int dropped = diis_solve<kDiisMax>(B, ldb, order, m, coef, wa, wx);
    scal[1] = (double)dropped;
}

hipError_t launch_finish_diis(const double* part, int nblk, int m, const double* part_max, int nblk_max, double* B,
                              int ldb, int newslot, const DiisOrder& order, double* coef, double* scal, hipStream_t st) {
    if (m < 1 || m > kDiisMax) return hipErrorInvalidValue;
    k_finish_diis<<<1, kThreads, 0, st>>>(part, nblk, m, part_max, nblk_max, B, ldb, newslot, order, coef, scal);
    return hipGetLastError();
}

// *count += number of non-finite values among x[0..n) (the caller zeroes *count)
__global__ __launch_bounds__(256) void k_count_nonfinite(const double* __restrict__ x, long long n,
                                                         unsigned long long* __restrict__ count) {
    __shared__ unsigned int sh[kThreads];
    unsigned int c = 0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads)
        c += isfinite(x[k]) ? 0u : 1u;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sh[0]) atomicAdd(count, (unsigned long long)sh[0]);
}

template <int ORDER>
__global__ __launch_bounds__(256) void k_dressed_denoms(const uint16_t* __restrict__ idx, const double* __restrict__ f,
                                                        int no, double floor, double* __restrict__ D, long long n) {
    const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    double d;
    if (ORDER == 2) {
        const ushort2 x = *(const ushort2*)(idx + 2 * k);
        d = f[x.x] - f[no + x.y];
    } else {
        const ushort4 x = *(const ushort4*)(idx + 4 * k);
        d = f[x.x] + f[x.y] - f[no + x.z] - f[no + x.w];
    }
    D[k] = fmin(d, -floor);
}

hipError_t launch_dressed_denoms(const uint16_t* idx, int order, const double* f, int no, double floor, double* D,
                                 long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((n + kThreads - 1) / kThreads);
    if (order == 2) k_dressed_denoms<2><<<grid, kThreads, 0, st>>>(idx, f, no, floor, D, n);
    else if (order == 4) k_dressed_denoms<4><<<grid, kThreads, 0, st>>>(idx, f, no, floor, D, n);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double* x, long long n, unsigned long long* count, hipStream_t st) {
    hipError_t e = hipMemsetAsync(count, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess || n <= 0) return e;
    const long long blocks = std::min<long long>((n + kThreads - 1) / kThreads, 4096);
    k_count_nonfinite<<<(unsigned)blocks, kThreads, 0, st>>>(x, n, count);
    return hipGetLastError();
}

// out = sum_j coef[j] xs[j]; coef[m] != 0 (a non-finite step) leaves out untouched
__global__ __launch_bounds__(256) void k_lincomb(double2* __restrict__ out, PtrList xs, const double* __restrict__ coef,
                                                 int m, long long n) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || coef[m] != 0.0) return;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < m; ++j) {
        double c = coef[j];
        if (c != 0.0) {
            double2 x = xs.p[j][k];
            sr += c * x.x;
            si += c * x.y;
        }
    }
    out[k] = make_double2(sr, si);
}

hipError_t launch_lincomb(double2* out, const double2* const* xs, const double* coef, int m, long long n,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (m < 0 || m > kDiisMax) return hipErrorInvalidValue;
    PtrList pl;
    for (int j = 0; j < kDiisMax; ++j) pl.p[j] = j < m ? xs[j] : nullptr;
    k_lincomb<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(out, pl, coef, m, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zdotu_part(const double2* __restrict__ x, const double2* __restrict__ y,
                                                    long long n, double* part) {
    __shared__ double sh[kThreads];
    double sr = 0.0, si = 0.0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads) {
        double2 a = x[k], b = y[k];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
    }
    double r = block_sum(sr, sh);
    double i = block_sum(si, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r;
        part[2 * blockIdx.x + 1] = i;
    }
}

__global__ __launch_bounds__(256) void k_sum2(const double* __restrict__ part, int nblk, double* out) {
    __shared__ double sh[kThreads];
    double r = 0.0, i = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
        r += part[2 * b];
        i += part[2 * b + 1];
    }
    r = block_sum(r, sh);
    i = block_sum(i, sh);
    if (threadIdx.x == 0) {
        out[0] = r;
        out[1] = i;
    }
}

hipError_t launch_zdotu(const double2* x, const double2* y, long long n, double* part, int nblk, double* out,
                        hipStream_t st) {
    k_zdotu_part<<<nblk, kThreads, 0, st>>>(x, y, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum2<<<1, kThreads, 0, st>>>(part, nblk, out);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// batched Jacobi + DIIS update and energy: blockIdx.y (or x) = system; each
// system keeps its own circular DIIS history on the device, so an iteration
// needs no host decision and can be replayed as a graph.

__global__ __launch_bounds__(256) void k_bjacobi(const double2* __restrict__ t1, const double2* __restrict__ t2,
                                                 const double2* __restrict__ r1, const double2* __restrict__ r2,
                                                 const double* __restrict__ D1, const double* __restrict__ D2,
                                                 const BSeg* __restrict__ segs, const BState* __restrict__ state,
                                                 double2* __restrict__ ht, double2* __restrict__ he,
                                                 double* __restrict__ part_max, double shift) {
    __shared__ double sh[kThreads];
    const int s = blockIdx.y;
    const BState stt = state[s];
    if (!stt.active) {
        if (threadIdx.x == 0) part_max[(long long)s * gridDim.x + blockIdx.x] = 0.0;
        return;
    }
    const BSeg g = segs[s];
    const long long n = g.n1 + g.n2;
    const int slot = (stt.newest + 1) % stt.nd;
    double2* hts = ht + g.hoff + (long long)slot * n;
    double2* hes = he + g.hoff + (long long)slot * n;
    double mx = 0.0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads) {
        double2 rr, tt;
        double d;
        if (k < g.n1) {
            rr = r1[g.off1 + k];
            tt = t1[g.off1 + k];
            d = D1[g.off1 + k];
        } else {
            rr = r2[g.off2 + k - g.n1];
            tt = t2[g.off2 + k - g.n1];
            d = D2[g.off2 + k - g.n1];
        }
        d -= shift;   // level shift: D < 0 for every amplitude, so |D| grows and the step is damped
        const double2 st = make_double2(rr.x / d, rr.y / d);
        hes[k] = st;
        hts[k] = make_double2(tt.x + st.x, tt.y + st.y);
        const double a = sqrt(st.x * st.x + st.y * st.y);
        mx = (a > mx || a != a) ? a : mx;
    }
    const double b = block_max(mx, sh);
    if (threadIdx.x == 0) part_max[(long long)s * gridDim.x + blockIdx.x] = b;
}

// live slots of system state `st` after adding the new vector: oldest first
__device__ inline int bslots(const BState& st, int* order) {
    const int nw = (st.newest + 1) % st.nd;
    const int m = min(st.count + 1, st.nd);
    for (int j = 0; j < m; ++j) order[j] = ((nw - (m - 1) + j) % st.nd + st.nd) % st.nd;
    return m;
}

__global__ __launch_bounds__(256) void k_bdots(const BSeg* __restrict__ segs, const BState* __restrict__ state,
                                               const double2* __restrict__ he, double* __restrict__ part) {
    __shared__ double sh[kThreads];
    const int s = blockIdx.y;
    const BState stt = state[s];
    if (!stt.active) return;
    const BSeg g = segs[s];
    const long long n = g.n1 + g.n2;
    int order[8];
    const int m = bslots(stt, order);
    const double2* enew = he + g.hoff + (long long)order[m - 1] * n;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads) {
        const double2 y = enew[k];
        for (int j = 0; j < m; ++j) {
            const double2 x = he[g.hoff + (long long)order[j] * n + k];
            acc[j] += x.x * y.x + x.y * y.y;
        }
    }
    for (int j = 0; j < m; ++j) {
        const double b = block_sum(acc[j], sh);
        if (threadIdx.x == 0) part[((long long)s * gridDim.x + blockIdx.x) * 8 + j] = b;
    }
}

// one workgroup per system: finish the dots, update B, solve, advance the
// circular history, apply the convergence test (max|step| < tol freezes the
// system after this update; a non-finite step freezes it as failed)
__global__ __launch_bounds__(256) void k_bfinish(BState* __restrict__ state, const double* __restrict__ part, int nblk,
                                                 const double* __restrict__ part_max, double* __restrict__ Bm,
                                                 double* __restrict__ coef, double* __restrict__ maxstep, double tol,
                                                 int* __restrict__ active, int* __restrict__ upd) {
    __shared__ double sh[kThreads];
    __shared__ double row[8];
    __shared__ double wa[9 * 10], wx[9];
    const int s = blockIdx.x;
    BState stt = state[s];
    if (!stt.active) {
        if (threadIdx.x == 0) {
            state[s].upd = 0;
            active[s] = 0;
            upd[s] = 0;
        }
        return;
    }
    int order[8];
    const int m = bslots(stt, order);
    for (int j = 0; j < m; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kThreads) v += part[((long long)s * nblk + b) * 8 + j];
        const double r = block_sum(v, sh);
        if (threadIdx.x == 0) row[j] = r;
    }
    double mx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
        const double a = part_max[(long long)s * nblk + b];
        mx = (a > mx || a != a) ? a : mx;
    }
    mx = block_max(mx, sh);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double* B = Bm + (long long)s * 64;
    const int nw = order[m - 1];
    for (int j = 0; j < m; ++j) {
        B[nw * 8 + order[j]] = row[j];
        B[order[j] * 8 + nw] = row[j];
    }
    const int dropped = diis_solve<8>(B, 8, order, m, coef + (long long)s * 8, wa, wx);
    stt.newest = nw;
    stt.count = max(1, m - dropped);
    stt.iters += 1;
    stt.upd = 1;
    if (!(mx == mx) || mx > 1.7976931348623157e308) {
        stt.failed = 1;
        stt.active = 0;
        stt.upd = 0;
    } else if (mx < tol) {
        stt.active = 0;
    }
    state[s] = stt;
    active[s] = stt.active;
    upd[s] = stt.upd;
    maxstep[s] = mx;
}

__global__ __launch_bounds__(256) void k_blincomb(double2* __restrict__ t1, double2* __restrict__ t2,
                                                  const BSeg* __restrict__ segs, const BState* __restrict__ state,
                                                  const double2* __restrict__ ht, const double* __restrict__ coef) {
    const int s = blockIdx.y;
    const BState stt = state[s];
    if (!stt.upd) return;
    const BSeg g = segs[s];
    const long long n = g.n1 + g.n2;
    double c[8];
    for (int j = 0; j < 8; ++j) c[j] = j < stt.nd ? coef[s * 8 + j] : 0.0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads) {
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < stt.nd; ++j)
            if (c[j] != 0.0) {
                const double2 x = ht[g.hoff + (long long)j * n + k];
                sr += c[j] * x.x;
                si += c[j] * x.y;
            }
        if (k < g.n1) t1[g.off1 + k] = make_double2(sr, si);
        else t2[g.off2 + k - g.n1] = make_double2(sr, si);
    }
}

__global__ __launch_bounds__(256) void k_benergy(const double2* __restrict__ x, const double2* __restrict__ y,
                                                 const BSeg* __restrict__ segs, double* __restrict__ part) {
    __shared__ double sh[kThreads];
    const int s = blockIdx.y;
    const BSeg g = segs[s];
    double sr = 0.0, si = 0.0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < g.n2; k += (long long)gridDim.x * kThreads) {
        const double2 a = x[g.off2 + k], b = y[g.off2 + k];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
    }
    const double r = block_sum(sr, sh);
    const double i = block_sum(si, sh);
    if (threadIdx.x == 0) {
        part[((long long)s * gridDim.x + blockIdx.x) * 2] = r;
        part[((long long)s * gridDim.x + blockIdx.x) * 2 + 1] = i;
    }
}

// per-system report row: E_re, E_im, max|step|, active, iterations, failed
__global__ __launch_bounds__(256) void k_breport(const double* __restrict__ part, int nblk,
                                                 const BState* __restrict__ state, const double* __restrict__ maxstep,
                                                 double* __restrict__ out) {
    __shared__ double sh[kThreads];
    const int s = blockIdx.x;
    double r = 0.0, i = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
        r += part[((long long)s * nblk + b) * 2];
        i += part[((long long)s * nblk + b) * 2 + 1];
    }
    r = block_sum(r, sh);
    i = block_sum(i, sh);
    if (threadIdx.x == 0) {
        const BState st = state[s];
        double* o = out + (long long)s * 6;
        o[0] = r;
        o[1] = i;
        o[2] = maxstep[s];
        o[3] = st.active;
        o[4] = st.iters;
        o[5] = st.failed;
    }
}

hipError_t launch_batch_update(const double2* t1, const double2* t2, const double2* r1, const double2* r2,
                               double2* t1o, double2* t2o, const double* D1, const double* D2, const BSeg* segs,
                               BState* state, double2* ht, double2* he, double* part_max, double* part, double* Bm,
                               double* coef, double* maxstep, double tol, double shift, int* active, int* upd,
                               int nsys, int nblk, hipStream_t st) {
    if (nsys <= 0) return hipSuccess;
    dim3 grid(nblk, nsys);
    k_bjacobi<<<grid, kThreads, 0, st>>>(t1, t2, r1, r2, D1, D2, segs, state, ht, he, part_max, shift);
    k_bdots<<<grid, kThreads, 0, st>>>(segs, state, he, part);
    k_bfinish<<<nsys, kThreads, 0, st>>>(state, part, nblk, part_max, Bm, coef, maxstep, tol, active, upd);
    k_blincomb<<<grid, kThreads, 0, st>>>(t1o, t2o, segs, state, ht, coef);
    return hipGetLastError();
}

hipError_t launch_batch_energy(const double2* oovv, const double2* tau, const BSeg* segs, const BState* state,
                               const double* maxstep, double* part, double* out, int nsys, int nblk, hipStream_t st) {
    if (nsys <= 0) return hipSuccess;
    k_benergy<<<dim3(nblk, nsys), kThreads, 0, st>>>(oovv, tau, segs, part);
    k_breport<<<nsys, kThreads, 0, st>>>(part, nblk, state, maxstep, out);
    return hipGetLastError();
}


// per-system max |r / D| over the T1 and T2 segments
__global__ __launch_bounds__(256) void k_bmaxnorm(const double2* __restrict__ r1, const double2* __restrict__ r2,
                                                  const double* __restrict__ D1, const double* __restrict__ D2,
                                                  const BSeg* __restrict__ segs, double* __restrict__ part) {
    __shared__ double sh[kThreads];
    const int s = blockIdx.y;
    const BSeg g = segs[s];
    const long long n = g.n1 + g.n2;
    double mx = 0.0;
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kThreads) {
        double2 rr;
        double d;
        if (k < g.n1) {
            rr = r1[g.off1 + k];
            d = D1[g.off1 + k];
        } else {
            rr = r2[g.off2 + k - g.n1];
            d = D2[g.off2 + k - g.n1];
        }
        const double a = sqrt(rr.x * rr.x + rr.y * rr.y) / fabs(d);
        mx = (a > mx || a != a) ? a : mx;
    }
    const double b = block_max(mx, sh);
    if (threadIdx.x == 0) part[(long long)s * gridDim.x + blockIdx.x] = b;
}

__global__ __launch_bounds__(256) void k_bmaxnorm_final(const double* __restrict__ part, int nblk,
                                                        double* __restrict__ out) {
    __shared__ double sh[kThreads];
    const int s = blockIdx.x;
    double mx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
        const double a = part[(long long)s * nblk + b];
        mx = (a > mx || a != a) ? a : mx;
    }
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) out[s] = mx;
}

hipError_t launch_batch_maxnorm(const double2* r1, const double2* r2, const double* D1, const double* D2,
                                const BSeg* segs, double* part, double* out, int nsys, int nblk, hipStream_t st) {
    if (nsys <= 0) return hipSuccess;
    k_bmaxnorm<<<dim3(nblk, nsys), kThreads, 0, st>>>(r1, r2, D1, D2, segs, part);
    k_bmaxnorm_final<<<nsys, kThreads, 0, st>>>(part, nblk, out);
    return hipGetLastError();
}

}  // namespace fscc
