// kernels_real.hip -- real-arithmetic forms of the FS-RCCSD hot-path kernels.
//
// For double groups whose integrals and amplitudes are real (the paper's
// symmetry-handling section: real groups such as C2v*, D2h*, C-inf-v* need
// no complex arithmetic), every contraction is a real GEMM: one FP64 MFMA
// chain per product instead of four, half the bytes per element.  Same tile
// lists, problems, maps and reductions as the complex kernels; only the
// element type differs.
//  * k_dgemm    grouped real GEMM on FP64 matrix cores (v_mfma_f64_16x16x4_f64)
//  * k_dtall / k_dred   the streaming vector-ALU forms (tall, reduction-shaped)
//  * gather, elementwise, Jacobi / DIIS / energy reductions on doubles
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fscc {

typedef double dbl4r __attribute__((ext_vector_type(4)));

namespace {

constexpr int kT = 256;

// ---------------------------------------------------------------------------
// grouped real GEMM: tiles as in the complex kernel, one LDS plane per
// operand, one MFMA chain per fragment

template <int BM, int BN, int WM, int WN, int BK, bool TA, bool TB, int ROLE>
__global__ __launch_bounds__(256, 3) void k_dgemm(const double* __restrict__ A, const double* __restrict__ B,
                                               double* __restrict__ C, const ZProb* __restrict__ probs,
                                               const ZTile* __restrict__ tiles, double alpha, int beta,
                                               const int* __restrict__ active) {
    constexpr int PAD = 1;   // odd row padding (bank spread of transposed stores and fragment reads)
    constexpr int FM = BM / (16 * WM);
    constexpr int FN = BN / (16 * WN);
    constexpr int KS_UNROLL = FM * FN >= 4 ? 2 : BK / 4;   // 4-deep steps unrolled per slice
    static_assert(WM * WN == 4, "four waves");
    static_assert(FM >= 1 && FN >= 1, "tile too small");
    __shared__ double As[BK][BM + PAD];
    __shared__ double Bs[BK][BN + PAD];

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

    dbl4r acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = dbl4r{0.0, 0.0, 0.0, 0.0};

    constexpr int AV = BM * BK / 4;
    constexpr int BV = BN * BK / 4;
    constexpr int AVT = (AV + kT - 1) / kT;
    constexpr int BVT = (BV + kT - 1) / kT;
    double ra[AVT][4], rb[BVT][4];

    auto load_slice = [&](int k0) {
#pragma unroll
        for (int u = 0; u < AVT; ++u) {
            int v = tid + u * kT;
#pragma unroll
            for (int e = 0; e < 4; ++e) ra[u][e] = 0.0;
            if (v < AV) {
                if (!TA) {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
                    int m = m0 + r;
                    if (m < M) {
                        const double* p = Ap + (long long)m * pr.lda + k0 + kk;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (k0 + kk + e < K) ra[u][e] = p[e];
                    }
                } else {
                    int kr = v / (BM / 4), mm = (v % (BM / 4)) * 4;
                    int k = k0 + kr;
                    if (k < K) {
                        const double* p = Ap + (long long)k * pr.lda + m0 + mm;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (m0 + mm + e < M) ra[u][e] = p[e];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < BVT; ++u) {
            int v = tid + u * kT;
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[u][e] = 0.0;
            if (v < BV) {
                if (!TB) {
                    int kr = v / (BN / 4), nn = (v % (BN / 4)) * 4;
                    int k = k0 + kr;
                    if (k < K) {
                        const double* p = Bp + (long long)k * pr.ldb + n0 + nn;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (n0 + nn + e < N) rb[u][e] = p[e];
                    }
                } else {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
                    int n = n0 + r;
                    if (n < N) {
                        const double* p = Bp + (long long)n * pr.ldb + k0 + kk;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (k0 + kk + e < K) rb[u][e] = p[e];
                    }
                }
            }
        }
    };

    auto store_slice = [&]() {
#pragma unroll
        for (int u = 0; u < AVT; ++u) {
            int v = tid + u * kT;
            if (v < AV) {
                if (!TA) {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) As[kk + e][r] = ra[u][e];
                } else {
                    int kr = v / (BM / 4), mm = (v % (BM / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) As[kr][mm + e] = ra[u][e];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < BVT; ++u) {
            int v = tid + u * kT;
            if (v < BV) {
                if (!TB) {
                    int kr = v / (BN / 4), nn = (v % (BN / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) Bs[kr][nn + e] = rb[u][e];
                } else {
                    int r = v / (BK / 4), kk = (v % (BK / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) Bs[kk + e][r] = rb[u][e];
                }
            }
        }
    };

    const int lr = lane & 15;
    const int lk = lane >> 4;
    const int wm0 = wm * FM * 16, wn0 = wn * FN * 16;
    const bool wave_live = m0 + wm0 < M && n0 + wn0 < N;

    if (K > 0) load_slice(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        store_slice();
        __syncthreads();
        if (k0 + BK < K) load_slice(k0 + BK);
#pragma unroll KS_UNROLL
        for (int ks = 0; ks < BK / 4; ++ks) {
            if (!wave_live) break;
            double a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[ks * 4 + lk][wm0 + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = Bs[ks * 4 + lk][wn0 + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }

    // accumulator element q of a lane: row 4*q + lane/16, column lane%16
    double* Cp = C + pr.c_off;
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
                double out = alpha * acc[i][j][q];
                double* c = Cp + (long long)row * pr.ldc + col;
                if (beta) out += *c;
                *c = out;
            }
        }
}

// tall products: B in LDS, one row of A per thread (as the complex form)
template <bool TB>
__global__ __launch_bounds__(256) void k_dtall(const double* __restrict__ A, const double* __restrict__ B,
                                               double* __restrict__ C, const ZProb* __restrict__ probs,
                                               const ZTile* __restrict__ tiles, double alpha, int beta,
                                               const int* __restrict__ active) {
    __shared__ double Bs[ZTALL_MAX_KN];
    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;
    const ZProb pr = probs[tl.prob];
    const int N = pr.N, K = pr.K;
    const double* Bp = B + pr.b_off;
    for (int e = threadIdx.x; e < K * N; e += kT) {
        const int k = e / N, n = e - k * N;
        Bs[e] = TB ? Bp[(long long)n * pr.ldb + k] : Bp[(long long)k * pr.ldb + n];
    }
    __syncthreads();
    const int m = tl.m0 + (int)threadIdx.x;
    if (m >= pr.M) return;
    const double* a = A + pr.a_off + (long long)m * pr.lda;
    double* c = C + pr.c_off + (long long)m * pr.ldc;
    for (int n0 = 0; n0 < N; n0 += 8) {
        double x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = 0.0;
        for (int k0 = 0; k0 < K; k0 += 8) {
            double av[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) av[j] = k0 + j < K ? a[k0 + j] : 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (k0 + j < K) {
                    const double* b = Bs + (k0 + j) * N + n0;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (n0 + q < N) x[q] += av[j] * b[q];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (n0 + q < N) {
                double out = alpha * x[q];
                if (beta) out += c[n0 + q];
                c[n0 + q] = out;
            }
    }
}

// reduction-shaped products: A chunk in LDS, P consecutive rows of B per step
template <bool TA, int MAXM, int U>
__global__ __launch_bounds__(256) void k_dred(const double* __restrict__ A, const double* __restrict__ B,
                                              double* __restrict__ C, const ZProb* __restrict__ probs,
                                              const ZTile* __restrict__ tiles, double alpha, int beta,
                                              const int* __restrict__ active) {
    __shared__ double As[ZRED_LDS];
    __shared__ double red[kT];
    const ZTile tl = tiles[blockIdx.x];
    if (active && !active[tl.sys]) return;
    const ZProb pr = probs[tl.prob];
    const int M = pr.M, N = pr.N, K = pr.K;
    if (M <= 0 || N <= 0) return;
    const int P = kT / N;
    const int tid = threadIdx.x, n = tid % N, kl = tid / N;
    const bool live = kl < P;
    const double* Ap = A + pr.a_off;
    const double* Bp = B + pr.b_off + n;
    for (int e = tid; e < M * K; e += kT) {
        int i, k;
        if (TA) {
            k = e / M;
            i = e - k * M;
        } else {
            i = e / K;
            k = e - i * K;
        }
        As[i * K + k] = TA ? Ap[(long long)k * pr.lda + i] : Ap[(long long)i * pr.lda + k];
    }
    __syncthreads();
    double x[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) x[i] = 0.0;
    auto fma_k = [&](const double b, int k) {
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
            if (i < M) x[i] += As[i * K + k] * b;
    };
    if (live) {
        const int step = U * P;
        int k = kl;
        double nb[U];
        if (k + (U - 1) * P < K) {
#pragma unroll
            for (int u = 0; u < U; ++u) nb[u] = Bp[(long long)(k + u * P) * pr.ldb];
        }
        for (; k + (U - 1) * P < K; k += step) {
            double cb[U];
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
    double* Cp = C + pr.c_off;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
        if (i >= M) break;
        __syncthreads();
        if (live) red[kl * N + n] = x[i];
        __syncthreads();
        if (tid < N) {
            double s = 0.0;
            for (int q = 0; q < P; ++q) s += red[q * N + tid];
            double out = alpha * s;
            double* c = Cp + (long long)i * pr.ldc + tid;
            if (beta) out += *c;
            *c = out;
        }
    }
}

template <int BM, int BN, int WM, int WN, int BK>
hipError_t dlaunch_cfg(bool tA, bool tB, const double* A, const double* B, double* C, const ZProb* probs,
                       const ZTile* tiles, int ntiles, double alpha, int beta, hipStream_t st, int role,
                       const int* active) {
    dim3 grid(ntiles), block(kT);
    if (!tA && !tB) {
        if (role == 2) k_dgemm<BM, BN, WM, WN, BK, false, false, 2><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        else k_dgemm<BM, BN, WM, WN, BK, false, false, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    } else if (!tA && tB) {
        if (role == 1) k_dgemm<BM, BN, WM, WN, BK, false, true, 1><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        else k_dgemm<BM, BN, WM, WN, BK, false, true, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    } else if (tA && !tB) {
        k_dgemm<BM, BN, WM, WN, BK, true, false, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    } else {
        k_dgemm<BM, BN, WM, WN, BK, true, true, 0><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
    }
    return hipGetLastError();
}

template <int BK>
hipError_t dlaunch_bk(int cfg, bool tA, bool tB, const double* A, const double* B, double* C, const ZProb* probs,
                      const ZTile* tiles, int ntiles, double alpha, int beta, hipStream_t st, int role,
                      const int* active) {
    switch (cfg) {
        case ZCFG_128x16: return dlaunch_cfg<128, 16, 4, 1, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_16x128: return dlaunch_cfg<16, 128, 1, 4, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_32x32: return dlaunch_cfg<32, 32, 2, 2, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x16: return dlaunch_cfg<64, 16, 4, 1, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_16x64: return dlaunch_cfg<16, 64, 1, 4, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x64: return dlaunch_cfg<64, 64, 2, 2, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_32x64: return dlaunch_cfg<32, 64, 2, 2, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x32: return dlaunch_cfg<64, 32, 2, 2, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x64R: return dlaunch_cfg<64, 64, 4, 1, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        case ZCFG_64x32R: return dlaunch_cfg<64, 32, 4, 1, BK>(tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// split-K pass, gathers, elementwise

__global__ __launch_bounds__(256) void k_dsplitk_reduce(double* __restrict__ C, const double* __restrict__ W,
                                                        const ZRed* __restrict__ reds, double alpha, int beta) {
    __shared__ double part[kT];
    const ZRed r = reds[blockIdx.y];
    const long long mn = (long long)r.M * r.N;
    const int o = threadIdx.x & 15, g = threadIdx.x >> 4;
    const long long e = (long long)blockIdx.x * 16 + o;
    double s = 0.0;
    if (e < mn) {
        const double* w = W + r.w_off + e;
        int q = g;
        for (; q + 48 < r.S; q += 64) {
            const double x0 = w[(long long)q * mn], x1 = w[(long long)(q + 16) * mn];
            const double x2 = w[(long long)(q + 32) * mn], x3 = w[(long long)(q + 48) * mn];
            s += x0;
            s += x1;
            s += x2;
            s += x3;
        }
        for (; q < r.S; q += 16) s += w[(long long)q * mn];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (g == 0 && e < mn) {
        s = 0.0;
        for (int q = 0; q < 16; ++q) s += part[q * 16 + o];
        const int m = (int)(e / r.N), n = (int)(e % r.N);
        double* c = C + r.c_off + (long long)m * r.ldc + n;
        double out = alpha * s;
        if (beta) out += *c;
        *c = out;
    }
}

// few K chunks: one output per thread, chunks summed in order
__global__ __launch_bounds__(256) void k_dsplitk_reduce_few(double* __restrict__ C, const double* __restrict__ W,
                                                            const ZRed* __restrict__ reds, double alpha, int beta) {
    const ZRed r = reds[blockIdx.y];
    const long long mn = (long long)r.M * r.N;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mn) return;
    const double* w = W + r.w_off + e;
    double s = 0.0;
    int q = 0;
    for (; q + 4 <= r.S; q += 4) {
        const double x0 = w[(long long)q * mn], x1 = w[(long long)(q + 1) * mn];
        const double x2 = w[(long long)(q + 2) * mn], x3 = w[(long long)(q + 3) * mn];
        s += x0;
        s += x1;
        s += x2;
        s += x3;
    }
    for (; q < r.S; ++q) s += w[(long long)q * mn];
    long long ci = e;   // contiguous rows: the output index is e
    if (r.ldc != r.N) {
        const unsigned ue = (unsigned)e, un = (unsigned)r.N;
        ci = (long long)(ue / un) * r.ldc + (ue % un);
    }
    double* c = C + r.c_off + ci;
    double out = alpha * s;
    if (beta) out += *c;
    *c = out;
}

__device__ __forceinline__ double dmap_load(const double* __restrict__ s, uint32_t m) {
    if (m == 0xFFFFFFFFu) return 0.0;
    const double x = s[m & 0x7FFFFFFFu];
    return (m & 0x80000000u) ? -x : x;
}

template <int NT, bool BIL>
__global__ __launch_bounds__(256) void k_dgather(double* __restrict__ dst, const double* __restrict__ src,
                                                 const double* __restrict__ src2, GatherMaps maps, long long n,
                                                 double alpha, int beta) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double x = dmap_load(maps.src[t] ? (const double*)maps.src[t] : src, maps.a[t][k]);
        if (BIL) x *= dmap_load(src2, maps.b[t][k]);
        s += x;
    }
    double out = alpha * s;
    if (beta) out += dst[k];
    dst[k] = out;
}

__global__ __launch_bounds__(256) void k_daxpby(double* __restrict__ dst, const double* __restrict__ src, long long n,
                                                double alpha, int beta) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double out = alpha * src[k];
    if (beta) out += dst[k];
    dst[k] = out;
}

__global__ __launch_bounds__(256) void k_ddiag(double* __restrict__ dst, const double* __restrict__ d,
                                               const double* __restrict__ src, long long n) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] -= d[k] * src[k];
}

__global__ __launch_bounds__(256) void k_dmul(double* __restrict__ dst, const double* __restrict__ d, long long n) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] *= d[k];
}

// ---------------------------------------------------------------------------
// reductions (deterministic: fixed grid, per-block partials, one final block)

__device__ __forceinline__ double dblock_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double dblock_max(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
            sh[threadIdx.x] = (a > b || a != a) ? a : b;
        }
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double ddyn_delta(double d, double S, int n) {
    const double q = S / (fmin(d, 0.0) + S);
    double p = q;
    for (int i = 1; i < n; ++i) p *= q;
    return S * p;
}

__global__ __launch_bounds__(256) void k_djacobi(const double* __restrict__ t, const double* __restrict__ r,
                                                 const double* __restrict__ D, double* __restrict__ ht,
                                                 double* __restrict__ he, long long n, double* part_max,
                                                 double shift, double dS, int dn) {
    __shared__ double sh[kT];
    double mx = 0.0;
    for (long long k = (long long)blockIdx.x * kT + threadIdx.x; k < n; k += (long long)gridDim.x * kT) {
        double rr = r[k];
        const double tt = t[k];
        double d = D[k];
        if (dS != 0.0) {
            const double dl = ddyn_delta(d, dS, dn);
            rr -= dl * tt;
            d += dl;
        }
        d -= shift;
        const double s = rr / d;
        he[k] = s;
        ht[k] = tt + s;
        const double a = fabs(s);
        mx = (a > mx || a != a) ? a : mx;
    }
    double b = dblock_max(mx, sh);
    if (threadIdx.x == 0) part_max[blockIdx.x] = b;
}

struct DPtrList {
    const double* p[kDiisMax];
};

__global__ __launch_bounds__(256) void k_ddots(DPtrList e, int m, const double* __restrict__ enew, long long n,
                                               double* part) {
    __shared__ double sh[kT];
    double acc[kDiisMax];
#pragma unroll
    for (int j = 0; j < kDiisMax; ++j) acc[j] = 0.0;
    for (long long k = (long long)blockIdx.x * kT + threadIdx.x; k < n; k += (long long)gridDim.x * kT) {
        const double y = enew[k];
#pragma unroll
        for (int j = 0; j < kDiisMax; ++j)
            if (j < m) acc[j] += e.p[j][k] * y;
    }
#pragma unroll
    for (int j = 0; j < kDiisMax; ++j)
        if (j < m) {
            double b = dblock_sum(acc[j], sh);
            if (threadIdx.x == 0) part[blockIdx.x * kDiisMax + j] = b;
        }
}

// out = sum_j coef[j] xs[j]; coef[m] != 0 (a non-finite step) leaves out untouched
__global__ __launch_bounds__(256) void k_dlincomb(double* __restrict__ out, DPtrList xs, const double* __restrict__ coef,
                                                  int m, long long n) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || coef[m] != 0.0) return;
    double s = 0.0;
    for (int j = 0; j < m; ++j) {
        const double c = coef[j];
        if (c != 0.0) s += c * xs.p[j][k];
    }
    out[k] = s;
}

__global__ __launch_bounds__(256) void k_ddot_part(const double* __restrict__ x, const double* __restrict__ y,
                                                   long long n, double* part) {
    __shared__ double sh[kT];
    double s = 0.0;
    for (long long k = (long long)blockIdx.x * kT + threadIdx.x; k < n; k += (long long)gridDim.x * kT) s += x[k] * y[k];
    double r = dblock_sum(s, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r;
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_dsum(const double* __restrict__ part, int nblk, double* out) {
    __shared__ double sh[kT];
    double r = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kT) r += part[2 * b];
    r = dblock_sum(r, sh);
    if (threadIdx.x == 0) {
        out[0] = r;
        out[1] = 0.0;
    }
}

inline unsigned grid_of(long long n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

hipError_t launch_dgemm(int cfg, int bk, bool tA, bool tB, const double* A, const double* B, double* C,
                        const ZProb* probs, const ZTile* tiles, int ntiles, double alpha, int beta, hipStream_t st,
                        int role, const int* active, int max_m, int lds) {
    if (ntiles <= 0) return hipSuccess;
    if (lds == LDS_DIRECT) {
        if (bk != 16 || !zcfg_has_dl(cfg)) return hipErrorInvalidValue;
        return launch_dgemm_dl(cfg, tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
    }
    if (lds != LDS_STAGED) return hipErrorInvalidValue;
    dim3 grid(ntiles), block(kT);
    if (cfg == ZCFG_TALL) {
        if (tA) return hipErrorInvalidValue;
        if (tB) k_dtall<true><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        else k_dtall<false><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        return hipGetLastError();
    }
    if (cfg == ZCFG_RED) {
        if (tB || max_m < 1 || max_m > ZRED_MAX_M) return hipErrorInvalidValue;
        if (max_m <= 2) {
            if (tA) k_dred<true, 2, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
            else k_dred<false, 2, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        } else if (max_m <= 4) {
            if (tA) k_dred<true, 4, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
            else k_dred<false, 4, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        } else {
            if (tA) k_dred<true, 8, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
            else k_dred<false, 8, 8><<<grid, block, 0, st>>>(A, B, C, probs, tiles, alpha, beta, active);
        }
        return hipGetLastError();
    }
    if (bk == 32) return dlaunch_bk<32>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
    if (bk == 16) return dlaunch_bk<16>(cfg, tA, tB, A, B, C, probs, tiles, ntiles, alpha, beta, st, role, active);
    return hipErrorInvalidValue;
}

hipError_t launch_dsplitk_reduce(double* C, const double* W, const ZRed* reds, int nred, int maxMN, int maxS,
                                 double alpha, int beta, hipStream_t st) {
    if (nred <= 0 || maxMN <= 0) return hipSuccess;
    if (maxS <= ZRED_FEW_S) {
        dim3 grid((unsigned)((maxMN + kT - 1) / kT), (unsigned)nred);
        k_dsplitk_reduce_few<<<grid, kT, 0, st>>>(C, W, reds, alpha, beta);
    } else {
        dim3 grid((unsigned)((maxMN + 15) / 16), (unsigned)nred);
        k_dsplitk_reduce<<<grid, kT, 0, st>>>(C, W, reds, alpha, beta);
    }
    return hipGetLastError();
}

hipError_t launch_dgather(double* dst, const double* src, const double* src2, GatherMaps maps, int nt, long long n,
                          double alpha, int beta, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const bool bil = src2 != nullptr;
#define FSCC_DG(NT)                                                                                     \
    if (bil) k_dgather<NT, true><<<grid_of(n), kT, 0, st>>>(dst, src, src2, maps, n, alpha, beta);     \
    else k_dgather<NT, false><<<grid_of(n), kT, 0, st>>>(dst, src, src2, maps, n, alpha, beta);
    switch (nt) {
        case 1: FSCC_DG(1); break;
        case 2: FSCC_DG(2); break;
        case 3: FSCC_DG(3); break;
        case 4: FSCC_DG(4); break;
        default: return hipErrorInvalidValue;
    }
#undef FSCC_DG
    return hipGetLastError();
}

hipError_t launch_daxpby(double* dst, const double* src, long long n, double alpha, int beta, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_daxpby<<<grid_of(n), kT, 0, st>>>(dst, src, n, alpha, beta);
    return hipGetLastError();
}

hipError_t launch_ddiag(double* dst, const double* d, const double* src, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_ddiag<<<grid_of(n), kT, 0, st>>>(dst, d, src, n);
    return hipGetLastError();
}

hipError_t launch_dmul(double* dst, const double* d, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_dmul<<<grid_of(n), kT, 0, st>>>(dst, d, n);
    return hipGetLastError();
}

hipError_t launch_djacobi(const double* t, const double* r, const double* D, double* hist_t, double* hist_e,
                          long long n, double* part_max, int nblk, hipStream_t st, double shift, double dyn_S,
                          int dyn_n) {
    if (dyn_S != 0.0 && !(dyn_S < 0.0 && dyn_n >= 1)) return hipErrorInvalidValue;
    k_djacobi<<<nblk, kT, 0, st>>>(t, r, D, hist_t, hist_e, n, part_max, shift, dyn_S, dyn_n);
    return hipGetLastError();
}

hipError_t launch_ddots(const double* const* e, int m, const double* enew, long long n, double* part, int nblk,
                        hipStream_t st) {
    if (m < 0 || m > kDiisMax) return hipErrorInvalidValue;
    DPtrList pl;
    for (int j = 0; j < kDiisMax; ++j) pl.p[j] = j < m ? e[j] : nullptr;
    k_ddots<<<nblk, kT, 0, st>>>(pl, m, enew, n, part);
    return hipGetLastError();
}

hipError_t launch_dlincomb(double* out, const double* const* xs, const double* coef, int m, long long n,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (m < 0 || m > kDiisMax) return hipErrorInvalidValue;
    DPtrList pl;
    for (int j = 0; j < kDiisMax; ++j) pl.p[j] = j < m ? xs[j] : nullptr;
    k_dlincomb<<<grid_of(n), kT, 0, st>>>(out, pl, coef, m, n);
    return hipGetLastError();
}

hipError_t launch_ddot(const double* x, const double* y, long long n, double* part, int nblk, double* out,
                       hipStream_t st) {
    k_ddot_part<<<nblk, kT, 0, st>>>(x, y, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_dsum<<<1, kT, 0, st>>>(part, nblk, out);
    return hipGetLastError();
}

}  // namespace fscc
