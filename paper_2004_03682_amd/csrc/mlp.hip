// mlp.hip -- learned warm start: features, a 3-layer FP32 MLP (8 -> 256 ->
// 256 -> 4) with hand-written forward / backward / Adam kernels on the fp32
// matrix cores (v_mfma_f32_16x16x4_f32), and the amplitude head.
//
// Per packed T2 element: u = MP2 amplitude, r = residual at u, D = its
// denominator, v = r / D (the next Jacobi correction), s = |u| + |v| + 1e-30;
// features x = (Re u/s, Im u/s, Re v/s, Im v/s, clip(ln((|v|+1e-30)/(|u|+1e-30)),
// -10, 10)/10, D/10, ln(s)/10, |v|/s); the network output y gives
// a = y0 + i y1, b = y2 + i y3 and the prediction t = u + v + a v + b u; the
// training loss is mean |t - t_converged|^2 / s^2 (relative) or
// sum |t - t_converged|^2 / sum s^2 (absolute).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fscc.h"
#include "kernels.hpp"

namespace fscc {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kT = 256;
constexpr int F_IN = 8, HID = 256, F_OUT = 4;
// flat parameter layout: W1 [8][256], b1, W2 [256][256], b2, W3 [256][4], b3
constexpr size_t OFF_W1 = 0, OFF_B1 = OFF_W1 + F_IN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
                 OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * F_OUT, N_PARAMS = OFF_B3 + F_OUT;

enum SgEpi { SG_PLAIN = 0, SG_BIAS_RELU = 1, SG_BIAS = 2, SG_MASK = 3 };

// C = op(A) op(B) (+ epilogue); op(A)(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// op(B)(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  64x64 tiles, 4 waves of 32x32.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_sgemm(const float* __restrict__ A, const float* __restrict__ B,
                                               float* __restrict__ C, int M, int N, int K, int lda, int ldb, int ldc,
                                               const float* __restrict__ bias, const float* __restrict__ mask, int ldm) {
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
    f4v c[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) c[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * kT;
            int mm, kk;
            if (!TA) {
                mm = idx / BK;
                kk = idx % BK;
            } else {
                kk = idx / BM;
                mm = idx % BM;
            }
            const int gm = m0 + mm, gk = k0 + kk;
            float v = 0.f;
            if (gm < M && gk < K) v = TA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
            As[kk][mm] = v;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * kT;
            int nn, kk;
            if (!TB) {
                kk = idx / BN;
                nn = idx % BN;
            } else {
                nn = idx / BK;
                kk = idx % BK;
            }
            const int gn = n0 + nn, gk = k0 + kk;
            float v = 0.f;
            if (gn < N && gk < K) v = TB ? B[(long long)gn * ldb + gk] : B[(long long)gk * ldb + gn];
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[ks + (lane >> 4)][wm0 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[ks + (lane >> 4)][wn0 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) c[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], c[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // fp32-accumulating MFMA: accumulator element q is row 4*(lane/16) + q, column lane%16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn0 + j * 16 + (lane & 15);
            if (col >= N) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm0 + i * 16 + 4 * (lane >> 4) + q;
                if (row >= M) continue;
                float v = c[i][j][q];
                if (EPI == SG_BIAS_RELU) v = fmaxf(v + bias[col], 0.f);
                if (EPI == SG_BIAS) v += bias[col];
                if (EPI == SG_MASK) v = mask[(long long)row * ldm + col] > 0.f ? v : 0.f;
                C[(long long)row * ldc + col] = v;
            }
        }
}

template <bool TA, bool TB, int EPI>
hipError_t sgemm(const float* A, const float* B, float* C, int M, int N, int K, int lda, int ldb, int ldc,
                 const float* bias, const float* mask, int ldm, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    k_sgemm<TA, TB, EPI><<<grid, kT, 0, st>>>(A, B, C, M, N, K, lda, ldb, ldc, bias, mask, ldm);
    return hipGetLastError();
}

__device__ inline void ws_v_s(double2 u, double2 r, double d, double2* v, double* s) {
    *v = make_double2(r.x / d, r.y / d);
    *s = hypot(u.x, u.y) + hypot(v->x, v->y) + 1e-30;
}

__global__ __launch_bounds__(256) void k_ws_features(const double2* __restrict__ u, const double2* __restrict__ r,
                                                     const double* __restrict__ D, long long n, float* __restrict__ X) {
    const long long k = (long long)blockIdx.x * kT + threadIdx.x;
    if (k >= n) return;
    const double2 uu = u[k];
    double2 v;
    double s;
    const double d = D[k];
    ws_v_s(uu, r[k], d, &v, &s);
    const double au = hypot(uu.x, uu.y), av = hypot(v.x, v.y);
    const double lr = fmin(fmax(log((av + 1e-30) / (au + 1e-30)), -10.0), 10.0);
    float* x = X + k * F_IN;
    x[0] = (float)(uu.x / s);
    x[1] = (float)(uu.y / s);
    x[2] = (float)(v.x / s);
    x[3] = (float)(v.y / s);
    x[4] = (float)(lr / 10.0);
    x[5] = (float)(d / 10.0);
    x[6] = (float)(log(s) / 10.0);
    x[7] = (float)(av / s);
}

// prediction u + v + a v + b u  (Y may be null: a = b = 0)
__global__ __launch_bounds__(256) void k_ws_apply(const float* __restrict__ Y, const double2* __restrict__ u,
                                                  const double2* __restrict__ r, const double* __restrict__ D,
                                                  long long n, double2* __restrict__ out) {
    const long long k = (long long)blockIdx.x * kT + threadIdx.x;
    if (k >= n) return;
    const double2 uu = u[k];
    double2 v;
    double s;
    ws_v_s(uu, r[k], D[k], &v, &s);
    double ar = 0, ai = 0, br = 0, bi = 0;
    if (Y) {
        ar = Y[k * F_OUT];
        ai = Y[k * F_OUT + 1];
        br = Y[k * F_OUT + 2];
        bi = Y[k * F_OUT + 3];
    }
    out[k] = make_double2(uu.x + v.x + (ar * v.x - ai * v.y) + (br * uu.x - bi * uu.y),
                          uu.y + v.y + (ar * v.y + ai * v.x) + (br * uu.y + bi * uu.x));
}

// per-block partial sums of s^2 (the absolute loss normaliser)
__global__ __launch_bounds__(256) void k_ws_s2(const double2* __restrict__ u, const double2* __restrict__ r,
                                               const double* __restrict__ D, long long n, double* __restrict__ part) {
    __shared__ double sh[kT];
    const long long k = (long long)blockIdx.x * kT + threadIdx.x;
    double q = 0.0;
    if (k < n) {
        double2 v;
        double s;
        ws_v_s(u[k], r[k], D[k], &v, &s);
        q = s * s;
    }
    sh[threadIdx.x] = q;
    __syncthreads();
    for (int s2 = kT / 2; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// loss rows and dL/dy; weight w_k = 1/(n s_k^2) (mode 0) or 1/sum s^2 (mode 1,
// *norm holds sum s^2); per-block loss partials (already weighted)
__global__ __launch_bounds__(256) void k_ws_head(const float* __restrict__ Y, const double2* __restrict__ u,
                                                 const double2* __restrict__ r, const double* __restrict__ D,
                                                 const double2* __restrict__ t, long long n, int mode,
                                                 const double* __restrict__ norm, float* __restrict__ dY,
                                                 double* __restrict__ part) {
    __shared__ double sh[kT];
    const long long k = (long long)blockIdx.x * kT + threadIdx.x;
    double l = 0.0;
    if (k < n) {
        const double2 uu = u[k];
        double2 v;
        double s;
        ws_v_s(uu, r[k], D[k], &v, &s);
        const double ar = Y[k * F_OUT], ai = Y[k * F_OUT + 1], br = Y[k * F_OUT + 2], bi = Y[k * F_OUT + 3];
        const double2 tt = t[k];
        const double er = uu.x + v.x + (ar * v.x - ai * v.y) + (br * uu.x - bi * uu.y) - tt.x;
        const double ei = uu.y + v.y + (ar * v.y + ai * v.x) + (br * uu.y + bi * uu.x) - tt.y;
        const double w = mode == 0 ? 1.0 / (s * s) / (double)n : 1.0 / *norm;
        l = (er * er + ei * ei) * w;
        const double f = 2.0 * w;
        // conj(e) * v = (er v.x + ei v.y) + i (er v.y - ei v.x)
        dY[k * F_OUT] = (float)(f * (er * v.x + ei * v.y));
        dY[k * F_OUT + 1] = (float)(-f * (er * v.y - ei * v.x));
        dY[k * F_OUT + 2] = (float)(f * (er * uu.x + ei * uu.y));
        dY[k * F_OUT + 3] = (float)(-f * (er * uu.y - ei * uu.x));
    }
    sh[threadIdx.x] = l;
    __syncthreads();
    for (int s2 = kT / 2; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nblk, double scale,
                                                   double* __restrict__ out) {
    __shared__ double sh[kT];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kT) v += part[b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s2 = kT / 2; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] * scale;
}

// column sums of H [M][N] in two deterministic passes: partial[chunk][col]
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ H, int M, int N, int rows_per,
                                                     float* __restrict__ part) {
    const int col = blockIdx.x * kT + threadIdx.x;
    const int chunk = blockIdx.y;
    if (col >= N) return;
    const int r0 = chunk * rows_per, r1 = min(M, r0 + rows_per);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += H[(long long)r * N + col];
    part[(long long)chunk * N + col] = s;
}

__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ part, int nchunk, int N,
                                                      float* __restrict__ out) {
    const int col = blockIdx.x * kT + threadIdx.x;
    if (col >= N) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += part[(long long)c * N + col];
    out[col] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ w, long long n, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
    const long long k = (long long)blockIdx.x * kT + threadIdx.x;
    if (k >= n) return;
    const float gg = g[k];
    const float mm = b1 * m[k] + (1.f - b1) * gg;
    const float ww = b2 * w[k] + (1.f - b2) * gg * gg;
    m[k] = mm;
    w[k] = ww;
    p[k] -= lr * (mm / bc1) / (sqrtf(ww / bc2) + eps);
}

__global__ __launch_bounds__(256) void k_gather_rows(const unsigned char* __restrict__ src, int eb,
                                                     const long long* __restrict__ idx, long long n,
                                                     unsigned char* __restrict__ dst) {
    const long long k = (long long)blockIdx.x * kT + threadIdx.x;
    if (k >= n) return;
    const long long i = idx[k];
    if (eb == 16) ((double2*)dst)[k] = ((const double2*)src)[i];
    else ((double*)dst)[k] = ((const double*)src)[i];
}

__global__ __launch_bounds__(256) void k_ws_step(const double2* __restrict__ t, const double2* __restrict__ r,
                                                 const double* __restrict__ D, long long n, double2* __restrict__ out) {
    const long long k = (long long)blockIdx.x * kT + threadIdx.x;
    if (k >= n) return;
    const double d = D[k];
    const double2 tt = t ? t[k] : make_double2(0.0, 0.0), rr = r[k];
    out[k] = make_double2(tt.x + rr.x / d, tt.y + rr.y / d);
}

unsigned grid1(long long n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace
}  // namespace fscc

using namespace fscc;

struct fscc_mlp {
    hipStream_t st = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *w = nullptr;
    long long step = 0;
    // training scratch (rows <= maxb)
    size_t maxb = 0;
    float *X = nullptr, *h1 = nullptr, *h2 = nullptr, *dh1 = nullptr, *dh2 = nullptr, *Y = nullptr, *dY = nullptr,
          *cpart = nullptr;
    double *part = nullptr, *loss = nullptr, *bD = nullptr;
    double2 *bu = nullptr, *br = nullptr, *bt = nullptr;
    // inference scratch (chunk rows)
    size_t chunk = 0;
    float *ih1 = nullptr, *ih2 = nullptr;
    double* hloss = nullptr;
    std::string err;

    void free_train() {
        void* ps[] = {X, h1, h2, dh1, dh2, Y, dY, cpart, part, loss, bD, bu, br, bt};
        for (void* q : ps)
            if (q) (void)hipFree(q);
        X = h1 = h2 = dh1 = dh2 = Y = dY = cpart = nullptr;
        part = loss = bD = nullptr;
        bu = br = bt = nullptr;
        maxb = 0;
    }
    ~fscc_mlp() {
        if (st) (void)hipStreamSynchronize(st);
        else (void)hipDeviceSynchronize();
        free_train();
        void* ps[] = {p, g, m, w, ih1, ih2};
        for (void* q : ps)
            if (q) (void)hipFree(q);
        if (hloss) (void)hipHostFree(hloss);
    }
};

namespace {

bool ok(hipError_t e) { return e == hipSuccess; }

fscc_status herr(fscc_mlp* n, hipError_t e, const char* what) {
    if (n) n->err = std::string(what) + ": " + hipGetErrorString(e);
    return FSCC_EHIP;
}

template <class T>
hipError_t dalloc(T** q, size_t count) {
    return hipMalloc((void**)q, sizeof(T) * (count ? count : 1));
}

hipError_t ensure_train(fscc_mlp* n, size_t rows) {
    if (rows <= n->maxb) return hipSuccess;
    n->free_train();
    size_t b = 1024;
    while (b < rows) b *= 2;
    hipError_t e = hipSuccess;
    if (ok(e)) e = dalloc(&n->X, b * F_IN);
    if (ok(e)) e = dalloc(&n->h1, b * HID);
    if (ok(e)) e = dalloc(&n->h2, b * HID);
    if (ok(e)) e = dalloc(&n->dh1, b * HID);
    if (ok(e)) e = dalloc(&n->dh2, b * HID);
    if (ok(e)) e = dalloc(&n->Y, b * F_OUT);
    if (ok(e)) e = dalloc(&n->dY, b * F_OUT);
    if (ok(e)) e = dalloc(&n->cpart, ((b + 255) / 256) * HID);
    if (ok(e)) e = dalloc(&n->part, (b + 255) / 256);
    if (ok(e)) e = dalloc(&n->loss, 2);
    if (ok(e)) e = dalloc(&n->bD, b);
    if (ok(e)) e = dalloc(&n->bu, b);
    if (ok(e)) e = dalloc(&n->br, b);
    if (ok(e)) e = dalloc(&n->bt, b);
    if (ok(e)) n->maxb = b;
    return e;
}

// h1, h2, Y of `rows` feature rows X
hipError_t forward_rows(fscc_mlp* n, const float* X, size_t rows, float* h1, float* h2, float* Y) {
    const float* P = n->p;
    const int M = (int)rows;
    hipError_t e = sgemm<false, false, SG_BIAS_RELU>(X, P + OFF_W1, h1, M, HID, F_IN, F_IN, HID, HID, P + OFF_B1,
                                                     nullptr, 0, n->st);
    if (ok(e)) e = sgemm<false, false, SG_BIAS_RELU>(h1, P + OFF_W2, h2, M, HID, HID, HID, HID, HID, P + OFF_B2,
                                                     nullptr, 0, n->st);
    if (ok(e)) e = sgemm<false, false, SG_BIAS>(h2, P + OFF_W3, Y, M, F_OUT, HID, HID, F_OUT, F_OUT, P + OFF_B3,
                                                nullptr, 0, n->st);
    return e;
}

hipError_t colsum(fscc_mlp* n, const float* H, int M, int N, float* out) {
    const int rows_per = 256, nchunk = (M + rows_per - 1) / rows_per;
    if (nchunk == 0) return hipMemsetAsync(out, 0, sizeof(float) * N, n->st);
    k_colsum_part<<<dim3((N + kT - 1) / kT, nchunk), kT, 0, n->st>>>(H, M, N, rows_per, n->cpart);
    k_colsum_final<<<(N + kT - 1) / kT, kT, 0, n->st>>>(n->cpart, nchunk, N, out);
    return hipGetLastError();
}

// forward + loss + backward on the staged rows (bu, br, bD, bt) -> n->g, n->loss
hipError_t loss_grad_staged(fscc_mlp* n, size_t rows, int mode) {
    const int M = (int)rows;
    const float* P = n->p;
    float* G = n->g;
    hipStream_t st = n->st;
    k_ws_features<<<grid1(M), kT, 0, st>>>(n->bu, n->br, n->bD, M, n->X);
    hipError_t e = hipGetLastError();
    if (ok(e)) e = forward_rows(n, n->X, rows, n->h1, n->h2, n->Y);
    if (!ok(e)) return e;
    if (mode == 1) {
        k_ws_s2<<<grid1(M), kT, 0, st>>>(n->bu, n->br, n->bD, M, n->part);
        k_sum_parts<<<1, kT, 0, st>>>(n->part, (int)grid1(M), 1.0, n->loss + 1);
    }
    k_ws_head<<<grid1(M), kT, 0, st>>>(n->Y, n->bu, n->br, n->bD, n->bt, M, mode, n->loss + 1, n->dY, n->part);
    k_sum_parts<<<1, kT, 0, st>>>(n->part, (int)grid1(M), 1.0, n->loss);
    e = hipGetLastError();
    // W3, b3
    if (ok(e)) e = sgemm<true, false, SG_PLAIN>(n->h2, n->dY, G + OFF_W3, HID, F_OUT, M, HID, F_OUT, F_OUT, nullptr,
                                                nullptr, 0, st);
    if (ok(e)) e = colsum(n, n->dY, M, F_OUT, G + OFF_B3);
    // dh2 = (dY W3^T) o (h2 > 0)
    if (ok(e)) e = sgemm<false, true, SG_MASK>(n->dY, P + OFF_W3, n->dh2, M, HID, F_OUT, F_OUT, F_OUT, HID, nullptr,
                                               n->h2, HID, st);
    if (ok(e)) e = sgemm<true, false, SG_PLAIN>(n->h1, n->dh2, G + OFF_W2, HID, HID, M, HID, HID, HID, nullptr,
                                                nullptr, 0, st);
    if (ok(e)) e = colsum(n, n->dh2, M, HID, G + OFF_B2);
    // dh1 = (dh2 W2^T) o (h1 > 0)
    if (ok(e)) e = sgemm<false, true, SG_MASK>(n->dh2, P + OFF_W2, n->dh1, M, HID, HID, HID, HID, HID, nullptr,
                                               n->h1, HID, st);
    if (ok(e)) e = sgemm<true, false, SG_PLAIN>(n->X, n->dh1, G + OFF_W1, F_IN, HID, M, F_IN, HID, HID, nullptr,
                                                nullptr, 0, st);
    if (ok(e)) e = colsum(n, n->dh1, M, HID, G + OFF_B1);
    return e;
}

hipError_t adam(fscc_mlp* n, float lr) {
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)n->step));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)n->step));
    k_adam<<<grid1(N_PARAMS), kT, 0, n->st>>>(n->p, n->g, n->m, n->w, (long long)N_PARAMS, lr, b1, b2, 1e-8f, bc1,
                                             bc2);
    return hipGetLastError();
}

// SplitMix64 (Steele, Lea, Flood 2014) + Box-Muller for the initial weights
struct InitRng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double normal() {
        const double u1 = ((double)(next() >> 11) + 1.0) * 0x1.0p-53, u2 = (double)(next() >> 11) * 0x1.0p-53;
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

}  // namespace

extern "C" {

fscc_status fscc_mlp_num_params(size_t* n) {
    if (!n) return FSCC_EINVAL;
    *n = N_PARAMS;
    return FSCC_OK;
}

fscc_status fscc_mlp_create(uint64_t seed, void* hip_stream, fscc_mlp** out) {
    if (!out) return FSCC_EINVAL;
    *out = nullptr;
    fscc_mlp* n = new (std::nothrow) fscc_mlp();
    if (!n) return FSCC_ENOMEM;
    n->st = (hipStream_t)hip_stream;
    hipError_t e = dalloc(&n->p, N_PARAMS);
    if (ok(e)) e = dalloc(&n->g, N_PARAMS);
    if (ok(e)) e = dalloc(&n->m, N_PARAMS);
    if (ok(e)) e = dalloc(&n->w, N_PARAMS);
    if (ok(e)) e = hipHostMalloc((void**)&n->hloss, sizeof(double), hipHostMallocDefault);
    if (ok(e)) {
        std::vector<float> h(N_PARAMS, 0.f);
        InitRng r{seed};
        const double s1 = std::sqrt(2.0 / F_IN), s2 = std::sqrt(2.0 / HID);
        for (size_t k = 0; k < (size_t)F_IN * HID; ++k) h[OFF_W1 + k] = (float)(s1 * r.normal());
        for (size_t k = 0; k < (size_t)HID * HID; ++k) h[OFF_W2 + k] = (float)(s2 * r.normal());
        std::vector<float> z(N_PARAMS, 0.f);
        e = hipMemcpy(n->p, h.data(), sizeof(float) * N_PARAMS, hipMemcpyHostToDevice);
        if (ok(e)) e = hipMemcpy(n->m, z.data(), sizeof(float) * N_PARAMS, hipMemcpyHostToDevice);
        if (ok(e)) e = hipMemcpy(n->w, z.data(), sizeof(float) * N_PARAMS, hipMemcpyHostToDevice);
        if (ok(e)) e = hipMemcpy(n->g, z.data(), sizeof(float) * N_PARAMS, hipMemcpyHostToDevice);
    }
    if (!ok(e)) {
        delete n;
        return e == hipErrorOutOfMemory ? FSCC_ENOMEM : FSCC_EHIP;
    }
    *out = n;
    return FSCC_OK;
}

void fscc_mlp_destroy(fscc_mlp* n) { delete n; }

const char* fscc_mlp_last_error(const fscc_mlp* n) { return n ? n->err.c_str() : "null network"; }

fscc_status fscc_mlp_set_params(fscc_mlp* n, const float* host, size_t count) {
    if (!n || !host || count != N_PARAMS) return FSCC_EINVAL;
    std::vector<float> z(N_PARAMS, 0.f);
    hipError_t e = hipMemcpy(n->p, host, sizeof(float) * N_PARAMS, hipMemcpyHostToDevice);
    if (ok(e)) e = hipMemcpy(n->m, z.data(), sizeof(float) * N_PARAMS, hipMemcpyHostToDevice);
    if (ok(e)) e = hipMemcpy(n->w, z.data(), sizeof(float) * N_PARAMS, hipMemcpyHostToDevice);
    n->step = 0;
    return ok(e) ? FSCC_OK : herr(n, e, "set params");
}

fscc_status fscc_mlp_get_params(fscc_mlp* n, float* host, size_t count) {
    if (!n || !host || count != N_PARAMS) return FSCC_EINVAL;
    hipError_t e = hipStreamSynchronize(n->st);
    if (ok(e)) e = hipMemcpy(host, n->p, sizeof(float) * N_PARAMS, hipMemcpyDeviceToHost);
    return ok(e) ? FSCC_OK : herr(n, e, "get params");
}

fscc_status fscc_mlp_get_grad(fscc_mlp* n, float* host, size_t count) {
    if (!n || !host || count != N_PARAMS) return FSCC_EINVAL;
    hipError_t e = hipStreamSynchronize(n->st);
    if (ok(e)) e = hipMemcpy(host, n->g, sizeof(float) * N_PARAMS, hipMemcpyDeviceToHost);
    return ok(e) ? FSCC_OK : herr(n, e, "get grad");
}

fscc_status fscc_ws_features(const fscc_c128* u, const fscc_c128* r, const double* D, size_t n, float* X,
                             void* hip_stream) {
    if (n && (!u || !r || !D || !X)) return FSCC_EINVAL;
    if (!n) return FSCC_OK;
    k_ws_features<<<grid1((long long)n), kT, 0, (hipStream_t)hip_stream>>>((const double2*)u, (const double2*)r, D,
                                                                           (long long)n, X);
    return ok(hipGetLastError()) ? FSCC_OK : FSCC_EHIP;
}

fscc_status fscc_ws_apply(const float* Y, const fscc_c128* u, const fscc_c128* r, const double* D, size_t n,
                          fscc_c128* out, void* hip_stream) {
    if (n && (!u || !r || !D || !out)) return FSCC_EINVAL;
    if (!n) return FSCC_OK;
    k_ws_apply<<<grid1((long long)n), kT, 0, (hipStream_t)hip_stream>>>(Y, (const double2*)u, (const double2*)r, D,
                                                                        (long long)n, (double2*)out);
    return ok(hipGetLastError()) ? FSCC_OK : FSCC_EHIP;
}

fscc_status fscc_ws_step(const fscc_c128* t, const fscc_c128* r, const double* D, size_t n, fscc_c128* out,
                         void* hip_stream) {
    if (n && (!r || !D || !out)) return FSCC_EINVAL;
    if (!n) return FSCC_OK;
    k_ws_step<<<grid1((long long)n), kT, 0, (hipStream_t)hip_stream>>>((const double2*)t, (const double2*)r, D,
                                                                       (long long)n, (double2*)out);
    return ok(hipGetLastError()) ? FSCC_OK : FSCC_EHIP;
}

fscc_status fscc_ws_gather(const void* src, size_t elem_bytes, const int64_t* idx, size_t n, void* dst,
                           void* hip_stream) {
    if ((elem_bytes != 8 && elem_bytes != 16) || (n && (!src || !idx || !dst))) return FSCC_EINVAL;
    if (!n) return FSCC_OK;
    k_gather_rows<<<grid1((long long)n), kT, 0, (hipStream_t)hip_stream>>>(
        (const unsigned char*)src, (int)elem_bytes, (const long long*)idx, (long long)n, (unsigned char*)dst);
    return ok(hipGetLastError()) ? FSCC_OK : FSCC_EHIP;
}

fscc_status fscc_mlp_forward(fscc_mlp* n, const float* X, size_t rows, float* Y) {
    if (!n || (rows && (!X || !Y))) return FSCC_EINVAL;
    const size_t ch = (size_t)1 << 20;
    hipError_t e = hipSuccess;
    if (!n->ih1) {
        e = dalloc(&n->ih1, ch * HID);
        if (ok(e)) e = dalloc(&n->ih2, ch * HID);
        if (!ok(e)) return herr(n, e, "inference scratch");
        n->chunk = ch;
    }
    for (size_t r0 = 0; r0 < rows && ok(e); r0 += ch) {
        const size_t m = rows - r0 < ch ? rows - r0 : ch;
        e = forward_rows(n, X + r0 * F_IN, m, n->ih1, n->ih2, Y + r0 * F_OUT);
    }
    return ok(e) ? FSCC_OK : herr(n, e, "forward");
}

fscc_status fscc_mlp_loss_grad(fscc_mlp* n, const fscc_c128* u, const fscc_c128* r, const double* D,
                               const fscc_c128* t, const int64_t* idx, size_t rows, int mode, double* loss) {
    if (!n || !loss || rows == 0 || !u || !r || !D || !t || rows > (size_t)1 << 24 || mode < 0 || mode > 1)
        return FSCC_EINVAL;
    hipError_t e = ensure_train(n, rows);
    if (!ok(e)) return herr(n, e, "training scratch");
    hipStream_t st = n->st;
    if (idx) {
        k_gather_rows<<<grid1(rows), kT, 0, st>>>((const unsigned char*)u, 16, (const long long*)idx, rows,
                                                  (unsigned char*)n->bu);
        k_gather_rows<<<grid1(rows), kT, 0, st>>>((const unsigned char*)r, 16, (const long long*)idx, rows,
                                                  (unsigned char*)n->br);
        k_gather_rows<<<grid1(rows), kT, 0, st>>>((const unsigned char*)t, 16, (const long long*)idx, rows,
                                                  (unsigned char*)n->bt);
        k_gather_rows<<<grid1(rows), kT, 0, st>>>((const unsigned char*)D, 8, (const long long*)idx, rows,
                                                  (unsigned char*)n->bD);
    } else {
        e = hipMemcpyAsync(n->bu, u, 16 * rows, hipMemcpyDeviceToDevice, st);
        if (ok(e)) e = hipMemcpyAsync(n->br, r, 16 * rows, hipMemcpyDeviceToDevice, st);
        if (ok(e)) e = hipMemcpyAsync(n->bt, t, 16 * rows, hipMemcpyDeviceToDevice, st);
        if (ok(e)) e = hipMemcpyAsync(n->bD, D, 8 * rows, hipMemcpyDeviceToDevice, st);
    }
    if (ok(e)) e = hipGetLastError();
    if (ok(e)) e = loss_grad_staged(n, rows, mode);
    if (ok(e)) e = hipMemcpyAsync(n->hloss, n->loss, sizeof(double), hipMemcpyDeviceToHost, st);
    if (ok(e)) e = hipStreamSynchronize(st);
    if (!ok(e)) return herr(n, e, "loss/grad");
    *loss = *n->hloss;
    return FSCC_OK;
}

fscc_status fscc_mlp_adam(fscc_mlp* n, float lr) {
    if (!n || !(lr > 0.f)) return FSCC_EINVAL;
    hipError_t e = adam(n, lr);
    return ok(e) ? FSCC_OK : herr(n, e, "adam");
}

}  // extern "C"
