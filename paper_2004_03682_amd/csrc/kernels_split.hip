// kernels_split.hip -- compensated mixed-precision complex GEMM for gfx950.
//
// An FP64 operand x is written as a short sum of low-precision pieces,
//   split-BF16:  x ~ h0 + h1 + h2   (three bf16; each piece rounds the
//                remainder of the previous ones, 3 x 8 significand bits)
//   split-FP32:  x ~ hi + lo        (two fp32)
// and a product a*b is the sum of the piece products whose order is at most
// the piece count minus one (bf16: 6 of the 9 cross products, fp32: 3 of 4).
// bf16 x bf16 products are exact in fp32, so the matrix cores
// (v_mfma_f32_16x16x32_bf16 / v_mfma_f32_16x16x4_f32) only round the fp32
// accumulation; the fp32 partial sums of every 32-deep k block are added into
// FP64 registers, and the epilogue applies alpha/beta in FP64.
//
//  * k_split         FP64 complex operand -> piece planes, once per operand
//                    (constant integrals) or per call (amplitudes).  Layout of
//                    one problem inside a plane: [Kp/32][rows_pad][32] so that
//                    a 32-deep slice of any 64-row panel is one contiguous run.
//  * k_zgemm_split   grouped tiles, LDS-staged, FP64 epilogue.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace fscc {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kT = 256;
constexpr int KB = 32;   // k depth of one staged block

// round-to-nearest-even fp32 -> bf16 bits (finite inputs)
__device__ inline uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ inline double bf16_value(uint32_t h) { return (double)__uint_as_float(h << 16); }

}  // namespace

template <bool BF>
__global__ __launch_bounds__(256) void k_split(const double2* __restrict__ src, void* __restrict__ dst,
                                               long long plane, const SplitProb* __restrict__ sps, int conj) {
    const SplitProb p = sps[blockIdx.y];
    const long long nchunk = (long long)p.rows_pad * (p.kpad / 8);
    const double sg = conj ? -1.0 : 1.0;
    for (long long c = (long long)blockIdx.x * kT + threadIdx.x; c < nchunk; c += (long long)gridDim.x * kT) {
        const int k8 = (int)(c & 3);
        const long long rest = c >> 2;
        const int r = (int)(rest % p.rows_pad);
        const int kb = (int)(rest / p.rows_pad);
        const int k0 = kb * KB + k8 * 8;
        double re[8], im[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + e;
            double2 v = make_double2(0.0, 0.0);
            if (r < p.rows && k < p.cols)
                v = p.trans ? src[p.src_off + (long long)k * p.ld + r] : src[p.src_off + (long long)r * p.ld + k];
            re[e] = v.x;
            im[e] = sg * v.y;
        }
        const long long o = p.dst_off + ((long long)kb * p.rows_pad + r) * KB + k8 * 8;
        if (BF) {
            uint16_t* d = (uint16_t*)dst;
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) {
                u4v w[3] = {u4v{0, 0, 0, 0}, u4v{0, 0, 0, 0}, u4v{0, 0, 0, 0}};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const double x = ri ? im[e] : re[e];
                    const uint32_t h0 = bf16_bits((float)x);
                    const double r1 = x - bf16_value(h0);
                    const uint32_t h1 = bf16_bits((float)r1);
                    const double r2 = r1 - bf16_value(h1);
                    const uint32_t h2 = bf16_bits((float)r2);
                    const int sh = 16 * (e & 1);
                    w[0][e >> 1] |= h0 << sh;
                    w[1][e >> 1] |= h1 << sh;
                    w[2][e >> 1] |= h2 << sh;
                }
#pragma unroll
                for (int pc = 0; pc < 3; ++pc) *(u4v*)(d + (long long)(2 * pc + ri) * plane + o) = w[pc];
            }
        } else {
            float* d = (float*)dst;
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) {
                f4v hi[2], lo[2];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const double x = ri ? im[e] : re[e];
                    const float h = (float)x;
                    hi[e >> 2][e & 3] = h;
                    lo[e >> 2][e & 3] = (float)(x - (double)h);
                }
                f4v* ph = (f4v*)(d + (long long)ri * plane + o);
                f4v* pl = (f4v*)(d + (long long)(2 + ri) * plane + o);
                ph[0] = hi[0];
                ph[1] = hi[1];
                pl[0] = lo[0];
                pl[1] = lo[1];
            }
        }
    }
}

// Planes: piece-major, re/im minor (plane 2*piece + ri).  Accumulator terms per
// fragment: 0 = sum Ar*Br, 1 = sum Ai*Bi, 2 = sum Ar*Bi, 3 = sum Ai*Br.
// ROLE only distinguishes kernel symbols in profiles (1 pp-ladder, 2 ring).
// BD: the B fragments are read by each wave straight from global memory into
// registers (the panel layout makes the 16 x 32 slice of one fragment 1 KB
// (bf16) or 2 KB (fp32) contiguous, lane l at offset 16 l or 32 l: the MFMA
// operand layout itself), one k block ahead; only A goes through LDS.  This
// takes the B stores and B fragment reads off the LDS, which otherwise
// carries more bytes per MFMA than it can serve.
template <bool BF, int BM, int BN, int WM, int WN, int ROLE, bool BD>
__global__ __launch_bounds__(256) void k_zgemm_split(const void* __restrict__ Av, long long sA,
                                                     const void* __restrict__ Bv, long long sB,
                                                     double2* __restrict__ C, const MProb* __restrict__ probs,
                                                     const ZTile* __restrict__ tiles, double ar, double ai, int beta) {
    constexpr int ES = BF ? 2 : 4;             // bytes per piece element
    constexpr int NPC = BF ? 3 : 2;            // pieces
    constexpr int NPL = 2 * NPC;               // planes
    constexpr int ROWB = KB * ES;              // bytes of one row of a k block
    // LDS rows: bf16 rows are 64 bytes, unpadded, with 16-byte chunk c of row r
    // at chunk c ^ swz(r): the stores (4 lanes per row, consecutive rows) and
    // the fragment reads (16 rows, one chunk each) then touch distinct banks
    // whether the LDS serves 8 or 16 lanes of a 16-byte access per cycle;
    // fp32 rows are padded by 16 bytes instead.
    constexpr int PITCH = BF ? ROWB : ROWB + 16;   // LDS row pitch (bytes)
    constexpr int VPR = ROWB / 16;             // 16-byte vectors per row
    constexpr int AVEC = NPL * BM * VPR, BVEC = NPL * BN * VPR;
    constexpr int AVT = (AVEC + kT - 1) / kT, BVT = (BVEC + kT - 1) / kT;
    constexpr int FM = BM / (16 * WM), FN = BN / (16 * WN);
    constexpr int FV = BF ? 1 : 2;             // 16-byte vectors per fragment and plane
    static_assert(WM * WN == 4 && FM >= 1 && FN >= 1, "tile");
    static_assert(BM % 16 == 0 && BN % 16 == 0, "row swizzle: rows mod 16 = fragment lane rows");
    __shared__ __attribute__((aligned(16))) unsigned char lds[NPL * (BM + (BD ? 0 : BN)) * PITCH];
    unsigned char* ldsA = lds;
    unsigned char* ldsB = lds + NPL * BM * PITCH;

    const ZTile tl = tiles[blockIdx.x];
    const MProb pr = probs[tl.prob];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm0 = (wave / WN) * FM * 16, wn0 = (wave % WN) * FN * 16;
    const int m0 = tl.m0, n0 = tl.n0;
    // a wave whose rows (or columns) all lie past the edge only helps load
    // the tile: the 64-row tiles over short pair-row blocks do no padded MFMAs
    const bool wave_live = m0 + wm0 < pr.M && n0 + wn0 < pr.N;
    const int nkb = pr.Kp / KB;
    const unsigned char* Ab = (const unsigned char*)Av + (pr.a_off + (long long)m0 * KB) * ES;
    const unsigned char* Bb = (const unsigned char*)Bv + (pr.b_off + (long long)n0 * KB) * ES;
    const long long stepA = (long long)pr.rows_a * KB * ES, stepB = (long long)pr.rows_b * KB * ES;

    const int lr = lane & 15, kq = lane >> 4;
    auto swz = [](int r) { return BF ? (((r >> 1) + (r >> 3)) & 3) : 0; };   // r: row mod 16
    const int sl = swz(lr);
    u4v ra[AVT], rb[BD ? 1 : BVT];
    u4v gb[NPC][2][FN][FV];   // BD: the next k block's B fragments
    auto load = [&](int kb) {
#pragma unroll
        for (int u = 0; u < AVT; ++u) {
            const int v = tid + u * kT;
            if (v < AVEC) {
                const int p = v / (BM * VPR), w = v % (BM * VPR);
                ra[u] = *(const u4v*)(Ab + (long long)p * sA * ES + kb * stepA + (long long)w * 16);
            }
        }
        if constexpr (BD) {
#pragma unroll
            for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int h = 0; h < FV; ++h)
                            gb[pc][ri][j][h] = *(const u4v*)(Bb + (long long)(2 * pc + ri) * sB * ES + kb * stepB +
                                                             (long long)(wn0 + j * 16 + lr) * ROWB + kq * 16 * FV +
                                                             h * 16);
        } else {
#pragma unroll
            for (int u = 0; u < BVT; ++u) {
                const int v = tid + u * kT;
                if (v < BVEC) {
                    const int p = v / (BN * VPR), w = v % (BN * VPR);
                    rb[u] = *(const u4v*)(Bb + (long long)p * sB * ES + kb * stepB + (long long)w * 16);
                }
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < AVT; ++u) {
            const int v = tid + u * kT;
            if (v < AVEC) {
                const int p = v / (BM * VPR), w = v % (BM * VPR);
                *(u4v*)(ldsA + (p * BM + w / VPR) * PITCH + ((w % VPR) ^ swz((w / VPR) & 15)) * 16) = ra[u];
            }
        }
        if constexpr (!BD) {
#pragma unroll
            for (int u = 0; u < BVT; ++u) {
                const int v = tid + u * kT;
                if (v < BVEC) {
                    const int p = v / (BN * VPR), w = v % (BN * VPR);
                    *(u4v*)(ldsB + (p * BN + w / VPR) * PITCH + ((w % VPR) ^ swz((w / VPR) & 15)) * 16) = rb[u];
                }
            }
        }
    };

    double dr[FM][FN][4], di[FM][FN][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) dr[i][j][q] = di[i][j][q] = 0.0;

    if (nkb > 0) load(0);
    for (int kb = 0; kb < nkb; ++kb) {
        __syncthreads();
        store();
        __syncthreads();
        // fragments: lane (lr, kq) holds k = 8*kq .. 8*kq+7 of row/column lr
        u4v fb[NPC][2][FN][FV];
        if constexpr (BD) {
#pragma unroll
            for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int h = 0; h < FV; ++h) fb[pc][ri][j][h] = gb[pc][ri][j][h];
        }
        if (kb + 1 < nkb) load(kb + 1);
        if (!wave_live) continue;
        if constexpr (!BD) {
#pragma unroll
            for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int h = 0; h < FV; ++h)
                            fb[pc][ri][j][h] = *(const u4v*)(ldsB + ((2 * pc + ri) * BN + wn0 + j * 16 + lr) * PITCH +
                                                             ((kq * FV + h) ^ sl) * 16);
        }
        f4v acc[FM][FN][4];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[i][j][t] = f4v{0.f, 0.f, 0.f, 0.f};
        // piece pairs from the smallest order to (0,0): the small cross products
        // accumulate among themselves and the leading product is added last, so
        // each fp32 accumulator is rounded at the scale of the full sum only once
#pragma unroll
        for (int pa = NPC - 1; pa >= 0; --pa) {
            u4v fa[2][FM][FV];
#pragma unroll
            for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int h = 0; h < FV; ++h)
                        fa[ri][i][h] = *(const u4v*)(ldsA + ((2 * pa + ri) * BM + wm0 + i * 16 + lr) * PITCH +
                                                     ((kq * FV + h) ^ sl) * 16);
#pragma unroll
            for (int pb = NPC - 1 - pa; pb >= 0; --pb) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int ra_ = (t == 1 || t == 3) ? 1 : 0;   // A re/im
                    const int rb_ = (t == 1 || t == 2) ? 1 : 0;   // B re/im
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            if constexpr (BF) {
                                acc[i][j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    __builtin_bit_cast(bf8v, fa[ra_][i][0]), __builtin_bit_cast(bf8v, fb[pb][rb_][j][0]),
                                    acc[i][j][t], 0, 0, 0);
                            } else {
#pragma unroll
                                for (int s = 0; s < 8; ++s) {
                                    const float a = __uint_as_float(fa[ra_][i][s >> 2][s & 3]);
                                    const float b = __uint_as_float(fb[pb][rb_][j][s >> 2][s & 3]);
                                    acc[i][j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i][j][t], 0, 0, 0);
                                }
                            }
                        }
                }
            }
        }
        // spill the fp32 block sums into FP64
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    dr[i][j][q] += (double)acc[i][j][0][q] - (double)acc[i][j][1][q];
                    di[i][j][q] += (double)acc[i][j][2][q] + (double)acc[i][j][3][q];
                }
    }

    // epilogue: for the fp32-accumulating MFMAs, accumulator element q of a lane
    // is row 4*(lane/16) + q, column lane%16 of the fragment
    double2* Cp = C + pr.c_off;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn0 + j * 16 + lr;
            if (col >= pr.N) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm0 + i * 16 + kq * 4 + q;
                if (row >= pr.M) continue;
                const double xr = dr[i][j][q], xi = di[i][j][q];
                double2 out = make_double2(ar * xr - ai * xi, ar * xi + ai * xr);
                double2* c = Cp + (long long)row * pr.ldc + col;
                if (beta) {
                    const double2 old = *c;
                    out.x += old.x;
                    out.y += old.y;
                }
                *c = out;
            }
        }
}

void mcfg_tile(int cfg, int* bm, int* bn) {
    switch (cfg % MCFG_TILES) {
        case MCFG_64x32: *bm = 64; *bn = 32; break;
        case MCFG_32x64: *bm = 32; *bn = 64; break;
        case MCFG_32x32: *bm = 32; *bn = 32; break;
        default: *bm = 64; *bn = 64; break;
    }
}

hipError_t launch_split(bool bf16, const double2* src, void* dst, long long plane, const SplitProb* sp, int nprob,
                        long long max_chunks, int conj, hipStream_t st) {
    if (nprob <= 0 || max_chunks <= 0) return hipSuccess;
    long long bx = (max_chunks + kT - 1) / kT;
    dim3 grid((unsigned)(bx < 2048 ? bx : 2048), (unsigned)nprob), block(kT);
    if (bf16) k_split<true><<<grid, block, 0, st>>>(src, dst, plane, sp, conj);
    else k_split<false><<<grid, block, 0, st>>>(src, dst, plane, sp, conj);
    return hipGetLastError();
}

template <bool BF, int BM, int BN, int WM, int WN, bool BD>
static hipError_t launch_split_cfg(const void* A, long long sA, const void* B, long long sB, double2* C,
                                   const MProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta,
                                   hipStream_t st, int role) {
    dim3 grid(ntiles), block(kT);
    if (role == 1)
        k_zgemm_split<BF, BM, BN, WM, WN, 1, BD><<<grid, block, 0, st>>>(A, sA, B, sB, C, probs, tiles, ar, ai, beta);
    else if (role == 2)
        k_zgemm_split<BF, BM, BN, WM, WN, 2, BD><<<grid, block, 0, st>>>(A, sA, B, sB, C, probs, tiles, ar, ai, beta);
    else
        k_zgemm_split<BF, BM, BN, WM, WN, 0, BD><<<grid, block, 0, st>>>(A, sA, B, sB, C, probs, tiles, ar, ai, beta);
    return hipGetLastError();
}

template <bool BF, bool BD>
static hipError_t launch_split_tile(int tile, const void* A, long long sA, const void* B, long long sB, double2* C,
                                    const MProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta,
                                    hipStream_t st, int role) {
    switch (tile) {
        case MCFG_64x64: return launch_split_cfg<BF, 64, 64, 2, 2, BD>(A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
        case MCFG_64x32: return launch_split_cfg<BF, 64, 32, 2, 2, BD>(A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
        case MCFG_32x64: return launch_split_cfg<BF, 32, 64, 2, 2, BD>(A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
        case MCFG_32x32: return launch_split_cfg<BF, 32, 32, 2, 2, BD>(A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
        default: return hipErrorInvalidValue;
    }
}

template <bool BF>
static hipError_t launch_split_bf(int cfg, const void* A, long long sA, const void* B, long long sB, double2* C,
                                  const MProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta,
                                  hipStream_t st, int role) {
    if (cfg < 0 || cfg >= MCFG_N) return hipErrorInvalidValue;
    if (cfg >= MCFG_TILES)
        return launch_split_tile<BF, true>(cfg - MCFG_TILES, A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
    return launch_split_tile<BF, false>(cfg, A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
}

hipError_t launch_zgemm_split(bool bf16, int cfg, const void* A, long long sA, const void* B, long long sB, double2* C,
                              const MProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta,
                              hipStream_t st, int role) {
    if (ntiles <= 0) return hipSuccess;
    if (bf16) return launch_split_bf<true>(cfg, A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
    return launch_split_bf<false>(cfg, A, sA, B, sB, C, probs, tiles, ntiles, ar, ai, beta, st, role);
}

}  // namespace fscc
