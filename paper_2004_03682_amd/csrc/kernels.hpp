// kernels.hpp -- launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gtile.hpp"

namespace fscc {

// one GEMM problem (offsets in complex elements)
struct ZProb {
    long long a_off, b_off, c_off;
    int M, N, K, lda, ldb, ldc;
};
// one output tile of one problem; sys = system index of a batched launch
struct ZTile {
    int prob, m0, n0, sys;
};

// tile shapes of the grouped complex GEMM
// ZCFG_SKINNY: one workgroup per (64 x 32 output block, K chunk) on the
// vector ALUs; always used with the split-K reduction.
// ZCFG_TALL: one workgroup per 256 rows, one row per thread, all columns, on
// the vector ALUs; needs !tA, K <= ZTALL_MAX_K, N <= ZTALL_MAX_KN and
// K*N <= ZTALL_MAX_KN (B is kept in LDS); never split.
// ZCFG_RED: one workgroup per K chunk of a problem with M <= ZRED_MAX_M and
// 1 <= N <= ZRED_MAX_N, !tB, on the vector ALUs; always split along K into
// chunks of at most ZRED_LDS / M.
// ZCFG_DOT: one workgroup per ZDOT_ROWS rows of B of a problem with
// M <= ZDOT_MAX_M, !tA, tB (every output a dot product of two contiguous
// K-vectors), on the vector ALUs; each B row is streamed once; never split.
// ZCFG_64x64R / ZCFG_64x32R: 64-row MFMA tiles with the four waves stacked
// along M (16 rows each): a problem of up to 64 rows reads each column panel
// of B once, and a wave whose 16 rows lie past M issues no MFMA, so the
// padding is that of 16-row tiles.
enum ZCfg {
    ZCFG_64x64 = 0, ZCFG_128x16, ZCFG_16x128, ZCFG_32x32, ZCFG_64x16, ZCFG_16x64, ZCFG_SKINNY, ZCFG_TALL, ZCFG_RED,
    ZCFG_32x64, ZCFG_64x32, ZCFG_DOT, ZCFG_64x64R, ZCFG_64x32R, ZCFG_N
};
constexpr int ZSKINNY_BM = 64, ZSKINNY_BN = 32, ZSKINNY_MAX_MN = ZSKINNY_BM * ZSKINNY_BN;
// deepest DIIS subspace of a single-system context (vectors kept; the dot
// partials of the DIIS kernels have this stride)
constexpr int kDiisMax = 16;
constexpr int ZTALL_ROWS = 256, ZTALL_MAX_K = 64, ZTALL_MAX_KN = 1024;
constexpr int ZRED_MAX_M = 8, ZRED_MAX_N = 256, ZRED_LDS = 2048;   // LDS: A chunk of M * K <= ZRED_LDS
constexpr int ZDOT_MAX_M = 8, ZDOT_ROWS = 16, ZDOT_KC = 256;       // LDS: A chunk of M * ZDOT_KC
void zcfg_tile(int cfg, int* bm, int* bn);

// C(m,n) = alpha * sum_k opA(m,k) opB(k,n) + beta*C(m,n)  for every tile in `tiles`
//   !tA: A(m,k) = A[a_off + m*lda + k]      tA: A(m,k) = A[a_off + k*lda + m]
//   !tB: B(k,n) = B[b_off + k*ldb + n]      tB: B(k,n) = B[b_off + n*ldb + k]
//   cA/cB conjugate the operand; beta is 0 (overwrite) or 1 (accumulate).
//   bk = 16 or 32 (K depth of one LDS stage); role only selects a distinct kernel symbol.
//   active (may be null): tiles whose active[tile.sys] == 0 are skipped.
//   max_m: largest M of the problems (used by ZCFG_RED and ZCFG_DOT only, 1..8).
//   m3: MFMA tiles form the complex product from three real products (3M)
//   instead of four (4M); ignored by the vector-ALU forms.
//   lds: how an MFMA tile stages its K slices in LDS: LDS_STAGED (through
//   registers, one buffer pair), LDS_DOUBLE (two buffer pairs, one barrier per
//   slice; bk = 16 and the tiles for which zcfg_has_db() holds) or
//   LDS_DIRECT (direct-to-LDS loads through a ring of stages; bk = 16 and the
//   tiles for which zcfg_has_dl() holds).
enum { LDS_STAGED = 0, LDS_DOUBLE = 1, LDS_DIRECT = 2 };
hipError_t launch_zgemm(int cfg, int bk, bool tA, bool tB, const double2* A, const double2* B, double2* C,
                        const ZProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA,
                        int cB, hipStream_t st, int role = 0, const int* active = nullptr, int max_m = 0,
                        bool m3 = false, int lds = LDS_STAGED);
bool zcfg_has_db(int cfg);
// The same GEMM with direct-to-LDS loads through a ring of LDS stages
// (kernels_dl.hip); 16-deep slices, the tiles for which zcfg_has_dl() holds.
hipError_t launch_zgemm_dl(int cfg, bool tA, bool tB, const double2* A, const double2* B, double2* C,
                           const ZProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta, int cA,
                           int cB, hipStream_t st, int role, const int* active, bool m3);
bool zcfg_has_dl(int cfg);

// ---- compensated mixed-precision GEMM (kernels_split.hip)
// element (r, k) of a rows x cols operand: src[src_off + r*ld + k] (trans = 0)
// or src[src_off + k*ld + r] (trans = 1); written as piece planes in the
// panel layout [kpad/32][rows_pad][32] at dst_off (rows_pad % 64 == 0,
// kpad % 32 == 0, zero fill outside rows x cols).
struct SplitProb {
    long long src_off, dst_off;
    int rows, cols, ld, trans, rows_pad, kpad;
};
// bf16: 6 planes (piece-major, re/im), fp32: 4 planes; `plane` = elements per
// plane (multiple of 64); conj negates the imaginary pieces.  max_chunks =
// max over problems of rows_pad*kpad/8.
hipError_t launch_split(bool bf16, const double2* src, void* dst, long long plane, const SplitProb* sp, int nprob,
                        long long max_chunks, int conj, hipStream_t st);
// C(m,n) = alpha * sum_k A(m,k) B(n,k) + beta*C(m,n), A/B in split planes
// (a_off/b_off: element offsets of the problem inside a plane, rows_a/rows_b
// the panel row counts, Kp the padded depth).
struct MProb {
    long long a_off, b_off, c_off;
    int M, N, Kp, ldc, rows_a, rows_b;
};
// split-kernel tiles; MCFG_TILES + t: tile t with the B fragments read from
// global memory straight into registers (only A staged in LDS)
enum MCfg { MCFG_64x64 = 0, MCFG_64x32, MCFG_32x64, MCFG_32x32, MCFG_TILES, MCFG_N = 2 * MCFG_TILES };
void mcfg_tile(int cfg, int* bm, int* bn);
hipError_t launch_zgemm_split(bool bf16, int cfg, const void* A, long long sA, const void* B, long long sB, double2* C,
                              const MProb* probs, const ZTile* tiles, int ntiles, double ar, double ai, int beta,
                              hipStream_t st, int role = 0);

// split-K second pass: C = alpha * sum_s W[w_off + s*M*N + m*N + n] + beta*C
// (sys: system of a batched launch; skipped when active[sys] == 0)
struct ZRed {
    long long c_off, w_off;
    int M, N, ldc, S, sys, pad;
};
// maxS = the largest number of K chunks over the problems
constexpr int ZRED_FEW_S = 8;
hipError_t launch_splitk_reduce(double2* C, const double2* W, const ZRed* reds, int nred, int maxMN, int maxS,
                                double ar, double ai, int beta, hipStream_t st, const int* active = nullptr);

// Block table of a segmented elementwise launch over a batched buffer: block b
// handles elements [start[b], min(start[b] + 256, end[b])) of system sys[b]
// and does nothing if active[sys[b]] == 0.  sys == nullptr: plain launch over
// [0, n).
struct SegBlocks {
    const int* sys = nullptr;
    const long long* start = nullptr;
    const long long* end = nullptr;
    const int* active = nullptr;
    int nblk = 0;
};

// dst[k] = beta*dst[k] + alpha * sum_t s_t cj(src_t[mA_t[k]]) * (src2 ? src2[mB_t[k]] : 1)
// src[t], when set, is term t's own source (a sum of reorders of different
// buffers into one destination); otherwise term t reads the call's src
struct GatherMaps {
    const uint32_t* a[4];
    const uint32_t* b[4];
    const void* src[4];
};
// the same gather over its affine tiles (no second operand): work units
// units[nunits] over tiles[], terms[tile * nt + t] (see RTerm); mapped terms
// read maps.a[t]
hipError_t launch_reorder(double2* dst, const double2* src, GatherMaps maps, int nt, const RUnit* units, int nunits,
                          const GTile* tiles, const RTerm* terms, double ar, double ai, int beta, int conj,
                          hipStream_t st);
hipError_t launch_gather(double2* dst, const double2* src, const double2* src2, GatherMaps maps, int nt,
                         long long n, double ar, double ai, int beta, int conj, hipStream_t st,
                         SegBlocks sb = SegBlocks());
// the same gather over the 16 x 16 destination tiles of `tiles` (device array)
hipError_t launch_gather_tiled(double2* dst, const double2* src, const double2* src2, GatherMaps maps, int nt,
                               const GTile* tiles, int ntiles, double ar, double ai, int beta, int conj,
                               hipStream_t st);

hipError_t launch_axpby(double2* dst, const double2* src, long long n, double ar, double ai, int beta, int conj,
                        hipStream_t st, SegBlocks sb = SegBlocks());
hipError_t launch_diag(double2* dst, const double* d, const double2* src, long long n, hipStream_t st,
                       SegBlocks sb = SegBlocks());
hipError_t launch_mul(double2* dst, const double* d, long long n, hipStream_t st,
                      SegBlocks sb = SegBlocks());   // dst *= d (real)

// Jacobi: step = r/(D - shift); tn = t + step (written to hist_t), e = step (hist_e);
// per-block max |step| into part_max[block].  dyn_S < 0: dynamic shifts
// Delta = dyn_S (dyn_S / (min(D,0) + dyn_S))^dyn_n, step = (r - Delta t) / (D + Delta - shift).
hipError_t launch_jacobi(const double2* t, const double2* r, const double* D, double2* hist_t, double2* hist_e,
                         long long n, double* part_max, int nblk, hipStream_t st, double shift = 0.0,
                         double dyn_S = 0.0, int dyn_n = 0);
// sum_b part[b*stride + j] -> out[j]  (j < cols), and max over part_max
hipError_t launch_dots(const double2* const* e, int m, const double2* enew, long long n, double* part, int nblk,
                       hipStream_t st);
// *count = number of non-finite doubles in x[0..n) (zeroes *count first; not
// for code under graph capture: it records a memset)
hipError_t launch_count_nonfinite(const double* x, long long n, unsigned long long* count, hipStream_t st);
// dressed Jacobi denominators: D[k] = min(f[i] - f[no + a], -floor) (order 2,
// idx = (i, a) per element) or min(f[i] + f[j] - f[no + a] - f[no + b], -floor)
// (order 4, idx = (i, j, a, b)); f = occupied then virtual one-particle energies
hipError_t launch_dressed_denoms(const uint16_t* idx, int order, const double* f, int no, double floor, double* D,
                                 long long n, hipStream_t st);
// coef holds ldb + 1 doubles: coef[ldb] = 1 marks a non-finite step.  The
// live slots (oldest first) travel as a kernel argument, so that enqueueing
// the update needs no copy from host memory.
struct DiisOrder {
    int v[kDiisMax];
};
hipError_t launch_finish_diis(const double* part, int nblk, int m, const double* part_max, int nblk_max, double* B,
                              int ldb, int newslot, const DiisOrder& order, double* coef, double* scal, hipStream_t st);
// out = sum_{j<m} coef[j] xs[j], unless coef[m] != 0 (out is then left untouched)
hipError_t launch_lincomb(double2* out, const double2* const* xs, const double* coef, int m, long long n,
                          hipStream_t st);
// complex dot sum_k x[k]*y[k] (no conjugation): per-block partials then final
hipError_t launch_zdotu(const double2* x, const double2* y, long long n, double* part, int nblk, double* out,
                        hipStream_t st);
hipError_t launch_zero(double2* dst, long long n, hipStream_t st);

int reduce_blocks(long long n);

// ---- real arithmetic (kernels_real.hip): the same operations on doubles for
// double groups with real integrals and amplitudes; alpha is real, no
// conjugation, plain (unsegmented) launches.  launch_dgemm takes the MFMA
// tile shapes and ZCFG_TALL / ZCFG_RED (not ZCFG_SKINNY).
hipError_t launch_dgemm(int cfg, int bk, bool tA, bool tB, const double* A, const double* B, double* C,
                        const ZProb* probs, const ZTile* tiles, int ntiles, double alpha, int beta, hipStream_t st,
                        int role = 0, const int* active = nullptr, int max_m = 0, int lds = LDS_STAGED);
// the real direct-to-LDS form (kernels_dl.hip); the tiles of zcfg_has_dl(), bk = 16
hipError_t launch_dgemm_dl(int cfg, bool tA, bool tB, const double* A, const double* B, double* C,
                           const ZProb* probs, const ZTile* tiles, int ntiles, double alpha, int beta, hipStream_t st,
                           int role, const int* active);
hipError_t launch_dsplitk_reduce(double* C, const double* W, const ZRed* reds, int nred, int maxMN, int maxS,
                                 double alpha, int beta, hipStream_t st);
hipError_t launch_dgather(double* dst, const double* src, const double* src2, GatherMaps maps, int nt, long long n,
                          double alpha, int beta, hipStream_t st);
hipError_t launch_daxpby(double* dst, const double* src, long long n, double alpha, int beta, hipStream_t st);
hipError_t launch_ddiag(double* dst, const double* d, const double* src, long long n, hipStream_t st);
hipError_t launch_dmul(double* dst, const double* d, long long n, hipStream_t st);
hipError_t launch_djacobi(const double* t, const double* r, const double* D, double* hist_t, double* hist_e,
                          long long n, double* part_max, int nblk, hipStream_t st, double shift = 0.0,
                          double dyn_S = 0.0, int dyn_n = 0);
hipError_t launch_ddots(const double* const* e, int m, const double* enew, long long n, double* part, int nblk,
                        hipStream_t st);
// real form of launch_lincomb (same coef[m] convention)
hipError_t launch_dlincomb(double* out, const double* const* xs, const double* coef, int m, long long n,
                           hipStream_t st);
// out[0] = sum x*y, out[1] = 0
hipError_t launch_ddot(const double* x, const double* y, long long n, double* part, int nblk, double* out,
                       hipStream_t st);

// ---- batched update (many independent systems in concatenated vectors)
// segment of system s: T1 part [off1, off1+n1), T2 part [off2, off2+n2);
// history: nd slots of n1+n2 elements at hoff
struct BSeg {
    long long off1, n1, off2, n2, hoff;
};
// per-system DIIS state: count live slots, newest slot, active (not yet
// converged), upd (updated in the current iteration), iterations, failed
// (non-finite step), nd = history depth (<= 8)
struct BState {
    int count, newest, active, upd, iters, failed, nd, pad;
};
// Jacobi step r/(D - shift) + per-system DIIS (t?o may alias t?); one launch sequence.
// active[s] / upd[s] receive the system's flags after / during this update
hipError_t launch_batch_update(const double2* t1, const double2* t2, const double2* r1, const double2* r2,
                               double2* t1o, double2* t2o, const double* D1, const double* D2, const BSeg* segs,
                               BState* state, double2* ht, double2* he, double* part_max, double* part, double* Bm,
                               double* coef, double* maxstep, double tol, double shift, int* active, int* upd,
                               int nsys, int nblk, hipStream_t st);
// per-system E = sum oovv*tau over the T2 segment, then the report rows
// out[s*6 + {0..5}] = E_re, E_im, max|step|, active, iterations, failed
// out[s] = max |r / D| over system s's T1 and T2 segments
hipError_t launch_batch_maxnorm(const double2* r1, const double2* r2, const double* D1, const double* D2,
                                const BSeg* segs, double* part, double* out, int nsys, int nblk, hipStream_t st);
hipError_t launch_batch_energy(const double2* oovv, const double2* tau, const BSeg* segs, const BState* state,
                               const double* maxstep, double* part, double* out, int nsys, int nblk, hipStream_t st);

}  // namespace fscc
