// fsgen_gpu.hip -- the integral generator of fsgen.c evaluated on the GPU.
//
// INPUT GENERATION only (no coupled-cluster arithmetic).  Same definition as
// fsgen.c: X_pqrs from SplitMix64 counters + Box-Muller, V = 1/8 of the
// antisymmetric-Hermitian projection evaluated at the canonical
// representative, exact sign / conjugation images, zero outside allowed
// irrep tuples.  The transcendental functions are the device library's, so
// values agree with the host generator to a few units in the last place
// rather than bit for bit.  Used to produce large class buffers (batched
// workloads) directly in device memory.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ inline uint64_t sm64_at(uint64_t key, uint64_t k) { return mix64(key + (k + 1ULL) * 0x9E3779B97F4A7C15ULL); }

__device__ inline void xval(uint64_t key, uint64_t n, int p, int q, int r, int s, double sc, double* re, double* im) {
    const uint64_t L = (((uint64_t)p * n + (uint64_t)q) * n + (uint64_t)r) * n + (uint64_t)s;
    const uint64_t h1 = sm64_at(key, 2ULL * L);
    const uint64_t h2 = sm64_at(key, 2ULL * L + 1ULL);
    const double u1 = (double)((h1 >> 11) + 1ULL) * 0x1.0p-53;
    const double u2 = (double)(h2 >> 11) * 0x1.0p-53;
    const double rad = sqrt(-2.0 * log(u1)) * sc;
    const double th = 6.283185307179586476925286766559 * u2;
    *re = rad * cos(th);
    *im = rad * sin(th);
}

__device__ inline double2 vval(uint64_t key, int n, const int* irrep, int G, int p, int q, int r, int s, double sc) {
    if (p == q || r == s) return make_double2(0.0, 0.0);
    if (((irrep[p] + irrep[q] - irrep[r] - irrep[s]) % G + G) % G != 0) return make_double2(0.0, 0.0);
    int sg = 1, t;
    if (p > q) { t = p; p = q; q = t; sg = -sg; }
    if (r > s) { t = r; r = s; s = t; sg = -sg; }
    bool cj = false;
    if (p > r || (p == r && q > s)) {
        t = p; p = r; r = t;
        t = q; q = s; s = t;
        cj = true;
    }
    double xr[4], xi[4], yr[4], yi[4];
    const uint64_t nn = (uint64_t)n;
    xval(key, nn, p, q, r, s, sc, &xr[0], &xi[0]);
    xval(key, nn, q, p, r, s, sc, &xr[1], &xi[1]);
    xval(key, nn, p, q, s, r, sc, &xr[2], &xi[2]);
    xval(key, nn, q, p, s, r, sc, &xr[3], &xi[3]);
    xval(key, nn, r, s, p, q, sc, &yr[0], &yi[0]);
    xval(key, nn, s, r, p, q, sc, &yr[1], &yi[1]);
    xval(key, nn, r, s, q, p, sc, &yr[2], &yi[2]);
    xval(key, nn, s, r, q, p, sc, &yr[3], &yi[3]);
    const double ar = ((xr[0] - xr[1]) - xr[2]) + xr[3];
    const double ai = ((xi[0] - xi[1]) - xi[2]) + xi[3];
    const double br = ((yr[0] - yr[1]) - yr[2]) + yr[3];
    const double bi = ((yi[0] - yi[1]) - yi[2]) + yi[3];
    double vr = (ar + br) * 0.125, vi = (ai - bi) * 0.125;
    if (cj) vi = -vi;
    if (sg < 0) {
        vr = -vr;
        vi = -vi;
    }
    return make_double2(vr, vi);
}

// one dense block of the class buffer: out[off + ((a*n2 + b)*n3 + c)*n4 + d]
struct GenBlock {
    long long off;
    int n[4];
    int mem[4];   // offsets into the member array (global spinor indices)
};

__global__ __launch_bounds__(256) void k_gen(uint64_t key, double sc, int n, const int* __restrict__ irrep, int G,
                                             const GenBlock* __restrict__ blocks, const int* __restrict__ mem,
                                             double2* __restrict__ out) {
    const GenBlock b = blocks[blockIdx.y];
    const long long cnt = (long long)b.n[0] * b.n[1] * b.n[2] * b.n[3];
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (long long)gridDim.x * blockDim.x) {
        long long x = e;
        const int d = (int)(x % b.n[3]);
        x /= b.n[3];
        const int c = (int)(x % b.n[2]);
        x /= b.n[2];
        const int bb = (int)(x % b.n[1]);
        const int a = (int)(x / b.n[1]);
        out[b.off + e] = vval(key, n, irrep, G, mem[b.mem[0] + a], mem[b.mem[1] + bb], mem[b.mem[2] + c],
                              mem[b.mem[3] + d], sc);
    }
}

}  // namespace

// Fill a class buffer (boundary layout, nblocks dense blocks) in device
// memory.  irrep_host[n]: labels; blocks_host / mem_host: block table and
// member lists (host arrays, copied here).  Synchronous on `stream`.
// Returns 0 on success, a HIP error code otherwise.
extern "C" int fsgen_gpu_class(uint64_t seed, double sigma, int n, const int* irrep_host, int G, const void* blocks_host,
                               int nblocks, const int* mem_host, int nmem, void* out_dev, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    int *dirr = nullptr, *dmem = nullptr;
    GenBlock* dblk = nullptr;
    hipError_t e = hipMalloc(&dirr, sizeof(int) * (n > 0 ? n : 1));
    if (e == hipSuccess) e = hipMalloc(&dmem, sizeof(int) * (nmem > 0 ? nmem : 1));
    if (e == hipSuccess) e = hipMalloc(&dblk, sizeof(GenBlock) * (nblocks > 0 ? nblocks : 1));
    if (e == hipSuccess && n > 0) e = hipMemcpy(dirr, irrep_host, sizeof(int) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && nmem > 0) e = hipMemcpy(dmem, mem_host, sizeof(int) * nmem, hipMemcpyHostToDevice);
    if (e == hipSuccess && nblocks > 0) e = hipMemcpy(dblk, blocks_host, sizeof(GenBlock) * nblocks, hipMemcpyHostToDevice);
    long long maxcnt = 0;
    const GenBlock* hb = (const GenBlock*)blocks_host;
    for (int k = 0; k < nblocks; ++k) {
        long long c = (long long)hb[k].n[0] * hb[k].n[1] * hb[k].n[2] * hb[k].n[3];
        if (c > maxcnt) maxcnt = c;
    }
    if (e == hipSuccess && nblocks > 0 && maxcnt > 0) {
        long long bx = (maxcnt + 255) / 256;
        dim3 grid((unsigned)(bx < 4096 ? bx : 4096), (unsigned)nblocks);
        k_gen<<<grid, 256, 0, st>>>(seed, sigma / sqrt(2.0), n, dirr, G, dblk, dmem, (double2*)out_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dirr) (void)hipFree(dirr);
    if (dmem) (void)hipFree(dmem);
    if (dblk) (void)hipFree(dblk);
    return (int)e;
}
