/*
 * fsgen.c -- seeded synthetic two-electron integrals for the relativistic
 * Fock-space coupled-cluster workloads (Hamiltonian of Eq. (1)).
 *
 * This file is INPUT GENERATION only.  It holds none of the coupled-cluster
 * arithmetic; both the CPU oracle and the HIP library's tests and benchmark
 * obtain their integrals from here, so that the two sides see identical
 * inputs while sharing no method code.
 *
 * Definition (order-free, counter based):
 *   X_pqrs  ~ CN(0, sigma^2): Re and Im independent N(0, sigma^2/2), drawn by
 *             Box-Muller from two SplitMix64 outputs at counters 2L and 2L+1,
 *             L = ((p*n + q)*n + r)*n + s, key = seed.
 *   V_pqrs  = 1/8 [ X_pqrs - X_qprs - X_pqsr + X_qpsr
 *                  + conj(X_rspq - X_srpq - X_rsqp + X_srqp) ]
 *             i.e. the projection of X onto tensors antisymmetric in (pq)
 *             and in (rs) and Hermitian under (pq) <-> (rs).
 *   V is evaluated only at the canonical representative (p<q, r<s,
 *   (p,q) <= (r,s) lexicographically) and every other element is obtained
 *   from it by an exact sign flip and/or complex conjugation, so the
 *   antisymmetry and Hermiticity hold bit for bit.
 *   Elements whose irrep labels violate g_p + g_q = g_r + g_s (mod nirrep)
 *   are exactly zero (Abelian double-group selection rule).
 *
 * SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state advances by the golden
 * gamma 0x9E3779B97F4A7C15 and each output is the "mix64" finaliser of the
 * state.  Output k (k >= 0) of the stream with initial state `key` is
 * mix64(key + (k+1)*gamma).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t sm64_at(uint64_t key, uint64_t k)
{
    return mix64(key + (k + 1ULL) * 0x9E3779B97F4A7C15ULL);
}

/* One complex Gaussian X_pqrs with E|X|^2 = sigma^2 (sc = sigma/sqrt(2)). */
static inline void xval(uint64_t key, uint64_t n, int p, int q, int r, int s,
                        double sc, double *re, double *im)
{
    uint64_t L = (((uint64_t)p * n + (uint64_t)q) * n + (uint64_t)r) * n + (uint64_t)s;
    uint64_t h1 = sm64_at(key, 2ULL * L);
    uint64_t h2 = sm64_at(key, 2ULL * L + 1ULL);
    double u1 = (double)((h1 >> 11) + 1ULL) * 0x1.0p-53; /* (0, 1] */
    double u2 = (double)(h2 >> 11) * 0x1.0p-53;          /* [0, 1) */
    double rad = sqrt(-2.0 * log(u1)) * sc;
    double th = 6.283185307179586476925286766559 * u2;
    *re = rad * cos(th);
    *im = rad * sin(th);
}

/* V at a canonical representative (P<Q, R<S, (P,Q) <= (R,S)). */
static void vcanon(uint64_t key, uint64_t n, int P, int Q, int R, int S, double sc,
                   double *re, double *im)
{
    double xr[4], xi[4], yr[4], yi[4];
    xval(key, n, P, Q, R, S, sc, &xr[0], &xi[0]);
    xval(key, n, Q, P, R, S, sc, &xr[1], &xi[1]);
    xval(key, n, P, Q, S, R, sc, &xr[2], &xi[2]);
    xval(key, n, Q, P, S, R, sc, &xr[3], &xi[3]);
    xval(key, n, R, S, P, Q, sc, &yr[0], &yi[0]);
    xval(key, n, S, R, P, Q, sc, &yr[1], &yi[1]);
    xval(key, n, R, S, Q, P, sc, &yr[2], &yi[2]);
    xval(key, n, S, R, Q, P, sc, &yr[3], &yi[3]);
    double ar = ((xr[0] - xr[1]) - xr[2]) + xr[3];
    double ai = ((xi[0] - xi[1]) - xi[2]) + xi[3];
    double br = ((yr[0] - yr[1]) - yr[2]) + yr[3];
    double bi = ((yi[0] - yi[1]) - yi[2]) + yi[3];
    *re = (ar + br) * 0.125;
    *im = (ai - bi) * 0.125;
}

/* V_pqrs for arbitrary global spinor indices. */
static void vval(uint64_t key, int n, const int *irrep, int nirrep, int p, int q, int r,
                 int s, double sc, double *re, double *im)
{
    *re = 0.0;
    *im = 0.0;
    if (p == q || r == s)
        return;
    if (((irrep[p] + irrep[q] - irrep[r] - irrep[s]) % nirrep + nirrep) % nirrep != 0)
        return;
    int sg = 1, t;
    if (p > q) { t = p; p = q; q = t; sg = -sg; }
    if (r > s) { t = r; r = s; s = t; sg = -sg; }
    int cj = 0;
    if (p > r || (p == r && q > s)) {
        t = p; p = r; r = t;
        t = q; q = s; s = t;
        cj = 1;
    }
    double vr, vi;
    vcanon(key, (uint64_t)n, p, q, r, s, sc, &vr, &vi);
    if (cj)
        vi = -vi;
    if (sg < 0) {
        vr = -vr;
        vi = -vi;
    }
    *re = vr;
    *im = vi;
}

/*
 * Dense block out[a][b][c][d] = V(P[a], Q[b], R[c], S[d]) as interleaved
 * (re, im) doubles.  n = total number of spinors, irrep[n] = labels.
 */
void fsgen_block(uint64_t seed, double sigma, int n, const int *irrep, int nirrep,
                 const int *P, int np_, const int *Q, int nq, const int *R, int nr,
                 const int *S, int ns, double *out)
{
    const double sc = sigma / sqrt(2.0);
    const long long nab = (long long)np_ * nq;
#pragma omp parallel for schedule(dynamic, 4)
    for (long long ab = 0; ab < nab; ++ab) {
        int a = (int)(ab / nq), b = (int)(ab % nq);
        double *o = out + 2 * ab * (long long)nr * ns;
        for (int c = 0; c < nr; ++c)
            for (int d = 0; d < ns; ++d) {
                double re, im;
                vval(seed, n, irrep, nirrep, P[a], Q[b], R[c], S[d], sc, &re, &im);
                o[2 * (c * ns + d)] = re;
                o[2 * (c * ns + d) + 1] = im;
            }
    }
}

/* The raw draw X_pqrs (exposed so tests can check the projection). */
void fsgen_xraw(uint64_t seed, double sigma, int n, int p, int q, int r, int s, double *out)
{
    xval(seed, (uint64_t)n, p, q, r, s, sigma / sqrt(2.0), &out[0], &out[1]);
}

/*
 * Whole class buffer for a class whose four spaces coincide (OOOO or VVVV),
 * in the boundary layout (allowed (g1,g2,g3) lexicographic, dense
 * [n(g1)][n(g2)][n(g3)][n(g4)] blocks).  Bit-identical to fsgen_block:
 *   pass 1 writes the raw draw X at every position;
 *   pass 2 visits each canonical representative once, reads the (at most 8)
 *   X values of its symmetry orbit and overwrites the orbit with V, using the
 *   same arithmetic as vcanon and exact sign / conjugation images.
 * Orbits are disjoint, so pass 2 runs in place and in parallel.
 *   base  : global index of the first spinor of the space (0 or nocc)
 *   m     : number of spinors of the space; sirrep[m] their labels
 *   n     : total number of spinors (defines the counter L)
 */
void fsgen_class_sym(uint64_t seed, double sigma, int n, int base, int m, const int *sirrep,
                     int nirrep, double *out)
{
    const double sc = sigma / sqrt(2.0);
    int G = nirrep;
    /* per-irrep members and local ranks */
    int *cnt = (int *)calloc(G, sizeof(int));
    int *loc = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    for (int p = 0; p < m; ++p) loc[p] = cnt[sirrep[p]]++;
    int *mstart = (int *)calloc(G + 1, sizeof(int));
    for (int g = 0; g < G; ++g) mstart[g + 1] = mstart[g] + cnt[g];
    int *mem = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    {
        int *fill = (int *)calloc(G, sizeof(int));
        for (int p = 0; p < m; ++p) mem[mstart[sirrep[p]] + fill[sirrep[p]]++] = p;
        free(fill);
    }
    long long *boff = (long long *)malloc(sizeof(long long) * G * G * G);
    long long off = 0;
    for (int g1 = 0; g1 < G; ++g1)
        for (int g2 = 0; g2 < G; ++g2)
            for (int g3 = 0; g3 < G; ++g3) {
                int g4 = ((g1 + g2 - g3) % G + G) % G;
                boff[(g1 * G + g2) * G + g3] = off;
                off += (long long)cnt[g1] * cnt[g2] * cnt[g3] * cnt[g4];
            }
    const long long total = off;
    /* pass 1: raw draws at every position */
#pragma omp parallel for schedule(dynamic, 8)
    for (long long pq = 0; pq < (long long)m * m; ++pq) {
        int p = (int)(pq / m), q = (int)(pq % m);
        int gp = sirrep[p], gq = sirrep[q];
        for (int gr = 0; gr < G; ++gr) {
            int gs = ((gp + gq - gr) % G + G) % G;
            long long b = boff[(gp * G + gq) * G + gr];
            int nr = cnt[gr], ns = cnt[gs];
            long long rowbase = b + ((long long)loc[p] * cnt[gq] + loc[q]) * nr * ns;
            for (int ir = 0; ir < nr; ++ir)
                for (int is = 0; is < ns; ++is) {
                    int r = mem[mstart[gr] + ir], s = mem[mstart[gs] + is];
                    double *o = out + 2 * (rowbase + (long long)ir * ns + is);
                    xval(seed, (uint64_t)n, base + p, base + q, base + r, base + s, sc, &o[0], &o[1]);
                }
        }
    }
    /* pass 2: canonical orbits, in place */
#define POS(a, b, c, d)                                                                  \
    (boff[(sirrep[a] * G + sirrep[b]) * G + sirrep[c]] +                                 \
     (((long long)loc[a] * cnt[sirrep[b]] + loc[b]) * cnt[sirrep[c]] + loc[c]) *         \
         cnt[sirrep[d]] + loc[d])
#pragma omp parallel for schedule(dynamic, 4)
    for (long long pq = 0; pq < (long long)m * m; ++pq) {
        int P = (int)(pq / m), Q = (int)(pq % m);
        if (P > Q) continue;
        if (P == Q) {
            /* X at (P,P,r,s) and (r,s,P,P) belong to no orbit: V is zero there */
            int gPP = (2 * sirrep[P]) % G;
            for (int R = 0; R < m; ++R) {
                int gS = ((gPP - sirrep[R]) % G + G) % G;
                for (int k = mstart[gS]; k < mstart[gS + 1]; ++k) {
                    int S = mem[k];
                    long long a1 = POS(P, P, R, S), a2 = POS(R, S, P, P);
                    out[2 * a1] = 0.0; out[2 * a1 + 1] = 0.0;
                    out[2 * a2] = 0.0; out[2 * a2 + 1] = 0.0;
                }
            }
            continue;
        }
        int gsum = sirrep[P] + sirrep[Q];
        for (int R = P; R < m; ++R) {
            int gS = ((gsum - sirrep[R]) % G + G) % G;
            for (int k = mstart[gS]; k < mstart[gS + 1]; ++k) {
                int S = mem[k];
                if (S <= R) continue;
                if (R == P && S < Q) continue;
                long long i1 = POS(P, Q, R, S), i2 = POS(Q, P, R, S), i3 = POS(P, Q, S, R), i4 = POS(Q, P, S, R);
                long long j1 = POS(R, S, P, Q), j2 = POS(S, R, P, Q), j3 = POS(R, S, Q, P), j4 = POS(S, R, Q, P);
                double ar = ((out[2 * i1] - out[2 * i2]) - out[2 * i3]) + out[2 * i4];
                double ai = ((out[2 * i1 + 1] - out[2 * i2 + 1]) - out[2 * i3 + 1]) + out[2 * i4 + 1];
                double br = ((out[2 * j1] - out[2 * j2]) - out[2 * j3]) + out[2 * j4];
                double bi = ((out[2 * j1 + 1] - out[2 * j2 + 1]) - out[2 * j3 + 1]) + out[2 * j4 + 1];
                double vr = (ar + br) * 0.125, vi = (ai - bi) * 0.125;
                /* images: (pq) and (rs) antisymmetry, Hermitian swap with conjugation */
                out[2 * i1] = vr;  out[2 * i1 + 1] = vi;
                out[2 * i2] = -vr; out[2 * i2 + 1] = -vi;
                out[2 * i3] = -vr; out[2 * i3 + 1] = -vi;
                out[2 * i4] = vr;  out[2 * i4 + 1] = vi;
                if (!(R == P && S == Q)) {
                    out[2 * j1] = vr;  out[2 * j1 + 1] = -vi;
                    out[2 * j2] = -vr; out[2 * j2 + 1] = vi;
                    out[2 * j3] = -vr; out[2 * j3 + 1] = vi;
                    out[2 * j4] = vr;  out[2 * j4 + 1] = -vi;
                }
            }
        }
    }
#undef POS
    (void)total;
    free(cnt); free(loc); free(mstart); free(mem); free(boff);
}
