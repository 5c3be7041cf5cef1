/*
 * fscc.h -- C ABI of the MI355X (gfx950) Fock-space relativistic CCSD hot path.
 *
 * What it computes (Oleynichenko, Zaitsevskii, Eliav, "Towards High
 * Performance Relativistic Electronic Structure Modelling: The EXP-T Program
 * Package", 2020):
 *   - the second-quantised Hamiltonian of Eq. (1) with antisymmetrised
 *     complex integrals <pq||rs> and a diagonal Fock operator (orbital
 *     energies eps), partitioned into dense blocks by irreps (the
 *     symmetry-handling section, Fig. 3);
 *   - the CCSD amplitude equations of Eq. (3)-(4) for the (0h,0p) sector
 *     (Eq. (5) sector partition), evaluated as transpose-transpose-GEMM-
 *     transpose contractions over block lists (algorithm-design section,
 *     Fig. 4), with the particle-particle ladder sum_{c<d} <ab||cd> t_ij^cd
 *     on FP64 matrix cores;
 *   - the Jacobi update t += R/D of Eq. (3) (D = negative H0-eigenvalue
 *     differences) accelerated by DIIS, and the correlation energy.
 *
 * Conventions
 *   Spinors: global index p in [0, nocc) occupied, [nocc, nocc+nvirt) virtual.
 *   Irreps: Abelian Z_nirrep labels; <pq||rs> != 0 only if
 *     irrep(p) + irrep(q) = irrep(r) + irrep(s) (mod nirrep).
 *   Inside an irrep, spinors are ordered by ascending global index
 *   ("irrep-sorted order" = irrep 0 first, then irrep 1, ...).
 *   Complex numbers: fscc_c128 = two doubles (re, im) = C99 double _Complex
 *   = torch.complex128.
 *
 * Packed amplitude / residual layouts (sector (0h,0p)):
 *   T1, R1: for g = 0..nirrep-1: dense [o_g][v_g] row-major block of
 *           t_i^a with irrep(i) = irrep(a) = g.
 *   T2, R2: for G = 0..nirrep-1: dense [n_oo(G)][n_vv(G)] row-major block;
 *           rows = occupied pairs i<j (irrep-sorted order) with
 *           irrep(i)+irrep(j) = G, columns = virtual pairs a<b with
 *           irrep(a)+irrep(b) = G.  Pairs are grouped by (g_p, g_q), g_p <= g_q,
 *           g_p ascending; inside a group p-major (for g_p = g_q the strict
 *           upper triangle, row-major).
 *   fscc_layout() returns the lengths n1 (T1) and n2 (T2).
 *
 * Packed layouts of the (0h,1p) sector (Eq. (5) sector partition; one valence
 * particle in the active virtual spinors A given at fscc_create):
 *   S1, R1: for g = 0..nirrep-1: dense [x_g][v_g] row-major block of s_x^a,
 *           x = active spinors of irrep g (ascending global index), a = ALL
 *           virtual spinors of irrep g.  Entries with a in A are model-space
 *           components, not amplitudes: they are ignored on input and are 0 in R1.
 *   S2, R2: for G = 0..nirrep-1: dense [n_xj(G)][n_vv(G)] row-major block of
 *           s_xj^ab (antisymmetric in ab, stored a<b); rows = pairs (x, j),
 *           x active, j occupied, irrep(x)+irrep(j) = G, grouped by
 *           (irrep(x), irrep(j)) with irrep(x) ascending, x-major inside;
 *           columns exactly as for T2.
 *
 * Integral classes at the boundary (fscc_set_integrals): one contiguous
 *   buffer per class, concatenating over (g1, g2, g3) in lexicographic order,
 *   g4 = (g1 + g2 - g3) mod nirrep, the dense row-major blocks
 *   [n_X1(g1)][n_X2(g2)][n_X3(g3)][n_X4(g4)] (full, not packed).  All
 *   other integrals follow by antisymmetry and Hermiticity
 *   (<pq||rs> = -<qp||rs> = -<pq||sr> = conj <rs||pq>).
 *
 * Ownership and errors
 *   Every pointer argument is owned by the caller.  Amplitude, residual and
 *   integral buffers are DEVICE memory on the context's device; scalar outputs
 *   (max_step, energies, counts) are HOST memory.  The library owns its packed
 *   integrals, intermediates and DIIS history (device memory allocated at
 *   fscc_create / fscc_set_integrals and released by fscc_destroy).
 *   All device work is ordered on the hip_stream given to fscc_create; a
 *   call with host outputs synchronises that stream before returning.
 *   No C++ exception crosses the ABI.  On error the outputs are untouched
 *   (one exception: FSCC_ENOCONV from fscc_update_amplitudes after sustained
 *   growth, where the amplitudes hold the last finite iterate), the call
 *   returns a negative status and fscc_last_error() describes it.
 *   A context must not be used from two host threads at once.
 */
#ifndef FSCC_H
#define FSCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fscc_ctx fscc_ctx;

typedef struct {
    double re, im;
} fscc_c128;

typedef enum {
    FSCC_OK = 0,
    FSCC_EINVAL = -1,  /* bad argument (sizes, pointers, sector, class)          */
    FSCC_ESYMM = -2,   /* input violates antisymmetry / Hermiticity              */
    FSCC_ENOMEM = -3,  /* device allocation failed                               */
    FSCC_EHIP = -4,    /* a HIP runtime call failed                              */
    FSCC_ESTATE = -5,  /* call out of order (e.g. integrals not all set)         */
    FSCC_ENOCONV = -6  /* the amplitude iteration diverges (fscc_update_amplitudes)
                          or an eigenvalue iteration fails (fscc_heff_eig)          */
} fscc_status;

/* Arithmetic of a context.  FSCC_REAL_FP64 (fscc_create only): real double
 * groups -- integrals, amplitudes and residuals are real, every device buffer
 * the caller passes holds DOUBLES (8 bytes per element, the same layouts and
 * element counts as the complex form), the fscc_c128 pointer types of the
 * calls are reinterpreted accordingly, fscc_energy returns e_im = 0 and the
 * host matrices of fscc_heff / fscc_heff2 stay complex with zero imaginary
 * parts; all three sectors, no split precision. */
typedef enum { FSCC_FP64 = 0, FSCC_SPLIT_FP32 = 1, FSCC_SPLIT_BF16 = 2, FSCC_REAL_FP64 = 3 } fscc_precision;

typedef enum { FSCC_S00 = 0, FSCC_S01 = 1, FSCC_S02 = 2 } fscc_sector; /* (0h,0p), (0h,1p), (0h,2p) */

typedef enum { FSCC_OOOO = 0, FSCC_OOOV, FSCC_OOVV, FSCC_OVOV, FSCC_OVVV, FSCC_VVVV } fscc_iclass;

typedef struct {
    int32_t nocc, nvirt, nirrep;
    const int32_t *irrep;  /* host [nocc+nvirt], labels in [0, nirrep)              */
    const double *eps;     /* host [nocc+nvirt], orbital energies (Eh)             */
    int32_t nact;          /* (0h,1p) active virtuals; 0 = (0h,0p) only            */
    const int32_t *active; /* host [nact], global indices of the active virtuals   */
} fscc_system;

/* Build the plan for one system (the second-quantised Hamiltonian of Eq. (1)
 * given by its orbital energies and irrep labels; active virtual spinors
 * select the model space of the (0h,1p) and (0h,2p) sectors of Eq. (5)):
 * irrep-sorted index spaces, block layouts,
 * reorder maps and grouped-GEMM problem lists (the TTGT decomposition of
 * every contraction of the CCSD residual).  hip_stream may be NULL (the null
 * stream).  prec selects the arithmetic of the dominant contractions (see
 * fscc_set_precision).  Device memory for intermediates is allocated here. */
fscc_status fscc_create(const fscc_system *sys, fscc_precision prec, void *hip_stream, fscc_ctx **out);

/* Import one integral class (boundary layout above, n complex elements) and
 * pack it into the library's block layouts (integral sorting, step I of the
 * flowchart).  dev_blocks may be freed on return.  All six classes must be
 * set before fscc_build_residual / fscc_energy.
 * Input checks, before anything is packed (the class then stays unset, so a
 * corrected buffer can be passed again):
 *   - every value is finite (a full scan of the buffer), else FSCC_EINVAL;
 *   - at a sample of elements (fscc_set_validation; 4096 per class by
 *     default, seeded, so a call is reproducible) the symmetries of Eq. (1)'s
 *     antisymmetrised integrals that relate two elements of the same class:
 *     <pq||rs> = -<qp||rs> and <pq||rs> = -<pq||sr> where both indices of a
 *     pair lie in one space, and Hermiticity <pq||rs> = conj <rs||pq> where
 *     (pq) and (rs) span the same spaces (OOOO, OVOV, VVVV; plain symmetry in
 *     a real context), each to 1e-10 of the largest sampled magnitude; a
 *     violation returns FSCC_ESYMM naming the element.  Sampling can miss an
 *     isolated bad element; systematic violations are caught. */
fscc_status fscc_set_integrals(fscc_ctx *ctx, fscc_iclass cls, const fscc_c128 *dev_blocks, size_t n);

/* Number of sampled elements per class for the symmetry checks of
 * fscc_set_integrals (0 = no symmetry checks; the finiteness scan always
 * runs).  0 <= nsample <= 2^20, else FSCC_EINVAL.  Applies to later
 * fscc_set_integrals calls. */
fscc_status fscc_set_validation(fscc_ctx *ctx, int nsample);

/* Streams of the residual evaluations (the block operations of the
 * algorithm-design section, executed as a dependency graph): n = 1 runs every
 * operation in order on the context's stream; n = 2 puts the GEMMs bound by
 * the matrix cores on the context's stream and the reorders, elementwise
 * operations and memory-bound GEMMs on a second stream of the library's
 * (default priority), with an event wait for every dependency between the
 * two (read after write, write after read and write after write on each
 * buffer), so that independent operations of the two kinds overlap.  Work
 * enqueued on the context's stream before a residual is seen by both
 * streams, and the context's stream waits for the second before the call
 * returns, so callers still see one stream.  Results are bitwise the same
 * (each operation's arithmetic is unchanged and the dependencies fix every
 * buffer's order of writes).  Out-of-core VVVV and batched contexts always
 * run on one stream.  n other than 1 or 2: FSCC_EINVAL. */
fscc_status fscc_set_streams(fscc_ctx *ctx, int n);

/* Packed lengths (complex elements) of T1/R1 and T2/R2 for a sector (for
 * FSCC_S02: n1 = 0 and n2 = the length of S_xy^ab, see fscc_heff2): the
 * amplitudes of the wave operator of Eq. (2) restricted to the sector of
 * Eq. (5), stored as the symmetry blocks of the block partition (Fig. 3) in
 * the layouts given at the top of this file.  FSCC_EINVAL for a sector the
 * system does not have (no active spinors, fewer than two for FSCC_S02). */
fscc_status fscc_layout(const fscc_ctx *ctx, fscc_sector sector, size_t *n1, size_t *n2);

/* R = RHS - D*t for the CCSD equations (Eq. (3)), D_i^a = e_i - e_a,
 * D_ij^ab = e_i + e_j - e_a - e_b.  t1, t2 inputs; r1, r2 outputs (device,
 * packed layouts; must not alias the inputs).  Asynchronous on the stream. */
fscc_status fscc_build_residual(fscc_ctx *ctx, fscc_sector sector, const fscc_c128 *t1, const fscc_c128 *t2,
                                fscc_c128 *r1, fscc_c128 *r2);

/* Jacobi step of Eq. (3): step = R/D, t' = t + step; then DIIS over the last
 * ndiis (t', step) pairs (B_kl = Re <step_k, step_l> over the packed unique
 * amplitudes, bordered Pulay system solved on the device in FP64) writes the
 * extrapolated amplitudes into t1, t2.  *max_step (host) = max |step|.
 * Divergence (the intruder-state failure of the iteration): the largest step
 * of every iteration is watched per sector; a step more than 1e3 times the
 * smallest one since the watch started (that smallest one taken as at least
 * 1e-8) clears the DIIS subspace and restarts the watch from that step; a
 * second such growth returns FSCC_ENOCONV with *max_step set and t1, t2
 * holding the last (finite) iterate.  A step that is not finite returns
 * FSCC_ENOCONV at once with t1, t2 left at their input values.  Either
 * failure clears the DIIS subspace; fscc_diis_reset, fscc_prepare_sector,
 * fscc_precondition and fscc_dynamic_shift restart the watch. */
fscc_status fscc_update_amplitudes(fscc_ctx *ctx, fscc_sector sector, fscc_c128 *t1, fscc_c128 *t2,
                                   const fscc_c128 *r1, const fscc_c128 *r2, double *max_step);

/* Prepare the (0h,1p) sector from converged (0h,0p) amplitudes t1, t2 (device):
 * builds the one- and two-body elements of Hbar = exp(-T) H exp(T) used by
 * the sector's equations (kept by the library) and clears the sector's DIIS
 * history.  Must be called before fscc_build_residual / fscc_heff with
 * sector FSCC_S01, and again if T changes. */
fscc_status fscc_prepare_sector(fscc_ctx *ctx, fscc_sector sector, const fscc_c128 *t1, const fscc_c128 *t2);

/* (0h,1p) sector, with sector = FSCC_S01 in fscc_build_residual: for every
 * active x, r(x) = e_x + s_x and sigma(x) = Hbar_N r(x) on the {1p, 2p1h}
 * space; H_eff[y][x] = sigma(x)^y (y in A) is the closed part of Eq. (3)'s
 * Omega (V Omega)_Cl, and the residual is the Bloch equation
 *   R1_x^a = sigma(x)^a - sum_y s_y^a H_eff[y][x]   (a not in A),
 *   R2_xj^ab = sigma(x)_j^ab - sum_y s_yj^ab H_eff[y][x],
 * with Jacobi denominators D_x^a = e_x - e_a, D_xj^ab = e_x + e_j - e_a - e_b
 * in fscc_update_amplitudes(FSCC_S01, ...).
 * fscc_heff returns H_eff = (H Omega)_Cl for amplitudes s1, s2 as a dense
 * row-major nact x nact complex matrix heff_host[y][x] (host memory), rows
 * and columns in the order of sys->active; its eigenvalues are the (0h,1p)
 * state energies relative to the (0h,0p) reference state.  Synchronises. */
fscc_status fscc_heff(fscc_ctx *ctx, const fscc_c128 *s1, const fscc_c128 *s2, fscc_c128 *heff_host);

/* (0h,2p) sector (the next step of the sector hierarchy of Eq. (5), two valence
 * particles; present when nact >= 2).  Prepared with fscc_prepare_sector(ctx,
 * FSCC_S02, s1, s2) from CONVERGED (0h,1p) amplitudes s1, s2 (device, the
 * FSCC_S01 layouts) after the (0h,1p) preparation; repeat if s1, s2 or T
 * change (a new (0h,1p) preparation invalidates it).  Amplitudes s_xy^ab for
 * active pairs x < y and virtual pairs a < b that are not both active,
 * layout [G][xy<][ab<] (G = irrep(x)+irrep(y) = irrep(a)+irrep(b), pairs as in
 * the T2 layout over the irrep-sorted active spinors; n1 = 0, pass t1 = r1 =
 * NULL).  With the normal-ordered wave operator, Omega|xy> = R_x R_y|Phi> +
 * S_xy|Phi> where R_x attaches the dressed particle r(x) = e_x + s_x of the
 * (0h,1p) sector; sigma2(xy) = [Hbar_N Omega|xy>] on the 2p space,
 * H_eff[zw][xy] = sigma2(xy)^zw, and fscc_build_residual(FSCC_S02, NULL, s,
 * NULL, r) writes the Bloch residual
 *   R_xy^ab = sigma2(xy)^ab - sum_{z<w} omega(zw)^ab H_eff[zw][xy],
 *   omega(zw)^ab = r(z)^a r(w)^b - r(z)^b r(w)^a + s_zw^ab,
 * zero on the model pairs; Jacobi denominators D_xy^ab = e_x + e_y - e_a - e_b
 * in fscc_update_amplitudes(FSCC_S02, NULL, s, NULL, r, ...); dynamic shifts
 * as for FSCC_S01.  fscc_heff2 returns H_eff for amplitudes s as a dense
 * row-major P x P complex matrix heff_host[pair(zw)][pair(xy)] (host memory,
 * P = nact(nact-1)/2), pairs i < j of positions in sys->active ordered
 * row-major over the upper triangle; its eigenvalues are the (0h,2p) state
 * energies relative to the (0h,0p) reference state.  Synchronises. */
fscc_status fscc_heff2(fscc_ctx *ctx, const fscc_c128 *s, fscc_c128 *heff_host);

/* Eigenvalues of an effective Hamiltonian (step V of the flowchart, Fig. 1:
 * diagonalise H_eff = (H Omega)_Cl of a sector; its eigenvalues are the state
 * energies relative to the (0h,0p) reference): heff_host is a dense row-major
 * n x n complex matrix in host memory (e.g. the output of fscc_heff or
 * fscc_heff2), eig_host receives its n eigenvalues sorted by real part (ties
 * by imaginary part).  Host code only (no device work, no context): Householder
 * reduction to Hessenberg form, then single-shift complex QR iterations with
 * the Wilkinson shift and deflation.  FSCC_EINVAL for n outside 0..4096, null
 * arrays or non-finite elements; FSCC_ENOCONV if the QR iteration does not
 * converge in 60 n steps. */
fscc_status fscc_heff_eig(int n, const fscc_c128 *heff_host, fscc_c128 *eig_host);

/* Jacobi denominators of a sector.  mode 0: D from the orbital energies
 * (Eq. (3)-(4), the default).  mode 1, dressed: sector FSCC_S01 (after
 * fscc_prepare_sector): D from the diagonal of Hbar, D_x^a = Re(Fbar_xx -
 * Fbar_aa), D_xj^ab = Re(Fbar_xx + Fbar_jj - Fbar_aa - Fbar_bb); sector
 * FSCC_S00 (after a (0h,0p) residual evaluation, FSCC_ESTATE before one): the
 * diagonal of the amplitude equations at the amplitudes of that residual,
 * f_p = e_p + Re F'_pp with the one-body intermediates F'_be (virtual) and
 * F'_mj (occupied) that multiply t2 in Eq. (3), D_i^a = f_i - f_a and
 * D_ij^ab = f_i + f_j - f_a - f_b; clamped to <= -floor (floor > 0, Eh).  The
 * dressed denominators are computed once per call (call again to refresh
 * them).  Only the step changes, not the solution of the amplitude or Bloch
 * equations; clears the sector's DIIS history. */
fscc_status fscc_precondition(fscc_ctx *ctx, fscc_sector sector, int mode, double floor);

/* Device copies of the Jacobi denominators the (0h,0p) update uses now
 * (sector = FSCC_S00: the bare e_i - e_a, e_i + e_j - e_a - e_b, or the
 * dressed ones after fscc_precondition mode 1), in the packed T1 / T2
 * layouts, without level shift.  D1, D2: device arrays of n1, n2 doubles
 * (fscc_layout), owned by the caller.  Asynchronous on the stream. */
fscc_status fscc_denominators(fscc_ctx *ctx, fscc_sector sector, double *D1, double *D2);

/* One whole (0h,0p) iteration with a single synchronisation: the residual
 * of t1, t2 into r1, r2 (as fscc_build_residual), the Jacobi + DIIS update of
 * t1, t2 (as fscc_update_amplitudes) and the energy of the updated amplitudes
 * (as fscc_energy), all enqueued before the host waits once for the step size
 * and the energy.  Same arguments, layouts and errors as those three calls;
 * on FSCC_ENOCONV *e_re, *e_im hold the energy of whatever t1, t2 then hold. */
fscc_status fscc_iterate(fscc_ctx *ctx, fscc_c128 *t1, fscc_c128 *t2, fscc_c128 *r1, fscc_c128 *r2, double *max_step,
                         double *e_re, double *e_im);

/* Correlation energy of the (0h,0p) sector, the expectation value of Eq. (1)'s
 * normal-ordered Hamiltonian in the coupled-cluster state of Eq. (2):
 * E = sum_{i<j,a<b} <ij||ab> (t_ij^ab + t_i^a t_j^b - t_i^b t_j^a) (the f_ia term
 * vanishes for the diagonal Fock operator), complex in general (complex
 * integrals without time-reversal symmetry; the real part is the correlation
 * energy).  t1, t2: device, packed (0h,0p) layouts; e_re, e_im: host.
 * FSCC_ESTATE before the OOVV class is set.  Synchronises the stream. */
fscc_status fscc_energy(fscc_ctx *ctx, const fscc_c128 *t1, const fscc_c128 *t2, double *e_re, double *e_im);

/* Clear the DIIS history of a sector and set its depth (0 or 1 = plain Jacobi
 * of Eq. (3), max 16; the context keeps 16 vector pairs per sector on the
 * device); also restarts the sector's divergence watch (see
 * fscc_update_amplitudes).  FSCC_EINVAL for a depth outside 0..16 or a sector
 * the system does not have. */
fscc_status fscc_diis_reset(fscc_ctx *ctx, fscc_sector sector, int ndiis);

/* The particle-particle ladder alone: out_ij^ab = sum_{c<d} <ab||cd> tau_ij^cd
 * (T2 layouts, device; out overwritten).  The dominant contraction of the
 * residual, exposed for parity checks and timing. */
fscc_status fscc_ladder(fscc_ctx *ctx, const fscc_c128 *tau, fscc_c128 *out);

/* Work counts of one residual evaluation: real flops of all grouped GEMMs,
 * of the ladder alone, and its vvvv bytes (host outputs). */
fscc_status fscc_work(const fscc_ctx *ctx, double *gemm_flops, double *ladder_flops, double *ladder_bytes);

/* Per-operation timing.  fscc_profile(ctx, 1) makes every residual
 * evaluation record HIP events around each operation on the stream;
 * fscc_op_count returns the number of operations; fscc_op_info(k) returns
 * the name (static until destroy), accumulated milliseconds, number of
 * timed calls and real flops per call of operation k (host outputs). */
fscc_status fscc_profile(fscc_ctx *ctx, int enable);

/* While profiling is enabled, record events only around operation k
 * (k = -1: every operation, the default).  Events are read back when the
 * next residual evaluation starts or by fscc_op_info / fscc_profile, so
 * profiling adds no stream synchronisation; timing one operation leaves the
 * others' launch sequence untouched.  FSCC_EINVAL if k is not an operation. */
fscc_status fscc_profile_select(fscc_ctx *ctx, int k);
fscc_status fscc_op_count(const fscc_ctx *ctx, int *count);
/* Kind and algorithmic bytes of one call of operation k (host outputs):
 * kind 0 = reorder / antisymmetriser (a gather: steps 1, 2 and 4 of the TTGT
 * scheme of the algorithm-design section), 1 = grouped GEMM (step 3),
 * 2 = elementwise.  Bytes: every destination element written once (and read
 * once when accumulating), every distinct source element read once (the
 * structural zeros of a reorder read nothing; index maps are not counted),
 * every GEMM operand element read once.  With the measured time per call
 * (fscc_op_info) this gives each operation's HBM rate. */
fscc_status fscc_op_traffic(const fscc_ctx *ctx, int k, int *kind, double *bytes);
fscc_status fscc_op_info(fscc_ctx *ctx, int k, const char **name, double *ms, int *calls, double *flops);
/* Run operation k alone, reps times (1..1000), on the buffers bound by the
 * last residual evaluation of its sector (FSCC_ESTATE before one): a single
 * reorder or GEMM of the TTGT scheme in isolation, for profiling its kernel
 * (e.g. its HBM counters per dispatch).  Accumulating operations keep
 * accumulating, so the sector's residual buffers hold no result afterwards.
 * Asynchronous on the stream. */
fscc_status fscc_op_run(fscc_ctx *ctx, int k, int reps);

/* Tile-shape autotuner for the grouped complex GEMMs (the block contractions
 * of Fig. 4 have very uneven shapes).  level 1: every candidate tile shape,
 * K depth (16/32) and split-K choice of each GEMM operation is timed on the
 * device (HIP events on the context's stream) and the fastest is kept, then
 * for an MFMA winner its four-product complex form is timed against the
 * default three-product form (FSCC_CFG_3M) and the faster kept;
 * in a split precision (fscc_set_precision) level 1 also times the split
 * kernel's tile shapes of the split operations; level 2 times only those;
 * level 0: restore the cost-model defaults chosen at fscc_create (FP64
 * shapes; 16-deep K slices, split-K allowed, the direct-to-LDS form
 * FSCC_CFG_DL wherever the tile has one).  Level 1 also times the double-buffered LDS form (FSCC_CFG_DB) and
 * the direct-to-LDS form (FSCC_CFG_DL) of every eligible tile.  Level 1 also times each reorder (gather) of a complex context in
 * destination order, by 16 x 16 destination tiles and by affine tiles (see
 * fscc_gather_order) and keeps the fastest.
 * Results are numerically equivalent (summation order may change). */
fscc_status fscc_autotune(fscc_ctx *ctx, int level);

/* Autotune result cache (the paper's proposal to choose each block
 * operation's parallelism from a first-iteration profile, kept across runs):
 * with a path set, fscc_autotune(ctx, 1 or 2) first looks in that JSON file
 * for an entry keyed by the GPU architecture, the precision, the level, the
 * library's kernel-set version and a hash of every operation of the
 * context's plans (kinds, sizes, GEMM problem shapes); if one fits it is
 * applied without timing anything, otherwise every candidate is timed as
 * usual and the choices are written to the file (entries of other keys are
 * kept; the file is replaced through a rename).  path NULL or "" switches the
 * cache off (the default).  An unreadable or unwritable file only costs the
 * timing.  fscc_autotune_cached reports whether the last fscc_autotune call
 * applied cached choices (1) or measured (0). */
fscc_status fscc_tune_cache(fscc_ctx *ctx, const char *path);
fscc_status fscc_autotune_cached(const fscc_ctx *ctx, int *from_cache);

/* Traversal of the reorders / antisymmetrisers (gathers) of every operation
 * list (steps 1, 2 and 4 of the TTGT scheme of the algorithm-design section):
 * tiled = 0 walks each destination in storage order through per-element
 * index maps, tiled = 1 in 16 x 16 tiles of its blocks, tiled = 2 in affine
 * tiles (at most 16 x 16) on which each term's source index is an affine
 * function of the destination row and column: no index map is read there,
 * the source is read with consecutive lanes on consecutive elements and a
 * transposed term is staged through LDS so that the destination is written
 * along its rows; a term without an affine form on a tile uses its map
 * (gathers with a second operand fall back to tiled = 1).  Complex contexts;
 * a real context always uses storage order.  The results are bitwise
 * identical.  Replaces the choice fscc_autotune(ctx, 1) made.  FSCC_EINVAL for
 * another value. */
fscc_status fscc_gather_order(fscc_ctx *ctx, int tiled);

/* MFMA tile ids of fscc_zgemm / fscc_gemm_config may carry this bit: the
 * complex product is formed from three real matrix products (Ar Br, Ai Bi,
 * (Ar + Ai)(Br + Bi); Re = P1 - P2, Im = P3 - P1 - P2) instead of four.
 * Contexts use it for every MFMA-tile GEMM unless the autotuner measured
 * the four-product form faster.  Rounding: the imaginary part's error bound
 * grows from ~u sum|Ar Bi| + |Ai Br| to ~u sum(|Ar| + |Ai|)(|Br| + |Bi|). */
#define FSCC_CFG_3M 256

/* MFMA tile ids may also carry this bit: double-buffered LDS (two buffer
 * pairs per operand, one barrier per K slice: the next slice is stored while
 * the matrix cores work on the current one).  Needs bk = 16 and one of the
 * tiles 3: 32x32, 4: 64x16, 5: 16x64, 9: 32x64, 10: 64x32, 13: 64x32 stacked
 * (their two buffer pairs stay within 64 KB of LDS); FSCC_EINVAL otherwise.
 * The result is the same (same summation order). */
#define FSCC_CFG_DB 512

/* MFMA tile ids may instead carry this bit: the K slices are loaded from
 * device memory straight into LDS (one complex element per lane and load,
 * no register staging) into two LDS stages: the next slice arrives while the
 * matrix cores work on the current one, and the smaller register and LDS
 * footprint lets more workgroups share a CU.
 * Needs bk = 16 and one of the tiles 0: 64x64, 3: 32x32, 4: 64x16,
 * 5: 16x64, 9: 32x64, 10: 64x32, 12: 64x64 stacked, 13: 64x32 stacked;
 * FSCC_EINVAL otherwise or together with FSCC_CFG_DB.  The result is the
 * same (same summation order). */
#define FSCC_CFG_DL 1024

/* Chosen configuration of operation k (cfg = tile shape id, with
 * FSCC_CFG_3M set for a three-product MFMA tile, FSCC_CFG_DB for a
 * double-buffered one and FSCC_CFG_DL for a direct-to-LDS one, or -1 if k
 * is not a GEMM;
 * bk = K depth; split = 1 if split along K); host outputs. */
fscc_status fscc_gemm_config(const fscc_ctx *ctx, int k, int *cfg, int *bk, int *split);

/* One complex GEMM through the grouped MFMA kernel, for kernel-level tests:
 * C = alpha * op(A) op(B) + beta*C with op = transpose (tA/tB) and/or
 * conjugate (cA/cB); A is M x K (lda) or, if tA, K x M; B is K x N (ldb) or,
 * if tB, N x K; all row-major, device pointers.  cfg = kernel form: MFMA tile
 * shapes 0: 64x64, 1: 128x16, 2: 16x128, 3: 32x32, 4: 64x16, 5: 16x64,
 * 9: 32x64, 10: 64x32, and 12: 64x64, 13: 64x32 with the four waves
 * stacked along M (a wave whose 16 rows lie past M issues no MFMA);
 * vector-ALU forms 6: skinny (64x32 output blocks), 7: tall (needs !tA,
 * K <= 64, K*N <= 1024), 8: reduction (needs !tB, M <= 8, N <= 256),
 * 11: dot (needs !tA, tB, M <= 8; every B row streamed once);
 * an MFMA tile id | FSCC_CFG_3M selects the three-product complex form,
 * | FSCC_CFG_DB or | FSCC_CFG_DL the LDS staging form (see above);
 * -1 = cost model (three-product form).  FSCC_EINVAL if the shape does not
 * fit the form.
 * bk = 16 or 32, allow_split = 1 permits split-K.  beta is 0 or 1.
 * Synchronises hip_stream. */
fscc_status fscc_zgemm(int cfg, int bk, int tA, int tB, int cA, int cB, int M, int N, int K, const fscc_c128 *A, int lda,
                       const fscc_c128 *B, int ldb, fscc_c128 *C, int ldc, double alpha_re, double alpha_im, int beta,
                       int allow_split, void *hip_stream);

/* Size of the static device array of fscc_zgemm_noalloc (bytes per GPU). */
#define FSCC_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* fscc_zgemm for callers that cannot allocate device memory (serving loops,
 * harnesses that forbid hipMalloc): the same arguments, kernels and result,
 * but the problem / tile / split-K tables and the split-K partial sums live in
 * one static device array of FSCC_NOALLOC_SCRATCH_BYTES per GPU (held until
 * the process ends) instead of buffers allocated per call; no hipMalloc or
 * hipFree is called.  A K split whose partial sums do not fit the array runs
 * unsplit; a plan whose tables alone do not fit returns FSCC_EINVAL.  Every
 * call on one GPU uses that GPU's array: calls that overlap on one GPU (from
 * two host threads at once) race.  Synchronises hip_stream.  The message of
 * a failed call (of this one or fscc_zgemm) is fscc_last_error(NULL) on the
 * calling thread. */
fscc_status fscc_zgemm_noalloc(int cfg, int bk, int tA, int tB, int cA, int cB, int M, int N, int K,
                               const fscc_c128 *A, int lda, const fscc_c128 *B, int ldb, fscc_c128 *C, int ldc,
                               double alpha_re, double alpha_im, int beta, int allow_split, void *hip_stream);

/* Real form of fscc_zgemm (kernel-level tests of the real-arithmetic path):
 * C = alpha * op(A) op(B) + beta*C on doubles, same layout conventions and
 * kernel forms except 6 (skinny), which has no real form (FSCC_EINVAL); an
 * MFMA tile id may carry FSCC_CFG_DL (the direct-to-LDS form: each double
 * moves as two 4-byte direct-to-LDS loads; bk = 16 and the tiles listed at
 * FSCC_CFG_DL), not FSCC_CFG_3M or FSCC_CFG_DB.  Synchronises hip_stream. */
fscc_status fscc_dgemm(int cfg, int bk, int tA, int tB, int M, int N, int K, const double *A, int lda, const double *B,
                       int ldb, double *C, int ldc, double alpha, int beta, int allow_split, void *hip_stream);

/* Level shift (Eh, >= 0) of the (0h,0p) Jacobi step: step = R / (D - shift)
 * with D < 0 for every T1/T2 denominator, so the update is damped; the fixed
 * point R = 0 is unchanged.  Default 0.  sector must be FSCC_S00.  Applies
 * from the next fscc_update_amplitudes. */
fscc_status fscc_level_shift(fscc_ctx *ctx, fscc_sector sector, double shift);

/* Out-of-core <ab||cd> (the paper's block-contraction loop that loads each
 * integral block from disk while the contraction runs, Fig. 4; for systems
 * whose packed VVVV does not fit the GPU): with staging_bytes > 0 the packed
 * VVVV integrals move to pinned host memory (their device copy is freed) and
 * every GEMM that reads them (the particle-particle ladders of both sectors)
 * streams them through two device staging buffers of staging_bytes / 2 each:
 * a copy stream brings one chunk of integral rows while the matrix cores
 * work on the previous one.  Problems are cut along the ladder's ab index to
 * fit a staging buffer; results equal the in-memory ones up to summation
 * order.  staging_bytes = 0 moves VVVV back to device memory.  Needs all
 * integrals set and FP64 precision; afterwards fscc_autotune and split
 * precision are refused (FSCC_ESTATE) until VVVV is back.  FSCC_EINVAL if a
 * staging buffer cannot hold one integral row (nvv pairs of the largest
 * block). */
fscc_status fscc_vvvv_out_of_core(fscc_ctx *ctx, size_t staging_bytes);

/* Dynamic denominator shifts against intruder states (the FS-RCC method's
 * shifting of ill-defined, nearly zero or positive, energy denominators,
 * followed by extrapolation to zero shift).  With S < 0 (Eh) and integer
 * exponent n (1..16) every amplitude K of the sector gets
 *   Delta_K = S * (S / (min(D_K, 0) + S))^n
 * (D_K: the sector's Jacobi denominator in use), and the solved equations
 * become R_K = Delta_K s_K: fscc_update_amplitudes takes the step
 * (R - Delta s) / (D + Delta).  Delta = S where D = 0 and decays as
 * S (S/D)^n for |D| >> |S|.  S = 0 switches the shift off (n ignored).
 * Clears the sector's DIIS history.  FSCC_EINVAL for S > 0, S <= -1e6, n out
 * of range, or FSCC_S01 / FSCC_S02 on a context without the sector.  Contexts of the
 * batch API do not take shifts. */
fscc_status fscc_dynamic_shift(fscc_ctx *ctx, fscc_sector sector, double S, int n);

/* Value at x0 of the [L/M] Pade approximant
 *   E(x) = (a_0 + a_1 x + ... + a_L x^L) / (1 + b_1 x + ... + b_M x^M)
 * fitted to npts points (x[i], y[i]) by linearised least squares
 * (sum_j a_j x^j - y sum_{j>=1} b_j x^j = y), e.g. state energies at shifts
 * x_i * S extrapolated to x0 = 0.  Host arrays; host code only (no device
 * work).  npts >= L + M + 1, L + M + 1 <= 17, npts <= 4096.  FSCC_EINVAL on
 * bad sizes, non-finite input, a rank-deficient system or a non-finite
 * result. */
fscc_status fscc_pade(int npts, const double *x, const fscc_c128 *y, int L, int M, double x0, fscc_c128 *out);

/* Arithmetic of the dominant (0h,0p) contractions: the particle-particle
 * ladder sum_{c<d} <ab||cd> tau_ij^cd and the two ring GEMM sets (the T2
 * part of W_mbej and sum_me t_im^ae W_mbej), which together carry most of
 * the flops of an iteration, and in FSCC_SPLIT_BF16 also the ladder's T1 part
 * Z_ij^am = sum_{e<f} <am||ef> tau_ij^ef and the (0h,1p) sector's ladder
 * sum_{e<f} <ab||ef> s_xj^ef (Eq. (6)).  Every other step -- the remaining contractions, the reorders,
 * the denominator (Jacobi) update, the DIIS subspace solve and the energy --
 * stays FP64 in every mode.
 *   FSCC_FP64        complex FP64 on the FP64 matrix cores.
 *   FSCC_SPLIT_BF16  each FP64 operand value is written as three bf16 pieces
 *                    (x ~ h0 + h1 + h2, each piece the rounded remainder of
 *                    the previous ones); a product keeps the six piece
 *                    products of order <= 2 (exact in fp32) on the bf16
 *                    matrix cores with fp32 accumulation; every 32-deep
 *                    k block of fp32 sums is added into FP64, and the
 *                    alpha/beta epilogue is FP64.  Relative error of one
 *                    output element ~1e-7 of sum_k |a_k||b_k|.
 *   FSCC_SPLIT_FP32  two fp32 pieces (hi + lo), three products (hi hi,
 *                    hi lo, lo hi) on the fp32 matrix cores, same
 *                    accumulation; same order of accuracy.
 * Constant operands (integrals) are split once and kept (12 B per complex
 * element for bf16, 16 B for fp32, beside their FP64 copy); amplitude
 * operands are split on every call.  Switching is allowed between residual
 * calls; DIIS history is kept.  The first switch to a split mode allocates
 * the piece buffers. */
fscc_status fscc_set_precision(fscc_ctx *ctx, fscc_precision prec);
fscc_status fscc_get_precision(const fscc_ctx *ctx, int *prec);

/* Split-kernel tile shape of operation k in the current precision (host
 * output; -1 if k does not run in split precision now).  Shapes: 0: 64x64,
 * 1: 64x32, 2: 32x64, 3: 32x32; 4..7: the same tiles with the B operand's
 * fragments loaded from device memory straight into registers (only A staged
 * in LDS).  fscc_autotune(ctx, 1) in a split mode also measures these
 * shapes. */
fscc_status fscc_mixed_config(const fscc_ctx *ctx, int k, int *cfg);

/* One complex GEMM through the split-precision kernel (kernel-level tests):
 * same operand conventions as fscc_zgemm; prec = FSCC_SPLIT_BF16 or
 * FSCC_SPLIT_FP32; cfg = split tile shape (0..7).  Allocates and frees its
 * piece buffers; synchronises hip_stream. */
fscc_status fscc_zgemm_split(int prec, int cfg, int tA, int tB, int cA, int cB, int M, int N, int K,
                             const fscc_c128 *A, int lda, const fscc_c128 *B, int ldb, fscc_c128 *C, int ldc,
                             double alpha_re, double alpha_im, int beta, void *hip_stream);

void fscc_destroy(fscc_ctx *ctx);
/* Message of the last failed call on ctx; with ctx = NULL, of the last failed
 * context-free GEMM call (fscc_zgemm, fscc_zgemm_noalloc) on this thread. */
const char *fscc_last_error(const fscc_ctx *ctx);

/* ---- batches of independent systems (the block-loop structure of Fig. 4
 * extended over systems) -------------------------------------------------
 * A batch holds nsys (0h,0p) systems (nact must be 0).  Their residual plans
 * are concatenated buffer by buffer, so every contraction runs as ONE grouped
 * GEMM launch over the symmetry blocks of all systems, and every reorder and
 * elementwise step as one launch over the concatenation.  Amplitude and
 * residual vectors of a batch are the concatenations of the systems' packed
 * vectors (fscc_layout order): T1 of system 0, T1 of system 1, ... and
 * likewise T2; fscc_batch_segment gives each system's offsets.  Each system
 * keeps its own Jacobi + DIIS subspace on the device; once its max|step|
 * falls below tol it is frozen (amplitudes no longer updated, its GEMM tiles
 * skipped) while the others continue.  A batch owns its device memory and is
 * not thread-safe; calls are asynchronous on hip_stream unless stated. */
typedef struct fscc_batch fscc_batch;

/* sys[nsys] as for fscc_create.  Plans are built in parallel host threads. */
fscc_status fscc_batch_create(const fscc_system *sys, int nsys, fscc_precision prec, void *hip_stream,
                              fscc_batch **out);
void fscc_batch_destroy(fscc_batch *b);
const char *fscc_batch_last_error(const fscc_batch *b);

/* Totals of the concatenated T1 / T2 vectors, and system s's segments. */
fscc_status fscc_batch_sizes(const fscc_batch *b, size_t *n1, size_t *n2);
fscc_status fscc_batch_segment(const fscc_batch *b, int s, size_t *off1, size_t *n1, size_t *off2, size_t *n2);

/* Integral class of system s, boundary layout as fscc_set_integrals
 * (synchronous; dev_blocks may be freed on return). */
fscc_status fscc_batch_set_integrals(fscc_batch *b, int s, fscc_iclass cls, const fscc_c128 *dev_blocks, size_t n);

/* Fresh DIIS subspaces (depth ndiis in 1..8) for every system, all systems
 * active, convergence threshold tol on max|step|, level shift >= 0 (Eh): the
 * Jacobi step is R / (D - shift) (D < 0), which damps the update and leaves
 * the fixed point R = 0 unchanged (default after create: 6, 1e-10, 0).
 * Drops a captured graph. */
fscc_status fscc_batch_reset(fscc_batch *b, int ndiis, double tol, double shift);

/* Residuals of all systems, R = RHS - D*t (Eq. (3)) (rows of frozen systems
 * are not meaningful). */
fscc_status fscc_batch_build_residual(fscc_batch *b, const fscc_c128 *t1, const fscc_c128 *t2, fscc_c128 *r1,
                                      fscc_c128 *r2);

/* One iteration for every active system: residual, Jacobi step, DIIS
 * extrapolation, energy of the new amplitudes.  use_graph = 1 replays a HIP
 * graph of the whole iteration (captured on first use for these four
 * pointers, re-captured when they change).  Synchronous: report[nsys*6]
 * (host) receives per system E_re, E_im, max|step| of this iteration (last
 * value for frozen systems), active (1 = not yet converged), iterations
 * taken, failed (1 = non-finite step; the system is frozen). */
fscc_status fscc_batch_step(fscc_batch *b, fscc_c128 *t1, fscc_c128 *t2, fscc_c128 *r1, fscc_c128 *r2,
                            int use_graph, double *report);

/* Fresh DIIS subspace for the systems with mask[s] != 0 (host array [nsys]):
 * they become active again and their next step starts from whatever
 * amplitudes their segments then hold; iteration counts keep running.
 * Synchronous. */
fscc_status fscc_batch_restart(fscc_batch *b, const int *mask);

/* Jacobi denominators of every system of the batch, as fscc_precondition for
 * the (0h,0p) sector: mode 0 the bare orbital-energy differences (default),
 * mode 1 the dressed ones, f_i + f_j - f_a - f_b with f_p = e_p + Re F'_pp
 * from each system's F'_be, F'_mj of the last residual evaluation (FSCC_ESTATE
 * before the first step or residual), clamped to <= -floor (floor > 0, Eh);
 * the step is R / (D - shift).  The solution R = 0 is unchanged.  Every
 * system's DIIS subspace restarts (active flags and iteration counts are
 * kept); switching between modes drops a captured graph.  Synchronous. */
fscc_status fscc_batch_precondition(fscc_batch *b, int mode, double floor);

/* Device copies of the batch's Jacobi denominators D (concatenated T1 / T2
 * layouts, e_i - e_a and e_i + e_j - e_a - e_b, without level shift). */
fscc_status fscc_batch_denominators(fscc_batch *b, double *D1, double *D2);

/* Per system s: out[s] = max |r / D| over its T1 and T2 segments (host
 * output, synchronous) -- the size of the Jacobi step a residual r implies. */
fscc_status fscc_batch_maxnorm(fscc_batch *b, const fscc_c128 *r1, const fscc_c128 *r2, double *out);

/* The batch's executor, for the introspection calls only (fscc_profile,
 * fscc_op_count, fscc_op_info, fscc_autotune, fscc_gemm_config): its
 * operations are the merged grouped launches.  Owned by the batch. */
fscc_ctx *fscc_batch_context(fscc_batch *b);

/* ---- matrix-core throughput probe -------------------------------------
 * The roofline of the GEMMs (the contractions of Eq. (3) and of the sector
 * equations run as block matrix products on the matrix cores) measured on
 * this GPU at the clock it runs: kind 0 = FP64 v_mfma_f64_16x16x4f64,
 * 1 = BF16 v_mfma_f32_16x16x32_bf16 (fp32 accumulation), 2 = FP32
 * v_mfma_f32_16x16x4f32.  Every wave runs 8 independent accumulator chains of
 * iters instructions each from register operands (no memory traffic), four
 * waves per workgroup, as many workgroups per compute unit as are resident
 * at once (hipOccupancyMaxActiveBlocksPerMultiprocessor); one untimed launch
 * first, then one launch timed with HIP events on hip_stream (NULL: the
 * default stream).  *tflops = issued flops (2*16*16*k per instruction) / time;
 * *ms (may be NULL) = the timed launch.  Allocates and frees a small device
 * buffer; synchronous.  FSCC_EINVAL for another kind, iters outside
 * 1..2^20 or tflops NULL; FSCC_ENOMEM / FSCC_EHIP on runtime failures. */
fscc_status fscc_probe_mfma(int kind, int iters, void *hip_stream, double *tflops, double *ms);

/* ---- learned warm start ----------------------------------------------
 * A small network predicts the converged T2 amplitudes from quantities of
 * the first two Jacobi iterates, to start the iteration of Eq. (3) closer to
 * its fixed point.  Per packed T2 element: u = MP2 amplitude (the Jacobi
 * iterate from t = 0), r = the residual at u, D = the denominator,
 * v = r / D, s = |u| + |v| + 1e-30.
 *   features x[8] = (Re u/s, Im u/s, Re v/s, Im v/s,
 *                    clip(ln((|v|+1e-30)/(|u|+1e-30)), -10, 10)/10, D/10,
 *                    ln(s)/10, |v|/s)                              (fp32)
 *   network  h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3,
 *            8 -> 256 -> 256 -> 4, fp32, W stored [in][out]; the flat
 *            parameter vector is W1, b1, W2, b2, W3, b3 (69124 floats)
 *   head     t = u + v + a v + b u with a = y0 + i y1, b = y2 + i y3
 *            (y = 0: the ordinary second Jacobi iterate u + v)
 *   loss     mode 0: mean over rows of |t - t_converged|^2 / s^2 (relative)
 *            mode 1: sum |t - t_converged|^2 / sum s^2 (absolute)
 *   update   Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * All arrays are device memory; n = rows.  The network's calls run on its
 * stream; the fscc_ws_* calls on the stream given. */
typedef struct fscc_mlp fscc_mlp;

fscc_status fscc_mlp_num_params(size_t *n);
/* He-normal W1, W2 from a SplitMix64 + Box-Muller stream keyed by seed; zero
 * W3 and biases (the untrained network returns the second Jacobi iterate). */
fscc_status fscc_mlp_create(uint64_t seed, void *hip_stream, fscc_mlp **out);
void fscc_mlp_destroy(fscc_mlp *net);
const char *fscc_mlp_last_error(const fscc_mlp *net);
/* Host parameter vectors (count = fscc_mlp_num_params); set resets Adam. */
fscc_status fscc_mlp_set_params(fscc_mlp *net, const float *host, size_t count);
fscc_status fscc_mlp_get_params(fscc_mlp *net, float *host, size_t count);
/* Gradient of the last fscc_mlp_loss_grad call (host copy). */
fscc_status fscc_mlp_get_grad(fscc_mlp *net, float *host, size_t count);

/* X[n][8] from u, r, D. */
fscc_status fscc_ws_features(const fscc_c128 *u, const fscc_c128 *r, const double *D, size_t n, float *X,
                             void *hip_stream);
/* Y[n][4] = network(X[n][8]) (row chunks of 2^20; allocates its scratch on
 * first use). */
fscc_status fscc_mlp_forward(fscc_mlp *net, const float *X, size_t n, float *Y);
/* out = u + v + a v + b u from Y (Y may be NULL: out = u + v). */
fscc_status fscc_ws_apply(const float *Y, const fscc_c128 *u, const fscc_c128 *r, const double *D, size_t n,
                          fscc_c128 *out, void *hip_stream);
/* out = t + r / D (t may be NULL: out = r / D, e.g. the MP2 amplitudes from
 * the residual at t = 0). */
fscc_status fscc_ws_step(const fscc_c128 *t, const fscc_c128 *r, const double *D, size_t n, fscc_c128 *out,
                         void *hip_stream);
/* dst[k] = src[idx[k]] for elements of 8 or 16 bytes. */
fscc_status fscc_ws_gather(const void *src, size_t elem_bytes, const int64_t *idx, size_t n, void *dst,
                           void *hip_stream);
/* Loss and gradient (kept in the network) on rows idx[0..n) of the arrays
 * (idx NULL: rows 0..n-1), n <= 2^24.  Synchronous; *loss on the host. */
fscc_status fscc_mlp_loss_grad(fscc_mlp *net, const fscc_c128 *u, const fscc_c128 *r, const double *D,
                               const fscc_c128 *t, const int64_t *idx, size_t n, int mode, double *loss);
/* One Adam step with the current gradient (asynchronous). */
fscc_status fscc_mlp_adam(fscc_mlp *net, float lr);

#ifdef __cplusplus
}
#endif

#endif /* FSCC_H */
