// plan.hpp -- the residual as a list of elementary operations.
//
// Every Goldstone-diagram contraction is evaluated by the TTGT scheme of the
// algorithm-design section: reorder the operands into supermatrix layouts
// (gather ops), one grouped complex GEMM over the symmetry blocks (one
// problem per pair irrep, the block loop of Fig. 4), then reorder and
// antisymmetrise the result into the residual (gather-accumulate ops).
// The plan is pure host data: buffers, gather maps and GEMM problem lists.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "gtile.hpp"
#include "layout.hpp"

namespace fscc {

using cplx = std::complex<double>;

enum BufKind { BUF_IN_T1, BUF_IN_T2, BUF_OUT_R1, BUF_OUT_R2, BUF_CONST, BUF_SCRATCH, BUF_REAL,
               BUF_IN_S1, BUF_IN_S2, BUF_OUT_RS1, BUF_OUT_RS2, BUF_IN_P2, BUF_OUT_RP2 };

inline bool caller_buffer(BufKind k) {
    return k == BUF_IN_T1 || k == BUF_IN_T2 || k == BUF_OUT_R1 || k == BUF_OUT_R2 || k == BUF_IN_S1 ||
           k == BUF_IN_S2 || k == BUF_OUT_RS1 || k == BUF_OUT_RS2 || k == BUF_IN_P2 || k == BUF_OUT_RP2;
}

struct BufDesc {
    std::string name;
    int64_t n;        // complex elements (doubles for BUF_REAL)
    BufKind kind;
};

struct GemmProblem {
    int64_t a_off, b_off, c_off;
    int M, N, K;
    int lda, ldb, ldc;
    int sys = 0;   // system of a batched plan (tiles of inactive systems are skipped)
};

enum OpKind {
    OP_GATHER,   // dst[k] = beta*dst[k] + alpha * sum_t s_t * cj(src[mA_t[k]]) * (src2 ? src2[mB_t[k]] : 1)
    OP_GEMM,     // grouped: C = alpha*op(A)op(B) + beta*C
    OP_AXPBY,    // dst[k] = alpha*cj(src[k]) + beta*dst[k]
    OP_DIAG,     // dst[k] -= d[k] * src[k]   (d real)
    OP_MUL,      // dst[k] *= d[k]            (d real)
};

struct Op {
    OpKind kind;
    std::string name;
    int dst = -1, src = -1, src2 = -1;
    std::vector<int> mapsA, mapsB;   // gather maps (map ids)
    std::vector<int> srcT;           // gathers summing reorders of several buffers: term t's source
    cplx alpha = 1.0;
    int beta = 0;
    bool conj = false;
    int64_t n = 0;
    std::vector<GTile> gtiles;       // gathers: 16 x 16 tiles covering the destination blocks
    const GTile* d_gtiles = nullptr; // device copy (set up with the context)
    bool use_gtiles = false;         // traverse the destination by tiles (chosen by timing)
    // affine traversal: destination tiles (at most 16 x 16, inside one of the
    // 16 x 16 tiles above) on which each term's source index is affine in
    // (row, column) -- rterms[tile * nterms + t] -- so no map is read there
    std::vector<GTile> rtiles;
    std::vector<RTerm> rterms;
    std::vector<RUnit> runits;       // consecutive affine tiles grouped into work units
    const GTile* d_rtiles = nullptr;
    const RTerm* d_rterms = nullptr;
    const RUnit* d_runits = nullptr;
    bool use_rtiles = false;         // chosen by timing
    // GEMM
    bool tA = false, tB = false, cA = false, cB = false;
    std::vector<GemmProblem> probs;
    double flops = 0;                // real flops (8 per complex MAC)
    double bytes = 0;                // algorithmic bytes per call (set when the context is built)
};

// integral classes
enum IClass { IC_OOOO = 0, IC_OOOV, IC_OOVV, IC_OVOV, IC_OVVV, IC_VVVV, IC_N };

// a derived constant built at set_integrals time from one class
struct SetupGather {
    int cls;
    int dst;          // buffer id
    int map;          // map id (from the class's FullBlocks buffer)
    bool conj;
    std::string name;
};

struct System {
    int nocc = 0, nvirt = 0, G = 1;
    std::vector<int> irrep;     // global order
    std::vector<double> eps;    // global order
    std::vector<int> active;    // global indices of active virtuals (0h1p)
};

struct Plan {
    int G = 1;
    Space O, V;
    std::vector<BufDesc> bufs;
    std::vector<std::vector<uint32_t>> maps;
    std::vector<std::string> map_names;
    std::vector<Op> ops;
    std::vector<SetupGather> setup;
    FullBlocks full[IC_N];
    // stored layouts of the caller's amplitudes
    Layout L_T1, L_T2;
    int b_t1 = -1, b_t2 = -1, b_r1 = -1, b_r2 = -1;
    int b_D1 = -1, b_D2 = -1;         // real denominators in T1/T2 layouts
    int b_oovv = -1;                  // <ij||ab> in the T2 layout (energy)
    int b_tau = -1;                   // tau in the T2 layout (energy scratch)
    std::vector<double> D1, D2;       // host copies (uploaded once)

    // ---- (0h,1p) sector (present when the system has active virtuals)
    bool has01 = false;
    Space X;                          // active virtuals, irrep-sorted
    std::vector<int> x_vpos;          // X position -> V position
    std::vector<int> x_order;         // X position -> index in the caller's active list
    Layout L_S1, L_S2, L_Heff;
    int b_s1 = -1, b_s2 = -1, b_rs1 = -1, b_rs2 = -1;
    int b_D1x = -1, b_D2x = -1, b_mask1 = -1, b_heff = -1;
    std::vector<double> D1x, D2x, mask1;
    int b_Fvv01 = -1, b_Foo01 = -1;   // Fbar_vv, Fbar_oo ([g][n_g][n_g] blocks)
    std::vector<int64_t> fvv_diag, foo_diag;   // offset of the diagonal element per V / O position
    // (0h,0p) dressed preconditioner: F'_be / F'_mj of the last residual and
    // the offsets of their diagonal elements; orbital energies by position
    int b_Fbe = -1, b_Fmj = -1;
    std::vector<int64_t> fbe_diag, fmj_diag;
    std::vector<double> eps_o, eps_v;
    std::vector<Op> ops01_prep;       // Hbar elements from the converged (0h,0p) amplitudes
    std::vector<Op> ops01;            // sigma + Bloch residual

    // ---- (0h,2p) sector (present when there are at least two active virtuals)
    bool has02 = false;
    Layout L_S02, L_Heff02;           // s_xy^ab: [G][xy<][ab<];  H_eff: [G][zw<][xy<]
    int b_s02 = -1, b_rs02 = -1, b_D02 = -1, b_mask02 = -1, b_heff02 = -1;
    std::vector<double> D02, mask02;
    std::vector<Op> ops02_prep;       // fixed part of sigma2 from the converged (0h,1p) amplitudes
    std::vector<Op> ops02;            // S_xy terms + Bloch residual
    struct HostConst {
        int buf;
        std::vector<cplx> data;
    };
    std::vector<HostConst> const_host;   // small complex constants uploaded at create

    int buf(const std::string& name, int64_t n, BufKind k) {
        bufs.push_back({name, n, k});
        return (int)bufs.size() - 1;
    }
    int map(const std::string& name, std::vector<uint32_t>&& m) {
        maps.push_back(std::move(m));
        map_names.push_back(name);
        return (int)maps.size() - 1;
    }
    double total_flops() const {
        double f = 0;
        for (auto& o : ops) f += o.flops;
        return f;
    }
};

void build_plan_ccsd(const System& S, Plan& P);

}  // namespace fscc
