// Internal declarations shared by the host driver and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/irk.h"

#define IRK_MAX_LEVELS 14
#define IRK_WG 256
#define IRK_RED_BLOCKS 512   // work-groups of the reduction kernels
#define IRK_MATVEC_DOT_BLOCKS 2048   // of the matvec fused with a projection (a stencil needs more waves)
#define IRK_LANE_PARTIALS (IRK_MATVEC_DOT_BLOCKS * 16)   // doubles of a lane's partial sums

namespace irk {

// Tableau and the real eigenbasis of A0^{-1} (host, float64 after a long
// double construction).
struct EigenBlocks {
    int s = 0, nblocks = 0;
    double A[IRK_MAX_STAGES * IRK_MAX_STAGES], Ainv[IRK_MAX_STAGES * IRK_MAX_STAGES];
    double b[IRK_MAX_STAGES], c[IRK_MAX_STAGES];
    double T[IRK_MAX_STAGES * IRK_MAX_STAGES], Tinv[IRK_MAX_STAGES * IRK_MAX_STAGES];
    double TLam[IRK_MAX_STAGES * IRK_MAX_STAGES];          // T Lambda
    int width[IRK_MAX_STAGES], first[IRK_MAX_STAGES];
    double eta[IRK_MAX_STAGES], beta[IRK_MAX_STAGES], gamma_star[IRK_MAX_STAGES];
    // off-diagonal entries of each 2x2 diagonal block [[eta, c12], [c21, eta]]
    // (eigenbasis: beta, -beta; real Schur basis: phi, -beta^2/phi)
    double c12[IRK_MAX_STAGES], c21[IRK_MAX_STAGES];
    // T^{-1} A0^{-1} T: Lambda (block diagonal) or, in the real Schur basis,
    // R0 (block upper triangular: its blocks above the diagonal couple blocks)
    double R[IRK_MAX_STAGES * IRK_MAX_STAGES];
    bool schur = false;
    int argmax_stage[IRK_MAX_STAGES];                     // per transformed row
};

bool build_tableau_ld(int family, int s, long double *A, long double *b, long double *c);
bool build_eigen_blocks(int family, int s, EigenBlocks *eb);
// the real Schur basis of A0^{-1}, built from the real eigenbasis
bool build_schur_blocks(int family, int s, EigenBlocks *eb);
void build_sdirk_stage_block(double gamma, double ci, EigenBlocks *eb);

// Small constant blocks passed to kernels by value.
struct StageCoefs {
    double A[IRK_MAX_STAGES * IRK_MAX_STAGES];
    double TLam[IRK_MAX_STAGES * IRK_MAX_STAGES];
    double Tinv[IRK_MAX_STAGES * IRK_MAX_STAGES];
    double b[IRK_MAX_STAGES];
    double tstage[IRK_MAX_STAGES];      // t_n + c_i dt
    double sin_t[IRK_MAX_STAGES], cos_t[IRK_MAX_STAGES];
};

// Entries of an eigen-block's diagonal block of Lambda (or R0):
// [[eta, c12], [c21, eta]] (1x1 blocks: eta).
struct BlockLam {
    double eta, c12, c21;
};

// Stage weights of an eigen-block's operator under Newton-like (2), (3):
// row a of the block applies sum_b sum_k w[a][b][k] L(U_k) to component b.
struct BlockWeights {
    double w[2][2][IRK_MAX_STAGES];
};

// A block of R0 above the diagonal in the real Schur basis, coupling block i
// (rows) to block j (columns): R0_ij M - dt sum_k w[a][b][k] L(U_k) (the
// Jacobian terms only under Newton-like (3)).
struct BlockCouple {
    int wi, wj;
    double R[2][2];
    BlockWeights W;
    int jac;
};

// Geometry and physical parameters of one grid level.
struct Grid {
    int nx, ny;
    double h;       // spacing on this level
    double nu;
};

// One multigrid level's work arrays (precision of the V-cycle).
struct Level {
    int nx, ny;
    double h;
    void *x, *x2, *d, *b;
};

// Operator-specific kernel launchers (defined in kernels.hip).
struct DeviceProblem {
    int kind;               // irk_op_kind
    int forcing;
    int nvar;               // 1, or 2 for (omega, psi)
    Grid g;
    const double *sinx, *cosx, *siny, *cosy;   // forcing tables (NLDIFF)
};

}  // namespace irk
