// Internal interface of the stage adjoint (idp_adjoint.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace idp {

// Work arrays of one stage's vector-Jacobian product (device).
// Per node: [n][nc] unless noted; per stencil entry (SELL order): [sell][nc]
// unless noted.  Written by one kernel each, read by later ones.
struct AdjArgs {
    double tau;
    const double *Eb;   // cotangent of the stage output E(U)
    double *Ub;         // result: cotangent of U
    double *Upb;        // pass-1 state's (= U^L's) cotangent
    double *bndb;       // [n][3] bounds' cotangent from pass 2
    double *Ub3, *Ub2;  // own parts of U's cotangent (low order, indicator)
    double *alb;        // [n] alpha's own cotangent (low order)
    double *sb1, *sb2;  // [sell] s1, s2 cotangents, one row's share
    double *Pb;         // P_ij's cotangent
    double *cnode;      // [sell][nc + 3] limiter contributions to the row's
                        // state (U^L or pass-1) and bounds
    double *cR, *cU;    // R's and U's cotangent contributions to the row's node
    double *cal;        // [sell] alpha's contribution to the row's node
    double *dbp;        // [npairs] d_ij's cotangent from the directions
    double *cUj, *cUj2; // contributions to the column node j (low order, indicator)
    double *calj, *db3; // [sell] alpha_j's and d_ij's contributions (low order)
    // totals kept for inspection: U^L's, R's, bounds', alpha's cotangents
    // (d_ij's total is left in dbp)
    double *ULt, *Rt, *bndt, *alt;
};

void launch_stage_vjp(const StageArgs &P, const AdjArgs &A, hipStream_t st);
void launch_adj_ssp(hipStream_t st, int64_t n, int nc, const uint8_t *hold, const double *outb,
                    double theta, double *Eb, double *U0b, int first);
void launch_adj_add(hipStream_t st, int64_t n, const double *x, double *y);

}  // namespace idp
