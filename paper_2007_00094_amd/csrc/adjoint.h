// Internal interface of the stage adjoint (idp_adjoint.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace idp {

// Record strides (doubles) of the adjoint's work arrays.  Records read by
// cooperative gathers have even strides (16-byte chunks).
constexpr int kEbS = 8;    // node: stage-output cotangent (nc), padded
constexpr int kUpS = 8;    // node: pass-1 state's cotangent (nc), bounds' (3)
constexpr int kLimS = 8;   // pair: the active candidate's state (nc) and bounds (3)
                           // cotangents of one limiter pass (written only if nonzero)
constexpr int kZS = 8;     // entry: direction cotangent +-Z (nc) [0, 5), alpha's share [5],
                           // d^H - d^L [6], the pass-1 limiter record of the row [7]
constexpr int kC5S = 6;    // entry: state cotangent (nc) from the graph viscosity
constexpr int kQS = 6;     // pair: cotangent of the pass-2 direction (nc)
constexpr int kNS = 16;    // node: Lw's (nc) [0, 5), R's (nc) [5, 10), bounds' [10, 13)
                           // cotangents, alpha [13], the neighbours that set the
                           // bounds [14, 16)
constexpr int kIS = 8;     // node: the indicator's a and b (nc) cotangents [0, 6),
                           // eta/rho [6]

// Work arrays of one stage's vector-Jacobian product (device).  The
// per-entry buffer C holds the direction records (kZS), then the
// graph-viscosity records (kC5S); the pair buffer Lim the pass-2, then the
// pass-1 limiter records.  Each is dead before the next is written.  A
// limiter record exists only where the active candidate's cotangents are
// nonzero (a limited pair); an entry finds it through its index (-1: none).
struct AdjArgs {
    double tau;
    const double *Ebp;  // [n][kEbS] cotangent of the stage output E(U)
    double *Ub;         // [n][nc] result: cotangent of U
    double *Upb;        // [n][kUpS]
    double *Nrec;       // [n][kNS]
    double *Irec;       // [n][kIS]
    double *Up4, *Up6;  // [n][nc] parts of U's cotangent (low order; indicator and
                        // the neighbours' low order)
    double *alb;        // [n] alpha's cotangent from the directions and its own R
    double *C;          // [sell][kZS]
    int32_t *lim2e;     // [sell] pass-2 limiter record of the entry's row, or -1
    double *Lim;        // [npairs][kLimS]
    double *db4;        // [sell] d_ij's cotangent from row i's low-order update
    double *Qb;         // [npairs][kQS]
    double *dLb;        // [npairs] d_ij's cotangent: the directions', then the total
    // totals kept for inspection: U^L's, R's, bounds', alpha's cotangents
    double *ULt, *Rt, *bndt, *alt;
};

void launch_stage_vjp(const StageArgs &P, const AdjArgs &A, hipStream_t st);
// Eb [n][kEbS] of a user array [n][nc]
void launch_adj_pad(hipStream_t st, int64_t n, int nc, const double *in, double *out);
void launch_adj_ssp(hipStream_t st, int64_t n, int nc, const uint8_t *hold, const double *outb,
                    double theta, double *Eb, double *U0b, int first);
void launch_adj_add(hipStream_t st, int64_t n, const double *x, double *y);

}  // namespace idp
