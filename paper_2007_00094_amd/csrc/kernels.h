// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "idp_device.h"

namespace idp {

constexpr int kBlock = 256;   // threads per block: 4 wavefronts = 4 slices
constexpr int kSlice = 64;    // SELL slice height = wavefront width
constexpr int kXcd = 8;       // XCDs of an MI355X; blocks are renumbered so
                              // that each XCD walks a contiguous slice range
constexpr int kPack = 16;     // doubles per node in the gather packs
constexpr int kPackAlpha = 12;  // pack A slot of alpha_i (written by k_diag)
constexpr int kPackCoef = 12;   // pack B slot of tau/(lambda_i m_i)
constexpr int kRowB = 8;      // doubles per node: U^L (nc), bounds (3)
constexpr int kRowU = 8;      // doubles per node: state after pass 1

// status bits (device int)
constexpr int kErrState = 1;
constexpr int kErrDt = 2;
constexpr int kWarnCfl = 4;
constexpr int kErrMask = kErrState | kErrDt;

// Everything a kernel needs, passed by value.
struct StageArgs {
    int dim;
    int64_t n;
    int64_t nslices;
    int per;                    // logical blocks per XCD
    double gamma, cfl, tol;
    GasC gas;                   // gamma-only constants of the wave-speed bound
    int newton_max, passes;
    // SELL-64 graph
    const int32_t *perm, *row_len, *diag_k;
    const int64_t *slice_off;
    const int32_t *scol, *stpos;
    // unordered pairs {i < j}: SELL positions of (i,j), (j,i); nodes
    int64_t npairs;
    int pper;                   // pair blocks per XCD
    const int32_t *pair_e, *pair_t, *pair_i, *pair_j;
    double *mp;                 // [npairs] m_ij in pair order
    double *dp, *l1p;           // [npairs] d_ij, min(l_ij, l_ji) pass 1
    // matrices (SELL order); written by the precompute only
    double *c0, *c1, *c2, *mij;
    double *ct0, *ct1, *ct2;    // c_ji at the position of c_ij
    double *mi, *lam;
    const uint8_t *hold;
    // per-stage work
    double *d;                  // [sell] d_ij, diagonal d_ii
    double *l1, *l2;            // [sell] min(l_ij, l_ji) of pass 1, 2
    double *packA, *alpha, *packB, *rowB, *upass, *taui;
    unsigned long long *taumin; // bits of min_i m_i/(-2 d_ii)
    double *tau, *bound;
    int *status;
};

void launch_matrices(const StageArgs &P, hipStream_t st, const double *coords,
                     const int32_t *cells, const int64_t *nc_ptr,
                     const int32_t *nc_list, const double gx[3], int *err);
void launch_begin(const StageArgs &P, hipStream_t st, int clear_status);
void launch_tau(const StageArgs &P, hipStream_t st, double dt_in, int mode);
void launch_node(const StageArgs &P, hipStream_t st, const double *U, int check);
void launch_dpair(const StageArgs &P, hipStream_t st);
void launch_diag(const StageArgs &P, hipStream_t st, int with_alpha);
void launch_low(const StageArgs &P, hipStream_t st);
void launch_lim1p(const StageArgs &P, hipStream_t st);
void launch_pass1a(const StageArgs &P, hipStream_t st);
void launch_lim2p(const StageArgs &P, hipStream_t st);
void launch_pass2(const StageArgs &P, hipStream_t st, const double *U0, double *out,
                  int mode);
void launch_math(hipStream_t st, int kind, int64_t n, const double *x, const double *y,
                 double *out);

}  // namespace idp
