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
constexpr int kPackAlpha = 12;  // pack A slot of alpha_i (written with the indicator)
constexpr int kPackCoef = 12;   // pack B slot of tau/(lambda_i m_i)
constexpr int kRowB = 8;      // doubles per node: U^L (nc), bounds (3)
constexpr int kRowU = 8;      // doubles per node: state after pass 1 (nc), the
                              // row's bounds (3)
constexpr int kPackL = 8;     // doubles per node: the low-order sweep's neighbour
                              // record U (nc), p, phi, alpha [kPackLAlpha]
constexpr int kPackLAlpha = 7;
// records of a row block's neighbourhood staged in LDS (3D at Morton order:
// about 600 with a 64-row SELL window, 700 with rows sorted over the whole
// mesh; 2D: about 350), at most 6 chunks each (75 KB, 48 KB)
constexpr int kHaloMax3 = 800;
constexpr int kHaloMax2 = 512;
template <int D> constexpr int kHaloMaxD = D == 3 ? kHaloMax3 : kHaloMax2;
// a smaller cap for the staged viscosity sweep (64-byte records): 632
// records in 3D keep its LDS under 40 KB, four blocks per CU instead of
// three (Morton blocks of 256 rows have 600 halo nodes in the bulk, 648 and
// more at faces of the Morton tree).  A context takes it when at most one
// block in 50 has a halo between the two caps: those blocks gather instead,
// several times slower (rows sorted by length over the whole mesh make
// most blocks' halos larger)
constexpr int kHaloPair3 = 632;

// status bits (device int)
constexpr int kErrState = 1;
constexpr int kErrDt = 2;
constexpr int kWarnCfl = 4;
constexpr int kErrWait = 8;     // a persistent launch gave up waiting on a dependency
constexpr int kErrMask = kErrState | kErrDt | kErrWait;

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
    double *dp, *l1p;           // [npairs] d_ij, min(l_ij, l_ji) pass 1; written
                                // only for stages that keep adjoint records
    // matrices (SELL order); written by the precompute only
    double *c0, *c1, *c2, *mij;
    double *ct0, *ct1, *ct2;    // c_ji at the position of c_ij
    double *mi, *lam;
    // [n] widening r_i = (m_i/|Omega|)^(1.5/d) of the bounds (remark of
    // Section 3.9), or null: the bounds of the paper, unrelaxed
    double *relax_r;
    const uint8_t *hold;
    // per-stage work
    double *d;                  // [sell] d_ij, diagonal d_ii
    double *l1, *l2;            // [sell] min(l_ij, l_ji) of pass 1, 2
    double *packA, *alpha, *packB, *rowB, *upass, *taui;
    double *packL;              // [n][kPackL]
    // [nslices] bits of the slice's minimum tau_i where the low-order sweep
    // sums d_ii (stages with tau held), folded into taumin by k_tau_fold
    unsigned long long *wmin;
    unsigned long long *wmin_blk;   // [nslices / kBlock] their block minima
    // [n] pass 2's limiter candidate of row i along a zero direction, from
    // its pass-1 state and bounds (written by pass 1): the candidate l_ij of
    // every pair that pass 1 left unlimited, min(l_ij, l_ji) = 1, whose
    // pass-2 direction (1 - 1) P_ij is zero
    double *l2self;
    // pass 2's work list, built by pass 1: per slice s the SELL positions of
    // the entries (i, j), j > i, whose s1 < 1, packed from slow_base[s]
    // ([nslices + 1]: the slice's entries with j > i before it) and counted
    // in slow_cnt[s].  Null: no list (every pair of pass 2 is swept).
    int32_t *slow, *slow_cnt;
    const int64_t *slow_base;
    // [sell / 64] bit l of word w: SELL entry 64 w + l has s1 < 1 (written
    // by pass 1 for slices up to 64 columns wide), or null: pass 2 visits
    // every entry
    unsigned long long *slowmask;
    // records for the stage adjoint (null: not kept): which orientation
    // set d_ij = max(...) (1: i -> j), which side of a pair set min(l_ij,
    // l_ji) (1: the row of pair_i) per limiter pass; and per node the row
    // positions k of the entries that set rho_min, rho_max and phi_min
    // (bits 0-7, 8-15, 16-23; 255: the node itself)
    uint8_t *sided, *side1, *side2;
    int32_t *argk;
    // neighbourhoods of the row blocks (4 slices) for LDS staging, or null:
    // [per * 8] start in halo_node and size (-1: too large, gathers instead);
    // [sell] position of entry e's column in its block's halo
    const int64_t *halo_start;
    const int32_t *halo_cnt, *halo_node;
    const uint16_t *loc;
    int dpair_cap;              // the staged viscosity sweep's cap in 3D:
                                // kHaloPair3 or kHaloMax3
    // [per * 8 + 1] the pairs of each row block (those of its rows), and
    // [npairs] the halo position of each pair's node i, or null (the
    // viscosity sweep then gathers both records)
    const int64_t *pair_blk;
    const uint16_t *pair_li;
    // [npairs * 2 dim] c_ij then c_ji of each pair, in pair order (the
    // viscosity sweep's coefficient stream)
    double *cpair;
    // instances: a batch of independent meshes shares one context; their
    // slices, pairs and nodes are contiguous and never mixed
    int ninst;
    const int32_t *inst_slice;  // [nslices] instance of each slice (null: one)
    unsigned long long *taumin; // [ninst] bits of min_i m_i/(-2 d_ii)
    double *tau, *bound;        // [ninst]
    // the paper's variant 3 (IDP_FLAG_SPLIT_P), or null: [nc][qstride] the
    // viscous part (d^H - d^L)(U_j - U_i) of P_ij per SELL entry, written by
    // the low-order sweep and read by the limiter sweeps and the passes
    double *q;
    int64_t qstride;
    const double *dt_inst;      // [ninst] per-instance dt of a batch call, or null
    int *status;
};

// One persistent launch over a batch: a queue of work items, each a few
// consecutive wavefront units (64 nodes, 64 pairs or 1 slice) of one sweep
// of one instance, in (stage, sweep, instance) order; an item starts once
// every item of the previous sweep of its instance has completed.
constexpr int kSweeps = 8;      // node, dpair, diag, low, lim1p, pass1a, lim2p, pass2
struct BatchArgs {
    int nsteps;
    int tile;                   // wavefront units per work item
    int check;                  // admissibility check of stage-1 inputs
    int64_t items_per_stage;
    int64_t total_items;
    int64_t sweep_off[kSweeps + 1];   // item offsets of the sweeps inside a stage
    const int32_t *item_inst;   // [items_per_stage] instance of each item
    const int32_t *item_tile;   // [items_per_stage] units of each item
    const int64_t *item_first;  // [items_per_stage] first node/pair/slice of each item
    const int64_t *pre;         // [ninst][kSweeps + 1] completions required before each
                                // sweep inside a stage; [kSweeps]: completions per stage
    const int64_t *unit_end;    // [ninst][3] end of the instance's nodes, pairs, slices
    unsigned long long *taumin2;  // [2][ninst] (stages alternate)
    unsigned int *done;         // [ninst] completed items (and tau updates)
    unsigned long long *head;   // next item
    double *U, *U1;             // state and the stage scratch, concatenated
    double *dt_rec;             // [nsteps][ninst] tau of every step
};

// decision traces of the last stage: [npairs] pair codes, [n] row codes
void launch_trace(const StageArgs &P, hipStream_t st, unsigned long long *pairs,
                  unsigned *rows);
// s2 at the pairs with s1 = 1, which the pass-2 limiter sweep leaves out
void launch_l2_fill(const StageArgs &P, hipStream_t st);
// pass 2's limiter: over the work list built by pass 1, or over every pair
// (stages that keep the adjoint's records, or no list)
void launch_lim2(const StageArgs &P, hipStream_t st);
// per-entry P_ij component / pass-1 / pass-2 candidates into out [sell]
void launch_debug_entries(const StageArgs &P, hipStream_t st, int what, int comp, double *out);
// r_i = (m_i / mass_total)^(1.5/d) into P.relax_r
void launch_relax(const StageArgs &P, hipStream_t st, double mass_total);
void launch_matrices(const StageArgs &P, hipStream_t st, const double *coords,
                     const int32_t *cells, const int64_t *nc_ptr,
                     const int32_t *nc_list, const double gx[3], int *err);
void launch_begin(const StageArgs &P, hipStream_t st, int clear_status);
void launch_batch_init(const StageArgs &P, const BatchArgs &B, hipStream_t st, int clear_status);
void launch_persistent(const StageArgs &P, const BatchArgs &B, hipStream_t st, int grid);
int persistent_blocks_per_cu(int dim);
// fold: first take in the block minima of launch_tau_fold(.., 0)
void launch_tau(const StageArgs &P, hipStream_t st, double dt_in, int mode, int fold);
// the per-slice minima of tau_i (wmin, left by the diagonal or low-order
// sweep) towards taumin: with reduce all the way, else to block minima
// that launch_tau with fold takes in
void launch_tau_fold(const StageArgs &P, hipStream_t st, int reduce);
void launch_node(const StageArgs &P, hipStream_t st, const double *U, int check);
// with_alpha: the row-block viscosity sweep also computes the indicator of
// its rows (the diagonal sweep then leaves it)
void launch_dpair(const StageArgs &P, hipStream_t st, int with_alpha);
// mode 0: d_ii and tau_i; 1: and the indicator; 2: d_ii and tau_i from d
// alone (the viscosity sweep computed the indicator)
void launch_diag(const StageArgs &P, hipStream_t st, int mode);
// with_diag: the low-order sweep also sums d_ii and tau_i (per-slice minima
// into wmin), for stages whose tau is held
void launch_low(const StageArgs &P, hipStream_t st, int with_diag);
void launch_lim1p(const StageArgs &P, hipStream_t st);
void launch_pass1a(const StageArgs &P, hipStream_t st);
void launch_lim2p(const StageArgs &P, hipStream_t st);
void launch_pass2(const StageArgs &P, hipStream_t st, const double *U0, double *out,
                  int mode);
void launch_math(hipStream_t st, int kind, int64_t n, const double *x, const double *y,
                 double *out);

}  // namespace idp
