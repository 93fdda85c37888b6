// HIP kernels of the IDP Q1 Euler scheme (arXiv:2007.00094) for gfx950.
//
// One forward-Euler stage of Alg. 1 is a node kernel, four row sweeps over
// the SELL-64 stencil layout and three sweeps over the unordered pairs:
//   k_node    step 0   per node: p, c, eta/rho, v = m/rho, phi   (pack A)
//   k_dpair   step 1   per pair: d_ij = d_ji (both orientations, the larger;
//                       one where c_ji = -c_ij makes them mirror images)
//   k_dpair_h step 1   the same by row block, and the indicator alpha_i of
//                       the block's rows
//   k_diag    step 2   per row: d_ii, tau_i, min tau; indicator alpha_i (k_dsum:
//                       d_ii and tau_i alone, after k_dpair_h)
//   k_low     step 3   per row: R_i, U^L_i, bounds rho_min, rho_max, phi_min
//   k_lim1p   step 4   per pair: P_ij, P_ji (eq. def-p), l_ij, l_ji (Alg. 2),
//                       s_ij = s_ji = min(l_ij, l_ji)
//   k_pass1a  step 5   per row: U_i = U^L_i + sum lambda_i s_ij P_ij
//   k_lim2p   step 5   per pair: candidates of pass 2 on (1 - s_ij) P_ij
//   k_pass2   step 6   per row: final pass, SSP-RK3 combination, hold
// Each sweep is a device function over a range of nodes, pairs or slices:
// the kernels above launch one sweep over a whole context, and
// k_persistent runs every sweep of many steps of a batch of independent
// meshes in one launch, from a queue of work items with per-instance
// dependency counts (no grid-wide barrier).
// A row sweep gives one wavefront lane one stencil row (a SELL slice holds
// 64 rows) and sums its columns in ascending order, sequentially, like the
// CPU oracle, so every row reduction has one writer and a fixed order.  A
// pair sweep evaluates each symmetric quantity once, with the operation
// order its two rows would use, and stores it at (i,j) and (j,i): no row
// ever reads a transposed entry.  Neighbour data are gathered from
// node-major packs (128 bytes per node), mostly by whole wavefronts at once
// (one cache line per record and load instruction, exchanged through LDS).
// Blocks are renumbered so that consecutive slices or pairs run on the same
// XCD (L2 locality of the gathers).  No MFMA: the sweeps are sparse, FP64
// and bound by the L1 address path of their gathers and by FP64 issue.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "idp_device.h"
#include "kernels.h"
#include "sweep_common.h"

namespace idp {

// ------------------------------------------------------------ matrices
// Eq. matrices by 3-point Gauss quadrature per direction on each cell;
// the row of node i accumulates the cell contributions in ascending cell
// order.  For each cell the local row of i is integrated point by point.
template <int D>
__global__ void __launch_bounds__(kBlock)
k_matrices(StageArgs P, const double *__restrict__ coords,
           const int32_t *__restrict__ cells, const int64_t *__restrict__ nc_ptr,
           const int32_t *__restrict__ nc_list, double gx0, double gx1, double gx2,
           int *__restrict__ err)
{
    ROW_SETUP(P)
    constexpr int NV = 1 << D;
    constexpr int NQ = D == 2 ? 9 : 27;
    const double gx[3] = {gx0, gx1, gx2};
    const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        P.mij[e] = 0.0;
        P.c0[e] = 0.0;
        P.c1[e] = 0.0;
        if (D == 3) P.c2[e] = 0.0;
    }
    for (int64_t q = nc_ptr[i]; q < nc_ptr[i + 1]; ++q) {
        const int32_t T = nc_list[q];
        int vx[NV];
        int a = 0;
        for (int b = 0; b < NV; ++b) {
            vx[b] = cells[int64_t(T) * NV + b];
            if (vx[b] == i) a = b;
        }
        double xb[NV][D];
        for (int b = 0; b < NV; ++b)
            for (int p = 0; p < D; ++p) xb[b][p] = coords[int64_t(vx[b]) * D + p];
        double mloc[NV], cloc[NV][D];
        for (int b = 0; b < NV; ++b) {
            mloc[b] = 0.0;
            for (int p = 0; p < D; ++p) cloc[b][p] = 0.0;
        }
        for (int qp = 0; qp < NQ; ++qp) {
            double xi[D];
            double w = 1.0;
            int qq = qp;
            for (int k = 0; k < D; ++k) {
                xi[k] = gx[qq % 3];
                w *= gw[qq % 3];
                qq /= 3;
            }
            double J[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
            double gr[NV][D], ph[NV];
            for (int b = 0; b < NV; ++b) {
                for (int k = 0; k < D; ++k) {
                    double v = ((b >> k) & 1) ? 1.0 : -1.0;
                    for (int l = 0; l < D; ++l)
                        if (l != k) v *= ((b >> l) & 1) ? xi[l] : 1.0 - xi[l];
                    gr[b][k] = v;
                }
                double v = 1.0;
                for (int k = 0; k < D; ++k) v *= ((b >> k) & 1) ? xi[k] : 1.0 - xi[k];
                ph[b] = v;
                for (int p = 0; p < D; ++p)
                    for (int k = 0; k < D; ++k) J[p][k] += xb[b][p] * gr[b][k];
            }
            double det, Ji[3][3];
            if (D == 2) {
                det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
                Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
            } else {
                det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
            }
            if (!(det > 0.0)) atomicOr(err, 1);
            const double wd = w * det;
            for (int b = 0; b < NV; ++b) {
                double gp[D];
                for (int p = 0; p < D; ++p) {
                    double s = 0.0;
                    for (int k = 0; k < D; ++k) s += Ji[k][p] * gr[b][k];
                    gp[p] = s;
                }
                mloc[b] += wd * (ph[a] * ph[b]);
                for (int p = 0; p < D; ++p) cloc[b][p] += wd * ph[a] * gp[p];
            }
        }
        for (int b = 0; b < NV; ++b) {
            int kk = 0;
            for (int k = 0; k < L; ++k)
                if (P.scol[ENTRY(k)] == vx[b]) kk = k;
            const int64_t e = ENTRY(kk);
            P.mij[e] += mloc[b];
            P.c0[e] += cloc[b][0];
            P.c1[e] += cloc[b][1];
            if (D == 3) P.c2[e] += cloc[b][D - 1];
        }
    }
}

// m_i = sum_j m_ij (ascending columns), lambda_i = 1/(card I(i) - 1)
__global__ void __launch_bounds__(kBlock) k_lumped(StageArgs P)
{
    ROW_SETUP(P)
    double s = 0.0;
    for (int k = 0; k < L; ++k) s += P.mij[ENTRY(k)];
    P.mi[i] = s;
    P.lam[i] = 1.0 / double(L - 1);
}

// c_ji stored at the position of c_ij (coalesced reads of the transpose)
template <int D>
__global__ void __launch_bounds__(kBlock) k_transpose_c(StageArgs P)
{
    ROW_SETUP(P)
    for (int k = 0; k < L; ++k) {
        const int64_t e = ENTRY(k);
        const int64_t t = P.stpos[e];
        P.ct0[e] = P.c0[t];
        P.ct1[e] = P.c1[t];
        if (D == 3) P.ct2[e] = P.c2[t];
    }
}

// m_ij in pair order (the pair sweeps read it without the position lookup)
__global__ void __launch_bounds__(kBlock) k_pair_mass(StageArgs P)
{
    const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= P.npairs) return;
    P.mp[p] = P.mij[P.pair_e[p]];
}

// c_ij and c_ji in pair order
template <int D>
__global__ void __launch_bounds__(kBlock) k_pair_c(StageArgs P)
{
    const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= P.npairs) return;
    const int64_t e = P.pair_e[p];
    double *o = P.cpair + p * (2 * D);
    o[0] = P.c0[e];
    o[1] = P.c1[e];
    if (D == 3) o[2] = P.c2[e];
    o[D] = P.ct0[e];
    o[D + 1] = P.ct1[e];
    if (D == 3) o[D + 2] = P.ct2[e];
}

// ------------------------------------------------------------ helpers
// Minimum over the wavefront's lanes of the bit patterns of non-negative
// doubles (their order as values; +inf for lanes without a row).
__device__ __forceinline__ unsigned long long wave_min_bits(unsigned long long t)
{
#pragma unroll
    for (int o = kSlice / 2; o > 0; o /= 2) {
        const unsigned long long u = __shfl_xor(t, o);
        t = u < t ? u : t;
    }
    return t;
}

// The low-order sweep's per-slice minima of tau_i towards each instance's
// minimum: a batch's slices by atomics into their instance's; a single
// mesh's by block into wmin_blk, which k_tau reduces (same-address atomics
// from many blocks at once queue for microseconds).
__global__ void __launch_bounds__(kBlock) k_tau_fold(StageArgs P)
{
    __shared__ unsigned long long red[kBlock / kSlice];
    const int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (P.ninst > 1) {
        if (s < P.nslices) atomicMin(P.taumin + P.inst_slice[s], P.wmin[s]);
        return;
    }
    const unsigned long long t = wave_min_bits(s < P.nslices ? P.wmin[s] : 0x7FF0000000000000ull);
    if (threadIdx.x % kSlice == 0) red[threadIdx.x / kSlice] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int w = 1; w < kBlock / kSlice; ++w) m = red[w] < m ? red[w] : m;
        P.wmin_blk[blockIdx.x] = m;
    }
}

__global__ void k_begin(StageArgs P, int clear_status)
{
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0 && clear_status) *P.status = 0;
    for (int k = threadIdx.x; k < P.ninst; k += blockDim.x)
        P.taumin[k] = 0x7FF0000000000000ull;  // +inf
}

// Per instance k.  mode 1 (stage 1 of a step): tau = dt if given (error if
// dt exceeds the bound) else cfl * bound; mode 2: tau = dt, warn if it
// exceeds the bound; mode 0 (stages 2, 3): warn if the held tau exceeds
// this stage's bound.
__device__ __forceinline__ void select_tau(const StageArgs &P, int k, double bound,
                                           double dt_in, int mode)
{
    P.bound[k] = bound;
    if (mode == 1) {
        if (dt_in > 0.0 && dt_in > bound) atomicOr(P.status, kErrDt);
        P.tau[k] = dt_in > 0.0 ? dt_in : P.cfl * bound;
    } else if (mode == 2) {
        P.tau[k] = dt_in;
        if (dt_in > bound) atomicOr(P.status, kWarnCfl);
    } else {
        if (P.tau[k] > bound) atomicOr(P.status, kWarnCfl);
    }
}

// k_tau_fold's block minima into the mesh's minimum (one block of kBlock
// threads; a single mesh only: a batch's slices went in by atomics).
__device__ __forceinline__ void tau_reduce(const StageArgs &P)
{
    __shared__ unsigned long long red[kBlock];
    if (P.ninst != 1) return;
    const int64_t nb = (P.nslices + kBlock - 1) / kBlock;
    unsigned long long m = 0x7FF0000000000000ull;
    for (int64_t q = threadIdx.x; q < nb; q += kBlock) {
        const unsigned long long v = P.wmin_blk[q];
        m = v < m ? v : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o && red[threadIdx.x + o] < red[threadIdx.x])
            red[threadIdx.x] = red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] < P.taumin[0]) P.taumin[0] = red[0];
    __syncthreads();
}

__global__ void __launch_bounds__(kBlock) k_tau_reduce(StageArgs P) { tau_reduce(P); }

// fold: take in k_tau_fold's block minima first
__global__ void __launch_bounds__(kBlock) k_tau(StageArgs P, double dt_in, int mode, int fold)
{
    if (blockIdx.x != 0) return;
    if (fold) tau_reduce(P);
    for (int k = threadIdx.x; k < P.ninst; k += blockDim.x) {
        const double bound = __longlong_as_double((long long)P.taumin[k]);
        select_tau(P, k, bound, P.dt_inst ? P.dt_inst[k] : dt_in, mode);
    }
}

// ----------------------------------------------------------- node pass
// Step 0: p, c, eta/rho, v = m/rho, phi of nodes i in [i0, i0 + 256) below
// iend; with check, flags inadmissible input.
template <int D>
__device__ __forceinline__ void node_sweep(const StageArgs &P, int64_t i, int64_t iend,
                                           const double *__restrict__ U, int check, double2 *lw)
{
    // whole wavefronts past the end leave; the rest store their records
    // with one cooperative scatter (lanes past the end store nothing)
    if (i - int64_t(threadIdx.x % kSlice) >= iend) return;
    if (failed(P)) return;
    constexpr int NC = D + 2, NCH = kPackAChunks<D>;
    const bool valid = i < iend;
    const int64_t ii = valid ? i : 0;
    double u[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) u[k] = U[ii * NC + k];
    const double g = P.gamma;
    const double eps = internal_energy<D>(u);
    double A[2 * NCH];
#pragma unroll
    for (int k = 0; k < NC; ++k) A[k] = u[k];
    A[NC + 0] = pressure<D>(u, g);
    A[NC + 1] = speed_of_sound<D>(u, g);
    A[NC + 2] = harten_entropy<D>(u, g) / u[0];
#pragma unroll
    for (int k = 0; k < D; ++k) A[NC + 3 + k] = u[1 + k] / u[0];
    A[NC + 3 + D] = specific_entropy<D>(u, g);
#pragma unroll
    for (int k = NC + 4 + D; k < 2 * NCH; ++k) A[k] = 0.0;
    // the forward sweeps read pack A's first kDiagChunks chunks; v and phi
    // only the stage adjoint, which runs on stages recomputed with records
    if (P.argk)
        scatter<NCH>(P.packA, kPack, valid ? int(i) : -1, lw, A);
    else
        scatter<kDiagChunks<D>>(P.packA, kPack, valid ? int(i) : -1, lw, A);
    // the low-order sweep's record: U, p, phi (alpha follows with the indicator)
    double L[kPackL];
#pragma unroll
    for (int k = 0; k < NC; ++k) L[k] = u[k];
    L[NC] = A[NC];
    L[NC + 1] = A[NC + 3 + D];
#pragma unroll
    for (int k = NC + 2; k < kPackL; ++k) L[k] = 0.0;
    scatter<kPackL / 2>(P.packL, kPackL, valid ? int(i) : -1, lw, L);
    if (check && valid) {
        bool ok = u[0] > 0.0 && eps > 0.0;
#pragma unroll
        for (int k = 0; k < NC; ++k) ok = ok && isfinite(u[k]);
        if (!ok) atomicOr(P.status, kErrState);
    }
}

// ------------------------------------------------------- pair viscosity
// Step 1, once per unordered pair {i, j}: d_ij = d_ji = max of
// lambda~(n_ij, U_i, U_j)|c_ij| and lambda~(n_ji, U_j, U_i)|c_ji|, from
// c_ij, c_ji (stored at the position of c_ij) and the two nodes' pack A
// records (U, p, c); p_ is the pair's index, e and t its two entries.
template <int D, bool TR = false>
__device__ __forceinline__ double pair_viscosity(const double *c, const double *ct,
                                                 const double *Ai, const double *Aj,
                                                 const GasC &G, bool &first,
                                                 unsigned *code = nullptr)
{
    constexpr int NC = D + 2;
    double aij = 0.0, aji = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        aij += c[q] * c[q];
        aji += ct[q] * ct[q];
    }
    aij = sqrt(aij);
    aji = sqrt(aji);
    // c_ij + c_ji integrates phi_i phi_j n over the boundary: it vanishes
    // (up to rounding) unless both nodes are boundary nodes, and then the
    // reversed problem (n_ji, U_j, U_i) mirrors (n_ij, U_i, U_j) and has
    // the same bound; the pair's orientation (lower caller id first) is
    // the one evaluated
    bool mirror;
    {
        double s = 0.0, m = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            s += fabs(c[q] + ct[q]);
            m += fabs(c[q]) + fabs(ct[q]);
        }
        mirror = s <= 0x1p-36 * m;
    }
    double t1 = 0.0, t2 = 0.0;
    unsigned cs = 0, c1 = 0, c2 = 0;
    // the psi_branch terms of the two states serve both orientations
    const double S = (aij > 0.0 || aji > 0.0)
        ? psi_sum<D, TR>(Ai[0], Ai[NC], Ai[NC + 1], Aj[0], Aj[NC], Aj[NC + 1], G, &cs)
        : 0.0;
    if (aij > 0.0) {
        const double inv = 1.0 / aij;
        double nn[D];
#pragma unroll
        for (int q = 0; q < D; ++q) nn[q] = c[q] * inv;
        t1 = lambda_max_s<D, TR>(nn, Ai, Ai[NC], Ai[NC + 1], Aj, Aj[NC], Aj[NC + 1], S, G, &c1) *
             aij;
    }
    if (!mirror && aji > 0.0) {
        const double inv = 1.0 / aji;
        double nn[D];
#pragma unroll
        for (int q = 0; q < D; ++q) nn[q] = ct[q] * inv;
        t2 = lambda_max_s<D, TR>(nn, Aj, Aj[NC], Aj[NC + 1], Ai, Ai[NC], Ai[NC + 1], S, G, &c2) *
             aji;
    }
    first = mirror || t1 > t2;
    // trace: bit 0 the state with p_max, bits 1-6 the (i, j) bound, bits
    // 7-12 the (j, i) bound, bit 13 which of the two set d_ij
    if constexpr (TR) *code = cs | (c1 << 1) | (c2 << 7) | (t1 > t2 ? 1u << 13 : 0u);
    return t1 > t2 ? t1 : t2;
}

template <int D>
__device__ __forceinline__ void dpair_eval(const StageArgs &P, int64_t p_, int64_t e,
                                           int64_t t, const double *c, const double *ct,
                                           const double *Ai, const double *Aj)
{
    bool first;
    const double dd = pair_viscosity<D>(c, ct, Ai, Aj, P.gas, first);
    P.d[e] = dd;
    P.d[t] = dd;
    if (P.sided) P.dp[p_] = dd;   // pair order: read by the stage adjoint only
    if (P.sided) P.sided[p_] = first;
}

// c_ij and c_ji of pair p (16-byte loads from the pair-order copy)
template <int D>
__device__ __forceinline__ void load_cp(const StageArgs &P, int64_t p, double *c, double *ct)
{
    const double2 *q = reinterpret_cast<const double2 *>(P.cpair + p * (2 * D));
    double v[2 * D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double2 w = q[k];
        v[2 * k] = w.x;
        v[2 * k + 1] = w.y;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        c[k] = v[k];
        ct[k] = v[D + k];
    }
}

// the sweep over pairs pidx (one per lane) below pend, both records gathered
template <int D>
__device__ __forceinline__ void dpair_sweep(const StageArgs &P, int64_t pidx, int64_t pend,
                                            double2 *lw)
{
    WAVE_PAIR_SETUP(P, pidx, pend)
    if (failed(P)) return;
    constexpr int NCH = (D + 5) / 2;   // U, p, c
    double c[D], ct[D];
    load_cp<D>(P, pq_, c, ct);
    double Ai[2 * NCH], Aj[2 * NCH];
    {
        // both records' loads in flight before either passes through LDS
        dchunk vi[GatherShape<NCH>::LPR], vj[GatherShape<NCH>::LPR];
        gather_issue<NCH>(P.packA, kPack, i, vi);
        gather_issue<NCH>(P.packA, kPack, j, vj);
        gather_exchange<NCH>(lw, vi, Ai);
        gather_exchange<NCH>(lw, vj, Aj);
    }
    if (!valid_) return;
    dpair_eval<D>(P, p_, e, t, c, ct, Ai, Aj);
}

// Section 3.8: alpha_i = N_i/D_i from the row sums a_i and b_i, with
// N_i = |a_i - eta'_i . b_i + (eta_i/rho_i)(b_i)_1| and
// D_i = |a_i| + sum_k |eta'_{i,k} - delta_1k eta_i/rho_i| |(b_i)_k|
// (0 if D_i = 0).  TR: *code receives the sign of each term under |.|
// (bit 0 that of N_i's argument, bit 1 a_i, bits 2.. (b_i)_k, bits
// 2 + nc.. the eta' terms) and bit 2 + 2 nc for D_i > 0.
template <int D, bool TR = false>
__device__ __forceinline__ double indicator(const double *U, double er, double a,
                                            const double *b, double g,
                                            unsigned *code = nullptr)
{
    constexpr int NC = D + 2;
    double etap[NC];
    harten_entropy_derivative<D>(U, g, etap);
    double etab = 0.0;
#pragma unroll
    for (int r = 0; r < NC; ++r) etab += etap[r] * b[r];
    const double x = a - etab + er * b[0];
    const double N = fabs(x);
    double Dn = fabs(a);
    unsigned bits = (x > 0.0 ? 1u : 0u) | (a > 0.0 ? 2u : 0u);
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        const double y = etap[r] - (r == 0 ? er : 0.0);
        Dn += fabs(y) * fabs(b[r]);
        bits |= (b[r] > 0.0 ? 1u << (2 + r) : 0u) | (y > 0.0 ? 1u << (2 + NC + r) : 0u);
    }
    if constexpr (TR) *code = bits | (Dn > 0.0 ? 1u << (2 + 2 * NC) : 0u);
    return Dn > 0.0 ? N / Dn : 0.0;
}

// --------------------------------------------------------- row diagonal
// d_ii = -sum_{j != i} d_ij in ascending column order (the diagonal at its
// known position) and tau_i, the slice's minimum into wmin: the diagonal
// sweep without the indicator, reading d alone.
__device__ __forceinline__ void diag_only(const StageArgs &P, int64_t sidx, int64_t send)
{
    WAVE_ROW_SETUP(P, sidx, send)
    (void)inst_;
    if (failed(P)) return;
    const int dk = valid_ ? P.diag_k[r_] : -1;
    // nine entries' loads in flight at a time (a Q1 row has 9 or 27), summed
    // in column order as they arrive
    constexpr int kU = 9;
    double dsum = 0.0;
    for (int k0 = 0; k0 < Lmax_; k0 += kU) {
        double dd[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            dd[u] = k0 + u < L ? ld_stream(P.d + ENTRY(k0 + u)) : 0.0;
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (k0 + u < L && k0 + u != dk) dsum += dd[u];
    }
    const double dii = -dsum;
    const double ti = valid_ ? P.mi[i] / (-2.0 * dii) : 0.0;
    const unsigned long long m = wave_min_bits(
        valid_ ? (unsigned long long)__double_as_longlong(ti) : 0x7FF0000000000000ull);
    if (lane_ == 0) P.wmin[s_] = m;
    if (!valid_) return;
    P.d[ENTRY(dk)] = dii;
    P.taui[i] = ti;
}

// Step 2: d_ii = -sum_{j != i} d_ij (columns ascending), tau_i, the
// instance's min tau_i (into taumin[instance], or with taumin null the
// slice's minimum into wmin); indicator alpha_i (Section 3.8) over all j in
// I(i).
template <int D, class F>
__device__ __forceinline__ void diag_sweep(const StageArgs &P, int64_t sidx, int64_t send,
                                           int with_alpha, unsigned long long *taumin,
                                           const F &fetch)
{
    WAVE_ROW_SETUP(P, sidx, send)
    if (failed(P)) return;
    constexpr int NC = D + 2;
    constexpr int NCH = kDiagChunks<D>;
    const double g = P.gamma;
    NodeA<D> Ai;
    load_a_fwd<D>(P.packA + int64_t(i) * kPack, Ai);
    double Fi[NC][D];
    flux<D>(Ai.U, Ai.v, Ai.p, Fi);
    double dsum = 0.0, a = 0.0;
    double b[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) b[r] = 0.0;
    int jn = Lmax_ > 0 ? ld_stream(P.scol + ENTRY(0)) : 0;
    for (int k = 0; k < Lmax_; ++k) {
        const int64_t e = ENTRY(k);
        const int j = jn;
        if (k + 1 < Lmax_) jn = ld_stream(P.scol + ENTRY(k + 1));
        const bool in = k < L;
        const double dd = ld_stream(P.d + e);
        if (in && j != i) dsum += dd;
        if (with_alpha) {
            double c[D];
            load_c_stream<D>(P, e, c);
            double rec[2 * NCH];
            fetch(fetch.token(e), in ? j : -1, rec);
            if (!in) continue;
            // U, p, c, eta/rho; v = m/rho exactly as the node pass has it
            NodeA<D> Aj;
#pragma unroll
            for (int r = 0; r < NC; ++r) Aj.U[r] = rec[r];
            Aj.p = rec[NC];
            Aj.er = rec[NC + 2];
#pragma unroll
            for (int q = 0; q < D; ++q) Aj.v[q] = Aj.U[1 + q] / Aj.U[0];
            double mc = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) mc += Aj.U[1 + q] * c[q];
            a += (Aj.er - Ai.er) * mc;
            double Fj[NC][D], fd[NC];
            flux<D>(Aj.U, Aj.v, Aj.p, Fj);
            flux_diff_dot<D>(Fi, Fj, c, fd);
#pragma unroll
            for (int r = 0; r < NC; ++r) b[r] += fd[r];
        }
    }
    const double dii = -dsum;
    const double ti = valid_ ? P.mi[i] / (-2.0 * dii) : 0.0;
    if (!taumin) {
        // the slice's minimum into wmin (k_tau_fold takes it in)
        const unsigned long long m = wave_min_bits(
            valid_ ? (unsigned long long)__double_as_longlong(ti) : 0x7FF0000000000000ull);
        if (lane_ == 0) P.wmin[s_] = m;
    }
    if (!valid_) return;
    P.d[ENTRY(P.diag_k[r_])] = dii;
    P.taui[i] = ti;
    if (taumin) atomicMin(taumin + inst_, (unsigned long long)__double_as_longlong(ti));
    if (with_alpha) {
        const double al = indicator<D>(Ai.U, Ai.er, a, b, g);
        P.alpha[i] = al;
        P.packL[int64_t(i) * kPackL + kPackLAlpha] = al;
        // pack A's copy is read only by the stage adjoint, which runs on
        // stages recomputed with their records kept
        if (P.argk) P.packA[int64_t(i) * kPack + kPackAlpha] = al;
    }
}

// ------------------------------------------------------ row low order
// Step 3.  The neighbours' records (pack L, 64 bytes) come from the row
// block's LDS staging, else from per-lane loads (3D: its per-entry
// arithmetic hides them better than a cooperative gather) or a cooperative
// gather (2D).
template <int D, bool SP = false, class F>
__device__ __forceinline__ void low_sweep(const StageArgs &P, int64_t sidx, int64_t send,
                                          const F &fetch, int with_diag = 0)
{
    WAVE_ROW_SETUP(P, sidx, send)
    if (failed(P)) return;
    constexpr int NC = D + 2;
    // the row's own record: U, p and phi from pack L, v recomputed
    NodeA<D> Ai;
    {
        const double *a = P.packL + int64_t(i) * kPackL;
#pragma unroll
        for (int r = 0; r < NC; ++r) Ai.U[r] = a[r];
        Ai.p = a[NC];
        Ai.phi = a[NC + 1];
#pragma unroll
        for (int k = 0; k < D; ++k) Ai.v[k] = Ai.U[1 + k] / Ai.U[0];
    }
    const double alpha_i = P.alpha[i];
    const double tau = P.tau[inst_];
    double Fi[NC][D];
    flux<D>(Ai.U, Ai.v, Ai.p, Fi);
    double R[NC], Lw[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) { R[r] = 0.0; Lw[r] = 0.0; }
    double rho_min = Ai.U[0], rho_max = Ai.U[0], phi_min = Ai.phi;
    double dsum = 0.0;   // with_diag: -d_ii, summed as the diagonal sweep sums it
    int kmn = 255, kmx = 255, kph = 255;
    int jn = Lmax_ > 0 ? ld_stream(P.scol + ENTRY(0)) : 0;
    for (int k = 0; k < Lmax_; ++k) {
        const int64_t e = ENTRY(k);
        const int j = jn;
        if (k + 1 < Lmax_) jn = ld_stream(P.scol + ENTRY(k + 1));
        const bool act = k < L && j != i;
        double c[D];
        load_c_stream<D>(P, e, c);
        const double dL = ld_stream(P.d + e);
        if (act) dsum += dL;
        // the neighbour's record U, p, phi, alpha (pack L); v = m/rho is
        // recomputed exactly as the node pass computes it
        double rec[kPackL];
        fetch(fetch.token(e), act ? j : -1, rec);
        if (!act) continue;
        NodeA<D> Aj;
#pragma unroll
        for (int r = 0; r < NC; ++r) Aj.U[r] = rec[r];
        Aj.p = rec[NC];
        Aj.phi = rec[NC + 1];
#pragma unroll
        for (int k = 0; k < D; ++k) Aj.v[k] = Aj.U[1 + k] / Aj.U[0];
        const double alpha_j = rec[kPackLAlpha];
        const double dH = dL * (alpha_i + alpha_j) / 2.0;
        double Fj[NC][D], fd[NC];
        flux<D>(Aj.U, Aj.v, Aj.p, Fj);
        flux_diff_dot<D>(Fi, Fj, c, fd);
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            R[r] += -fd[r] + dH * (Aj.U[r] - Ai.U[r]);
            Lw[r] += -fd[r] + dL * (Aj.U[r] - Ai.U[r]);
        }
        if constexpr (SP) {
            // variant 3: the direction's viscous part for steps 4 to 6
#pragma unroll
            for (int r = 0; r < NC; ++r)
                P.q[int64_t(r) * P.qstride + e] = (dH - dL) * (Aj.U[r] - Ai.U[r]);
        }
        double rbar = 0.5 * (Ai.U[0] + Aj.U[0]);
        if (dL > 0.0) rbar -= fd[0] / (2.0 * dL);
        if (rbar < rho_min) { rho_min = rbar; kmn = k; }
        if (rbar > rho_max) { rho_max = rbar; kmx = k; }
        if (Aj.phi < phi_min) { phi_min = Aj.phi; kph = k; }
    }
    if (with_diag) {
        // tau held (stages 2 and 3): d_ii and tau_i for the CFL check, the
        // slice's minimum into wmin
        const double dii = -dsum;
        const double ti = P.mi[i] / (-2.0 * dii);
        const unsigned long long m = wave_min_bits(
            valid_ ? (unsigned long long)__double_as_longlong(ti) : 0x7FF0000000000000ull);
        if (lane_ == 0) P.wmin[s_] = m;
        if (valid_) {
            P.d[ENTRY(P.diag_k[r_])] = dii;
            P.taui[i] = ti;
        }
    }
    if (!valid_) return;
    if (P.argk) P.argk[i] = kmn | (kmx << 8) | (kph << 16);
    const double mi = P.mi[i];
    double *B = P.packB + int64_t(i) * kPack;
    double *W = P.rowB + int64_t(i) * kRowB;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        B[r] = Ai.U[r];
        B[NC + r] = R[r];
        W[r] = Ai.U[r] + tau / mi * Lw[r];
    }
    B[2 * NC] = alpha_i;
    B[2 * NC + 1] = mi;
    // the records are written whole (unused slots zero): a partly written
    // line costs the memory a read-modify-write
#pragma unroll
    for (int r = 2 * NC + 2; r < kPackCoef; ++r) B[r] = 0.0;
    B[kPackCoef] = tau / (P.lam[i] * mi);   // tau/(lambda_i m_i) of eq. def-p
#pragma unroll
    for (int r = kPackCoef + 1; r < kPack; ++r) B[r] = 0.0;
    if (P.relax_r) {
        // widened bounds (remark of Section 3.9), r_i fixed by the mesh
        const double rr = P.relax_r[i];
        rho_min *= (1.0 - rr);
        rho_max *= (1.0 + rr);
        phi_min *= (1.0 - rr);
    }
    W[NC + 0] = rho_min;
    W[NC + 1] = rho_max;
    W[NC + 2] = phi_min;
#pragma unroll
    for (int r = NC + 3; r < kRowB; ++r) W[r] = 0.0;
}

// ------------------------------------------------------ pair limiter 1
// Step 4, once per unordered pair: l_ij from (U^L_i, P_ij, bounds_i) and
// l_ji from (U^L_j, P_ji, bounds_j), each evaluated exactly as its own row
// would; s_ij = s_ji = min(l_ij, l_ji) stored at (i,j) and (j,i).
template <int D, bool SP = false>
__device__ __forceinline__ void lim1_sweep(const StageArgs &P, int64_t pidx, int64_t pend,
                                           double2 *lw)
{
    WAVE_PAIR_SETUP(P, pidx, pend)
    if (failed(P)) return;
    constexpr int NC = D + 2;
    using CH = Chunks<D>;
    const double dL = P.d[e], m = P.mp[pq_];   // d_ij at (i, j): the viscosity sweep's value
    // both directions first, so that the node packs are dead before the
    // rows' bounds are gathered.  2D: each phase has the loads of both rows
    // in flight before either passes through LDS; 3D (more registers per
    // record): one row at a time, which keeps four waves per SIMD
    double Pij[NC], Pji[NC];
    {
        NodeB<D> Bi, Bj;
        if constexpr (D == 2) {
            gather_b2<D>(P.packB, i, j, lw, Bi, Bj);
        } else {
            gather_b<D>(P.packB, i, lw, Bi);
            gather_b<D>(P.packB, j, lw, Bj);
        }
        if constexpr (SP) {
            double Q[NC], nQ[NC];
#pragma unroll
            for (int r = 0; r < NC; ++r) {
                Q[r] = P.q[int64_t(r) * P.qstride + e];
                nQ[r] = -Q[r];
            }
            direction_q<D>(Bi, Bj, Bi.coef, m, Q, Pij);
            direction_q<D>(Bj, Bi, Bj.coef, m, nQ, Pji);
        } else {
            direction<D>(Bi, Bj, Bi.coef, dL, m, Pij);
            direction<D>(Bj, Bi, Bj.coef, dL, m, Pji);
        }
    }
    constexpr int NW = CH::rowB;
    double lij, lji;
    if constexpr (D == 2) {
        dchunk vi[GatherShape<NW>::LPR], vj[GatherShape<NW>::LPR];
        gather_issue<NW>(P.rowB, kRowB, i, vi);
        gather_issue<NW>(P.rowB, kRowB, j, vj);
        double Wi[2 * NW], Wj[2 * NW];
        gather_exchange<NW>(lw, vi, Wi);
        gather_exchange<NW>(lw, vj, Wj);
        if (!valid_) return;
        lij = row_limiter<D>(Wi, Wi, Pij, P);
        lji = row_limiter<D>(Wj, Wj, Pji, P);
    } else {
        double W[2 * NW];
        gather<NW>(P.rowB, kRowB, i, lw, W);
        lij = valid_ ? row_limiter<D>(W, W, Pij, P) : 0.0;
        gather<NW>(P.rowB, kRowB, j, lw, W);
        if (!valid_) return;
        lji = row_limiter<D>(W, W, Pji, P);
    }
    const double sv = lij < lji ? lij : lji;
    P.l1[e] = sv;
    P.l1[t] = sv;

    if (P.side1) P.l1p[p_] = sv;   // pair order: read by the stage adjoint only
    if (P.side1) P.side1[p_] = lij < lji;
}

// -------------------------------------------------------- row pass 1
// Step 5, first half: U_i = U^L_i + sum_{j != i} lambda_i s_ij P_ij.
template <int D, bool SP = false, class F>
__device__ __forceinline__ void pass1_sweep(const StageArgs &P, int64_t sidx, int64_t send,
                                            const F &fetch)
{
    WAVE_ROW_SETUP(P, sidx, send)
    if (failed(P)) return;
    constexpr int NC = D + 2;
    using CH = Chunks<D>;
    NodeB<D> Bi;
    load_b<D>(P.packB + int64_t(i) * kPack, Bi);
    const double *W = P.rowB + int64_t(i) * kRowB;
    double V[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) V[r] = W[r];
    const double tau = P.tau[inst_];
    const double lam = P.lam[i];
    const double coef = tau / (lam * Bi.m);
    // pass 2's work list: the entries (i, j), j > i, with s1 < 1, packed at
    // the slice's base (not for stages that keep the adjoint's records,
    // whose pass-2 limiter sweeps all pairs)
    const bool list = P.slow && P.passes >= 2 && !P.side2;
    const int64_t sbase = list ? P.slow_base[s_] : 0;
    int nslow = 0;
    // and the slice's mask words of the entries with s1 < 1 (word k: the
    // 64 rows' entries k), which pass 2 visits
    unsigned long long *const mw =
        P.slowmask && P.passes >= 2 && Lmax_ <= kSlice ? P.slowmask + (P.slice_off[s_] >> 6)
                                                       : nullptr;
    unsigned long long mword = 0ull;
    // the next entry's column, scalars and fetch token are loaded one
    // entry ahead
    int jn = 0, tn = 0;
    double ln = 0.0, dn = 0.0, mn = 0.0;
    if (Lmax_ > 0) {
        const int64_t e0 = ENTRY(0);
        jn = P.scol[e0];
        tn = fetch.token(e0);
        ln = P.l1[e0];
        dn = P.d[e0];
        mn = P.mij[e0];
    }
    for (int k = 0; k < Lmax_; ++k) {
        const int j = jn, tk = tn;
        const double l = ln, dL = dn, m = mn;
        if (k + 1 < Lmax_) {
            const int64_t e1 = ENTRY(k + 1);
            jn = P.scol[e1];
            tn = fetch.token(e1);
            ln = P.l1[e1];
            dn = P.d[e1];
            mn = P.mij[e1];
        }
        const bool act = k < L && j != i;
        if (mw) {
            // column k's word, kept by lane k and stored after the loop
            const unsigned long long bm = __ballot(act && !(l == 1.0));
            mword = lane_ == k ? bm : mword;
        }
        if (list) {
            const bool slow = act && j > i && !(l == 1.0);
            const unsigned long long bal = __ballot(slow);
            if (slow) {
                const unsigned below = __builtin_amdgcn_mbcnt_hi(
                    unsigned(bal >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(bal), 0u));
                P.slow[sbase + nslow + below] = int32_t(ENTRY(k));
            }
            nslow += __popcll(bal);
        }
        double rec[2 * CH::packBrow];
        fetch(tk, act ? j : -1, rec);
        if (!act) continue;
        NodeB<D> Bj;
        unpack_b<D, false>(rec, Bj);
        double Pd[NC];
        if constexpr (SP) {
            double Q[NC];
#pragma unroll
            for (int r = 0; r < NC; ++r) Q[r] = P.q[int64_t(r) * P.qstride + ENTRY(k)];
            direction_q<D>(Bi, Bj, coef, m, Q, Pd);
        } else {
            direction<D>(Bi, Bj, coef, dL, m, Pd);
        }
#pragma unroll
        for (int r = 0; r < NC; ++r) V[r] += lam * l * Pd[r];
    }
    if (list && lane_ == 0) P.slow_cnt[s_] = nslow;
    if (mw && lane_ < Lmax_) mw[lane_] = mword;
    if (!valid_) return;
    P.l1[ENTRY(P.diag_k[r_])] = 1.0;   // the diagonal's s1 (pass 2 reads it as 1)
    // whole 64-byte records (a partly written line costs the memory a
    // read-modify-write): the state, and the row's bounds beside it so that
    // the pass-2 limiter gathers one record per row
    double *Up = P.upass + int64_t(i) * kRowU;
#pragma unroll
    for (int r = 0; r < NC; ++r) Up[r] = V[r];
#pragma unroll
    for (int q = 0; q < 3; ++q) Up[NC + q] = W[NC + q];
#pragma unroll
    for (int r = NC + 3; r < kRowU; ++r) Up[r] = 0.0;
    if (P.passes >= 2) {
        // pass 2's candidate of this row along a zero direction: the one
        // every pair with s_ij = 1 gets, since its (1 - s_ij) P_ij is zero
        // (the limiter's outcome is the same for +0 and -0 components)
        double Z[NC];
#pragma unroll
        for (int r = 0; r < NC; ++r) Z[r] = 0.0;
        P.l2self[i] = limiter<D>(V, Z, W[NC], W[NC + 1], W[NC + 2], P.gamma, P.newton_max,
                                 P.tol);
    }
}

// ------------------------------------------------------ pair limiter 2
// Step 5, second half, once per unordered pair: candidates of pass 2 on the
// rescaled directions (1 - s_ij) P_ij from the pass-1 states.  A pair that
// pass 1 left unlimited (s_ij = 1) has the pass-2 direction (1 - 1) P_ij =
// 0, along which the candidate of each side depends on that side's row only
// (pass 1 stores it: l2self); its pass-2 term is a zero whatever s2 is, and
// pass 2 does not read s2 there.  So only the pairs with s_ij < 1 need the
// limiter: pass 1 lists them (slow), and k_lim2s runs over that list.  The
// full sweep over all pairs (k_lim2p) runs for stages that keep the
// adjoint's records and in the persistent batch schedule; a wavefront of it
// whose pairs all have s_ij = 1 stores min of the two l2self (bit for bit
// what the limiter returns along a zero direction) where records are kept
// and skips them otherwise.  A debug export of s2 fills the skipped pairs in.

// The limiter of one pair (i, j) at SELL positions e = (i,j), t = (j,i)
// with m = m_ij; p: the pair's index for the records (< 0: none).  Every
// lane of the wavefront calls it (cooperative gathers); valid_: whether
// the lane has a pair.
template <int D, bool SP = false>
__device__ __forceinline__ void lim2_pair(const StageArgs &P, bool valid_, int64_t p_,
                                          int64_t e, int64_t t, int i, int j, double m,
                                          double l, double2 *lw)
{
    constexpr int NC = D + 2;
    using CH = Chunks<D>;
    const double dL = P.d[e];   // d_ij at (i, j): the viscosity sweep's value
    double Pij[NC], Pji[NC];
    {
        NodeB<D> Bi, Bj;
        if constexpr (D == 2) {
            gather_b2<D>(P.packB, i, j, lw, Bi, Bj);
        } else {
            gather_b<D>(P.packB, i, lw, Bi);
            gather_b<D>(P.packB, j, lw, Bj);
        }
        if constexpr (SP) {
            double Q[NC], nQ[NC];
#pragma unroll
            for (int r = 0; r < NC; ++r) {
                Q[r] = P.q[int64_t(r) * P.qstride + e];
                nQ[r] = -Q[r];
            }
            direction_q<D>(Bi, Bj, Bi.coef, m, Q, Pij);
            direction_q<D>(Bj, Bi, Bj.coef, m, nQ, Pji);
        } else {
            direction<D>(Bi, Bj, Bi.coef, dL, m, Pij);
            direction<D>(Bj, Bi, Bj.coef, dL, m, Pji);
        }
    }
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        Pij[r] = (1.0 - l) * Pij[r];
        Pji[r] = (1.0 - l) * Pji[r];
    }
    // per side: the pass-1 state with the row's bounds (one record); in 2D
    // the loads of both sides are in flight before the first passes
    // through LDS
    constexpr int NU = CH::upassb;
    double lij, lji;
    if constexpr (D == 2) {
        dchunk ui[GatherShape<NU>::LPR], uj[GatherShape<NU>::LPR];
        gather_issue<NU>(P.upass, kRowU, i, ui);
        gather_issue<NU>(P.upass, kRowU, j, uj);
        double Ui[2 * NU], Uj[2 * NU];
        gather_exchange<NU>(lw, ui, Ui);
        gather_exchange<NU>(lw, uj, Uj);
        if (!valid_) return;
        lij = limiter<D>(Ui, Pij, Ui[NC], Ui[NC + 1], Ui[NC + 2], P.gamma, P.newton_max, P.tol);
        lji = limiter<D>(Uj, Pji, Uj[NC], Uj[NC + 1], Uj[NC + 2], P.gamma, P.newton_max, P.tol);
    } else {
        double U[2 * NU];
        gather<NU>(P.upass, kRowU, i, lw, U);
        lij = valid_ ? limiter<D>(U, Pij, U[NC], U[NC + 1], U[NC + 2], P.gamma, P.newton_max,
                                  P.tol)
                     : 0.0;
        gather<NU>(P.upass, kRowU, j, lw, U);
        if (!valid_) return;
        lji = limiter<D>(U, Pji, U[NC], U[NC + 1], U[NC + 2], P.gamma, P.newton_max, P.tol);
    }
    const double sv = lij < lji ? lij : lji;
    P.l2[e] = sv;
    P.l2[t] = sv;
    if (P.side2 && p_ >= 0) P.side2[p_] = lij < lji;
}

template <int D, bool SP = false>
__device__ __forceinline__ void lim2_sweep(const StageArgs &P, int64_t pidx, int64_t pend,
                                           double2 *lw)
{
    const int64_t p_ = pidx;
    if (p_ - threadIdx.x % kSlice >= pend) return;
    if (failed(P)) return;
    const bool valid_ = p_ < pend;
    const int64_t pq_ = valid_ ? p_ : 0;
    const int64_t e = P.pair_e[pq_];
    const double l = P.l1[e];
    if (__all(!valid_ || l == 1.0)) {
        if (!valid_ || !P.side2) return;
        const int64_t t = P.pair_t[pq_];
        const int i = P.pair_i[pq_], j = P.pair_j[pq_];
        const double lij = P.l2self[i], lji = P.l2self[j];
        const double sv = lij < lji ? lij : lji;
        P.l2[e] = sv;
        P.l2[t] = sv;
        P.side2[p_] = lij < lji;
        return;
    }
    lim2_pair<D, SP>(P, valid_, p_, e, P.pair_t[pq_], P.pair_i[pq_], P.pair_j[pq_], P.mp[pq_],
                     l, lw);
}

// -------------------------------------------------------- row pass 2

// Step 6: U_i += sum_{j != i} lambda_i s2_ij (1 - s1_ij) P_ij, then
// mode 0: out = E(U); 1: out = E (stage 1); 2: out = U0 + 1/4 (E - U0);
// 3: out = U0 + 2/3 (E - U0); modes 1-3 keep held nodes at U0.
template <int D, bool SP = false, class F>
__device__ __forceinline__ void pass2_sweep(const StageArgs &P, int64_t sidx, int64_t send,
                                            const double *U0, double *out, int mode,
                                            const F &fetch)
{
    WAVE_ROW_SETUP(P, sidx, send)
    if (failed(P)) return;
    constexpr int NC = D + 2;
    using CH = Chunks<D>;
    NodeB<D> Bi;   // loaded once an entry of the wavefront needs it
    double V[NC];
    const double *Up = P.upass + int64_t(i) * kRowU;
#pragma unroll
    for (int r = 0; r < NC; ++r) V[r] = Up[r];
    if (P.passes >= 2) {
        const double tau = P.tau[inst_];
        const double lam = P.lam[i];
        double coef = 0.0;
        bool have_b = false;
        // An entry with s1 = 1 or s2 = 0 adds lambda s2 (1 - s1) P_ij = +-0,
        // which leaves V as it is unless a component of V is zero (whose sign
        // the term could change).  The entries with s1 < 1 are marked in the
        // slice's mask words (word k: the 64 rows' entries k), so only they,
        // and any entry of a row whose V has a zero component, are visited;
        // without the mask every entry is.
        // (pass 1 writes the words of slices up to 64 columns wide; wider
        // ones visit every entry)
        const unsigned long long *mw = P.slowmask && Lmax_ <= kSlice
                                           ? P.slowmask + (P.slice_off[s_] >> 6)
                                           : nullptr;
        // the slice's mask words held by the lanes (lane q: word q) and the
        // set of columns with a marked entry, so that unmarked columns cost
        // no memory access (loading the next marked column's scalars ahead
        // measured slower: 140 registers, three waves per SIMD)
        const bool held = mw != nullptr;
        unsigned long long wq = 0ull;
        if (held && lane_ < Lmax_) wq = mw[lane_];
        const unsigned long long kset = held ? __ballot(wq != 0ull) : ~0ull;
        for (int k = 0; k < Lmax_; ++k) {
            bool vzero = false;
#pragma unroll
            for (int r = 0; r < NC; ++r) vzero = vzero || V[r] == 0.0;
            if (held && !((kset >> k) & 1ull) && !__any(k < L && vzero)) continue;
            const bool marked = held ? ((__shfl(wq, k) >> lane_) & 1ull) != 0 : true;
            const bool need = k < L && (marked || vzero);
            if (!__any(need)) continue;
            if (!have_b) {
                load_b<D>(P.packB + int64_t(i) * kPack, Bi);
                coef = tau / (lam * Bi.m);
                have_b = true;
            }
            int j = i, tk = 0;
            double s1 = 1.0, s2 = 1.0, dL = 0.0, m = 0.0;
            if (need) {
                const int64_t ek = ENTRY(k);
                j = P.scol[ek];
                tk = fetch.token(ek);
                s1 = P.l1[ek];
                s2 = P.l2[ek];
                dL = P.d[ek];
                m = P.mij[ek];
            }
            const bool act = need && j != i;
            double rec[2 * CH::packBrow];
            fetch(tk, act ? j : -1, rec);
            if (!act) continue;
            NodeB<D> Bj;
            unpack_b<D, false>(rec, Bj);
            double Pd[NC];
            if constexpr (SP) {
                double Q[NC];
#pragma unroll
                for (int r = 0; r < NC; ++r) Q[r] = P.q[int64_t(r) * P.qstride + ENTRY(k)];
                direction_q<D>(Bi, Bj, coef, m, Q, Pd);
            } else {
                direction<D>(Bi, Bj, coef, dL, m, Pd);
            }
            // s1 = 1: the term is a zero with the sign of P_ij, s2 being +0
            // or 1 there (its stored value may be skipped: see lim2_pair)
            const double s2e = s1 == 1.0 ? 1.0 : s2;
#pragma unroll
            for (int r = 0; r < NC; ++r) {
                const double P2 = (1.0 - s1) * Pd[r];
                V[r] += lam * s2e * P2;
            }
        }
    }
    if (!valid_) return;
    if (P.passes >= 2) P.l2[ENTRY(P.diag_k[r_])] = 1.0;   // the diagonal's s2
    double *o = out + int64_t(i) * NC;
    if (mode == 0) {
#pragma unroll
        for (int r = 0; r < NC; ++r) o[r] = V[r];
        return;
    }
    const double *u0 = U0 + int64_t(i) * NC;
    double w[NC];
    if (P.hold && P.hold[i]) {
#pragma unroll
        for (int r = 0; r < NC; ++r) w[r] = u0[r];
    } else if (mode == 1) {
#pragma unroll
        for (int r = 0; r < NC; ++r) w[r] = V[r];
    } else if (mode == 2) {
#pragma unroll
        for (int r = 0; r < NC; ++r) w[r] = u0[r] + 0.25 * (V[r] - u0[r]);
    } else {
#pragma unroll
        for (int r = 0; r < NC; ++r) w[r] = u0[r] + (2.0 / 3.0) * (V[r] - u0[r]);
    }
#pragma unroll
    for (int r = 0; r < NC; ++r) o[r] = w[r];
}

// ------------------------------------------------- one launch per sweep
template <int D>
__global__ void __launch_bounds__(kBlock) k_node(StageArgs P, const double *__restrict__ U,
                                                 int check)
{
    WAVE_LDS(kPackAChunks<D>)
    node_sweep<D>(P, int64_t(blockIdx.x) * kBlock + threadIdx.x, P.n, U, check, lw);
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_dpair(StageArgs P)
{
    WAVE_LDS((D + 5) / 2)
    dpair_sweep<D>(P, PAIR_INDEX(P), P.npairs, lw);
}

// Staged viscosity sweep: one block per row block takes the pairs of its
// rows, whose two nodes are both in the block's halo; with the halo's
// records in LDS every node record is read from memory once per block
// instead of once per pair (a node has 2 x 13 pairs in 3D).  A block whose
// halo did not fit gathers as above.  Then the block computes the indicator
// of its rows.

// ------------------------------------------- indicator in the staged block
// Step 1's indicator (Section 3.8) for the rows of a row block: after the
// block's pairs, one lane per row sums the row's entries in ascending
// column order, exactly as the diagonal sweep does, from the neighbours'
// records (U, p, eta/rho: pack A's first 64 bytes) staged in LDS (STAGED)
// or read from pack A (blocks whose halo did not fit).
template <int D, bool STAGED>
__device__ __forceinline__ void alpha_rows(const StageArgs &P, int64_t b, const double2 *halo)
{
    constexpr int NC = D + 2;
    const int64_t s = b * (kBlock / kSlice) + threadIdx.x / kSlice;
    if (s >= P.nslices) return;
    const int lane = int(threadIdx.x % kSlice);
    const int64_t r = s * kSlice + lane;
    const int i = P.perm[r];
    if (i < 0) return;
    const int L = P.row_len[r];
    const int64_t off = P.slice_off[s] + lane;
    const double g = P.gamma;
    NodeA<D> Ai;
    load_a_fwd<D>(P.packA + int64_t(i) * kPack, Ai);
    double Fi[NC][D];
    flux<D>(Ai.U, Ai.v, Ai.p, Fi);
    double a = 0.0, bs[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) bs[q] = 0.0;
    for (int k = 0; k < L; ++k) {
        const int64_t e = off + int64_t(k) * kSlice;
        double c[D];
        load_c_stream<D>(P, e, c);
        double a8[8];
        if constexpr (STAGED) {
            const double2 *rec = halo + 4 * int(P.loc[e]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 v = rec[q];
                a8[2 * q] = v.x;
                a8[2 * q + 1] = v.y;
            }
        } else {
            const double *rec = P.packA + int64_t(P.scol[e]) * kPack;
#pragma unroll
            for (int q = 0; q < 8; ++q) a8[q] = rec[q];
        }
        NodeA<D> Aj;
#pragma unroll
        for (int q = 0; q < NC; ++q) Aj.U[q] = a8[q];
        Aj.p = a8[NC];
        Aj.er = a8[NC + 2];
#pragma unroll
        for (int q = 0; q < D; ++q) Aj.v[q] = Aj.U[1 + q] / Aj.U[0];
        double mc = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) mc += Aj.U[1 + q] * c[q];
        a += (Aj.er - Ai.er) * mc;
        double Fj[NC][D], fd[NC];
        flux<D>(Aj.U, Aj.v, Aj.p, Fj);
        flux_diff_dot<D>(Fi, Fj, c, fd);
#pragma unroll
        for (int q = 0; q < NC; ++q) bs[q] += fd[q];
    }
    const double al = indicator<D>(Ai.U, Ai.er, a, bs, g);
    P.alpha[i] = al;
    P.packL[int64_t(i) * kPackL + kPackLAlpha] = al;
    // pack A's copy is read only by the stage adjoint, which runs on stages
    // recomputed with their records kept
    if (P.argk) P.packA[int64_t(i) * kPack + kPackAlpha] = al;
}

template <int D, int CAP>
__global__ void __launch_bounds__(kBlock) k_dpair_h(StageArgs P, int with_alpha)
{
    constexpr int NCH = (D + 5) / 2;   // gathered chunks per record
    // staged record: pack A's first 64 bytes (U, p, c, eta/rho), which the
    // pairs and then the indicator read (3D: 40 KB per block and four
    // blocks per CU at the smaller cap, 51 KB and three at the larger)
    constexpr int NS = 4;
    static_assert(CAP * NS >= (kBlock / kSlice) * NCH * kLdsRow, "gather tiles fit");
    __shared__ double2 sh_[CAP * NS];
    const int64_t b = logical_block(P.per);
    const int64_t p0 = P.pair_blk[b], p1 = P.pair_blk[b + 1];
    const bool staged = stage_halo<NS, NS - 1, kPack, CAP>(P, b, P.packA, sh_);
    if (staged) {
        // block-uniform: the indicator phase below has block barriers
        if (__syncthreads_or(failed(P))) return;
        // the next pair's entries, halo positions and coefficients are
        // loaded one pair ahead
        int64_t p = p0 + threadIdx.x, en = 0, tn = 0;
        int lin = 0, ljn = 0;
        double cn[D], ctn[D];
        if (p < p1) {
            en = P.pair_e[p];
            tn = P.pair_t[p];
            lin = P.pair_li[p];
            ljn = P.loc[en];
            load_cp<D>(P, p, cn, ctn);
        }
        for (; p < p1; p += kBlock) {
            const int64_t e = en, t = tn;
            const int li = lin, lj = ljn;
            double c[D], ct[D];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                c[q] = cn[q];
                ct[q] = ctn[q];
            }
            if (p + kBlock < p1) {
                en = P.pair_e[p + kBlock];
                tn = P.pair_t[p + kBlock];
                lin = P.pair_li[p + kBlock];
                ljn = P.loc[en];
                load_cp<D>(P, p + kBlock, cn, ctn);
            }
            const double2 *ri = sh_ + li * NS;
            const double2 *rj = sh_ + lj * NS;
            double Ai[2 * NCH], Aj[2 * NCH];
#pragma unroll
            for (int k = 0; k < NCH; ++k) {
                const double2 a = ri[k], q = rj[k];
                Ai[2 * k] = a.x;
                Ai[2 * k + 1] = a.y;
                Aj[2 * k] = q.x;
                Aj[2 * k + 1] = q.y;
            }
            dpair_eval<D>(P, p, e, t, c, ct, Ai, Aj);
        }
        if (with_alpha) alpha_rows<D, true>(P, b, sh_);
    } else {
        double2 *lw = sh_ + (threadIdx.x / kSlice) * NCH * kLdsRow;
        for (int64_t q0 = p0; q0 < p1; q0 += kBlock) dpair_sweep<D>(P, q0 + threadIdx.x, p1, lw);
        if (with_alpha) alpha_rows<D, false>(P, b, nullptr);
    }
}

// d_ii and tau_i alone (the viscosity sweep computed the indicator): a
// kernel of its own, whose few registers leave room for eight waves per SIMD
__global__ void __launch_bounds__(kBlock) k_dsum(StageArgs P)
{
    diag_only(P, ROW_SLICE(P), P.nslices);
}

template <int D>
__global__ void __launch_bounds__(kBlock, 4) k_diag(StageArgs P, int mode)
{
    WAVE_LDS(kDiagChunks<D>)
    diag_sweep<D>(P, ROW_SLICE(P), P.nslices, mode != 0, nullptr,
                  GatherFetch<kDiagChunks<D>>{P.packA, lw});
}

template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_low(StageArgs P, int with_diag)
{
    constexpr int NCH = kPackL / 2;
    if constexpr (D == 3) {
        low_sweep<D, SP>(P, ROW_SLICE(P), P.nslices,
                         LaneTailFetch<NCH, NCH - 1, kPackL>{P.packL}, with_diag);
    } else {
        WAVE_LDS(NCH)
        low_sweep<D, SP>(P, ROW_SLICE(P), P.nslices,
                         GatherTailFetch<NCH, NCH - 1, kPackL>{P.packL, lw}, with_diag);
    }
}

// the persistent worker's low-order fetch: per lane in 3D, gathered in 2D
template <int D>
struct LowFetch {
    const double *base;
    double2 *lw;
    __device__ __forceinline__ int token(int64_t e) const
    {
        (void)e;
        return 0;
    }
    __device__ __forceinline__ void operator()(int tok, int node, double *rec) const
    {
        constexpr int NCH = kPackL / 2;
        if constexpr (D == 3)
            LaneTailFetch<NCH, NCH - 1, kPackL>{base}(tok, node, rec);
        else
            GatherTailFetch<NCH, NCH - 1, kPackL>{base, lw}(tok, node, rec);
    }
};

template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_lim1p(StageArgs P)
{
    WAVE_LDS(Chunks<D>::packB)
    lim1_sweep<D, SP>(P, PAIR_INDEX(P), P.npairs, lw);
}

template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_pass1a(StageArgs P)
{
    WAVE_LDS(Chunks<D>::packBrow)
    pass1_sweep<D, SP>(P, ROW_SLICE(P), P.nslices,
                       GatherFetch<Chunks<D>::packBrow>{P.packB, lw});
}

template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_lim2p(StageArgs P)
{
    WAVE_LDS(Chunks<D>::packB)
    lim2_sweep<D, SP>(P, PAIR_INDEX(P), P.npairs, lw);
}

// Pass 2's limiter over the work list: one wavefront per slice takes the
// slice's listed pairs, 64 at a time.  The listed pairs cluster where the
// flow is limited, so consecutive slices go to consecutive blocks, which
// the hardware deals out over the XCDs (the XCD-aware order of the sweeps,
// a contiguous range of slices per XCD, measured 1.44 against 1.13 ms;
// 4 and 16 slices per wavefront 1.18 and 1.29 ms).
template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_lim2s(StageArgs P)
{
    WAVE_LDS(Chunks<D>::packB)
    const int64_t s = int64_t(blockIdx.x) * (kBlock / kSlice) + threadIdx.x / kSlice;
    if (s >= P.nslices || failed(P)) return;
    const int64_t base = P.slow_base[s];
    const int cap = int(P.slow_base[s + 1] - base);
    int cnt = P.slow_cnt[s];
    cnt = cnt < cap ? cnt : cap;
    const int lane = int(threadIdx.x % kSlice);
    for (int q0 = 0; q0 < cnt; q0 += kSlice) {
        const int q = q0 + lane;
        const bool valid = q < cnt;
        const int64_t e = P.slow[base + (valid ? q : q0)];
        const int64_t t = P.stpos[e];
        const int j = P.scol[e], i = P.scol[t];
        lim2_pair<D, SP>(P, valid, -1, e, t, i, j, P.mij[e], P.l1[e], lw);
    }
}

template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_pass2(StageArgs P, const double *U0, double *out,
                                                  int mode)
{
    WAVE_LDS(Chunks<D>::packBrow)
    // consecutive slices to consecutive blocks, dealt out over the XCDs by
    // the hardware: pass 2's work clusters where the flow is limited, and
    // the XCD-aware order (a contiguous range of slices per XCD) left one
    // XCD with most of it (3.30 against 2.44 ms per launch at 257^3)
    pass2_sweep<D, SP>(P, int64_t(blockIdx.x) * (kBlock / kSlice) + threadIdx.x / kSlice,
                       P.nslices, U0, out, mode,
                       GatherFetch<Chunks<D>::packBrow>{P.packB, lw});
}

// LDS-staged row sweeps: the block first stages its rows' neighbourhood
// (the records of its halo nodes, up to 75 KB in 3D, 48 KB in 2D) and its
// rows then read their neighbours from LDS; a block whose halo did not fit
// gathers as above, with its wavefront tiles inside the same buffer.
// Staged: the two passes, and in 2D the low-order sweep.  The diagonal
// sweep measured slower staged in both dimensions (3D 7.8 vs 5.7 ms at
// 257^3, 2D 0.77 vs 0.58 ms on the 64-mesh batch) and keeps the gathers.
#define HALO_SWEEP(NCH, LAST, STRIDE, BASE, CALL)                            \
    __shared__ double2 sh_[kHaloMaxD<D> * (NCH)];                            \
    const int64_t hb_ = logical_block(P.per);                                \
    if (stage_halo<NCH, LAST, STRIDE>(P, hb_, BASE, sh_)) {                  \
        const HaloFetch<NCH> f_{sh_, P.loc};                                 \
        CALL;                                                                \
    } else {                                                                 \
        const GatherTailFetch<NCH, LAST, STRIDE> f_{BASE,                    \
                                            sh_ + (threadIdx.x / kSlice) * (NCH) * kLdsRow}; \
        CALL;                                                                \
    }

template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_pass1a_h(StageArgs P)
{
    constexpr int NCH = Chunks<D>::packBrow;
    HALO_SWEEP(NCH, NCH - 1, kPack, P.packB, (pass1_sweep<D, SP>(P, ROW_SLICE(P), P.nslices, f_)))
}

template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_pass2_h(StageArgs P, const double *U0, double *out,
                                                    int mode)
{
    constexpr int NCH = Chunks<D>::packBrow;
    HALO_SWEEP(NCH, NCH - 1, kPack, P.packB,
               (pass2_sweep<D, SP>(P, ROW_SLICE(P), P.nslices, U0, out, mode, f_)))
}

// staged low-order sweep
template <int D, bool SP>
__global__ void __launch_bounds__(kBlock) k_low_h(StageArgs P, int with_diag)
{
    HALO_SWEEP(kPackL / 2, kPackL / 2 - 1, kPackL, P.packL,
               (low_sweep<D, SP>(P, ROW_SLICE(P), P.nslices, f_, with_diag)))
}

// ------------------------------------------------ persistent batch launch
// Every wavefront is an independent worker that pops work items from one
// queue in (stage, sweep, instance) order.  An item of sweep s of instance
// k waits until every item of the earlier sweeps of that instance's stage
// (and the instance's tau update) has completed; items only ever wait on
// items earlier in the queue, which running workers hold, so the queue
// always drains, whatever the number of resident wavefronts.  The last
// diagonal item of an instance to complete also selects the instance's tau
// (the kernel-launch path's k_tau).  A wait that outlives kWaitPolls polls
// sets kErrWait and gives up; every later item then skips its work, so
// every wavefront reaches the end.  All control flow of the worker loop is
// wavefront-uniform (values through readfirstlane, atomics issued by every
// lane with the increment on lane 0 only): there is no block barrier and
// no lane-divergent region around the queue, so the compiler cannot split
// the loop between lanes.
constexpr unsigned kWaitPolls = 1u << 22;
constexpr unsigned long long kPosInf = 0x7FF0000000000000ull;

__device__ __forceinline__ uint32_t uniform32(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint64_t u = uint64_t(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ unsigned load_done(unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_batch_init(StageArgs P, BatchArgs B, int clear_status)
{
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) {
        *B.head = 0;
        if (clear_status) *P.status = 0;
    }
    for (int k = threadIdx.x; k < P.ninst; k += blockDim.x) {
        B.done[k] = 0;
        B.taumin2[k] = kPosInf;
        B.taumin2[P.ninst + k] = kPosInf;
    }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_persistent(StageArgs P, BatchArgs B)
{
    __shared__ double2 lds_[kBlock / kSlice][kMaxChunks * kLdsRow];
    double2 *const lw = lds_[threadIdx.x / kSlice];
    const int lane = threadIdx.x % kSlice;
    const unsigned one = lane == 0 ? 1u : 0u;   // per-wavefront increments
    for (;;) {
        const int64_t q = uniform64(int64_t(atomicAdd(B.head, (unsigned long long)one)));
        if (q >= B.total_items) return;
        const int64_t sg = q / B.items_per_stage;   // stage index of the whole run
        const int64_t r = q - sg * B.items_per_stage;
        int s = 0;
        while (s + 1 < kSweeps && B.sweep_off[s + 1] <= r) ++s;
        const int k = int(uniform32(uint32_t(B.item_inst[r])));
        const int64_t first = uniform64(B.item_first[r]);
        const int64_t *pre = B.pre + int64_t(k) * (kSweeps + 1);
        const unsigned base = uniform32(unsigned(sg * pre[kSweeps]));
        const unsigned need = base + uniform32(unsigned(pre[s]));
        for (unsigned polls = 0;;) {
            if (uniform32(load_done(B.done + k)) >= need) break;
            if (++polls > kWaitPolls) {
                atomicOr(P.status, kErrWait);
                break;
            }
            if ((polls & 1023u) == 0 &&
                (uniform32(__hip_atomic_load(P.status, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) & kErrWait))
                break;
            __builtin_amdgcn_s_sleep(8);
        }
        __threadfence();   // acquire: the stores of the items waited for
        const int stage = int(sg % 3);
        const int64_t *end = B.unit_end + int64_t(k) * 3;   // nodes, pairs, slices
        const int64_t e0 = uniform64(end[0]), e1 = uniform64(end[1]), e2 = uniform64(end[2]);
        const int ntile = int(uniform32(uint32_t(B.item_tile[r])));
        for (int u = 0; u < ntile; ++u) {
            const int64_t lin = first + int64_t(u) * kSlice + lane;   // node, pair
            const int64_t sl = first + u;                               // slice
            switch (s) {
            case 0: node_sweep<D>(P, lin, e0, stage == 0 ? B.U : B.U1,
                                  stage == 0 ? B.check : 0, lw); break;
            case 1: dpair_sweep<D>(P, lin, e1, lw); break;
            case 2:
                diag_sweep<D>(P, sl, e2, 1, B.taumin2 + (sg & 1) * P.ninst,
                              GatherFetch<kDiagChunks<D>>{P.packA, lw});
                break;
            case 3: low_sweep<D>(P, sl, e2, LowFetch<D>{P.packL, lw}); break;
            case 4: lim1_sweep<D>(P, lin, e1, lw); break;
            case 5:
                pass1_sweep<D>(P, sl, e2, GatherFetch<Chunks<D>::packBrow>{P.packB, lw});
                break;
            case 6: lim2_sweep<D>(P, lin, e1, lw); break;
            default:
                pass2_sweep<D>(P, sl, e2, B.U, stage == 2 ? B.U : B.U1, stage + 1,
                               GatherFetch<Chunks<D>::packBrow>{P.packB, lw});
            }
        }
        __threadfence();   // release: this item's stores before its completion count
        const unsigned old = uniform32(atomicAdd(B.done + k, one));
        if (s == 2 && old + 1 == base + unsigned(pre[3]) - 1) {
            // every diagonal item of the instance is in: select its tau (every
            // lane writes the same values)
            __threadfence();
            const unsigned long long bits = __hip_atomic_load(
                B.taumin2 + (sg & 1) * P.ninst + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const double bound = __longlong_as_double((long long)uniform64(int64_t(bits)));
            select_tau(P, k, bound, P.dt_inst ? P.dt_inst[k] : 0.0, stage == 0 ? 1 : 0);
            if (stage == 0) B.dt_rec[(sg / 3) * P.ninst + k] = P.tau[k];
            B.taumin2[((sg + 1) & 1) * P.ninst + k] = kPosInf;   // next stage's slot
            __threadfence();
            (void)atomicAdd(B.done + k, one);
        }
    }
}

// ------------------------------------------------------- device math
__global__ void k_math(int kind, int64_t n, const double *x, const double *y, double *out)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    if (kind == 0) out[i] = fpow(x[i], y[i]);
    else if (kind == 1) out[i] = sqrt(x[i]);
    else out[i] = x[i] / y[i];
}

// Debug export of per-entry quantities the pair sweeps compute and do not
// keep, from the buffers of the last stage, with the sweeps' own device
// functions: what 0: component `comp` of P_ij (eq. def-p); 1: the pass-1
// candidate l_ij (Alg. 2 on U^L_i, P_ij, bounds_i); 2: the pass-2 candidate
// on (pass-1 state of i, (1 - s1_ij) P_ij, bounds_i).  Diagonal: P_ii = 0,
// candidates 1.  One thread per row, SELL positions.
template <int D>
__global__ void k_debug_entries(StageArgs P, int what, int comp, double *out)
{
    constexpr int NC = D + 2;
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (r >= P.nslices * kSlice) return;
    const int i = P.perm[r];
    if (i < 0) return;
    const int L = P.row_len[r];
    const int64_t off = P.slice_off[r / kSlice] + r % kSlice;
    NodeB<D> Bi;
    load_b<D>(P.packB + int64_t(i) * kPack, Bi);
    const double *W = P.rowB + int64_t(i) * kRowB;
    const double *Up = P.upass + int64_t(i) * kRowU;
    for (int k = 0; k < L; ++k) {
        const int64_t e = off + int64_t(k) * kSlice;
        const int j = P.scol[e];
        if (j == i) {
            out[e] = what == 0 ? 0.0 : 1.0;
            continue;
        }
        NodeB<D> Bj;
        load_b<D>(P.packB + int64_t(j) * kPack, Bj);
        double Pd[NC];
        direction<D>(Bi, Bj, Bi.coef, P.d[e], P.mij[e], Pd);
        if (what == 0) {
            out[e] = Pd[comp];
        } else if (what == 1) {
            out[e] = row_limiter<D>(W, W, Pd, P);
        } else {
            const double l = P.l1[e];
#pragma unroll
            for (int q = 0; q < NC; ++q) Pd[q] = (1.0 - l) * Pd[q];
            out[e] = limiter<D>(Up, Pd, Up[NC], Up[NC + 1], Up[NC + 2], P.gamma, P.newton_max,
                                P.tol);
        }
    }
}

// Decision traces (tests only): after a stage, the branch every
// comparison, clamp, max and min of the stage took, recomputed from the
// stage's buffers with the sweeps' own device functions.
//  k_trace_pairs, one thread per pair: bits 0-13 the viscosity's
//    (pair_viscosity), bits 16-23 / 24-31 the pass-1 limiter of (i,j) /
//    (j,i), bits 32-39 / 40-47 those of pass 2 (kLim* bits), bit 48 / 49
//    whether l_ij < l_ji in pass 1 / 2;
//  k_trace_rows, one thread per row: the indicator's signs (indicator).
template <int D>
__global__ void k_trace_pairs(StageArgs P, unsigned long long *out)
{
    constexpr int NC = D + 2;
    const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= P.npairs) return;
    const int64_t e = P.pair_e[p];
    const int i = P.pair_i[p], j = P.pair_j[p];
    double c[D], ct[D];
    c[0] = P.c0[e];
    c[1] = P.c1[e];
    ct[0] = P.ct0[e];
    ct[1] = P.ct1[e];
    if constexpr (D == 3) {
        c[2] = P.c2[e];
        ct[2] = P.ct2[e];
    }
    double Ai[NC + 2], Aj[NC + 2];
#pragma unroll
    for (int k = 0; k < NC + 2; ++k) {
        Ai[k] = P.packA[int64_t(i) * kPack + k];
        Aj[k] = P.packA[int64_t(j) * kPack + k];
    }
    bool first;
    unsigned cv = 0;
    pair_viscosity<D, true>(c, ct, Ai, Aj, P.gas, first, &cv);
    NodeB<D> Bi, Bj;
    load_b<D>(P.packB + int64_t(i) * kPack, Bi);
    load_b<D>(P.packB + int64_t(j) * kPack, Bj);
    const double dL = P.d[e], m = P.mij[e];
    double Pij[NC], Pji[NC];
    direction<D>(Bi, Bj, Bi.coef, dL, m, Pij);
    direction<D>(Bj, Bi, Bj.coef, dL, m, Pji);
    const double *Wi = P.rowB + int64_t(i) * kRowB, *Wj = P.rowB + int64_t(j) * kRowB;
    unsigned a1 = 0, b1 = 0, a2 = 0, b2 = 0;
    const double lij = limiter<D, true>(Wi, Pij, Wi[NC], Wi[NC + 1], Wi[NC + 2], P.gamma,
                                        P.newton_max, P.tol, &a1);
    const double lji = limiter<D, true>(Wj, Pji, Wj[NC], Wj[NC + 1], Wj[NC + 2], P.gamma,
                                        P.newton_max, P.tol, &b1);
    unsigned long long code = cv | (a1 << 16) | (b1 << 24) | (lij < lji ? 1ull << 48 : 0ull);
    if (P.passes >= 2) {
        const double l = P.l1[e];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            Pij[q] = (1.0 - l) * Pij[q];
            Pji[q] = (1.0 - l) * Pji[q];
        }
        const double *Ui = P.upass + int64_t(i) * kRowU, *Uj = P.upass + int64_t(j) * kRowU;
        const double mij2 = limiter<D, true>(Ui, Pij, Ui[NC], Ui[NC + 1], Ui[NC + 2], P.gamma,
                                             P.newton_max, P.tol, &a2);
        const double mji2 = limiter<D, true>(Uj, Pji, Uj[NC], Uj[NC + 1], Uj[NC + 2], P.gamma,
                                             P.newton_max, P.tol, &b2);
        code |= (static_cast<unsigned long long>(a2) << 32) |
                (static_cast<unsigned long long>(b2) << 40) | (mij2 < mji2 ? 1ull << 49 : 0ull);
    }
    out[p] = code;
}

template <int D>
__global__ void k_trace_rows(StageArgs P, unsigned *out)
{
    constexpr int NC = D + 2;
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (r >= P.nslices * kSlice) return;
    const int i = P.perm[r];
    if (i < 0) return;
    const int L = P.row_len[r];
    const int64_t off = P.slice_off[r / kSlice] + r % kSlice;
    NodeA<D> Ai;
    load_a_fwd<D>(P.packA + int64_t(i) * kPack, Ai);
    double Fi[NC][D];
    flux<D>(Ai.U, Ai.v, Ai.p, Fi);
    double a = 0.0, b[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) b[q] = 0.0;
    // the row sums of the diagonal sweep, in its order
    for (int k = 0; k < L; ++k) {
        const int64_t e = off + int64_t(k) * kSlice;
        NodeA<D> Aj;
        load_a_fwd<D>(P.packA + int64_t(P.scol[e]) * kPack, Aj);
        double c[D];
        c[0] = P.c0[e];
        c[1] = P.c1[e];
        if constexpr (D == 3) c[2] = P.c2[e];
        double mc = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) mc += Aj.U[1 + q] * c[q];
        a += (Aj.er - Ai.er) * mc;
        double Fj[NC][D], fd[NC];
        flux<D>(Aj.U, Aj.v, Aj.p, Fj);
        flux_diff_dot<D>(Fi, Fj, c, fd);
#pragma unroll
        for (int q = 0; q < NC; ++q) b[q] += fd[q];
    }
    unsigned code = 0;
    indicator<D, true>(Ai.U, Ai.er, a, b, P.gamma, &code);
    out[i] = code;
}

// Widening of the bounds: r_i = (m_i/|Omega|)^(1.5/d), |Omega| = sum_i m_i
// (summed on the host in the caller's node order).
__global__ void k_relax(StageArgs P, double mass_total, double expo)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= P.n) return;
    P.relax_r[i] = fpow(P.mi[i] / mass_total, expo);
}

// ------------------------------------------------------------ launches
static inline int grid_rows(const StageArgs &P) { return P.per * kXcd; }
static inline int grid_nodes(int64_t n) { return int((n + kBlock - 1) / kBlock); }

void launch_matrices(const StageArgs &P, hipStream_t st, const double *coords,
                     const int32_t *cells, const int64_t *nc_ptr,
                     const int32_t *nc_list, const double gx[3], int *err)
{
    if (P.dim == 2)
        hipLaunchKernelGGL(k_matrices<2>, dim3(grid_rows(P)), dim3(kBlock), 0, st, P,
                           coords, cells, nc_ptr, nc_list, gx[0], gx[1], gx[2], err);
    else
        hipLaunchKernelGGL(k_matrices<3>, dim3(grid_rows(P)), dim3(kBlock), 0, st, P,
                           coords, cells, nc_ptr, nc_list, gx[0], gx[1], gx[2], err);
    hipLaunchKernelGGL(k_lumped, dim3(grid_rows(P)), dim3(kBlock), 0, st, P);
    if (P.dim == 2)
        hipLaunchKernelGGL(k_transpose_c<2>, dim3(grid_rows(P)), dim3(kBlock), 0, st, P);
    else
        hipLaunchKernelGGL(k_transpose_c<3>, dim3(grid_rows(P)), dim3(kBlock), 0, st, P);
    if (P.npairs > 0) {
        const dim3 gp(unsigned((P.npairs + kBlock - 1) / kBlock));
        hipLaunchKernelGGL(k_pair_mass, gp, dim3(kBlock), 0, st, P);
        if (P.dim == 2)
            hipLaunchKernelGGL(k_pair_c<2>, gp, dim3(kBlock), 0, st, P);
        else
            hipLaunchKernelGGL(k_pair_c<3>, gp, dim3(kBlock), 0, st, P);
    }
}

// s2 of every pair that pass 1 left unlimited (s1 = 1), which the pass-2
// limiter sweep skips unless records are kept: the smaller of the two rows'
// l2self, as the limiter returns it along the zero direction
__global__ void __launch_bounds__(kBlock) k_l2_fill(StageArgs P)
{
    const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= P.npairs) return;
    const int64_t e = P.pair_e[p];
    if (P.l1[e] != 1.0) return;
    const double a = P.l2self[P.pair_i[p]], b = P.l2self[P.pair_j[p]];
    const double sv = a < b ? a : b;
    P.l2[e] = sv;
    P.l2[P.pair_t[p]] = sv;
}

void launch_l2_fill(const StageArgs &P, hipStream_t st)
{
    if (P.npairs == 0) return;
    const dim3 g(unsigned((P.npairs + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_l2_fill, g, dim3(kBlock), 0, st, P);
}

void launch_debug_entries(const StageArgs &P, hipStream_t st, int what, int comp, double *out)
{
    const dim3 g(unsigned((P.nslices * kSlice + kBlock - 1) / kBlock));
    if (P.dim == 2)
        hipLaunchKernelGGL(k_debug_entries<2>, g, dim3(kBlock), 0, st, P, what, comp, out);
    else
        hipLaunchKernelGGL(k_debug_entries<3>, g, dim3(kBlock), 0, st, P, what, comp, out);
}

void launch_trace(const StageArgs &P, hipStream_t st, unsigned long long *pairs,
                  unsigned *rows)
{
    const dim3 gp(unsigned((P.npairs + kBlock - 1) / kBlock));
    const dim3 gr(unsigned((P.nslices * kSlice + kBlock - 1) / kBlock));
    if (P.dim == 2) {
        if (P.npairs) hipLaunchKernelGGL(k_trace_pairs<2>, gp, dim3(kBlock), 0, st, P, pairs);
        hipLaunchKernelGGL(k_trace_rows<2>, gr, dim3(kBlock), 0, st, P, rows);
    } else {
        if (P.npairs) hipLaunchKernelGGL(k_trace_pairs<3>, gp, dim3(kBlock), 0, st, P, pairs);
        hipLaunchKernelGGL(k_trace_rows<3>, gr, dim3(kBlock), 0, st, P, rows);
    }
}

void launch_relax(const StageArgs &P, hipStream_t st, double mass_total)
{
    hipLaunchKernelGGL(k_relax, dim3(grid_nodes(P.n)), dim3(kBlock), 0, st, P, mass_total,
                       1.5 / double(P.dim));
}

void launch_begin(const StageArgs &P, hipStream_t st, int clear_status)
{
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(kBlock), 0, st, P, clear_status);
}

void launch_tau(const StageArgs &P, hipStream_t st, double dt_in, int mode, int fold)
{
    hipLaunchKernelGGL(k_tau, dim3(1), dim3(kBlock), 0, st, P, dt_in, mode, fold);
}

void launch_node(const StageArgs &P, hipStream_t st, const double *U, int check)
{
    if (P.dim == 2)
        hipLaunchKernelGGL(k_node<2>, dim3(grid_nodes(P.n)), dim3(kBlock), 0, st, P, U, check);
    else
        hipLaunchKernelGGL(k_node<3>, dim3(grid_nodes(P.n)), dim3(kBlock), 0, st, P, U, check);
}

static inline int grid_pairs(const StageArgs &P) { return P.pper * kXcd; }

#define LAUNCH_D(K, grid, ...)                                                          \
    do {                                                                                \
        if (P.dim == 2)                                                                 \
            hipLaunchKernelGGL(K<2>, dim3(grid), dim3(kBlock), 0, st, __VA_ARGS__);     \
        else                                                                            \
            hipLaunchKernelGGL(K<3>, dim3(grid), dim3(kBlock), 0, st, __VA_ARGS__);     \
    } while (0)
// sweeps with a variant-3 instantiation (the viscous part of P_ij stored)
#define LAUNCH_DS(K, grid, ...)                                                         \
    do {                                                                                \
        if (P.q) {                                                                      \
            if (P.dim == 2)                                                             \
                hipLaunchKernelGGL((K<2, true>), dim3(grid), dim3(kBlock), 0, st, __VA_ARGS__); \
            else                                                                        \
                hipLaunchKernelGGL((K<3, true>), dim3(grid), dim3(kBlock), 0, st, __VA_ARGS__); \
        } else {                                                                        \
            if (P.dim == 2)                                                             \
                hipLaunchKernelGGL((K<2, false>), dim3(grid), dim3(kBlock), 0, st, __VA_ARGS__); \
            else                                                                        \
                hipLaunchKernelGGL((K<3, false>), dim3(grid), dim3(kBlock), 0, st, __VA_ARGS__); \
        }                                                                               \
    } while (0)

void launch_dpair(const StageArgs &P, hipStream_t st, int with_alpha)
{
    const dim3 g(unsigned(grid_rows(P)));
    if (P.halo_cnt && P.pair_blk) {
        if (P.dim == 2)
            hipLaunchKernelGGL((k_dpair_h<2, kHaloMax2>), g, dim3(kBlock), 0, st, P, with_alpha);
        else if (P.dpair_cap == kHaloPair3)
            hipLaunchKernelGGL((k_dpair_h<3, kHaloPair3>), g, dim3(kBlock), 0, st, P, with_alpha);
        else
            hipLaunchKernelGGL((k_dpair_h<3, kHaloMax3>), g, dim3(kBlock), 0, st, P, with_alpha);
    } else
        LAUNCH_D(k_dpair, grid_pairs(P), P);
}
void launch_diag(const StageArgs &P, hipStream_t st, int mode)
{
    if (mode == 2)
        hipLaunchKernelGGL(k_dsum, dim3(grid_rows(P)), dim3(kBlock), 0, st, P);
    else
        LAUNCH_D(k_diag, grid_rows(P), P, mode);
}
void launch_low(const StageArgs &P, hipStream_t st, int with_diag)
{
    if (P.halo_cnt)
        LAUNCH_DS(k_low_h, grid_rows(P), P, with_diag);
    else
        LAUNCH_DS(k_low, grid_rows(P), P, with_diag);
}
void launch_tau_fold(const StageArgs &P, hipStream_t st, int reduce)
{
    if (P.nslices == 0) return;
    hipLaunchKernelGGL(k_tau_fold, dim3(unsigned((P.nslices + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, P);
    if (reduce) hipLaunchKernelGGL(k_tau_reduce, dim3(1), dim3(kBlock), 0, st, P);
}
void launch_lim1p(const StageArgs &P, hipStream_t st) { LAUNCH_DS(k_lim1p, grid_pairs(P), P); }
void launch_pass1a(const StageArgs &P, hipStream_t st)
{
    if (P.halo_cnt)
        LAUNCH_DS(k_pass1a_h, grid_rows(P), P);
    else
        LAUNCH_DS(k_pass1a, grid_rows(P), P);
}
void launch_lim2p(const StageArgs &P, hipStream_t st) { LAUNCH_DS(k_lim2p, grid_pairs(P), P); }

void launch_lim2(const StageArgs &P, hipStream_t st)
{
    if (!P.slow || P.side2) {
        launch_lim2p(P, st);
        return;
    }
    if (P.nslices == 0) return;
    const int grid = int((P.nslices + kBlock / kSlice - 1) / (kBlock / kSlice));
    LAUNCH_DS(k_lim2s, grid, P);
}
void launch_pass2(const StageArgs &P, hipStream_t st, const double *U0, double *out, int mode)
{
    if (P.halo_cnt && !P.slowmask)
        LAUNCH_DS(k_pass2_h, grid_rows(P), P, U0, out, mode);
    else
        LAUNCH_DS(k_pass2, grid_rows(P), P, U0, out, mode);
}

void launch_batch_init(const StageArgs &P, const BatchArgs &B, hipStream_t st, int clear_status)
{
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(kBlock), 0, st, P, B, clear_status);
}

void launch_persistent(const StageArgs &P, const BatchArgs &B, hipStream_t st, int grid)
{
    LAUNCH_D(k_persistent, grid, P, B);
}

int persistent_blocks_per_cu(int dim)
{
    int nb = 0;
    hipError_t e = dim == 2
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<2>, kBlock, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<3>, kBlock, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

void launch_math(hipStream_t st, int kind, int64_t n, const double *x, const double *y,
                 double *out)
{
    hipLaunchKernelGGL(k_math, dim3(grid_nodes(n)), dim3(kBlock), 0, st, kind, n, x, y, out);
}

}  // namespace idp
