// Pieces shared by the forward sweeps and their adjoints: block
// numbering, the SELL row and pair setups, node records and their
// gathers, and the limiter direction P_ij of eq. def-p.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "idp_device.h"
#include "kernels.h"

namespace idp {

__device__ __forceinline__ int64_t logical_block(int per)
{
    const int b = blockIdx.x;
    return int64_t(b % kXcd) * per + b / kXcd;
}

#define ROW_SETUP(P)                                                         \
    const int64_t s_ = logical_block(P.per) * (kBlock / kSlice) +            \
                       threadIdx.x / kSlice;                                 \
    if (s_ >= P.nslices) return;                                             \
    const int lane_ = threadIdx.x % kSlice;                                  \
    const int64_t r_ = s_ * kSlice + lane_;                                  \
    const int i = P.perm[r_];                                                \
    if (i < 0) return;                                                       \
    const int L = P.row_len[r_];                                             \
    const int64_t off_ = P.slice_off[s_] + lane_;

#define ENTRY(k) (off_ + int64_t(k) * kSlice)

__device__ __forceinline__ bool failed(const StageArgs &P)
{
    return (*P.status & kErrMask) != 0;
}

template <int D>
struct NodeA {
    double U[D + 2];
    double p, c, er, v[D], phi;
};

template <int D>
__device__ __forceinline__ void load_a(const double *__restrict__ A, NodeA<D> &o)
{
    constexpr int NC = D + 2;
#pragma unroll
    for (int k = 0; k < NC; ++k) o.U[k] = A[k];
    o.p = A[NC];
    o.c = A[NC + 1];
    o.er = A[NC + 2];
#pragma unroll
    for (int k = 0; k < D; ++k) o.v[k] = A[NC + 3 + k];
    o.phi = A[NC + 3 + D];
}

// The forward part of a pack A record (U, p, c, eta/rho) with v = m/rho
// recomputed exactly as the node pass computes it; phi is not set.
template <int D>
__device__ __forceinline__ void load_a_fwd(const double *__restrict__ A, NodeA<D> &o)
{
    constexpr int NC = D + 2;
#pragma unroll
    for (int k = 0; k < NC; ++k) o.U[k] = A[k];
    o.p = A[NC];
    o.c = A[NC + 1];
    o.er = A[NC + 2];
#pragma unroll
    for (int k = 0; k < D; ++k) o.v[k] = o.U[1 + k] / o.U[0];
    o.phi = 0.0;
}

// Streamed per-entry arrays of the diagonal and low-order sweeps (read once
// per sweep) carry the non-temporal hint, which leaves the L2 to the reused
// node records (measured: 1-3% faster there, slower in the passes).
template <class T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}

// ------------------------------------------------- cooperative gathers
// A lane that fetches a neighbour's record with its own 16-byte loads
// touches a different cache line per lane, so every load instruction costs
// the L1 address path 64 line lookups, and a 104-byte record costs seven
// instructions.  Instead the 64 lanes of a wavefront fetch the records of
// all its lanes together: lane l loads chunk l % LPR of the record wanted
// by lane it * (64 / LPR) + l / LPR, so one instruction covers 64 / LPR
// records (one line each), and the chunks reach their owners through a
// per-wavefront LDS tile.  All loads are issued before the first is used.
// Every lane of the wavefront must call it (node < 0: nothing wanted).
constexpr int kLdsRow = kSlice + 1;   // double2 per chunk row (+1: bank skew)
constexpr int kMaxChunks = 7;         // largest record gathered (pack B with coefficient)

// A 16-byte chunk in registers (a native vector: its copies stay loads and
// stores that the optimiser can keep in registers)
typedef double dchunk __attribute__((ext_vector_type(2)));

// Lanes per record and records per load instruction of an NCH-chunk gather.
template <int NCH> struct GatherShape {
    static_assert(NCH >= 1 && NCH <= 8, "record of 1 to 8 chunks");
    static constexpr int LPR = NCH > 4 ? 8 : (NCH > 2 ? 4 : (NCH > 1 ? 2 : 1));
    static constexpr int RPI = kSlice / LPR;
};

// The loads of a gather: chunks 0 .. NCH-2 and chunk LAST of the records
// the lanes want, as lane l holds them (val[it] = chunk l % LPR of the
// record of lane it * RPI + l / LPR); nothing waits for them yet.
template <int NCH, int LAST = NCH - 1>
__device__ __forceinline__ void gather_issue(const double *__restrict__ base, int stride,
                                             int node, dchunk (&val)[GatherShape<NCH>::LPR])
{
    static_assert(LAST >= NCH - 1, "prefix plus one chunk");
    using S = GatherShape<NCH>;
    const int lane = threadIdx.x % kSlice;
    const int c = lane % S::LPR;
    const int cc = c < NCH ? c : NCH - 1;   // spare lanes repeat the last chunk
    const int src = cc == NCH - 1 ? LAST : cc;
    int nd[S::LPR];
#pragma unroll
    for (int it = 0; it < S::LPR; ++it) {
        const int v = __shfl(node, it * S::RPI + lane / S::LPR);
        nd[it] = v < 0 ? 0 : v;
    }
#pragma unroll
    for (int it = 0; it < S::LPR; ++it)
        val[it] = *reinterpret_cast<const dchunk *>(base + int64_t(nd[it]) * stride + 2 * src);
}

// The chunks of gather_issue() to their owners through the wavefront's LDS
// tile: out = the lane's own record (NCH chunks).
template <int NCH>
__device__ __forceinline__ void gather_exchange(double2 *lds,
                                                const dchunk (&val)[GatherShape<NCH>::LPR],
                                                double *out)
{
    using S = GatherShape<NCH>;
    const int lane = threadIdx.x % kSlice;
    const int c = lane % S::LPR;
    const int cc = c < NCH ? c : NCH - 1;
    dchunk *const t = reinterpret_cast<dchunk *>(lds);
#pragma unroll
    for (int it = 0; it < S::LPR; ++it) t[cc * kLdsRow + it * S::RPI + lane / S::LPR] = val[it];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        const dchunk v = t[k * kLdsRow + lane];
        out[2 * k] = v.x;
        out[2 * k + 1] = v.y;
    }
    __builtin_amdgcn_wave_barrier();
}

template <int NCH>
__device__ __forceinline__ void gather(const double *__restrict__ base, int stride, int node,
                                       double2 *lds, double *out)
{
    dchunk val[GatherShape<NCH>::LPR];
    gather_issue<NCH>(base, stride, node, val);
    gather_exchange<NCH>(lds, val, out);
}

// Variant of gather() whose last chunk is chunk LAST of the record (the
// first NCH - 1 are chunks 0 .. NCH - 2): a record prefix plus one far slot.
template <int NCH, int LAST>
__device__ __forceinline__ void gather_tail(const double *__restrict__ base, int stride, int node,
                                            double2 *lds, double *out)
{
    static_assert(NCH >= 2 && NCH <= 8 && LAST >= NCH - 1, "prefix plus one chunk");
    dchunk val[GatherShape<NCH>::LPR];
    gather_issue<NCH, LAST>(base, stride, node, val);
    gather_exchange<NCH>(lds, val, out);
}

// The store counterpart of gather(): lane l's record `in` (NCH chunks) goes
// to base + node_l * stride (node < 0: nothing stored).  The records pass
// through the per-wavefront LDS tile so that each store instruction writes
// 64 / LPR whole records (one line each) instead of one chunk of 64 lines.
// Every lane of the wavefront must call it.
template <int NCH>
__device__ __forceinline__ void scatter(double *__restrict__ base, int stride, int node,
                                        double2 *lds, const double *in)
{
    static_assert(NCH >= 1 && NCH <= 8, "record of 1 to 8 chunks");
    constexpr int LPR = NCH > 4 ? 8 : (NCH > 2 ? 4 : (NCH > 1 ? 2 : 1));
    constexpr int RPI = kSlice / LPR;
    const int lane = threadIdx.x % kSlice;
    const int c = lane % LPR;
#pragma unroll
    for (int k = 0; k < NCH; ++k) lds[k * kLdsRow + lane] = make_double2(in[2 * k], in[2 * k + 1]);
    __builtin_amdgcn_wave_barrier();
    int nd[LPR];
#pragma unroll
    for (int it = 0; it < LPR; ++it) nd[it] = __shfl(node, it * RPI + lane / LPR);
    if (c < NCH) {
#pragma unroll
        for (int it = 0; it < LPR; ++it)
            if (nd[it] >= 0)
                *reinterpret_cast<double2 *>(base + int64_t(nd[it]) * stride + 2 * c) =
                    lds[c * kLdsRow + it * RPI + lane / LPR];
    }
    __builtin_amdgcn_wave_barrier();
}

// chunks of pack A as the node pass writes it: U, p, c, eta/rho, v, phi;
// the diagonal sweep reads U, p, c, eta/rho (and recomputes v = m/rho)
template <int D> constexpr int kPackAChunks = (D + 2 + 4 + D) / 2;
template <int D> constexpr int kDiagChunks = (D + 2 + 3 + 1) / 2;

// Where a row sweep takes its neighbours' records from.  GatherFetch: the
// wavefront's cooperative gather from global memory (every lane of the
// wavefront calls it).  HaloFetch: the block's neighbourhood staged in LDS,
// entry e's record at halo position loc[e] (per lane).  token(e) is loaded
// one entry ahead; node < 0: nothing wanted, rec untouched.
template <int NCH>
struct GatherFetch {
    const double *base;
    double2 *lw;
    // what the fetch of entry e needs ahead of time (nothing here)
    __device__ __forceinline__ int token(int64_t e) const
    {
        (void)e;
        return 0;
    }
    __device__ __forceinline__ void operator()(int tok, int node, double *rec) const
    {
        (void)tok;
        gather<NCH>(base, kPack, node, lw, rec);
    }
};

template <int NCH>
struct HaloFetch {
    const double2 *halo;
    const uint16_t *loc;
    __device__ __forceinline__ int token(int64_t e) const { return int(ld_stream(loc + e)); }
    __device__ __forceinline__ void operator()(int tok, int node, double *rec) const
    {
        if (node < 0) return;
        const double2 *h = halo + tok * NCH;
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const double2 v = h[k];
            rec[2 * k] = v.x;
            rec[2 * k + 1] = v.y;
        }
    }
};

// LDS staging of a row block's neighbourhood: the first NCH chunks of the
// record (STRIDE doubles per node) of every node in the block's halo, in halo order.
// Every thread of the block calls it (it ends in a block barrier); false
// if the block's halo did not fit (its rows then gather from memory): more
// than the host's cap (count -1) or than CAP records.
template <int NCH, int LAST = NCH - 1, int STRIDE = kPack, int CAP = 0x7fffffff>
__device__ __forceinline__ bool stage_halo(const StageArgs &P, int64_t b, const double *base,
                                           double2 *halo)
{
    static_assert(NCH <= 6 && LAST >= NCH - 1, "halo record");
    const int cnt = P.halo_cnt[b];
    if (cnt < 0 || cnt > CAP) return false;
    const int64_t h0 = P.halo_start[b];
    const int tot = cnt * NCH;
#pragma unroll 4
    for (int q = int(threadIdx.x); q < tot; q += kBlock) {
        const int r = q / NCH, c = q - r * NCH;
        const int src = c == NCH - 1 ? LAST : c;
        halo[q] = *reinterpret_cast<const double2 *>(
            base + int64_t(P.halo_node[h0 + r]) * STRIDE + 2 * src);
    }
    __syncthreads();
    return true;
}

// Fetches of chunks 0 .. NCH-2 and chunk LAST of a record: per lane
// (LaneTailFetch) or wavefront-cooperative (GatherTailFetch).
template <int NCH, int LAST, int STRIDE = kPack>
struct LaneTailFetch {
    const double *base;
    __device__ __forceinline__ int token(int64_t e) const
    {
        (void)e;
        return 0;
    }
    __device__ __forceinline__ void operator()(int tok, int node, double *rec) const
    {
        (void)tok;
        if (node < 0) return;
        const double *a = base + int64_t(node) * STRIDE;
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int src = k == NCH - 1 ? LAST : k;
            rec[2 * k] = a[2 * src];
            rec[2 * k + 1] = a[2 * src + 1];
        }
    }
};

template <int NCH, int LAST, int STRIDE = kPack>
struct GatherTailFetch {
    const double *base;
    double2 *lw;
    __device__ __forceinline__ int token(int64_t e) const
    {
        (void)e;
        return 0;
    }
    __device__ __forceinline__ void operator()(int tok, int node, double *rec) const
    {
        (void)tok;
        gather_tail<NCH, LAST>(base, STRIDE, node, lw, rec);
    }
};

// Launch shapes of the wavefront sweeps: row sweeps take slice 4 b + w in
// wavefront w of logical block b; pair sweeps one pair per lane.
#define ROW_SLICE(P) (logical_block(P.per) * (kBlock / kSlice) + threadIdx.x / kSlice)
#define PAIR_INDEX(P) (logical_block(P.pper) * kBlock + threadIdx.x)
#define WAVE_LDS(NCH)                                                        \
    [[maybe_unused]] constexpr int kTile_ = (NCH);  /* chunks per record */ \
    __shared__ double2 lds_[kBlock / kSlice][(NCH) * kLdsRow];               \
    double2 *const lw = lds_[threadIdx.x / kSlice];

// Row sweeps: one wavefront per slice s (below send); every lane stays to
// the end of the slice's longest row; lanes past the node count take node
// 0 and write nothing.  inst_ is the slice's instance.
#define WAVE_ROW_SETUP(P, S, SEND)                                           \
    const int64_t s_ = (S);                                                  \
    if (s_ >= (SEND)) return;                                                \
    const int lane_ = threadIdx.x % kSlice;                                  \
    const int64_t r_ = s_ * kSlice + lane_;                                  \
    const int iraw_ = P.perm[r_];                                            \
    const bool valid_ = iraw_ >= 0;                                          \
    const int i = valid_ ? iraw_ : 0;                                        \
    const int L = valid_ ? P.row_len[r_] : 0;                                \
    const int64_t off_ = P.slice_off[s_] + lane_;                            \
    /* the slice's instance, wavefront-uniform: keeps atomics on its tau */  \
    /* combined per wavefront                                            */  \
    const int inst_ = __builtin_amdgcn_readfirstlane(                        \
        P.inst_slice ? P.inst_slice[s_] : 0);                                \
    int Lmax_ = L;                                                           \
    for (int o_ = kSlice / 2; o_ > 0; o_ /= 2) {                             \
        const int v_ = __shfl_xor(Lmax_, o_);                                \
        Lmax_ = v_ > Lmax_ ? v_ : Lmax_;                                     \
    }

// Pair sweeps: one lane per pair p (below pend); lanes past the end take
// pair 0 and write nothing; a wavefront with no pair leaves.
#define WAVE_PAIR_SETUP(P, PIDX, PEND)                                       \
    const int64_t p_ = (PIDX);                                               \
    if (p_ - threadIdx.x % kSlice >= (PEND)) return;                         \
    const bool valid_ = p_ < (PEND);                                         \
    const int64_t pq_ = valid_ ? p_ : 0;                                     \
    const int64_t e = P.pair_e[pq_];                                         \
    const int64_t t = P.pair_t[pq_];                                         \
    const int i = P.pair_i[pq_];                                             \
    const int j = P.pair_j[pq_];

template <int D>
__device__ __forceinline__ void load_c(const StageArgs &P, int64_t e, double *c)
{
    c[0] = P.c0[e];
    c[1] = P.c1[e];
    if (D == 3) c[D - 1] = P.c2[e];
}

// the same for c_ij
template <int D>
__device__ __forceinline__ void load_c_stream(const StageArgs &P, int64_t e, double *c)
{
    c[0] = ld_stream(P.c0 + e);
    c[1] = ld_stream(P.c1 + e);
    if (D == 3) c[D - 1] = ld_stream(P.c2 + e);
}

template <int D>
struct NodeB {
    double U[D + 2], R[D + 2], alpha, m, coef;
};

template <int D>
__device__ __forceinline__ void load_b(const double *__restrict__ B, NodeB<D> &o)
{
    constexpr int NC = D + 2;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        o.U[k] = B[k];
        o.R[k] = B[NC + k];
    }
    o.alpha = B[2 * NC];
    o.m = B[2 * NC + 1];
    o.coef = B[kPackCoef];
}

// pack B record as gathered: U, R, alpha, m (and the coefficient if
// WITH_COEF, i.e. if the gather reached slot kPackCoef)
template <int D, bool WITH_COEF>
__device__ __forceinline__ void unpack_b(const double *o, NodeB<D> &B)
{
    constexpr int NC = D + 2;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        B.U[k] = o[k];
        B.R[k] = o[NC + k];
    }
    B.alpha = o[2 * NC];
    B.m = o[2 * NC + 1];
    B.coef = WITH_COEF ? o[kPackCoef] : 0.0;
}

// Pack B record of `node` with the coefficient, gathered cooperatively:
// U, R, alpha, m (2 nc + 2 doubles) and the coefficient's chunk (in 2D the
// record's middle chunk is skipped).  Every lane of the wavefront calls it.
template <int D>
__device__ __forceinline__ void gather_b(const double *__restrict__ packB, int node, double2 *lw,
                                         NodeB<D> &B)
{
    constexpr int NC = D + 2, NB = (2 * NC + 2) / 2;
    double rec[2 * (NB + 1)];
    gather_tail<NB + 1, kPackCoef / 2>(packB, kPack, node, lw, rec);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        B.U[k] = rec[k];
        B.R[k] = rec[NC + k];
    }
    B.alpha = rec[2 * NC];
    B.m = rec[2 * NC + 1];
    B.coef = rec[2 * NB];
}

// Pack B records (with the coefficient) of two nodes, the loads of both
// in flight before either passes through the LDS tile.
template <int D>
__device__ __forceinline__ void gather_b2(const double *__restrict__ packB, int na, int nb,
                                          double2 *lw, NodeB<D> &A, NodeB<D> &B)
{
    constexpr int NC = D + 2, NB = (2 * NC + 2) / 2, NCH = NB + 1;
    dchunk va[GatherShape<NCH>::LPR], vb[GatherShape<NCH>::LPR];
    gather_issue<NCH, kPackCoef / 2>(packB, kPack, na, va);
    gather_issue<NCH, kPackCoef / 2>(packB, kPack, nb, vb);
    double rec[2 * NCH];
    gather_exchange<NCH>(lw, va, rec);
    unpack_b<D, false>(rec, A);
    A.coef = rec[2 * NB];
    gather_exchange<NCH>(lw, vb, rec);
    unpack_b<D, false>(rec, B);
    B.coef = rec[2 * NB];
}

// eq. def-p: P_ij = tau/(lambda_i m_i) (b_ij R_j - b_ji R_i + (d^H - d^L)(U_j - U_i)),
// b_ij = -m_ij/m_j, b_ji = -m_ij/m_i (j != i)
template <int D>
__device__ __forceinline__ void direction(const NodeB<D> &Bi, const NodeB<D> &Bj,
                                          double coef, double dL, double mij,
                                          double *Pd)
{
    const double dH = dL * (Bi.alpha + Bj.alpha) / 2.0;
    const double bij = -mij / Bj.m;
    const double bji = -mij / Bi.m;
#pragma unroll
    for (int r = 0; r < D + 2; ++r)
        Pd[r] = coef * (bij * Bj.R[r] - bji * Bi.R[r] + (dH - dL) * (Bj.U[r] - Bi.U[r]));
}

// The same with the viscous part Q = (d^H - d^L)(U_j - U_i) given (the
// paper's variant 3 stores it in step 3): the same value, bit for bit.
template <int D>
__device__ __forceinline__ void direction_q(const NodeB<D> &Bi, const NodeB<D> &Bj,
                                            double coef, double mij, const double *Q,
                                            double *Pd)
{
    const double bij = -mij / Bj.m;
    const double bji = -mij / Bi.m;
#pragma unroll
    for (int r = 0; r < D + 2; ++r) Pd[r] = coef * (bij * Bj.R[r] - bji * Bi.R[r] + Q[r]);
}

// Candidate of row i on the line U + t P_ij under the bounds of row i.
template <int D>
__device__ __forceinline__ double row_limiter(const double *Urow, const double *W,
                                              const double *Pd, const StageArgs &P)
{
    constexpr int NC = D + 2;
    return limiter<D>(Urow, Pd, W[NC], W[NC + 1], W[NC + 2], P.gamma, P.newton_max, P.tol);
}

// record sizes in 16-byte chunks
template <int D> struct Chunks {
    static constexpr int NC = D + 2;
    static constexpr int packB = kPackCoef / 2 + 1;   // U, R, alpha, m, coefficient
    static constexpr int packBrow = NC + 1;           // U, R, alpha, m
    static constexpr int rowB = (NC + 4) / 2;         // U^L, bounds
    static constexpr int upass = (NC + 1) / 2;        // pass-1 state
    static constexpr int upassb = (NC + 4) / 2;       // pass-1 state and bounds
};
static_assert(Chunks<3>::packB <= kMaxChunks && Chunks<2>::packB <= kMaxChunks, "LDS tile");

}  // namespace idp
