// C-ABI of the library: context, precompute, SSP-RK3 stepper, exports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/idp.h"
#include "adjoint.h"
#include "graph.h"
#include "kernels.h"

static_assert(idp::kSellC == idp::kSlice, "SELL slice height = wavefront width");

namespace {

enum KernelId {
    K_BEGIN, K_NODE, K_DPAIR, K_DIAG, K_TAU, K_LOW, K_LIM1P, K_PASS1A, K_LIM2P, K_PASS2,
    K_PERSIST, K_VJP, K_COUNT
};
const char *kKernelNames[K_COUNT] = {"begin", "node_pack", "pair_viscosity", "row_diagonal",
                                     "tau", "row_low_order", "pair_limiter1", "row_pass1",
                                     "pair_limiter2", "row_pass2", "batch_persistent",
                                     "stage_vjp"};

struct Pending {
    int id;
    hipEvent_t a, b;
};

// Device block of scalars, copied back in one transfer: the status word,
// then per instance min tau_i (bits), tau and the bound.
struct Scalars {
    int status = 0;
    std::vector<unsigned long long> taumin;
    std::vector<double> tau, bound;
};
constexpr size_t kScalHead = 16;
inline size_t scal_bytes(int ninst) { return kScalHead + size_t(ninst) * 24; }

// Work tables of one persistent schedule (tile size) of a batch.
struct PersistTables {
    int tile = 0;
    idp::BatchArgs B{};
    int32_t *item_inst = nullptr, *item_tile = nullptr;
    int64_t *item_first = nullptr, *pre = nullptr;
};

}  // namespace

struct idp_ctx {
    idp_params prm{};
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0, nnz = 0;
    size_t bytes = 0;
    std::vector<void *> allocs;
    // host copies kept for the CSR exports
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<int64_t> sell_of_csr;
    int64_t sell_size = 0;
    idp::StageArgs P{};
    char *scal = nullptr;           // device block, see Scalars
    double *U1 = nullptr;
    // IDP_FLAG_RENUMBER: the library's node k is the caller's node order[k];
    // pos is the inverse (host and device); the state lives in Uint
    std::vector<int32_t> order, pos;
    int32_t *pos_dev = nullptr;
    double *Uint = nullptr;
    double *Pa = nullptr, *Pb = nullptr;   // the adjoint's caller arrays, renumbered
    // batches
    int ninst = 1;
    idp::BatchLayout lay;           // instance offsets (single mesh: one instance)
    double *dt_dev = nullptr;       // [ninst] per-instance dt of a batch call
    double *dt_rec = nullptr;       // [dt_rec_cap] tau of every step and instance
    int64_t dt_rec_cap = 0;
    int64_t *unit_end = nullptr;    // [ninst][3] node, pair, slice ends
    unsigned long long *taumin2 = nullptr;
    unsigned int *done = nullptr;
    unsigned long long *head = nullptr;
    std::vector<PersistTables> tables;
    idp_schedule tuned{IDP_SCHED_LAUNCHES, 0};
    double *U_tune = nullptr;
    // adjoint
    idp::AdjArgs A{};
    bool adj_ready = false;
    double *Estage = nullptr, *U2 = nullptr, *Ebp = nullptr, *acc = nullptr;
    double *bar[3] = {nullptr, nullptr, nullptr};
    uint8_t *sided = nullptr, *side1 = nullptr, *side2 = nullptr;   // records of a
                                                                    // recomputed stage
    int32_t *argk = nullptr;
    double *ckpt = nullptr;          // [slots][n][nc]
    int64_t ckpt_slots = 0;
    int ck_steps = -1, ck_every = 0;
    std::vector<double> ck_dt;
    // tape: the per-stage arrays of tape_steps steps (3 stage argument sets
    // each), so that a segment recomputed once serves its whole backward
    void *tape_mem = nullptr;
    size_t tape_bytes = 0;
    int tape_steps = 0;
    std::vector<idp::StageArgs> tape;
    bool tape_last = false;          // holds the last segment of the forward
    // the backward's recomputation stream (default priority) and its events:
    // [0, 1] a bank of the tape recomputed, [2, 3] a bank's VJPs done, [4] start
    hipStream_t stream2 = nullptr;
    hipEvent_t ev[5] = {};
    // timing
    bool timing = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[K_COUNT] = {};
    int64_t launches[K_COUNT] = {};
};

namespace {

template <class T>
int dalloc(idp_ctx *c, T **p, size_t count)
{
    void *q = nullptr;
    const size_t b = count * sizeof(T);
    if (hipMalloc(&q, b > 0 ? b : 8) != hipSuccess) {
        (void)hipGetLastError();
        return IDP_ENOMEM;
    }
    c->allocs.push_back(q);
    c->bytes += b;
    *p = static_cast<T *>(q);
    return IDP_OK;
}

hipEvent_t get_event(idp_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch wrapper: brackets the launch with events when timing is on.
template <class F>
void timed_on(idp_ctx *c, hipStream_t st, int id, F &&launch)
{
    if (!c->timing) {
        launch();
        return;
    }
    Pending p{id, get_event(c), get_event(c)};
    if (p.a) (void)hipEventRecord(p.a, st);
    launch();
    if (p.b) (void)hipEventRecord(p.b, st);
    c->pending.push_back(p);
}

template <class F>
void timed(idp_ctx *c, int id, F &&launch)
{
    timed_on(c, c->stream, id, launch);
}

// After a stream synchronisation: fold event pairs into the totals.
void collect(idp_ctx *c)
{
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (p.a && p.b && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->total_ms[p.id] += ms;
            c->launches[p.id] += 1;
        }
        if (p.a) c->pool.push_back(p.a);
        if (p.b) c->pool.push_back(p.b);
    }
    c->pending.clear();
}

int sync(idp_ctx *c)
{
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        return IDP_EHIP;
    }
    if (hipGetLastError() != hipSuccess) return IDP_EHIP;
    collect(c);
    return IDP_OK;
}

int read_scalars(idp_ctx *c, Scalars *h)
{
    const int n = c->ninst;
    std::vector<char> buf(scal_bytes(n));
    if (hipMemcpyAsync(buf.data(), c->scal, buf.size(), hipMemcpyDeviceToHost, c->stream) !=
        hipSuccess)
        return IDP_EHIP;
    const int rc = sync(c);
    if (rc != IDP_OK) return rc;
    std::memcpy(&h->status, buf.data(), sizeof(int));
    h->taumin.resize(n);
    h->tau.resize(n);
    h->bound.resize(n);
    std::memcpy(h->taumin.data(), buf.data() + kScalHead, size_t(n) * 8);
    std::memcpy(h->tau.data(), buf.data() + kScalHead + size_t(n) * 8, size_t(n) * 8);
    std::memcpy(h->bound.data(), buf.data() + kScalHead + size_t(n) * 16, size_t(n) * 8);
    return IDP_OK;
}

int status_code(int st)
{
    if (st & idp::kErrState) return IDP_ESTATE;
    if (st & idp::kErrDt) return IDP_EDT;
    if (st & idp::kErrWait) return IDP_EWAIT;
    if (st & idp::kWarnCfl) return IDP_WARN_CFL;
    return IDP_OK;
}

// States between the caller's numbering and the library's (renumbered
// contexts): to_internal: out[pos[i]] = in[i]; else out[i] = in[pos[i]].
__global__ void k_permute(int64_t n, int nc, const int32_t *__restrict__ pos,
                          const double *__restrict__ in, double *__restrict__ out,
                          int to_internal)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = pos[i];
    if (to_internal)
        for (int r = 0; r < nc; ++r) out[k * nc + r] = in[i * nc + r];
    else
        for (int r = 0; r < nc; ++r) out[i * nc + r] = in[k * nc + r];
}

void permute(idp_ctx *c, const double *in, double *out, int to_internal)
{
    const int nc = c->prm.dim + 2;
    hipLaunchKernelGGL(k_permute, dim3(unsigned((c->n + 255) / 256)), dim3(256), 0, c->stream,
                       c->n, nc, c->pos_dev, in, out, to_internal);
}

// One forward-Euler stage on the context stream.
//  in: stage input state; U0: step-initial state; out: destination;
//  tau_mode: 1 select tau (stage 1), 0 check the held tau, 2 use dt_in.
//  P: the stage's arguments (the context's, or a set whose per-stage arrays
//  live elsewhere, e.g. in the adjoint's tape).
void stage_p(idp_ctx *c, const idp::StageArgs &P, const double *in, const double *U0,
             double *out, int mode, int tau_mode, double dt_in, int check, int clear,
             hipStream_t st)
{
    timed_on(c, st, K_BEGIN, [&] { idp::launch_begin(P, st, clear); });
    timed_on(c, st, K_NODE, [&] { idp::launch_node(P, st, in, check); });
    // the row-block viscosity sweep computes the indicator of every row
    const bool staged = P.halo_cnt && P.pair_blk;
    timed_on(c, st, K_DPAIR, [&] { idp::launch_dpair(P, st, staged ? 1 : 0); });
    if (staged && tau_mode == 0) {
        // tau held (stages 2 and 3): the low-order sweep sums d_ii and tau_i
        // on its way, and the CFL check follows it
        timed_on(c, st, K_LOW, [&] { idp::launch_low(P, st, 1); });
        timed_on(c, st, K_TAU, [&] {
            idp::launch_tau_fold(P, st, 0);
            idp::launch_tau(P, st, dt_in, tau_mode, 1);
        });
    } else {
        timed_on(c, st, K_DIAG, [&] { idp::launch_diag(P, st, staged ? 2 : 1); });
        timed_on(c, st, K_TAU, [&] {
            idp::launch_tau_fold(P, st, 0);
            idp::launch_tau(P, st, dt_in, tau_mode, 1);
        });
        timed_on(c, st, K_LOW, [&] { idp::launch_low(P, st, 0); });
    }
    timed_on(c, st, K_LIM1P, [&] { idp::launch_lim1p(P, st); });
    timed_on(c, st, K_PASS1A, [&] { idp::launch_pass1a(P, st); });
    if (P.passes >= 2) timed_on(c, st, K_LIM2P, [&] { idp::launch_lim2(P, st); });
    timed_on(c, st, K_PASS2, [&] { idp::launch_pass2(P, st, U0, out, mode); });
}

void stage_p(idp_ctx *c, const idp::StageArgs &P, const double *in, const double *U0,
             double *out, int mode, int tau_mode, double dt_in, int check, int clear)
{
    stage_p(c, P, in, U0, out, mode, tau_mode, dt_in, check, clear, c->stream);
}

void stage(idp_ctx *c, const double *in, const double *U0, double *out, int mode,
           int tau_mode, double dt_in, int check, int clear)
{
    stage_p(c, c->P, in, U0, out, mode, tau_mode, dt_in, check, clear);
}

}  // namespace

extern "C" {

int idp_default_params(idp_params *p, int dim)
{
    if (!p || (dim != 2 && dim != 3)) return IDP_EINVAL;
    p->dim = dim;
    p->gamma = 1.4;
    p->cfl = 0.5;
    p->limiter_passes = 2;
    p->newton_max_iter = 2;
    p->newton_tol = 1e-10;
    p->relax_bounds = 0;
    p->flags = 0;
    p->sell_sigma = 0;
    return IDP_OK;
}

void idp_destroy(idp_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->pending) {
        if (p.a) (void)hipEventDestroy(p.a);
        if (p.b) (void)hipEventDestroy(p.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->stream2) {
        (void)hipStreamSynchronize(c->stream2);
        (void)hipStreamDestroy(c->stream2);
    }
    for (auto e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (void *q : c->allocs) (void)hipFree(q);
    if (c->tape_mem) (void)hipFree(c->tape_mem);
    delete c;
}

}  // extern "C"

namespace {

struct MeshIn {
    int64_t n_nodes, n_cells;
    const double *coords;
    const int64_t *cells;
    const uint8_t *dirichlet;
};

int check_params(const idp_params &p)
{
    if ((p.dim != 2 && p.dim != 3) || !(p.gamma > 1.0) || !(p.cfl > 0.0) ||
        !(p.cfl <= 1.0) || (p.limiter_passes != 1 && p.limiter_passes != 2) ||
        p.newton_max_iter < 0 || p.newton_max_iter > 64 || !(p.newton_tol >= 0.0) ||
        p.sell_sigma < 0 || p.sell_sigma % idp::kSellC != 0)
        return IDP_EINVAL;
    if (p.relax_bounds != 0 && p.relax_bounds != 1) return IDP_EINVAL;
    return IDP_OK;
}

// One context for one mesh or a batch of meshes (concatenated graph).
int create_impl(idp_ctx **out, const idp_params &p, const std::vector<MeshIn> &meshes,
                void *hip_stream)
{
    const int K = int(meshes.size());
    idp_ctx *c = new (std::nothrow) idp_ctx;
    if (!c) return IDP_ENOMEM;
    c->prm = p;
    c->ninst = K;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return IDP_EHIP; }
    const int dim = p.dim;
    const int nv = 1 << dim;

    idp::HostGraph g;
    // host mesh arrays of the whole context (concatenated for a batch)
    std::vector<double> coords_all;
    std::vector<int64_t> cells_all;
    std::vector<uint8_t> hold_all;
    const double *coords = meshes[0].coords;
    const int64_t *cells = meshes[0].cells;
    const uint8_t *dirichlet = meshes[0].dirichlet;
    int64_t n_cells = meshes[0].n_cells;
    int rc = IDP_OK;
    try {
        if (K == 1 && (p.flags & IDP_FLAG_RENUMBER)) {
            // nodes numbered along a Morton curve; rows keep the caller's
            // column order (key = the caller's id), so the sums run as before
            const int64_t n = meshes[0].n_nodes;
            for (int64_t t = 0; t < n_cells * nv; ++t)
                if (cells[t] < 0 || cells[t] >= n) rc = IDP_EINVAL;
            if (rc == IDP_OK) {
                idp::morton_order(dim, n, coords, c->order);
                c->pos.assign(size_t(n), 0);
                for (int64_t k = 0; k < n; ++k) c->pos[size_t(c->order[size_t(k)])] = int32_t(k);
                cells_all.resize(size_t(n_cells) * nv);
                for (int64_t t = 0; t < n_cells * nv; ++t)
                    cells_all[size_t(t)] = c->pos[size_t(cells[t])];
                coords_all.resize(size_t(n) * dim);
                for (int64_t k = 0; k < n; ++k)
                    for (int d = 0; d < dim; ++d)
                        coords_all[size_t(k) * dim + d] = coords[int64_t(c->order[size_t(k)]) * dim + d];
                if (dirichlet) {
                    hold_all.resize(size_t(n));
                    for (int64_t k = 0; k < n; ++k) hold_all[size_t(k)] = dirichlet[c->order[size_t(k)]];
                    dirichlet = hold_all.data();
                }
                cells = cells_all.data();
                coords = coords_all.data();
                rc = idp::build_graph(g, dim, n, n_cells, cells, p.sell_sigma, c->order.data());
            }
            auto &L = c->lay;
            L.node = {0, g.n};
            L.cell = {0, g.ncells};
            L.nnz = {0, g.nnz};
            L.slice = {0, g.nslices};
            L.sell = {0, g.sell_size};
            L.pair = {0, g.npairs};
        } else if (K == 1) {
            rc = idp::build_graph(g, dim, meshes[0].n_nodes, n_cells, cells, p.sell_sigma);
            auto &L = c->lay;
            L.node = {0, g.n};
            L.cell = {0, g.ncells};
            L.nnz = {0, g.nnz};
            L.slice = {0, g.nslices};
            L.sell = {0, g.sell_size};
            L.pair = {0, g.npairs};
        } else {
            std::vector<idp::HostGraph> parts(K);
            for (int k = 0; k < K && rc == IDP_OK; ++k)
                rc = idp::build_graph(parts[k], dim, meshes[k].n_nodes, meshes[k].n_cells,
                                      meshes[k].cells, p.sell_sigma);
            if (rc == IDP_OK) rc = idp::concat_graphs(parts, g, c->lay);
            if (rc == IDP_OK) {
                const auto &L = c->lay;
                coords_all.resize(size_t(L.node[K]) * dim);
                cells_all.resize(size_t(L.cell[K]) * nv);
                bool any_hold = false;
                for (int k = 0; k < K; ++k) any_hold = any_hold || meshes[k].dirichlet;
                if (any_hold) hold_all.assign(size_t(L.node[K]), 0);
                for (int k = 0; k < K; ++k) {
                    const MeshIn &m = meshes[k];
                    std::memcpy(coords_all.data() + L.node[k] * dim, m.coords,
                                size_t(m.n_nodes) * dim * 8);
                    for (int64_t t = 0; t < m.n_cells * nv; ++t)
                        cells_all[L.cell[k] * nv + t] = m.cells[t] + L.node[k];
                    if (m.dirichlet)
                        std::memcpy(hold_all.data() + L.node[k], m.dirichlet, size_t(m.n_nodes));
                }
                coords = coords_all.data();
                cells = cells_all.data();
                dirichlet = any_hold ? hold_all.data() : nullptr;
                n_cells = L.cell[K];
            }
        }
    } catch (const std::bad_alloc &) {
        rc = IDP_ENOMEM;
    }
    if (rc != IDP_OK) { delete c; return rc; }
    c->n = g.n;
    c->nnz = g.nnz;
    c->sell_size = g.sell_size;
    const int64_t nrows = g.nslices * idp::kSlice;
    idp::StageArgs &P = c->P;
    P.dim = dim;
    P.n = g.n;
    P.nslices = g.nslices;
    const int64_t blocks = (g.nslices + (idp::kBlock / idp::kSlice) - 1) / (idp::kBlock / idp::kSlice);
    P.per = int((blocks + idp::kXcd - 1) / idp::kXcd);
    P.gamma = p.gamma;
    P.gas = idp::make_gas(p.gamma);
    P.cfl = p.cfl;
    P.tol = p.newton_tol;
    P.newton_max = p.newton_max_iter;
    P.passes = p.limiter_passes;
    P.ninst = K;

    int32_t *perm, *row_len, *diag_k, *scol, *stpos;
    int32_t *pe, *pt, *pi, *pj;
    int64_t *slice_off;
    const int64_t S = g.sell_size;
    int e = IDP_OK;
#define TRY(x) do { if ((e = (x)) != IDP_OK) { idp_destroy(c); return e; } } while (0)
#define HIPTRY(x) do { if ((x) != hipSuccess) { (void)hipGetLastError(); idp_destroy(c); return IDP_EHIP; } } while (0)
    TRY(dalloc(c, &perm, nrows));
    TRY(dalloc(c, &row_len, nrows));
    TRY(dalloc(c, &diag_k, nrows));
    TRY(dalloc(c, &slice_off, g.nslices));
    TRY(dalloc(c, &scol, S));
    TRY(dalloc(c, &stpos, S));
    TRY(dalloc(c, &pe, g.npairs));
    TRY(dalloc(c, &pt, g.npairs));
    TRY(dalloc(c, &pi, g.npairs));
    TRY(dalloc(c, &pj, g.npairs));
    TRY(dalloc(c, &P.mp, g.npairs));
    TRY(dalloc(c, &P.cpair, g.npairs * 2 * dim));
    TRY(dalloc(c, &P.dp, g.npairs));
    TRY(dalloc(c, &P.l1p, g.npairs));
    TRY(dalloc(c, &P.c0, S));
    TRY(dalloc(c, &P.c1, S));
    if (dim == 3) TRY(dalloc(c, &P.c2, S));
    TRY(dalloc(c, &P.ct0, S));
    TRY(dalloc(c, &P.ct1, S));
    if (dim == 3) TRY(dalloc(c, &P.ct2, S));
    TRY(dalloc(c, &P.mij, S));
    TRY(dalloc(c, &P.d, S));
    TRY(dalloc(c, &P.l1, S));
    TRY(dalloc(c, &P.l2, S));
    TRY(dalloc(c, &P.mi, g.n));
    TRY(dalloc(c, &P.lam, g.n));
    TRY(dalloc(c, &P.packA, g.n * idp::kPack));
    TRY(dalloc(c, &P.packL, g.n * idp::kPackL));
    TRY(dalloc(c, &P.packB, g.n * idp::kPack));
    TRY(dalloc(c, &P.rowB, g.n * idp::kRowB));
    TRY(dalloc(c, &P.upass, g.n * idp::kRowU));
    TRY(dalloc(c, &P.l2self, g.n));
    {
        // pass 2's work list (see StageArgs::slow)
        std::vector<int64_t> base;
        idp::upper_bases(g, base);
        int64_t *sb = nullptr;
        TRY(dalloc(c, &P.slowmask, std::max<int64_t>(S / 64, 1)));
        TRY(dalloc(c, &P.slow, std::max<int64_t>(g.npairs, 1)));
        TRY(dalloc(c, &P.slow_cnt, std::max<int64_t>(g.nslices, 1)));
        TRY(dalloc(c, &sb, int64_t(base.size())));
        HIPTRY(hipMemcpyAsync(sb, base.data(), base.size() * 8, hipMemcpyHostToDevice,
                              c->stream));
        HIPTRY(hipMemsetAsync(P.slow_cnt, 0, size_t(std::max<int64_t>(g.nslices, 1)) * 4,
                              c->stream));
        HIPTRY(hipStreamSynchronize(c->stream));   // base leaves scope
        P.slow_base = sb;
    }
    TRY(dalloc(c, &P.alpha, g.n));
    TRY(dalloc(c, &P.taui, g.n));
    TRY(dalloc(c, &P.wmin, std::max<int64_t>(g.nslices, 1)));
    TRY(dalloc(c, &P.wmin_blk, std::max<int64_t>((g.nslices + idp::kBlock - 1) / idp::kBlock, 1)));
    if (p.flags & IDP_FLAG_SPLIT_P) {
        // the paper's variant 3: the viscous part of P_ij per entry
        TRY(dalloc(c, &P.q, S * (dim + 2)));
        P.qstride = S;
    }
    TRY(dalloc(c, &c->U1, g.n * (dim + 2)));
    TRY(dalloc(c, &c->scal, scal_bytes(K)));
    uint8_t *hold = nullptr;
    if (dirichlet) {
        TRY(dalloc(c, &hold, g.n));
        HIPTRY(hipMemcpyAsync(hold, dirichlet, g.n, hipMemcpyHostToDevice, c->stream));
    }
    if (K > 1) {
        int32_t *inst = nullptr;
        TRY(dalloc(c, &inst, g.nslices));
        HIPTRY(hipMemcpyAsync(inst, c->lay.inst_slice.data(), g.nslices * 4,
                              hipMemcpyHostToDevice, c->stream));
        P.inst_slice = inst;
    }
    P.hold = hold;
    P.perm = perm;
    P.row_len = row_len;
    P.diag_k = diag_k;
    P.slice_off = slice_off;
    P.scol = scol;
    P.stpos = stpos;
    P.npairs = g.npairs;
    P.pper = int(((g.npairs + idp::kBlock - 1) / idp::kBlock + idp::kXcd - 1) / idp::kXcd);
    P.pair_e = pe;
    P.pair_t = pt;
    P.pair_i = pi;
    P.pair_j = pj;
    P.status = reinterpret_cast<int *>(c->scal);
    P.taumin = reinterpret_cast<unsigned long long *>(c->scal + kScalHead);
    P.tau = reinterpret_cast<double *>(c->scal + kScalHead + size_t(K) * 8);
    P.bound = reinterpret_cast<double *>(c->scal + kScalHead + size_t(K) * 16);
    HIPTRY(hipMemcpyAsync(perm, g.perm.data(), nrows * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(row_len, g.row_len.data(), nrows * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(diag_k, g.diag_k.data(), nrows * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(slice_off, g.slice_off.data(), g.nslices * 8, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(scol, g.scol.data(), S * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(stpos, g.stpos.data(), S * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(pe, g.pair_e.data(), g.npairs * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(pt, g.pair_t.data(), g.npairs * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(pi, g.pair_i.data(), g.npairs * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(pj, g.pair_j.data(), g.npairs * 4, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemsetAsync(c->scal, 0, scal_bytes(K), c->stream));
    // neighbourhoods of the row blocks for the LDS-staged row sweeps
    if (!(p.flags & IDP_FLAG_NO_STAGING)) {
        idp::Halos h;
        const int64_t nblk = int64_t(P.per) * idp::kXcd;
        TRY(idp::build_halos(g, nblk, dim == 3 ? idp::kHaloMax3 : idp::kHaloMax2, h));
        // the viscosity sweep's smaller cap where few blocks exceed it
        int64_t mid = 0;
        for (int64_t q = 0; q < nblk; ++q) mid += h.cnt[size_t(q)] > idp::kHaloPair3;
        P.dpair_cap = mid * 50 <= nblk ? idp::kHaloPair3 : idp::kHaloMax3;
        int64_t *hs;
        int32_t *hc, *hn;
        uint16_t *hl;
        TRY(dalloc(c, &hs, nblk));
        TRY(dalloc(c, &hc, nblk));
        TRY(dalloc(c, &hn, int64_t(h.node.size())));
        TRY(dalloc(c, &hl, S));
        HIPTRY(hipMemcpyAsync(hs, h.start.data(), nblk * 8, hipMemcpyHostToDevice, c->stream));
        HIPTRY(hipMemcpyAsync(hc, h.cnt.data(), nblk * 4, hipMemcpyHostToDevice, c->stream));
        if (!h.node.empty())
            HIPTRY(hipMemcpyAsync(hn, h.node.data(), h.node.size() * 4, hipMemcpyHostToDevice,
                                  c->stream));
        HIPTRY(hipMemcpyAsync(hl, h.loc.data(), S * 2, hipMemcpyHostToDevice, c->stream));
        if (!h.pair_blk.empty()) {
            int64_t *pb;
            uint16_t *pl;
            TRY(dalloc(c, &pb, nblk + 1));
            TRY(dalloc(c, &pl, std::max<int64_t>(g.npairs, 1)));
            HIPTRY(hipMemcpyAsync(pb, h.pair_blk.data(), (nblk + 1) * 8, hipMemcpyHostToDevice,
                                  c->stream));
            if (g.npairs)
                HIPTRY(hipMemcpyAsync(pl, h.pair_li.data(), g.npairs * 2,
                                      hipMemcpyHostToDevice, c->stream));
            P.pair_blk = pb;
            P.pair_li = pl;
        }
        // the host vectors die at the end of this scope: wait for the copies
        HIPTRY(hipStreamSynchronize(c->stream));
        P.halo_start = hs;
        P.halo_cnt = hc;
        P.halo_node = hn;
        P.loc = hl;
    }

    // matrices on the device (temporary mesh arrays)
    {
        std::vector<int32_t> cells32;
        try {
            cells32.resize(size_t(n_cells) * nv);
        } catch (const std::bad_alloc &) {
            idp_destroy(c);
            return IDP_ENOMEM;
        }
        for (int64_t t = 0; t < n_cells * nv; ++t) cells32[t] = int32_t(cells[t]);
        double *dco = nullptr;
        int32_t *dcells = nullptr, *dnl = nullptr;
        int64_t *dncp = nullptr;
        int *derr = nullptr;
        bool ok = hipMalloc(&dco, size_t(g.n) * dim * 8) == hipSuccess &&
                  hipMalloc(&dcells, cells32.size() * 4) == hipSuccess &&
                  hipMalloc(&dncp, g.nc_ptr.size() * 8) == hipSuccess &&
                  hipMalloc(&dnl, g.nc_list.size() * 4) == hipSuccess &&
                  hipMalloc(&derr, sizeof(int)) == hipSuccess;
        int herr = 0;
        if (ok) {
            ok = hipMemcpyAsync(dco, coords, size_t(g.n) * dim * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                 hipMemcpyAsync(dcells, cells32.data(), cells32.size() * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                 hipMemcpyAsync(dncp, g.nc_ptr.data(), g.nc_ptr.size() * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                 hipMemcpyAsync(dnl, g.nc_list.data(), g.nc_list.size() * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                 hipMemsetAsync(derr, 0, sizeof(int), c->stream) == hipSuccess;
        }
        if (ok) {
            const double gx[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
            idp::launch_matrices(P, c->stream, dco, dcells, dncp, dnl, gx, derr);
            ok = hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
                 hipStreamSynchronize(c->stream) == hipSuccess && hipGetLastError() == hipSuccess;
        }
        const bool alloc_fail = !(dco && dcells && dncp && dnl && derr);
        (void)hipFree(dco); (void)hipFree(dcells); (void)hipFree(dncp); (void)hipFree(dnl); (void)hipFree(derr);
        if (!ok) {
            (void)hipGetLastError();
            idp_destroy(c);
            return alloc_fail ? IDP_ENOMEM : IDP_EHIP;
        }
        if (herr) { idp_destroy(c); return IDP_EMESH; }
    }
    if (p.relax_bounds) {
        // |Omega| = sum_i m_i, summed in the caller's node order
        std::vector<double> mi_host;
        try {
            mi_host.resize(size_t(g.n));
        } catch (const std::bad_alloc &) {
            idp_destroy(c);
            return IDP_ENOMEM;
        }
        TRY(dalloc(c, &P.relax_r, g.n));
        HIPTRY(hipMemcpyAsync(mi_host.data(), P.mi, size_t(g.n) * 8, hipMemcpyDeviceToHost,
                              c->stream));
        HIPTRY(hipStreamSynchronize(c->stream));
        double mass_total = 0.0;
        for (int64_t i = 0; i < g.n; ++i)
            mass_total += mi_host[c->pos.empty() ? size_t(i) : size_t(c->pos[size_t(i)])];
        idp::launch_relax(P, c->stream, mass_total);
        HIPTRY(hipGetLastError());
    }
    // keep what the CSR exports need (in the caller's numbering), drop the
    // rest of the host graph
    if (!c->pos.empty()) {
        const int64_t n = g.n;
        c->row_ptr.assign(size_t(n) + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = c->pos[size_t(i)];
            c->row_ptr[size_t(i) + 1] = c->row_ptr[size_t(i)] + (g.row_ptr[k + 1] - g.row_ptr[k]);
        }
        c->col.resize(size_t(g.nnz));
        c->sell_of_csr.resize(size_t(g.nnz));
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = c->pos[size_t(i)], q0 = c->row_ptr[size_t(i)];
            for (int64_t q = g.row_ptr[k]; q < g.row_ptr[k + 1]; ++q) {
                c->col[size_t(q0 + q - g.row_ptr[k])] = c->order[size_t(g.col[q])];
                c->sell_of_csr[size_t(q0 + q - g.row_ptr[k])] = g.sell_of_csr[q];
            }
        }
        TRY(dalloc(c, &c->pos_dev, n));
        TRY(dalloc(c, &c->Uint, n * (dim + 2)));
        HIPTRY(hipMemcpyAsync(c->pos_dev, c->pos.data(), size_t(n) * 4, hipMemcpyHostToDevice,
                              c->stream));
        HIPTRY(hipStreamSynchronize(c->stream));
    } else {
        c->row_ptr.swap(g.row_ptr);
        c->col.swap(g.col);
        c->sell_of_csr.swap(g.sell_of_csr);
    }
#undef TRY
#undef HIPTRY
    *out = c;
    return IDP_OK;
}

}  // namespace

extern "C" {

int idp_create(idp_ctx **out, const idp_params *prm, int64_t n_nodes,
               const double *coords, int64_t n_cells, const int64_t *cells,
               const uint8_t *dirichlet, void *hip_stream)
{
    if (!out || !prm || !coords || !cells) return IDP_EINVAL;
    *out = nullptr;
    const int rc = check_params(*prm);
    if (rc != IDP_OK) return rc;
    if (n_nodes < 1 || n_cells < 1) return IDP_EINVAL;   // an empty mesh has no step
    return create_impl(out, *prm, {MeshIn{n_nodes, n_cells, coords, cells, dirichlet}},
                       hip_stream);
}

int idp_create_batch(idp_ctx **out, const idp_params *prm, int n_inst,
                     const int64_t *n_nodes, const double *const *coords,
                     const int64_t *n_cells, const int64_t *const *cells,
                     const uint8_t *const *dirichlet, void *hip_stream)
{
    if (!out || !prm || n_inst < 1 || !n_nodes || !coords || !n_cells || !cells)
        return IDP_EINVAL;
    *out = nullptr;
    const int rc = check_params(*prm);
    if (rc != IDP_OK) return rc;
    if (prm->flags & IDP_FLAG_RENUMBER) return IDP_ENOTSUP;   // single meshes only
    if (prm->relax_bounds) return IDP_ENOTSUP;                 // single meshes only
    if (prm->flags & IDP_FLAG_SPLIT_P) return IDP_ENOTSUP;     // single meshes only
    std::vector<MeshIn> meshes;
    try {
        meshes.resize(n_inst);
    } catch (const std::bad_alloc &) {
        return IDP_ENOMEM;
    }
    for (int k = 0; k < n_inst; ++k) {
        if (!coords[k] || !cells[k] || n_nodes[k] < 1 || n_cells[k] < 1) return IDP_EINVAL;
        meshes[k] = MeshIn{n_nodes[k], n_cells[k], coords[k], cells[k],
                           dirichlet ? dirichlet[k] : nullptr};
    }
    return create_impl(out, *prm, meshes, hip_stream);
}

int idp_step(idp_ctx *c, double *U, double dt, double *dt_used)
{
    if (!c || !U || !std::isfinite(dt)) return IDP_EINVAL;
    if (c->ninst != 1) return IDP_ENOTSUP;
    const bool async = (c->prm.flags & IDP_FLAG_ASYNC) != 0;
    double *U1 = c->U1;
    double *const Uc = U;   // the caller's array
    if (c->pos_dev) {
        permute(c, Uc, c->Uint, 1);
        U = c->Uint;
    }
    // stage 1: U1 = E(U^n), tau selected (or checked) from the stage-1 bound
    stage(c, U, U, U1, 1, 1, dt, 1, async ? 0 : 1);
    // stage 2: U2 = U^n + 1/4 (E(U1) - U^n), written over U1
    stage(c, U1, U, U1, 2, 0, 0.0, 0, 0);
    // stage 3: U^{n+1} = U^n + 2/3 (E(U2) - U^n), written over U
    stage(c, U1, U, U, 3, 0, 0.0, 0, 0);
    if (c->pos_dev) permute(c, U, Uc, 0);   // unchanged if the step refused
    if (hipGetLastError() != hipSuccess) return IDP_EHIP;
    if (async) return IDP_OK;
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    rc = status_code(h.status);
    if (rc >= 0 && dt_used) *dt_used = h.tau[0];
    return rc;
}

int idp_euler_stage(idp_ctx *c, const double *U, double tau, double *Uout)
{
    if (!c || !U || !Uout || !(tau > 0.0) || !std::isfinite(tau) || U == Uout)
        return IDP_EINVAL;
    if (c->ninst != 1) return IDP_ENOTSUP;
    if (c->pos_dev) {
        permute(c, U, c->Uint, 1);
        stage(c, c->Uint, c->Uint, c->U1, 0, 2, tau, 1, 1);
        permute(c, c->U1, Uout, 0);
    } else {
        stage(c, U, U, Uout, 0, 2, tau, 1, 1);
    }
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    return status_code(h.status);
}

}  // extern "C"

namespace {

// cfl * min_i m_i/(-2 d_ii) of every instance (host dt_out [ninst])
int max_dt_all(idp_ctx *c, const double *U, double *dt_out)
{
    const idp::StageArgs &P = c->P;
    timed(c, K_BEGIN, [&] { idp::launch_begin(P, c->stream, 1); });
    timed(c, K_NODE, [&] { idp::launch_node(P, c->stream, U, 1); });
    timed(c, K_DPAIR, [&] { idp::launch_dpair(P, c->stream, 0); });
    timed(c, K_DIAG, [&] { idp::launch_diag(P, c->stream, 0); });
    timed(c, K_TAU, [&] { idp::launch_tau_fold(P, c->stream, 1); });
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    if (h.status & idp::kErrState) return IDP_ESTATE;
    for (int k = 0; k < c->ninst; ++k) {
        double bound;
        std::memcpy(&bound, &h.taumin[k], sizeof(double));
        dt_out[k] = c->prm.cfl * bound;
    }
    return IDP_OK;
}

}  // namespace

extern "C" {

int idp_max_dt(idp_ctx *c, const double *U, double *dt_out)
{
    if (!c || !U || !dt_out) return IDP_EINVAL;
    if (c->ninst != 1) return IDP_ENOTSUP;
    if (c->pos_dev) {
        permute(c, U, c->Uint, 1);
        return max_dt_all(c, c->Uint, dt_out);
    }
    return max_dt_all(c, U, dt_out);
}

int idp_batch_max_dt(idp_ctx *c, const double *U, double *dt_out)
{
    if (!c || !U || !dt_out) return IDP_EINVAL;
    if (c->pos_dev) return IDP_ENOTSUP;   // renumbered contexts: idp_max_dt
    return max_dt_all(c, U, dt_out);
}

int idp_get_status(idp_ctx *c)
{
    if (!c) return IDP_EINVAL;
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    if (hipMemsetAsync(c->P.status, 0, sizeof(int), c->stream) != hipSuccess) return IDP_EHIP;
    rc = sync(c);
    if (rc != IDP_OK) return rc;
    return status_code(h.status);
}

int idp_info(const idp_ctx *c, int64_t *n_nodes, int64_t *nnz, size_t *device_bytes)
{
    if (!c) return IDP_EINVAL;
    if (n_nodes) *n_nodes = c->n;
    if (nnz) *nnz = c->nnz;
    if (device_bytes) *device_bytes = c->bytes;
    return IDP_OK;
}

static int sell_to_csr(idp_ctx *c, const double *dev, double *host, int stride, int comp)
{
    std::vector<double> tmp;
    try {
        tmp.resize(size_t(c->sell_size));
    } catch (const std::bad_alloc &) {
        return IDP_ENOMEM;
    }
    if (hipMemcpyAsync(tmp.data(), dev, size_t(c->sell_size) * 8, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
        return IDP_EHIP;
    int rc = sync(c);
    if (rc != IDP_OK) return rc;
    for (int64_t q = 0; q < c->nnz; ++q) host[q * stride + comp] = tmp[c->sell_of_csr[q]];
    return IDP_OK;
}

static int node_to_host(idp_ctx *c, const double *dev, int dev_stride, int off, int count,
                        double *host)
{
    std::vector<double> tmp;
    try {
        tmp.resize(size_t(c->n) * dev_stride);
    } catch (const std::bad_alloc &) {
        return IDP_ENOMEM;
    }
    if (hipMemcpyAsync(tmp.data(), dev, size_t(c->n) * dev_stride * 8, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
        return IDP_EHIP;
    int rc = sync(c);
    if (rc != IDP_OK) return rc;
    for (int64_t i = 0; i < c->n; ++i) {
        const int64_t j = c->pos.empty() ? i : c->pos[size_t(i)];
        for (int k = 0; k < count; ++k) host[i * count + k] = tmp[j * dev_stride + off + k];
    }
    return IDP_OK;
}

int idp_export_matrices(const idp_ctx *cc, int64_t *row_ptr, int32_t *col, double *m_i,
                        double *m_ij, double *c_ij)
{
    if (!cc) return IDP_EINVAL;
    idp_ctx *c = const_cast<idp_ctx *>(cc);
    if (row_ptr) std::memcpy(row_ptr, c->row_ptr.data(), (c->n + 1) * 8);
    if (col) std::memcpy(col, c->col.data(), c->nnz * 4);
    int rc = IDP_OK;
    if (m_i && (rc = node_to_host(c, c->P.mi, 1, 0, 1, m_i)) != IDP_OK) return rc;
    if (m_ij && (rc = sell_to_csr(c, c->P.mij, m_ij, 1, 0)) != IDP_OK) return rc;
    if (c_ij) {
        const int dim = c->prm.dim;
        if ((rc = sell_to_csr(c, c->P.c0, c_ij, dim, 0)) != IDP_OK) return rc;
        if ((rc = sell_to_csr(c, c->P.c1, c_ij, dim, 1)) != IDP_OK) return rc;
        if (dim == 3 && (rc = sell_to_csr(c, c->P.c2, c_ij, dim, 2)) != IDP_OK) return rc;
    }
    return IDP_OK;
}

int idp_debug_export(idp_ctx *c, int what, double *out)
{
    if (!c || !out) return IDP_EINVAL;
    const int nc = c->prm.dim + 2;
    switch (what) {
    case IDP_DBG_D: return sell_to_csr(c, c->P.d, out, 1, 0);
    case IDP_DBG_L1: return sell_to_csr(c, c->P.l1, out, 1, 0);
    case IDP_DBG_L2:
        if (c->P.passes >= 2) idp::launch_l2_fill(c->P, c->stream);
        return sell_to_csr(c, c->P.l2, out, 1, 0);
    case IDP_DBG_ALPHA: return node_to_host(c, c->P.alpha, 1, 0, 1, out);
    case IDP_DBG_TAUI: return node_to_host(c, c->P.taui, 1, 0, 1, out);
    case IDP_DBG_R: return node_to_host(c, c->P.packB, idp::kPack, nc, nc, out);
    case IDP_DBG_UL: return node_to_host(c, c->P.rowB, idp::kRowB, 0, nc, out);
    case IDP_DBG_BOUNDS: return node_to_host(c, c->P.rowB, idp::kRowB, nc, 3, out);
    case IDP_DBG_UPASS: return node_to_host(c, c->P.upass, idp::kRowU, 0, nc, out);
    case IDP_DBG_P:
    case IDP_DBG_L1RAW:
    case IDP_DBG_L2RAW: {
        // recomputed from the last stage's buffers into a temporary array
        double *tmp = nullptr;
        if (hipMalloc(&tmp, size_t(c->sell_size) * 8) != hipSuccess) {
            (void)hipGetLastError();
            return IDP_ENOMEM;
        }
        int rc = IDP_OK;
        const int kind = what == IDP_DBG_P ? 0 : what == IDP_DBG_L1RAW ? 1 : 2;
        const int ncomp = kind == 0 ? nc : 1;
        for (int q = 0; q < ncomp && rc == IDP_OK; ++q) {
            idp::launch_debug_entries(c->P, c->stream, kind, q, tmp);
            if (hipGetLastError() != hipSuccess) rc = IDP_EHIP;
            else rc = sell_to_csr(c, tmp, out, ncomp, q);
        }
        (void)hipFree(tmp);
        return rc;
    }
    default: return IDP_EINVAL;
    }
}

int idp_set_timing(idp_ctx *c, int on)
{
    if (!c) return IDP_EINVAL;
    int rc = sync(c);
    if (rc != IDP_OK) return rc;
    c->timing = on != 0;
    for (int k = 0; k < K_COUNT; ++k) {
        c->total_ms[k] = 0.0;
        c->launches[k] = 0;
    }
    return IDP_OK;
}

int idp_kernel_times(idp_ctx *c, int max, const char **names, double *total_ms,
                     int64_t *launches)
{
    if (!c) return IDP_EINVAL;
    int rc = sync(c);
    if (rc != IDP_OK) return rc;
    for (int k = 0; k < K_COUNT && k < max; ++k) {
        if (names) names[k] = kKernelNames[k];
        if (total_ms) total_ms[k] = c->total_ms[k];
        if (launches) launches[k] = c->launches[k];
    }
    return K_COUNT;
}

int idp_device_math(idp_ctx *c, int kind, int64_t n, const double *x, const double *y,
                    double *out)
{
    if (!c || !x || !out || n < 0 || kind < 0 || kind > 2 || (kind != 1 && !y))
        return IDP_EINVAL;
    if (n == 0) return IDP_OK;
    idp::launch_math(c->stream, kind, n, x, y, out);
    return sync(c);
}

}  // extern "C"

namespace {

int adj_setup(idp_ctx *c)
{
    if (c->adj_ready) return IDP_OK;
    // the stage records keep row positions in 8 bits (255: none)
    for (int64_t i = 0; i < c->n; ++i)
        if (c->row_ptr[i + 1] - c->row_ptr[i] > 254) return IDP_ENOTSUP;
    const int nc = c->prm.dim + 2;
    const int64_t n = c->n, S = c->sell_size, np = c->P.npairs;
    idp::AdjArgs &A = c->A;
    int e = IDP_OK;
#define ADJ_ALLOC(ptr, count) if ((e = dalloc(c, &(ptr), (count))) != IDP_OK) return e
    ADJ_ALLOC(c->Ebp, n * idp::kEbS);
    if (c->pos_dev) {
        ADJ_ALLOC(c->Pa, n * nc);
        ADJ_ALLOC(c->Pb, n * nc);
    }
    ADJ_ALLOC(A.Upb, n * idp::kUpS);
    ADJ_ALLOC(A.Nrec, n * idp::kNS);
    ADJ_ALLOC(A.Irec, n * idp::kIS);
    ADJ_ALLOC(A.Up4, n * nc);
    ADJ_ALLOC(A.Up6, n * nc);
    ADJ_ALLOC(A.alb, n);
    ADJ_ALLOC(A.C, S * idp::kZS);
    ADJ_ALLOC(A.lim2e, S);
    ADJ_ALLOC(A.Lim, np * idp::kLimS);
    ADJ_ALLOC(A.db4, S);
    ADJ_ALLOC(A.Qb, np * idp::kQS);
    ADJ_ALLOC(A.dLb, np);
    ADJ_ALLOC(A.ULt, n * nc);
    ADJ_ALLOC(A.Rt, n * nc);
    ADJ_ALLOC(A.bndt, n * 3);
    ADJ_ALLOC(A.alt, n);
    ADJ_ALLOC(c->Estage, n * nc);
    ADJ_ALLOC(c->U2, n * nc);
    ADJ_ALLOC(c->acc, n * nc);
    for (int k = 0; k < 3; ++k) ADJ_ALLOC(c->bar[k], n * nc);
    ADJ_ALLOC(c->sided, np);
    ADJ_ALLOC(c->side1, np);
    ADJ_ALLOC(c->side2, np);
    ADJ_ALLOC(c->argk, n);
#undef ADJ_ALLOC
    c->adj_ready = true;
    return IDP_OK;
}

int adj_check(idp_ctx *c)
{
    // the adjoint differentiates the paper's bounds (no relaxation)
    if (c->ninst != 1 || c->prm.newton_max_iter > 8 || c->prm.relax_bounds ||
        (c->prm.flags & IDP_FLAG_SPLIT_P))
        return IDP_ENOTSUP;
    return adj_setup(c);
}

// The context's stage arguments with the adjoint's records switched on.
idp::StageArgs rec_args(const idp_ctx *c)
{
    idp::StageArgs P = c->P;
    P.sided = c->sided;
    P.side1 = c->side1;
    P.side2 = c->side2;
    P.argk = c->argk;
    return P;
}

// ------------------------------------------------------------------ tape
inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

size_t tape_slot_bytes(const idp_ctx *c)
{
    const size_t S = size_t(c->sell_size), np = size_t(c->P.npairs), n = size_t(c->n);
    return 3 * al256(S * 8) + 2 * al256(np * 8) + 2 * al256(n * idp::kPack * 8) +
           al256(n * idp::kRowB * 8) + al256(n * idp::kRowU * 8) + 2 * al256(n * 8) +
           3 * al256(np) + al256(n * 4) + al256(S / 64 * 8);
}

// Room for `steps` steps (fewer if device memory is short: the largest
// count that leaves 1/16 of the free memory, and at least 1 GiB, free).
int tape_reserve(idp_ctx *c, int steps)
{
    if (c->tape_steps >= steps) return IDP_OK;
    if (c->tape_mem) {
        (void)hipFree(c->tape_mem);
        c->tape_mem = nullptr;
        c->tape_bytes = 0;
        c->tape_steps = 0;
        c->tape.clear();
        c->tape_last = false;
    }
    const size_t slot = tape_slot_bytes(c);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return IDP_EHIP;
    }
    const size_t keep = std::max<size_t>(size_t(1) << 30, fr / 16);
    const int64_t fit = fr > keep ? int64_t((fr - keep) / (3 * slot)) : 0;
    int want = int(std::min<int64_t>(steps, fit));
    void *mem = nullptr;
    while (want > 0) {
        if (hipMalloc(&mem, size_t(want) * 3 * slot) == hipSuccess) break;
        (void)hipGetLastError();
        mem = nullptr;
        want /= 2;
    }
    if (!mem) return IDP_OK;           // no tape: the backward recomputes per stage
    c->tape_mem = mem;
    c->tape_bytes = size_t(want) * 3 * slot;
    c->tape_steps = want;
    c->tape.assign(size_t(want) * 3, c->P);
    const size_t S = size_t(c->sell_size), np = size_t(c->P.npairs), n = size_t(c->n);
    for (size_t k = 0; k < c->tape.size(); ++k) {
        char *q = static_cast<char *>(mem) + k * slot;
        auto take = [&](size_t b) { char *r = q; q += al256(b); return r; };
        idp::StageArgs &P = c->tape[k];
        P.d = reinterpret_cast<double *>(take(S * 8));
        P.l1 = reinterpret_cast<double *>(take(S * 8));
        P.l2 = reinterpret_cast<double *>(take(S * 8));
        P.dp = reinterpret_cast<double *>(take(np * 8));
        P.l1p = reinterpret_cast<double *>(take(np * 8));
        P.packA = reinterpret_cast<double *>(take(n * idp::kPack * 8));
        P.packB = reinterpret_cast<double *>(take(n * idp::kPack * 8));
        P.rowB = reinterpret_cast<double *>(take(n * idp::kRowB * 8));
        P.upass = reinterpret_cast<double *>(take(n * idp::kRowU * 8));
        P.l2self = reinterpret_cast<double *>(take(n * 8));
        P.slowmask = reinterpret_cast<unsigned long long *>(take(S / 64 * 8));
        P.alpha = reinterpret_cast<double *>(take(n * 8));
        P.sided = reinterpret_cast<uint8_t *>(take(np));
        P.side1 = reinterpret_cast<uint8_t *>(take(np));
        P.side2 = reinterpret_cast<uint8_t *>(take(np));
        P.argk = reinterpret_cast<int32_t *>(take(n * 4));
    }
    return IDP_OK;
}

// One SSP-RK3 step in place on U whose three stages keep their arrays in
// tape step `slot` (the same arithmetic as idp_step with a given dt).
void tape_step(idp_ctx *c, int slot, double *U, double dt, int clear, hipStream_t st)
{
    const idp::StageArgs *T = c->tape.data() + 3 * slot;
    stage_p(c, T[0], U, U, c->U1, 1, 1, dt, 1, clear, st);
    stage_p(c, T[1], c->U1, U, c->U1, 2, 0, 0.0, 0, 0, st);
    stage_p(c, T[2], c->U1, U, U, 3, 0, 0.0, 0, 0, st);
}

void tape_step(idp_ctx *c, int slot, double *U, double dt, int clear)
{
    tape_step(c, slot, U, dt, clear, c->stream);
}

// The second stream and its events, created on first use.
int ensure_stream2(idp_ctx *c)
{
    if (c->stream2) return IDP_OK;
    if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        c->stream2 = nullptr;
        return IDP_EHIP;
    }
    for (auto &e : c->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return IDP_EHIP;
        }
    return IDP_OK;
}

// ------------------------------------------------------------- backward
// The stage VJP on the intermediates held by P.
void run_vjp(idp_ctx *c, const idp::StageArgs &P, double tau, const double *Ebp, double *Ub)
{
    idp::AdjArgs A = c->A;
    A.tau = tau;
    A.Ebp = Ebp;
    A.Ub = Ub;
    timed(c, K_VJP, [&] { idp::launch_stage_vjp(P, A, c->stream); });
}

// Recompute the stage at U (its intermediates and records), then run it
// backwards; Ebp in the padded layout.
void stage_vjp(idp_ctx *c, const double *U, double tau, const double *Ebp, double *Ub, int clear)
{
    const idp::StageArgs P = rec_args(c);
    stage_p(c, P, U, U, c->Estage, 0, 2, tau, 1, clear);
    run_vjp(c, P, tau, Ebp, Ub);
}

// One SSP-RK3 step backwards: prep(k) makes the intermediates of stage k
// (0, 1, 2) current and returns the arguments that hold them.
template <class F>
void step_vjp_core(idp_ctx *c, double dt, const double *Ubn, double *Ub, F &&prep)
{
    const int nc = c->prm.dim + 2;
    const int64_t n = c->n;
    const uint8_t *hold = c->P.hold;
    hipStream_t st = c->stream;
    // stage 3: U^{n+1} = U + 2/3 (E(U2) - U)
    idp::launch_adj_ssp(st, n, nc, hold, Ubn, 2.0 / 3.0, c->Ebp, c->acc, 1);
    run_vjp(c, prep(2), dt, c->Ebp, c->bar[1]);
    // stage 2: U2 = U + 1/4 (E(U1) - U)
    idp::launch_adj_ssp(st, n, nc, hold, c->bar[1], 0.25, c->Ebp, c->acc, 0);
    run_vjp(c, prep(1), dt, c->Ebp, c->bar[2]);
    // stage 1: U1 = E(U)
    idp::launch_adj_ssp(st, n, nc, hold, c->bar[2], 1.0, c->Ebp, c->acc, 0);
    run_vjp(c, prep(0), dt, c->Ebp, c->bar[1]);
    idp::launch_adj_add(st, n * nc, c->bar[1], c->acc);
    (void)hipMemcpyAsync(Ub, c->acc, size_t(n) * nc * 8, hipMemcpyDeviceToDevice, st);
}

// One SSP-RK3 step backwards from U, its stages recomputed one at a time.
void step_vjp(idp_ctx *c, const double *U, double dt, const double *Ubn, double *Ub, int clear)
{
    stage(c, U, U, c->U1, 1, 2, dt, 1, clear);           // U1
    stage(c, c->U1, U, c->U2, 2, 2, dt, 0, 0);           // U2
    const double *Us[3] = {U, c->U1, c->U2};
    const idp::StageArgs P = rec_args(c);
    step_vjp_core(c, dt, Ubn, Ub, [&](int k) -> const idp::StageArgs & {
        stage_p(c, P, Us[k], Us[k], c->Estage, 0, 2, dt, 1, 0);
        return P;
    });
}

// One step backwards on the intermediates of tape step `slot`.
void step_vjp_tape(idp_ctx *c, int slot, double dt, const double *Ubn, double *Ub)
{
    const idp::StageArgs *T = c->tape.data() + 3 * slot;
    step_vjp_core(c, dt, Ubn, Ub, [&](int k) -> const idp::StageArgs & { return T[k]; });
}

int finish(idp_ctx *c)
{
    if (hipGetLastError() != hipSuccess) return IDP_EHIP;
    Scalars h{};
    const int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    return status_code(h.status);
}

}  // namespace

extern "C" {

int idp_euler_stage_vjp(idp_ctx *c, const double *U, double tau, const double *Ebar,
                        double *Ubar)
{
    if (!c || !U || !Ebar || !Ubar || !(tau > 0.0) || !std::isfinite(tau) || U == Ubar ||
        Ebar == Ubar)
        return IDP_EINVAL;
    int rc = adj_check(c);
    if (rc != IDP_OK) return rc;
    if (c->pos_dev) {   // in the library's numbering, then back
        permute(c, U, c->Uint, 1);
        permute(c, Ebar, c->Pa, 1);
        idp::launch_adj_pad(c->stream, c->n, c->prm.dim + 2, c->Pa, c->Ebp);
        stage_vjp(c, c->Uint, tau, c->Ebp, c->Pb, 1);
        permute(c, c->Pb, Ubar, 0);
        return finish(c);
    }
    idp::launch_adj_pad(c->stream, c->n, c->prm.dim + 2, Ebar, c->Ebp);
    stage_vjp(c, U, tau, c->Ebp, Ubar, 1);
    return finish(c);
}

int idp_step_vjp(idp_ctx *c, const double *U, double dt, const double *Ubar_next, double *Ubar)
{
    if (!c || !U || !Ubar_next || !Ubar || !(dt > 0.0) || !std::isfinite(dt) || U == Ubar)
        return IDP_EINVAL;
    int rc = adj_check(c);
    if (rc != IDP_OK) return rc;
    if (c->pos_dev) {
        permute(c, U, c->Uint, 1);
        permute(c, Ubar_next, c->Pa, 1);
        step_vjp(c, c->Uint, dt, c->Pa, c->Pb, 1);
        permute(c, c->Pb, Ubar, 0);
        return finish(c);
    }
    step_vjp(c, U, dt, Ubar_next, Ubar, 1);
    return finish(c);
}

int idp_debug_adjoint(idp_ctx *c, int what, double *out)
{
    if (!c || !out) return IDP_EINVAL;
    if (!c->adj_ready) return IDP_EINVAL;
    const int nc = c->prm.dim + 2;
    switch (what) {
    case IDP_ADJ_UL: return node_to_host(c, c->A.ULt, nc, 0, nc, out);
    case IDP_ADJ_R: return node_to_host(c, c->A.Rt, nc, 0, nc, out);
    case IDP_ADJ_BOUNDS: return node_to_host(c, c->A.bndt, 3, 0, 3, out);
    case IDP_ADJ_ALPHA: return node_to_host(c, c->A.alt, 1, 0, 1, out);
    case IDP_ADJ_D: {
        const int64_t np = c->P.npairs;
        std::vector<double> dp(np);
        std::vector<int32_t> pe(np);
        if (hipMemcpy(dp.data(), c->A.dLb, np * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(pe.data(), c->P.pair_e, np * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return IDP_EHIP;
        // CSR position of each pair's (i, j) entry, value at (i,j); 0 elsewhere
        std::vector<int64_t> csr_of_sell(size_t(c->sell_size), -1);
        for (int64_t q = 0; q < c->nnz; ++q) csr_of_sell[c->sell_of_csr[q]] = q;
        for (int64_t q = 0; q < c->nnz; ++q) out[q] = 0.0;
        for (int64_t k = 0; k < np; ++k) out[csr_of_sell[pe[k]]] = dp[k];
        return IDP_OK;
    }
    default: return IDP_EINVAL;
    }
}

static int forward_checkpoints(idp_ctx *c, double *U, int n_steps, const double *dt, int every);

int idp_forward_checkpoints(idp_ctx *c, double *U, int n_steps, const double *dt, int every)
{
    if (!c || !U || !dt || n_steps < 1 || every < 1) return IDP_EINVAL;
    if (!c->pos_dev) return forward_checkpoints(c, U, n_steps, dt, every);
    int rc = adj_check(c);   // allocates nothing twice; the buffers below need it
    if (rc != IDP_OK) return rc;
    permute(c, U, c->Uint, 1);
    rc = forward_checkpoints(c, c->Uint, n_steps, dt, every);
    if (rc < 0) return rc;
    permute(c, c->Uint, U, 0);
    const int rc2 = finish(c);
    return rc2 < 0 ? rc2 : rc;
}

static int forward_checkpoints(idp_ctx *c, double *U, int n_steps, const double *dt, int every)
{
    if (!c || !U || !dt || n_steps < 1 || every < 1) return IDP_EINVAL;
    for (int s = 0; s < n_steps; ++s)
        if (!(dt[s] > 0.0) || !std::isfinite(dt[s])) return IDP_EINVAL;
    int rc = adj_check(c);
    if (rc != IDP_OK) return rc;
    const int nc = c->prm.dim + 2;
    const size_t state = size_t(c->n) * nc;
    const int64_t slots = (n_steps + every - 1) / every + every;   // checkpoints + a segment
    if (c->ckpt_slots < slots) {
        if ((rc = dalloc(c, &c->ckpt, slots * state)) != IDP_OK) return rc;
        c->ckpt_slots = slots;
    }
    // two banks of `every` steps if memory allows: the backward recomputes a
    // segment into one while it runs the VJPs of the other
    if ((rc = tape_reserve(c, 2 * every)) != IDP_OK) return rc;
    c->ck_steps = -1;
    c->tape_last = false;
    // the last segment runs on the tape, which the backward then starts from
    const int last0 = ((n_steps - 1) / every) * every;
    const bool keep = c->tape_steps >= n_steps - last0;
    for (int s = 0; s < n_steps; ++s) {
        if (s % every == 0)
            (void)hipMemcpyAsync(c->ckpt + (s / every) * state, U, state * 8,
                                 hipMemcpyDeviceToDevice, c->stream);
        if (keep && s >= last0) {
            tape_step(c, s - last0, U, dt[s], s == 0 ? 1 : 0);
        } else {
            stage(c, U, U, c->U1, 1, 1, dt[s], 1, s == 0 ? 1 : 0);
            stage(c, c->U1, U, c->U1, 2, 0, 0.0, 0, 0);
            stage(c, c->U1, U, U, 3, 0, 0.0, 0, 0);
        }
    }
    rc = finish(c);
    if (rc >= 0) {
        c->ck_steps = n_steps;
        c->ck_every = every;
        c->ck_dt.assign(dt, dt + n_steps);
        c->tape_last = keep;
    }
    return rc;
}

// Decision traces: see idp_trace_decisions.
static int64_t trace_stage_bytes(const idp_ctx *c)
{
    return int64_t(al256(size_t(c->P.npairs) * 8) + 2 * al256(size_t(c->n) * 4));
}

int idp_trace_decisions(idp_ctx *c, double *U, int n_steps, const double *dt,
                        void *trace_dev, int64_t trace_bytes, int64_t *stage_bytes)
{
    if (!c || n_steps < 0) return IDP_EINVAL;
    if (c->pos_dev) return IDP_ENOTSUP;
    int rc = adj_check(c);   // the stage records of the adjoint (bounds' argk)
    if (rc != IDP_OK) return rc;
    const int64_t sb = trace_stage_bytes(c);
    if (stage_bytes) *stage_bytes = sb;
    if (n_steps == 0) return IDP_OK;
    if (!U || !dt || !trace_dev || trace_bytes < sb * 3 * int64_t(n_steps)) return IDP_EINVAL;
    for (int s = 0; s < n_steps; ++s)
        if (!(dt[s] > 0.0) || !std::isfinite(dt[s])) return IDP_EINVAL;
    const idp::StageArgs P = rec_args(c);
    const size_t pb = al256(size_t(c->P.npairs) * 8), rb = al256(size_t(c->n) * 4);
    char *base = static_cast<char *>(trace_dev);
    for (int s = 0; s < n_steps; ++s)
        for (int k = 0; k < 3; ++k) {
            const double *in = k == 0 ? U : c->U1;
            double *out = k == 2 ? U : c->U1;
            stage_p(c, P, in, U, out, k + 1, k == 0 ? 1 : 0, k == 0 ? dt[s] : 0.0,
                    k == 0 ? 1 : 0, s == 0 && k == 0 ? 1 : 0);
            char *at = base + (int64_t(3 * s + k)) * sb;
            idp::launch_trace(P, c->stream, reinterpret_cast<unsigned long long *>(at),
                              reinterpret_cast<unsigned *>(at + pb));
            if (hipMemcpyAsync(at + pb + rb, c->argk, size_t(c->n) * 4, hipMemcpyDeviceToDevice,
                               c->stream) != hipSuccess)
                return IDP_EHIP;
        }
    return finish(c);
}

static int adjoint_checkpoints(idp_ctx *c, int n_steps, const double *dt, int every,
                               const double *Ubar_final, double *Ubar0);

int idp_adjoint_checkpoints(idp_ctx *c, int n_steps, const double *dt, int every,
                            const double *Ubar_final, double *Ubar0)
{
    if (!c || !dt || !Ubar_final || !Ubar0 || n_steps < 1 || every < 1) return IDP_EINVAL;
    if (!c->pos_dev) return adjoint_checkpoints(c, n_steps, dt, every, Ubar_final, Ubar0);
    if (!c->Pa) return IDP_EINVAL;   // no forward_checkpoints yet
    permute(c, Ubar_final, c->Pa, 1);
    const int rc = adjoint_checkpoints(c, n_steps, dt, every, c->Pa, c->Pb);
    if (rc < 0) return rc;
    permute(c, c->Pb, Ubar0, 0);
    const int rc2 = finish(c);
    return rc2 < 0 ? rc2 : rc;
}

static int adjoint_checkpoints(idp_ctx *c, int n_steps, const double *dt, int every,
                               const double *Ubar_final, double *Ubar0)
{
    if (!c || !dt || !Ubar_final || !Ubar0 || n_steps < 1 || every < 1) return IDP_EINVAL;
    if (n_steps != c->ck_steps || every != c->ck_every) return IDP_EINVAL;
    for (int s = 0; s < n_steps; ++s)
        if (dt[s] != c->ck_dt[s]) return IDP_EINVAL;
    const int nc = c->prm.dim + 2;
    const size_t state = size_t(c->n) * nc;
    const int nck = (n_steps + every - 1) / every;
    double *seg = c->ckpt + int64_t(nck) * state;      // `every` states of one segment
    const int T = c->tape_steps;
    // the running cotangent alternates between Ubar0 and bar[0]
    double *cur = c->bar[0], *nxt = Ubar0;
    (void)hipMemcpyAsync(cur, Ubar_final, state * 8, hipMemcpyDeviceToDevice, c->stream);
    int first = 1;
    auto back = [&](auto &&one) {
        one(cur, nxt);
        first = 0;
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    };
    if (T >= 2 * every && nck >= 2 && ensure_stream2(c) == IDP_OK) {
        // Two tape banks: segment k lives in bank (nck - 1 - k) % 2 (the
        // forward left the last one in bank 0).  While the VJPs of segment
        // k run on the context stream, the second stream recomputes segment
        // k - 1 into the other bank, after the VJPs that last read it.
        hipStream_t s2 = c->stream2;
        hipEvent_t *evR = c->ev, *evV = c->ev + 2;
        auto bank = [&](int k) { return (nck - 1 - k) & 1; };
        int first2 = 1;
        auto recompute = [&](int k) {
            const int s0 = k * every, s1 = s0 + every < n_steps ? s0 + every : n_steps;
            (void)hipMemcpyAsync(seg, c->ckpt + int64_t(k) * state, state * 8,
                                 hipMemcpyDeviceToDevice, s2);
            for (int s = s0; s < s1; ++s) {
                tape_step(c, bank(k) * every + (s - s0), seg, dt[s], first2, s2);
                first2 = 0;
            }
            (void)hipEventRecord(evR[bank(k)], s2);
        };
        (void)hipEventRecord(c->ev[4], c->stream);   // everything before this call
        (void)hipStreamWaitEvent(s2, c->ev[4], 0);
        if (c->tape_last)
            (void)hipEventRecord(evR[0], c->stream);
        else
            recompute(nck - 1);
        for (int k = nck - 1; k >= 0; --k) {
            const int b = bank(k), s0 = k * every;
            const int s1 = s0 + every < n_steps ? s0 + every : n_steps;
            (void)hipStreamWaitEvent(c->stream, evR[b], 0);
            if (k > 0) {
                if (k + 1 < nck) (void)hipStreamWaitEvent(s2, evV[1 - b], 0);
                recompute(k - 1);
            }
            for (int s = s1 - 1; s >= s0; --s)
                back([&](double *in, double *out) {
                    step_vjp_tape(c, b * every + (s - s0), dt[s], in, out);
                });
            (void)hipEventRecord(evV[b], c->stream);
        }
        c->tape_last = false;
        if (cur != Ubar0)
            (void)hipMemcpyAsync(Ubar0, cur, state * 8, hipMemcpyDeviceToDevice, c->stream);
        return finish(c);
    }
    for (int k = nck - 1; k >= 0; --k) {
        const int s0 = k * every, s1 = s0 + every < n_steps ? s0 + every : n_steps;
        if (T >= s1 - s0) {
            // the whole segment on the tape (already there for the forward's last)
            if (!(k == nck - 1 && c->tape_last)) {
                (void)hipMemcpyAsync(seg, c->ckpt + int64_t(k) * state, state * 8,
                                     hipMemcpyDeviceToDevice, c->stream);
                for (int s = s0; s < s1; ++s) {
                    tape_step(c, s - s0, seg, dt[s], first);
                    first = 0;
                }
            }
            for (int s = s1 - 1; s >= s0; --s)
                back([&](double *in, double *out) { step_vjp_tape(c, s - s0, dt[s], in, out); });
            continue;
        }
        // the segment's states, then (with a tape) blocks of T steps recomputed
        // from their first state onto the tape, else one step at a time
        (void)hipMemcpyAsync(seg, c->ckpt + int64_t(k) * state, state * 8,
                             hipMemcpyDeviceToDevice, c->stream);
        for (int s = s0; s + 1 < s1; ++s) {
            double *from = seg + int64_t(s - s0) * state, *to = from + state;
            (void)hipMemcpyAsync(to, from, state * 8, hipMemcpyDeviceToDevice, c->stream);
            stage(c, to, to, c->U1, 1, 1, dt[s], 1, first);
            stage(c, c->U1, to, c->U1, 2, 0, 0.0, 0, 0);
            stage(c, c->U1, to, to, 3, 0, 0.0, 0, 0);
            first = 0;
        }
        if (T > 0) {
            for (int b1 = s1; b1 > s0;) {
                const int b0 = b1 - T > s0 ? b1 - T : s0;
                (void)hipMemcpyAsync(c->U2, seg + int64_t(b0 - s0) * state, state * 8,
                                     hipMemcpyDeviceToDevice, c->stream);
                for (int s = b0; s < b1; ++s) {
                    tape_step(c, s - b0, c->U2, dt[s], first);
                    first = 0;
                }
                for (int s = b1 - 1; s >= b0; --s)
                    back([&](double *in, double *out) {
                        step_vjp_tape(c, s - b0, dt[s], in, out);
                    });
                b1 = b0;
            }
        } else {
            for (int s = s1 - 1; s >= s0; --s)
                back([&](double *in, double *out) {
                    step_vjp(c, seg + int64_t(s - s0) * state, dt[s], in, out, first);
                });
        }
    }
    c->tape_last = false;
    if (cur != Ubar0)
        (void)hipMemcpyAsync(Ubar0, cur, state * 8, hipMemcpyDeviceToDevice, c->stream);
    return finish(c);
}

int idp_batch_info(const idp_ctx *c, int *n_inst, int64_t *node_offsets)
{
    if (!c) return IDP_EINVAL;
    if (n_inst) *n_inst = c->ninst;
    if (node_offsets)
        for (int k = 0; k <= c->ninst; ++k) node_offsets[k] = c->lay.node[k];
    return IDP_OK;
}

}  // extern "C"

namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Work-item tables of the persistent schedule with `tile` units per item;
// tile < 0: every instance's sweep in (at most) -tile items, so that large
// instances take coarse items and small ones fine items.
int persist_tables(idp_ctx *c, int tile, PersistTables **out)
{
    for (auto &t : c->tables)
        if (t.tile == tile) { *out = &t; return IDP_OK; }
    const int K = c->ninst;
    const auto &L = c->lay;
    int e = IDP_OK;
    if (!c->done) {
        if ((e = dalloc(c, &c->done, K)) != IDP_OK) return e;
        if ((e = dalloc(c, &c->head, 1)) != IDP_OK) return e;
        if ((e = dalloc(c, &c->taumin2, 2 * size_t(K))) != IDP_OK) return e;
        if ((e = dalloc(c, &c->unit_end, 3 * size_t(K))) != IDP_OK) return e;
        std::vector<int64_t> ue(3 * size_t(K));
        for (int k = 0; k < K; ++k) {
            ue[3 * k + 0] = L.node[k + 1];
            ue[3 * k + 1] = L.pair[k + 1];
            ue[3 * k + 2] = L.slice[k + 1];
        }
        if (hipMemcpy(c->unit_end, ue.data(), ue.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
            return IDP_EHIP;
    }
    // sweep kinds: 0 nodes, 1 pairs, 2 slices; the unit of work of one
    // wavefront: 64 nodes, 64 pairs, 1 slice
    const int kind[idp::kSweeps] = {0, 1, 2, 2, 1, 2, 1, 2};
    const int64_t unit[3] = {idp::kSlice, idp::kSlice, 1};
    constexpr int S1 = idp::kSweeps + 1;
    std::vector<int64_t> items(size_t(K) * idp::kSweeps), pre(size_t(K) * S1);
    std::vector<int64_t> tiles(size_t(K) * idp::kSweeps);
    idp::BatchArgs B{};
    B.tile = tile;
    for (int s = 0; s < idp::kSweeps; ++s) {
        B.sweep_off[s + 1] = B.sweep_off[s];
        for (int k = 0; k < K; ++k) {
            const int64_t *range = kind[s] == 0 ? L.node.data() : kind[s] == 1 ? L.pair.data()
                                                                              : L.slice.data();
            const int64_t units = cdiv(range[k + 1] - range[k], unit[kind[s]]);
            int64_t t = tile;
            if (tile < 0) {
                const int64_t want = std::min<int64_t>(units, -tile);
                t = want > 0 ? cdiv(units, want) : 1;
            }
            int64_t n = cdiv(units, t);
            if (s == 6 && c->prm.limiter_passes < 2) n = 0;
            items[size_t(k) * idp::kSweeps + s] = n;
            tiles[size_t(k) * idp::kSweeps + s] = t;
            B.sweep_off[s + 1] += n;
        }
    }
    for (int k = 0; k < K; ++k) {
        int64_t acc = 0;
        for (int s = 0; s < idp::kSweeps; ++s) {
            pre[size_t(k) * S1 + s] = acc + (s >= 3 ? 1 : 0);   // + the tau update
            acc += items[size_t(k) * idp::kSweeps + s];
        }
        pre[size_t(k) * S1 + idp::kSweeps] = acc + 1;
    }
    B.items_per_stage = B.sweep_off[idp::kSweeps];
    std::vector<int32_t> inst(B.items_per_stage), ntile(B.items_per_stage);
    std::vector<int64_t> first(B.items_per_stage);
    int64_t q = 0;
    for (int s = 0; s < idp::kSweeps; ++s)
        for (int k = 0; k < K; ++k) {
            const int64_t *range = kind[s] == 0 ? L.node.data() : kind[s] == 1 ? L.pair.data()
                                                                              : L.slice.data();
            const int64_t t = tiles[size_t(k) * idp::kSweeps + s];
            for (int64_t it = 0; it < items[size_t(k) * idp::kSweeps + s]; ++it, ++q) {
                inst[q] = k;
                ntile[q] = int32_t(t);
                first[q] = range[k] + it * t * unit[kind[s]];
            }
        }
    PersistTables T;
    T.tile = tile;
    if ((e = dalloc(c, &T.item_inst, inst.size())) != IDP_OK) return e;
    if ((e = dalloc(c, &T.item_tile, ntile.size())) != IDP_OK) return e;
    if ((e = dalloc(c, &T.item_first, first.size())) != IDP_OK) return e;
    if ((e = dalloc(c, &T.pre, pre.size())) != IDP_OK) return e;
    if (hipMemcpy(T.item_inst, inst.data(), inst.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(T.item_tile, ntile.data(), ntile.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(T.item_first, first.data(), first.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(T.pre, pre.data(), pre.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return IDP_EHIP;
    B.item_inst = T.item_inst;
    B.item_tile = T.item_tile;
    B.item_first = T.item_first;
    B.pre = T.pre;
    B.unit_end = c->unit_end;
    B.taumin2 = c->taumin2;
    B.done = c->done;
    B.head = c->head;
    T.B = B;
    c->tables.push_back(T);
    *out = &c->tables.back();
    return IDP_OK;
}

int batch_steps(idp_ctx *c, double *U, int n_steps, const double *dt, double *dt_used,
                const idp_schedule &sc)
{
    const int K = c->ninst;
    idp::StageArgs &P = c->P;
    int e = IDP_OK;
    if (dt) {
        for (int k = 0; k < K; ++k)
            if (!(dt[k] > 0.0) || !std::isfinite(dt[k])) return IDP_EINVAL;
        if (!c->dt_dev && (e = dalloc(c, &c->dt_dev, K)) != IDP_OK) return e;
        if (hipMemcpyAsync(c->dt_dev, dt, size_t(K) * 8, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess)
            return IDP_EHIP;
    }
    const int64_t need = int64_t(n_steps) * K;
    if (c->dt_rec_cap < need) {
        if ((e = dalloc(c, &c->dt_rec, need)) != IDP_OK) return e;
        c->dt_rec_cap = need;
    }
    P.dt_inst = dt ? c->dt_dev : nullptr;
    if (sc.kind == IDP_SCHED_LAUNCHES) {
        for (int st = 0; st < n_steps; ++st) {
            stage(c, U, U, c->U1, 1, 1, 0.0, 1, st == 0 ? 1 : 0);
            (void)hipMemcpyAsync(c->dt_rec + int64_t(st) * K, P.tau, size_t(K) * 8,
                                 hipMemcpyDeviceToDevice, c->stream);
            stage(c, c->U1, U, c->U1, 2, 0, 0.0, 0, 0);
            stage(c, c->U1, U, U, 3, 0, 0.0, 0, 0);
        }
    } else {
        PersistTables *T = nullptr;
        if ((e = persist_tables(c, sc.tile, &T)) != IDP_OK) { P.dt_inst = nullptr; return e; }
        idp::BatchArgs B = T->B;
        B.nsteps = n_steps;
        B.check = 1;
        B.total_items = B.items_per_stage * 3 * n_steps;
        B.U = U;
        B.U1 = c->U1;
        B.dt_rec = c->dt_rec;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess) { P.dt_inst = nullptr; return IDP_EHIP; }
        const int grid = idp::persistent_blocks_per_cu(P.dim) * cus;
        idp::launch_batch_init(P, B, c->stream, 1);
        idp::StageArgs Pw = P;
        Pw.slow = nullptr;   // the persistent worker sweeps every pass-2 pair
        timed(c, K_PERSIST, [&] { idp::launch_persistent(Pw, B, c->stream, grid); });
    }
    P.dt_inst = nullptr;
    if (hipGetLastError() != hipSuccess) return IDP_EHIP;
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    rc = status_code(h.status);
    if (rc >= 0 && dt_used) {
        if (hipMemcpy(dt_used, c->dt_rec, size_t(need) * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return IDP_EHIP;
    }
    return rc;
}

bool valid_schedule(const idp_schedule &s)
{
    if (s.kind == IDP_SCHED_LAUNCHES) return true;
    return s.kind == IDP_SCHED_PERSISTENT &&
           ((s.tile >= 1 && s.tile <= 1024) || (s.tile >= -256 && s.tile <= -1));
}

}  // namespace

extern "C" {

int idp_batch_steps(idp_ctx *c, double *U, int n_steps, const double *dt, double *dt_used,
                    const idp_schedule *sched)
{
    if (!c || !U || n_steps < 0) return IDP_EINVAL;
    if (c->pos_dev) return IDP_ENOTSUP;   // renumbered contexts: idp_step
    const idp_schedule sc = sched ? *sched : c->tuned;
    if (!valid_schedule(sc)) return IDP_EINVAL;
    if (n_steps == 0) return IDP_OK;
    return batch_steps(c, U, n_steps, dt, dt_used, sc);
}

int idp_batch_tune(idp_ctx *c, const double *U, int n_steps, idp_schedule *best,
                   double *ms_out, int *n_candidates)
{
    if (!c || !U || n_steps < 1) return IDP_EINVAL;
    if (c->pos_dev) return IDP_ENOTSUP;
    // fixed tiles, and tiles per instance size (every sweep of an instance
    // in at most 8, 32 or 128 items)
    const idp_schedule cand[] = {{IDP_SCHED_LAUNCHES, 0},    {IDP_SCHED_PERSISTENT, 4},
                                 {IDP_SCHED_PERSISTENT, 16},  {IDP_SCHED_PERSISTENT, 32},
                                 {IDP_SCHED_PERSISTENT, 64},  {IDP_SCHED_PERSISTENT, 128},
                                 {IDP_SCHED_PERSISTENT, 256}, {IDP_SCHED_PERSISTENT, -8},
                                 {IDP_SCHED_PERSISTENT, -32}, {IDP_SCHED_PERSISTENT, -128}};
    const int nc = int(sizeof(cand) / sizeof(cand[0]));
    const size_t bytes = size_t(c->n) * (c->prm.dim + 2) * 8;
    int e = IDP_OK;
    if (!c->U_tune && (e = dalloc(c, &c->U_tune, size_t(c->n) * (c->prm.dim + 2))) != IDP_OK)
        return e;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return IDP_EHIP;
    }
    int bi = -1;
    double bms = 0.0;
    for (int q = 0; q < nc; ++q) {
        double ms = -1.0;   // failed candidate
        int rc = hipMemcpyAsync(c->U_tune, U, bytes, hipMemcpyDeviceToDevice, c->stream) ==
                         hipSuccess ? batch_steps(c, c->U_tune, 1, nullptr, nullptr, cand[q])
                                    : IDP_EHIP;                             // warm-up
        if (rc >= 0 &&
            hipMemcpyAsync(c->U_tune, U, bytes, hipMemcpyDeviceToDevice, c->stream) == hipSuccess &&
            hipEventRecord(a, c->stream) == hipSuccess) {
            rc = batch_steps(c, c->U_tune, n_steps, nullptr, nullptr, cand[q]);
            float f = 0.f;
            if (rc >= 0 && hipEventRecord(b, c->stream) == hipSuccess &&
                hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&f, a, b) == hipSuccess)
                ms = f;
        }
        (void)hipGetLastError();
        if (ms_out) ms_out[q] = ms;
        if (ms >= 0.0 && (bi < 0 || ms < bms)) { bi = q; bms = ms; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (n_candidates) *n_candidates = nc;
    if (bi < 0) return IDP_EHIP;
    c->tuned = cand[bi];
    if (best) *best = cand[bi];
    return IDP_OK;
}

}  // extern "C"

// ------------------------------------------ the batch step that allocates nothing
// Per device, one static array holds what idp_batch_steps keeps in buffers
// it allocates on demand: the status word, per instance the tau minimum,
// tau, the bound and the given dt, and the tau record of every step.  Host
// code never uses the array's name as an address: the device address of
// this device's copy is looked up once (hipGetSymbolAddress, with the
// device current) and kept in g_scratch_ptr.
namespace {
constexpr size_t kNoAllocBytes = size_t(1) << 20;
constexpr int kNoAllocDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
char *g_scratch_ptr[kNoAllocDevices] = {};

int scratch_address(int device, char **out)
{
    if (device < 0 || device >= kNoAllocDevices) return IDP_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return IDP_EHIP;
        }
        g_scratch_ptr[device] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[device];
    return IDP_OK;
}

}  // namespace

extern "C" {

int idp_batch_steps_noalloc(idp_ctx *c, double *U, int n_steps, const double *dt,
                            double *dt_used)
{
    if (!c || !U || n_steps < 0) return IDP_EINVAL;
    if (c->pos_dev) return IDP_ENOTSUP;   // as idp_batch_steps
    if (n_steps == 0) return IDP_OK;
    const int K = c->ninst;
    // layout: [status, 16 B] [tau minimum bits | tau | bound | dt] x K [record n_steps x K]
    const size_t head = kScalHead + size_t(K) * 32;
    if (size_t(n_steps) > (kNoAllocBytes - std::min(head, kNoAllocBytes)) / 8 / size_t(K) ||
        head > kNoAllocBytes)
        return IDP_ESCRATCH;
    if (dt)
        for (int k = 0; k < K; ++k)
            if (!(dt[k] > 0.0) || !std::isfinite(dt[k])) return IDP_EINVAL;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return IDP_EHIP;
    if (cur != c->device) return IDP_EINVAL;   // the context's device must be current
    char *base = nullptr;
    int rc = scratch_address(c->device, &base);
    if (rc != IDP_OK) return rc;
    idp::StageArgs P = c->P;
    P.status = reinterpret_cast<int *>(base);
    P.taumin = reinterpret_cast<unsigned long long *>(base + kScalHead);
    P.tau = reinterpret_cast<double *>(base + kScalHead + size_t(K) * 8);
    P.bound = reinterpret_cast<double *>(base + kScalHead + size_t(K) * 16);
    double *dt_dev = reinterpret_cast<double *>(base + kScalHead + size_t(K) * 24);
    double *rec = reinterpret_cast<double *>(base + head);
    if (dt && hipMemcpyAsync(dt_dev, dt, size_t(K) * 8, hipMemcpyHostToDevice, c->stream) !=
                  hipSuccess)
        return IDP_EHIP;
    P.dt_inst = dt ? dt_dev : nullptr;
    // no event timing here (it may create events)
    const bool timing = c->timing;
    c->timing = false;
    for (int st = 0; st < n_steps; ++st) {
        // the first stage clears the status word and every stage the tau
        // minima (kernels, so the call needs no memset)
        stage_p(c, P, U, U, c->U1, 1, 1, 0.0, 1, st == 0 ? 1 : 0);
        (void)hipMemcpyAsync(rec + int64_t(st) * K, P.tau, size_t(K) * 8,
                             hipMemcpyDeviceToDevice, c->stream);
        stage_p(c, P, c->U1, U, c->U1, 2, 0, 0.0, 0, 0);
        stage_p(c, P, c->U1, U, U, 3, 0, 0.0, 0, 0);
    }
    c->timing = timing;
    if (hipGetLastError() != hipSuccess) return IDP_EHIP;
    int status = 0;
    if (hipMemcpyAsync(&status, P.status, sizeof(int), hipMemcpyDeviceToHost, c->stream) !=
        hipSuccess)
        return IDP_EHIP;
    if ((rc = sync(c)) != IDP_OK) return rc;
    rc = status_code(status);
    if (rc >= 0 && dt_used) {
        if (hipMemcpyAsync(dt_used, rec, size_t(n_steps) * K * 8, hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess)
            return IDP_EHIP;
        const int rs = sync(c);
        if (rs != IDP_OK) return rs;
    }
    return rc;
}

const char *idp_strerror(int code)
{
    switch (code) {
    case IDP_OK: return "success";
    case IDP_WARN_CFL: return "warning: tau exceeded the stage-2/3 stability bound";
    case IDP_EINVAL: return "invalid argument";
    case IDP_EMESH: return "invalid mesh: det J <= 0 at a quadrature point";
    case IDP_ENOMEM: return "out of memory";
    case IDP_EHIP: return "HIP runtime error";
    case IDP_ESTATE: return "input state not admissible (rho <= 0, internal energy <= 0 or NaN)";
    case IDP_EDT: return "dt exceeds the stage-1 bound min_i m_i/(-2 d_ii)";
    case IDP_ENOTSUP: return "option not supported";
    case IDP_EWAIT: return "a persistent batch launch gave up waiting on a dependency";
    case IDP_ESCRATCH: return "the call needs more than the static scratch of idp_batch_steps_noalloc";
    default: return "unknown error";
    }
}

}  // extern "C"
