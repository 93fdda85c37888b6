// C-ABI of the library: context, precompute, SSP-RK3 stepper, exports.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/idp.h"
#include "graph.h"
#include "kernels.h"

static_assert(idp::kSellC == idp::kSlice, "SELL slice height = wavefront width");

namespace {

enum KernelId {
    K_BEGIN, K_NODE, K_DPAIR, K_DIAG, K_TAU, K_LOW, K_LIM1P, K_PASS1A, K_LIM2P, K_PASS2,
    K_COUNT
};
const char *kKernelNames[K_COUNT] = {"begin", "node_pack", "pair_viscosity", "row_diagonal",
                                     "tau", "row_low_order", "pair_limiter1", "row_pass1",
                                     "pair_limiter2", "row_pass2"};

struct Pending {
    int id;
    hipEvent_t a, b;
};

struct Scalars {        // device-side scalars, copied back in one transfer
    unsigned long long taumin;
    double tau;
    double bound;
    int status;
    int pad;
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
    Scalars *scal = nullptr;
    double *U1 = nullptr;
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
void timed(idp_ctx *c, int id, F &&launch)
{
    if (!c->timing) {
        launch();
        return;
    }
    Pending p{id, get_event(c), get_event(c)};
    if (p.a) (void)hipEventRecord(p.a, c->stream);
    launch();
    if (p.b) (void)hipEventRecord(p.b, c->stream);
    c->pending.push_back(p);
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
    if (hipMemcpyAsync(h, c->scal, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream) !=
        hipSuccess)
        return IDP_EHIP;
    return sync(c);
}

int status_code(int st)
{
    if (st & idp::kErrState) return IDP_ESTATE;
    if (st & idp::kErrDt) return IDP_EDT;
    if (st & idp::kWarnCfl) return IDP_WARN_CFL;
    return IDP_OK;
}

// One forward-Euler stage on the context stream.
//  in: stage input state; U0: step-initial state; out: destination;
//  tau_mode: 1 select tau (stage 1), 0 check the held tau, 2 use dt_in.
void stage(idp_ctx *c, const double *in, const double *U0, double *out, int mode,
           int tau_mode, double dt_in, int check, int clear)
{
    const idp::StageArgs &P = c->P;
    hipStream_t st = c->stream;
    timed(c, K_BEGIN, [&] { idp::launch_begin(P, st, clear); });
    timed(c, K_NODE, [&] { idp::launch_node(P, st, in, check); });
    timed(c, K_DPAIR, [&] { idp::launch_dpair(P, st); });
    timed(c, K_DIAG, [&] { idp::launch_diag(P, st, 1); });
    timed(c, K_TAU, [&] { idp::launch_tau(P, st, dt_in, tau_mode); });
    timed(c, K_LOW, [&] { idp::launch_low(P, st); });
    timed(c, K_LIM1P, [&] { idp::launch_lim1p(P, st); });
    timed(c, K_PASS1A, [&] { idp::launch_pass1a(P, st); });
    if (P.passes >= 2) timed(c, K_LIM2P, [&] { idp::launch_lim2p(P, st); });
    timed(c, K_PASS2, [&] { idp::launch_pass2(P, st, U0, out, mode); });
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
    for (void *q : c->allocs) (void)hipFree(q);
    delete c;
}

int idp_create(idp_ctx **out, const idp_params *prm, int64_t n_nodes,
               const double *coords, int64_t n_cells, const int64_t *cells,
               const uint8_t *dirichlet, void *hip_stream)
{
    if (!out || !prm || !coords || !cells) return IDP_EINVAL;
    *out = nullptr;
    const idp_params p = *prm;
    if ((p.dim != 2 && p.dim != 3) || !(p.gamma > 1.0) || !(p.cfl > 0.0) ||
        !(p.cfl <= 1.0) || (p.limiter_passes != 1 && p.limiter_passes != 2) ||
        p.newton_max_iter < 0 || p.newton_max_iter > 64 || !(p.newton_tol >= 0.0))
        return IDP_EINVAL;
    if (p.relax_bounds) return IDP_ENOTSUP;
    idp_ctx *c = new (std::nothrow) idp_ctx;
    if (!c) return IDP_ENOMEM;
    c->prm = p;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return IDP_EHIP; }

    idp::HostGraph g;
    int rc = idp::build_graph(g, p.dim, n_nodes, n_cells, cells);
    if (rc != IDP_OK) { delete c; return rc; }
    c->n = g.n;
    c->nnz = g.nnz;
    c->sell_size = g.sell_size;
    const int64_t nrows = g.nslices * idp::kSlice;
    const int dim = p.dim;
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
    TRY(dalloc(c, &P.packB, g.n * idp::kPack));
    TRY(dalloc(c, &P.rowB, g.n * idp::kRowB));
    TRY(dalloc(c, &P.upass, g.n * idp::kRowU));
    TRY(dalloc(c, &P.alpha, g.n));
    TRY(dalloc(c, &P.taui, g.n));
    TRY(dalloc(c, &c->U1, g.n * (dim + 2)));
    TRY(dalloc(c, &c->scal, 1));
    uint8_t *hold = nullptr;
    if (dirichlet) {
        TRY(dalloc(c, &hold, g.n));
        HIPTRY(hipMemcpyAsync(hold, dirichlet, g.n, hipMemcpyHostToDevice, c->stream));
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
    P.taumin = &c->scal->taumin;
    P.tau = &c->scal->tau;
    P.bound = &c->scal->bound;
    P.status = &c->scal->status;
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
    HIPTRY(hipMemsetAsync(c->scal, 0, sizeof(Scalars), c->stream));

    // matrices on the device (temporary mesh arrays)
    {
        const int nv = 1 << dim;
        std::vector<int32_t> cells32;
        try {
            cells32.resize(size_t(n_cells) * nv);
        } catch (const std::bad_alloc &) {
            idp_destroy(c);
            return IDP_ENOMEM;
        }
        for (int64_t t = 0; t < n_cells * nv; ++t) cells32[t] = int32_t(cells[t]);
        double *dco = nullptr, *dummy = nullptr;
        int32_t *dcells = nullptr, *dnl = nullptr;
        int64_t *dncp = nullptr;
        int *derr = nullptr;
        bool ok = hipMalloc(&dco, size_t(g.n) * dim * 8) == hipSuccess &&
                  hipMalloc(&dcells, cells32.size() * 4) == hipSuccess &&
                  hipMalloc(&dncp, g.nc_ptr.size() * 8) == hipSuccess &&
                  hipMalloc(&dnl, g.nc_list.size() * 4) == hipSuccess &&
                  hipMalloc(&derr, sizeof(int)) == hipSuccess;
        (void)dummy;
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
    // keep what the CSR exports need, drop the rest of the host graph
    c->row_ptr.swap(g.row_ptr);
    c->col.swap(g.col);
    c->sell_of_csr.swap(g.sell_of_csr);
#undef TRY
#undef HIPTRY
    *out = c;
    return IDP_OK;
}

int idp_step(idp_ctx *c, double *U, double dt, double *dt_used)
{
    if (!c || !U || !std::isfinite(dt)) return IDP_EINVAL;
    const bool async = (c->prm.flags & IDP_FLAG_ASYNC) != 0;
    double *U1 = c->U1;
    // stage 1: U1 = E(U^n), tau selected (or checked) from the stage-1 bound
    stage(c, U, U, U1, 1, 1, dt, 1, async ? 0 : 1);
    // stage 2: U2 = U^n + 1/4 (E(U1) - U^n), written over U1
    stage(c, U1, U, U1, 2, 0, 0.0, 0, 0);
    // stage 3: U^{n+1} = U^n + 2/3 (E(U2) - U^n), written over U
    stage(c, U1, U, U, 3, 0, 0.0, 0, 0);
    if (hipGetLastError() != hipSuccess) return IDP_EHIP;
    if (async) return IDP_OK;
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    rc = status_code(h.status);
    if (rc >= 0 && dt_used) *dt_used = h.tau;
    return rc;
}

int idp_euler_stage(idp_ctx *c, const double *U, double tau, double *Uout)
{
    if (!c || !U || !Uout || !(tau > 0.0) || !std::isfinite(tau) || U == Uout)
        return IDP_EINVAL;
    stage(c, U, U, Uout, 0, 2, tau, 1, 1);
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    return status_code(h.status);
}

int idp_max_dt(idp_ctx *c, const double *U, double *dt_out)
{
    if (!c || !U || !dt_out) return IDP_EINVAL;
    const idp::StageArgs &P = c->P;
    timed(c, K_BEGIN, [&] { idp::launch_begin(P, c->stream, 1); });
    timed(c, K_NODE, [&] { idp::launch_node(P, c->stream, U, 1); });
    timed(c, K_DPAIR, [&] { idp::launch_dpair(P, c->stream); });
    timed(c, K_DIAG, [&] { idp::launch_diag(P, c->stream, 0); });
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    if (h.status & idp::kErrState) return IDP_ESTATE;
    double bound;
    std::memcpy(&bound, &h.taumin, sizeof(double));
    *dt_out = c->prm.cfl * bound;
    return IDP_OK;
}

int idp_get_status(idp_ctx *c)
{
    if (!c) return IDP_EINVAL;
    Scalars h{};
    int rc = read_scalars(c, &h);
    if (rc != IDP_OK) return rc;
    if (hipMemsetAsync(&c->scal->status, 0, sizeof(int), c->stream) != hipSuccess) return IDP_EHIP;
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
    for (int64_t i = 0; i < c->n; ++i)
        for (int k = 0; k < count; ++k) host[i * count + k] = tmp[i * dev_stride + off + k];
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
    case IDP_DBG_L2: return sell_to_csr(c, c->P.l2, out, 1, 0);
    case IDP_DBG_ALPHA: return node_to_host(c, c->P.alpha, 1, 0, 1, out);
    case IDP_DBG_TAUI: return node_to_host(c, c->P.taui, 1, 0, 1, out);
    case IDP_DBG_R: return node_to_host(c, c->P.packB, idp::kPack, nc, nc, out);
    case IDP_DBG_UL: return node_to_host(c, c->P.rowB, idp::kRowB, 0, nc, out);
    case IDP_DBG_BOUNDS: return node_to_host(c, c->P.rowB, idp::kRowB, nc, 3, out);
    case IDP_DBG_UPASS: return node_to_host(c, c->P.upass, idp::kRowU, 0, nc, out);
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
    default: return "unknown error";
    }
}

}  // extern "C"
