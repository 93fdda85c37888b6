// Host-side construction of the stencil graph and the SELL-64 layout.
#include "graph.h"

#include <algorithm>
#include <new>

#include "../../include/idp.h"

namespace idp {

static int build(HostGraph &g, int dim, int64_t n, int64_t ncells,
                 const int64_t *cells, int sigma, const int32_t *key)
{
    // column order within a row: ascending key (the node id by default)
    auto before = [key](int32_t a, int32_t b) { return key ? key[a] < key[b] : a < b; };
    const int nv = 1 << dim;
    g.dim = dim;
    g.nv = nv;
    g.n = n;
    g.ncells = ncells;
    if (n <= 0 || ncells <= 0 || n >= (int64_t(1) << 31) ||
        ncells * nv >= (int64_t(1) << 31))
        return IDP_EINVAL;
    const int64_t inc = ncells * nv;
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int64_t t = 0; t < inc; ++t)
        if (cells[t] < 0 || cells[t] >= n) bad = 1;
    if (bad) return IDP_EINVAL;

    // node -> cells (ascending cell id): counting sort of the incidences
    g.nc_ptr.assign(n + 1, 0);
    for (int64_t t = 0; t < inc; ++t) g.nc_ptr[cells[t] + 1]++;
    for (int64_t i = 0; i < n; ++i) g.nc_ptr[i + 1] += g.nc_ptr[i];
    g.nc_list.resize(inc);
    {
        std::vector<int64_t> fill(g.nc_ptr.begin(), g.nc_ptr.end() - 1);
        for (int64_t c = 0; c < ncells; ++c)
            for (int b = 0; b < nv; ++b)
                g.nc_list[fill[cells[c * nv + b]]++] = int32_t(c);
    }

    // rows: sorted unique vertices of the cells around each node
    g.row_ptr.assign(n + 1, 0);
    int maxlen = 0;
#pragma omp parallel reduction(max : maxlen)
    {
        std::vector<int32_t> cand;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            cand.clear();
            for (int64_t q = g.nc_ptr[i]; q < g.nc_ptr[i + 1]; ++q) {
                const int64_t c = g.nc_list[q];
                for (int b = 0; b < nv; ++b) cand.push_back(int32_t(cells[c * nv + b]));
            }
            std::sort(cand.begin(), cand.end(), before);
            const int len = int(std::unique(cand.begin(), cand.end()) - cand.begin());
            g.row_ptr[i + 1] = len;
            maxlen = std::max(maxlen, len);
        }
    }
    for (int64_t i = 0; i < n; ++i) g.row_ptr[i + 1] += g.row_ptr[i];
    g.nnz = g.row_ptr[n];
    g.max_len = maxlen;
    g.col.resize(g.nnz);
#pragma omp parallel
    {
        std::vector<int32_t> cand;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            cand.clear();
            for (int64_t q = g.nc_ptr[i]; q < g.nc_ptr[i + 1]; ++q) {
                const int64_t c = g.nc_list[q];
                for (int b = 0; b < nv; ++b) cand.push_back(int32_t(cells[c * nv + b]));
            }
            std::sort(cand.begin(), cand.end(), before);
            auto end = std::unique(cand.begin(), cand.end());
            std::copy(cand.begin(), end, g.col.begin() + g.row_ptr[i]);
        }
    }
    // transposed positions: the stencil relation is symmetric
    g.tpos.resize(g.nnz);
    bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = g.row_ptr[i]; q < g.row_ptr[i + 1]; ++q) {
            const int32_t j = g.col[q];
            auto b = g.col.begin() + g.row_ptr[j], e = g.col.begin() + g.row_ptr[j + 1];
            auto it = std::lower_bound(b, e, int32_t(i), before);
            if (it == e || *it != i) { bad = 1; continue; }
            g.tpos[q] = it - g.col.begin();
        }
    if (bad) return IDP_EINVAL;

    // SELL-64: rows by length, longest first, stable in node id, within
    // windows of sigma rows (all rows if sigma = 0)
    g.nslices = (n + kSellC - 1) / kSellC;
    const int64_t nrows = g.nslices * kSellC;
    g.perm.assign(nrows, -1);
    g.row_len.assign(nrows, 0);
    g.diag_k.assign(nrows, 0);
    {
        const int64_t win = sigma > 0 ? int64_t(sigma) : (n > 0 ? n : 1);
        std::vector<int64_t> cnt(maxlen + 2), start(maxlen + 2);
        for (int64_t w0 = 0; w0 < n; w0 += win) {
            const int64_t w1 = w0 + win < n ? w0 + win : n;
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int64_t i = w0; i < w1; ++i) cnt[g.row_ptr[i + 1] - g.row_ptr[i]]++;
            int64_t acc = w0;
            for (int L = maxlen; L >= 0; --L) { start[L] = acc; acc += cnt[L]; }
            for (int64_t i = w0; i < w1; ++i) {
                const int L = int(g.row_ptr[i + 1] - g.row_ptr[i]);
                const int64_t r = start[L]++;
                g.perm[r] = int32_t(i);
                g.row_len[r] = L;
            }
        }
    }
    g.slice_w.resize(g.nslices);
    g.slice_off.resize(g.nslices);
    int64_t off = 0;
    for (int64_t s = 0; s < g.nslices; ++s) {
        g.slice_w[s] = g.row_len[s * kSellC];
        g.slice_off[s] = off;
        off += int64_t(g.slice_w[s]) * kSellC;
    }
    g.sell_size = off;
    if (g.sell_size >= (int64_t(1) << 31)) return IDP_EINVAL;
    g.sell_of_csr.resize(g.nnz);
    g.scol.resize(g.sell_size);
    g.stpos.resize(g.sell_size);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t s = r / kSellC, lane = r % kSellC;
        const int32_t i = g.perm[r];
        for (int k = 0; k < g.slice_w[s]; ++k) {
            const int64_t e = g.slice_off[s] + int64_t(k) * kSellC + lane;
            if (i >= 0 && k < g.row_len[r]) {
                const int64_t q = g.row_ptr[i] + k;
                g.sell_of_csr[q] = e;
                g.scol[e] = g.col[q];
                if (g.col[q] == i) g.diag_k[r] = k;
            } else {
                g.scol[e] = i >= 0 ? i : 0;  // padding: a valid node id
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t s = r / kSellC, lane = r % kSellC;
        const int32_t i = g.perm[r];
        for (int k = 0; k < g.slice_w[s]; ++k) {
            const int64_t e = g.slice_off[s] + int64_t(k) * kSellC + lane;
            if (i >= 0 && k < g.row_len[r])
                g.stpos[e] = int32_t(g.sell_of_csr[g.tpos[g.row_ptr[i] + k]]);
            else
                g.stpos[e] = int32_t(e);
        }
    }
    // pairs: the entries (i, j) with j after i in the column order (j > i,
    // or key[j] > key[i]), slice by slice in SELL order
    {
        std::vector<int64_t> cnt(g.nslices + 1, 0);
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < g.nslices; ++s) {
            int64_t c = 0;
            for (int k = 0; k < g.slice_w[s]; ++k)
                for (int lane = 0; lane < kSellC; ++lane) {
                    const int64_t r = s * kSellC + lane;
                    const int32_t i = g.perm[r];
                    if (i < 0 || k >= g.row_len[r]) continue;
                    if (before(i, g.scol[g.slice_off[s] + int64_t(k) * kSellC + lane])) ++c;
                }
            cnt[s + 1] = c;
        }
        for (int64_t s = 0; s < g.nslices; ++s) cnt[s + 1] += cnt[s];
        g.npairs = cnt[g.nslices];
        if (2 * g.npairs + n != g.nnz) return IDP_EINVAL;  // stencil not symmetric
        g.pair_e.resize(g.npairs);
        g.pair_t.resize(g.npairs);
        g.pair_i.resize(g.npairs);
        g.pair_j.resize(g.npairs);
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < g.nslices; ++s) {
            int64_t p = cnt[s];
            for (int k = 0; k < g.slice_w[s]; ++k)
                for (int lane = 0; lane < kSellC; ++lane) {
                    const int64_t r = s * kSellC + lane;
                    const int32_t i = g.perm[r];
                    if (i < 0 || k >= g.row_len[r]) continue;
                    const int64_t e = g.slice_off[s] + int64_t(k) * kSellC + lane;
                    const int32_t j = g.scol[e];
                    if (!before(i, j)) continue;
                    g.pair_e[p] = int32_t(e);
                    g.pair_t[p] = g.stpos[e];
                    g.pair_i[p] = i;
                    g.pair_j[p] = j;
                    ++p;
                }
        }
    }
    return IDP_OK;
}

int build_graph(HostGraph &g, int dim, int64_t n, int64_t ncells,
                const int64_t *cells, int sigma, const int32_t *key)
{
    try {
        return build(g, dim, n, ncells, cells, sigma, key);
    } catch (const std::bad_alloc &) {
        return IDP_ENOMEM;
    }
}

static int concat(const std::vector<HostGraph> &parts, HostGraph &g, BatchLayout &lay)
{
    const size_t K = parts.size();
    const HostGraph &p0 = parts[0];
    g = HostGraph();
    g.dim = p0.dim;
    g.nv = p0.nv;
    for (auto *v : {&lay.node, &lay.cell, &lay.nnz, &lay.slice, &lay.sell, &lay.pair})
        v->assign(K + 1, 0);
    for (size_t k = 0; k < K; ++k) {
        const HostGraph &h = parts[k];
        lay.node[k + 1] = lay.node[k] + h.n;
        lay.cell[k + 1] = lay.cell[k] + h.ncells;
        lay.nnz[k + 1] = lay.nnz[k] + h.nnz;
        lay.slice[k + 1] = lay.slice[k] + h.nslices;
        lay.sell[k + 1] = lay.sell[k] + h.sell_size;
        lay.pair[k + 1] = lay.pair[k] + h.npairs;
        if (h.max_len > g.max_len) g.max_len = h.max_len;
    }
    // positions and node ids stay 32-bit on the device
    if (lay.sell[K] >= (int64_t(1) << 31) || lay.node[K] >= (int64_t(1) << 31)) return IDP_EINVAL;
    g.n = lay.node[K];
    g.ncells = lay.cell[K];
    g.nnz = lay.nnz[K];
    g.nslices = lay.slice[K];
    g.sell_size = lay.sell[K];
    g.npairs = lay.pair[K];
    g.row_ptr.resize(g.n + 1);
    g.col.resize(g.nnz);
    g.tpos.resize(g.nnz);
    g.nc_ptr.resize(g.n + 1);
    g.nc_list.resize(size_t(g.ncells) * g.nv);
    const int64_t nr = g.nslices * kSellC;
    g.perm.resize(nr);
    g.row_len.resize(nr);
    g.diag_k.resize(nr);
    g.slice_w.resize(g.nslices);
    g.slice_off.resize(g.nslices);
    g.sell_of_csr.resize(g.nnz);
    g.scol.resize(g.sell_size);
    g.stpos.resize(g.sell_size);
    g.pair_e.resize(g.npairs);
    g.pair_t.resize(g.npairs);
    g.pair_i.resize(g.npairs);
    g.pair_j.resize(g.npairs);
    lay.inst_slice.resize(g.nslices);
    for (size_t k = 0; k < K; ++k) {
        const HostGraph &h = parts[k];
        const int64_t no = lay.node[k], co = lay.cell[k], zo = lay.nnz[k];
        const int64_t so = lay.slice[k], eo = lay.sell[k], po = lay.pair[k];
        for (int64_t i = 0; i < h.n; ++i) {
            g.row_ptr[no + i] = zo + h.row_ptr[i];
            g.nc_ptr[no + i] = co * g.nv + h.nc_ptr[i];
        }
        for (int64_t q = 0; q < h.nnz; ++q) {
            g.col[zo + q] = int32_t(no + h.col[q]);
            g.tpos[zo + q] = zo + h.tpos[q];
            g.sell_of_csr[zo + q] = eo + h.sell_of_csr[q];
        }
        for (int64_t q = 0; q < h.ncells * h.nv; ++q)
            g.nc_list[co * g.nv + q] = int32_t(co + h.nc_list[q]);
        for (int64_t r = 0; r < h.nslices * kSellC; ++r) {
            g.perm[so * kSellC + r] = h.perm[r] >= 0 ? int32_t(no + h.perm[r]) : -1;
            g.row_len[so * kSellC + r] = h.row_len[r];
            g.diag_k[so * kSellC + r] = h.diag_k[r];
        }
        for (int64_t t = 0; t < h.nslices; ++t) {
            g.slice_w[so + t] = h.slice_w[t];
            g.slice_off[so + t] = eo + h.slice_off[t];
            lay.inst_slice[so + t] = int32_t(k);
        }
        for (int64_t e = 0; e < h.sell_size; ++e) {
            g.scol[eo + e] = int32_t(no + h.scol[e]);
            g.stpos[eo + e] = int32_t(eo + h.stpos[e]);
        }
        for (int64_t q = 0; q < h.npairs; ++q) {
            g.pair_e[po + q] = int32_t(eo + h.pair_e[q]);
            g.pair_t[po + q] = int32_t(eo + h.pair_t[q]);
            g.pair_i[po + q] = int32_t(no + h.pair_i[q]);
            g.pair_j[po + q] = int32_t(no + h.pair_j[q]);
        }
    }
    g.row_ptr[g.n] = g.nnz;
    g.nc_ptr[g.n] = g.ncells * g.nv;
    return IDP_OK;
}

// The pair ranges of the row blocks and the halo position of each pair's
// row node (see Halos); left empty unless the pair entries ascend and every
// pair's row diagonal holds its node i.
static void pair_ranges(const HostGraph &g, int64_t nblocks, Halos &h)
{
    const int64_t np = g.npairs, nb = (g.nslices + 3) / 4;
    for (int64_t p = 1; p < np; ++p)
        if (g.pair_e[size_t(p)] <= g.pair_e[size_t(p - 1)]) return;
    std::vector<int64_t> blk(size_t(nblocks + 1), np);
    for (int64_t b = 0; b < nb; ++b)
        blk[size_t(b)] = std::lower_bound(g.pair_e.begin(), g.pair_e.end(),
                                          g.slice_off[size_t(4 * b)],
                                          [](int32_t a, int64_t v) { return a < v; }) -
                         g.pair_e.begin();
    std::vector<uint16_t> li(size_t(np), 0);
    bool bad = false;
#pragma omp parallel for schedule(dynamic, 64) reduction(|| : bad)
    for (int64_t b = 0; b < nb; ++b) {
        if (h.cnt[size_t(b)] < 0) continue;
        int64_t s = 4 * b;
        for (int64_t p = blk[size_t(b)]; p < blk[size_t(b + 1)]; ++p) {
            const int64_t e = g.pair_e[size_t(p)];
            while (s + 1 < g.nslices && g.slice_off[size_t(s + 1)] <= e) ++s;
            const int lane = int((e - g.slice_off[size_t(s)]) % kSellC);
            const int64_t r = s * kSellC + lane;
            const int64_t ed = g.slice_off[size_t(s)] + int64_t(g.diag_k[size_t(r)]) * kSellC + lane;
            if (s >= 4 * b + 4 || g.scol[size_t(ed)] != g.pair_i[size_t(p)]) {
                bad = true;
                break;
            }
            li[size_t(p)] = h.loc[size_t(ed)];
        }
    }
    if (bad) return;
    h.pair_blk.swap(blk);
    h.pair_li.swap(li);
}

int build_halos(const HostGraph &g, int64_t nblocks, int hmax, Halos &h)
{
    try {
        const int64_t nb = (g.nslices + 3) / 4;
        h.cnt.assign(size_t(nblocks), 0);
        h.start.assign(size_t(nblocks), 0);
        h.loc.assign(size_t(g.sell_size), 0);
        std::vector<std::vector<int32_t>> lists(static_cast<size_t>(nb));
        bool oom = false;
#pragma omp parallel
        {
            std::vector<int32_t> stamp;
            std::vector<uint16_t> pos;
            try {
                stamp.assign(size_t(g.n), -1);
                pos.assign(size_t(g.n), 0);
            } catch (const std::bad_alloc &) {
#pragma omp atomic write
                oom = true;
            }
#pragma omp for schedule(dynamic, 64)
            for (int64_t b = 0; b < nb; ++b) {
                if (stamp.empty()) continue;
                std::vector<int32_t> &L = lists[size_t(b)];
                const int64_t s1 = std::min<int64_t>(4 * b + 4, g.nslices);
                for (int64_t s = 4 * b; s < s1; ++s)
                    for (int lane = 0; lane < kSellC; ++lane) {
                        const int64_t r = s * kSellC + lane;
                        if (g.perm[r] < 0) continue;
                        for (int k = 0; k < g.row_len[r]; ++k) {
                            const int32_t c = g.scol[g.slice_off[s] + int64_t(k) * kSellC + lane];
                            if (stamp[c] != int32_t(b)) {
                                stamp[c] = int32_t(b);
                                L.push_back(c);
                            }
                        }
                    }
                if (int64_t(L.size()) > hmax) {
                    h.cnt[size_t(b)] = -1;
                    std::vector<int32_t>().swap(L);
                    continue;
                }
                std::sort(L.begin(), L.end());
                h.cnt[size_t(b)] = int32_t(L.size());
                for (size_t q = 0; q < L.size(); ++q) pos[L[q]] = uint16_t(q);
                for (int64_t s = 4 * b; s < s1; ++s)
                    for (int lane = 0; lane < kSellC; ++lane) {
                        const int64_t r = s * kSellC + lane;
                        if (g.perm[r] < 0) continue;
                        for (int k = 0; k < g.row_len[r]; ++k) {
                            const int64_t e = g.slice_off[s] + int64_t(k) * kSellC + lane;
                            h.loc[size_t(e)] = pos[g.scol[e]];
                        }
                    }
            }
        }
        if (oom) return IDP_ENOMEM;
        int64_t tot = 0;
        for (int64_t b = 0; b < nb; ++b) {
            h.start[size_t(b)] = tot;
            tot += int64_t(lists[size_t(b)].size());
        }
        for (int64_t b = nb; b < nblocks; ++b) h.start[size_t(b)] = tot;
        h.node.resize(size_t(tot));
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < nb; ++b)
            std::copy(lists[size_t(b)].begin(), lists[size_t(b)].end(),
                      h.node.begin() + h.start[size_t(b)]);
        pair_ranges(g, nblocks, h);
    } catch (const std::bad_alloc &) {
        return IDP_ENOMEM;
    }
    return IDP_OK;
}

void upper_bases(const HostGraph &g, std::vector<int64_t> &base)
{
    const int64_t ns = g.nslices;
    base.assign(size_t(ns) + 1, 0);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t cnt = 0;
        for (int l = 0; l < kSellC; ++l) {
            const int64_t r = s * kSellC + l;
            const int32_t i = g.perm[size_t(r)];
            if (i < 0) continue;
            for (int k = 0; k < g.row_len[size_t(r)]; ++k)
                cnt += g.scol[size_t(g.slice_off[size_t(s)] + l + int64_t(k) * kSellC)] > i;
        }
        base[size_t(s) + 1] = cnt;
    }
    for (int64_t s = 0; s < ns; ++s) base[size_t(s) + 1] += base[size_t(s)];
}

int concat_graphs(const std::vector<HostGraph> &parts, HostGraph &g, BatchLayout &lay)
{
    if (parts.empty()) return IDP_EINVAL;
    try {
        return concat(parts, g, lay);
    } catch (const std::bad_alloc &) {
        return IDP_ENOMEM;
    }
}

// Morton code: the coordinates scaled to 2^(63/dim) steps of their bounding
// box, bits interleaved (x lowest)
void morton_order(int dim, int64_t n, const double *coords, std::vector<int32_t> &order)
{
    const int bits = dim == 3 ? 21 : 31;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        lo[d] = hi[d] = n > 0 ? coords[d] : 0.0;
        for (int64_t i = 1; i < n; ++i) {
            lo[d] = std::min(lo[d], coords[i * dim + d]);
            hi[d] = std::max(hi[d], coords[i * dim + d]);
        }
    }
    const double top = double((uint64_t(1) << bits) - 1);
    std::vector<uint64_t> code(size_t(n), 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t c = 0;
        for (int d = 0; d < dim; ++d) {
            const double w = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
            const double x = (coords[i * dim + d] - lo[d]) / w * top + 0.5;
            const uint64_t q = x >= 0.0 ? (x < top ? uint64_t(x) : uint64_t(top)) : 0;  // NaN: 0
            for (int b = 0; b < bits; ++b) c |= ((q >> b) & 1u) << (b * dim + d);
        }
        code[size_t(i)] = c;
    }
    order.resize(size_t(n));
    for (int64_t i = 0; i < n; ++i) order[size_t(i)] = int32_t(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return code[size_t(a)] < code[size_t(b)]; });
}

}  // namespace idp
