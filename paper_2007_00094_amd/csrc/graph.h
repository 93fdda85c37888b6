// Host-side stencil graph of a Q1 mesh and its SELL-64 device layout.
//
// The stencil I(i) (Section 3.1) is the set of nodes that share a cell with
// node i, i included.  Rows are kept in CSR with ascending columns; for the
// device the rows are additionally packed as SELL-C-sigma with C = 64 (one
// wavefront lane per row) and sigma = all rows by default: rows sorted by
// length, longest first, stable in node id, so that the slices of
// full-stencil interior rows carry no padding (the paper's SELL-C-sigma layout, Section
// 4.3, with the slice height set to the wavefront width instead of the
// SIMD width).  Entry k of the row in lane l of slice s sits at
// slice_off[s] + 64 k + l.
#pragma once

#include <cstdint>
#include <vector>

namespace idp {

constexpr int kSellC = 64;

struct HostGraph {
    int dim = 0;
    int nv = 0;              // vertices per cell, 2^dim
    int64_t n = 0;           // nodes
    int64_t ncells = 0;
    int64_t nnz = 0;         // CSR entries, diagonal included
    int max_len = 0;         // longest row

    std::vector<int64_t> row_ptr;   // [n+1]
    std::vector<int32_t> col;       // [nnz] ascending within a row
    std::vector<int64_t> tpos;      // [nnz] CSR position of (j,i)

    std::vector<int64_t> nc_ptr;    // [n+1] node -> cells, ascending cell id
    std::vector<int32_t> nc_list;   // [ncells*nv]

    // SELL-64
    int64_t nslices = 0;
    int64_t sell_size = 0;          // entries incl. padding
    std::vector<int32_t> perm;      // [nslices*64] sorted row -> node (-1 pad)
    std::vector<int32_t> row_len;   // [nslices*64] length of sorted row (0 pad)
    std::vector<int32_t> diag_k;    // [nslices*64] position of i in its row
    std::vector<int32_t> slice_w;   // [nslices]
    std::vector<int64_t> slice_off; // [nslices]
    std::vector<int64_t> sell_of_csr;  // [nnz]
    std::vector<int32_t> scol;      // [sell_size] column node id (pad: own)
    std::vector<int32_t> stpos;     // [sell_size] SELL position of (j,i)

    // unordered pairs {i, j}, i < j, in SELL order of the entry (i, j):
    // SELL positions of (i,j) and (j,i) and the two nodes
    int64_t npairs = 0;
    std::vector<int32_t> pair_e, pair_t, pair_i, pair_j;
};

// Returns 0 or a negative idp error code (IDP_EINVAL for ids out of range,
// IDP_ENOMEM).  cells is [ncells][2^dim] (int64 node ids).  Rows are sorted
// by length within windows of sigma rows (a multiple of 64; 0: all rows).
// The columns of a row ascend by key[j] (the node id itself if key is
// null): a renumbered mesh passes each node's original id, so that every
// row keeps the original column order.
int build_graph(HostGraph &g, int dim, int64_t n, int64_t ncells,
                const int64_t *cells, int sigma = 0, const int32_t *key = nullptr);

// A numbering of the nodes along a Morton curve of their coordinates
// (coords [n][dim]): order[k] = the node placed k-th (ties: by node id).
void morton_order(int dim, int64_t n, const double *coords, std::vector<int32_t> &order);

// Neighbourhoods of row blocks, for staging in LDS.  Block b holds the rows
// of slices 4b .. 4b+3; its halo is the ascending set of the columns of
// those rows.  cnt[b] = its size, or -1 if it exceeds hmax (the block then
// gathers from memory); node[start[b] + q] is its q-th node and loc[e] the
// halo position of entry e's column (entries of blocks with cnt < 0: 0).
// The pairs of block b (those whose row i lies in it: pairs are ordered by
// entry) are pair_blk[b] .. pair_blk[b+1]-1, and pair_li[p] is the halo
// position of pair p's node i (its row's diagonal entry); pair_blk stays
// empty if the pair entries are not ascending.
struct Halos {
    std::vector<int64_t> start;   // [nblocks]
    std::vector<int32_t> cnt;     // [nblocks]
    std::vector<int32_t> node;
    std::vector<uint16_t> loc;    // [sell_size]
    std::vector<int64_t> pair_blk;   // [nblocks + 1]
    std::vector<uint16_t> pair_li;   // [npairs]
};

// nblocks >= ceil(nslices / 4) (blocks past the last slice: empty).
// Returns 0 or IDP_ENOMEM.
int build_halos(const HostGraph &g, int64_t nblocks, int hmax, Halos &h);

// base[s] = the number of SELL entries (i, j) with j > i in the slices
// before s (s = 0..nslices): each unordered pair has one such entry, so
// base[nslices] = npairs.
void upper_bases(const HostGraph &g, std::vector<int64_t> &base);

// Where each instance of a concatenated batch lives (k = 0..ninst, the
// last entry is the total): nodes, cells, CSR entries, slices, SELL
// entries, pairs.
struct BatchLayout {
    std::vector<int64_t> node, cell, nnz, slice, sell, pair;
    std::vector<int32_t> inst_slice;   // [nslices] instance of each slice
};

// Concatenates independent graphs into one: instance k's ids, positions
// and slices are shifted past those of instances 0..k-1, so a slice or a
// pair never mixes instances and every row keeps its columns and order.
// Returns 0 or IDP_ENOMEM.
int concat_graphs(const std::vector<HostGraph> &parts, HostGraph &g, BatchLayout &lay);

}  // namespace idp
