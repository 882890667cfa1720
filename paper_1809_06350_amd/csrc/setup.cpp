// Host-side setup of the node-graph block pattern (integer work only).
//
// The tangent [[A, B], [C, D]] of the P1 discretisation couples every pair of
// nodes that share a tetrahedron, so one block pattern over nodes serves all
// four value arrays.  Rows are stored in fixed-width slots: row i owns blocks
// b = W*i + s, s < W, with W the largest row length rounded up to a multiple
// of 16; its row_len[i] real blocks come first with sorted columns (diagonal
// included), the padding slots hold column i, zero values and no
// contributions.  Products then find a row without reading row pointers, and
// every row starts on a 16-block boundary.
// Besides the pattern this file builds
//   tpos[b]        position of block (j, i) for the block b = (i, j),
//   diag_pos[i]    position of block (i, i),
//   blk_src_ptr / blk_src: for every block, the element-local pairs that add
//                  into it, as e*16 + A*4 + B (element e, rows of node
//                  tets[e][A], columns of node tets[e][B]), in increasing
//                  element order; the gather that sums element matrices into
//                  the blocks follows this order, so the assembled values do not
//                  depend on scheduling.  The contributions of a diagonal
//                  block are exactly the (element, local node) incidences of
//                  its node, which also serves the nodal gathers,
//   shat_col: the off-diagonal distance-2 node pattern (every other node
//                  reachable in two graph steps), the pattern of
//                  S^ = D - C diag(A)^-1 B without its diagonal, in rows of
//                  shat_width fixed slots (a multiple of 64: one wavefront
//                  per row, one entry per lane): sorted columns first,
//                  padding slots hold the row's own node,
//   node -> loaded boundary face lists (for the dead-load vector).
#include <algorithm>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <vector>

#include "vms_internal.h"

namespace {

struct Graph {
  std::vector<int32_t> row_ptr, col;
};

Graph build_graph(int32_t n, int32_t m, const int32_t *tets) {
  std::vector<int32_t> deg(n, 0);
  for (int64_t e = 0; e < m; ++e)
    for (int a = 0; a < 4; ++a) deg[tets[4 * e + a]] += 4;
  std::vector<int64_t> off(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg[i];
  std::vector<int32_t> tmp(off[n]);
  std::vector<int64_t> fill(off.begin(), off.end() - 1);
  for (int64_t e = 0; e < m; ++e)
    for (int a = 0; a < 4; ++a) {
      int32_t i = tets[4 * e + a];
      for (int b = 0; b < 4; ++b) tmp[fill[i]++] = tets[4 * e + b];
    }
  Graph g;
  g.row_ptr.assign(n + 1, 0);
  g.col.reserve(off[n] / 3);
  for (int32_t i = 0; i < n; ++i) {
    auto first = tmp.begin() + off[i], last = tmp.begin() + off[i + 1];
    std::sort(first, last);
    auto uend = std::unique(first, last);
    if (first == uend) {          // isolated node: keep a diagonal block
      g.col.push_back(i);
    } else {
      g.col.insert(g.col.end(), first, uend);
    }
    g.row_ptr[i + 1] = (int32_t)g.col.size();
  }
  return g;
}

inline int32_t find_block(const Graph &g, int32_t i, int32_t j) {
  auto first = g.col.begin() + g.row_ptr[i], last = g.col.begin() + g.row_ptr[i + 1];
  auto it = std::lower_bound(first, last, j);
  if (it == last || *it != j) return -1;
  return (int32_t)(it - g.col.begin());
}

}  // namespace

// off-diagonal distance-2 pattern: row i lists every j != i with a k in N(i) and j in N(k)
static void build_ring2(const Graph &g, int32_t n, std::vector<int64_t> &ptr, std::vector<int32_t> *col) {
  ptr.assign(n + 1, 0);
  std::vector<int32_t> mark(n, -1), row;
  for (int32_t i = 0; i < n; ++i) {
    row.clear();
    mark[i] = i;
    for (int32_t a = g.row_ptr[i]; a < g.row_ptr[i + 1]; ++a) {
      const int32_t k = g.col[a];
      for (int32_t b = g.row_ptr[k]; b < g.row_ptr[k + 1]; ++b) {
        const int32_t j = g.col[b];
        if (mark[j] != i) { mark[j] = i; row.push_back(j); }
      }
    }
    if (col) {
      std::sort(row.begin(), row.end());
      col->insert(col->end(), row.begin(), row.end());
    }
    ptr[i + 1] = ptr[i] + (int64_t)row.size();
  }
}

static int32_t ring2_width(const std::vector<int64_t> &p2, int32_t n) {
  int64_t mx = 1;
  for (int32_t i = 0; i < n; ++i) mx = std::max(mx, p2[i + 1] - p2[i]);
  return (int32_t)(64 * ((mx + 63) / 64));
}

static int32_t slot_width(const Graph &g, int32_t n) {
  int32_t mx = 1;
  for (int32_t i = 0; i < n; ++i) mx = std::max(mx, g.row_ptr[i + 1] - g.row_ptr[i]);
  return 16 * ((mx + 15) / 16);
}

extern "C" int vms_setup_sizes(int32_t n_nodes, int32_t n_tets, const int32_t *tets, int64_t *nnzb,
                               int32_t *slot_width_out, int32_t *shat_width_out, int32_t *shat_span_out) {
  if (n_nodes <= 0 || n_tets < 0 || (!tets && n_tets > 0) || !nnzb || !slot_width_out || !shat_width_out)
    return VMS_ERR_ARG;
  if ((int64_t)n_tets > VMS_MAX_TETS) return VMS_ERR_ARG;
  for (int64_t k = 0; k < 4 * (int64_t)n_tets; ++k)
    if (tets[k] < 0 || tets[k] >= n_nodes) return VMS_ERR_ARG;
  Graph g = build_graph(n_nodes, n_tets, tets);
  const int32_t W = slot_width(g, n_nodes);
  if ((int64_t)W * n_nodes >= ((int64_t)1 << 31)) return VMS_ERR_ARG;
  std::vector<int64_t> p2;
  std::vector<int32_t> c2;
  build_ring2(g, n_nodes, p2, shat_span_out ? &c2 : nullptr);
  const int32_t W2 = ring2_width(p2, n_nodes);
  if (W2 > VMS_MAX_SHAT_ROW || (int64_t)W2 * n_nodes >= ((int64_t)1 << 31)) return VMS_ERR_ARG;
  *slot_width_out = W;
  *nnzb = (int64_t)W * n_nodes;
  *shat_width_out = W2;
  if (shat_span_out) {
    int64_t span = 0;
    for (int32_t i = 0; i < n_nodes; ++i)
      for (int64_t k = p2[i]; k < p2[i + 1]; ++k) span = std::max<int64_t>(span, std::abs((int64_t)c2[k] - i));
    *shat_span_out = (int32_t)span;
  }
  return VMS_OK;
}

extern "C" int vms_setup_build(int32_t n_nodes, int32_t n_tets, const int32_t *tets,
                               int32_t n_bfaces, const int32_t *bfaces,
                               int32_t *row_len, int32_t *col, int32_t *tpos, int32_t *diag_pos,
                               int32_t *blk_src_ptr, int32_t *blk_src, int32_t *shat_col, int16_t *shat_off,
                               int32_t *nf_ptr, int32_t *nf_face) {
  if (n_nodes <= 0 || n_tets < 0 || (int64_t)n_tets > VMS_MAX_TETS || !row_len || !col || !tpos || !diag_pos ||
      !shat_col ||
      !blk_src_ptr || (n_tets > 0 && (!tets || !blk_src)) || !nf_ptr || (n_bfaces > 0 && (!bfaces || !nf_face)))
    return VMS_ERR_ARG;
  for (int64_t k = 0; k < 4 * (int64_t)n_tets; ++k)
    if (tets[k] < 0 || tets[k] >= n_nodes) return VMS_ERR_ARG;
  for (int64_t k = 0; k < 3 * (int64_t)n_bfaces; ++k)
    if (bfaces[k] < 0 || bfaces[k] >= n_nodes) return VMS_ERR_ARG;
  Graph g = build_graph(n_nodes, n_tets, tets);
  const int32_t W = slot_width(g, n_nodes);
  if ((int64_t)W * n_nodes >= ((int64_t)1 << 31)) return VMS_ERR_ARG;
  const int64_t nnzb = (int64_t)W * n_nodes;
  // slot position of the CSR block k of row i
  auto slot = [&](int32_t i, int32_t k) { return (int32_t)((int64_t)W * i + (k - g.row_ptr[i])); };
  for (int32_t i = 0; i < n_nodes; ++i) {
    const int32_t len = g.row_ptr[i + 1] - g.row_ptr[i];
    row_len[i] = len;
    for (int32_t s = 0; s < W; ++s) {
      const int64_t b = (int64_t)W * i + s;
      if (s < len) {
        col[b] = g.col[g.row_ptr[i] + s];
        const int32_t j = col[b];
        tpos[b] = slot(j, find_block(g, j, i));
      } else {
        col[b] = i;
        tpos[b] = (int32_t)b;
      }
    }
    diag_pos[i] = slot(i, find_block(g, i, i));
  }
  // block <- (element, local pair): counting sort of the 16 m pairs by block, element order kept
  std::vector<int32_t> eb(16 * (size_t)n_tets);
  for (int64_t e = 0; e < n_tets; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int32_t i = tets[4 * e + a];
        eb[16 * e + 4 * a + b] = slot(i, find_block(g, i, tets[4 * e + b]));
      }
  std::fill(blk_src_ptr, blk_src_ptr + nnzb + 1, 0);
  for (size_t k = 0; k < eb.size(); ++k) blk_src_ptr[eb[k] + 1]++;
  for (int64_t b = 0; b < nnzb; ++b) blk_src_ptr[b + 1] += blk_src_ptr[b];
  std::vector<int32_t> fill(blk_src_ptr, blk_src_ptr + nnzb);
  for (size_t k = 0; k < eb.size(); ++k) blk_src[fill[eb[k]]++] = (int32_t)k;

  // off-diagonal distance-2 pattern of S^ in fixed-width rows
  {
    std::vector<int64_t> p2;
    std::vector<int32_t> c2;
    build_ring2(g, n_nodes, p2, &c2);
    const int32_t W2 = ring2_width(p2, n_nodes);
    if (W2 > VMS_MAX_SHAT_ROW || (int64_t)W2 * n_nodes >= ((int64_t)1 << 31)) return VMS_ERR_ARG;
    for (int32_t i = 0; i < n_nodes; ++i) {
      const int64_t len = p2[i + 1] - p2[i];
      for (int32_t s2 = 0; s2 < W2; ++s2) {
        const int32_t c = (s2 < len) ? c2[p2[i] + s2] : i;
        shat_col[(int64_t)W2 * i + s2] = c;
        if (shat_off) {
          const int32_t d = c - i;
          if (d < -32768 || d > 32767) return VMS_ERR_ARG;
          shat_off[(int64_t)W2 * i + s2] = (int16_t)d;
        }
      }
    }
  }

  // node -> loaded faces
  std::fill(nf_ptr, nf_ptr + n_nodes + 1, 0);
  for (int64_t k = 0; k < 3 * (int64_t)n_bfaces; ++k) nf_ptr[bfaces[k] + 1]++;
  for (int32_t i = 0; i < n_nodes; ++i) nf_ptr[i + 1] += nf_ptr[i];
  std::vector<int32_t> ff(nf_ptr, nf_ptr + n_nodes);
  for (int64_t f = 0; f < n_bfaces; ++f)
    for (int a = 0; a < 3; ++a) nf_face[ff[bfaces[3 * f + a]]++] = (int32_t)f;
  return VMS_OK;
}
