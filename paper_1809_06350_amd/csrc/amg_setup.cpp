// Host-side set-up of the aggregation multigrid for the A-block solves: the
// parts that depend on the mesh only (aggregates, near-null space,
// prolongators, coarse patterns and the lists that sum the Galerkin products),
// built once per mesh; the coarse operators themselves are formed on the
// device for every linear system (amg.h).
//
// Method (the paper preconditions its A-solves with algebraic multigrid; this
// is plain aggregation multigrid after Vanek, Mandel and Brezina):
//  - aggregates: greedy, in node order, on the level's node graph: (1) a node
//    whose whole neighbourhood is free forms an aggregate of it; (2) each node
//    still free joins the aggregate of its first neighbour (increasing index)
//    placed in phase 1; (3) a node still free forms an aggregate with its free
//    neighbours;
//  - near-null space of the finest level: the ten conformal motions (three
//    translations, three rotations, the dilation y and the fields
//    2 (a.y) y - |y|^2 a), the kernel of the linearised isochoric stiffness,
//    at y = (X - c)/h per aggregate (c the centroid of its nodes, h the
//    largest |X - c| component), zero on Dirichlet velocity components;
//  - tentative prolongator: modified Gram-Schmidt of the ten columns over the
//    aggregate's rows (nodes ascending, dofs in order), a column whose
//    remainder is at most 1e-10 of its norm dropped; B = Q R, and R gives the
//    next level's near-null space (ten dofs per coarse node);
//  - coarse pattern: coarse nodes I, J couple when some node of I couples to
//    some node of J; the Galerkin list of a coarse block holds the blocks of
//    the finer level that add into it, in the finer level's block order.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "vms_internal.h"

namespace {

constexpr int NM = VMS_AMG_MODES;
constexpr double DROP_TOL = 1e-10;

struct LevelGraph {   // node graph of one level (sorted neighbours, self loops included)
  std::vector<int32_t> ptr, idx;
};

void aggregate(const LevelGraph &g, std::vector<int32_t> &agg, int32_t &na) {
  const int32_t n = (int32_t)g.ptr.size() - 1;
  agg.assign(n, -1);
  na = 0;
  for (int32_t i = 0; i < n; ++i) {   // phase 1: whole free neighbourhoods
    if (agg[i] >= 0) continue;
    bool free_nb = true;
    for (int32_t k = g.ptr[i]; k < g.ptr[i + 1] && free_nb; ++k) free_nb = agg[g.idx[k]] < 0;
    if (!free_nb) continue;
    for (int32_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) agg[g.idx[k]] = na;
    agg[i] = na++;
  }
  const std::vector<int32_t> phase1 = agg;
  for (int32_t i = 0; i < n; ++i) {   // phase 2: join the first neighbour placed in phase 1
    if (agg[i] >= 0) continue;
    for (int32_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) {
      const int32_t j = g.idx[k];
      if (j != i && phase1[j] >= 0) {
        agg[i] = phase1[j];
        break;
      }
    }
  }
  for (int32_t i = 0; i < n; ++i) {   // phase 3: leftovers with their free neighbours
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int32_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k)
      if (agg[g.idx[k]] < 0) agg[g.idx[k]] = na;
    ++na;
  }
}

// modes at point y: B[d][k], d the velocity component, k the mode
void conformal_modes(const double y[3], double B[3][NM]) {
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < NM; ++k) B[d][k] = 0.0;
  for (int d = 0; d < 3; ++d) B[d][d] = 1.0;
  B[1][3] = -y[2]; B[2][3] = y[1];       // rotation about e_x
  B[0][4] = y[2];  B[2][4] = -y[0];      // about e_y
  B[0][5] = -y[1]; B[1][5] = y[0];       // about e_z
  for (int d = 0; d < 3; ++d) B[d][6] = y[d];   // dilation
  const double s2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  for (int a = 0; a < 3; ++a) {
    for (int d = 0; d < 3; ++d) B[d][7 + a] = 2.0 * y[a] * y[d];
    B[a][7 + a] -= s2;
  }
}

// modified Gram-Schmidt with the drop rule on M (rows x NM, row-major), in place -> Q; R (NM x NM)
void mgs_drop(std::vector<double> &M, int rows, double R[NM][NM]) {
  for (int i = 0; i < NM; ++i)
    for (int j = 0; j < NM; ++j) R[i][j] = 0.0;
  std::vector<double> v(rows);
  for (int j = 0; j < NM; ++j) {
    double n0 = 0.0;
    for (int r = 0; r < rows; ++r) {
      v[r] = M[(size_t)r * NM + j];
      n0 += v[r] * v[r];
    }
    n0 = std::sqrt(n0);
    for (int i = 0; i < j; ++i) {
      if (R[i][i] == 0.0) continue;
      double d = 0.0;
      for (int r = 0; r < rows; ++r) d += M[(size_t)r * NM + i] * v[r];
      R[i][j] = d;
      for (int r = 0; r < rows; ++r) v[r] -= d * M[(size_t)r * NM + i];
    }
    double nv = 0.0;
    for (int r = 0; r < rows; ++r) nv += v[r] * v[r];
    nv = std::sqrt(nv);
    const bool keep = n0 > 0.0 && nv > DROP_TOL * n0;
    if (keep) R[j][j] = nv;
    for (int r = 0; r < rows; ++r) M[(size_t)r * NM + j] = keep ? v[r] / nv : 0.0;
  }
}

}  // namespace

struct vms_amg {
  struct Level {
    int32_t n = 0, bs = 3;
    int64_t nnzb = 0;                              // level >= 1: CSR blocks
    std::vector<int32_t> ptr, col, brow, dpos;     // level >= 1 pattern
    std::vector<uint8_t> dropped;                  // level >= 1: [n * 10]
    std::vector<int32_t> agg, mptr, mem;           // transfer to the next level
    std::vector<double> P;                         // [n][bs][10]
    std::vector<float> P32;
    std::vector<int32_t> gptr, gsrc;               // Galerkin lists of the next level
  };
  struct Offsets {   // byte offsets of the level's arrays in the device copy
    size_t ptr, col, brow, dpos, dropped, agg, mptr, mem, P, P32, gptr, gsrc;
  };
  int n_levels = 0;
  Level h[VMS_AMG_MAX_LEVELS];
  Offsets offs[VMS_AMG_MAX_LEVELS] = {};
  vms_amg_opts opts{};
  int32_t fine_W = 0;
  int64_t fine_nnzb = 0;
  vms_amg_dev dev{};
  size_t dev_bytes = 0;
};

namespace {

struct Layout {   // byte layout of the device copy (256-byte aligned arrays)
  size_t off = 0;
  template <typename X>
  size_t take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    const size_t at = off;
    off += sizeof(X) * count;
    return at;
  }
};

}  // namespace

extern "C" int vms_amg_create(int32_t n_nodes, int32_t slot_width, const int32_t *row_len, const int32_t *col,
                              const double *X, const uint8_t *dir_mask, const vms_amg_opts *opts, vms_amg **out) {
  if (!out) return VMS_ERR_ARG;
  *out = nullptr;
  if (n_nodes <= 0 || slot_width <= 0 || !row_len || !col || !X || !dir_mask || !opts) return VMS_ERR_ARG;
  if (opts->max_levels < 2 || opts->max_levels > VMS_AMG_MAX_LEVELS || opts->min_coarse < 0 ||
      opts->degree < 1 || opts->degree > 16 || opts->coarse_degree < 1 || opts->coarse_degree > 64 ||
      opts->mid_degree < 0 || opts->mid_degree > 16)
    return VMS_ERR_ARG;
  if ((int64_t)slot_width * n_nodes >= ((int64_t)1 << 31)) return VMS_ERR_ARG;
  for (int32_t i = 0; i < n_nodes; ++i) {
    if (row_len[i] < 1 || row_len[i] > slot_width) return VMS_ERR_ARG;
    for (int32_t s = 0; s < row_len[i]; ++s) {
      const int32_t j = col[(int64_t)slot_width * i + s];
      if (j < 0 || j >= n_nodes || (s > 0 && j <= col[(int64_t)slot_width * i + s - 1])) return VMS_ERR_ARG;
    }
  }
  vms_amg *a = new vms_amg();
  a->opts = *opts;
  a->fine_W = slot_width;
  a->fine_nnzb = (int64_t)slot_width * n_nodes;
  // finest graph from the block pattern (sorted, diagonal included)
  LevelGraph g;
  g.ptr.assign(n_nodes + 1, 0);
  for (int32_t i = 0; i < n_nodes; ++i) g.ptr[i + 1] = g.ptr[i] + row_len[i];
  g.idx.resize(g.ptr[n_nodes]);
  for (int32_t i = 0; i < n_nodes; ++i)
    for (int32_t s = 0; s < row_len[i]; ++s) g.idx[g.ptr[i] + s] = col[(int64_t)slot_width * i + s];
  // near-null space of the current level: [n][bs][NM]
  std::vector<double> B;
  int lev = 0;
  a->h[0].n = n_nodes;
  a->h[0].bs = 3;
  for (;; ++lev) {
    vms_amg::Level &L = a->h[lev];
    const int32_t n = L.n, bs = L.bs;
    if (lev == opts->max_levels - 1 || n <= opts->min_coarse) break;
    int32_t na = 0;
    aggregate(g, L.agg, na);
    // members of each aggregate, ascending
    L.mptr.assign(na + 1, 0);
    for (int32_t i = 0; i < n; ++i) L.mptr[L.agg[i] + 1]++;
    for (int32_t I = 0; I < na; ++I) L.mptr[I + 1] += L.mptr[I];
    L.mem.resize(n);
    {
      std::vector<int32_t> fill(L.mptr.begin(), L.mptr.end() - 1);
      for (int32_t i = 0; i < n; ++i) L.mem[fill[L.agg[i]]++] = i;
    }
    if (lev == 0) {   // conformal modes per aggregate
      B.assign((size_t)n * 3 * NM, 0.0);
      for (int32_t I = 0; I < na; ++I) {
        const int32_t m0 = L.mptr[I], m1 = L.mptr[I + 1];
        double c[3] = {0.0, 0.0, 0.0};
        for (int32_t k = m0; k < m1; ++k)
          for (int d = 0; d < 3; ++d) c[d] += X[3 * (int64_t)L.mem[k] + d];
        for (int d = 0; d < 3; ++d) c[d] /= (double)(m1 - m0);
        double h = 0.0;
        for (int32_t k = m0; k < m1; ++k)
          for (int d = 0; d < 3; ++d) h = std::max(h, std::fabs(X[3 * (int64_t)L.mem[k] + d] - c[d]));
        if (!(h > 0.0)) h = 1.0;
        for (int32_t k = m0; k < m1; ++k) {
          const int32_t i = L.mem[k];
          double y[3], Bm[3][NM];
          for (int d = 0; d < 3; ++d) y[d] = (X[3 * (int64_t)i + d] - c[d]) / h;
          conformal_modes(y, Bm);
          for (int d = 0; d < 3; ++d)
            for (int q = 0; q < NM; ++q)
              B[((size_t)i * 3 + d) * NM + q] = dir_mask[4 * (int64_t)i + d] ? 0.0 : Bm[d][q];
        }
      }
    }
    // tentative prolongator and the next level's near-null space
    vms_amg::Level &C = a->h[lev + 1];
    C.n = na;
    C.bs = NM;
    L.P.assign((size_t)n * bs * NM, 0.0);
    std::vector<double> Bc((size_t)na * NM * NM, 0.0);
    C.dropped.assign((size_t)na * NM, 0);
    std::vector<double> M;
    for (int32_t I = 0; I < na; ++I) {
      const int32_t m0 = L.mptr[I], m1 = L.mptr[I + 1];
      const int rows = (m1 - m0) * bs;
      M.assign((size_t)rows * NM, 0.0);
      for (int32_t k = m0; k < m1; ++k)
        for (int d = 0; d < bs; ++d)
          for (int q = 0; q < NM; ++q)
            M[((size_t)(k - m0) * bs + d) * NM + q] = B[((size_t)L.mem[k] * bs + d) * NM + q];
      double R[NM][NM];
      mgs_drop(M, rows, R);
      for (int32_t k = m0; k < m1; ++k)
        for (int d = 0; d < bs; ++d)
          for (int q = 0; q < NM; ++q)
            L.P[((size_t)L.mem[k] * bs + d) * NM + q] = M[((size_t)(k - m0) * bs + d) * NM + q];
      for (int r = 0; r < NM; ++r) {
        for (int q = 0; q < NM; ++q) Bc[((size_t)I * NM + r) * NM + q] = R[r][q];
        C.dropped[(size_t)I * NM + r] = R[r][r] == 0.0 ? 1 : 0;
      }
    }
    L.P32.assign(L.P.begin(), L.P.end());
    // coarse graph and pattern
    LevelGraph gc;
    gc.ptr.assign(na + 1, 0);
    {
      std::vector<std::vector<int32_t>> rows(na);
      for (int32_t i = 0; i < n; ++i)
        for (int32_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) rows[L.agg[i]].push_back(L.agg[g.idx[k]]);
      for (int32_t I = 0; I < na; ++I) {
        auto &r = rows[I];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        gc.ptr[I + 1] = gc.ptr[I] + (int32_t)r.size();
      }
      gc.idx.resize(gc.ptr[na]);
      for (int32_t I = 0; I < na; ++I) std::copy(rows[I].begin(), rows[I].end(), gc.idx.begin() + gc.ptr[I]);
    }
    C.ptr = gc.ptr;
    C.col = gc.idx;
    C.nnzb = gc.ptr[na];
    C.brow.resize(C.nnzb);
    C.dpos.resize(na);
    for (int32_t I = 0; I < na; ++I)
      for (int32_t k = gc.ptr[I]; k < gc.ptr[I + 1]; ++k) {
        C.brow[k] = I;
        if (gc.idx[k] == I) C.dpos[I] = k;
      }
    // Galerkin lists: every block of this level in its block order, grouped by coarse block
    {
      std::vector<int64_t> src_blk;     // this level's block ids
      std::vector<int32_t> dst;         // coarse block of each
      for (int32_t i = 0; i < n; ++i) {
        const int32_t I = L.agg[i];
        const int32_t *cb = gc.idx.data() + gc.ptr[I], *ce = gc.idx.data() + gc.ptr[I + 1];
        const int32_t k0 = lev == 0 ? 0 : L.ptr[i], k1 = lev == 0 ? row_len[i] : L.ptr[i + 1];
        for (int32_t k = k0; k < k1; ++k) {
          const int64_t b = lev == 0 ? (int64_t)slot_width * i + k : (int64_t)k;
          const int32_t j = lev == 0 ? col[b] : L.col[k];
          const int32_t J = L.agg[j];
          const int32_t pos = (int32_t)(std::lower_bound(cb, ce, J) - gc.idx.data());
          src_blk.push_back(b);
          dst.push_back(pos);
        }
      }
      L.gptr.assign(C.nnzb + 1, 0);
      for (int32_t d : dst) L.gptr[d + 1]++;
      for (int64_t k = 0; k < C.nnzb; ++k) L.gptr[k + 1] += L.gptr[k];
      L.gsrc.resize(dst.size());
      std::vector<int32_t> fill(L.gptr.begin(), L.gptr.end() - 1);
      for (size_t k = 0; k < dst.size(); ++k) L.gsrc[fill[dst[k]]++] = (int32_t)src_blk[k];
    }
    g = std::move(gc);
    B = std::move(Bc);
  }
  a->n_levels = lev + 1;
  // device layout
  Layout lay;
  for (int l = 0; l < a->n_levels; ++l) {
    vms_amg::Level &L = a->h[l];
    vms_amg::Offsets &o = a->offs[l];
    vms_amg_level_dev &D = a->dev.lev[l];
    D.n = L.n;
    D.bs = L.bs;
    D.nnzb = l == 0 ? a->fine_nnzb : L.nnzb;
    if (l > 0) {
      o.ptr = lay.take<int32_t>(L.ptr.size());
      o.col = lay.take<int32_t>(L.col.size());
      o.brow = lay.take<int32_t>(L.brow.size());
      o.dpos = lay.take<int32_t>(L.dpos.size());
      o.dropped = lay.take<uint8_t>(L.dropped.size());
    }
    if (l < a->n_levels - 1) {
      o.agg = lay.take<int32_t>(L.agg.size());
      o.mptr = lay.take<int32_t>(L.mptr.size());
      o.mem = lay.take<int32_t>(L.mem.size());
      o.P = lay.take<double>(L.P.size());
      o.P32 = lay.take<float>(L.P32.size());
      o.gptr = lay.take<int32_t>(L.gptr.size());
      o.gsrc = lay.take<int32_t>(L.gsrc.size());
    }
  }
  a->dev.n_levels = a->n_levels;
  a->dev.degree = opts->degree;
  a->dev.coarse_degree = opts->coarse_degree;
  a->dev.mid_degree = opts->mid_degree > 0 ? opts->mid_degree : opts->degree;
  a->dev.uploaded = 0;
  a->dev_bytes = lay.off + 256;
  *out = a;
  return VMS_OK;
}

extern "C" void vms_amg_destroy(vms_amg *amg) { delete amg; }

extern "C" int vms_amg_get_info(const vms_amg *amg, vms_amg_info *info) {
  if (!amg || !info) return VMS_ERR_ARG;
  std::memset(info, 0, sizeof(*info));
  info->n_levels = amg->n_levels;
  for (int l = 0; l < amg->n_levels; ++l) {
    info->n[l] = amg->h[l].n;
    info->bs[l] = amg->h[l].bs;
    info->nnzb[l] = l == 0 ? amg->fine_nnzb : amg->h[l].nnzb;
  }
  info->device_bytes = amg->dev_bytes;
  return VMS_OK;
}

extern "C" int vms_amg_level_arrays(const vms_amg *amg, int level, const int32_t **agg, const double **P,
                                    const int32_t **ptr, const int32_t **col, const uint8_t **dropped) {
  if (!amg || level < 0 || level >= amg->n_levels) return VMS_ERR_ARG;
  const vms_amg::Level &L = amg->h[level];
  const bool has_next = level < amg->n_levels - 1;
  if (agg) *agg = has_next ? L.agg.data() : nullptr;
  if (P) *P = has_next ? L.P.data() : nullptr;
  if (ptr) *ptr = level > 0 ? L.ptr.data() : nullptr;
  if (col) *col = level > 0 ? L.col.data() : nullptr;
  if (dropped) *dropped = level > 0 ? L.dropped.data() : nullptr;
  return VMS_OK;
}

extern "C" size_t vms_amg_device_bytes(const vms_amg *amg) { return amg ? amg->dev_bytes : 0; }

extern "C" int vms_amg_upload(vms_ctx *ctx, vms_amg *amg, void *device_buffer, size_t bytes) {
  if (!ctx) return VMS_ERR_ARG;
  if (!amg || !device_buffer) return vms_set_error(ctx, VMS_ERR_ARG, "vms_amg_upload: missing argument");
  if (bytes < amg->dev_bytes)
    return vms_set_error(ctx, VMS_ERR_WORKSPACE, "vms_amg_upload: buffer too small: %zu < %zu", bytes,
                         amg->dev_bytes);
  // dev_bytes includes 256 bytes of alignment slack
  char *base = (char *)(((uintptr_t)device_buffer + 255) & ~(uintptr_t)255);
  vms_amg_dev &D = amg->dev;
  D.uploaded = 0;
  for (int l = 0; l < amg->n_levels; ++l) {
    const vms_amg::Level &L = amg->h[l];
    const vms_amg::Offsets &o = amg->offs[l];
    vms_amg_level_dev &lv = D.lev[l];
    auto put = [&](size_t off, const void *src, size_t nbytes) -> void * {
      void *dst = base + off;
      if (nbytes && hipMemcpyAsync(dst, src, nbytes, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        return nullptr;
      return dst;
    };
    bool ok = true;
    if (l > 0) {
      ok = ok && (lv.ptr = (const int32_t *)put(o.ptr, L.ptr.data(), L.ptr.size() * 4));
      ok = ok && (lv.col = (const int32_t *)put(o.col, L.col.data(), L.col.size() * 4));
      ok = ok && (lv.brow = (const int32_t *)put(o.brow, L.brow.data(), L.brow.size() * 4));
      ok = ok && (lv.dpos = (const int32_t *)put(o.dpos, L.dpos.data(), L.dpos.size() * 4));
      ok = ok && (lv.dropped = (const uint8_t *)put(o.dropped, L.dropped.data(), L.dropped.size()));
    }
    if (l < amg->n_levels - 1) {
      ok = ok && (lv.agg = (const int32_t *)put(o.agg, L.agg.data(), L.agg.size() * 4));
      ok = ok && (lv.mptr = (const int32_t *)put(o.mptr, L.mptr.data(), L.mptr.size() * 4));
      ok = ok && (lv.mem = (const int32_t *)put(o.mem, L.mem.data(), L.mem.size() * 4));
      ok = ok && (lv.P = (const double *)put(o.P, L.P.data(), L.P.size() * 8));
      ok = ok && (lv.P32 = (const float *)put(o.P32, L.P32.data(), L.P32.size() * 4));
      ok = ok && (lv.gptr = (const int32_t *)put(o.gptr, L.gptr.data(), L.gptr.size() * 4));
      ok = ok && (lv.gsrc = (const int32_t *)put(o.gsrc, L.gsrc.data(), L.gsrc.size() * 4));
    }
    if (!ok) return vms_set_error(ctx, VMS_ERR_HIP, "vms_amg_upload: copy to the device failed");
  }
  VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  D.uploaded = 1;
  D.device = ctx->device;
  return VMS_OK;
}

const vms_amg_dev *vms_amg_device(const vms_amg *amg) { return amg ? &amg->dev : nullptr; }
