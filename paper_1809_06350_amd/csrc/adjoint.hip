// Adjoint of the generalized-alpha time step (implicit differentiation at the
// converged state, section 3.3 block structure).
//
// One step solves G(y-dot_{n+1}; y_n, y-dot_n, theta) = 0 with
// G = (R-bar_k, R_p, R_m) and y_{n+1} = y_n + dt y-dot_n + gamma dt (y-dot_{n+1} - y-dot_n).
// Given the cotangents (y-bar_{n+1}, y-dot-bar_{n+1}) of J with respect to the
// step's output, with g = y-dot-bar_{n+1} + gamma dt y-bar_{n+1}:
//   K^T lam = g, K = dG/dy-dot_{n+1}.  With the block factorisation of K
//   (eq. K_block_decomposition): mu_u = g_u/am, mu_p = g_p,
//   mu_v = g_v + (c2/am) g_u;  [A B; C D]^T (lam_m, lam_p) = (mu_v, mu_p);
//   lam_k = mu_u - (c2/am) (dR/du_{alpha_f})^T (lam_m, lam_p).
//   y-bar_n      = y-bar_{n+1} - lam^T dG/dy_{n+alpha_f}
//   y-dot-bar_n  = (1-gamma) dt y-bar_{n+1}
//                  - [(1-am) lam^T dG/dy-dot_{n+alpha_m} + af (1-gamma) dt lam^T dG/dy_{n+alpha_f}]
//   dJ/dtheta   -= lam^T dG/dtheta   (R-bar_k does not depend on theta)
// since y_{n+alpha_f} = y_n + af((1-gamma) dt y-dot_n + gamma dt y-dot_{n+1}) and
// y-dot_{n+alpha_m} = (1-am) y-dot_n + am y-dot_{n+1}.
// Nodal cotangent layout [n][7] = (u 3, p, v 3) and (u-dot 3, p-dot, v-dot 3).
#include <chrono>
#include <cstring>

#include "vms_internal.h"

namespace {

inline int grid1(int64_t n) { return (int)((n + VMS_BLOCK - 1) / VMS_BLOCK); }

// block (i, j) of K^T = transpose of block (j, i) of K: A' = A^T, B' = C^T, C' = B^T, D' = D^T
__global__ void k_transpose(int64_t nnzb, const int32_t *tpos, const double *A, const double *B, const double *C,
                            const double *D, double *At, double *Bt, double *Ct, double *Dt, float *At32,
                            float *Bt32, float *Ct32, float *Dt32) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int64_t t = tpos[b];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const double v = A[(3 * c + r) * nnzb + t];
      At[(3 * r + c) * nnzb + b] = v;
      if (At32) At32[(3 * r + c) * nnzb + b] = (float)v;
    }
  for (int r = 0; r < 3; ++r) {
    const double vb = C[r * nnzb + t], vc = B[r * nnzb + t];
    Bt[r * nnzb + b] = vb;
    Ct[r * nnzb + b] = vc;
    if (Bt32) { Bt32[r * nnzb + b] = (float)vb; Ct32[r * nnzb + b] = (float)vc; }
  }
  Dt[b] = D[t];
  if (Dt32) Dt32[b] = (float)D[t];
}

// rhs* = W (mu_v, mu_p), mu_u kept; Dirichlet components do not carry cotangents
__global__ void k_adj_seed(int n, vms_ga ga, const uint8_t *dir, const double *W, const double *yb1,
                           const double *ydb1, double *rhs, double *mu_u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o7 = 7 * (int64_t)i, o4 = 4 * (int64_t)i;
  const double gdt = ga.gm * ga.dt;
  for (int c = 0; c < 3; ++c) {
    const bool d = dir[o4 + c];
    const double gu = ydb1[o7 + c] + gdt * yb1[o7 + c];
    const double gv = ydb1[o7 + 4 + c] + gdt * yb1[o7 + 4 + c];
    mu_u[3 * (int64_t)i + c] = d ? 0.0 : gu / ga.am;
    rhs[o4 + c] = d ? 0.0 : W[o4 + c] * (gv + ga.c2 / ga.am * gu);
  }
  const double gp = ydb1[o7 + 3] + gdt * yb1[o7 + 3];
  rhs[o4 + 3] = dir[o4 + 3] ? 0.0 : W[o4 + 3] * gp;
}

__global__ void k_unscale(int64_t n4, const double *W, const double *xs, double *x) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n4) x[k] = W[k] * xs[k];
}

// lam_k, then the cotangents of y_n and y-dot_n (vjp = [n][11] staged-field cotangents of lam_(m,p))
__global__ void k_adj_back(int n, vms_ga ga, const uint8_t *dir, const double *mu_u, const double *vjp,
                           const double *yb1, double *yb0, double *ydb0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o7 = 7 * (int64_t)i, o11 = 11 * (int64_t)i, o4 = 4 * (int64_t)i;
  const double a1 = 1.0 - ga.am, b1 = ga.af * (1.0 - ga.gm) * ga.dt, e1 = (1.0 - ga.gm) * ga.dt;
  for (int c = 0; c < 3; ++c) {
    const double lk = dir[o4 + c] ? 0.0 : mu_u[3 * (int64_t)i + c] - ga.c2 / ga.am * vjp[o11 + c];
    const double Yu = vjp[o11 + c], Yv = vjp[o11 + 4 + c] - lk;     // lam^T dG/dy_{alpha_f}
    const double Ydu = lk, Ydv = vjp[o11 + 7 + c];                  // lam^T dG/dy-dot_{alpha_m}
    yb0[o7 + c] = yb1[o7 + c] - Yu;
    yb0[o7 + 4 + c] = yb1[o7 + 4 + c] - Yv;
    ydb0[o7 + c] = e1 * yb1[o7 + c] - (a1 * Ydu + b1 * Yu);
    ydb0[o7 + 4 + c] = e1 * yb1[o7 + 4 + c] - (a1 * Ydv + b1 * Yv);
  }
  const double Yp = vjp[o11 + 3], Ydp = vjp[o11 + 10];
  yb0[o7 + 3] = yb1[o7 + 3] - Yp;
  ydb0[o7 + 3] = e1 * yb1[o7 + 3] - (a1 * Ydp + b1 * Yp);
}

// column sums of sens[m][5] in a fixed order: partials per workgroup, then one workgroup
__global__ void __launch_bounds__(VMS_BLOCK) k_sens_part(int m, const double *sens, double *part) {
  __shared__ double sm[4];
  for (int k = 0; k < 5; ++k) {
    double acc = 0.0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) acc += sens[5 * (int64_t)e + k];
    acc = block_sum(acc, sm);
    if (threadIdx.x == 0) part[5 * blockIdx.x + k] = acc;
  }
}
__global__ void __launch_bounds__(VMS_BLOCK) k_sens_final(int nb, const double *part, double *out) {
  __shared__ double sm[4];
  for (int k = 0; k < 5; ++k) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) acc += part[5 * q + k];
    acc = block_sum(acc, sm);
    if (threadIdx.x == 0) out[k] = acc;
  }
}

struct Bump {
  char *base;
  size_t off = 0;
  template <typename X>
  X *take(int64_t count) {
    off = (off + 255) & ~(size_t)255;
    X *p = base ? (X *)(base + off) : nullptr;
    off += sizeof(X) * (size_t)count;
    return p;
  }
};

int sens_sum(vms_ctx *ctx, int m, const double *sens, double *part, double *dout, double *host_out) {
  int nb = vms_red_blocks(m);
  hipLaunchKernelGGL(k_sens_part, dim3(nb), dim3(VMS_BLOCK), 0, ctx->stream, m, sens, part);
  hipLaunchKernelGGL(k_sens_final, dim3(1), dim3(VMS_BLOCK), 0, ctx->stream, nb, (const double *)part, dout);
  VMS_LAUNCH_CHECK(ctx);
  VMS_HIP(ctx, hipMemcpyAsync(ctx->h_d, dout, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < 5; ++k) host_out[k] = ctx->h_d[k];
  return VMS_OK;
}

size_t sens_bytes(const vms_mesh *mesh) {
  Bump b{nullptr};
  b.take<double>(5 * (int64_t)mesh->n_tets);
  b.take<double>(5 * VMS_MAX_RED_BLOCKS);
  b.take<double>(8);
  return b.off + 256;
}

}  // namespace

int vms_launch_transpose(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, vms_matrix *Kt, bool m32) {
  if (!Kt || !Kt->A || !Kt->B || !Kt->C || !Kt->D)
    return vms_set_error(ctx, VMS_ERR_ARG, "transposed solve: storage for the transposed blocks missing");
  if (m32 && (!Kt->A32 || !Kt->B32 || !Kt->C32 || !Kt->D32))
    return vms_set_error(ctx, VMS_ERR_ARG, "mixed precision needs FP32 storage for the transpose");
  const int64_t nnzb = mesh->nnzb;
  hipLaunchKernelGGL(k_transpose, dim3(grid1(nnzb)), dim3(VMS_BLOCK), 0, ctx->stream, nnzb, mesh->tpos, K->A, K->B,
                     K->C, K->D, Kt->A, Kt->B, Kt->C, Kt->D, m32 ? Kt->A32 : nullptr, m32 ? Kt->B32 : nullptr,
                     m32 ? Kt->C32 : nullptr, m32 ? Kt->D32 : nullptr);
  VMS_LAUNCH_CHECK(ctx);
  Kt->W = K->W;
  return VMS_OK;
}

extern "C" int vms_solve_transpose_scaled(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, vms_matrix *Kt,
                                          const double *rhs_scaled, double *lam_scaled, const vms_solver_opts *opts,
                                          void *workspace, size_t workspace_bytes, vms_solve_stats *stats) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if (!K || !K->A || !K->B || !K->C || !K->D || !Kt || !opts)
    return vms_set_error(ctx, VMS_ERR_ARG, "vms_solve_transpose_scaled: matrix arrays missing");
  vms_matrix T = *Kt;
  if ((rc = vms_launch_transpose(ctx, mesh, K, &T, opts->precision == VMS_MIXED))) return rc;
  return vms_solve_scaled(ctx, mesh, &T, rhs_scaled, lam_scaled, opts, workspace, workspace_bytes, stats);
}

extern "C" int vms_solve_transpose(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, vms_matrix *Kt, const double *g,
                                   double *lam, double eps_diag, const vms_solver_opts *opts, void *workspace,
                                   size_t workspace_bytes, vms_solve_stats *stats) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_solve(ctx, mesh, K, opts, workspace, workspace_bytes, vms_solve_workspace(mesh, opts), stats,
                           "vms_solve_transpose");
  if (rc) return rc;
  if (!g || !lam || !K->W || !Kt) return vms_set_error(ctx, VMS_ERR_ARG, "vms_solve_transpose: missing argument");
  std::memset(stats, 0, sizeof(*stats));
  vms_phase_reset(ctx);
  const auto t0 = std::chrono::steady_clock::now();
  vms_matrix T = *Kt;
  rc = vms_solve_full(ctx, mesh, K, g, nullptr, nullptr, lam, eps_diag, opts, workspace, stats, &T);
  if (rc >= 0) {
    VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    vms_phase_finish(ctx, stats);
  }
  stats->status = rc;
  stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

extern "C" int vms_param_sensitivity(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat,
                                     const vms_timeint *ti, const vms_state *st, const double *dfibre,
                                     const double *lam, int pmask, double *out, void *workspace,
                                     size_t workspace_bytes) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if (!mat || !ti || !st || !lam || !out || !workspace || pmask <= 0 || pmask > 31)
    return vms_set_error(ctx, VMS_ERR_ARG, "vms_param_sensitivity: bad arguments");
  if (workspace_bytes < sens_bytes(mesh)) return vms_set_error(ctx, VMS_ERR_WORKSPACE, "workspace too small");
  Bump b{(char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255)};
  double *sens = b.take<double>(5 * (int64_t)mesh->n_tets);
  double *part = b.take<double>(5 * VMS_MAX_RED_BLOCKS);
  double *dout = b.take<double>(8);
  const vms_ga ga = vms_genalpha(ti);
  if ((rc = vms_launch_clear_inverted(ctx))) return rc;
  if ((rc = vms_launch_assemble(ctx, mesh, mat, ga, st, nullptr, nullptr, nullptr, nullptr, VMS_ASM_SENS, nullptr, 0,
                                lam, nullptr, dfibre, pmask, sens)))
    return rc;
  return sens_sum(ctx, mesh->n_tets, sens, part, dout, out);
}

extern "C" size_t vms_adjoint_workspace(const vms_mesh *mesh, const vms_solver_opts *opts) {
  if (!mesh || !opts || mesh->n_nodes <= 0) return 0;
  Bump b{nullptr};
  const int64_t n = mesh->n_nodes;
  b.take<double>(4 * n);   // rhs
  b.take<double>(4 * n);   // lam*
  b.take<double>(4 * n);   // lam
  b.take<double>(3 * n);   // mu_u
  b.take<double>(11 * n);  // vjp
  // the solver's bases and the assembly's element buffers share one region (used in turn)
  const size_t asm_b = vms_asm_scratch_bytes(mesh, VMS_ASM_TANGENT) > vms_asm_scratch_bytes(mesh, VMS_ASM_VJP)
                           ? vms_asm_scratch_bytes(mesh, VMS_ASM_TANGENT)
                           : vms_asm_scratch_bytes(mesh, VMS_ASM_VJP);
  const size_t sol_b = vms_solve_workspace(mesh, opts);
  return b.off + sens_bytes(mesh) + (sol_b > asm_b ? sol_b : asm_b) + 1024;
}

extern "C" int vms_adjoint_step(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_timeint *ti,
                                const vms_state *st, const double *dfibre, vms_matrix *K, vms_matrix *Kt,
                                const double *ybar1, const double *ydbar1, double *ybar0, double *ydbar0, int pmask,
                                double *dJdtheta, const vms_solver_opts *opts, double eps_diag, void *workspace,
                                size_t workspace_bytes, vms_solve_stats *stats) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if (!mat || !ti || !st || !K || !Kt || !ybar1 || !ydbar1 || !ybar0 || !ydbar0 || !opts || !stats || !workspace ||
      (pmask && !dJdtheta))
    return vms_set_error(ctx, VMS_ERR_ARG, "vms_adjoint_step: missing argument");
  if (workspace_bytes < vms_adjoint_workspace(mesh, opts))
    return vms_set_error(ctx, VMS_ERR_WORKSPACE, "workspace too small");
  const int n = mesh->n_nodes;
  const vms_ga ga = vms_genalpha(ti);
  Bump b{(char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255)};
  double *rhs = b.take<double>(4 * (int64_t)n);
  double *lams = b.take<double>(4 * (int64_t)n);
  double *lam = b.take<double>(4 * (int64_t)n);
  double *mu_u = b.take<double>(3 * (int64_t)n);
  double *vjp = b.take<double>(11 * (int64_t)n);
  double *sens = b.take<double>(5 * (int64_t)mesh->n_tets);
  double *part = b.take<double>(5 * VMS_MAX_RED_BLOCKS);
  double *dout = b.take<double>(8);
  char *sws = b.take<char>(0);
  const size_t sws_bytes = workspace_bytes - (size_t)(sws - (char *)workspace);
  hipStream_t s = ctx->stream;
  const bool m32 = opts->precision == VMS_MIXED;
  // tangent at the converged state, Dirichlet rows, scaling
  if ((rc = vms_launch_clear_inverted(ctx))) return rc;
  if ((rc = vms_launch_assemble(ctx, mesh, mat, ga, st, nullptr, K, nullptr, nullptr, VMS_ASM_TANGENT, sws,
                                sws_bytes)))
    return rc;
  if ((rc = vms_launch_prepare(ctx, mesh, K, nullptr, nullptr, nullptr, eps_diag, 0))) return rc;
  hipLaunchKernelGGL(k_adj_seed, dim3(grid1(n)), dim3(VMS_BLOCK), 0, s, n, ga, mesh->dir_mask, (const double *)K->W,
                     ybar1, ydbar1, rhs, mu_u);
  VMS_LAUNCH_CHECK(ctx);
  // transposed nested solve, lam = W lam*
  vms_matrix Kt2 = *Kt;
  if (!m32) { Kt2.A32 = Kt2.B32 = Kt2.C32 = Kt2.D32 = nullptr; }
  rc = vms_solve_transpose_scaled(ctx, mesh, K, &Kt2, rhs, lams, opts, sws, sws_bytes, stats);
  if (rc < 0) return rc;
  const int solve_rc = rc;
  hipLaunchKernelGGL(k_unscale, dim3(grid1(4 * (int64_t)n)), dim3(VMS_BLOCK), 0, s, 4 * (int64_t)n,
                     (const double *)K->W, (const double *)lams, lam);
  // staged-field cotangents, then y-bar_n, y-dot-bar_n
  if ((rc = vms_launch_assemble(ctx, mesh, mat, ga, st, nullptr, nullptr, nullptr, nullptr, VMS_ASM_VJP, sws,
                                sws_bytes, lam, vjp)))
    return rc;
  hipLaunchKernelGGL(k_adj_back, dim3(grid1(n)), dim3(VMS_BLOCK), 0, s, n, ga, mesh->dir_mask, (const double *)mu_u,
                     (const double *)vjp, ybar1, ybar0, ydbar0);
  VMS_LAUNCH_CHECK(ctx);
  if (pmask) {
    if ((rc = vms_launch_assemble(ctx, mesh, mat, ga, st, nullptr, nullptr, nullptr, nullptr, VMS_ASM_SENS, nullptr,
                                  0, lam, nullptr, dfibre, pmask, sens)))
      return rc;
    double g[5];
    if ((rc = sens_sum(ctx, mesh->n_tets, sens, part, dout, g))) return rc;
    for (int k = 0; k < 5; ++k)
      if (pmask & (1 << k)) dJdtheta[k] -= g[k];
  }
  VMS_HIP(ctx, hipMemcpyAsync(ctx->h_i, &ctx->dstat->inverted, sizeof(int), hipMemcpyDeviceToHost, s));
  VMS_HIP(ctx, hipStreamSynchronize(s));
  if (ctx->h_i[0]) return vms_set_error(ctx, VMS_ERR_INVERTED_ELEMENT, "element with J <= 0");
  return solve_rc;
}
