// Internal declarations shared by the HIP translation units of libvms.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "vms.h"

#define VMS_BLOCK 256
#define VMS_MAX_RED_BLOCKS 1024
// internal assembly mode: cotangents lam^T dR/d(staged fields), [n][11] = (u 3, p, v 3, v-dot 3, p-dot)
#define VMS_ASM_VJP 8u
// internal assembly mode: per-element lam_e^T dR_e/dtheta, [m][5] for (mu, kappa, k1, k2, phi)
#define VMS_ASM_SENS 16u

// Small device-side status area owned by a context (allocated at create).
struct vms_dev_status {
  int inverted;        // an element had J <= 0 (sticky until cleared)
  int pad0;
  int pad1;
  int pad2;
  double norm2;        // result of the residual-norm reduction
  double part[VMS_MAX_RED_BLOCKS];
};

#define VMS_AMG_MODES 10      // near-null modes per aggregate (coarse dofs per coarse node)

// device arrays of one multigrid level (fixed per mesh; amg_setup.cpp)
struct vms_amg_level_dev {
  int32_t n = 0, bs = 3;
  int64_t nnzb = 0;                     // level 0: the mesh's slots; level >= 1: CSR blocks
  const int32_t *ptr = nullptr, *col = nullptr, *brow = nullptr, *dpos = nullptr;   // level >= 1
  const uint8_t *dropped = nullptr;     // level >= 1: [n * 10], coarse dofs without a mode
  const int32_t *agg = nullptr, *mptr = nullptr, *mem = nullptr;   // to the next level
  const double *P = nullptr;            // [n][bs][10]
  const float *P32 = nullptr;
  const int32_t *gptr = nullptr, *gsrc = nullptr;   // Galerkin lists of the next level's blocks
};
struct vms_amg_dev {
  int n_levels = 0, degree = 2, coarse_degree = 8, mid_degree = 2, uploaded = 0, device = -1;
  vms_amg_level_dev lev[VMS_AMG_MAX_LEVELS];
};
const vms_amg_dev *vms_amg_device(const vms_amg *amg);

#define VMS_MAX_TIMED 65536   // timed launches per kind between two reads
#define VMS_PHASE_EVENTS 1024 // event pairs of the solver's phase timing (created with the context)

// Phases of a solve timed with HIP events (vms_solve_stats.ms_*)
enum { VMS_PH_SCALE = 0, VMS_PH_SETUP, VMS_PH_OUTER, VMS_PH_A, VMS_PH_S, VMS_PH_INNER, VMS_PH_N };

// Device time of nested solver phases: begin() records a start event on the
// context stream, end() the stop event; completed pairs are folded into ms[]
// as their stop events finish (harvest), all of them at finish().  The
// events come from a fixed pool created with the context; when every pair is
// in flight a phase goes untimed and `complete` turns false.
struct vms_phase_timer {
  std::vector<hipEvent_t> ev;      // 2 * VMS_PHASE_EVENTS, pair k = (ev[2k], ev[2k+1])
  std::vector<int> free_pairs;
  struct open_t { int pair, kind; };
  std::vector<open_t> pending;     // stop recorded, not yet folded in
  double ms[VMS_PH_N] = {};
  bool complete = true;
};

struct vms_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  vms_dev_status *dstat = nullptr;   // device
  int32_t *h_i = nullptr;            // pinned host scratch (ints)
  double *h_d = nullptr;             // pinned host scratch (doubles)
  int est_A = 8, est_I = 8, est_S = 8;  // Krylov iteration estimates (batching)
  // launch timing of the A-block product (vms_ctx_set_timing): per kind (0 FP64, 1 FP32) a pool of
  // event pairs and a device flag per launch that the kernel sets when it did work
  bool timing = false;
  std::vector<hipEvent_t> tev[2];
  int tused[2] = {0, 0};
  int *tflag = nullptr;              // device [2][VMS_MAX_TIMED]
  // low-latency flag readback: a one-thread kernel copies a level's flags and a
  // sequence number into pinned coherent host memory, the host spins on it
  volatile int32_t *h_post = nullptr;   // [8]: seq, flags[4]
  int32_t post_seq = 0;
  vms_phase_timer ph;
  void *scratch = nullptr;           // device address of this device's static scratch (vms_step_noalloc)
};

// Phase timing of the solver (see vms_phase_timer): reset before a solve,
// begin/end around a phase (begin returns -1 when no event pair is free;
// end(-1) is a no-op), finish after the stream has drained.
void vms_phase_reset(vms_ctx *ctx);
int vms_phase_begin(vms_ctx *ctx);
void vms_phase_end(vms_ctx *ctx, int pair, int kind);
void vms_phase_finish(vms_ctx *ctx, vms_solve_stats *stats);

// Read the 4 ints at dev (device) into ctx->h_i once every earlier kernel of
// the stream has finished, by the low-latency path (falls back to a stream
// synchronisation if the posted sequence number does not arrive).
int vms_read_flags(vms_ctx *ctx, const int *dev);
// Wait until sequence number seq has been posted to ctx->h_post by a kernel
// already enqueued, then copy the posted flags to ctx->h_i (on a failed or
// drained stream: as vms_read_flags, reading the flags at dev).
int vms_wait_post(vms_ctx *ctx, int32_t seq, const int *dev);

// Next timed launch of the A-block product (kind 0 FP64, 1 FP32) when timing
// is on: the start/stop events that the launch passes to hipExtLaunchKernelGGL
// (they take the kernel's own start and end times) and its work flag;
// slot < 0 when timing is off or the pool is full.
struct vms_timed {
  int slot = -1;
  int *worked = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};
vms_timed vms_timer_next(vms_ctx *ctx, int kind);

int vms_set_error(vms_ctx *ctx, int code, const char *fmt, ...);

#define VMS_HIP(ctx, call)                                                          \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return vms_set_error((ctx), VMS_ERR_HIP, "%s failed: %s (%s:%d)", #call,      \
                           hipGetErrorString(e_), __FILE__, __LINE__);              \
  } while (0)

#define VMS_LAUNCH_CHECK(ctx) VMS_HIP(ctx, hipGetLastError())

// ---------------------------------------------------------------------------
// device helpers

// Workgroups of a launch are handed to the 8 XCDs round-robin; remap the
// hardware block id so that each XCD processes one contiguous slab of rows
// (better reuse of gathered vector entries in that XCD's L2).
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int full = (nblocks / 8) * 8;
  if (bid >= full) return bid;
  return (bid & 7) * (nblocks >> 3) + (bid >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread block; every thread receives the same value.
// Fixed order, hence deterministic.
__device__ __forceinline__ double block_sum(double v, double *sm) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  const double r = (sm[0] + sm[1]) + (sm[2] + sm[3]);
  __syncthreads();
  return r;
}

inline int vms_red_blocks(int64_t n) {
  int64_t nb = (n + 2 * VMS_BLOCK - 1) / (2 * VMS_BLOCK);
  if (nb < 1) nb = 1;
  if (nb > VMS_MAX_RED_BLOCKS) nb = VMS_MAX_RED_BLOCKS;
  return (int)nb;
}

// ---------------------------------------------------------------------------
// launchers implemented in assembly.hip / linalg.hip, used by solver.hip

struct vms_ga {   // generalized-alpha constants
  double am, af, gm, dt, c2, c3, load;
};
vms_ga vms_genalpha(const vms_timeint *ti);

int vms_check_mesh(vms_ctx *ctx, const vms_mesh *m);
// Bytes of element buffers the assembly needs for these flags.
size_t vms_asm_scratch_bytes(const vms_mesh *mesh, unsigned flags);
int vms_launch_assemble(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat,
                        const vms_ga &ga, const vms_state *st, const double *f_ext,
                        vms_matrix *K, double *R, double *corr, unsigned flags,
                        void *scratch, size_t scratch_bytes,
                        const double *lam = nullptr, double *vjp = nullptr, const double *dfibre = nullptr,
                        int pmask = 0, double *sens = nullptr);
int vms_launch_clear_inverted(vms_ctx *ctx);
int vms_launch_norm(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, const vms_state *st,
                    const double *R);
int vms_launch_prepare(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *R,
                       const double *corr, double *rhs, double eps_diag, int mirror32);
int vms_launch_update(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, vms_state *st,
                      const double *W, const double *x, int lift);
int vms_launch_predictor(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, double t_np1,
                         vms_state *st, int lift);
int vms_launch_spmv(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, int op,
                    const void *x, void *y, int fp32);
// Kt = blocks of K^T (FP32 copies too when m32)
int vms_launch_transpose(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, vms_matrix *Kt, bool m32);

// ---------------------------------------------------------------------------
// the nested solve shared by the entry points of solver.hip and adjoint.hip

// argument checks common to the solve entry points (need: the workspace bytes they require)
int vms_check_solve(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, const vms_solver_opts *opts,
                    const void *workspace, size_t workspace_bytes, size_t need, const vms_solve_stats *stats,
                    const char *who);
// bytes of the nested solve's own workspace (Krylov bases, control blocks, temporaries)
size_t vms_solve_core_bytes(const vms_mesh *mesh, const vms_solver_opts *opts);
// (scaled K) x = rhs by the nested solver; fills the iteration counts, residuals and phase events of
// stats (the caller resets the phase timer and finishes it)
int vms_solve_core(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, const double *rhs, double *x,
                   const vms_solver_opts *opts, void *ws, vms_solve_stats *stats);
// Dirichlet rows and scaling of K in place, rhs* = W(-R + corr) (R given) or W g (g given), the
// nested solve of W K W (Kt == NULL) or of its transpose (blocks written to Kt), delta = W x*.
// Workspace: rhs*, x*, then the nested solve's (vms_solve_workspace bytes).
int vms_solve_full(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *g, const double *R,
                   const double *corr, double *delta, double eps_diag, const vms_solver_opts *opts, void *workspace,
                   vms_solve_stats *stats, vms_matrix *Kt);
