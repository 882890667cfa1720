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

#define VMS_MAX_TIMED 65536   // timed launches per kind between two reads

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
};

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
                      const double *W, const double *x);
int vms_launch_predictor(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, double t_np1,
                         vms_state *st);
int vms_launch_spmv(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, int op,
                    const void *x, void *y, int fp32);
