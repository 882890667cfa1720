// Context management and the thin C-ABI wrappers around the assembly kernels.
#include <cstring>

#include <atomic>
#include <mutex>

#include "vms_internal.h"

// Workspace of vms_step_noalloc: one static device array per GPU, held from the
// code object's load until the process ends.  In host code `scratch` names a
// host-side stand-in; its device address comes from hipGetSymbolAddress, taken
// once per device in vms_ctx_create with that device current.
static __device__ __align__(256) unsigned char scratch[VMS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_call_mu[kMaxDevices];
}  // namespace

// device address of this device's scratch array (the current device must be `device`)
static int scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return VMS_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VMS_ERR_HIP;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return VMS_OK;
}

int vms_set_error(vms_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

static void ctx_free(vms_ctx *c) {
  for (int k = 0; k < 2; ++k)
    for (hipEvent_t e : c->tev[k]) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ph.ev) (void)hipEventDestroy(e);
  if (c->tflag) (void)hipFree(c->tflag);
  if (c->dstat) (void)hipFree(c->dstat);
  if (c->h_i) (void)hipHostFree(c->h_i);
  if (c->h_d) (void)hipHostFree(c->h_d);
  if (c->h_post) (void)hipHostFree((void *)c->h_post);
  delete c;
}

extern "C" int vms_ctx_create(vms_ctx **out, int device, void *stream) {
  if (!out) return VMS_ERR_ARG;
  *out = nullptr;
  vms_ctx *c = new vms_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return VMS_ERR_HIP;
  }
  // everything the context owns on the device is allocated here: the status area, the per-launch
  // flags of the A-product launch timing and the events of the phase timing
  bool ok = hipMalloc((void **)&c->dstat, sizeof(vms_dev_status)) == hipSuccess &&
            hipMalloc((void **)&c->tflag, 2 * VMS_MAX_TIMED * sizeof(int)) == hipSuccess &&
            hipHostMalloc((void **)&c->h_i, 64 * sizeof(int32_t), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&c->h_d, 64 * sizeof(double), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&c->h_post, 64 * sizeof(int32_t), hipHostMallocCoherent | hipHostMallocMapped) ==
                hipSuccess;
  if (ok) {
    c->ph.ev.reserve(2 * VMS_PHASE_EVENTS);
    for (int k = 0; k < 2 * VMS_PHASE_EVENTS && ok; ++k) {
      hipEvent_t e;
      ok = hipEventCreate(&e) == hipSuccess;
      if (ok) c->ph.ev.push_back(e);
    }
  }
  if (ok) {
    for (int q = 0; q < 64; ++q) c->h_post[q] = 0;
    ok = hipMemset(c->dstat, 0, sizeof(vms_dev_status)) == hipSuccess &&
         hipMemset(c->tflag, 0, 2 * VMS_MAX_TIMED * sizeof(int)) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
  }
  if (ok && device < kMaxDevices) ok = scratch_address(device, &c->scratch) == VMS_OK;
  if (!ok) {
    ctx_free(c);
    return VMS_ERR_HIP;
  }
  vms_phase_reset(c);
  *out = c;
  return VMS_OK;
}

extern "C" void vms_ctx_destroy(vms_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  ctx_free(ctx);
}

// ---- phase timing of the solver --------------------------------------------------
void vms_phase_reset(vms_ctx *ctx) {
  vms_phase_timer &t = ctx->ph;
  t.free_pairs.clear();
  for (int k = (int)t.ev.size() / 2 - 1; k >= 0; --k) t.free_pairs.push_back(k);
  t.pending.clear();
  for (double &m : t.ms) m = 0.0;
  t.complete = true;
}

// fold every pending pair whose stop event has completed into ms[] (all of them when wait is set)
static void phase_harvest(vms_ctx *ctx, bool wait) {
  vms_phase_timer &t = ctx->ph;
  size_t keep = 0;
  for (size_t i = 0; i < t.pending.size(); ++i) {
    const auto p = t.pending[i];
    hipEvent_t e0 = t.ev[2 * p.pair], e1 = t.ev[2 * p.pair + 1];
    bool done = wait ? hipEventSynchronize(e1) == hipSuccess : hipEventQuery(e1) == hipSuccess;
    if (!done) {
      if (wait) t.complete = false;
      else { t.pending[keep++] = p; continue; }
    } else {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) t.ms[p.kind] += ms;
      else t.complete = false;
    }
    t.free_pairs.push_back(p.pair);
  }
  t.pending.resize(keep);
}

int vms_phase_begin(vms_ctx *ctx) {
  vms_phase_timer &t = ctx->ph;
  if (t.free_pairs.empty()) phase_harvest(ctx, false);
  if (t.free_pairs.empty()) {
    t.complete = false;
    return -1;
  }
  const int pair = t.free_pairs.back();
  if (hipEventRecord(t.ev[2 * pair], ctx->stream) != hipSuccess) {
    t.complete = false;
    return -1;
  }
  t.free_pairs.pop_back();
  return pair;
}

void vms_phase_end(vms_ctx *ctx, int pair, int kind) {
  if (pair < 0) return;
  vms_phase_timer &t = ctx->ph;
  if (hipEventRecord(t.ev[2 * pair + 1], ctx->stream) != hipSuccess) {
    t.complete = false;
    t.free_pairs.push_back(pair);   // its start event is harmless
    return;
  }
  t.pending.push_back({pair, kind});
}

void vms_phase_finish(vms_ctx *ctx, vms_solve_stats *stats) {
  phase_harvest(ctx, true);
  const vms_phase_timer &t = ctx->ph;
  stats->ms_scale = t.ms[VMS_PH_SCALE];
  stats->ms_setup = t.ms[VMS_PH_SETUP];
  stats->ms_outer = t.ms[VMS_PH_OUTER];
  stats->ms_A = t.ms[VMS_PH_A];
  stats->ms_S = t.ms[VMS_PH_S];
  stats->ms_inner = t.ms[VMS_PH_INNER];
  stats->phases_timed = t.complete ? 1 : 0;
}

// ---- low-latency flag readback ---------------------------------------------------
// One thread copies the flags, then (after a system-scope fence) the sequence
// number, into the coherent host buffer.
__global__ void k_post_flags(const int *dev, volatile int32_t *host, int32_t seq) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < 4; ++q) host[1 + q] = dev[q];
  __threadfence_system();
  host[0] = seq;
}

int vms_wait_post(vms_ctx *ctx, int32_t seq, const int *dev) {
  for (long spin = 0;; ++spin) {
    if (ctx->h_post[0] == seq) {
      std::atomic_thread_fence(std::memory_order_acquire);
      for (int q = 0; q < 4; ++q) ctx->h_i[q] = ctx->h_post[1 + q];
      return VMS_OK;
    }
    if ((spin & 1023) == 1023) {   // now and then: has the stream failed, or drained without the post?
      const hipError_t e = hipStreamQuery(ctx->stream);
      if (e != hipErrorNotReady) {
        if (e != hipSuccess)
          return vms_set_error(ctx, VMS_ERR_HIP, "stream failed: %s", hipGetErrorString(e));
        if (ctx->h_post[0] == seq) continue;
        // drained but the post is not visible: read the flags the ordinary way
        VMS_HIP(ctx, hipMemcpyAsync(ctx->h_i, dev, 4 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return VMS_OK;
      }
    }
  }
}

int vms_read_flags(vms_ctx *ctx, const int *dev) {
  const int32_t seq = ++ctx->post_seq;
  hipLaunchKernelGGL(k_post_flags, dim3(1), dim3(64), 0, ctx->stream, dev, ctx->h_post, seq);
  VMS_LAUNCH_CHECK(ctx);
  return vms_wait_post(ctx, seq, dev);
}

// ---- launch timing of the A-block product --------------------------------------
vms_timed vms_timer_next(vms_ctx *ctx, int kind) {
  vms_timed t;
  if (!ctx->timing || ctx->tused[kind] >= VMS_MAX_TIMED) return t;
  const int i = ctx->tused[kind];
  auto &ev = ctx->tev[kind];
  while ((int)ev.size() < 2 * (i + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return t;
    ev.push_back(e);
  }
  ctx->tused[kind] = i + 1;
  t.slot = i;
  t.worked = ctx->tflag + (int64_t)kind * VMS_MAX_TIMED + i;
  t.e0 = ev[2 * i];
  t.e1 = ev[2 * i + 1];
  return t;
}

extern "C" int vms_ctx_set_timing(vms_ctx *ctx, int enable) {
  if (!ctx) return VMS_ERR_ARG;
  VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  VMS_HIP(ctx, hipMemset(ctx->tflag, 0, 2 * VMS_MAX_TIMED * sizeof(int)));
  ctx->tused[0] = ctx->tused[1] = 0;
  ctx->timing = enable != 0;
  return VMS_OK;
}

extern "C" int vms_ctx_kernel_time(vms_ctx *ctx, int kind, double *ms_total, int64_t *launches) {
  if (!ctx || kind < 0 || kind > 1 || !ms_total || !launches) return VMS_ERR_ARG;
  *ms_total = 0.0;
  *launches = 0;
  if (!ctx->timing) return vms_set_error(ctx, VMS_ERR_STATE, "vms_ctx_kernel_time: launch timing is off");
  VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int used = ctx->tused[kind];
  if (used == 0) return VMS_OK;
  std::vector<int> flag(used);
  VMS_HIP(ctx, hipMemcpy(flag.data(), ctx->tflag + (int64_t)kind * VMS_MAX_TIMED, used * sizeof(int),
                         hipMemcpyDeviceToHost));
  for (int i = 0; i < used; ++i) {
    if (!flag[i]) continue;   // the level had converged: the kernel returned at once
    float ms = 0.0f;
    VMS_HIP(ctx, hipEventElapsedTime(&ms, ctx->tev[kind][2 * i], ctx->tev[kind][2 * i + 1]));
    *ms_total += ms;
    ++*launches;
  }
  VMS_HIP(ctx, hipMemset(ctx->tflag + (int64_t)kind * VMS_MAX_TIMED, 0, used * sizeof(int)));
  ctx->tused[kind] = 0;
  return VMS_OK;
}

extern "C" const char *vms_last_error(const vms_ctx *ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

static int check_state(vms_ctx *ctx, const vms_state *st) {
  if (!st || !st->u_n || !st->p_n || !st->v_n || !st->du_n || !st->dp_n || !st->dv_n || !st->u || !st->p ||
      !st->v || !st->du || !st->dp || !st->dv)
    return vms_set_error(ctx, VMS_ERR_ARG, "incomplete state");
  return VMS_OK;
}

extern "C" int vms_predictor(vms_ctx *ctx, const vms_mesh *mesh, const vms_timeint *ti, vms_state *st,
                             int dir_lift) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if ((rc = check_state(ctx, st))) return rc;
  if (!ti || !(ti->dt > 0.0)) return vms_set_error(ctx, VMS_ERR_ARG, "bad time-integration parameters");
  const vms_ga ga = vms_genalpha(ti);
  if (dir_lift != 0 && dir_lift != 1) return vms_set_error(ctx, VMS_ERR_ARG, "dir_lift must be 0 or 1");
  return vms_launch_predictor(ctx, mesh, ga, ti->t_n + ti->dt, st, dir_lift);
}

extern "C" size_t vms_assemble_workspace(const vms_mesh *mesh, unsigned flags) {
  if (!mesh || mesh->n_tets < 0) return 0;
  return vms_asm_scratch_bytes(mesh, flags & 7u);
}

extern "C" int vms_assemble(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_timeint *ti,
                            const vms_state *st, const double *f_ext, vms_matrix *K, double *R, double *corr,
                            unsigned flags, void *workspace, size_t workspace_bytes) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if ((rc = check_state(ctx, st))) return rc;
  if (!mat || !ti || !(ti->dt > 0.0)) return vms_set_error(ctx, VMS_ERR_ARG, "material/timeint missing");
  if ((flags & VMS_ASM_RESIDUAL) && !R) return vms_set_error(ctx, VMS_ERR_ARG, "R missing");
  if ((flags & VMS_ASM_RKCORR) && !corr) return vms_set_error(ctx, VMS_ERR_ARG, "corr missing");
  if ((flags & VMS_ASM_TANGENT) && (!K || !K->A || !K->B || !K->C || !K->D))
    return vms_set_error(ctx, VMS_ERR_ARG, "K arrays missing");
  if ((flags & 7u) == 0 || (flags & ~7u)) return vms_set_error(ctx, VMS_ERR_ARG, "bad assembly flags");
  const vms_ga ga = vms_genalpha(ti);
  if ((rc = vms_launch_clear_inverted(ctx))) return rc;
  rc = vms_launch_assemble(ctx, mesh, mat, ga, st, f_ext, K, R, corr, flags, workspace, workspace_bytes);
  if (rc) return rc;
  VMS_HIP(ctx, hipMemcpyAsync(ctx->h_i, &ctx->dstat->inverted, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->h_i[0]) return vms_set_error(ctx, VMS_ERR_INVERTED_ELEMENT, "element with J <= 0");
  return VMS_OK;
}

extern "C" int vms_residual_norm(vms_ctx *ctx, const vms_mesh *mesh, const vms_timeint *ti, const vms_state *st,
                                 const double *R, double *norm_host) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if ((rc = check_state(ctx, st))) return rc;
  if (!ti || !R || !norm_host) return vms_set_error(ctx, VMS_ERR_ARG, "vms_residual_norm: bad arguments");
  const vms_ga ga = vms_genalpha(ti);
  if ((rc = vms_launch_norm(ctx, mesh, ga, st, R))) return rc;
  VMS_HIP(ctx, hipMemcpyAsync(ctx->h_d, &ctx->dstat->norm2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *norm_host = sqrt(ctx->h_d[0]);
  if (!std::isfinite(*norm_host)) return vms_set_error(ctx, VMS_ERR_NAN, "residual norm is not finite");
  return VMS_OK;
}

extern "C" int vms_prepare_system(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *R,
                                  const double *corr, double *rhs_scaled, double eps_diag, int mirror32) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if (rhs_scaled && !R) return vms_set_error(ctx, VMS_ERR_ARG, "R missing");
  return vms_launch_prepare(ctx, mesh, K, R, corr, rhs_scaled, eps_diag, mirror32);
}

extern "C" int vms_newton_update(vms_ctx *ctx, const vms_mesh *mesh, const vms_timeint *ti, vms_state *st,
                                 const double *W, const double *x_scaled, int dir_lift) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if ((rc = check_state(ctx, st))) return rc;
  if (!ti || !x_scaled) return vms_set_error(ctx, VMS_ERR_ARG, "vms_newton_update: bad arguments");
  const vms_ga ga = vms_genalpha(ti);
  if (dir_lift != 0 && dir_lift != 1) return vms_set_error(ctx, VMS_ERR_ARG, "dir_lift must be 0 or 1");
  return vms_launch_update(ctx, mesh, ga, st, W, x_scaled, dir_lift);
}

// ---- allocation-free time step ----------------------------------------------------
extern "C" size_t vms_noalloc_scratch_bytes(void) { return (size_t)VMS_NOALLOC_SCRATCH_BYTES; }

extern "C" int vms_step_noalloc(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_timeint *ti,
                                vms_state *st, const double *f_ext, vms_matrix *K, const vms_newton_opts *nopts,
                                const vms_solver_opts *sopts, vms_step_stats *stats) {
  if (!ctx) return VMS_ERR_ARG;
  if (!mesh || !sopts) return vms_set_error(ctx, VMS_ERR_ARG, "vms_step_noalloc: missing argument");
  if (!ctx->scratch) return vms_set_error(ctx, VMS_ERR_STATE, "vms_step_noalloc: no device scratch on this context");
  // launch timing creates its events on demand; this entry point creates nothing
  if (ctx->timing) return vms_set_error(ctx, VMS_ERR_STATE, "vms_step_noalloc: launch timing is on");
  const size_t need = vms_step_workspace(mesh, sopts);
  if (need == 0) return vms_set_error(ctx, VMS_ERR_ARG, "vms_step_noalloc: empty mesh");
  if (need > (size_t)VMS_NOALLOC_SCRATCH_BYTES)
    return vms_set_error(ctx, VMS_ERR_WORKSPACE,
                         "vms_step_noalloc: the step needs %zu bytes of workspace, the static scratch holds %zu",
                         need, (size_t)VMS_NOALLOC_SCRATCH_BYTES);
  // one call at a time per device from this process's host threads; calls on other streams
  // still race on the device (documented in the header)
  std::lock_guard<std::mutex> lk(g_scratch_call_mu[ctx->device]);
  return vms_step(ctx, mesh, mat, ti, st, f_ext, K, nopts, sopts, ctx->scratch, (size_t)VMS_NOALLOC_SCRATCH_BYTES,
                  stats);
}
