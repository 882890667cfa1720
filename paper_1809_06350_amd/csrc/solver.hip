// Nested block-preconditioned Krylov solver (section 4) and the time step
// driver (section 3.3).
//
// Levels (section 4.4):
//   outer         FGMRES on the scaled K* = [[A, B], [C, D]], FP64, right-
//                 preconditioned by the Schur complement reduction (Alg. 1;
//                 or its partial factorizations, or SIMPLE of section 4.3);
//   intermediate  GMRES or CG on A (3x3 block-Jacobi right preconditioner,
//                 the stand-in for the paper's AMG) and GMRES on
//                 S = D - C A^-1 B (right preconditioner from
//                 S^ = D - C diag(A)^-1 B: diag(S^)^-1, a Chebyshev
//                 polynomial, or a fixed number of CG steps on S^);
//   inner         GMRES or CG on A inside the matrix-free Schur product
//                 (Alg. 2); CG is the inner solver the conclusions suggest.
// Every level starts from x0 = 0 and stops on ||r|| <= max(rtol ||b||, atol)
// (GMRES: its least-squares residual) or at maxit.
//
// Device-resident Krylov: the Hessenberg matrix, Givens rotations, CG
// scalars and the convergence flags live in a per-level control block in
// device memory; the kernels of an iteration read the `done` flag and return
// immediately once the level has converged, so the host can enqueue several
// A-level iterations before it reads the flags back (posted by the last
// kernel of a batch into pinned host memory).  GMRES orthogonalisation is
// classical Gram-Schmidt -- one multi-dot and one multi-update pass per
// iteration (CGS1), a second pass always (CGS2) or when the first removed
// more than half of the vector ("if needed") -- or modified Gram-Schmidt
// (one dot/axpy launch pair per basis vector).  The outer FGMRES always uses
// CGS2 (or MGS).
//
// Mixed form: the intermediate and inner levels run on FP32 copies of the
// scaled blocks with FP32 Krylov vectors (FP64 accumulation of every sum and
// FP64 Hessenberg/Givens/CG scalars); the outer FGMRES, its vectors and the
// Newton update stay FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "linalg.h"
#include "vms_internal.h"

namespace {

enum { PC_NONE = 0, PC_BJ33 = 1, PC_DIAG = 2 };

// Arnoldi vector kernels: 1024-thread workgroups, at most 256 of them (their
// partials are reduced inside the consuming kernel)
#define KRY_BLOCK 1024
#define KRY_MAX_BLOCKS 256
inline int kry_blocks(int64_t nvec) {
  int64_t nb = (nvec + 2 * KRY_BLOCK - 1) / (2 * KRY_BLOCK);
  return (int)std::min<int64_t>(std::max<int64_t>(nb, 1), KRY_MAX_BLOCKS);
}
enum { KS_OK = 0, KS_MAXIT = 1, KS_NAN = 2, KS_BREAKDOWN = 3 };
enum { IF_DONE = 0, IF_ITS = 1, IF_STATUS = 2 };

struct KOff {
  int m;
  int64_t H, cs, sn, g, y, h1, h2, scal, pn, pn2, part;
};

inline KOff make_off(int m) {
  KOff o;
  o.m = m;
  int64_t p = 0;
  o.H = p; p += (int64_t)(m + 1) * m;
  o.cs = p; p += m;
  o.sn = p; p += m;
  o.g = p; p += m + 1;
  o.y = p; p += m;
  o.h1 = p; p += m + 1;
  o.h2 = p; p += m + 1;
  o.scal = p; p += 8;
  o.pn = p; p += VMS_MAX_RED_BLOCKS;
  o.pn2 = p; p += VMS_MAX_RED_BLOCKS;
  o.part = p; p += (int64_t)(m + 1) * VMS_MAX_RED_BLOCKS;
  return o;
}
inline int64_t ctrl_doubles(int m) {
  KOff o = make_off(m);
  return o.part + (int64_t)(m + 1) * VMS_MAX_RED_BLOCKS;
}

template <typename T>
__device__ __forceinline__ double dl(const T *p, int64_t i) { return (double)p[i]; }

// ---- reductions ------------------------------------------------------------
// Every reduction writes one partial per workgroup (part[blk * ld + k]) and a
// separate single-workgroup kernel sums them in a fixed order: no atomics and
// no device-scope fences (on a multi-XCD device those write back the L2),
// deterministic results; the kernel boundary makes the partials visible.

// partial sums of ||b||^2
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_norm_part(int64_t nvec, const T *__restrict__ b, double *part, const int *iflag) {
  if (iflag && iflag[IF_DONE]) return;
  __shared__ double sm[4];
  double acc = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nvec; r += (int64_t)gridDim.x * blockDim.x) {
    const double v = dl(b, r);
    acc += v * v;
  }
  acc = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__device__ __forceinline__ double sum_partials1(const double *part, int nb, double *sm) {
  double s = 0.0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x) s += part[q];
  return block_sum(s, sm);
}

// V_j = w / scale; Z_j = M^-1 V_j (block-Jacobi 3x3 or point diagonal)
template <typename T>
__device__ __forceinline__ void scale_and_precond(int64_t nvec, const T *w, double inv, T *V, T *Z, int pc,
                                                  const T *pcd) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (pc == PC_BJ33) {
    const int64_t nn = nvec / 3;
    for (int64_t i = t0; i < nn; i += stride) {
      const T v0 = (T)(dl(w, 3 * i) * inv), v1 = (T)(dl(w, 3 * i + 1) * inv), v2 = (T)(dl(w, 3 * i + 2) * inv);
      V[3 * i] = v0; V[3 * i + 1] = v1; V[3 * i + 2] = v2;
      const T *M = pcd + 9 * i;
      const double a0 = (double)v0, a1 = (double)v1, a2 = (double)v2;
      Z[3 * i] = (T)(dl(M, 0) * a0 + dl(M, 1) * a1 + dl(M, 2) * a2);
      Z[3 * i + 1] = (T)(dl(M, 3) * a0 + dl(M, 4) * a1 + dl(M, 5) * a2);
      Z[3 * i + 2] = (T)(dl(M, 6) * a0 + dl(M, 7) * a1 + dl(M, 8) * a2);
    }
  } else {
    for (int64_t r = t0; r < nvec; r += stride) {
      const T vv = (T)(dl(w, r) * inv);
      V[r] = vv;
      if (pc == PC_DIAG) Z[r] = (T)(dl(pcd, r) * (double)vv);
    }
  }
}

// Relative tolerance of a level: rtol, or -- for the inner A-solve of a Schur
// product with relaxation on (relax = the Schur level's control scalars: its
// initial residual norm and current estimate) -- rtol * ||r_0|| / ||r_k|| of
// the Schur level, at most max(rtol, RELAX_MAX).
#ifndef RELAX_MAX
#define RELAX_MAX 1e-2
#endif
__device__ __forceinline__ double relaxed_rtol(double rtol, const double *relax) {
  if (!relax) return rtol;
  const double r0 = relax[0], rk = relax[2];
  if (!(rk > 0.0) || !(r0 > rk)) return rtol;
  return fmin(rtol * (r0 / rk), fmax(rtol, RELAX_MAX));
}

// Start of a level: beta = ||b|| from the k_norm_part partials (every
// workgroup reduces them in the same order), V_0 = b / beta, Z_0 = M^-1 V_0;
// workgroup 0 also sets the tolerance, g_0 and the level flags.
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_kinit(int64_t nvec, const T *__restrict__ b, T *V0, T *Z0, double *ctrl, KOff off, int *iflag, int nb,
        double rtol, double atol, int pc, const T *pcd, const double *relax) {
  __shared__ double sm[4];
  const double beta = sqrt(sum_partials1(ctrl + off.part, nb, sm));
  const bool done = !isfinite(beta) || beta == 0.0 || beta <= atol;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl[off.scal + 0] = beta;
    ctrl[off.scal + 1] = fmax(relaxed_rtol(rtol, relax) * beta, atol);
    ctrl[off.scal + 2] = beta;
    ctrl[off.g] = beta;
    iflag[IF_ITS] = 0;
    iflag[IF_STATUS] = isfinite(beta) ? KS_OK : KS_NAN;
    iflag[IF_DONE] = done ? 1 : 0;
  }
  if (done) return;
  scale_and_precond(nvec, b, 1.0 / beta, V0, Z0, pc, pcd);
}

// sum of the nbp (<= KRY_MAX_BLOCKS) partials p[0], p[ld], ... in a fixed order
__device__ __forceinline__ double kry_sum_partials(const double *p, int nbp, int ld, double *sm) {
  double v = (threadIdx.x < (unsigned)nbp) ? p[(int64_t)threadIdx.x * ld] : 0.0;
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < nw; ++q) r += sm[q];
  __syncthreads();
  return r;
}

// Workgroup total of one value per thread, in a fixed order; every thread
// receives it. Lets a kernel load its partials, issue its first streaming
// loads, and only then reduce.
__device__ __forceinline__ double kry_block_total(double v, double *sm) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < nw; ++q) r += sm[q];
  __syncthreads();
  return r;
}
// Reorthogonalisation test of the "if needed" mode (Daniel-Gragg-Kaufman-
// Stewart with eta^2 = 1/2): after the first pass w' = w - V h, a second pass
// is needed when ||w'||^2 < (||w'||^2 + ||h||^2) / 2, i.e. when more than half
// of ||w||^2 was removed.  Every kernel of the step evaluates it from the same
// data in the same order, so they all take the same decision.
__device__ __forceinline__ bool kry_need_reorth(const double *ctrl, const KOff &off, int nbp, int nk, double *sm) {
  const double w2 = kry_sum_partials(ctrl + off.pn, nbp, 1, sm);
  double hh = 0.0;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) hh += ctrl[off.h1 + k] * ctrl[off.h1 + k];
  hh = wave_sum(hh);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[w] = hh;
  __syncthreads();
  double h2 = 0.0;
  for (int q = 0; q < nw; ++q) h2 += sm[q];
  __syncthreads();
  return w2 < 0.5 * (w2 + h2);
}

// partial dots <V_k, w>, k < nk, eight basis vectors per pass over the rows;
// one partial per workgroup (up to 16 wavefronts), summed over the waves in
// wave order
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_mdot_part(int64_t nvec, const T *__restrict__ V, int nk, const T *__restrict__ w, double *part, int ld,
            const int *iflag, const double *sel_ctrl = nullptr, KOff sel_off = KOff{}, int sel_nbp = 0) {
  if (iflag[IF_DONE]) return;
  __shared__ double sm[16][8];
  if (sel_ctrl && !kry_need_reorth(sel_ctrl, sel_off, sel_nbp, nk, &sm[0][0])) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int k0 = 0; k0 < nk; k0 += 8) {
    const int kk = min(8, nk - k0);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const T *Vk = V + (int64_t)k0 * nvec;
    for (int64_t r = t0; r < nvec; r += stride) {
      const double wr = dl(w, r);
      // every load unconditional (slots q >= kk read basis vector k0 again and
      // are not used), so that the eight loads are issued together
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = dl(Vk, (int64_t)(q < kk ? q : 0) * nvec + r);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < kk) acc[q] += v[q] * wr;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double v = wave_sum(acc[q]);
      if (lane == 0) sm[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kk) {
      double t = 0.0;
      for (int q = 0; q < nw; ++q) t += sm[q][threadIdx.x];
      part[(int64_t)blockIdx.x * ld + k0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// ---- fused Arnoldi kernels (classical Gram-Schmidt) ------------------------
// Workgroups of KRY_BLOCK threads, at most KRY_MAX_BLOCKS of them, so that a
// consumer can reduce the producer's partials itself: every workgroup sums
// the same partials in the same fixed order and obtains identical values,
// which removes a separate finalize launch per reduction.

// cs[k] = sum_b part[b * ld + k] for k < nk: 16 coefficients per round, the
// partials split over 64 thread groups and combined by a fixed binary tree
// (needs exactly KRY_BLOCK = 1024 threads)
__device__ __forceinline__ void kry_reduce_coefs(const double *part, int nbp, int ld, int nk, double *cs,
                                                 double (*red)[17]) {
  const int kl = threadIdx.x & 15, bg = threadIdx.x >> 4;   // bg < 64 for 1024 threads
  for (int k0 = 0; k0 < nk; k0 += 16) {
    const int k = k0 + kl;
    double a = 0.0;
    if (k < nk)
      for (int b = bg; b < nbp; b += 64) a += part[(int64_t)b * ld + k];
    red[bg][kl] = a;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
      if (bg < h) red[bg][kl] += red[bg + h][kl];
      __syncthreads();
    }
    if (bg == 0 && k < nk) cs[k] = red[0][kl];
    __syncthreads();
  }
}

// w -= sum_k h_k V_k with h reduced in-kernel from the k_mdot_part partials;
// workgroup 0 stores h (Hessenberg column part); with NORM also the partial
// sums of the updated ||w||^2 (pn[blockIdx.x])
template <typename T, bool NORM>
__global__ void __launch_bounds__(KRY_BLOCK)
k_mupdate_fin(int64_t nvec, const T *__restrict__ V, int nk, T *w, const double *part, int nbp, int ld,
              double *hout, double *pn, const int *iflag, const double *sel_ctrl = nullptr, KOff sel_off = KOff{}) {
  if (iflag[IF_DONE]) return;
  __shared__ double cs[1024];
  __shared__ double red[64][17];
  __shared__ double sm[16];
  if (sel_ctrl && !kry_need_reorth(sel_ctrl, sel_off, nbp, nk, sm)) return;
  kry_reduce_coefs(part, nbp, ld, nk, cs, red);
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < nk; k += blockDim.x) hout[k] = cs[k];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double ss = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nvec; r += stride) {
    // eight basis vectors per round, every load unconditional (slots past nk
    // read vector k0 again and are not used) so that they are issued together;
    // term k goes to accumulator k mod 4
    const double wr = dl(w, r);
    double a[4] = {0, 0, 0, 0};
    for (int k0 = 0; k0 < nk; k0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = dl(V, (int64_t)(k0 + q < nk ? k0 + q : k0) * nvec + r);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q < nk) a[q & 3] += cs[k0 + q] * v[q];
    }
    const T out = (T)(wr - ((a[0] + a[1]) + (a[2] + a[3])));
    w[r] = out;
    if (NORM) ss += (double)out * (double)out;
  }
  if (!NORM) return;
  ss = wave_sum(ss);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[wv] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += sm[q];
    pn[blockIdx.x] = t;
  }
}

// out[k] = sum_b part[b * ld + k]: a workgroup owns 16 consecutive k (16-wide
// coalesced segments) and splits the partials over 16 groups of threads with
// four independent accumulators each; fixed combination order.
#define FIN_K 16
__global__ void __launch_bounds__(VMS_BLOCK)
k_dot_finalize(const double *part, int nb, int ld, int nk, double *out, const int *iflag) {
  if (iflag[IF_DONE]) return;
  __shared__ double sm[16][FIN_K + 1];
  const int kl = threadIdx.x & (FIN_K - 1), bg = threadIdx.x / FIN_K;
  const int k = blockIdx.x * FIN_K + kl;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  if (k < nk) {
    int b = bg;
    for (; b + 48 < nb; b += 64) {
      a0 += part[(int64_t)b * ld + k];
      a1 += part[(int64_t)(b + 16) * ld + k];
      a2 += part[(int64_t)(b + 32) * ld + k];
      a3 += part[(int64_t)(b + 48) * ld + k];
    }
    for (; b < nb; b += 16) a0 += part[(int64_t)b * ld + k];
  }
  sm[bg][kl] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (bg == 0 && k < nk) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += sm[q][kl];
    out[k] = t;
  }
}

// w -= sum_k coef[k] V_k (four independent partial sums per row); with NORM
// also the partial sums of the updated ||w||^2
template <typename T, bool NORM>
__global__ void __launch_bounds__(VMS_BLOCK)
k_mupdate(int64_t nvec, const T *__restrict__ V, int nk, T *w, const double *coef, double *part, const int *iflag) {
  if (iflag[IF_DONE]) return;
  __shared__ double cs[256];
  __shared__ double sm[4];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double ss = 0.0;
  for (int c0 = 0; c0 < nk; c0 += 256) {
    const int kn = min(256, nk - c0);
    __syncthreads();
    if (threadIdx.x < kn) cs[threadIdx.x] = coef[c0 + threadIdx.x];
    __syncthreads();
    const bool last = (c0 + 256 >= nk);
    const T *Vc = V + (int64_t)c0 * nvec;
    for (int64_t r = t0; r < nvec; r += stride) {
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      int k = 0;
      for (; k + 4 <= kn; k += 4) {
        a0 += cs[k] * dl(Vc, (int64_t)k * nvec + r);
        a1 += cs[k + 1] * dl(Vc, (int64_t)(k + 1) * nvec + r);
        a2 += cs[k + 2] * dl(Vc, (int64_t)(k + 2) * nvec + r);
        a3 += cs[k + 3] * dl(Vc, (int64_t)(k + 3) * nvec + r);
      }
      for (; k < kn; ++k) a0 += cs[k] * dl(Vc, (int64_t)k * nvec + r);
      const T out = (T)(dl(w, r) - ((a0 + a1) + (a2 + a3)));
      w[r] = out;
      if (NORM && last) ss += (double)out * (double)out;
    }
  }
  if (!NORM) return;
  ss = block_sum(ss, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = ss;
}

// finish Arnoldi step j (one thread): Hessenberg column (h1, plus h2 after a
// reorthogonalisation pass), h_{j+1,j} = ||w|| = hn, previous rotations, new
// Givens rotation, least-squares residual |g_{j+1}|, flags
__device__ void givens_update(double *ctrl, const KOff &off, int *iflag, int j, int nsum, int maxit, double hn) {
  const int m1 = off.m + 1;
  double *col = ctrl + off.H + (int64_t)j * m1;
  double *cs = ctrl + off.cs, *sn = ctrl + off.sn, *g = ctrl + off.g;
  if (nsum == 1)
    for (int i = 0; i <= j; ++i) col[i] = ctrl[off.h1 + i];
  else if (nsum == 2)
    for (int i = 0; i <= j; ++i) col[i] = ctrl[off.h1 + i] + ctrl[off.h2 + i];
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  double c = 1.0, sv = 0.0;
  if (den > 0.0) { c = col[j] / den; sv = col[j + 1] / den; }
  cs[j] = c;
  sn[j] = sv;
  col[j] = den;
  col[j + 1] = 0.0;
  g[j + 1] = -sv * g[j];
  g[j] = c * g[j];
  const double res = fabs(g[j + 1]);
  ctrl[off.scal + 2] = res;
  ctrl[off.scal + 3] = hn;
  iflag[IF_ITS] = j + 1;
  if (!isfinite(res) || !isfinite(hn)) {
    iflag[IF_STATUS] = KS_NAN;
    iflag[IF_DONE] = 1;
  } else if (den == 0.0) {
    iflag[IF_STATUS] = KS_BREAKDOWN;
    iflag[IF_ITS] = j;   // singular column: keep the previous iterate
    iflag[IF_DONE] = 1;
  } else if (res <= ctrl[off.scal + 1] || hn == 0.0) {
    iflag[IF_STATUS] = KS_OK;
    iflag[IF_DONE] = 1;
  } else if (j + 1 >= maxit) {
    iflag[IF_STATUS] = KS_MAXIT;
    iflag[IF_DONE] = 1;
  }
}

// Copy the level flags, then (after a system-scope fence) the sequence number,
// into the coherent host buffer the host spins on.
__device__ __forceinline__ void post_flags(const int *iflag, volatile int32_t *post, int32_t seq) {
  for (int q = 0; q < 4; ++q) post[1 + q] = iflag[q];
  __threadfence_system();
  post[0] = seq;
}

// MGS path: Hessenberg column already in place, ||w||^2 partials in part
__global__ void __launch_bounds__(VMS_BLOCK)
k_givens(int nb, double *ctrl, KOff off, int *iflag, int j, int maxit) {
  if (iflag[IF_DONE]) return;
  __shared__ double sm[4];
  const double s = sum_partials1(ctrl + off.part, nb, sm);
  if (threadIdx.x == 0) givens_update(ctrl, off, iflag, j, 0, maxit, sqrt(s));
}

// CGS path: h_{j+1,j} = ||w|| from the k_mupdate_fin norm partials (reduced by
// every workgroup), V_{j+1} = w / h_{j+1,j}, Z_{j+1} = M^-1 V_{j+1}; thread 0
// of workgroup 0 also finishes the Givens step.  nsum: 1 = one pass (h1,
// norm partials pn), 2 = two passes (h1 + h2, pn2), 3 = decide as the
// "if needed" test does.  (Workgroups that start after
// it has set the done flag skip the normalisation, whose result is then not
// used.)
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_normalize_givens(int64_t nvec, const T *__restrict__ w, T *V1, T *Z1, double *ctrl, KOff off, int *iflag, int nbp,
                   int j, int nsum, int maxit, int pc, const T *pcd, volatile int32_t *post, int32_t seq) {
  __shared__ double sm[16];
  __shared__ int done0;   // one read per workgroup: workgroup 0 may set the flag during this kernel
  if (threadIdx.x == 0) done0 = iflag[IF_DONE];
  __syncthreads();
  if (done0) {
    if (post && blockIdx.x == 0 && threadIdx.x == 0) post_flags(iflag, post, seq);
    return;
  }
  if (nsum == 3) nsum = kry_need_reorth(ctrl, off, nbp, j + 1, sm) ? 2 : 1;   // "if needed" mode
  const double *pn = ctrl + (nsum == 2 ? off.pn2 : off.pn);
  const double pl = (threadIdx.x < (unsigned)nbp) ? pn[threadIdx.x] : 0.0;
  if (pc != PC_BJ33) {
    const double hn = sqrt(kry_block_total(pl, sm));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      givens_update(ctrl, off, iflag, j, nsum, maxit, hn);
      if (post) post_flags(iflag, post, seq);   // the host may decide while the normalisation runs
    }
    scale_and_precond(nvec, w, hn > 0.0 ? 1.0 / hn : 0.0, V1, Z1, pc, pcd);
    return;
  }
  // block-Jacobi: the first node's w and M^-1 block are loaded while the partials are reduced
  const int64_t nn = nvec / 3, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double fw[3] = {0, 0, 0}, fm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (i0 < nn) {
#pragma unroll
    for (int c = 0; c < 3; ++c) fw[c] = dl(w, 3 * i0 + c);
#pragma unroll
    for (int e = 0; e < 9; ++e) fm[e] = dl(pcd, 9 * i0 + e);
  }
  const double hn = sqrt(kry_block_total(pl, sm));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    givens_update(ctrl, off, iflag, j, nsum, maxit, hn);
    if (post) post_flags(iflag, post, seq);   // the host may decide while the normalisation runs
  }
  const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int64_t i = i0; i < nn; i += stride) {
    const bool pre = (i == i0);
    const T v0 = (T)((pre ? fw[0] : dl(w, 3 * i)) * inv), v1 = (T)((pre ? fw[1] : dl(w, 3 * i + 1)) * inv),
            v2 = (T)((pre ? fw[2] : dl(w, 3 * i + 2)) * inv);
    V1[3 * i] = v0; V1[3 * i + 1] = v1; V1[3 * i + 2] = v2;
    double M[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) M[e] = pre ? fm[e] : dl(pcd, 9 * i + e);
    const double a0 = (double)v0, a1 = (double)v1, a2 = (double)v2;
    Z1[3 * i] = (T)(M[0] * a0 + M[1] * a1 + M[2] * a2);
    Z1[3 * i + 1] = (T)(M[3] * a0 + M[4] * a1 + M[5] * a2);
    Z1[3 * i + 2] = (T)(M[6] * a0 + M[7] * a1 + M[8] * a2);
  }
}

// MGS step k: w -= H[k-1,j] V_{k-1} (k > 0), then partial dots <w, V_k>
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_mgs_part(int64_t nvec, const T *__restrict__ V, int k, T *w, const double *hprev_p, double *part,
           const int *iflag) {
  if (iflag[IF_DONE]) return;
  __shared__ double sm[4];
  const double hprev = (k > 0) ? *hprev_p : 0.0;
  const T *Vp = V + (int64_t)(k > 0 ? k - 1 : 0) * nvec;
  const T *Vk = V + (int64_t)k * nvec;
  double acc = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nvec; r += (int64_t)gridDim.x * blockDim.x) {
    double wr = dl(w, r);
    if (k > 0) {
      const T u = (T)(wr - hprev * dl(Vp, r));
      w[r] = u;
      wr = (double)u;
    }
    acc += wr * dl(Vk, r);
  }
  acc = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_normalize(int64_t nvec, const T *__restrict__ w, T *V1, T *Z1, const double *ctrl, KOff off, const int *iflag,
            int pc, const T *pcd) {
  if (iflag[IF_DONE]) return;
  scale_and_precond(nvec, w, 1.0 / ctrl[off.scal + 3], V1, Z1, pc, pcd);
}

// y = R^-1 g (column-oriented back substitution on the rotated Hessenberg)
__global__ void __launch_bounds__(VMS_BLOCK) k_trisolve(double *ctrl, KOff off, const int *iflag) {
  __shared__ double gs[1024];
  const int k = iflag[IF_ITS];
  const int m1 = off.m + 1;
  const double *H = ctrl + off.H;
  double *y = ctrl + off.y;
  for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = ctrl[off.g + i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double yi = gs[i] / H[(int64_t)i * m1 + i];
    __syncthreads();
    for (int l = threadIdx.x; l < i; l += blockDim.x) gs[l] -= H[(int64_t)i * m1 + l] * yi;
    if (threadIdx.x == 0) y[i] = yi;
    __syncthreads();
  }
}

// x = sum_{l < its} y_l Z_l
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_combine(int64_t nvec, const T *__restrict__ Z, const double *ctrl, KOff off, const int *iflag, T *x) {
  __shared__ double ys[64];
  const int k = iflag[IF_ITS];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t r = t0; r < nvec; r += stride) x[r] = (T)0;
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int kn = min(64, k - c0);
    __syncthreads();
    if (threadIdx.x < kn) ys[threadIdx.x] = ctrl[off.y + c0 + threadIdx.x];
    __syncthreads();
    for (int64_t r = t0; r < nvec; r += stride) {
      double acc = (c0 == 0) ? 0.0 : dl(x, r);
      for (int l = 0; l < kn; ++l) acc += ys[l] * dl(Z, (int64_t)(c0 + l) * nvec + r);
      x[r] = (T)acc;
    }
  }
}

// Back substitution and x = sum_l y_l Z_l in one kernel for short bases: every
// workgroup solves the (its x its) triangular system in LDS (same order, same
// result) before its rows of the combination.
#define COMBINE_SOLVE_MAX 64
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_solve_combine(int64_t nvec, const T *__restrict__ Z, const double *ctrl, KOff off, const int *iflag, T *x) {
  __shared__ double gs[COMBINE_SOLVE_MAX];
  __shared__ double ys[COMBINE_SOLVE_MAX];
  const int k = iflag[IF_ITS];
  const int m1 = off.m + 1;
  const double *H = ctrl + off.H;
  if (threadIdx.x < k) gs[threadIdx.x] = ctrl[off.g + threadIdx.x];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) ys[i] = gs[i] / H[(int64_t)i * m1 + i];
    __syncthreads();
    if (threadIdx.x < i) gs[threadIdx.x] -= H[(int64_t)i * m1 + threadIdx.x] * ys[i];
    __syncthreads();
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nvec; r += stride) {
    double acc = 0.0;
    for (int l = 0; l < k; ++l) acc += ys[l] * dl(Z, (int64_t)l * nvec + r);
    x[r] = (T)acc;
  }
}

// ---- preconditioner setup --------------------------------------------------
// inverse of the 3x3 diagonal blocks of the scaled A
template <typename T>
__global__ void k_bj33_setup(int n, const int32_t *diag_pos, int64_t nnzb, const double *A, T *Minv, int sym) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = diag_pos[i];
  double a[9];
  for (int e = 0; e < 9; ++e) a[e] = A[e * nnzb + b];
  if (sym) {   // inverse of the symmetric part of the diagonal block
    for (int r = 0; r < 3; ++r)
      for (int c = r + 1; c < 3; ++c) a[3 * r + c] = a[3 * c + r] = 0.5 * (a[3 * r + c] + a[3 * c + r]);
  }
  const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  const double id = (det != 0.0) ? 1.0 / det : 0.0;
  double inv[9];
  inv[0] = c00 * id;
  inv[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  inv[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  inv[3] = c01 * id;
  inv[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  inv[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  inv[6] = c02 * id;
  inv[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  inv[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  for (int e = 0; e < 9; ++e) Minv[9 * (int64_t)i + e] = (T)inv[e];
}

// ---- conjugate gradients on the symmetrised A --------------------------------
// The paper's conclusions suggest symmetrising the inner A system and solving
// it by CG.  A_s = (A + A^T)/2 is formed on the block pattern: block (i,j)
// and the transpose of block (j,i) (slot tpos) are averaged entry by entry in
// FP64 and stored in the level precision.  Padding slots (tpos = self, zero
// values) stay zero.
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_sym_A(int64_t nnzb, const int32_t *__restrict__ tpos, const double *__restrict__ A, T *As) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int64_t t = tpos[b];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      As[(3 * r + c) * nnzb + b] = (T)(0.5 * (A[(3 * r + c) * nnzb + b] + A[(3 * c + r) * nnzb + t]));
}

// Sum of nbp partials (any count) by one workgroup in a fixed order; every
// thread receives the same value.
__device__ __forceinline__ double cg_sum_partials(const double *p, int nbp, double *sm) {
  double v = 0.0;
  for (int q = threadIdx.x; q < nbp; q += blockDim.x) v += p[q];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < nw; ++q) r += sm[q];
  __syncthreads();
  return r;
}

// Two sums over a 1024-thread workgroup (fixed order), written by thread 0.
__device__ __forceinline__ void cg_block_sums2(double a, double b, double *pa, double *pb, double (*sm)[16]) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) { sm[0][w] = a; sm[1][w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int q = 0; q < nw; ++q) { ta += sm[0][q]; tb += sm[1][q]; }
    *pa = ta;
    *pb = tb;
  }
}

// z = M^-1 r for one node (3x3 block-Jacobi), rounded to T
template <typename T>
__device__ __forceinline__ void bj33_apply(const T *M, const double r[3], T z[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) z[c] = (T)(dl(M, 3 * c) * r[0] + dl(M, 3 * c + 1) * r[1] + dl(M, 3 * c + 2) * r[2]);
}

// CG start with x0 = 0: r = b, z = M^-1 r, x = 0, and the partials of <r,z>
// and <r,r> (one per workgroup); resets the level flags.
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_cg_init(int64_t nn, const T *__restrict__ b, T *x, T *r, T *z, const T *__restrict__ Minv, double *prz,
          double *prr, int *iflag) {
  __shared__ double sm[2][16];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    iflag[IF_DONE] = 0;
    iflag[IF_ITS] = 0;
    iflag[IF_STATUS] = KS_OK;
  }
  double rz = 0.0, rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nn; i += stride) {
    double rv[3];
    T zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rv[c] = dl(b, 3 * i + c);
      r[3 * i + c] = (T)rv[c];
      x[3 * i + c] = (T)0;
    }
    bj33_apply(Minv + 9 * i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[3 * i + c] = zv[c];
      rz += rv[c] * (double)zv[c];
      rr += rv[c] * rv[c];
    }
  }
  cg_block_sums2(rz, rr, prz + blockIdx.x, prr + blockIdx.x, sm);
}

// CG iteration j, first half.  Every workgroup sums the partials of
// rz_j = <r_j, z_j> and rr_j = <r_j, r_j> and takes the same decision: stop
// when ||r_j|| <= max(rtol ||b||, atol) (or at maxit, or on NaN); workgroup 0
// records the flags (and posts them to host memory when asked).  Otherwise,
// with beta_j = rz_j / rz_{j-1} (beta_0 = 0), w = A z_j is formed and the
// rows' own entries of p_j = z_j + beta_j p_{j-1} and
// q_j = A p_j = w + beta_j q_{j-1} are updated in place (only z is gathered),
// with one partial of <p_j, q_j> per workgroup.  Layout of the A-block product
// (16 lanes per row, 16 rows per workgroup); a workgroup takes a contiguous
// range of row groups (XCD-aware order) when the grid is capped.  The cap is
// 8 resident 256-thread workgroups on each of the 256 CUs, so the capped grid
// runs as one wave: the FP64 instance is held to 8 waves per SIMD (at most 64
// VGPRs; with 7 resident the last 256 workgroups would run as a second, nearly
// empty wave).  In FP64 the row's own z, p, q are loaded after the product
// loop: held across it they push the kernel past that bound, and the compiler
// then recycles registers between the matrix loads and waits after each one
// instead of keeping all of a row group's loads in flight.
#ifndef CG_SPMV_BLOCKS
#define CG_SPMV_BLOCKS 2048
#endif
inline int cg_spmv_blocks(int n) {
  const int ng = (n + SPMV_ROWS_PER_BLOCK - 1) / SPMV_ROWS_PER_BLOCK;
  return std::max(1, std::min(ng, CG_SPMV_BLOCKS));
}
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 8 : 1)))
k_cg_spmv(int n, int64_t nnzb, int W, const int32_t *__restrict__ col, const T *__restrict__ A,
          const T *__restrict__ z, T *p, T *q, double *ctrl, KOff off, double *ppart, int *iflag, int j, int nbk,
          double rtol, double atol, int maxit, volatile int32_t *post, int32_t seq, int *worked,
          const double *relax) {
  __shared__ double sm[16];
  __shared__ int done0;
  if (threadIdx.x == 0) done0 = iflag[IF_DONE];
  __syncthreads();
  if (done0) {
    if (post && blockIdx.x == 0 && threadIdx.x == 0) post_flags(iflag, post, seq);
    return;
  }
  const double rz = cg_sum_partials(ctrl + off.pn, nbk, sm);
  const double rr = cg_sum_partials(ctrl + off.pn2, nbk, sm);
  const double rn = sqrt(rr);
  const double tol = (j == 0) ? fmax(relaxed_rtol(rtol, relax) * rn, atol) : ctrl[off.scal + 1];
  const bool bad = !isfinite(rr) || !isfinite(rz);
  const bool conv = !bad && rn <= tol;
  const bool stop = bad || conv || j >= maxit;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (j == 0) {
      ctrl[off.scal + 0] = rn;
      ctrl[off.scal + 1] = tol;
    }
    ctrl[off.scal + 2] = rn;
    ctrl[off.scal + 3 + (j & 1)] = rz;   // rz_j; rz_{j-1} sits in the other slot
    if (stop) {
      iflag[IF_ITS] = j;
      iflag[IF_STATUS] = bad ? KS_NAN : (conv ? KS_OK : KS_MAXIT);
      iflag[IF_DONE] = 1;
    }
    if (post) post_flags(iflag, post, seq);
  }
  if (stop) return;
  if (worked && blockIdx.x == 0 && threadIdx.x == 0) *worked = 1;   // launch timing: this launch did the product
  const bool first = (j == 0);
  const double beta = first ? 0.0 : rz / ctrl[off.scal + 3 + ((j - 1) & 1)];
  constexpr bool NT = sizeof(T) == 8;
  constexpr bool LATE = sizeof(T) == 8;
  const int lane = threadIdx.x & 15, sub = threadIdx.x >> 4;
  const int ng = (n + SPMV_ROWS_PER_BLOCK - 1) / SPMV_ROWS_PER_BLOCK;
  const int vb = xcd_block(blockIdx.x, gridDim.x);   // even split: every workgroup gets floor or ceil(ng / grid)
  const int g0 = (int)((int64_t)vb * ng / gridDim.x), g1 = (int)((int64_t)(vb + 1) * ng / gridDim.x);
  double pq = 0.0;
  // FP64, rows of 16 slots: one block per lane, and the next group's column index is requested
  // before this group's gathers, so a group waits for one load latency (A and z together), not two
  const bool pf = LATE && W == 16;
  int cnext = 0;
  if (pf && g0 < g1) {
    const int row = g0 * SPMV_ROWS_PER_BLOCK + sub;
    cnext = row < n ? ldc<NT>(col, 16 * (int64_t)row + lane) : 0;
  }
  for (int g = g0; g < g1; ++g) {
    const int row = g * SPMV_ROWS_PER_BLOCK + sub;
    const bool act = row < n;
    const int b0 = act ? W * row : 0, b1 = act ? b0 + W : 0;
    // lanes 0-2 own component `lane` of the row: its z, p, q are loaded ahead of the
    // product in FP32 and after it in FP64 (LATE)
    const bool own = act && lane < 3;
    const int64_t oc = 3 * (int64_t)(act ? row : 0) + (lane < 3 ? lane : 0);
    double zc = 0.0, pc = 0.0, qc = 0.0;
    if (!LATE && own) {
      zc = ld(z, oc);
      if (!first) { pc = ld(p, oc); qc = ld(q, oc); }
    }
    double a0 = 0, a1 = 0, a2 = 0;
    if (pf) {
      const int64_t o = 3 * (int64_t)cnext;
      if (g + 1 < g1) {
        const int rn = row + SPMV_ROWS_PER_BLOCK;
        cnext = rn < n ? ldc<NT>(col, 16 * (int64_t)rn + lane) : 0;
      }
      if (act) {
        const int b = b0 + lane;
        const double x0 = ld(z, o), x1 = ld(z, o + 1), x2 = ld(z, o + 2);
        a0 = ldm<NT>(A, 0 * nnzb + b) * x0 + ldm<NT>(A, 1 * nnzb + b) * x1 + ldm<NT>(A, 2 * nnzb + b) * x2;
        a1 = ldm<NT>(A, 3 * nnzb + b) * x0 + ldm<NT>(A, 4 * nnzb + b) * x1 + ldm<NT>(A, 5 * nnzb + b) * x2;
        a2 = ldm<NT>(A, 6 * nnzb + b) * x0 + ldm<NT>(A, 7 * nnzb + b) * x1 + ldm<NT>(A, 8 * nnzb + b) * x2;
      }
    } else {
      for (int b = b0 + lane; b < b1; b += 16) {
        const int64_t o = 3 * (int64_t)ldc<NT>(col, b);
        const double x0 = ld(z, o), x1 = ld(z, o + 1), x2 = ld(z, o + 2);
        a0 += ldm<NT>(A, 0 * nnzb + b) * x0 + ldm<NT>(A, 1 * nnzb + b) * x1 + ldm<NT>(A, 2 * nnzb + b) * x2;
        a1 += ldm<NT>(A, 3 * nnzb + b) * x0 + ldm<NT>(A, 4 * nnzb + b) * x1 + ldm<NT>(A, 5 * nnzb + b) * x2;
        a2 += ldm<NT>(A, 6 * nnzb + b) * x0 + ldm<NT>(A, 7 * nnzb + b) * x1 + ldm<NT>(A, 8 * nnzb + b) * x2;
      }
    }
    if (LATE && own) {
      zc = ld(z, oc);
      if (!first) { pc = ld(p, oc); qc = ld(q, oc); }
    }
    a0 = reduce16(a0);
    a1 = reduce16(a1);
    a2 = reduce16(a2);
    if (own) {
      const double w = lane == 0 ? a0 : (lane == 1 ? a1 : a2);
      const T pn = first ? (T)zc : (T)(zc + beta * pc);
      const T qn = first ? (T)w : (T)(w + beta * qc);
      p[oc] = pn;
      q[oc] = qn;
      pq += (double)pn * (double)qn;
    }
  }
  pq = block_sum(pq, sm);
  if (threadIdx.x == 0) ppart[blockIdx.x] = pq;
}

// CG iteration j, second half: alpha = rz_j / <p_j, q> (partials summed by
// every workgroup), x += alpha p_j, r -= alpha q, z = M^-1 r, and the
// partials of <r,z> and <r,r> for the next iteration's test.  A non-positive
// <p, A_s p> ends the level (status breakdown; x keeps the last iterate).
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_cg_update(int64_t nn, T *x, T *r, T *z, const T *__restrict__ p, const T *__restrict__ q,
            const T *__restrict__ Minv, double *ctrl, KOff off, const double *ppart, int nps, int *iflag, int j) {
  __shared__ double sm[2][16];
  __shared__ int done0;
  if (threadIdx.x == 0) done0 = iflag[IF_DONE];
  __syncthreads();
  if (done0) return;
  const double pq = cg_sum_partials(ppart, nps, sm[0]);
  const double alpha = ctrl[off.scal + 3 + (j & 1)] / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      iflag[IF_ITS] = j;
      iflag[IF_STATUS] = isfinite(pq) ? KS_BREAKDOWN : KS_NAN;
      iflag[IF_DONE] = 1;
    }
    return;
  }
  double rz = 0.0, rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nn; i += stride) {
    // every load of the node before any store (x and r are not restrict: loads
    // placed after their stores would be issued only once the stores are done)
    double xo[3], po[3], ro[3], qo[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t o = 3 * i + c;
      xo[c] = dl(x, o);
      po[c] = dl(p, o);
      ro[c] = dl(r, o);
      qo[c] = dl(q, o);
    }
    double rv[3];
    T xn[3], rt[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xn[c] = (T)(xo[c] + alpha * po[c]);
      rt[c] = (T)(ro[c] - alpha * qo[c]);
      rv[c] = (double)rt[c];
    }
    bj33_apply(Minv + 9 * i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] = xn[c];
      r[3 * i + c] = rt[c];
      z[3 * i + c] = zv[c];
      rz += rv[c] * (double)zv[c];
      rr += rv[c] * rv[c];
    }
  }
  cg_block_sums2(rz, rr, ctrl + off.pn + blockIdx.x, ctrl + off.pn2 + blockIdx.x, sm);
}

// ---- CG with the preconditioner applied by separate kernels (the multigrid V-cycle) -----------
// The iteration is the one above with z = M^-1 r formed between the update and the product: an
// update kernel (x += alpha p, r -= alpha q), the V-cycle r -> z, the partials of <r,z> and
// <r,r>, then k_cg_spmv, which reads those partials, tests convergence and forms p and q.

// start: r = b, x = 0, the level flags reset
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_cgx_init(int64_t nn, const T *__restrict__ b, T *x, T *r, int *iflag) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    iflag[IF_DONE] = 0;
    iflag[IF_ITS] = 0;
    iflag[IF_STATUS] = KS_OK;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * nn; i += stride) {
    r[i] = b[i];
    x[i] = (T)0;
  }
}

// partials of <r,z> and <r,r> (one per workgroup, the layout k_cg_spmv reads)
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_cgx_rz(int64_t nn, const T *__restrict__ r, const T *__restrict__ z, double *prz, double *prr, const int *iflag) {
  __shared__ double sm[2][16];
  if (iflag[IF_DONE]) return;
  double rz = 0.0, rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nn; i += stride) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double rv = dl(r, 3 * i + c);
      rz += rv * dl(z, 3 * i + c);
      rr += rv * rv;
    }
  }
  cg_block_sums2(rz, rr, prz + blockIdx.x, prr + blockIdx.x, sm);
}

// second half of iteration j without the preconditioner: alpha = rz_j / <p_j, q>, x += alpha p,
// r -= alpha q (a non-positive <p, A p> ends the level, as in k_cg_update)
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_cgx_update(int64_t nn, T *x, T *r, const T *__restrict__ p, const T *__restrict__ q, double *ctrl, KOff off,
             const double *ppart, int nps, int *iflag, int j) {
  __shared__ double sm[16];
  __shared__ int done0;
  if (threadIdx.x == 0) done0 = iflag[IF_DONE];
  __syncthreads();
  if (done0) return;
  const double pq = cg_sum_partials(ppart, nps, sm);
  const double alpha = ctrl[off.scal + 3 + (j & 1)] / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      iflag[IF_ITS] = j;
      iflag[IF_STATUS] = isfinite(pq) ? KS_BREAKDOWN : KS_NAN;
      iflag[IF_DONE] = 1;
    }
    return;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * nn; i += stride) {
    const double xo = dl(x, i), po = dl(p, i), ro = dl(r, i), qo = dl(q, i);
    x[i] = (T)(xo + alpha * po);
    r[i] = (T)(ro - alpha * qo);
  }
}

#include "amg.h"

// ---- CG steps on S^ as the Schur-level preconditioner ---------------------------
// A fixed number k of diag(S^)-preconditioned CG steps on S^ z = v from
// z = 0: for each right-hand side the Krylov-optimal polynomial of degree k,
// where the Chebyshev option applies one fixed polynomial.  The result
// depends nonlinearly on v, which the flexible Schur-level GMRES (it keeps
// the Z vectors) tolerates.  The steps use the pipelined recurrences of
// Ghysels and Vanroose (2014), equivalent to CG in exact arithmetic: the
// product n = S^ m is a plain kernel with no reduction, and one vector kernel
// per step reduces the previous step's <r,u> and <w,u>, updates every vector
// and forms the next step's partials.  A zero or non-finite <r,u> or a
// non-positive curvature ends the steps early (x keeps the last iterate); the
// host never waits on them.

// Off-diagonal part of row ro of S^ times z: lane l of the row's 16 takes
// slots l, l + 16, l + 32, l + 48 of each 64-slot segment (four column loads
// and four gathers in flight per lane).  With sorted columns the 16 lanes of
// one gather touch neighbouring columns; giving each lane four consecutive
// slots instead (one vector load each for columns and values) measured
// slower, since each gather instruction then spans the whole row.  The
// columns come as 2-byte offsets from the row when so != NULL (a quarter of
// the FP32 product's bytes saved), else as 4-byte indices.
template <typename T, bool OFF>
__device__ __forceinline__ double shat_row_dot_t(int W2, const int32_t *__restrict__ sc,
                                                 const int16_t *__restrict__ so, const T *__restrict__ S,
                                                 const T *__restrict__ z, int64_t r0, int ro, int lane) {
  double a = 0.0;
  for (int q0 = 0; q0 < W2; q0 += 64) {
    int c[4];
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = OFF ? ro + (int)so[r0 + q0 + lane + 16 * u] : sc[r0 + q0 + lane + 16 * u];
      v[u] = ld(S, r0 + q0 + lane + 16 * u);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) a += v[u] * ld(z, c[u]);
  }
  return a;
}
template <typename T>
__device__ __forceinline__ double shat_row_dot(int W2, const int32_t *__restrict__ sc,
                                               const int16_t *__restrict__ so, const T *__restrict__ S,
                                               const T *__restrict__ z, int ro, int lane) {
  const int64_t r0 = (int64_t)W2 * ro;
  return so ? shat_row_dot_t<T, true>(W2, sc, so, S, z, r0, ro, lane)
            : shat_row_dot_t<T, false>(W2, sc, so, S, z, r0, ro, lane);
}

// y = S^ x (off-diagonal distance-2 slots plus the diagonal), skipped when
// *done is set.  LPR lanes per row, each taking the slots lane + LPR u of
// every 64-slot segment; specialised for 64-slot rows and for 2-byte offsets.
// 8 lanes per row measured fastest in FP32 (22.7 against 24.5 us at 64^3),
// 16 in FP64 (8: same).
template <typename T, int LPR, bool OFF, int W2F>
__global__ void __launch_bounds__(VMS_BLOCK)
k_shat_spmv(int n, int W2rt, const int32_t *__restrict__ sc, const int16_t *__restrict__ so, const T *__restrict__ S,
            const T *__restrict__ Sd, const T *__restrict__ x, T *y, const int *done, const double *rpa,
            const double *rpb, int nred, double *rtot) {
  if (done && *done) return;
  if (rpa && blockIdx.x == 0) {
    // the totals of the previous CG step's two partial sums (fixed order), for the next vector step
    __shared__ double sm[2][VMS_BLOCK / 64];
    double ta = 0.0, tb = 0.0;
    for (int q = threadIdx.x; q < nred; q += VMS_BLOCK) {
      ta += rpa[q];
      tb += rpb[q];
    }
    ta = wave_sum(ta);
    tb = wave_sum(tb);
    if ((threadIdx.x & 63) == 0) { sm[0][threadIdx.x >> 6] = ta; sm[1][threadIdx.x >> 6] = tb; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
      for (int q = 0; q < VMS_BLOCK / 64; ++q) { a += sm[0][q]; b += sm[1][q]; }
      rtot[0] = a;
      rtot[1] = b;
    }
  }
  constexpr int RPB = VMS_BLOCK / LPR, PER = 64 / LPR;
  const int W2 = W2F ? W2F : W2rt;
  const int lane = threadIdx.x % LPR;
  const int row = xcd_block(blockIdx.x, gridDim.x) * RPB + threadIdx.x / LPR;
  const bool act = row < n;
  const int ro = act ? row : 0;
  const int64_t r0 = (int64_t)W2 * ro;
  const double xi = ld(x, ro), sii = ld(Sd, ro);
  double a = 0.0;
  for (int q0 = 0; q0 < W2; q0 += 64) {
    int c[PER];
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t k = r0 + q0 + lane + LPR * u;
      c[u] = OFF ? ro + (int)so[k] : sc[k];
      v[u] = ld(S, k);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) a += v[u] * ld(x, c[u]);
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, LPR);
  a += sii * xi;
  if (act && lane == 0) y[row] = (T)a;
}

// y = S^ x; with rpa, workgroup 0 also writes the totals of the partials rpa[0..nred) and
// rpb[0..nred) to rtot[0..1] (the next pipelined CG step reads them instead of the partials).
template <typename T>
void launch_shat_spmv(hipStream_t s, const vms_mesh *mesh, const T *S, const T *Sd, const T *x, T *y,
                      const int *done, const double *rpa = nullptr, const double *rpb = nullptr, int nred = 0,
                      double *rtot = nullptr) {
  constexpr int LPR = sizeof(T) == 4 ? 8 : 16;
  const int n = mesh->n_nodes, W2 = mesh->shat_width;
  const dim3 g((n + VMS_BLOCK / LPR - 1) / (VMS_BLOCK / LPR)), b(VMS_BLOCK);
  const bool off = mesh->shat_off != nullptr;
  if (W2 == 64) {
    if (off)
      hipLaunchKernelGGL((k_shat_spmv<T, LPR, true, 64>), g, b, 0, s, n, W2, mesh->shat_col, mesh->shat_off, S, Sd,
                         x, y, done, rpa, rpb, nred, rtot);
    else
      hipLaunchKernelGGL((k_shat_spmv<T, LPR, false, 64>), g, b, 0, s, n, W2, mesh->shat_col, mesh->shat_off, S, Sd,
                         x, y, done, rpa, rpb, nred, rtot);
  } else {
    if (off)
      hipLaunchKernelGGL((k_shat_spmv<T, LPR, true, 0>), g, b, 0, s, n, W2, mesh->shat_col, mesh->shat_off, S, Sd,
                         x, y, done, rpa, rpb, nred, rtot);
    else
      hipLaunchKernelGGL((k_shat_spmv<T, LPR, false, 0>), g, b, 0, s, n, W2, mesh->shat_col, mesh->shat_off, S, Sd,
                         x, y, done, rpa, rpb, nred, rtot);
  }
}

// ---- pipelined CG steps on S^ --------------------------------------------------
// Vector kernels of the steps: 1024-thread workgroups, PCG_THREAD_NODES nodes
// per thread (at most VMS_MAX_RED_BLOCKS workgroups, one partial each).
#ifndef PCG_THREAD_NODES
#define PCG_THREAD_NODES 2
#endif
inline int pcg_blocks(int64_t n) {
  const int64_t per = (int64_t)KRY_BLOCK * PCG_THREAD_NODES;
  return (int)std::min<int64_t>(std::max<int64_t>((n + per - 1) / per, 1), VMS_MAX_RED_BLOCKS);
}
// Work vectors of one application, each [n]: r, u, w, m, nv, z, q, s, p.
template <typename T>
struct PcgVec {
  T *r, *u, *w, *m, *nv, *z, *q, *s, *p;
};

// start: x = 0, r = v, u = diag(S^)^-1 v; resets the flag
template <typename T>
__global__ void k_pcg_init(int n, const T *__restrict__ v, const T *__restrict__ dinv, T *x, PcgVec<T> V, int *flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
  if (i >= n) return;
  const double vi = ld(v, i);
  x[i] = (T)0;
  V.r[i] = (T)vi;
  V.u[i] = (T)(ld(dinv, i) * vi);
}

// after w = S^ u: partials of gamma = <r,u> and delta = <w,u>, and m = diag(S^)^-1 w
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_pcg_start(int n, const T *__restrict__ dinv, PcgVec<T> V, double *pg, double *pd) {
  __shared__ double sm[2][16];
  double g = 0.0, d = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double ui = ld(V.u, i), wi = ld(V.w, i);
    g += ld(V.r, i) * ui;
    d += wi * ui;
    V.m[i] = (T)(ld(dinv, i) * wi);
  }
  cg_block_sums2(g, d, pg + blockIdx.x, pd + blockIdx.x, sm);
}

// step i (nv = S^ m already formed, and gamma_i, delta_i, the totals of the
// partials of buffer i & 1, in tot: the product kernel forms both); beta_i = gamma_i / gamma_{i-1}, alpha_i = gamma_i /
// (delta_i - beta_i gamma_i / alpha_{i-1}) (step 0: beta = 0, alpha =
// gamma / delta); z = nv + beta z, q = m + beta q, s = w + beta s,
// p = u + beta p, x += alpha p; unless last: r -= alpha s, u -= alpha q,
// w -= alpha z, m = diag(S^)^-1 w and the partials of the next gamma, delta
// into buffer (i + 1) & 1.  ctl: gamma and alpha of the last two steps.
template <typename T>
__global__ void __launch_bounds__(KRY_BLOCK)
k_pcg_step(int n, int i, int last, T *x, PcgVec<T> V, const T *__restrict__ dinv, double *ctl, double *pg0,
           double *pd0, double *pg1, double *pd1, const double *tot, int *flag) {
  __shared__ double sm[2][16];
  __shared__ int done0;
  if (threadIdx.x == 0) done0 = *flag;
  __syncthreads();
  if (done0) return;
  const double g = tot[0], d = tot[1];   // totals of the partials of buffer i & 1 (the product kernel's)
  double beta = 0.0, den = d;
  if (i > 0) {
    beta = g / ctl[(i - 1) & 1];
    den = d - beta * g / ctl[2 + ((i - 1) & 1)];
  }
  const double alpha = g / den;
  if (!(g > 0.0) || !(den > 0.0) || !isfinite(alpha) || !isfinite(beta)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[i & 1] = g;
    ctl[2 + (i & 1)] = alpha;
  }
  const bool first = (i == 0);
  double gn = 0.0, dn = 0.0;
  const int stride = gridDim.x * blockDim.x;
  if (last) {   // only x changes
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
      const double uo = ld(V.u, k), po = first ? 0.0 : ld(V.p, k), xo = ld(x, k);
      const double pk = uo + (first ? 0.0 : beta * po);
      x[k] = (T)(xo + alpha * pk);
    }
    return;
  }
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    // every load of the node before any store (the work vectors are not
    // restrict: loads placed after stores would wait for them).  On the first
    // step z, q, s, p are read but not used (the select keeps 0).
    const double nvo = ld(V.nv, k), mo = ld(V.m, k), wo = ld(V.w, k), uo = ld(V.u, k), ro = ld(V.r, k);
    const double zo = ld(V.z, k), qo = ld(V.q, k), so = ld(V.s, k), po = ld(V.p, k);
    const double xo = ld(x, k), dk = ld(dinv, k);
    const double zk = nvo + (first ? 0.0 : beta * zo);
    const double qk = mo + (first ? 0.0 : beta * qo);
    const double sk = wo + (first ? 0.0 : beta * so);
    const double pk = uo + (first ? 0.0 : beta * po);
    x[k] = (T)(xo + alpha * pk);
    V.z[k] = (T)zk;
    V.q[k] = (T)qk;
    V.s[k] = (T)sk;
    V.p[k] = (T)pk;
    const T rk = (T)(ro - alpha * sk);
    const T uk = (T)(uo - alpha * qk);
    const T wk = (T)(wo - alpha * zk);
    V.r[k] = rk;
    V.u[k] = uk;
    V.w[k] = wk;
    V.m[k] = (T)(dk * (double)wk);
    gn += (double)rk * (double)uk;
    dn += (double)wk * (double)uk;
  }
  cg_block_sums2(gn, dn, ((i + 1) & 1 ? pg1 : pg0) + blockIdx.x, ((i + 1) & 1 ? pd1 : pd0) + blockIdx.x, sm);
}

// ---- S^ = D - C diag(A)^-1 B, assembled on the distance-2 pattern ----------
// Off-diagonal part in rows of W2 fixed slots (sorted columns, then padding
// slots that hold the row's own node), diagonal apart.  16 lanes per row i
// (one per block slot of a 1-ring row), 16 rows per workgroup.  The row's
// columns and accumulators live in LDS; the neighbours k of i are visited in
// slot order, and for each k the 16 lanes take the blocks (k, j) of row k:
// lane l adds -sum_c C_ik,c B_kj,c / A_kk,cc to the accumulator of column j
// (one lane per j within a k, so no two lanes of a step touch one
// accumulator), then D_ij is added.  Fixed order: deterministic.  Also
// writes diag(S^)^-1 (1 where S^_ii is 0 or not finite).
#define SHAT_ROWS 16
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_shat_form(int n, int W, const int32_t *__restrict__ col, const int32_t *__restrict__ diag_pos, int64_t nnzb,
            const double *__restrict__ A, const double *__restrict__ B, const double *__restrict__ C,
            const double *__restrict__ D, int W2, const int32_t *__restrict__ sc, T *S, T *Sd, T *sdinv) {
  __shared__ int32_t scol[SHAT_ROWS][VMS_MAX_SHAT_ROW];
  __shared__ double acc[SHAT_ROWS][VMS_MAX_SHAT_ROW];
  __shared__ double dacc[SHAT_ROWS];
  const int lane = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int row = blockIdx.x * SHAT_ROWS + g;
  if (row >= n) return;   // a row's 16 lanes share one wavefront and use only their own LDS rows
  const int64_t r0 = (int64_t)W2 * row;
  int cnt = 0;
  for (int q = lane; q < W2; q += 16) {
    const int j = sc[r0 + q];
    scol[g][q] = j;
    acc[g][q] = 0.0;
    cnt += (j != row);
  }
  if (lane == 0) dacc[g] = 0.0;
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 16);
  const int len = cnt;   // real (sorted) entries come first
  auto slot = [&](int j) {   // position of column j != row in the row's sorted list
    int lo = 0, hi = len - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (scol[g][mid] < j) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  if (W == 16) {
    // lane kk forms the weights C_ik,c / A_kk,cc of neighbour slot kk (all sixteen at once); the
    // slots are then taken in order, each lane holding block (k, lane) of row k, and the next
    // slot's blocks are requested before this slot's accumulation
    const int64_t bi = (int64_t)W * row + lane;
    const double c0 = C[bi], c1 = C[nnzb + bi], c2 = C[2 * nnzb + bi];
    const bool use = !(c0 == 0.0 && c1 == 0.0 && c2 == 0.0);   // padding slot, or no coupling
    const int kme = col[bi];
    const int64_t dk = diag_pos[kme];
    const double a0 = A[dk], a1 = A[4 * nnzb + dk], a2 = A[8 * nnzb + dk];
    const double w0m = (a0 != 0.0) ? c0 / a0 : 0.0, w1m = (a1 != 0.0) ? c1 / a1 : 0.0;
    const double w2m = (a2 != 0.0) ? c2 / a2 : 0.0;
    const unsigned long long usem = __ballot(use);
    const int gl = (threadIdx.x & 63) & ~15;   // first lane of this row's sixteen
    auto fetch = [&](int kk, double &b0, double &b1, double &b2, int &j) {
      const int k = __shfl(kme, gl + kk, 64);
      const int64_t bkj = (int64_t)W * k + lane;
      b0 = B[bkj]; b1 = B[nnzb + bkj]; b2 = B[2 * nnzb + bkj];
      j = col[bkj];
    };
    double nb0 = 0.0, nb1 = 0.0, nb2 = 0.0;
    int nj = 0;
    fetch(0, nb0, nb1, nb2, nj);
    for (int kk = 0; kk < W; ++kk) {
      const double b0 = nb0, b1 = nb1, b2 = nb2;
      const int j = nj;
      if (kk + 1 < W) fetch(kk + 1, nb0, nb1, nb2, nj);
      const double w0 = __shfl(w0m, gl + kk, 64), w1 = __shfl(w1m, gl + kk, 64), w2 = __shfl(w2m, gl + kk, 64);
      if (!((usem >> (gl + kk)) & 1ull)) continue;
      const double v = w0 * b0 + w1 * b1 + w2 * b2;
      if (v != 0.0) {
        if (j == row) dacc[g] -= v;
        else acc[g][slot(j)] -= v;
      }
    }
  } else {
    for (int kk = 0; kk < W; ++kk) {
      const int64_t bik = (int64_t)W * row + kk;
      const double c0 = C[bik], c1 = C[nnzb + bik], c2 = C[2 * nnzb + bik];
      if (c0 == 0.0 && c1 == 0.0 && c2 == 0.0) continue;   // padding slot, or no coupling
      const int k = col[bik];
      const int64_t dk = diag_pos[k];
      const double a0 = A[dk], a1 = A[4 * nnzb + dk], a2 = A[8 * nnzb + dk];
      const double w0 = (a0 != 0.0) ? c0 / a0 : 0.0, w1 = (a1 != 0.0) ? c1 / a1 : 0.0, w2 = (a2 != 0.0) ? c2 / a2 : 0.0;
      for (int l = lane; l < W; l += 16) {
        const int64_t bkj = (int64_t)W * k + l;
        const double v = w0 * B[bkj] + w1 * B[nnzb + bkj] + w2 * B[2 * nnzb + bkj];
        if (v != 0.0) {
          const int j = col[bkj];
          if (j == row) dacc[g] -= v;
          else acc[g][slot(j)] -= v;
        }
      }
    }
  }
  for (int l = lane; l < W; l += 16) {
    const int64_t b = (int64_t)W * row + l;
    const double dv = D[b];
    if (dv != 0.0) {
      const int j = col[b];
      if (j == row) dacc[g] += dv;
      else acc[g][slot(j)] += dv;
    }
  }
  for (int q = lane; q < W2; q += 16) S[r0 + q] = (T)acc[g][q];
  if (lane == 0) {
    const double v = dacc[g];
    Sd[row] = (T)v;
    sdinv[row] = (T)((v != 0.0 && isfinite(v)) ? 1.0 / v : 1.0);
  }
}

// Chebyshev scalars for step k on [lmax/ratio, lmax] (lmax read on the device)
__device__ __forceinline__ void cheb_coef(const double *lam, double ratio, int k, double &rho0, double &rho1,
                                          double &delta, double &theta) {
  const double lmax = 1.1 * (*lam);
  const double lmin = lmax / ratio;
  theta = 0.5 * (lmax + lmin);
  delta = 0.5 * (lmax - lmin);
  const double s1 = theta / delta;
  double r = 1.0 / s1;
  for (int q = 0; q < k; ++q) r = 1.0 / (2.0 * s1 - r);
  rho0 = r;
  rho1 = 1.0 / (2.0 * s1 - r);
}

// y = S^ d: 16 lanes per row, 16 rows per workgroup; lane l takes the
// off-diagonal slots l, l + 16, l + 32, l + 48 of each 64-slot segment (four
// column loads and four gathers in flight per lane), the diagonal is added by
// lane 0; then
// MODE 0 (power iteration): y = diag(S^)^-1 S^ d
// MODE 1 (Chebyshev step k): x += d; r -= S^ d; y = rho1 rho0 d + 2 rho1/delta diag(S^)^-1 r
template <typename T, int MODE>
__global__ void __launch_bounds__(VMS_BLOCK)
k_shat_cheb(int n, int W2, const int32_t *__restrict__ sc, const int16_t *__restrict__ so, const T *__restrict__ S,
            const T *__restrict__ Sd, const T *__restrict__ d, const T *__restrict__ sdinv, T *y, T *x, T *r,
            const double *lam, double ratio, int k) {
  const int lane = threadIdx.x & 15;
  const int row = xcd_block(blockIdx.x, gridDim.x) * SPMV_ROWS_PER_BLOCK + (threadIdx.x >> 4);
  const bool act = row < n;
  const int ro = act ? row : 0;
  // the row's own values and the Chebyshev scalars ahead of the product (latency overlap)
  const double sdi = ld(sdinv, ro), sii = ld(Sd, ro), di = ld(d, ro);
  double xi = 0.0, ri = 0.0, rho0 = 0.0, rho1 = 0.0, delta = 1.0, theta = 1.0;
  if (MODE == 1) {
    xi = ld(x, ro);
    ri = ld(r, ro);
    cheb_coef(lam, ratio, k, rho0, rho1, delta, theta);
  }
  const double a = reduce16(shat_row_dot(W2, sc, so, S, d, ro, lane)) + sii * di;
  if (act && lane == 0) {
    if (MODE == 0) {
      y[row] = (T)(sdi * a);
    } else {
      x[row] = (T)(xi + di);
      const double rn = ri - a;
      r[row] = (T)rn;
      y[row] = (T)(rho1 * rho0 * di + 2.0 * rho1 / delta * sdi * rn);
    }
  }
}

// r = v, x = 0, d0 = diag(S^)^-1 r / theta
template <typename T>
__global__ void k_cheb_init(int n, const T *v, const T *sdinv, T *x, T *r, T *d, const double *lam, double ratio) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double rho0, rho1, delta, theta;
  cheb_coef(lam, ratio, 0, rho0, rho1, delta, theta);
  const double vi = ld(v, i);
  r[i] = (T)vi;
  x[i] = (T)0;
  d[i] = (T)(ld(sdinv, i) * vi / theta);
}

// deterministic oscillatory start vector of the power iteration
template <typename T>
__global__ void k_power_init(int n, T *x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)i * 2654435761u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  x[i] = (T)((double)(h & 0xffff) / 32768.0 - 1.0);
}

// lam = ||y|| from the norm partials
__global__ void __launch_bounds__(VMS_BLOCK) k_store_norm(int nb, const double *part, double *lam) {
  __shared__ double sm[4];
  const double s = sum_partials1(part, nb, sm);
  if (threadIdx.x == 0) *lam = sqrt(s);
}

template <typename T>
__global__ void k_power_scale(int n, const T *y, const double *lam, T *x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double l = *lam;
  x[i] = (T)((l > 0.0) ? ld(y, i) / l : 0.0);
}

// full [n][4] FP64 <-> split velocity [n][3] / pressure [n] of type T
template <typename T>
__global__ void k_split(int n, const double *full, T *v, T *p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = 4 * (int64_t)i;
  v[3 * (int64_t)i] = (T)full[o];
  v[3 * (int64_t)i + 1] = (T)full[o + 1];
  v[3 * (int64_t)i + 2] = (T)full[o + 2];
  p[i] = (T)full[o + 3];
}
template <typename T>
__global__ void k_merge(int n, const T *v, const T *p, double *full) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = 4 * (int64_t)i;
  full[o] = (double)v[3 * (int64_t)i];
  full[o + 1] = (double)v[3 * (int64_t)i + 1];
  full[o + 2] = (double)v[3 * (int64_t)i + 2];
  full[o + 3] = (double)p[i];
}
// z = d .* v
template <typename T>
__global__ void k_diag_scale(int n, const T *d, const T *v, T *z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = (T)(ld(d, i) * ld(v, i));
}

// z += d .* v
template <typename T>
__global__ void k_diag_axpy(int n, const T *d, const T *v, T *z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = (T)(ld(z, i) + ld(d, i) * ld(v, i));
}

// Lumped pressure mass of node i in the reference configuration -- the sum of
// vol_e / 4 over the elements at i, read from the (element, local node)
// incidences that the contribution list of i's diagonal block holds -- in the
// scaled variables: mlw_i = W_p,i^2 m_i.  one_i = 1 on free pressure dofs, 0
// on prescribed ones.
template <typename T>
__global__ void k_mass_lumped(int n, const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ ptr,
                              const int32_t *__restrict__ src, const double *__restrict__ X,
                              const int32_t *__restrict__ tets, const uint8_t *__restrict__ dir,
                              const double *__restrict__ W, double *mlw, T *one) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int blk = diag_pos[i];
  double m = 0.0;
  for (int k = ptr[blk]; k < ptr[blk + 1]; ++k) {
    const int64_t e = src[k] >> 4;
    const int32_t *t = tets + 4 * e;
    const double *x0 = X + 3 * (int64_t)t[0], *x1 = X + 3 * (int64_t)t[1], *x2 = X + 3 * (int64_t)t[2],
                 *x3 = X + 3 * (int64_t)t[3];
    const double a0 = x1[0] - x0[0], a1 = x1[1] - x0[1], a2 = x1[2] - x0[2];
    const double b0 = x2[0] - x0[0], b1 = x2[1] - x0[1], b2 = x2[2] - x0[2];
    const double c0 = x3[0] - x0[0], c1 = x3[1] - x0[1], c2 = x3[2] - x0[2];
    const double det = a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
    m += fabs(det) / 24.0;   // vol_e / 4
  }
  const double w = W[4 * (int64_t)i + 3];
  const bool fixed = dir[4 * (int64_t)i + 3] != 0;
  mlw[i] = w * w * m;
  one[i] = (T)(fixed ? 0.0 : 1.0);
}

// One workgroup: sums[0] = sum of (S 1)_i and sums[1] = sum of mlw_i over the
// free pressure dofs, each thread in a fixed order, then a fixed block order.
template <typename T>
__global__ void __launch_bounds__(1024) k_mass_sums(int n, const T *__restrict__ s1, const double *__restrict__ mlw,
                                                    const uint8_t *__restrict__ dir, double *sums) {
  __shared__ double sm[2][16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if (dir[4 * (int64_t)i + 3]) continue;
    a += ld(s1, i);
    b += mlw[i];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) { sm[0][w] = a; sm[1][w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int q = 0; q < nw; ++q) { ta += sm[0][q]; tb += sm[1][q]; }
    sums[0] = ta;
    sums[1] = tb;
  }
}

// minv_i = w / (c mlw_i) with c = sums[0] / sums[1] (the Rayleigh quotient of
// S and the scaled lumped mass on the constant vector; c = 1 if it is not
// positive or sums is null), w on prescribed pressure dofs (their S row is the identity);
// with pdiag, also pdiag = minv (+ diag(S^)^-1 when sdinv is given).
template <typename T>
__global__ void k_mass_inv(int n, const double *__restrict__ mlw, const double *__restrict__ sums,
                           const uint8_t *__restrict__ dir, double w, const T *sdinv, T *minv, T *pdiag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double c = sums ? sums[0] / sums[1] : 1.0;
  if (!(c > 0.0) || !isfinite(c)) c = 1.0;
  const double m = mlw[i];
  const double v = (dir[4 * (int64_t)i + 3] || !(m > 0.0)) ? w : w / (c * m);
  minv[i] = (T)v;
  if (pdiag) pdiag[i] = (T)(v + (sdinv ? ld(sdinv, i) : 0.0));
}

// diag(A)^-1: the diagonal entries of the 3x3 diagonal blocks (1 where zero)
template <typename T>
__global__ void k_diagA_inv(int n, const int32_t *diag_pos, int64_t nnzb, const double *A, T *dAinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = diag_pos[i];
  for (int c = 0; c < 3; ++c) {
    const double a = A[(4 * c) * nnzb + b];
    dAinv[3 * (int64_t)i + c] = (T)((a != 0.0 && isfinite(a)) ? 1.0 / a : 1.0);
  }
}

// last factor of the SIMPLE preconditioner: x_v = y_v - diag(A)^-1 w, w = B x_p
template <typename T>
__global__ void k_simple_vel(int64_t nv, const T *y, const T *w, const T *dAinv, T *x) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < nv) x[k] = (T)(ld(y, k) - ld(dAinv, k) * ld(w, k));
}

__global__ void k_clear_ints(int *p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0;
}

inline int grid1(int64_t n) { return (int)((n + VMS_BLOCK - 1) / VMS_BLOCK); }

// y = A x (A-block product, the solver's dominant kernel).  With launch timing
// on, the launch carries start/stop events taken by the dispatch itself.
template <typename T>
void launch_spmv_A(vms_ctx *ctx, const vms_mesh *mesh, const T *A, const T *x, T *y, const int *done) {
  const dim3 gr(spmv_grid(mesh->n_nodes)), bl(VMS_BLOCK);
  const vms_timed tm = vms_timer_next(ctx, std::is_same<T, float>::value ? 1 : 0);
  if (tm.slot >= 0)
    hipExtLaunchKernelGGL((k_spmv_A<T, T>), gr, bl, 0, ctx->stream, tm.e0, tm.e1, 0, (int)mesh->n_nodes,
                          (int64_t)mesh->nnzb, (int)mesh->slot_width, mesh->col, A, x, y, (const T *)nullptr, 1.0,
                          done, tm.worked);
  else
    hipLaunchKernelGGL((k_spmv_A<T, T>), gr, bl, 0, ctx->stream, (int)mesh->n_nodes, (int64_t)mesh->nnzb,
                       (int)mesh->slot_width, mesh->col, A, x, y, (const T *)nullptr, 1.0, done, (int *)nullptr);
}

// ---- workspace carving -------------------------------------------------------
struct Carver {
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

template <typename T>
struct KLevel {
  int64_t nvec = 0;
  int m = 0, nb = 1, nbk = 1;
  T *V = nullptr, *Z = nullptr, *W = nullptr;
  double *ctrl = nullptr;
  int *iflag = nullptr;
  KOff off{};
  void carve(Carver &cv, int64_t nv, int mm) {
    nvec = nv;
    m = std::max(mm, 1);
    nb = vms_red_blocks(nv);
    nbk = kry_blocks(nv);
    V = cv.take<T>((int64_t)(m + 1) * nv);
    Z = cv.take<T>((int64_t)(m + 1) * nv);
    W = cv.take<T>(nv);
    off = make_off(m);
    ctrl = cv.take<double>(ctrl_doubles(m));
    iflag = cv.take<int>(8);
  }
};

inline int sync_level_flags(vms_ctx *ctx, const int *iflag) { return vms_read_flags(ctx, iflag); }

// Arnoldi step j of level L: orthogonalise W against V_0..V_j, finish the
// Hessenberg/Givens update and the convergence flags, and form V_{j+1} and
// Z_{j+1} = M^-1 V_{j+1}.
//   CGS1: multi-dot, multi-update (+ norm partials), normalize/Givens
//   CGS2: the same with a second multi-dot/multi-update pass
//   CGS "if needed": the second pass only where the test of
//         kry_need_reorth asks for it (its kernels return at once otherwise)
//   MGS:  one dot/axpy launch pair per basis vector
template <typename T>
int orth_level(vms_ctx *ctx, KLevel<T> &L, int j, int maxit, int mode, int pc, const T *pcd,
               volatile int32_t *post = nullptr, int32_t seq = 0) {
  hipStream_t s = ctx->stream;
  double *part = L.ctrl + L.off.part;
  const int ld = L.m + 1;
  T *V1 = L.V + (int64_t)(j + 1) * L.nvec, *Z1 = L.Z + (int64_t)(j + 1) * L.nvec;
  if (mode == VMS_ORTH_MGS) {
    const dim3 gr(L.nb), bl(VMS_BLOCK);
    double *col = L.ctrl + L.off.H + (int64_t)j * ld;
    for (int k = 0; k <= j; ++k) {
      hipLaunchKernelGGL(k_mgs_part<T>, gr, bl, 0, s, L.nvec, L.V, k, L.W, (const double *)(col + (k > 0 ? k - 1 : 0)),
                         part, L.iflag);
      hipLaunchKernelGGL(k_dot_finalize, dim3(1), bl, 0, s, (const double *)part, L.nb, 1, 1, col + k, L.iflag);
    }
    hipLaunchKernelGGL((k_mupdate<T, true>), gr, bl, 0, s, L.nvec, L.V + (int64_t)j * L.nvec, 1, L.W,
                       (const double *)(col + j), part, L.iflag);
    hipLaunchKernelGGL(k_givens, dim3(1), bl, 0, s, L.nb, L.ctrl, L.off, L.iflag, j, maxit);
    hipLaunchKernelGGL(k_normalize<T>, gr, bl, 0, s, L.nvec, L.W, V1, Z1, L.ctrl, L.off, L.iflag, pc, pcd);
  } else {
    const dim3 gk(L.nbk), bk(KRY_BLOCK);
    double *h1 = L.ctrl + L.off.h1, *h2 = L.ctrl + L.off.h2;
    double *pn = L.ctrl + L.off.pn, *pn2 = L.ctrl + L.off.pn2;
    hipLaunchKernelGGL(k_mdot_part<T>, gk, bk, 0, s, L.nvec, L.V, j + 1, L.W, part, ld, L.iflag,
                       (const double *)nullptr, KOff{}, 0);
    if (mode == VMS_ORTH_CGS2) {
      hipLaunchKernelGGL((k_mupdate_fin<T, false>), gk, bk, 0, s, L.nvec, L.V, j + 1, L.W, (const double *)part,
                         L.nbk, ld, h1, pn, L.iflag, (const double *)nullptr, KOff{});
      hipLaunchKernelGGL(k_mdot_part<T>, gk, bk, 0, s, L.nvec, L.V, j + 1, L.W, part, ld, L.iflag,
                         (const double *)nullptr, KOff{}, 0);
      hipLaunchKernelGGL((k_mupdate_fin<T, true>), gk, bk, 0, s, L.nvec, L.V, j + 1, L.W, (const double *)part,
                         L.nbk, ld, h2, pn2, L.iflag, (const double *)nullptr, KOff{});
    } else {
      hipLaunchKernelGGL((k_mupdate_fin<T, true>), gk, bk, 0, s, L.nvec, L.V, j + 1, L.W, (const double *)part,
                         L.nbk, ld, h1, pn, L.iflag, (const double *)nullptr, KOff{});
      if (mode == VMS_ORTH_CGS_IFNEEDED) {   // second pass only where the test asks for it
        hipLaunchKernelGGL(k_mdot_part<T>, gk, bk, 0, s, L.nvec, L.V, j + 1, L.W, part, ld, L.iflag,
                           (const double *)L.ctrl, L.off, L.nbk);
        hipLaunchKernelGGL((k_mupdate_fin<T, true>), gk, bk, 0, s, L.nvec, L.V, j + 1, L.W, (const double *)part,
                           L.nbk, ld, h2, pn2, L.iflag, (const double *)L.ctrl, L.off);
      }
    }
    const int nsum = (mode == VMS_ORTH_CGS2) ? 2 : (mode == VMS_ORTH_CGS_IFNEEDED) ? 3 : 1;
    hipLaunchKernelGGL(k_normalize_givens<T>, gk, bk, 0, s, L.nvec, (const T *)L.W, V1, Z1, L.ctrl, L.off, L.iflag,
                       L.nbk, j, nsum, maxit, pc, pcd, post, seq);
  }
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

// Iterations to enqueue before the host next reads a level's flags.  The first batch is most of
// the previous solve's count on the level (consecutive solves differ by a few iterations), later
// ones start at an eighth of it and double: a launch past convergence still costs a few
// microseconds per kernel, a host round trip about as much as one iteration's kernels.
inline int next_batch(int est, int round) {
  if (round == 0) return std::max(1, (7 * est + 7) / 8);
  return std::min(64, std::max(2, (est + 7) / 8) << std::min(round - 1, 5));
}

// Right-preconditioned (F)GMRES with x0 = 0 on level L.  op(j) enqueues
// W = Op Z_j; for pc != PC_NONE the device preconditioner fills Z_{j+1} from
// V_{j+1}, otherwise op(j) itself must first fill Z_j (flexible variant).
// Without sync_each the host enqueues `batch` iterations before it reads the
// level flags (kernels past convergence return at once).
template <typename T, typename OpF>
int gmres_run(vms_ctx *ctx, KLevel<T> &L, const T *b, T *x, double rtol, double atol, int maxit, int orth, int pc,
              const T *pcd, bool sync_each, int &est, OpF op, int &its_out, int &status_out,
              const double *relax = nullptr) {
  hipStream_t s = ctx->stream;
  maxit = std::min(maxit, L.m);
  const dim3 gr(L.nb), bl(VMS_BLOCK);
  hipLaunchKernelGGL(k_norm_part<T>, gr, bl, 0, s, L.nvec, b, L.ctrl + L.off.part, (const int *)nullptr);
  hipLaunchKernelGGL(k_kinit<T>, gr, bl, 0, s, L.nvec, b, L.V, L.Z, L.ctrl, L.off, L.iflag, L.nb, rtol, atol, pc, pcd,
                     relax);
  VMS_LAUNCH_CHECK(ctx);
  int j = 0, rc;
  bool done = false, read = false;
  if (sync_each) {
    if ((rc = sync_level_flags(ctx, L.iflag))) return rc;
    done = ctx->h_i[IF_DONE] != 0;
    read = true;
  }
  const bool posting = (orth != VMS_ORTH_MGS);   // the last normalisation kernel of a batch posts the flags
  int round = 0;
  int batch = sync_each ? 1 : next_batch(est, round++);
  while (!done && j < maxit) {
    const int nbt = std::min(batch, maxit - j);
    int32_t seq = 0;
    for (int i = 0; i < nbt; ++i, ++j) {
      if ((rc = op(j))) return rc;
      const bool last = posting && (i == nbt - 1);
      if (last) seq = ++ctx->post_seq;
      if ((rc = orth_level<T>(ctx, L, j, maxit, orth, pc, pcd, last ? ctx->h_post : nullptr, seq))) return rc;
    }
    VMS_LAUNCH_CHECK(ctx);
    if ((rc = posting ? vms_wait_post(ctx, seq, L.iflag) : sync_level_flags(ctx, L.iflag))) return rc;
    done = ctx->h_i[IF_DONE] != 0;
    read = true;
    if (!sync_each) batch = next_batch(est, round++);
  }
  if (!read && (rc = sync_level_flags(ctx, L.iflag))) return rc;
  status_out = ctx->h_i[IF_STATUS];
  its_out = ctx->h_i[IF_ITS];
  if (its_out <= COMBINE_SOLVE_MAX) {
    hipLaunchKernelGGL(k_solve_combine<T>, gr, bl, 0, s, L.nvec, (const T *)L.Z, (const double *)L.ctrl, L.off,
                       (const int *)L.iflag, x);
  } else {
    hipLaunchKernelGGL(k_trisolve, dim3(1), bl, 0, s, L.ctrl, L.off, L.iflag);
    hipLaunchKernelGGL(k_combine<T>, gr, bl, 0, s, L.nvec, L.Z, L.ctrl, L.off, L.iflag, x);
  }
  VMS_LAUNCH_CHECK(ctx);
  est = std::max(1, its_out);
  if (status_out == KS_NAN) return vms_set_error(ctx, VMS_ERR_NAN, "NaN/Inf in a Krylov level");
  return VMS_OK;
}

// Preconditioned CG (3x3 block-Jacobi) on the symmetrised A of level L with
// x0 = 0: two kernels per iteration (product with the direction update, then
// the vector update); the level's vectors hold r, z, the two alternating
// directions and q = A_s p.  The stopping test runs at the start of the
// product kernel, so the host enqueues batches of iterations and reads the
// flags that the last product kernel of a batch posts.
template <typename T>
int cg_run(vms_ctx *ctx, KLevel<T> &L, const vms_mesh *mesh, const T *Acg, double *ppart, const T *b, T *x,
           double rtol, double atol, int maxit, const T *Minv, int &est, int &its_out, int &status_out,
           const double *relax = nullptr) {
  hipStream_t s = ctx->stream;
  const int n = mesh->n_nodes;
  const int64_t nn = n;
  T *r = L.V, *z = L.Z, *p = L.V + L.nvec, *q = L.W;
  const int gs = cg_spmv_blocks(n);
  // vector kernels: two nodes per thread (measured faster than one per thread with twice the workgroups)
  const dim3 gk(kry_blocks(nn)), bk(KRY_BLOCK), gsp(gs), bl(VMS_BLOCK);
  const int nbk = (int)gk.x;
  hipLaunchKernelGGL(k_cg_init<T>, gk, bk, 0, s, nn, b, x, r, z, Minv, L.ctrl + L.off.pn, L.ctrl + L.off.pn2,
                     L.iflag);
  // with launch timing on, the product launches of a CG level are the A-block
  // products that the context times (kind 0 FP64, 1 FP32)
  auto spmv = [&](int j, volatile int32_t *post, int32_t seq) {
    const vms_timed tm = vms_timer_next(ctx, std::is_same<T, float>::value ? 1 : 0);
    if (tm.slot >= 0)
      hipExtLaunchKernelGGL(k_cg_spmv<T>, gsp, bl, 0, s, tm.e0, tm.e1, 0, n, (int64_t)mesh->nnzb,
                            (int)mesh->slot_width, mesh->col, Acg, (const T *)z, p, q, L.ctrl, L.off, ppart, L.iflag,
                            j, nbk, rtol, atol, maxit, post, seq, tm.worked, relax);
    else
      hipLaunchKernelGGL(k_cg_spmv<T>, gsp, bl, 0, s, n, (int64_t)mesh->nnzb, (int)mesh->slot_width, mesh->col,
                         Acg, (const T *)z, p, q, L.ctrl, L.off, ppart, L.iflag, j, nbk, rtol, atol, maxit, post, seq,
                         (int *)nullptr, relax);
  };
  int j = 0;
  spmv(0, nullptr, 0);
  VMS_LAUNCH_CHECK(ctx);
  int round = 0;
  int batch = next_batch(est, round++);
  bool done = false;
  while (!done) {
    const int nbt = std::min(batch, maxit - j);
    if (nbt <= 0) {   // not reached: the product kernel of iteration maxit always ends the level
      int rc = sync_level_flags(ctx, L.iflag);
      if (rc) return rc;
      break;
    }
    const int32_t seq = ++ctx->post_seq;
    for (int i = 0; i < nbt; ++i) {
      hipLaunchKernelGGL(k_cg_update<T>, gk, bk, 0, s, nn, x, r, z, (const T *)p, (const T *)q, Minv, L.ctrl, L.off,
                         (const double *)ppart, gs, L.iflag, j);
      ++j;
      spmv(j, i == nbt - 1 ? ctx->h_post : nullptr, seq);
    }
    VMS_LAUNCH_CHECK(ctx);
    int rc = vms_wait_post(ctx, seq, L.iflag);
    if (rc) return rc;
    done = ctx->h_i[IF_DONE] != 0;
    batch = next_batch(est, round++);
  }
  status_out = ctx->h_i[IF_STATUS];
  its_out = ctx->h_i[IF_ITS];
  est = std::max(1, its_out);
  if (status_out == KS_NAN) return vms_set_error(ctx, VMS_ERR_NAN, "NaN/Inf in a CG level");
  return VMS_OK;
}

// The multigrid of one linear system: coarse operators, block-diagonal inverses, Chebyshev bounds
// and the V-cycle work vectors in the level precision T (FP64 copies of the coarse operators for
// the Galerkin products), carved from the solve's workspace.
template <typename T>
struct AmgSys {
  const vms_amg_dev *h = nullptr;
  int L = 0;
  double *Ac64[VMS_AMG_MAX_LEVELS] = {};
  T *Ac[VMS_AMG_MAX_LEVELS] = {};
  T *Dinv[VMS_AMG_MAX_LEVELS] = {};
  T *xv[VMS_AMG_MAX_LEVELS] = {}, *bv[VMS_AMG_MAX_LEVELS] = {}, *rv[VMS_AMG_MAX_LEVELS] = {};
  T *d0[VMS_AMG_MAX_LEVELS] = {}, *d1[VMS_AMG_MAX_LEVELS] = {};
  T *tv[VMS_AMG_MAX_LEVELS] = {};   // mode contributions of the residual (restriction), [n_l][10]
  double *lam = nullptr, *ltmp = nullptr, *part = nullptr;
  int *bad = nullptr;
  // finest level: the A-level operator and its 3x3 block-Jacobi inverses
  const T *A0 = nullptr, *M0 = nullptr;
  const vms_mesh *mesh = nullptr;
  const double *Wsc = nullptr;

  void carve(Carver &cv, const vms_mesh *m) {
    h = vms_amg_device(m->amg);   // checked by check_opts before any solve; absent: nothing to carve
    L = h ? h->n_levels : 0;
    for (int l = 0; l < L; ++l) {
      const vms_amg_level_dev &lv = h->lev[l];
      const int64_t nv = (int64_t)lv.n * lv.bs;
      if (l > 0) {
        Ac64[l] = cv.take<double>(lv.nnzb * AMG_NM * AMG_NM);
        Ac[l] = std::is_same<T, double>::value ? (T *)Ac64[l] : cv.take<T>(lv.nnzb * AMG_NM * AMG_NM);
        Dinv[l] = cv.take<T>((int64_t)lv.n * AMG_NM * AMG_NM);
        xv[l] = cv.take<T>(nv);
        bv[l] = cv.take<T>(nv);
      }
      rv[l] = cv.take<T>(nv);
      d0[l] = cv.take<T>(nv);
      d1[l] = cv.take<T>(nv);
      if (l + 1 < L) tv[l] = cv.take<T>((int64_t)lv.n * AMG_NM);
    }
    lam = cv.take<double>(VMS_AMG_MAX_LEVELS);
    ltmp = cv.take<double>(8);
    part = cv.take<double>(VMS_MAX_RED_BLOCKS);
    bad = cv.take<int>(4);
  }

  // per linear system: Galerkin products from the FP64 scaled A (symmetrised when sym), inverses
  // of the coarse diagonal blocks, FP32 copies, and lmax of every level
  int setup(vms_ctx *ctx, const vms_mesh *m, const vms_matrix *K, const T *A0_, const T *M0_, int sym) {
    hipStream_t s = ctx->stream;
    mesh = m;
    A0 = A0_;
    M0 = M0_;
    Wsc = K->W;
    const dim3 bl(VMS_BLOCK);
    hipLaunchKernelGGL(k_clear_ints, dim3(1), dim3(64), 0, s, bad, 1);
    for (int l = 1; l < L; ++l) {
      const vms_amg_level_dev &c = h->lev[l], &f = h->lev[l - 1];
      const int64_t ne = c.nnzb * AMG_NM * AMG_NM;
      const dim3 g((unsigned)((ne + VMS_BLOCK - 1) / VMS_BLOCK));
      if (l == 1)
        hipLaunchKernelGGL(k_amg_gal0, g, bl, 0, s, c.nnzb, c.brow, c.col, c.dropped, f.gptr, f.gsrc,
                           m->slot_width, m->nnzb, m->col, m->tpos, (const double *)K->A, sym,
                           (const double *)K->W, f.P, Ac64[1]);
      else
        hipLaunchKernelGGL(k_amg_gal, g, bl, 0, s, c.nnzb, c.brow, c.col, c.dropped, f.gptr, f.gsrc, f.brow, f.col,
                           (const double *)Ac64[l - 1], f.P, Ac64[l]);
      hipLaunchKernelGGL(k_amg_dinv<T>, dim3(grid1(c.n)), bl, 0, s, c.n, c.dpos, (const double *)Ac64[l], Dinv[l],
                         bad);
      if (!std::is_same<T, double>::value) hipLaunchKernelGGL(k_amg_cvt<T>, g, bl, 0, s, ne, (const double *)Ac64[l], Ac[l]);
    }
    for (int l = 0; l < L; ++l) power(ctx, l);
    VMS_LAUNCH_CHECK(ctx);
    return VMS_OK;
  }

  // lam[l] = 1.1 ||D^-1 A x|| / ||x|| after AMG_POWER_STEPS power steps from a SplitMix64 vector
  void power(vms_ctx *ctx, int l) {
    hipStream_t s = ctx->stream;
    const vms_amg_level_dev &lv = h->lev[l];
    const int64_t nv = (int64_t)lv.n * lv.bs;
    const int nb = vms_red_blocks(nv);
    const dim3 bl(VMS_BLOCK), gv((unsigned)((nv + VMS_BLOCK - 1) / VMS_BLOCK));
    T *x = d0[l], *y = d1[l];
    hipLaunchKernelGGL(k_amg_power_init<T>, gv, bl, 0, s, nv, (uint64_t)(l + 1), x);
    hipLaunchKernelGGL(k_norm_part<T>, dim3(nb), bl, 0, s, nv, (const T *)x, part, (const int *)nullptr);
    hipLaunchKernelGGL(k_store_norm, dim3(1), bl, 0, s, nb, (const double *)part, ltmp);
    hipLaunchKernelGGL(k_power_scale<T>, gv, bl, 0, s, (int)nv, (const T *)x, (const double *)ltmp, x);
    for (int it = 0; it < AMG_POWER_STEPS; ++it) {
      if (l == 0)
        hipLaunchKernelGGL(k_amgf_dapply<T>, dim3(spmv_grid(lv.n)), bl, 0, s, lv.n, mesh->nnzb, mesh->slot_width,
                           mesh->col, A0, M0, (const T *)x, y);
      else
        hipLaunchKernelGGL(k_amgc_dapply<T>, dim3(amg_wgrid(lv.n)), dim3(256), 0, s, lv.n, lv.ptr, lv.col,
                           (const T *)Ac[l], (const T *)Dinv[l], (const T *)x, y);
      hipLaunchKernelGGL(k_norm_part<T>, dim3(nb), bl, 0, s, nv, (const T *)y, part, (const int *)nullptr);
      hipLaunchKernelGGL(k_store_norm, dim3(1), bl, 0, s, nb, (const double *)part, ltmp);
      hipLaunchKernelGGL(k_power_scale<T>, gv, bl, 0, s, (int)nv, (const T *)y, (const double *)ltmp, x);
    }
    hipLaunchKernelGGL(k_amg_lam_final, dim3(1), dim3(1), 0, s, (const double *)ltmp, lam + l);
  }

  // degree-k Chebyshev smoothing of level l for A x = b, from zero (zero) or from x
  void smooth(hipStream_t s, int l, const T *b, T *x, bool zero, int deg, const int *done) {
    const vms_amg_level_dev &lv = h->lev[l];
    const int n = lv.n;
    const double *lm = lam + l;
    const dim3 bl(VMS_BLOCK), gf(spmv_grid(n)), gc(amg_cgrid(n)), gw(amg_wgrid(n)), bc(256);
    T *dk = d0[l], *dn = d1[l], *r = rv[l];
    if (l == 0) {
      if (zero)
        hipLaunchKernelGGL(k_amgf_cheb0<T>, dim3(grid1(n)), bl, 0, s, n, M0, b, x, r, dk, lm, done);
      else
        hipLaunchKernelGGL(k_amgf_chebres<T>, gf, bl, 0, s, n, mesh->nnzb, mesh->slot_width, mesh->col, A0, M0, b,
                           (const T *)x, r, dk, lm, done);
    } else {
      if (zero)
        hipLaunchKernelGGL(k_amgc_cheb0<T>, gc, bc, 0, s, n, (const T *)Dinv[l], b, x, r, dk, lm, done);
      else
        hipLaunchKernelGGL((k_amgc_cheb<T, 0>), gw, bc, 0, s, n, lv.ptr, lv.col, (const T *)Ac[l],
                           (const T *)Dinv[l], b, (const T *)x, dk, r, x, lm, 0, 0, done);
    }
    const int pending = zero ? 0 : 1;
    for (int k = 0; k + 1 < deg; ++k) {
      if (l == 0 && zero)
        hipLaunchKernelGGL((k_amgf_step<T, false>), gf, bl, 0, s, n, mesh->nnzb, mesh->slot_width, mesh->col, A0,
                           M0, (const T *)dk, dn, r, x, lm, k, k == 0 ? pending : 0, done);
      else if (l == 0)
        hipLaunchKernelGGL((k_amgf_step<T, true>), gf, bl, 0, s, n, mesh->nnzb, mesh->slot_width, mesh->col, A0,
                           M0, (const T *)dk, dn, r, x, lm, k, k == 0 ? pending : 0, done);
      else
        hipLaunchKernelGGL((k_amgc_cheb<T, 1>), gw, bc, 0, s, n, lv.ptr, lv.col, (const T *)Ac[l],
                           (const T *)Dinv[l], (const T *)nullptr, (const T *)dk, dn, r, x, lm, k,
                           k == 0 ? pending : 0, done);
      std::swap(dk, dn);
    }
    if (deg == 1 && !zero) {
      const int64_t nv = (int64_t)n * lv.bs;
      hipLaunchKernelGGL(k_amg_axpy<T>, dim3((unsigned)((nv + VMS_BLOCK - 1) / VMS_BLOCK)), bl, 0, s, nv,
                         (const T *)dk, x, done);
    }
  }

  // x = V-cycle(b) on level l
  void vcycle(hipStream_t s, int l, const T *b, T *x, const int *done) {
    const vms_amg_level_dev &lv = h->lev[l];
    if (l == L - 1) {
      smooth(s, l, b, x, true, h->coarse_degree, done);
      return;
    }
    const vms_amg_level_dev &c = h->lev[l + 1];
    const int deg = l == 0 ? h->degree : h->mid_degree;
    smooth(s, l, b, x, true, deg, done);
    const dim3 bl(VMS_BLOCK);
    constexpr bool F32 = std::is_same<T, float>::value;
    using TP = typename std::conditional<F32, float, double>::type;
    const TP *P = F32 ? (const TP *)lv.P32 : (const TP *)lv.P;
    // restriction: residual with its mode contributions per node, then the sums over aggregates
    if (l == 0)
      hipLaunchKernelGGL((k_amgf_resid_t<T, TP>), dim3(spmv_grid(lv.n)), bl, 0, s, lv.n, mesh->nnzb,
                         mesh->slot_width, mesh->col, A0, b, (const T *)x, P, Wsc, tv[0], done);
    else
      hipLaunchKernelGGL((k_amgc_resid_t<T, TP>), dim3(amg_wgrid(lv.n)), dim3(256), 0, s, lv.n, lv.ptr, lv.col,
                         (const T *)Ac[l], b, (const T *)x, P, tv[l], done);
    const dim3 gr((unsigned)(((int64_t)c.n * AMG_NM + VMS_BLOCK - 1) / VMS_BLOCK));
    const dim3 gp((unsigned)(((int64_t)lv.n * lv.bs + VMS_BLOCK - 1) / VMS_BLOCK));
    hipLaunchKernelGGL(k_amg_aggsum<T>, gr, bl, 0, s, c.n, lv.mptr, lv.mem, (const T *)tv[l], bv[l + 1], done);
    vcycle(s, l + 1, bv[l + 1], xv[l + 1], done);
    if (l == 0)
      hipLaunchKernelGGL((k_amg_prolong<T, TP, 3>), gp, bl, 0, s, lv.n, lv.agg, P, Wsc, (const T *)xv[1], x, done);
    else
      hipLaunchKernelGGL((k_amg_prolong<T, TP, AMG_NM>), gp, bl, 0, s, lv.n, lv.agg, P, (const double *)nullptr,
                         (const T *)xv[l + 1], x, done);
    smooth(s, l, b, x, false, deg, done);
  }
};

// Preconditioned CG with the multigrid V-cycle as the preconditioner (same stopping test, flags
// and batching as cg_run): update, V-cycle, <r,z> partials, product.
template <typename T>
int amg_cg_run(vms_ctx *ctx, KLevel<T> &L, const vms_mesh *mesh, const T *Acg, double *ppart, const T *b, T *x,
               double rtol, double atol, int maxit, AmgSys<T> &mg, int &est, int &its_out, int &status_out,
               const double *relax = nullptr) {
  hipStream_t s = ctx->stream;
  const int n = mesh->n_nodes;
  const int64_t nn = n;
  T *r = L.V, *z = L.Z, *p = L.V + L.nvec, *q = L.W;
  const int gs = cg_spmv_blocks(n);
  const dim3 gk(kry_blocks(nn)), bk(KRY_BLOCK), gsp(gs), bl(VMS_BLOCK);
  const int nbk = (int)gk.x;
  const int *done = L.iflag + IF_DONE;
  hipLaunchKernelGGL(k_cgx_init<T>, gk, bk, 0, s, nn, b, x, r, L.iflag);
  auto precond = [&]() {
    mg.vcycle(s, 0, (const T *)r, z, done);
    hipLaunchKernelGGL(k_cgx_rz<T>, gk, bk, 0, s, nn, (const T *)r, (const T *)z, L.ctrl + L.off.pn,
                       L.ctrl + L.off.pn2, (const int *)L.iflag);
  };
  auto spmv = [&](int j, volatile int32_t *post, int32_t seq) {
    const vms_timed tm = vms_timer_next(ctx, std::is_same<T, float>::value ? 1 : 0);
    if (tm.slot >= 0)
      hipExtLaunchKernelGGL(k_cg_spmv<T>, gsp, bl, 0, s, tm.e0, tm.e1, 0, n, (int64_t)mesh->nnzb,
                            (int)mesh->slot_width, mesh->col, Acg, (const T *)z, p, q, L.ctrl, L.off, ppart, L.iflag,
                            j, nbk, rtol, atol, maxit, post, seq, tm.worked, relax);
    else
      hipLaunchKernelGGL(k_cg_spmv<T>, gsp, bl, 0, s, n, (int64_t)mesh->nnzb, (int)mesh->slot_width, mesh->col,
                         Acg, (const T *)z, p, q, L.ctrl, L.off, ppart, L.iflag, j, nbk, rtol, atol, maxit, post, seq,
                         (int *)nullptr, relax);
  };
  precond();
  int j = 0;
  spmv(0, nullptr, 0);
  VMS_LAUNCH_CHECK(ctx);
  int round = 0;
  int batch = next_batch(est, round++);
  bool fin = false;
  while (!fin) {
    const int nbt = std::min(batch, maxit - j);
    if (nbt <= 0) {   // not reached: the product kernel of iteration maxit always ends the level
      int rc = sync_level_flags(ctx, L.iflag);
      if (rc) return rc;
      break;
    }
    const int32_t seq = ++ctx->post_seq;
    for (int i = 0; i < nbt; ++i) {
      hipLaunchKernelGGL(k_cgx_update<T>, gk, bk, 0, s, nn, x, r, (const T *)p, (const T *)q, L.ctrl, L.off,
                         (const double *)ppart, gs, L.iflag, j);
      precond();
      ++j;
      spmv(j, i == nbt - 1 ? ctx->h_post : nullptr, seq);
    }
    VMS_LAUNCH_CHECK(ctx);
    int rc = vms_wait_post(ctx, seq, L.iflag);
    if (rc) return rc;
    fin = ctx->h_i[IF_DONE] != 0;
    batch = next_batch(est, round++);
  }
  status_out = ctx->h_i[IF_STATUS];
  its_out = ctx->h_i[IF_ITS];
  est = std::max(1, its_out);
  if (status_out == KS_NAN) return vms_set_error(ctx, VMS_ERR_NAN, "NaN/Inf in a CG level");
  return VMS_OK;
}

template <typename T>
struct Nested {
  vms_ctx *ctx;
  const vms_mesh *mesh;
  const vms_matrix *K;
  const vms_solver_opts *o;
  int n;
  int64_t nnzb;
  const T *A, *B, *C, *D;  // scaled blocks in the level precision
  KLevel<T> LA, LS;
  T *rv, *rp, *xh, *xp, *xv, *xbar, *xt, *Minv, *sdinv;
  // pressure-mass term of the Schur preconditioner (schur_mass > 0)
  double *mlw = nullptr, *msum = nullptr;
  T *minv = nullptr, *pdiag = nullptr, *mone = nullptr, *ms1 = nullptr;
  T *Shat, *Shd, *cr, *cd0, *cd1, *px, *py;  // S^ (off-diagonal, diagonal); Chebyshev / power-iteration vectors
  T *As = nullptr;                            // (A + A^T)/2 for the CG levels (when symmetrised)
  double *cgpart = nullptr;                   // partials of <p, A p> of the CG product kernel
  double *sctl = nullptr;                     // CG steps on S^: gamma, alpha of two steps [4], partials [4][...]
  int *sflag = nullptr;
  PcgVec<T> pv{};                             // their work vectors
  T *dAinv = nullptr;                         // SIMPLE: diag(A)^-1
  double *lam = nullptr;                      // device: lmax estimate of diag(S^)^-1 S^
  AmgSys<T> mg;                               // multigrid of the A-levels (a_prec = AMG)
  vms_solve_stats *stats;
  int err = VMS_OK;

  void carve(Carver &cv, const vms_mesh *m_, const vms_solver_opts *o_) {
    const int64_t nn = m_->n_nodes;
    LA.carve(cv, 3 * nn, std::max(o_->maxit_A, o_->maxit_I));
    LS.carve(cv, nn, o_->maxit_S);
    rv = cv.take<T>(3 * nn);
    rp = cv.take<T>(nn);
    xh = cv.take<T>(3 * nn);
    xp = cv.take<T>(nn);
    xv = cv.take<T>(3 * nn);
    xbar = cv.take<T>(3 * nn);
    xt = cv.take<T>(3 * nn);
    Minv = cv.take<T>(9 * nn);
    sdinv = cv.take<T>(nn);
    Shat = cv.take<T>((int64_t)m_->shat_width * nn);
    Shd = cv.take<T>(nn);
    cr = cv.take<T>(nn);
    cd0 = cv.take<T>(nn);
    cd1 = cv.take<T>(nn);
    px = cv.take<T>(nn);
    py = cv.take<T>(nn);
    if (o_->precond == VMS_PC_SIMPLE) dAinv = cv.take<T>(3 * nn);
    if (o_->shat_method == VMS_SHAT_CG && o_->shat_degree > 0) {
      sctl = cv.take<double>(4 + 4 * VMS_MAX_RED_BLOCKS + 2);
      sflag = cv.take<int>(1);
      T **vs[9] = {&pv.r, &pv.u, &pv.w, &pv.m, &pv.nv, &pv.z, &pv.q, &pv.s, &pv.p};
      for (T **v : vs) *v = cv.take<T>(nn);
    }
    if (o_->a_krylov != VMS_AK_GMRES) {
      cgpart = cv.take<double>(cg_spmv_blocks(m_->n_nodes));
      if (o_->cg_symmetrise) As = cv.take<T>(9 * m_->nnzb);
    }
    if (o_->a_prec == VMS_APC_AMG) mg.carve(cv, m_);
    if (o_->schur_mass > 0.0) {
      mlw = cv.take<double>(nn);
      msum = cv.take<double>(4);
      minv = cv.take<T>(nn);
      pdiag = cv.take<T>(nn);
      mone = cv.take<T>(nn);
      ms1 = cv.take<T>(nn);
    }
  }

  // z = p(diag(S^)^-1 S^) diag(S^)^-1 v: degree-k Chebyshev iteration for S^ z = v
  void cheb_apply(const T *v, T *z) {
    hipStream_t s = ctx->stream;
    const int deg = o->shat_degree;
    const double ratio = o->shat_ratio > 1.0 ? o->shat_ratio : 20.0;
    const dim3 g1((n + VMS_BLOCK - 1) / VMS_BLOCK), gw(spmv_grid(n)), bl(VMS_BLOCK);
    hipLaunchKernelGGL(k_cheb_init<T>, g1, bl, 0, s, n, v, (const T *)sdinv, z, cr, cd0, (const double *)lam, ratio);
    T *d = cd0, *dn = cd1;
    for (int k = 0; k < deg; ++k) {
      hipLaunchKernelGGL((k_shat_cheb<T, 1>), gw, bl, 0, s, n, mesh->shat_width, mesh->shat_col, mesh->shat_off,
                         (const T *)Shat,
                         (const T *)Shd, (const T *)d, (const T *)sdinv, dn, z, cr, (const double *)lam, ratio, k);
      std::swap(d, dn);
    }
  }

  // z = k diag(S^)-preconditioned CG steps on S^ z = v (k = shat_degree), pipelined
  void scg_apply(const T *v, T *z) {
    hipStream_t s = ctx->stream;
    const int k = o->shat_degree;
    const int nbv = pcg_blocks(n);
    double *pg0 = sctl + 4, *pd0 = pg0 + VMS_MAX_RED_BLOCKS, *pg1 = pd0 + VMS_MAX_RED_BLOCKS,
           *pd1 = pg1 + VMS_MAX_RED_BLOCKS, *tot = pd1 + VMS_MAX_RED_BLOCKS;
    const dim3 gp(spmv_grid(n)), bl(VMS_BLOCK), gv(nbv), bk(KRY_BLOCK);
    hipLaunchKernelGGL(k_pcg_init<T>, dim3(grid1(n)), bl, 0, s, n, v, (const T *)sdinv, z, pv, sflag);
    launch_shat_spmv<T>(s, mesh, (const T *)Shat, (const T *)Shd, (const T *)pv.u, pv.w, (const int *)sflag);
    hipLaunchKernelGGL(k_pcg_start<T>, gv, bk, 0, s, n, (const T *)sdinv, pv, pg0, pd0);
    for (int i = 0; i < k; ++i) {
      // the product also totals step i's partials (buffer i & 1) for the vector step
      launch_shat_spmv<T>(s, mesh, (const T *)Shat, (const T *)Shd, (const T *)pv.m, pv.nv, (const int *)sflag,
                          (i & 1) ? pg1 : pg0, (i & 1) ? pd1 : pd0, nbv, tot);
      hipLaunchKernelGGL(k_pcg_step<T>, gv, bk, 0, s, n, i, (int)(i == k - 1), z, pv, (const T *)sdinv, sctl, pg0,
                         pd0, pg1, pd1, (const double *)tot, sflag);
    }
  }

  // lmax of diag(S^)^-1 S^ by power iteration, kept on the device
  void power_lmax(int iters) {
    hipStream_t s = ctx->stream;
    const dim3 g1((n + VMS_BLOCK - 1) / VMS_BLOCK), gw(spmv_grid(n)), bl(VMS_BLOCK);
    const int nb = vms_red_blocks(n);
    double *part = LS.ctrl + LS.off.part;
    hipLaunchKernelGGL(k_power_init<T>, g1, bl, 0, s, n, px);
    for (int it = 0; it < iters; ++it) {
      hipLaunchKernelGGL((k_shat_cheb<T, 0>), gw, bl, 0, s, n, mesh->shat_width, mesh->shat_col, mesh->shat_off,
                         (const T *)Shat,
                         (const T *)Shd, (const T *)px, (const T *)sdinv, py, (T *)nullptr, (T *)nullptr,
                         (const double *)nullptr, 0.0, 0);
      hipLaunchKernelGGL(k_norm_part<T>, dim3(nb), bl, 0, s, (int64_t)n, (const T *)py, part, (const int *)nullptr);
      hipLaunchKernelGGL(k_store_norm, dim3(1), bl, 0, s, nb, (const double *)part, lam);
      hipLaunchKernelGGL(k_power_scale<T>, g1, bl, 0, s, n, (const T *)py, (const double *)lam, px);
    }
  }

  // x = A^-1 b by GMRES with block-Jacobi (intermediate or inner level)
  int solve_A(const T *b, T *x, bool inner, bool may_relax = true) {
    int its = 0;
    const double rtol = inner ? o->rtol_I : o->rtol_A, atol = inner ? o->atol_I : o->atol_A;
    const int maxit = inner ? o->maxit_I : o->maxit_A;
    int &est = inner ? ctx->est_I : ctx->est_A;
    const bool amg = o->a_prec == VMS_APC_AMG;
    auto op = [&](int j) -> int {
      // multigrid: flexible form, Z_j = V-cycle(V_j) before the product
      if (amg) mg.vcycle(ctx->stream, 0, LA.V + (int64_t)j * LA.nvec, LA.Z + (int64_t)j * LA.nvec, LA.iflag + IF_DONE);
      launch_spmv_A<T>(ctx, mesh, A, LA.Z + (int64_t)j * LA.nvec, LA.W, LA.iflag + IF_DONE);
      return VMS_OK;
    };
    int st = 0;
    const int ph = vms_phase_begin(ctx);
    const bool cg = inner ? (o->a_krylov != VMS_AK_GMRES) : (o->a_krylov == VMS_AK_CG);
    // the inner solve of a Schur product (called only from the Schur level's
    // operator) may relax its tolerance with the Schur level's progress
    const double *relax = (inner && may_relax && o->relax_inner) ? LS.ctrl + LS.off.scal : nullptr;
    const T *Acg = o->cg_symmetrise ? (const T *)As : A;
    int rc;
    if (cg && amg)
      rc = amg_cg_run<T>(ctx, LA, mesh, Acg, cgpart, b, x, rtol, atol, maxit, mg, est, its, st, relax);
    else if (cg)
      rc = cg_run<T>(ctx, LA, mesh, Acg, cgpart, b, x, rtol, atol, maxit, Minv, est, its, st, relax);
    else
      rc = gmres_run<T>(ctx, LA, b, x, rtol, atol, maxit, o->orth, amg ? PC_NONE : PC_BJ33, Minv, false, est, op,
                        its, st, relax);
    vms_phase_end(ctx, ph, inner ? VMS_PH_INNER : VMS_PH_A);
    if (inner) { stats->n_I_solves++; stats->it_I += its; }
    else { stats->n_A_solves++; stats->it_A += its; }
    return rc;
  }

  // x_p = S^-1 b by GMRES with the matrix-free Schur product (Algorithm 2)
  int solve_S(const T *b, T *x) {
    int its = 0;
    // right preconditioner: CG steps or a Chebyshev polynomial on S^ (poly), else
    // diag(S^)^-1; plus the pressure-mass term; a diagonal one is applied inside
    // the level's normalisation
    const bool poly = o->shat_method != VMS_SHAT_NONE && o->shat_degree > 0;
    const bool mass = o->schur_mass > 0.0;
    auto op = [&](int j) -> int {
      T *z = LS.Z + (int64_t)j * LS.nvec;
      if (poly) {
        const T *v = LS.V + (int64_t)j * LS.nvec;
        if (o->shat_method == VMS_SHAT_CG) scg_apply(v, z);
        else cheb_apply(v, z);
        if (mass)
          hipLaunchKernelGGL(k_diag_axpy<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, (const T *)minv, v, z);
      }
      // x-bar = B z
      hipLaunchKernelGGL((k_spmv_B<T, T>), dim3(spmv_grid(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, nnzb,
                         mesh->slot_width, mesh->col, B, z, xbar, (const T *)nullptr, 1.0, (const int *)nullptr);
      // x-tilde = A^-1 x-bar (inner solver)
      int rc = solve_A(xbar, xt, true);
      if (rc) return rc;
      // W = D z - C x-tilde
      hipLaunchKernelGGL((k_spmv_CD<T, T>), dim3(spmv_grid(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, nnzb,
                         mesh->slot_width, mesh->col, C, D, xt, z, LS.W, (const T *)nullptr, -1.0, 1.0,
                         (const int *)nullptr);
      return VMS_OK;
    };
    int st = 0;
    int rc = gmres_run<T>(ctx, LS, b, x, o->rtol_S, o->atol_S, o->maxit_S, o->orth, poly ? PC_NONE : PC_DIAG,
                          mass ? (const T *)pdiag : (const T *)sdinv, true, ctx->est_S, op, its, st);
    stats->n_S_solves++;
    stats->it_S += its;
    return rc;
  }

  // z ~ S^-1 v by the Schur solve's preconditioner: diag(S^)^-1, Chebyshev or CG steps on S^
  void shat_prec(const T *v, T *z) {
    if (o->shat_degree <= 0)
      hipLaunchKernelGGL(k_diag_scale<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, (const T *)sdinv, v, z);
    else if (o->shat_method == VMS_SHAT_CG)
      scg_apply(v, z);
    else
      cheb_apply(v, z);
  }

  // x = S^-1 b by flexible GMRES on the assembled S^ (SIMPLE, section 4.3), right-preconditioned
  // like the Schur solve
  int solve_shat(const T *b, T *x) {
    int its = 0, st = 0;
    auto op = [&](int j) -> int {
      T *z = LS.Z + (int64_t)j * LS.nvec;
      shat_prec(LS.V + (int64_t)j * LS.nvec, z);
      launch_shat_spmv<T>(ctx->stream, mesh, (const T *)Shat, (const T *)Shd, (const T *)z, LS.W,
                          (const int *)(LS.iflag + IF_DONE));
      return VMS_OK;
    };
    int rc = gmres_run<T>(ctx, LS, b, x, o->rtol_S, o->atol_S, o->maxit_S, o->orth, PC_NONE, (const T *)nullptr,
                          true, ctx->est_S, op, its, st);
    stats->n_S_solves++;
    stats->it_S += its;
    return rc;
  }

  // x_p for the Schur step: a Krylov solve (S by Algorithm 2, or S^ for SIMPLE) or one application
  // of the S^ preconditioner
  int schur_step(const T *b, T *x) {
    const int ph = vms_phase_begin(ctx);
    int rc = VMS_OK;
    if (o->schur_solve == VMS_SCHUR_SHAT) {
      shat_prec(b, x);
      stats->n_S_solves++;
    } else {
      rc = (o->precond == VMS_PC_SIMPLE) ? solve_shat(b, x) : solve_S(b, x);
    }
    vms_phase_end(ctx, ph, VMS_PH_S);
    VMS_LAUNCH_CHECK(ctx);
    return rc;
  }

  // z = P_SCR^-1 v (Algorithm 1 and its partial-factorization variants) or P_SIMPLE^-1 v (section 4.3)
  int apply(const double *v_full, double *z_full) {
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_split<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, s, n, v_full, rv, rp);
    VMS_LAUNCH_CHECK(ctx);
    int rc;
    const int var = o->precond;
    if (var == VMS_PC_SIMPLE) {
      if ((rc = solve_A(rv, xh, false))) return rc;                 // y_v = A^-1 r_v
      hipLaunchKernelGGL((k_spmv_CD<T, T>), dim3(spmv_grid(n)), dim3(VMS_BLOCK), 0, s, n, nnzb, mesh->slot_width,
                         mesh->col, C, D, xh, (const T *)nullptr, rp, rp, -1.0, 0.0, (const int *)nullptr);
      if ((rc = schur_step(rp, xp))) return rc;                      // x_p = S^-1 (r_p - C y_v)
      hipLaunchKernelGGL((k_spmv_B<T, T>), dim3(spmv_grid(n)), dim3(VMS_BLOCK), 0, s, n, nnzb, mesh->slot_width,
                         mesh->col, B, xp, xbar, (const T *)nullptr, 1.0, (const int *)nullptr);
      hipLaunchKernelGGL(k_simple_vel<T>, dim3(grid1(3 * (int64_t)n)), dim3(VMS_BLOCK), 0, s, 3 * (int64_t)n,
                         (const T *)xh, (const T *)xbar, (const T *)dAinv, xv);  // x_v = y_v - diag(A)^-1 B x_p
      hipLaunchKernelGGL(k_merge<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, s, n, xv, xp, z_full);
      VMS_LAUNCH_CHECK(ctx);
      return VMS_OK;
    }
    if (var == VMS_PC_LDU || var == VMS_PC_LOWER) {
      if ((rc = solve_A(rv, xh, false))) return rc;                 // step 1
      hipLaunchKernelGGL((k_spmv_CD<T, T>), dim3(spmv_grid(n)), dim3(VMS_BLOCK), 0, s, n, nnzb, mesh->slot_width,
                         mesh->col, C, D, xh, (const T *)nullptr, rp, rp, -1.0, 0.0, (const int *)nullptr);  // step 2
    }
    if ((rc = schur_step(rp, xp))) return rc;                        // step 3
    if (var == VMS_PC_LDU || var == VMS_PC_UPPER) {
      hipLaunchKernelGGL((k_spmv_B<T, T>), dim3(spmv_grid(n)), dim3(VMS_BLOCK), 0, s, n, nnzb, mesh->slot_width,
                         mesh->col, B, xp, rv, rv, -1.0, (const int *)nullptr);  // step 4
      if ((rc = solve_A(rv, xv, false))) return rc;                 // step 5
    } else if (var == VMS_PC_LOWER) {
      hipLaunchKernelGGL(k_merge<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, s, n, xh, xp, z_full);
      VMS_LAUNCH_CHECK(ctx);
      return VMS_OK;
    } else {  // block diagonal
      if ((rc = solve_A(rv, xv, false))) return rc;
    }
    hipLaunchKernelGGL(k_merge<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, s, n, xv, xp, z_full);
    VMS_LAUNCH_CHECK(ctx);
    return VMS_OK;
  }

  int setup_precond() {
    const int sym = (o->a_krylov != VMS_AK_GMRES && o->cg_symmetrise);
    hipLaunchKernelGGL(k_bj33_setup<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, mesh->diag_pos, nnzb,
                       K->A, Minv, sym);
    if (sym)
      hipLaunchKernelGGL(k_sym_A<T>, dim3(grid1(nnzb)), dim3(VMS_BLOCK), 0, ctx->stream, nnzb, mesh->tpos, K->A, As);
    if (o->a_prec == VMS_APC_AMG) {
      if (!K->W) return vms_set_error(ctx, VMS_ERR_ARG, "a_prec AMG needs the scaling K->W");
      int rc = mg.setup(ctx, mesh, K, sym ? (const T *)As : A, Minv, sym);
      if (rc) return rc;
    }
    if (o->precond == VMS_PC_SIMPLE)
      hipLaunchKernelGGL(k_diagA_inv<T>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, mesh->diag_pos, nnzb,
                         K->A, dAinv);
    // S^ from the FP64 scaled blocks (stored in the level precision), and diag(S^)^-1
    hipLaunchKernelGGL(k_shat_form<T>, dim3((n + SHAT_ROWS - 1) / SHAT_ROWS), dim3(VMS_BLOCK), 0, ctx->stream, n,
                       mesh->slot_width, mesh->col, mesh->diag_pos, nnzb, K->A, K->B, K->C, K->D, mesh->shat_width,
                       mesh->shat_col, Shat, Shd, sdinv);
    if (o->shat_degree > 0 && o->shat_method == VMS_SHAT_CHEBYSHEV) {
      lam = LS.ctrl + LS.off.scal + 5;
      power_lmax(12);
    }
    if (o->schur_mass > 0.0) {
      hipStream_t s = ctx->stream;
      const dim3 g1(grid1(n)), bl(VMS_BLOCK);
      hipLaunchKernelGGL(k_mass_lumped<T>, g1, bl, 0, s, n, mesh->diag_pos, mesh->blk_src_ptr, mesh->blk_src, mesh->X,
                         mesh->tets, mesh->dir_mask, (const double *)K->W, mlw, mone);
      // The fit c = 1^T S 1 / 1^T M 1 weighs the term against the S^ part.  Alone (VMS_SHAT_NONE) the
      // term is the whole right preconditioner of the Schur level's GMRES, whose iterates do not
      // depend on its scale: c = 1 there, and no Schur product is spent on it.
      const bool fit = o->shat_method != VMS_SHAT_NONE;
      if (fit) {
        // S 1 = D 1 - C A^-1 B 1 (one Schur product, its inner solve counted with the others)
        hipLaunchKernelGGL((k_spmv_B<T, T>), dim3(spmv_grid(n)), bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, B,
                           (const T *)mone, xbar, (const T *)nullptr, 1.0, (const int *)nullptr);
        int rc = solve_A(xbar, xt, true, false);   // no Schur level is running: no relaxation
        if (rc) return rc;
        hipLaunchKernelGGL((k_spmv_CD<T, T>), dim3(spmv_grid(n)), bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, C,
                           D, (const T *)xt, (const T *)mone, ms1, (const T *)nullptr, -1.0, 1.0, (const int *)nullptr);
        hipLaunchKernelGGL(k_mass_sums<T>, dim3(1), dim3(1024), 0, s, n, (const T *)ms1, (const double *)mlw,
                           mesh->dir_mask, msum);
      }
      const bool poly = o->shat_method != VMS_SHAT_NONE && o->shat_degree > 0;
      hipLaunchKernelGGL(k_mass_inv<T>, g1, bl, 0, s, n, (const double *)mlw, fit ? (const double *)msum : nullptr,
                         mesh->dir_mask,
                         o->schur_mass, o->shat_method == VMS_SHAT_NONE ? (const T *)nullptr : (const T *)sdinv,
                         minv, poly ? (T *)nullptr : pdiag);
    }
    VMS_LAUNCH_CHECK(ctx);
    return VMS_OK;
  }
};

struct Outer {
  KLevel<double> L;
  void carve(Carver &cv, const vms_mesh *m, const vms_solver_opts *o) { L.carve(cv, 4 * (int64_t)m->n_nodes, o->maxit); }
};

// the nested solve's own workspace (Krylov bases, control blocks, temporaries)
size_t core_bytes(const vms_mesh *m, const vms_solver_opts *o) {
  Carver cv{nullptr};
  Outer ou;
  ou.carve(cv, m, o);
  if (o->precision == VMS_MIXED) {
    Nested<float> ne;
    ne.carve(cv, m, o);
  } else {
    Nested<double> ne;
    ne.carve(cv, m, o);
  }
  return cv.off + 256;
}

int check_opts(vms_ctx *ctx, const vms_solver_opts *o, const vms_mesh *m) {
  if (!o || o->maxit <= 0 || o->maxit_A <= 0 || o->maxit_S <= 0 || o->maxit_I <= 0 || o->maxit > 1000 ||
      o->maxit_A > 1000 || o->maxit_S > 1000 || o->maxit_I > 1000)
    return vms_set_error(ctx, VMS_ERR_ARG, "solver options: maxit must be in [1, 1000]");
  if (o->precond < VMS_PC_LDU || o->precond > VMS_PC_SIMPLE)
    return vms_set_error(ctx, VMS_ERR_ARG, "unknown preconditioner variant");
  if (o->precision != VMS_FP64 && o->precision != VMS_MIXED)
    return vms_set_error(ctx, VMS_ERR_ARG, "unknown precision");
  if (o->shat_degree < 0 || o->shat_degree > 64)
    return vms_set_error(ctx, VMS_ERR_ARG, "shat_degree must be in [0, 64]");
  if (o->orth != VMS_ORTH_CGS2 && o->orth != VMS_ORTH_MGS && o->orth != VMS_ORTH_CGS1 &&
      o->orth != VMS_ORTH_CGS_IFNEEDED)
    return vms_set_error(ctx, VMS_ERR_ARG, "unknown orthogonalisation");
  if (o->a_krylov != VMS_AK_GMRES && o->a_krylov != VMS_AK_CG_INNER && o->a_krylov != VMS_AK_CG)
    return vms_set_error(ctx, VMS_ERR_ARG, "unknown A-level Krylov method");
  if (o->cg_symmetrise != 0 && o->cg_symmetrise != 1)
    return vms_set_error(ctx, VMS_ERR_ARG, "cg_symmetrise must be 0 or 1");
  if (o->shat_method != VMS_SHAT_CHEBYSHEV && o->shat_method != VMS_SHAT_CG && o->shat_method != VMS_SHAT_NONE)
    return vms_set_error(ctx, VMS_ERR_ARG, "unknown S^ preconditioner method");
  if (!(o->schur_mass >= 0.0) || !std::isfinite(o->schur_mass))
    return vms_set_error(ctx, VMS_ERR_ARG, "schur_mass must be finite and >= 0");
  if (o->shat_method == VMS_SHAT_NONE && !(o->schur_mass > 0.0))
    return vms_set_error(ctx, VMS_ERR_ARG, "shat_method NONE needs schur_mass > 0");
  if ((o->schur_mass > 0.0 || o->shat_method == VMS_SHAT_NONE) &&
      (o->precond == VMS_PC_SIMPLE || o->schur_solve != VMS_SCHUR_KRYLOV))
    return vms_set_error(ctx, VMS_ERR_ARG, "the pressure-mass term needs the Krylov Schur step of P_SCR");
  if (o->schur_solve != VMS_SCHUR_KRYLOV && o->schur_solve != VMS_SCHUR_SHAT)
    return vms_set_error(ctx, VMS_ERR_ARG, "unknown Schur step");
  if (o->relax_inner != 0 && o->relax_inner != 1)
    return vms_set_error(ctx, VMS_ERR_ARG, "relax_inner must be 0 or 1");
  if (o->a_prec != VMS_APC_BJ && o->a_prec != VMS_APC_AMG)
    return vms_set_error(ctx, VMS_ERR_ARG, "unknown A-level preconditioner");
  if (o->a_prec == VMS_APC_AMG) {
    const vms_amg_dev *h = m ? vms_amg_device(m->amg) : nullptr;
    if (!h) return vms_set_error(ctx, VMS_ERR_ARG, "a_prec AMG needs mesh->amg");
    if (!h->uploaded || h->device != ctx->device)
      return vms_set_error(ctx, VMS_ERR_STATE, "the multigrid hierarchy is not uploaded to this device");
    if (h->lev[0].n != m->n_nodes || h->lev[0].nnzb != m->nnzb)
      return vms_set_error(ctx, VMS_ERR_ARG, "the multigrid hierarchy belongs to another mesh");
  }
  return VMS_OK;
}

template <typename T>
int solve_impl(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, const double *rhs, double *x,
               const vms_solver_opts *o, void *ws, vms_solve_stats *stats) {
  Carver cv{(char *)ws};
  Outer ou;
  ou.carve(cv, mesh, o);
  Nested<T> ne;
  ne.carve(cv, mesh, o);
  ne.ctx = ctx;
  ne.mesh = mesh;
  ne.K = K;
  ne.o = o;
  ne.n = mesh->n_nodes;
  ne.nnzb = mesh->nnzb;
  ne.stats = stats;
  if (std::is_same<T, float>::value) {
    ne.A = (const T *)K->A32; ne.B = (const T *)K->B32; ne.C = (const T *)K->C32; ne.D = (const T *)K->D32;
  } else {
    ne.A = (const T *)K->A; ne.B = (const T *)K->B; ne.C = (const T *)K->C; ne.D = (const T *)K->D;
  }
  const int ph_setup = vms_phase_begin(ctx);
  int rc = ne.setup_precond();
  vms_phase_end(ctx, ph_setup, VMS_PH_SETUP);
  if (rc) return rc;
  KLevel<double> &L = ou.L;
  const int n = mesh->n_nodes;
  int est_outer = 1;
  auto op = [&](int j) -> int {
    // host-driven preconditioner: Z_j = P_SCR^-1 V_j, then W = K Z_j
    int r = ne.apply(L.V + (int64_t)j * L.nvec, L.Z + (int64_t)j * L.nvec);
    if (r) return r;
    hipLaunchKernelGGL(k_spmv_full, dim3(spmv_grid(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, mesh->nnzb,
                       mesh->slot_width, mesh->col, K->A, K->B, K->C, K->D, L.Z + (int64_t)j * L.nvec, L.W,
                       L.iflag + IF_DONE);
    return VMS_OK;
  };
  // outer FGMRES: FP64, host-driven preconditioner, flags read every iteration
  hipStream_t s = ctx->stream;
  const int maxit = std::min(o->maxit, L.m);
  int status = 0, its = 0;
  // the outer FGMRES (a few iterations) always reorthogonalises, so its least-squares residual is that of a
  // numerically orthonormal basis whatever the inner levels use
  const int orth_outer = (o->orth == VMS_ORTH_MGS) ? VMS_ORTH_MGS : VMS_ORTH_CGS2;
  const int ph_outer = vms_phase_begin(ctx);
  rc = gmres_run<double>(ctx, L, rhs, x, o->rtol, o->atol, maxit, orth_outer, PC_NONE, (const double *)nullptr, true,
                         est_outer, op, its, status);
  vms_phase_end(ctx, ph_outer, VMS_PH_OUTER);
  if (rc) return rc;
  stats->n_outer = its;
  VMS_HIP(ctx, hipMemcpyAsync(ctx->h_d, L.ctrl + L.off.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  VMS_HIP(ctx, hipStreamSynchronize(s));
  stats->res0 = ctx->h_d[0];
  stats->res = (its > 0) ? ctx->h_d[2] : ctx->h_d[0];
  if (status == KS_NAN) return vms_set_error(ctx, VMS_ERR_NAN, "NaN/Inf in the outer FGMRES");
  if (status == KS_BREAKDOWN) return vms_set_error(ctx, VMS_ERR_BREAKDOWN, "outer Arnoldi breakdown");
  if (status == KS_MAXIT) {
    vms_set_error(ctx, VMS_NOT_CONVERGED, "outer FGMRES reached maxit = %d", maxit);
    return VMS_NOT_CONVERGED;
  }
  return VMS_OK;
}

// the unscaled entry points keep rhs* and x* in front of the nested solve's workspace
size_t workspace_bytes(const vms_mesh *m, const vms_solver_opts *o) {
  Carver cv{nullptr};
  cv.take<double>(4 * (int64_t)m->n_nodes);
  cv.take<double>(4 * (int64_t)m->n_nodes);
  cv.take<char>(0);
  return cv.off + core_bytes(m, o);
}

__global__ void k_wscale(int64_t n4, const double *W, const double *x, double *y) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n4) y[k] = W[k] * x[k];
}

// rhs* = W g on free dofs, 0 on Dirichlet dofs
__global__ void k_wrhs(int64_t n4, const uint8_t *dir, const double *W, const double *g, double *rhs) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n4) rhs[k] = dir[k] ? 0.0 : W[k] * g[k];
}

}  // namespace

int vms_check_solve(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, const vms_solver_opts *opts,
                    const void *workspace, size_t workspace_bytes_in, size_t need, const vms_solve_stats *stats,
                    const char *who) {
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if ((rc = check_opts(ctx, opts, mesh))) return rc;
  if (!K || !K->A || !K->B || !K->C || !K->D || !stats || !workspace)
    return vms_set_error(ctx, VMS_ERR_ARG, "%s: missing argument", who);
  if (workspace_bytes_in < need)
    return vms_set_error(ctx, VMS_ERR_WORKSPACE, "%s: workspace too small: %zu < %zu", who, workspace_bytes_in,
                         need);
  return VMS_OK;
}

size_t vms_solve_core_bytes(const vms_mesh *mesh, const vms_solver_opts *opts) { return core_bytes(mesh, opts); }

int vms_solve_core(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, const double *rhs, double *x,
                   const vms_solver_opts *opts, void *ws, vms_solve_stats *stats) {
  if (opts->precision == VMS_MIXED && (!K->A32 || !K->B32 || !K->C32 || !K->D32))
    return vms_set_error(ctx, VMS_ERR_ARG, "mixed precision needs the FP32 mirrors");
  ws = (void *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  return opts->precision == VMS_MIXED ? solve_impl<float>(ctx, mesh, K, rhs, x, opts, ws, stats)
                                      : solve_impl<double>(ctx, mesh, K, rhs, x, opts, ws, stats);
}

int vms_solve_full(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *g, const double *R,
                   const double *corr, double *delta, double eps_diag, const vms_solver_opts *opts, void *workspace,
                   vms_solve_stats *stats, vms_matrix *Kt) {
  const int64_t n4 = 4 * (int64_t)mesh->n_nodes;
  Carver cv{(char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255)};
  double *rhs = cv.take<double>(n4);
  double *xs = cv.take<double>(n4);
  char *core = cv.take<char>(0);
  const int mirror = (opts->precision == VMS_MIXED && !Kt) ? 1 : 0;
  const dim3 g4((unsigned)((n4 + VMS_BLOCK - 1) / VMS_BLOCK)), bl(VMS_BLOCK);
  int ph = vms_phase_begin(ctx);
  int rc = vms_launch_prepare(ctx, mesh, K, R, corr, R ? rhs : nullptr, eps_diag, mirror);
  if (rc) return rc;
  if (g) hipLaunchKernelGGL(k_wrhs, g4, bl, 0, ctx->stream, n4, mesh->dir_mask, (const double *)K->W, g, rhs);
  const vms_matrix *Ks = K;
  if (Kt) {
    if ((rc = vms_launch_transpose(ctx, mesh, K, Kt, opts->precision == VMS_MIXED))) return rc;
    Ks = Kt;
  }
  vms_phase_end(ctx, ph, VMS_PH_SCALE);
  rc = vms_solve_core(ctx, mesh, Ks, rhs, xs, opts, core, stats);
  if (rc < 0) return rc;
  ph = vms_phase_begin(ctx);
  hipLaunchKernelGGL(k_wscale, g4, bl, 0, ctx->stream, n4, (const double *)K->W, (const double *)xs, delta);
  vms_phase_end(ctx, ph, VMS_PH_SCALE);
  VMS_LAUNCH_CHECK(ctx);
  return rc;
}

extern "C" size_t vms_solve_workspace(const vms_mesh *mesh, const vms_solver_opts *opts) {
  if (!mesh || !opts || mesh->n_nodes <= 0) return 0;
  return workspace_bytes(mesh, opts);
}

extern "C" int vms_solve(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *R, const double *corr,
                         double *delta, double eps_diag, const vms_solver_opts *opts, void *workspace,
                         size_t workspace_bytes_in, vms_solve_stats *stats) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_solve(ctx, mesh, K, opts, workspace, workspace_bytes_in,
                           workspace_bytes(mesh, opts), stats, "vms_solve");
  if (rc) return rc;
  if (!R || !delta || !K->W) return vms_set_error(ctx, VMS_ERR_ARG, "vms_solve: missing argument");
  std::memset(stats, 0, sizeof(*stats));
  vms_phase_reset(ctx);
  const auto t0 = std::chrono::steady_clock::now();
  rc = vms_solve_full(ctx, mesh, K, nullptr, R, corr, delta, eps_diag, opts, workspace, stats, nullptr);
  if (rc >= 0) {
    VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    vms_phase_finish(ctx, stats);
  }
  stats->status = rc;
  stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

extern "C" int vms_solve_scaled(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, const double *rhs_scaled,
                                double *x_scaled, const vms_solver_opts *opts, void *workspace,
                                size_t workspace_bytes_in, vms_solve_stats *stats) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_solve(ctx, mesh, K, opts, workspace, workspace_bytes_in, core_bytes(mesh, opts), stats,
                           "vms_solve_scaled");
  if (rc) return rc;
  if (!rhs_scaled || !x_scaled) return vms_set_error(ctx, VMS_ERR_ARG, "vms_solve_scaled: missing argument");
  std::memset(stats, 0, sizeof(*stats));
  vms_phase_reset(ctx);
  const auto t0 = std::chrono::steady_clock::now();
  rc = vms_solve_core(ctx, mesh, K, rhs_scaled, x_scaled, opts, workspace, stats);
  if (rc >= 0) {
    VMS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    vms_phase_finish(ctx, stats);
  }
  stats->status = rc;
  stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

int vms_launch_spmv(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, int op, const void *x, void *y,
                    int fp32) {
  const int n = mesh->n_nodes;
  const int64_t nnzb = mesh->nnzb;
  dim3 gr(spmv_grid(n)), bl(VMS_BLOCK);
  hipStream_t s = ctx->stream;
  if (fp32 && op == VMS_OP_FULL) return vms_set_error(ctx, VMS_ERR_ARG, "FULL product is FP64 only");
  if (fp32 ? (!K->A32 || !K->B32 || !K->C32 || !K->D32) : (!K->A || !K->B || !K->C || !K->D))
    return vms_set_error(ctx, VMS_ERR_ARG, "matrix arrays missing");
  const int *nd = nullptr;
  switch (op) {
    case VMS_OP_FULL:
      hipLaunchKernelGGL(k_spmv_full, gr, bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, K->A, K->B, K->C, K->D,
                         (const double *)x, (double *)y, nd);
      break;
    case VMS_OP_A:
      if (fp32)
        launch_spmv_A<float>(ctx, mesh, K->A32, (const float *)x, (float *)y, nd);
      else
        launch_spmv_A<double>(ctx, mesh, K->A, (const double *)x, (double *)y, nd);
      break;
    case VMS_OP_B:
      if (fp32)
        hipLaunchKernelGGL((k_spmv_B<float, float>), gr, bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, K->B32,
                           (const float *)x, (float *)y, (const float *)nullptr, 1.0, nd);
      else
        hipLaunchKernelGGL((k_spmv_B<double, double>), gr, bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, K->B,
                           (const double *)x, (double *)y, (const double *)nullptr, 1.0, nd);
      break;
    case VMS_OP_C:
      if (fp32)
        hipLaunchKernelGGL((k_spmv_CD<float, float>), gr, bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, K->C32,
                           K->D32, (const float *)x, (const float *)nullptr, (float *)y, (const float *)nullptr, 1.0,
                           0.0, nd);
      else
        hipLaunchKernelGGL((k_spmv_CD<double, double>), gr, bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, K->C, K->D,
                           (const double *)x, (const double *)nullptr, (double *)y, (const double *)nullptr, 1.0,
                           0.0, nd);
      break;
    case VMS_OP_D:
      if (fp32)
        hipLaunchKernelGGL((k_spmv_CD<float, float>), gr, bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, K->C32,
                           K->D32, (const float *)nullptr, (const float *)x, (float *)y, (const float *)nullptr, 0.0,
                           1.0, nd);
      else
        hipLaunchKernelGGL((k_spmv_CD<double, double>), gr, bl, 0, s, n, nnzb, mesh->slot_width, mesh->col, K->C, K->D,
                           (const double *)nullptr, (const double *)x, (double *)y, (const double *)nullptr, 0.0,
                           1.0, nd);
      break;
    default:
      return vms_set_error(ctx, VMS_ERR_ARG, "unknown operator id %d", op);
  }
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

extern "C" int vms_spmv(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, int op, const void *x, void *y,
                        int fp32) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if (!K || !x || !y) return vms_set_error(ctx, VMS_ERR_ARG, "vms_spmv: missing argument");
  return vms_launch_spmv(ctx, mesh, K, op, x, y, fp32);
}

extern "C" int vms_schur_hat(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, double *S, double *Sdiag,
                             double *sdinv) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if (!K || !K->A || !K->B || !K->C || !K->D || !S || !Sdiag || !sdinv)
    return vms_set_error(ctx, VMS_ERR_ARG, "vms_schur_hat: missing argument");
  const int n = mesh->n_nodes;
  hipLaunchKernelGGL(k_shat_form<double>, dim3((n + SHAT_ROWS - 1) / SHAT_ROWS), dim3(VMS_BLOCK), 0, ctx->stream, n,
                     mesh->slot_width, mesh->col, mesh->diag_pos, mesh->nnzb, K->A, K->B, K->C, K->D,
                     mesh->shat_width, mesh->shat_col, S, Sdiag, sdinv);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

extern "C" int vms_shat_spmv(vms_ctx *ctx, const vms_mesh *mesh, const void *S, const void *Sd, const void *x,
                             void *y, int fp32) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if (!S || !Sd || !x || !y) return vms_set_error(ctx, VMS_ERR_ARG, "vms_shat_spmv: missing argument");
  if (x == y) return vms_set_error(ctx, VMS_ERR_ARG, "vms_shat_spmv: x and y must not alias");
  if (fp32)
    launch_shat_spmv<float>(ctx->stream, mesh, (const float *)S, (const float *)Sd, (const float *)x, (float *)y,
                            nullptr);
  else
    launch_shat_spmv<double>(ctx->stream, mesh, (const double *)S, (const double *)Sd, (const double *)x,
                             (double *)y, nullptr);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

// ---- one multigrid V-cycle (the A-levels' preconditioner on its own) -------------
namespace {
struct AmgApplyWs {
  double *Minv = nullptr, *As = nullptr;
  AmgSys<double> mg;
  void carve(Carver &cv, const vms_mesh *m, int sym) {
    Minv = cv.take<double>(9 * (int64_t)m->n_nodes);
    if (sym) As = cv.take<double>(9 * m->nnzb);
    mg.carve(cv, m);
  }
};
}  // namespace

extern "C" size_t vms_amg_apply_workspace(const vms_mesh *mesh, int sym) {
  if (!mesh || mesh->n_nodes <= 0 || !vms_amg_device(mesh->amg)) return 0;
  Carver cv{nullptr};
  AmgApplyWs w;
  w.carve(cv, mesh, sym ? 1 : 0);
  return cv.off + 256;
}

extern "C" int vms_amg_apply(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, int sym, const double *r,
                             double *z, void *workspace, size_t workspace_bytes) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  vms_solver_opts o{};
  o.maxit = o.maxit_A = o.maxit_S = o.maxit_I = 1;
  o.a_prec = VMS_APC_AMG;
  o.orth = VMS_ORTH_CGS1;
  o.a_krylov = VMS_AK_GMRES;
  o.shat_method = VMS_SHAT_CG;
  if ((rc = check_opts(ctx, &o, mesh))) return rc;
  if (!K || !K->A || !K->W || !r || !z || !workspace)
    return vms_set_error(ctx, VMS_ERR_ARG, "vms_amg_apply: missing argument");
  if (sym != 0 && sym != 1) return vms_set_error(ctx, VMS_ERR_ARG, "vms_amg_apply: sym must be 0 or 1");
  const size_t need = vms_amg_apply_workspace(mesh, sym);
  if (workspace_bytes < need)
    return vms_set_error(ctx, VMS_ERR_WORKSPACE, "vms_amg_apply: workspace too small: %zu < %zu", workspace_bytes,
                         need);
  Carver cv{(char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255)};
  AmgApplyWs w;
  w.carve(cv, mesh, sym);
  hipStream_t s = ctx->stream;
  const int n = mesh->n_nodes;
  hipLaunchKernelGGL(k_bj33_setup<double>, dim3(grid1(n)), dim3(VMS_BLOCK), 0, s, n, mesh->diag_pos, mesh->nnzb,
                     (const double *)K->A, w.Minv, sym);
  if (sym)
    hipLaunchKernelGGL(k_sym_A<double>, dim3(grid1(mesh->nnzb)), dim3(VMS_BLOCK), 0, s, mesh->nnzb, mesh->tpos,
                       (const double *)K->A, w.As);
  if ((rc = w.mg.setup(ctx, mesh, K, sym ? (const double *)w.As : (const double *)K->A, (const double *)w.Minv,
                       sym)))
    return rc;
  w.mg.vcycle(s, 0, r, z, nullptr);
  VMS_LAUNCH_CHECK(ctx);
  VMS_HIP(ctx, hipMemcpyAsync(ctx->h_i, w.mg.bad, sizeof(int), hipMemcpyDeviceToHost, s));
  VMS_HIP(ctx, hipStreamSynchronize(s));
  if (ctx->h_i[0]) return vms_set_error(ctx, VMS_ERR_BREAKDOWN, "vms_amg_apply: singular coarse diagonal block");
  return VMS_OK;
}

// ---- time step ---------------------------------------------------------------
extern "C" size_t vms_step_workspace(const vms_mesh *mesh, const vms_solver_opts *opts) {
  if (!mesh || !opts || mesh->n_nodes <= 0) return 0;
  // R, corr and Delta, then one region that the assembly's element buffers and the solver use in turn
  const size_t asm_b = vms_asm_scratch_bytes(mesh, VMS_ASM_TANGENT | VMS_ASM_RKCORR);
  const size_t sol_b = workspace_bytes(mesh, opts);
  return (sol_b > asm_b ? sol_b : asm_b) + 3 * (size_t)(4 * mesh->n_nodes) * sizeof(double) + 4 * 256;
}

extern "C" int vms_step(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_timeint *ti,
                        vms_state *st, const double *f_ext, vms_matrix *K, const vms_newton_opts *no,
                        const vms_solver_opts *so, void *workspace, size_t workspace_bytes_in,
                        vms_step_stats *stats) {
  if (!ctx) return VMS_ERR_ARG;
  int rc = vms_check_mesh(ctx, mesh);
  if (rc) return rc;
  if ((rc = check_opts(ctx, so, mesh))) return rc;
  if (!mat || !ti || !st || !K || !no || !stats || !workspace || no->l_max <= 0 || !(ti->dt > 0.0))
    return vms_set_error(ctx, VMS_ERR_ARG, "vms_step: missing argument");
  if (no->dir_lift != 0 && no->dir_lift != 1) return vms_set_error(ctx, VMS_ERR_ARG, "dir_lift must be 0 or 1");
  if (no->dir_lift && !no->rk_corr)
    return vms_set_error(ctx, VMS_ERR_ARG, "the lifted Dirichlet predictor needs rk_corr");
  const size_t need = vms_step_workspace(mesh, so);
  if (workspace_bytes_in < need)
    return vms_set_error(ctx, VMS_ERR_WORKSPACE, "workspace too small: %zu < %zu", workspace_bytes_in, need);
  if (so->precision == VMS_MIXED && (!K->A32 || !K->B32 || !K->C32 || !K->D32))
    return vms_set_error(ctx, VMS_ERR_ARG, "mixed precision needs the FP32 mirrors");
  std::memset(stats, 0, sizeof(*stats));
  const auto t_start = std::chrono::steady_clock::now();
  const int n = mesh->n_nodes;
  Carver cv{(char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255)};
  double *R = cv.take<double>(4 * (int64_t)n);
  double *corr = cv.take<double>(4 * (int64_t)n);
  double *delta = cv.take<double>(4 * (int64_t)n);
  char *sws = (char *)cv.take<char>(0);
  const size_t sws_bytes = workspace_bytes_in - (size_t)(sws - (char *)workspace);
  const vms_ga ga = vms_genalpha(ti);
  hipStream_t s = ctx->stream;
  if ((rc = vms_launch_predictor(ctx, mesh, ga, ti->t_n + ti->dt, st, no->dir_lift))) return rc;
  hipLaunchKernelGGL(k_clear_ints, dim3(1), dim3(64), 0, s, &ctx->dstat->inverted, 1);
  double R0 = -1.0;
  stats->status = VMS_NOT_CONVERGED;
  for (int l = 1; l <= no->l_max; ++l) {
    auto ta = std::chrono::steady_clock::now();
    if ((rc = vms_launch_assemble(ctx, mesh, mat, ga, st, f_ext, nullptr, R, nullptr, VMS_ASM_RESIDUAL, sws,
                                  sws_bytes)))
      return rc;
    if ((rc = vms_launch_norm(ctx, mesh, ga, st, R))) return rc;
    VMS_HIP(ctx, hipMemcpyAsync(ctx->h_d, ctx->dstat, 24, hipMemcpyDeviceToHost, s));
    VMS_HIP(ctx, hipStreamSynchronize(s));
    const int inverted = ((const int *)ctx->h_d)[0];
    const double nrm = sqrt(ctx->h_d[2]);
    if (inverted) return vms_set_error(ctx, VMS_ERR_INVERTED_ELEMENT, "element with J <= 0 at iteration %d", l);
    if (!std::isfinite(nrm)) return vms_set_error(ctx, VMS_ERR_NAN, "residual norm is not finite");
    if (l - 1 < 32) stats->res_norm[l - 1] = nrm;
    if (R0 < 0.0) R0 = nrm;
    // lifted form: the predictor's residual lacks the prescribed motion (it arrives with the first
    // corrector), so the relative test takes the largest residual of the iterates so far
    if (no->dir_lift && nrm > R0) R0 = nrm;
    if ((R0 > 0.0 && nrm / R0 <= no->tol_R) || nrm <= no->tol_A) {
      stats->status = VMS_OK;
      stats->ms_assemble += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
      break;
    }
    const unsigned fl = VMS_ASM_TANGENT | (no->rk_corr ? VMS_ASM_RKCORR : 0u);
    if ((rc = vms_launch_assemble(ctx, mesh, mat, ga, st, f_ext, K, nullptr, no->rk_corr ? corr : nullptr, fl, sws,
                                  sws_bytes)))
      return rc;
    VMS_HIP(ctx, hipStreamSynchronize(s));
    auto tb = std::chrono::steady_clock::now();
    stats->ms_assemble += std::chrono::duration<double, std::milli>(tb - ta).count();
    // solve(K, R) -> Delta: Dirichlet rows, scaling, nested solve, Delta = W x*
    vms_solve_stats ss;
    std::memset(&ss, 0, sizeof(ss));
    vms_phase_reset(ctx);
    rc = vms_solve_full(ctx, mesh, K, nullptr, R, no->rk_corr ? corr : nullptr, delta, no->eps_diag, so, sws, &ss,
                        nullptr);
    if (rc >= 0) {
      VMS_HIP(ctx, hipStreamSynchronize(s));
      vms_phase_finish(ctx, &ss);
    }
    ss.status = rc;
    ss.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
    stats->ms_solve += ss.ms_total;
    stats->last = ss;
    stats->it_outer_total += ss.n_outer;
    stats->it_A_total += ss.it_A;
    stats->it_S_total += ss.it_S;
    stats->it_I_total += ss.it_I;
    stats->ms_scale_total += ss.ms_scale;
    stats->ms_setup_total += ss.ms_setup;
    stats->ms_outer_total += ss.ms_outer;
    stats->ms_A_solve_total += ss.ms_A;
    stats->ms_S_solve_total += ss.ms_S;
    stats->ms_inner_total += ss.ms_inner;
    if (rc < 0) return rc;
    if ((rc = vms_launch_update(ctx, mesh, ga, st, nullptr, delta, no->dir_lift))) return rc;
    stats->n_newton = l;
  }
  VMS_HIP(ctx, hipStreamSynchronize(s));
  stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (stats->status != VMS_OK) {
    vms_set_error(ctx, VMS_NOT_CONVERGED, "Newton did not converge in %d iterations", no->l_max);
    return VMS_NOT_CONVERGED;
  }
  return VMS_OK;
}
