// Device part of the aggregation multigrid that preconditions the A-level
// solves (included by solver.hip inside its anonymous namespace).  The
// mesh-dependent arrays (aggregates, tentative prolongators, coarse patterns,
// Galerkin lists) come from amg_setup.cpp; per linear system the kernels here
// form
//   A_1 = P*^T A P*  with P* = W^-1 Q (the scaled system x = W x*: the W of
//                    the velocity dofs divides the unscaled prolongator Q),
//   A_{l+1} = Q_l^T A_l Q_l on coarser levels (FP64, summed over each coarse
//                    block's list in the finer level's block order),
// the inverses of their 10x10 diagonal blocks (the finest level uses the 3x3
// block-Jacobi inverses of the solver) and the Chebyshev bound lmax of
// D^-1 A_l (1.1 times the ratio after 12 power steps from a SplitMix64
// vector).  A V-cycle is then: Chebyshev pre-smoothing from zero, residual,
// restriction, the coarser level, prolongation, Chebyshev post-smoothing; the
// coarsest level only smooths from zero.  Every kernel returns at once when
// the Krylov level's `done` flag is set (iterations enqueued past convergence).
//
// Layouts.  Finest level: the mesh's fixed-slot 3x3 blocks (entry-major),
// vectors [n][3], 16 lanes per row as in the block products.  Coarse levels:
// CSR of 10x10 blocks stored block-major ([nnzb][10][10], row-major blocks),
// vectors [n][10]; the products take one wavefront per row (each lane owns two
// adjacent entries of every block, so the blocks are read contiguously), the
// row's ten sums go through LDS to the ten lanes that apply the 10x10
// block-diagonal inverse.
#pragma once

#define AMG_NM 10
#define AMG_CROWS 25
#define AMG_RATIO 30.0
#define AMG_POWER_STEPS 12
#define AMG_LMAX_SAFETY 1.1

inline int amg_cgrid(int n) { return (n + AMG_CROWS - 1) / AMG_CROWS; }

// output i of SplitMix64 (Steele, Lea and Flood 2014) started at `seed`, mapped to [-1, 1)
__device__ __forceinline__ double splitmix_unit(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

// Chebyshev constants on [lmax / AMG_RATIO, lmax]: theta, and for step k the coefficients of
// d_{k+1} = c1 d_k + c2 r with rho_0 = 1/sigma, rho_{k+1} = 1 / (2 sigma - rho_k)
__device__ __forceinline__ void amg_cheb(double lmax, int k, double &theta, double &c1, double &c2) {
  const double lmin = lmax / AMG_RATIO;
  theta = 0.5 * (lmax + lmin);
  const double delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma, rn = 0.0;
  for (int q = 0; q <= k; ++q) {
    rn = 1.0 / (2.0 * sigma - rho);
    if (q < k) rho = rn;
  }
  c1 = rn * rho;
  c2 = 2.0 * rn / delta;
}

__device__ __forceinline__ bool amg_done(const int *done) { return done && *done; }

// ---- finest level (3x3 fixed-slot blocks, 16 lanes per row) ---------------------------------

// row sums (A x)_row for all three components, valid in all 16 lanes of the row; in FP64 the
// matrix values and column indices, read once per pass, are loaded non-temporally so that they
// do not evict the gathered vector from the caches
template <typename T, bool NT = sizeof(T) == 8>
__device__ __forceinline__ void amgf_row(int64_t nnzb, int b0, int b1, int lane, const int32_t *__restrict__ col,
                                         const T *__restrict__ A, const T *__restrict__ x, double &a0, double &a1,
                                         double &a2) {
  a0 = a1 = a2 = 0.0;
  for (int b = b0 + lane; b < b1; b += 16) {
    const int64_t o = 3 * (int64_t)ldc<NT>(col, b);
    const double x0 = ld(x, o), x1 = ld(x, o + 1), x2 = ld(x, o + 2);
    a0 += ldm<NT>(A, 0 * nnzb + b) * x0 + ldm<NT>(A, 1 * nnzb + b) * x1 + ldm<NT>(A, 2 * nnzb + b) * x2;
    a1 += ldm<NT>(A, 3 * nnzb + b) * x0 + ldm<NT>(A, 4 * nnzb + b) * x1 + ldm<NT>(A, 5 * nnzb + b) * x2;
    a2 += ldm<NT>(A, 6 * nnzb + b) * x0 + ldm<NT>(A, 7 * nnzb + b) * x1 + ldm<NT>(A, 8 * nnzb + b) * x2;
  }
  a0 = reduce16(a0);
  a1 = reduce16(a1);
  a2 = reduce16(a2);
}

// component c of M w for the row's 3x3 block M (row-major)
template <typename T>
__device__ __forceinline__ double bj3_comp(const T *M, int c, double w0, double w1, double w2) {
  return ld(M, 3 * c) * w0 + ld(M, 3 * c + 1) * w1 + ld(M, 3 * c + 2) * w2;
}

// zero start: r = M b, d = r / theta, x = d (no product)
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_amgf_cheb0(int n, const T *__restrict__ Minv, const T *__restrict__ b, T *x, T *r, T *d, const double *lam,
             const int *done) {
  if (amg_done(done)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double th, c1, c2;
  amg_cheb(*lam, 0, th, c1, c2);
  const double b0 = ld(b, 3 * (int64_t)i), b1 = ld(b, 3 * (int64_t)i + 1), b2 = ld(b, 3 * (int64_t)i + 2);
  const T *M = Minv + 9 * (int64_t)i;
  for (int c = 0; c < 3; ++c) {
    const double z = bj3_comp(M, c, b0, b1, b2);
    r[3 * (int64_t)i + c] = (T)z;
    const T dz = (T)(z / th);
    d[3 * (int64_t)i + c] = dz;
    x[3 * (int64_t)i + c] = dz;
  }
}

// start from x: r = M (b - A x), d = r / theta (x += d is left to the next step)
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_amgf_chebres(int n, int64_t nnzb, int W, const int32_t *__restrict__ col, const T *__restrict__ A,
               const T *__restrict__ Minv, const T *__restrict__ b, const T *__restrict__ x, T *r, T *d,
               const double *lam, const int *done) {
  SPMV_PROLOGUE
  // the row's own operands are requested before the product, so their loads overlap its loads
  const bool own = act && lane < 3;
  const int64_t o = 3 * (int64_t)(act ? row : 0);
  const int c = own ? lane : 0;
  double bo0 = 0.0, bo1 = 0.0, bo2 = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
  if (own) {
    bo0 = ld(b, o); bo1 = ld(b, o + 1); bo2 = ld(b, o + 2);
    const T *M = Minv + 9 * (int64_t)row + 3 * c;
    m0 = ld(M, 0); m1 = ld(M, 1); m2 = ld(M, 2);
  }
  const double lamv = *lam;
  double a0, a1, a2;
  amgf_row(nnzb, b0, b1, lane, col, A, x, a0, a1, a2);
  if (!own) return;
  double th, c1, c2;
  amg_cheb(lamv, 0, th, c1, c2);
  const double w0 = bo0 - a0, w1 = bo1 - a1, w2 = bo2 - a2;
  const double z = m0 * w0 + m1 * w1 + m2 * w2;
  r[o + c] = (T)z;
  d[o + c] = (T)(z / th);
}

// Chebyshev step k: r -= M A d_k, d_{k+1} = c1 d_k + c2 r, x += (pending ? d_k : 0) + d_{k+1}.
// CACHED: plain loads of the matrix (the post-smoothing steps, so that the A-values they leave in
// the caches serve the Krylov product that follows the V-cycle).
template <typename T, bool CACHED = false>
__global__ void __launch_bounds__(VMS_BLOCK)
k_amgf_step(int n, int64_t nnzb, int W, const int32_t *__restrict__ col, const T *__restrict__ A,
            const T *__restrict__ Minv, const T *__restrict__ dk, T *dn, T *r, T *x, const double *lam, int k,
            int pending, const int *done) {
  SPMV_PROLOGUE
  // the row's own operands are requested before the product, so their loads overlap its loads
  const bool own = act && lane < 3;
  const int64_t o = 3 * (int64_t)(act ? row : 0) + (own ? lane : 0);
  double ro = 0.0, dko = 0.0, xo = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
  if (own) {
    ro = ld(r, o); dko = ld(dk, o); xo = ld(x, o);
    const T *M = Minv + 9 * (int64_t)row + 3 * lane;
    m0 = ld(M, 0); m1 = ld(M, 1); m2 = ld(M, 2);
  }
  const double lamv = *lam;
  double a0, a1, a2;
  amgf_row<T, sizeof(T) == 8 && !CACHED>(nnzb, b0, b1, lane, col, A, dk, a0, a1, a2);
  if (!own) return;
  double th, c1, c2;
  amg_cheb(lamv, k, th, c1, c2);
  const double z = m0 * a0 + m1 * a1 + m2 * a2;
  const double rn = ro - z;
  const double dnv = c1 * dko + c2 * rn;
  r[o] = (T)rn;
  dn[o] = (T)dnv;
  x[o] = (T)(xo + (pending ? dko : 0.0) + dnv);
}

// restriction, first half: the residual res = b - A x of the row and its ten mode contributions
// t[i][a] = sum_r Q[i][r][a] res_r / W[i][r] (lane a of the row's 16)
template <typename T, typename TP>
__global__ void __launch_bounds__(VMS_BLOCK)
k_amgf_resid_t(int n, int64_t nnzb, int W, const int32_t *__restrict__ col, const T *__restrict__ A,
               const T *__restrict__ b, const T *__restrict__ x, const TP *__restrict__ Q,
               const double *__restrict__ Wsc, T *t, const int *done) {
  SPMV_PROLOGUE
  // the row's own operands are requested before the product, so their loads overlap its loads
  const bool own = act && lane < AMG_NM;
  const int64_t o = 3 * (int64_t)(act ? row : 0);
  double bo0 = 0.0, bo1 = 0.0, bo2 = 0.0, w0 = 1.0, w1 = 1.0, w2 = 1.0, q0 = 0.0, q1 = 0.0, q2 = 0.0;
  if (own) {
    bo0 = ld(b, o); bo1 = ld(b, o + 1); bo2 = ld(b, o + 2);
    w0 = Wsc[4 * (int64_t)row]; w1 = Wsc[4 * (int64_t)row + 1]; w2 = Wsc[4 * (int64_t)row + 2];
    const TP *q = Q + (int64_t)row * 3 * AMG_NM + lane;
    q0 = ld(q, 0); q1 = ld(q, AMG_NM); q2 = ld(q, 2 * AMG_NM);
  }
  double a0, a1, a2;
  amgf_row(nnzb, b0, b1, lane, col, A, x, a0, a1, a2);
  if (!own) return;
  const double r0 = (bo0 - a0) / w0;
  const double r1 = (bo1 - a1) / w1;
  const double r2 = (bo2 - a2) / w2;
  t[(int64_t)row * AMG_NM + lane] = (T)(q0 * r0 + q1 * r1 + q2 * r2);
}

// y = M A x (power iteration)
template <typename T>
__global__ void __launch_bounds__(VMS_BLOCK)
k_amgf_dapply(int n, int64_t nnzb, int W, const int32_t *__restrict__ col, const T *__restrict__ A,
              const T *__restrict__ Minv, const T *__restrict__ x, T *y) {
  const int *done = nullptr;
  SPMV_PROLOGUE
  double a0, a1, a2;
  amgf_row(nnzb, b0, b1, lane, col, A, x, a0, a1, a2);
  if (!act || lane >= 3) return;
  y[3 * (int64_t)row + lane] = (T)bj3_comp(Minv + 9 * (int64_t)row, lane, a0, a1, a2);
}

// ---- coarse levels (10x10 CSR blocks) -----------------------------------------------------
// Block-row products: one wavefront per row.  Lane j < 50 owns the entries 2j and 2j+1 of every
// block of the row (block row j / 5, columns 2 (j % 5) and 2 (j % 5) + 1), so each block is read
// as 800 (FP64) or 400 (FP32) contiguous bytes in one load per lane, and the row's blocks are
// contiguous in CSR order.  The five partial sums of a block row are added in lane order
// through LDS; lanes 0..9 then finish the row's ten components.

template <typename T> struct Pair2;
template <> struct Pair2<double> { using V = double2; };
template <> struct Pair2<float> { using V = float2; };

// lane j's partial of (A x) over the row's blocks; j < 50, A and x 2-element aligned
template <typename T>
__device__ __forceinline__ double amgc_row_part(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                const T *__restrict__ A, const T *__restrict__ x, int row, int j) {
  using V = typename Pair2<T>::V;
  const int c = 2 * (j % 5);
  const int k0 = ptr[row], k1 = ptr[row + 1];
  double acc = 0.0;
#pragma unroll 4
  for (int k = k0; k < k1; ++k) {
    const V a = *(const V *)(A + (int64_t)k * (AMG_NM * AMG_NM) + 2 * j);
    const V xv = *(const V *)(x + (int64_t)col[k] * AMG_NM + c);
    acc += (double)a.x * (double)xv.x;
    acc += (double)a.y * (double)xv.y;
  }
  return acc;
}

// The ten block-row sums of (A x) for the wavefront's row into sw[0..9].  Every thread of the
// workgroup calls it (two barriers); rows past n give zeros.
template <typename T>
__device__ __forceinline__ void amgc_row_sums(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                              const T *__restrict__ A, const T *__restrict__ x, int row, bool act,
                                              int j, double *sp, double *sw) {
  sp[j] = act && j < 5 * AMG_NM ? amgc_row_part(ptr, col, A, x, row, j) : 0.0;
  __syncthreads();
  if (j < AMG_NM) sw[j] = sp[5 * j] + sp[5 * j + 1] + sp[5 * j + 2] + sp[5 * j + 3] + sp[5 * j + 4];
  __syncthreads();
}

#define AMG_WROWS 4   // rows (wavefronts) per 256-thread workgroup of the block-row products
inline int amg_wgrid(int n) { return (n + AMG_WROWS - 1) / AMG_WROWS; }

// the wavefront's row and lane: the row index is made wave-uniform for the CSR bounds
#define AMGC_WAVE_PROLOGUE                                                        \
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));       \
  const int j = threadIdx.x & 63;                                                \
  const int row = blockIdx.x * AMG_WROWS + wv;                                   \
  const bool act = row < n;

template <typename T>
__device__ __forceinline__ double amgc_dapply(const T *__restrict__ Dinv, int row, int rr, const double *w) {
  const T *m = Dinv + (int64_t)row * (AMG_NM * AMG_NM) + rr * AMG_NM;
  double z = 0.0;
#pragma unroll
  for (int c = 0; c < AMG_NM; ++c) z += ld(m, c) * w[c];
  return z;
}

// ten lanes per row, 25 rows per 256-thread workgroup (no product)
template <typename T>
__global__ void __launch_bounds__(256)
k_amgc_cheb0(int n, const T *__restrict__ Dinv, const T *__restrict__ b, T *x, T *r, T *d, const double *lam,
             const int *done) {
  if (amg_done(done)) return;
  const int t = threadIdx.x, row = blockIdx.x * AMG_CROWS + t / AMG_NM, rr = t % AMG_NM;
  if (t >= AMG_CROWS * AMG_NM || row >= n) return;
  double th, c1, c2;
  amg_cheb(*lam, 0, th, c1, c2);
  double w[AMG_NM];
#pragma unroll
  for (int c = 0; c < AMG_NM; ++c) w[c] = ld(b, (int64_t)row * AMG_NM + c);
  const double z = amgc_dapply(Dinv, row, rr, w);
  const int64_t o = (int64_t)row * AMG_NM + rr;
  r[o] = (T)z;
  const T dz = (T)(z / th);
  d[o] = dz;
  x[o] = dz;
}

// MODE 0: start from x (r = D^-1 (b - A x), d = r / theta); MODE 1: step k (as the finest level's)
template <typename T, int MODE>
__global__ void __launch_bounds__(256)
k_amgc_cheb(int n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col, const T *__restrict__ A,
            const T *__restrict__ Dinv, const T *__restrict__ b, const T *__restrict__ v, T *dn, T *r, T *x,
            const double *lam, int k, int pending, const int *done) {
  __shared__ double sp[AMG_WROWS][64], sw[AMG_WROWS][AMG_NM];
  if (amg_done(done)) return;
  AMGC_WAVE_PROLOGUE
  amgc_row_sums(ptr, col, A, v, row, act, j, sp[wv], sw[wv]);
  if (!act || j >= AMG_NM) return;
  const int64_t o = (int64_t)row * AMG_NM + j;
  double w[AMG_NM];
#pragma unroll
  for (int c = 0; c < AMG_NM; ++c) w[c] = MODE == 0 ? ld(b, (int64_t)row * AMG_NM + c) - sw[wv][c] : sw[wv][c];
  double th, c1, c2;
  amg_cheb(*lam, k, th, c1, c2);
  const double z = amgc_dapply(Dinv, row, j, w);
  if (MODE == 0) {
    r[o] = (T)z;
    dn[o] = (T)(z / th);
  } else {
    const double rn = ld(r, o) - z;
    const double dko = ld(v, o);
    const double dnv = c1 * dko + c2 * rn;
    r[o] = (T)rn;
    dn[o] = (T)dnv;
    x[o] = (T)(ld(x, o) + (pending ? dko : 0.0) + dnv);
  }
}

// coarse level: residual of the row and its mode contributions t[i][a] = sum_r Q[i][r][a] res_r
template <typename T, typename TP>
__global__ void __launch_bounds__(256)
k_amgc_resid_t(int n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col, const T *__restrict__ A,
               const T *__restrict__ b, const T *__restrict__ x, const TP *__restrict__ Q, T *t, const int *done) {
  __shared__ double sp[AMG_WROWS][64], sw[AMG_WROWS][AMG_NM];
  if (amg_done(done)) return;
  AMGC_WAVE_PROLOGUE
  amgc_row_sums(ptr, col, A, x, row, act, j, sp[wv], sw[wv]);
  if (!act || j >= AMG_NM) return;
  const TP *q = Q + (int64_t)row * AMG_NM * AMG_NM + j;   // column j of the row's 10x10 block
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < AMG_NM; ++r) acc += ld(q, r * AMG_NM) * (ld(b, (int64_t)row * AMG_NM + r) - sw[wv][r]);
  t[(int64_t)row * AMG_NM + j] = (T)acc;
}

// y = D^-1 A x (power iteration)
template <typename T>
__global__ void __launch_bounds__(256)
k_amgc_dapply(int n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col, const T *__restrict__ A,
              const T *__restrict__ Dinv, const T *__restrict__ x, T *y) {
  __shared__ double sp[AMG_WROWS][64], sw[AMG_WROWS][AMG_NM];
  AMGC_WAVE_PROLOGUE
  amgc_row_sums(ptr, col, A, x, row, act, j, sp[wv], sw[wv]);
  if (act && j < AMG_NM) y[(int64_t)row * AMG_NM + j] = (T)amgc_dapply(Dinv, row, j, sw[wv]);
}

// x += d (the pending step of a degree-1 smoothing from a nonzero start)
template <typename T>
__global__ void k_amg_axpy(int64_t nv, const T *__restrict__ d, T *x, const int *done) {
  if (amg_done(done)) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nv) x[i] = (T)(ld(x, i) + ld(d, i));
}

// ---- transfers -----------------------------------------------------------------------------
// restriction, second half: bc[I][a] = sum of t[i][a] over the members i of I (ascending)
template <typename T>
__global__ void k_amg_aggsum(int nc, const int32_t *__restrict__ mptr, const int32_t *__restrict__ mem,
                             const T *__restrict__ t, T *bc, const int *done) {
  if (amg_done(done)) return;
  const int64_t th = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (th >= (int64_t)nc * AMG_NM) return;
  const int I = (int)(th / AMG_NM), a = (int)(th % AMG_NM);
  const int k0 = mptr[I], k1 = mptr[I + 1];
  double acc = 0.0;
#pragma unroll 4
  for (int k = k0; k < k1; ++k) acc += ld(t, (int64_t)mem[k] * AMG_NM + a);
  bc[th] = (T)acc;
}

// prolongation x[i][r] += s[i][r] sum_a P[i][r][a] xc[agg(i)][a]
template <typename T, typename TP, int BS>
__global__ void k_amg_prolong(int n, const int32_t *__restrict__ agg, const TP *__restrict__ P,
                              const double *__restrict__ Wsc, const T *__restrict__ xc, T *x, const int *done) {
  if (amg_done(done)) return;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * BS) return;
  const int i = (int)(t / BS), r = (int)(t % BS);
  const T *e = xc + (int64_t)agg[i] * AMG_NM;
  const TP *p = P + t * AMG_NM;
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < AMG_NM; ++a) acc += ld(p, a) * ld(e, a);
  const double s = Wsc ? 1.0 / Wsc[4 * (int64_t)i + r] : 1.0;
  x[t] = (T)(ld(x, t) + s * acc);
}

// ---- coarse operators (per linear system, FP64) ---------------------------------------------
// A_1[cb][a][c] = sum over the finest blocks b of the list of cb, with b = (i, j):
//   sum_{r,q} (Q[i][r][a] / W[i][r]) A_b[r][q] (Q[j][q][c] / W[j][q]),
// A_b from the entry-major fine blocks, symmetrised ((A_b + A_{tpos b}^T) / 2) when sym; plus a
// unit diagonal on dropped coarse dofs.  One thread per coarse entry.
__global__ void k_amg_gal0(int64_t nbc, const int32_t *__restrict__ cbrow, const int32_t *__restrict__ ccol,
                           const uint8_t *__restrict__ dropped, const int32_t *__restrict__ gptr,
                           const int32_t *__restrict__ gsrc, int Wslot, int64_t nnzb, const int32_t *__restrict__ fcol,
                           const int32_t *__restrict__ tpos, const double *__restrict__ A, int sym,
                           const double *__restrict__ Wsc, const double *__restrict__ Q, double *Ac) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nbc * (AMG_NM * AMG_NM)) return;
  const int64_t cb = t / (AMG_NM * AMG_NM);
  const int e = (int)(t % (AMG_NM * AMG_NM)), a = e / AMG_NM, c = e % AMG_NM;
  double acc = 0.0;
  for (int k = gptr[cb]; k < gptr[cb + 1]; ++k) {
    const int b = gsrc[k];
    const int i = b / Wslot, j = fcol[b];
    const int bt = sym ? tpos[b] : b;
    double pj[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) pj[q] = Q[((int64_t)j * 3 + q) * AMG_NM + c] / Wsc[4 * (int64_t)j + q];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double row = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double v = sym ? 0.5 * (A[(int64_t)(3 * r + q) * nnzb + b] + A[(int64_t)(3 * q + r) * nnzb + bt])
                             : A[(int64_t)(3 * r + q) * nnzb + b];
        row += v * pj[q];
      }
      acc += Q[((int64_t)i * 3 + r) * AMG_NM + a] / Wsc[4 * (int64_t)i + r] * row;
    }
  }
  if (a == c && cbrow[cb] == ccol[cb] && dropped[(int64_t)cbrow[cb] * AMG_NM + a]) acc += 1.0;
  Ac[t] = acc;
}

// A_{l+1}[cb][a][c] = sum over the level-l blocks k of the list (row i, column j) of
// sum_r Q[i][r][a] sum_q A_l[k][r][q] Q[j][q][c]; unit diagonal on dropped coarse dofs
__global__ void k_amg_gal(int64_t nbc, const int32_t *__restrict__ cbrow, const int32_t *__restrict__ ccol,
                          const uint8_t *__restrict__ dropped, const int32_t *__restrict__ gptr,
                          const int32_t *__restrict__ gsrc, const int32_t *__restrict__ fbrow,
                          const int32_t *__restrict__ fcol, const double *__restrict__ Af,
                          const double *__restrict__ Q, double *Ac) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nbc * (AMG_NM * AMG_NM)) return;
  const int64_t cb = t / (AMG_NM * AMG_NM);
  const int e = (int)(t % (AMG_NM * AMG_NM)), a = e / AMG_NM, c = e % AMG_NM;
  double acc = 0.0;
  for (int k = gptr[cb]; k < gptr[cb + 1]; ++k) {
    const int fb = gsrc[k];
    const int i = fbrow[fb], j = fcol[fb];
    const double *Ab = Af + (int64_t)fb * (AMG_NM * AMG_NM);
    double pj[AMG_NM];
#pragma unroll
    for (int q = 0; q < AMG_NM; ++q) pj[q] = Q[((int64_t)j * AMG_NM + q) * AMG_NM + c];
    for (int r = 0; r < AMG_NM; ++r) {
      double row = 0.0;
#pragma unroll
      for (int q = 0; q < AMG_NM; ++q) row += Ab[r * AMG_NM + q] * pj[q];
      acc += Q[((int64_t)i * AMG_NM + r) * AMG_NM + a] * row;
    }
  }
  if (a == c && cbrow[cb] == ccol[cb] && dropped[(int64_t)cbrow[cb] * AMG_NM + a]) acc += 1.0;
  Ac[t] = acc;
}

// inverse of the 10x10 diagonal block of every row (Gauss-Jordan, partial pivoting, FP64); a
// singular block leaves its row's inverse zero and raises the level's flag
template <typename T>
__global__ void k_amg_dinv(int n, const int32_t *__restrict__ dpos, const double *__restrict__ Ac, T *Dinv,
                           int *bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m[AMG_NM][2 * AMG_NM];
  const double *blk = Ac + (int64_t)dpos[i] * (AMG_NM * AMG_NM);
  for (int r = 0; r < AMG_NM; ++r)
    for (int c = 0; c < AMG_NM; ++c) {
      m[r][c] = blk[r * AMG_NM + c];
      m[r][AMG_NM + c] = (r == c) ? 1.0 : 0.0;
    }
  bool ok = true;
  for (int c = 0; c < AMG_NM && ok; ++c) {
    int p = c;
    for (int r = c + 1; r < AMG_NM; ++r)
      if (fabs(m[r][c]) > fabs(m[p][c])) p = r;
    if (!(fabs(m[p][c]) > 0.0)) { ok = false; break; }
    if (p != c)
      for (int q = 0; q < 2 * AMG_NM; ++q) { const double tmp = m[c][q]; m[c][q] = m[p][q]; m[p][q] = tmp; }
    const double inv = 1.0 / m[c][c];
    for (int q = 0; q < 2 * AMG_NM; ++q) m[c][q] *= inv;
    for (int r = 0; r < AMG_NM; ++r) {
      if (r == c) continue;
      const double f = m[r][c];
      if (f != 0.0)
        for (int q = 0; q < 2 * AMG_NM; ++q) m[r][q] -= f * m[c][q];
    }
  }
  T *out = Dinv + (int64_t)i * (AMG_NM * AMG_NM);
  for (int r = 0; r < AMG_NM; ++r)
    for (int c = 0; c < AMG_NM; ++c) out[r * AMG_NM + c] = ok ? (T)m[r][AMG_NM + c] : (T)0;
  if (!ok) *bad = 1;
}

template <typename T>
__global__ void k_amg_cvt(int64_t count, const double *__restrict__ src, T *dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = (T)src[i];
}

template <typename T>
__global__ void k_amg_power_init(int64_t nv, uint64_t seed, T *x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nv) x[i] = (T)splitmix_unit(seed, (uint64_t)i);
}

__global__ void k_amg_lam_final(const double *lam_tmp, double *lam) { *lam = AMG_LMAX_SAFETY * *lam_tmp; }
