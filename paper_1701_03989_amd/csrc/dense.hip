// Tall-skinny kernels: the recovery Y*coef, the reductions that finish the
// partial sums of the other kernels, and small vector helpers.  (The Gram
// matrix is in gram.hip.)
#include "common.h"

namespace {

constexpr int WG = 256;
constexpr int MAXD = 2 * SSCG_S_LIMIT + 1;


// ---------------------------------------------------------------- finalizers
//
// Sum `nparts` dd partials of reduction blockIdx.x in a fixed order and
// round once.
__device__ __forceinline__ dd reduce_parts(const double* __restrict__ p, int nparts) {
  __shared__ double ls[WG / SSCG_WAVE], le[WG / SSCG_WAVE];
  dd a = dd_zero();
  // batches of independent loads (all in flight at once), merged in index order
  constexpr int U = 8;
  int q = threadIdx.x;
  for (; q + (U - 1) * WG < nparts; q += U * WG) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = reinterpret_cast<const double2*>(p)[q + u * WG];
#pragma unroll
    for (int u = 0; u < U; ++u) dd_merge(a, dd{v[u].x, v[u].y});
  }
  for (; q < nparts; q += WG) dd_merge(a, dd{p[2 * q], p[2 * q + 1]});
  a = dd_wave_reduce(a);
  int wv = threadIdx.x / SSCG_WAVE;
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) {
    ls[wv] = a.s;
    le[wv] = a.e;
  }
  __syncthreads();
  dd t{ls[0], le[0]};
  for (int q = 1; q < WG / SSCG_WAVE; ++q) dd_merge(t, dd{ls[q], le[q]});
  return t;
}

__global__ __launch_bounds__(WG) void k_finalize(const double* __restrict__ part, int nparts,
                                                 double* __restrict__ out) {
  int k = blockIdx.x;
  dd t = reduce_parts(part + (int64_t)k * nparts * 2, nparts);
  if (threadIdx.x == 0) out[k] = dd_round(t);
}

// out[0] = sqrt(RN(sum)): the finalize and the square root of a norm.
__global__ __launch_bounds__(WG) void k_finalize_sqrt(const double* __restrict__ part, int nparts,
                                                      double* __restrict__ out) {
  dd t = reduce_parts(part, nparts);
  if (threadIdx.x == 0) out[0] = sqrt(dd_round(t));
}

__global__ __launch_bounds__(WG) void k_max_finalize(const double* __restrict__ part, int nparts,
                                                     double* __restrict__ out) {
  __shared__ double lm[WG / SSCG_WAVE];
  double m = 0.0;
  for (int q = threadIdx.x; q < nparts; q += WG) m = fmax(m, part[q]);
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) m = fmax(m, __shfl_xor(m, k, SSCG_WAVE));
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) lm[threadIdx.x / SSCG_WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = lm[0];
    for (int q = 1; q < WG / SSCG_WAVE; ++q) t = fmax(t, lm[q]);
    out[0] = t;
  }
}

// max of width[0..n) into *out (one workgroup).
__global__ __launch_bounds__(WG) void k_max_width(const int32_t* __restrict__ width, int n,
                                                  int32_t* __restrict__ out) {
  __shared__ int lm[WG / SSCG_WAVE];
  int m = 0;
  for (int q = threadIdx.x; q < n; q += WG) m = max(m, (int)width[q]);
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) m = max(m, __shfl_xor(m, k, SSCG_WAVE));
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) lm[threadIdx.x / SSCG_WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = lm[0];
    for (int q = 1; q < WG / SSCG_WAVE; ++q) t = max(t, lm[q]);
    out[0] = t;
  }
}

// ---------------------------------------------------------------- recovery
//
// x_i <- RN(x_i + sum_a Y_ia x'_a), r_i <- RN(sum_a Y_ia r'_a),
// p_i <- RN(sum_a Y_ia p'_a) (eq. coords).  Columns whose three coefficients
// are all zero contribute nothing to the exact sums and are not read.
template <class Cols>
__device__ __forceinline__ void recover_row(const Cols& cols, int d,
                                            const double* __restrict__ coef, int i,
                                            const double* x_in, double* x_out, double* r,
                                            double* p);

// The 3d coefficients of a block into LDS (every thread of the workgroup
// must call it): the per-column zero tests then cost no memory waits.
__device__ __forceinline__ void stage_coef(const double* __restrict__ coef, int d, double* cf) {
  for (int e = threadIdx.x; e < 3 * d; e += blockDim.x) cf[e] = coef[e];
  __syncthreads();
}

__global__ __launch_bounds__(WG) void k_recover(ColPtr cols, int n, int d,
                                                const double* __restrict__ coef,
                                                const double* x_in, double* x_out, double* r,
                                                double* p, Gate gate) {
  if (gate_closed(gate)) return;
  int nb = (n + WG - 1) / WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  __shared__ double cf[3 * MAXD];
  stage_coef(coef, d, cf);
  int i = lb * WG + threadIdx.x;
  if (i >= n) return;
  recover_row(cols, d, cf, i, x_in, x_out, r, p);
}

template <class Cols>
__device__ __forceinline__ void recover_row(const Cols& cols, int d,
                                            const double* __restrict__ coef, int i,
                                            const double* x_in, double* x_out, double* r,
                                            double* p) {
  dd ax = dd_zero(), ar = dd_zero(), ap = dd_zero();
  dd_add(ax, x_in[i]);
  // groups of RC columns: all loads of a group are in flight before the sums
  constexpr int RC = 8;
  for (int a0 = 0; a0 < d; a0 += RC) {
    double y[RC];
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      // unconditional loads (a branch per load would serialise them): a
      // column past d or with three zero coefficients reads column 0's row
      // again instead (a cache hit, and its value is not used)
      const int a = a0 + u;
      const bool use =
          a < d && (coef[a] != 0.0 || coef[d + a] != 0.0 || coef[2 * d + a] != 0.0);
      y[u] = cols.at(use ? a : 0)[i];
    }
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      const int a = a0 + u;
      if (a < d) {
        const double cx = coef[a], cr = coef[d + a], cp = coef[2 * d + a];
        if (cx == 0.0 && cr == 0.0 && cp == 0.0) continue;
        dd_add_prod(ax, y[u], cx);
        dd_add_prod(ar, y[u], cr);
        dd_add_prod(ap, y[u], cp);
      }
    }
  }
  x_out[i] = dd_round(ax);
  r[i] = dd_round(ar);
  p[i] = dd_round(ap);
}

// Finish the residual fused into a block's first matrix-powers pass.
__global__ __launch_bounds__(WG) void k_res_finalize(const double* __restrict__ part, int nparts,
                                                     const double* __restrict__ b2, double tol,
                                                     sscg_block_info* info, int* stop) {
  if (*stop) return;
  dd t = reduce_parts(part, nparts);
  if (threadIdx.x == 0) {
    double rel = sqrt(dd_round(t)) / sqrt(b2[0]);
    info->relres_in = rel;
    if (rel <= tol) *stop = 1;
    else if (!isfinite(rel)) *stop = 3;
  }
}

// ---------------------------------------------------------------- helpers

__global__ __launch_bounds__(WG) void k_scale_vec(const double* __restrict__ in,
                                                  const double* __restrict__ s, int mul, int n,
                                                  double* __restrict__ out) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n) out[i] = mul ? in[i] * s[i] : in[i] / s[i];
}

__global__ __launch_bounds__(WG) void k_copy(const double* __restrict__ in, int n,
                                             double* __restrict__ out) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ __launch_bounds__(WG) void k_fill(double* __restrict__ out, int n, double v) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n) out[i] = v;
}

// out = sqrt(r2) / sqrt(b2): the true relative residual.
__global__ void k_relres(const double* __restrict__ r2, const double* __restrict__ b2,
                         double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = sqrt(r2[0]) / sqrt(b2[0]);
}

// SplitMix64 (Steele, Lea & Flood 2014): z_i from state seed + (i+1)*golden.
__global__ __launch_bounds__(WG) void k_splitmix(double* __restrict__ out, int n, uint64_t seed) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  out[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
}

// w_i <- w_i - alpha v_i (two roundings); partials of w.w.
__global__ __launch_bounds__(WG) void k_axpy_dot(double* __restrict__ w,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ alpha, int n,
                                                 double* __restrict__ part) {
  __shared__ double ls[WG / SSCG_WAVE], le[WG / SSCG_WAVE];
  int nb = (n + WG - 1) / WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  int i = lb * WG + threadIdx.x;
  dd a = dd_zero();
  if (i < n) {
    double t = (*alpha) * v[i];
    double wi = w[i] - t;
    w[i] = wi;
    dd_add_prod(a, wi, wi);
  }
  a = dd_wave_reduce(a);
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) {
    ls[threadIdx.x / SSCG_WAVE] = a.s;
    le[threadIdx.x / SSCG_WAVE] = a.e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    dd t{ls[0], le[0]};
    for (int q = 1; q < WG / SSCG_WAVE; ++q) dd_merge(t, dd{ls[q], le[q]});
    part[2 * lb] = t.s;
    part[2 * lb + 1] = t.e;
  }
}

__global__ __launch_bounds__(WG) void k_dot_parts(const double* __restrict__ x,
                                                  const double* __restrict__ y, int n,
                                                  double* __restrict__ part) {
  __shared__ double ls[WG / SSCG_WAVE], le[WG / SSCG_WAVE];
  int nb = (n + WG - 1) / WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  int i = lb * WG + threadIdx.x;
  dd a = dd_zero();
  if (i < n) dd_add_prod(a, x[i], y[i]);
  a = dd_wave_reduce(a);
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) {
    ls[threadIdx.x / SSCG_WAVE] = a.s;
    le[threadIdx.x / SSCG_WAVE] = a.e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    dd t{ls[0], le[0]};
    for (int q = 1; q < WG / SSCG_WAVE; ++q) dd_merge(t, dd{ls[q], le[q]});
    part[2 * lb] = t.s;
    part[2 * lb + 1] = t.e;
  }
}

__global__ __launch_bounds__(WG) void k_div_vec(const double* __restrict__ w,
                                                const double* __restrict__ beta, int n,
                                                double* __restrict__ out) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n) out[i] = w[i] / (*beta);
}


// ---------------------------------------------------------------- batches

// Gram columns of a system in this block: P_0..P_s, then R_0..R_{s-1}; the
// address is computed (an array of pointers would live in scratch memory).
// x <- x + Y x', r = Y r' (into R_0), p = Y p' (into P_0), per system; over
// the blocks listed in ablk (a workgroup takes every gridDim.x-th entry).
__global__ __launch_bounds__(WG) void k_recover_batch(BatchCfg c) {
  __shared__ double cf[3 * MAXD];
  const int nl = c.active[1];
  for (int li = blockIdx.x; li < nl; li += gridDim.x) {  // uniform over the workgroup
    const int lb = c.ablk[li];
    const int q = c.blk_sys[lb];
    if (q < 0 || c.sys[q].done) continue;
    const sscg_block_params prm = c.prm[q];
    const int d = prm.first ? prm.s + 1 : 2 * prm.s + 1;
    const int i = lb * BATCH_ROWS + threadIdx.x;
    stage_coef(c.coef + (int64_t)q * BATCH_CSZ, d, cf);
    if (c.sys[q].p32)  // an FP32 block's columns, widened
      recover_row(batch_cols32(c, prm.s), d, cf, i, c.x, c.x, batch_col(c, c.S + 1),
                  batch_col(c, 0));
    else
      recover_row(batch_cols(c, prm.s, prm.first), d, cf, i, c.x, c.x, batch_col(c, c.S + 1),
                  batch_col(c, 0));
    // the (p, r) pairs the next block's first pass gathers (each thread its own row)
    if (c.sys[q].il) c.T[0][i] = make_double2(batch_col(c, 0)[i], batch_col(c, c.S + 1)[i]);
    // and the FP32 P_0 = RN32(p), R_0 = RN32(r) the next block reads if the
    // plan makes it an FP32 block (its other columns the passes write)
    if (c.vprec && c.Y32) {
      c.Y32[i] = (float)batch_col(c, 0)[i];
      c.Y32[(int64_t)(c.S + 1) * c.ld + i] = (float)batch_col(c, c.S + 1)[i];
    }
    __syncthreads();  // cf is read before the next block's system rewrites it
  }
}

// Set-up per system from the residual and ||b||^2 partials of its blocks.
__global__ __launch_bounds__(WG) void k_batch_init(BatchCfg c, int q0) {
  const int q = q0 + blockIdx.x;
  BatchSys& sy = c.sys[q];
  dd r = reduce_parts(c.rpart + (int64_t)sy.blk0 * 2, sy.blk1 - sy.blk0);
  __syncthreads();
  dd bb = reduce_parts(c.bpart + (int64_t)sy.blk0 * 2, sy.blk1 - sy.blk0);
  if (threadIdx.x == 0) {
    const double r2 = dd_round(r), b2 = dd_round(bb);
    sy.b2 = b2;
    sy.eps_star = sy.tol * sqrt(b2);
    sy.first = 1;
    sy.m = 0;
    sy.s_prev = 0;
    sy.blocks = 0;
    sy.s_bar = 0;
    sy.bp = make_basis(c.basis, sy.lmin, sy.lmax);
    if (b2 == 0.0) {  // x = 0 solves A x = 0
      sy.relres = 0.0;
      sy.done = 1;
      sy.status = SSCG_OK;
    } else {
      const double rel = sqrt(r2) / sqrt(b2);
      sy.relres = rel;
      sy.done = rel <= sy.tol ? 1 : 0;
      sy.status = SSCG_OK;
    }
  }
}

// The true residual of each system's starting iterate (fused into the first
// matrix-powers pass) decides convergence; after block 0 only.
__global__ __launch_bounds__(WG) void k_batch_res_finalize(BatchCfg c) {
  const int q = blockIdx.x;
  BatchSys& sy = c.sys[q];
  if (sy.done || sy.first) return;
  dd t = reduce_parts(c.rpart + (int64_t)sy.blk0 * 2, sy.blk1 - sy.blk0);
  if (threadIdx.x == 0) {
    const double rel = sqrt(dd_round(t)) / sqrt(sy.b2);
    sy.relres = rel;
    if (sy.blocks >= 1 && sy.blocks - 1 < c.cap)
      c.hist[(int64_t)q * c.cap + sy.blocks - 1].relres_true = rel;
    if (rel <= sy.tol) {
      sy.done = 1;
      sy.status = SSCG_OK;
    } else if (!isfinite(rel)) {
      sy.done = 1;
      sy.status = SSCG_BREAKDOWN;
    } else if (sy.m >= c.max_iters) {
      sy.done = 1;
      sy.status = SSCG_NOT_CONVERGED;
    }
  }
}

// The systems not done: their number (active[0]), and the offsets (loff) and
// lengths (active[1], active[2]) of their entries in the block and chunk
// lists, in system order.  One workgroup; thread t takes a contiguous run of
// systems.
__global__ __launch_bounds__(WG) void k_batch_count(BatchCfg c) {
  __shared__ int ls[3][WG];
  const int t = threadIdx.x;
  const int per = (c.nsys + WG - 1) / WG;
  const int q0 = min(t * per, c.nsys), q1 = min(q0 + per, c.nsys);
  int a = 0, nb = 0, nc = 0;
  for (int q = q0; q < q1; ++q) {
    const BatchSys& y = c.sys[q];
    if (y.done) continue;
    ++a;
    nb += y.blk1 - y.blk0;
    nc += y.ch1 - y.ch0;
  }
  ls[0][t] = a;
  ls[1][t] = nb;
  ls[2][t] = nc;
  __syncthreads();
  for (int h = 1; h < WG; h <<= 1) {  // inclusive scans
    int v0 = 0, v1 = 0, v2 = 0;
    if (t >= h) {
      v0 = ls[0][t - h];
      v1 = ls[1][t - h];
      v2 = ls[2][t - h];
    }
    __syncthreads();
    ls[0][t] += v0;
    ls[1][t] += v1;
    ls[2][t] += v2;
    __syncthreads();
  }
  int ob = ls[1][t] - nb, oc = ls[2][t] - nc;
  for (int q = q0; q < q1; ++q) {
    const BatchSys& y = c.sys[q];
    if (y.done) continue;
    c.loff[2 * q] = ob;
    c.loff[2 * q + 1] = oc;
    ob += y.blk1 - y.blk0;
    oc += y.ch1 - y.ch0;
  }
  if (t == WG - 1) {
    c.active[0] = ls[0][t];
    c.active[1] = ls[1][t];
    c.active[2] = ls[2][t];
  }
}

// The lists themselves: the blocks and chunks of each system not done, at its
// offsets (after k_batch_count).
__global__ __launch_bounds__(WG) void k_batch_lists(BatchCfg c) {
  for (int q = blockIdx.x; q < c.nsys; q += gridDim.x) {
    const BatchSys& y = c.sys[q];
    if (y.done) continue;
    const int ob = c.loff[2 * q], oc = c.loff[2 * q + 1];
    for (int k = threadIdx.x; k < y.blk1 - y.blk0; k += WG) c.ablk[ob + k] = y.blk0 + k;
    for (int k = threadIdx.x; k < y.ch1 - y.ch0; k += WG) c.achk[oc + k] = y.ch0 + k;
  }
}


// ---------------------------------------------------------------- FP32 basis
// dx_i += sum_a Y_ia x'_a; r_i = RN32(sum_a Y_ia r'_a); p_i likewise (FP64 sums).
__global__ __launch_bounds__(WG) void k_recover32(Cols32 cols, int n, int d,
                                                  const double* __restrict__ coef, double* dx,
                                                  float* r, float* p) {
  int nb = (n + WG - 1) / WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  __shared__ double cf[3 * MAXD];
  stage_coef(coef, d, cf);
  int i = lb * WG + threadIdx.x;
  if (i >= n) return;
  double ax = 0.0, ar = 0.0, ap = 0.0;
  // groups of RC columns, every load of a group in flight before the sums (a
  // column with three zero coefficients reads column 0 again, unused); the
  // sums keep the column order
  constexpr int RC = 8;
  for (int a0 = 0; a0 < d; a0 += RC) {
    float y[RC];
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      const int a = a0 + u;
      const bool use = a < d && (cf[a] != 0.0 || cf[d + a] != 0.0 || cf[2 * d + a] != 0.0);
      y[u] = cols.at(use ? a : 0)[i];
    }
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      const int a = a0 + u;
      if (a >= d) continue;
      const double cx = cf[a], cr = cf[d + a], cp = cf[2 * d + a];
      if (cx == 0.0 && cr == 0.0 && cp == 0.0) continue;
      const double yy = (double)y[u];
      ax = ax + yy * cx;
      ar = ar + yy * cr;
      ap = ap + yy * cp;
    }
  }
  dx[i] = dx[i] + ax;
  r[i] = (float)ar;
  p[i] = (float)ap;
}

__global__ __launch_bounds__(WG) void k_add(double* __restrict__ x, const double* __restrict__ d,
                                            int n) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i < n) x[i] = x[i] + d[i];
}
}  // namespace

// ---------------------------------------------------------------- launches

hipError_t launch_res_finalize(const double* part, int nparts, const double* b2, double tol,
                               sscg_block_info* info, int* stop, hipStream_t st) {
  hipLaunchKernelGGL(k_res_finalize, dim3(1), dim3(WG), 0, st, part, nparts, b2, tol, info, stop);
  return hipGetLastError();
}

hipError_t launch_finalize_sqrt(const double* part, int nparts, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_sqrt, dim3(1), dim3(WG), 0, st, part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* part, int nparts, int count, double* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(count), dim3(WG), 0, st, part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_max_finalize(const double* part, int nparts, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_max_finalize, dim3(1), dim3(WG), 0, st, part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_max_width(const int32_t* width, int n, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_max_width, dim3(1), dim3(WG), 0, st, width, n, out);
  return hipGetLastError();
}

hipError_t launch_recover(const ColPtr& cols, int n, int d, const double* coef, const double* x_in,
                          double* x_out, double* r, double* p, Gate g, hipStream_t st) {
  int nb = (n + WG - 1) / WG;
  hipLaunchKernelGGL(k_recover, dim3(xcd_grid(nb)), dim3(WG), 0, st, cols, n, d, coef, x_in, x_out,
                     r, p, g);
  return hipGetLastError();
}

hipError_t launch_scale_vec(const double* in, const double* s, int mul, int n, double* out,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_scale_vec, dim3((n + WG - 1) / WG), dim3(WG), 0, st, in, s, mul, n, out);
  return hipGetLastError();
}

hipError_t launch_copy(const double* in, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3((n + WG - 1) / WG), dim3(WG), 0, st, in, n, out);
  return hipGetLastError();
}

hipError_t launch_fill(double* out, int n, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((n + WG - 1) / WG), dim3(WG), 0, st, out, n, v);
  return hipGetLastError();
}

hipError_t launch_relres(const double* r2, const double* b2, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_relres, dim3(1), dim3(SSCG_WAVE), 0, st, r2, b2, out);
  return hipGetLastError();
}

hipError_t launch_splitmix_vec(double* out, int n, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_splitmix, dim3((n + WG - 1) / WG), dim3(WG), 0, st, out, n, seed);
  return hipGetLastError();
}

hipError_t launch_axpy_dot(double* w, const double* v, const double* alpha, double* part,
                           int* nparts, int n, hipStream_t st) {
  int nb = (n + WG - 1) / WG;
  *nparts = nb;
  hipLaunchKernelGGL(k_axpy_dot, dim3(xcd_grid(nb)), dim3(WG), 0, st, w, v, alpha, n, part);
  return hipGetLastError();
}

hipError_t launch_dot_parts(const double* x, const double* y, int n, double* part, int* nparts,
                            hipStream_t st) {
  int nb = (n + WG - 1) / WG;
  *nparts = nb;
  hipLaunchKernelGGL(k_dot_parts, dim3(xcd_grid(nb)), dim3(WG), 0, st, x, y, n, part);
  return hipGetLastError();
}

hipError_t launch_div_vec(const double* w, const double* beta, int n, double* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_div_vec, dim3((n + WG - 1) / WG), dim3(WG), 0, st, w, beta, n, out);
  return hipGetLastError();
}

hipError_t launch_recover_batch(const BatchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_recover_batch, dim3(batch_grid(c.gblk)), dim3(WG), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_batch_init(const BatchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_init, dim3(c.nsys), dim3(WG), 0, st, c, 0);
  return hipGetLastError();
}

hipError_t launch_batch_init_range(const BatchCfg& c, int q0, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_init, dim3(count), dim3(WG), 0, st, c, q0);
  return hipGetLastError();
}

hipError_t launch_batch_res_finalize(const BatchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_res_finalize, dim3(c.nsys), dim3(WG), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_batch_count(const BatchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_count, dim3(1), dim3(WG), 0, st, c);
  hipLaunchKernelGGL(k_batch_lists, dim3(c.nsys < 1024 ? c.nsys : 1024), dim3(WG), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_recover32(const Cols32& cols, int n, int d, const double* coef, double* dx,
                            float* r, float* p, hipStream_t st) {
  int nb = (n + WG - 1) / WG;
  hipLaunchKernelGGL(k_recover32, dim3(xcd_grid(nb)), dim3(WG), 0, st, cols, n, d, coef, dx, r, p);
  return hipGetLastError();
}

hipError_t launch_add(double* x, const double* d, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3((n + WG - 1) / WG), dim3(WG), 0, st, x, d, n);
  return hipGetLastError();
}
