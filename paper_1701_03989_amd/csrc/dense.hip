// Tall-skinny kernels: the Gram matrix G = Y^T Y, the recovery Y*coef, the
// reductions that finish them, and small vector helpers.
#include "common.h"

namespace {

constexpr int WG = 256;
constexpr int GT = 32;            // rows of Y per LDS tile
constexpr int MAXD = 2 * SSCG_S_LIMIT + 1;
constexpr int MAXPAIRS = MAXD * (MAXD + 1) / 2;
constexpr int PAIRS_PER_THREAD = (MAXPAIRS + WG - 1) / WG;


// ---------------------------------------------------------------- Gram
//
// Each workgroup owns a contiguous range of row tiles (XCD-aware) and keeps
// one dd accumulator per upper-triangle entry (a <= b) it is assigned; tiles
// of GT rows x d columns are staged in LDS (row-major, so the lanes of a wave
// reading different columns of one row hit different banks).  Output: one dd
// partial per (entry, workgroup), entry-major.
//
// Upper-triangle dd partials of the Gram matrix of columns cols[0..d) over
// rows [rb, re): entry q (a <= b, row-major over the triangle) goes to
// part[(q * nparts + slot) * 2].
template <int PPT, class Cols>
__device__ __forceinline__ void gram_rows(const Cols& cols, int d, int rb, int re,
                                          double* __restrict__ part, int nparts, int slot) {
  // two LDS tiles: tile t+1 is loaded into registers while tile t is used
  __shared__ double tile[2][GT][MAXD + 1];
  constexpr int LPT = (GT * MAXD + WG - 1) / WG;  // tile elements per thread
  const int npairs = d * (d + 1) / 2;
  const int nel = GT * d;
  int pa[PPT], pb[PPT];
  dd acc[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    int q = threadIdx.x + u * WG;
    int a = 0, rem = q;
    while (a < d && rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    pa[u] = a < d ? a : 0;
    pb[u] = a < d ? a + rem : 0;
    acc[u] = dd_zero();
  }
  // element e of a tile: column e / GT, row e % GT (a wave reads whole column runs)
  double nx[LPT];
  auto fetch = [&](int r0) {
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const int e = threadIdx.x + k * WG;
      const int a = e / GT, row = r0 + (e - a * GT);
      nx[k] = (e < nel && row < re) ? cols.at(a)[row] : 0.0;
    }
  };
  if (rb < re) fetch(rb);
  int buf = 0;
  for (int r0 = rb; r0 < re; r0 += GT) {
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const int e = threadIdx.x + k * WG;
      const int a = e / GT;
      if (e < nel) tile[buf][e - a * GT][a] = nx[k];
    }
    // one barrier per tile: a thread writes tile[buf] again two tiles later,
    // after every thread has passed the next barrier, i.e. finished this tile
    __syncthreads();
    if (r0 + GT < re) fetch(r0 + GT);
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      if (threadIdx.x + u * WG < npairs) {
        const int a = pa[u], b = pb[u];
#pragma unroll 4
        for (int r = 0; r < GT; ++r) dd_add_prod(acc[u], tile[buf][r][a], tile[buf][r][b]);
      }
    }
    buf ^= 1;
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    int q = threadIdx.x + u * WG;
    if (q < npairs) {
      part[((int64_t)q * nparts + slot) * 2] = acc[u].s;
      part[((int64_t)q * nparts + slot) * 2 + 1] = acc[u].e;
    }
  }
}

// PPT: upper-triangle entries per thread (1 covers d <= 22)
template <int PPT>
__global__ __launch_bounds__(WG) void k_gram(ColPtr cols, int n, int d, double* __restrict__ part,
                                             int nparts, Gate gate) {
  if (gate_closed(gate)) return;
  int lb = xcd_block(nparts);
  if (lb >= nparts) return;
  int ntiles = (n + GT - 1) / GT;
  int per = (ntiles + nparts - 1) / nparts;
  int t0 = lb * per, t1 = min(t0 + per, ntiles);
  gram_rows<PPT>(cols, d, t0 * GT, min(t1 * GT, n), part, nparts, lb);
}

// Sum `nparts` dd partials of reduction blockIdx.x in a fixed order and
// round once.  Gram variant writes both triangles of G.
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

__global__ __launch_bounds__(WG) void k_gram_finalize(const double* __restrict__ part, int nparts,
                                                      int d, double* __restrict__ G,
                                                      const int* __restrict__ stop) {
  if (stop && *stop) return;
  int q = blockIdx.x;
  dd t = reduce_parts(part + (int64_t)q * nparts * 2, nparts);
  if (threadIdx.x == 0) {
    int a = 0, rem = q;
    while (rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    int b = a + rem;
    double g = dd_round(t);
    G[a * d + b] = g;
    G[b * d + a] = g;
  }
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
struct BatchCols {
  double* Y;
  int64_t ld;
  int s, S;
  __device__ __forceinline__ const double* at(int a) const {
    return Y + (int64_t)(a <= s ? a : S + 1 + (a - s - 1)) * ld;
  }
};

__device__ __forceinline__ BatchCols batch_cols(const BatchCfg& c, int s, int first) {
  (void)first;  // block 0 uses P_0..P_s only: d = s + 1 never reaches the R columns
  return BatchCols{c.Y, c.ld, s, c.S};
}

template <int PPT>
__global__ __launch_bounds__(WG) void k_gram_batch(BatchCfg c) {
  int lb = blockIdx.x;  // natural order, no XCD remap (see xcd_block)
  if (lb >= c.nchunks) return;
  const BatchChunk ch = c.chunks[lb];
  const int q = c.blk_sys[ch.r0 / BATCH_ROWS];  // the system that owns the chunk's rows now
  if (q < 0 || c.sys[q].done) return;
  const sscg_block_params prm = c.prm[q];
  const int d = prm.first ? prm.s + 1 : 2 * prm.s + 1;
  gram_rows<PPT>(batch_cols(c, prm.s, prm.first), d, ch.r0, ch.r1, c.gpart, c.nchunks, lb);
}

// grid (pairs, systems): entry blockIdx.x of system blockIdx.y.
__global__ __launch_bounds__(WG) void k_gram_finalize_batch(BatchCfg c) {
  const int q = blockIdx.y, e = blockIdx.x;
  const BatchSys& sy = c.sys[q];
  if (sy.done) return;
  const sscg_block_params prm = c.prm[q];
  const int d = prm.first ? prm.s + 1 : 2 * prm.s + 1;
  if (e >= d * (d + 1) / 2) return;
  dd t = reduce_parts(c.gpart + ((int64_t)e * c.nchunks + sy.ch0) * 2, sy.ch1 - sy.ch0);
  if (threadIdx.x == 0) {
    int a = 0, rem = e;
    while (rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    int b = a + rem;
    double g = dd_round(t);
    double* G = c.G + (int64_t)q * BATCH_GSZ;
    G[a * d + b] = g;
    G[b * d + a] = g;
  }
}

// x <- x + Y x', r = Y r' (into R_0), p = Y p' (into P_0), per system.
__global__ __launch_bounds__(WG) void k_recover_batch(BatchCfg c) {
  int lb = blockIdx.x;  // natural order, no XCD remap (see xcd_block)
  if (lb >= c.nblk) return;
  const int q = c.blk_sys[lb];
  if (q < 0 || c.sys[q].done) return;
  const sscg_block_params prm = c.prm[q];
  const int d = prm.first ? prm.s + 1 : 2 * prm.s + 1;
  const int i = lb * BATCH_ROWS + threadIdx.x;
  __shared__ double cf[3 * MAXD];
  stage_coef(c.coef + (int64_t)q * BATCH_CSZ, d, cf);
  recover_row(batch_cols(c, prm.s, prm.first), d, cf, i, c.x, c.x, batch_col(c, c.S + 1),
              batch_col(c, 0));
  // the (p, r) pairs the next block's first pass gathers (each thread its own row)
  if (c.sys[q].il) c.T[0][i] = make_double2(batch_col(c, 0)[i], batch_col(c, c.S + 1)[i]);
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

__global__ __launch_bounds__(WG) void k_batch_count(BatchCfg c) {
  __shared__ int ls[WG];
  int a = 0;
  for (int q = threadIdx.x; q < c.nsys; q += WG) a += c.sys[q].done ? 0 : 1;
  ls[threadIdx.x] = a;
  __syncthreads();
  for (int h = WG / 2; h >= 1; h >>= 1) {
    if (threadIdx.x < h) ls[threadIdx.x] += ls[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *c.active = ls[0];
}


// ---------------------------------------------------------------- FP32 basis
// Gram of FP32 columns: the products are exact in FP64 and summed in FP64 per
// thread (tiles of GT rows in LDS as before); partials as dd pairs (lo = 0).
__global__ __launch_bounds__(WG) void k_gram32(Cols32 cols, int n, int d,
                                               double* __restrict__ part, int nparts) {
  __shared__ double tile[GT][MAXD + 1];
  int lb = xcd_block(nparts);
  if (lb >= nparts) return;
  const int npairs = d * (d + 1) / 2;
  int pa[PAIRS_PER_THREAD], pb[PAIRS_PER_THREAD];
  double acc[PAIRS_PER_THREAD];
#pragma unroll
  for (int u = 0; u < PAIRS_PER_THREAD; ++u) {
    int q = threadIdx.x + u * WG;
    int a = 0, rem = q;
    while (a < d && rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    pa[u] = a < d ? a : 0;
    pb[u] = a < d ? a + rem : 0;
    acc[u] = 0.0;
  }
  int ntiles = (n + GT - 1) / GT;
  int per = (ntiles + nparts - 1) / nparts;
  int t0 = lb * per, t1 = min(t0 + per, ntiles);
  for (int t = t0; t < t1; ++t) {
    int r0 = t * GT;
    for (int e = threadIdx.x; e < GT * d; e += WG) {
      int a = e / GT, r = e - a * GT;
      int row = r0 + r;
      tile[r][a] = row < n ? (double)cols.at(a)[row] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PAIRS_PER_THREAD; ++u) {
      if (threadIdx.x + u * WG < npairs) {
        int a = pa[u], b = pb[u];
#pragma unroll 8
        for (int r = 0; r < GT; ++r) acc[u] = acc[u] + tile[r][a] * tile[r][b];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < PAIRS_PER_THREAD; ++u) {
    int q = threadIdx.x + u * WG;
    if (q < npairs) {
      part[((int64_t)q * nparts + lb) * 2] = acc[u];
      part[((int64_t)q * nparts + lb) * 2 + 1] = 0.0;
    }
  }
}

// dx_i += sum_a Y_ia x'_a; r_i = RN32(sum_a Y_ia r'_a); p_i likewise (FP64 sums).
// Gram of FP32 columns for d <= D, one row per lane: wavefront w of the W
// accumulates the entries [w NP / W, (w + 1) NP / W) of the row-major upper
// triangle over the workgroup's rows from registers (no LDS, no barrier).
// Products are exact in FP64 and summed with fma per lane (the same roundings
// as sum + product), the 64 lane sums added in a fixed tree; partials as dd
// pairs (lo = 0).
template <int D>
constexpr int g32_waves() {
  return D <= 11 ? 4 : 8;  // at most 29 entries (58 VGPRs of sums) per wavefront
}

template <int D, int w>
__device__ __forceinline__ void gram32_lr_wave(const Cols32& cols, int d, int r0, int r1,
                                               double* __restrict__ part, int nparts, int slot) {
  constexpr int NP = D * (D + 1) / 2;
  constexpr int W = g32_waves<D>();
  constexpr int Q0 = w * NP / W, Q1 = (w + 1) * NP / W;
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  const float* cp[D];
#pragma unroll
  for (int a = 0; a < D; ++a) cp[a] = a < d ? cols.at(a) : cols.Y;
  double acc[Q1 - Q0];
#pragma unroll
  for (int q = 0; q < Q1 - Q0; ++q) acc[q] = 0.0;
  float nx[D];
  auto fetch = [&](int r) {
#pragma unroll
    for (int a = 0; a < D; ++a) nx[a] = (a < d && r < r1) ? cp[a][r] : 0.0f;
  };
  fetch(r0 + lane);
  for (int base = r0; base < r1; base += SSCG_WAVE) {
    double v[D];
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = (double)nx[a];
    if (base + SSCG_WAVE < r1) fetch(base + SSCG_WAVE + lane);
    // (a, b) and the entry index q are constants after unrolling, so v stays in registers
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
      for (int b = a; b < D; ++b) {
        const int q = a * D - a * (a - 1) / 2 + (b - a);
        if (q >= Q0 && q < Q1) acc[q - Q0] = __builtin_fma(v[a], v[b], acc[q - Q0]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int b = a; b < D; ++b) {
      const int q = a * D - a * (a - 1) / 2 + (b - a);
      if (q < Q0 || q >= Q1) continue;
      double t = acc[q - Q0];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) t = t + shfl_xor_d(t, m);
      if (lane == 0 && b < d) {
        const int qd = a * d - a * (a - 1) / 2 + (b - a);  // the entry's index for dimension d
        part[((int64_t)qd * nparts + slot) * 2] = t;
        part[((int64_t)qd * nparts + slot) * 2 + 1] = 0.0;
      }
    }
  }
}

template <int D>
__global__ __launch_bounds__(g32_waves<D>() * SSCG_WAVE) void k_gram32_lr(Cols32 cols, int n, int d,
                                                                double* __restrict__ part,
                                                                int nparts) {
  const int lb = xcd_block(nparts);
  if (lb >= nparts) return;
  const int nb = (n + SSCG_WAVE - 1) / SSCG_WAVE, per = (nb + nparts - 1) / nparts;
  const int r0 = min(lb * per, nb) * SSCG_WAVE, r1 = min((lb + 1) * per * SSCG_WAVE, n);
  switch (threadIdx.x / SSCG_WAVE) {
    case 0: gram32_lr_wave<D, 0>(cols, d, r0, r1, part, nparts, lb); break;
    case 1: gram32_lr_wave<D, 1>(cols, d, r0, r1, part, nparts, lb); break;
    case 2: gram32_lr_wave<D, 2>(cols, d, r0, r1, part, nparts, lb); break;
    case 3: gram32_lr_wave<D, 3>(cols, d, r0, r1, part, nparts, lb); break;
    case 4: if constexpr (g32_waves<D>() > 4) gram32_lr_wave<D, 4>(cols, d, r0, r1, part, nparts, lb); break;
    case 5: if constexpr (g32_waves<D>() > 5) gram32_lr_wave<D, 5>(cols, d, r0, r1, part, nparts, lb); break;
    case 6: if constexpr (g32_waves<D>() > 6) gram32_lr_wave<D, 6>(cols, d, r0, r1, part, nparts, lb); break;
    default: if constexpr (g32_waves<D>() > 7) gram32_lr_wave<D, 7>(cols, d, r0, r1, part, nparts, lb); break;
  }
}

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

int gram_nparts(int n) {
  int ntiles = (n + GT - 1) / GT;
  // about 8 tiles per workgroup, at most 2048 workgroups
  int np = (ntiles + 7) / 8;
  if (np > 2048) np = 2048;
  return np < 1 ? 1 : np;
}

hipError_t launch_gram(const ColPtr& cols, int n, int d, double* part, int nparts, Gate g,
                       hipStream_t st) {
  if (d * (d + 1) / 2 <= WG)
    hipLaunchKernelGGL(k_gram<1>, dim3(xcd_grid(nparts)), dim3(WG), 0, st, cols, n, d, part,
                       nparts, g);
  else
    hipLaunchKernelGGL(k_gram<PAIRS_PER_THREAD>, dim3(xcd_grid(nparts)), dim3(WG), 0, st, cols, n,
                       d, part, nparts, g);
  return hipGetLastError();
}

hipError_t launch_gram_finalize(const double* part, int nparts, int d, double* G,
                                const int* stop, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_finalize, dim3(d * (d + 1) / 2), dim3(WG), 0, st, part, nparts, d, G,
                     stop);
  return hipGetLastError();
}

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

hipError_t launch_gram_batch(const BatchCfg& c, hipStream_t st) {
  const int dmax = 2 * c.S + 1;  // the largest basis of any system
  if (dmax * (dmax + 1) / 2 <= WG)
    hipLaunchKernelGGL(k_gram_batch<1>, dim3(xcd_grid(c.nchunks)), dim3(WG), 0, st, c);
  else
    hipLaunchKernelGGL(k_gram_batch<PAIRS_PER_THREAD>, dim3(xcd_grid(c.nchunks)), dim3(WG), 0, st,
                       c);
  return hipGetLastError();
}

hipError_t launch_gram_finalize_batch(const BatchCfg& c, hipStream_t st) {
  const int dm = 2 * c.S + 1;
  hipLaunchKernelGGL(k_gram_finalize_batch, dim3(dm * (dm + 1) / 2, c.nsys), dim3(WG), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_recover_batch(const BatchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_recover_batch, dim3(xcd_grid(c.nblk)), dim3(WG), 0, st, c);
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
  return hipGetLastError();
}

int gram32_nparts(int n) {
  // at least 32 row blocks of 64 per workgroup (the lane sums stay cheap), at most 512
  int nb = (n + SSCG_WAVE - 1) / SSCG_WAVE;
  int np = (nb + 31) / 32;
  if (np > 512) np = 512;
  return np < 1 ? 1 : np;
}

hipError_t launch_gram32(const Cols32& cols, int n, int d, double* part, int nparts,
                         hipStream_t st) {
  if (d <= 11)
    hipLaunchKernelGGL(k_gram32_lr<11>, dim3(xcd_grid(nparts)), dim3(g32_waves<11>() * SSCG_WAVE),
                       0, st, cols, n, d, part, nparts);
  else if (d <= 21)
    hipLaunchKernelGGL(k_gram32_lr<21>, dim3(xcd_grid(nparts)), dim3(g32_waves<21>() * SSCG_WAVE),
                       0, st, cols, n, d, part, nparts);
  else
    hipLaunchKernelGGL(k_gram32, dim3(xcd_grid(nparts)), dim3(WG), 0, st, cols, n, d, part,
                       nparts);
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
