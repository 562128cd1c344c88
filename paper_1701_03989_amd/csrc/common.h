// Shared device helpers and launch declarations of libsscg (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sscg.h"

#define SSCG_WAVE 64
#define SSCG_XCDS 8  // MI355X: 8 accelerator complex dies, one L2 each

// ---------------------------------------------------------------- dd sums
//
// A correctly rounded sum is approximated by a double-double accumulator:
// the running sum s and a plain sum e of the exact errors.  Each product
// enters exactly as fl(x*y) + fma(x, y, -fl(x*y)); each addition's error comes
// from TwoSum (Knuth).  The result fl(s + e) differs from the correctly
// rounded exact sum only if that sum lies within about n^2 2^-106 sum|terms|
// of a rounding boundary.  The code is compiled with -ffp-contract=off, so no
// other multiply-add is fused.
struct dd {
  double s, e;
};

__device__ __forceinline__ dd dd_zero() { return dd{0.0, 0.0}; }

__device__ __forceinline__ void dd_add(dd& a, double p) {
  double t = a.s + p;
  double bp = t - a.s;
  double err = (a.s - (t - bp)) + (p - bp);
  a.s = t;
  a.e = a.e + err;
}

__device__ __forceinline__ void dd_add_prod(dd& a, double x, double y) {
  double p = x * y;
  double pe = __builtin_fma(x, y, -p);
  double t = a.s + p;
  double bp = t - a.s;
  double err = (a.s - (t - bp)) + (p - bp);
  a.s = t;
  a.e = a.e + (err + pe);
}

__device__ __forceinline__ void dd_merge(dd& a, const dd& b) {
  double t = a.s + b.s;
  double bp = t - a.s;
  double err = (a.s - (t - bp)) + (b.s - bp);
  a.s = t;
  a.e = a.e + (b.e + err);
}

__device__ __forceinline__ double dd_round(const dd& a) { return a.s + a.e; }

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, SSCG_WAVE);
}

// Reduce a dd over the 64 lanes of a wave; every lane gets the total.
__device__ __forceinline__ dd dd_wave_reduce(dd a) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    dd o{shfl_xor_d(a.s, m), shfl_xor_d(a.e, m)};
    dd_merge(a, o);
  }
  return a;
}

// Workgroup index remapped so that each XCD works on one contiguous range of
// logical blocks (workgroups are dispatched to XCDs round-robin): neighbouring
// rows then share an L2.  Launch exactly xcd_grid(nb) workgroups; a
// workgroup whose logical index is >= nb must return.
__host__ __device__ __forceinline__ int xcd_grid(int nb) {
  int per = (nb + SSCG_XCDS - 1) / SSCG_XCDS;
  return per * SSCG_XCDS;
}
__device__ __forceinline__ int xcd_block(int nb) {
  int per = (nb + SSCG_XCDS - 1) / SSCG_XCDS;
  int b = blockIdx.x;
  return (b % SSCG_XCDS) * per + b / SSCG_XCDS;
}

// ---------------------------------------------------------------- matrix
//
// SELL-64 copy of a CSR matrix (built on the device once per call): rows in
// their original order, cut into slices of 64 (one wavefront); slice t holds
// width[t] = max row length of its rows, stored column-major so that lane l
// reads element j of row 64 t + l at off[t] + 64 j + l.  Padding: value 0,
// column = own row (rows past n: column 0).
struct DevMat {
  int32_t n;
  int32_t nslices;
  const int64_t* off;   // nslices + 1
  const int32_t* col;
  const double* val;
};

// Basis parameters of the three-term recurrence (monomial: theta = 0,
// gamma = sigma = 1 unused).  Chebyshev on [lmin, lmax]:
// theta_j = c0, gamma_0 = h, gamma_j = h/2, sigma_j = h/2.
struct BasisPrm {
  int cheb;
  double c0, h, h2;
};

__host__ __device__ inline BasisPrm make_basis(int basis, double lmin, double lmax) {
  BasisPrm b;
  b.cheb = basis == SSCG_BASIS_CHEBYSHEV;
  b.c0 = (lmax + lmin) * 0.5;
  b.h = (lmax - lmin) * 0.5;
  b.h2 = b.h * 0.5;
  return b;
}

// ---------------------------------------------------------------- launches
// (host wrappers; every one enqueues on `st` and returns the launch error)

// Launch gate of the streaming kernels.  A launch stands down (every
// workgroup returns at once) while *stop != 0; when `ran` is set, the first
// workgroup of a launch that does run stores 1 there, so kernel timing can
// tell launches that moved their bytes from launches that stood down.
struct Gate {
  const int* stop;
  int* ran;
};

__device__ __forceinline__ bool gate_closed(const Gate& g) {
  if (g.stop && *g.stop) return true;
  if (g.ran && blockIdx.x == 0 && threadIdx.x == 0) *g.ran = 1;
  return false;
}

// Sets *flag if rowptr decreases or a column index lies outside [0, n).
hipError_t launch_check_csr(const int32_t* rowptr, const int32_t* col, int n, int nnz,
                            int32_t* flag, hipStream_t st);
hipError_t launch_sell_widths(const int32_t* rowptr, int n, int32_t* width, hipStream_t st);
hipError_t launch_scan_offsets(const int32_t* width, int nslices, int64_t* off, hipStream_t st);
hipError_t launch_row_scale(const int32_t* rowptr, const double* val, int n, double* scale,
                            hipStream_t st);
hipError_t launch_sell_fill(const int32_t* rowptr, const int32_t* col, const double* val, int n,
                            const double* scale, const int64_t* off, int32_t* scol, double* sval,
                            hipStream_t st);

// One matrix-powers pass: for each of nrhs (1 or 2) sequences v,
// out = RN(A u - theta u - sigma w) / gamma_{j-1}, j >= 1 (w unused for j = 1).
struct MpkSeq {
  const double* u;  // rho_{j-1}(A) v
  const double* w;  // rho_{j-2}(A) v  (j >= 2, Chebyshev)
  double* out;      // rho_j(A) v
};
// Optional fused true residual of the block's starting iterate (x != NULL):
// per-workgroup dd partials of sum (b - A x)_i^2 into part.
struct MpkResidual {
  const double* x;
  const double* b;
  double* part;
};
hipError_t launch_mpk_pass(const DevMat& A, int j, BasisPrm bp, int nrhs, MpkSeq s0, MpkSeq s1,
                           Gate g, const MpkResidual& res, hipStream_t st);

// res_i = RN(b_i - (A x)_i) (written if r != NULL); per-workgroup dd partials
// of sum res_i^2 and (if bpart != NULL) sum b_i^2.
hipError_t launch_residual(const DevMat& A, const double* b, const double* x, double* r,
                           double* rpart, double* bpart, int* nparts, hipStream_t st);
int residual_nparts(int n);

// Sum dd partials (pairs) of `count` independent reductions, each with
// nparts parts stored at part[(k * nparts + q) * 2]; out[k] = RN(sum).
// If sqrt_div_by != NULL: out[k] = sqrt(sum) / *sqrt_div_by... see kernels.
hipError_t launch_finalize(const double* part, int nparts, int count, double* out,
                           hipStream_t st);

// The d basis columns of a block in G's order [P_0..P_s, R_0..R_{s-1}].
struct ColPtr {
  const double* c[2 * SSCG_S_LIMIT + 1];
};

// Gram of the d columns; partials then the finalize.  stop may be NULL.
int gram_nparts(int n);
hipError_t launch_gram(const ColPtr& cols, int n, int d, double* part, int nparts, Gate g,
                       hipStream_t st);
hipError_t launch_gram_finalize(const double* part, int nparts, int d, double* G,
                                const int* stop, hipStream_t st);

// Coordinate solve.  stop may be NULL.
hipError_t launch_kappa(const double* G, int d, int s, int first, sscg_block_info* info,
                        const int* stop, hipStream_t st);
// The coordinate recurrence; with stop != NULL a block that cannot take a
// single step (BREAKDOWN) sets *stop = 3.
hipError_t launch_inner(const double* G, const sscg_block_params& prm, double* coef,
                        sscg_block_info* info, int* stop, hipStream_t st);
// Replays the decisions of eq. condy and eq. check from the kappa list and
// the recorded r'^T G r' of a block run speculatively with s~ = s and no
// break; if they would have chosen s_k != s, sets *stop = 2 (redo the block).
hipError_t launch_validate(const double* G, const sscg_block_params& prm, sscg_block_info* info,
                           int* stop, hipStream_t st);
// Sum the fused residual partials: info->relres_in = sqrt(sum)/sqrt(*b2);
// sets *stop = 1 if relres_in <= tol (or 3 if it is not finite).
hipError_t launch_res_finalize(const double* part, int nparts, const double* b2, double tol,
                               sscg_block_info* info, int* stop, hipStream_t st);

// Recovery: x_out = RN(x_in + Y x'), r = RN(Y r'), p = RN(Y p').  x_out may
// equal x_in; r and p may alias columns (each row is read before it is
// written).
hipError_t launch_recover(const ColPtr& cols, int n, int d, const double* coef, const double* x_in,
                          double* x_out, double* r, double* p, Gate g, hipStream_t st);

// Small helpers.
hipError_t launch_scale_vec(const double* in, const double* s, int mul, int n, double* out,
                            hipStream_t st);  // out = mul ? in*s : in/s
hipError_t launch_copy(const double* in, int n, double* out, hipStream_t st);
hipError_t launch_fill(double* out, int n, double v, hipStream_t st);
hipError_t launch_relres(const double* r2, const double* b2, double* out, hipStream_t st);

// Spectral bounds.
hipError_t launch_gershgorin(const DevMat& A, double* part, int* nparts, hipStream_t st);
hipError_t launch_max_finalize(const double* part, int nparts, double* out, hipStream_t st);
hipError_t launch_splitmix_vec(double* out, int n, uint64_t seed, hipStream_t st);
hipError_t launch_lanczos_step(const DevMat& A, const double* v, const double* vprev,
                               const double* beta_prev, double* w, double* part, int* nparts,
                               hipStream_t st);
hipError_t launch_axpy_dot(double* w, const double* v, const double* alpha, double* part,
                           int* nparts, int n, hipStream_t st);
hipError_t launch_sqrt_scalar(double* x, hipStream_t st);
hipError_t launch_div_vec(const double* w, const double* beta, int n, double* out,
                          hipStream_t st);
hipError_t launch_dot_parts(const double* x, const double* y, int n, double* part, int* nparts,
                            hipStream_t st);
hipError_t launch_tridiag_eig(const double* alpha, const double* beta, int k, double* lmin,
                              double* lmax, hipStream_t st);
