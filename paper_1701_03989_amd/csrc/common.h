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

// Batched kernels keep the natural workgroup order instead: consecutive
// 256-row blocks then run on all eight XCDs at once, so the whole device
// sweeps one system at a time and that system's vectors stay in the shared
// Infinity Cache while its (possibly random) gathers reuse them; with one
// contiguous range per XCD, eight systems' streams would share the cache at
// once.  Measured: 256-system batch 609 -> 675 systems/s, serving 5.2 -> 8.6
// solves/s; the single solve of a stencil keeps the remap (1.4 % faster).
//
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
  const int64_t* off;     // start of each slice's entries
  const int32_t* width;   // entries per row of each slice
  const int32_t* col;
  const double* val;
  // Optional copy of col as 16-bit offsets from the slice's first row
  // (col = 64 t + col16 for an entry of slice t; padding rows past n hold 0),
  // present when every offset fits: the matrix-powers pass then reads 10
  // bytes per entry instead of 12.
  const int16_t* col16 = nullptr;
  // Optional value indices, present when no slice holds more than VTAB
  // distinct stored values (bitwise, padding zeros included): entry k of slice
  // t has the value vtab[VTAB t + vidx[k]], the same bits as val[k].  With
  // col16 the matrix-powers pass then reads 3 bytes per entry.
  const uint8_t* vidx = nullptr;
  const double* vtab = nullptr;
  // Optional slice-diagonal form, present when every slice couples its rows
  // to at most SD_DIAG column distances d = col - row and holds at most
  // SD_VALS distinct stored values (bitwise, padding excluded), and no row has
  // two entries at one distance: per slice the number of distances sd_nd, the
  // distances sd_delta[SD_DIAG t + k] and values sd_tab[4 t + c]; per row
  // (padded to the slices) a 16-bit word whose bits 2k, 2k+1 give the value
  // code of the row's entry at distance k, SD_ABSENT for none.  The
  // matrix-powers pass then reads 2 bytes of A per row and gathers from
  // addresses known without an index load.
  const int32_t* sd_nd = nullptr;
  const int32_t* sd_delta = nullptr;
  const double* sd_tab = nullptr;
  const uint16_t* sd_code = nullptr;
  // With the slice-diagonal form: 1 when every pair of slices (2t, 2t + 1)
  // has the same distances and values (their tables are stored in one
  // canonical order), so that the pass may take the pair's 128 rows in one
  // wavefront with the tables uniform over it.
  int32_t sd_pair = 0;
  // With the slice-diagonal form: per slice, bits 2k, 2k + 1 the value code
  // that every row with an entry at distance k has (3 where no row has one),
  // when every distance of every slice has one value (stencils with constant
  // coefficients); else null.  With sd_pair as well, both slices of each pair
  // agree on these codes.
  const uint32_t* sd_vk = nullptr;
};
constexpr int VTAB = 4;  // values in the table of a slice
constexpr int SD_DIAG = 8, SD_VALS = 3, SD_ABSENT = 3;

// Basis parameters of the three-term recurrence (monomial: theta = 0,
// gamma = sigma = 1 unused).  Chebyshev on [lmin, lmax]:
// theta_j = c0, gamma_0 = h, gamma_j = h/2, sigma_j = h/2.  Newton:
// theta_j = th[j] (the shifts), gamma_j = 1, sigma_j = 0; th is a host array
// read by the host-side launchers only (device code takes the shifts from
// the block parameters).
struct BasisPrm {
  int cheb;
  int newton;
  double c0, h, h2;
  const double* th;
};

__host__ __device__ inline BasisPrm make_basis(int basis, double lmin, double lmax,
                                               const double* th = nullptr) {
  BasisPrm b;
  b.cheb = basis == SSCG_BASIS_CHEBYSHEV;
  b.newton = basis == SSCG_BASIS_NEWTON;
  b.c0 = (lmax + lmin) * 0.5;
  b.h = (lmax - lmin) * 0.5;
  b.h2 = b.h * 0.5;
  b.th = th;
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
// The two halves of gate_closed, for kernels whose loads at the start should
// come before any store (a store there may alias what they read, which keeps
// uniform loads off the scalar path): the stop test first, the ran mark at
// the end (workgroup 0, thread 0 must reach it).
__device__ __forceinline__ bool gate_stopped(const Gate& g) { return g.stop && *g.stop; }
__device__ __forceinline__ void gate_mark_ran(const Gate& g) {
  if (g.ran && blockIdx.x == 0 && threadIdx.x == 0) *g.ran = 1;
}

// Sets *flag if rowptr decreases or a column index lies outside [0, n).
hipError_t launch_check_csr(const int32_t* rowptr, const int32_t* col, int n, int64_t nnz,
                            int32_t* flag, hipStream_t st);
hipError_t launch_sell_widths(const int32_t* rowptr, int n, int32_t* width, hipStream_t st);
hipError_t launch_scan_offsets(const int32_t* width, int nslices, int64_t* off, hipStream_t st);
// off[i] = base + 64 * (width[0] + ... + width[i-1]) for i < nslices, the
// total (base included) to *end.
hipError_t launch_scan_offsets_base(const int32_t* width, int nslices, int64_t base, int64_t* off,
                                    int64_t* end, hipStream_t st);
hipError_t launch_row_scale(const int32_t* rowptr, const double* val, int n, double* scale,
                            hipStream_t st);
hipError_t launch_sell_fill(const int32_t* rowptr, const int32_t* col, const double* val, int n,
                            const double* scale, const int64_t* off, const int32_t* width,
                            int32_t* scol, double* sval, hipStream_t st);
// col16[e] = scol[e] - 64 t for the entries of slice t (0 for rows >= n); sets
// *flag if an offset falls outside the int16 range.
// Value tables and indices of the SELL copy (vtab: VTAB per slice); *flag = 1
// if some slice holds more than VTAB distinct values (the indices are then
// not usable).
hipError_t launch_sell_vidx(const double* val, const int64_t* off, const int32_t* width,
                            int nslices, double* vtab, uint8_t* vidx, int32_t* flag,
                            hipStream_t st);
hipError_t launch_sell_compact(const int32_t* scol, int n, const int64_t* off,
                               const int32_t* width, int16_t* col16, int32_t* flag,
                               hipStream_t st);
// The slice-diagonal form of the SELL copy (DevMat::sd_*; sd_code has one
// word per row of the padded slices); *flag = 1 if some slice does not fit it.
// *flag = 1 if some pair of slices (2t, 2t + 1) differs in its distances or
// values.
hipError_t launch_sd_pairs(const int32_t* sd_nd, const int32_t* sd_delta, const double* sd_tab,
                           int nslices, int32_t* flag, hipStream_t st);
// sd_vk[t] for every slice t (see DevMat::sd_vk); flag[0] = 1 if a distance
// of some slice has two values, flag[1] = 1 if slices 2t and 2t + 1 differ in
// sd_vk for some t.
hipError_t launch_sd_values(const int32_t* sd_nd, const uint16_t* sd_code, int nslices,
                            uint32_t* sd_vk, int32_t* flag, hipStream_t st);
hipError_t launch_sell_sdia(const int32_t* rowptr, int n, const int32_t* scol, const double* sval,
                            const int64_t* off, const int32_t* width, int nslices, int32_t* sd_nd,
                            int32_t* sd_delta, double* sd_tab, uint16_t* sd_code, int32_t* flag,
                            hipStream_t st);

// One matrix-powers pass: for each of nrhs (1 or 2) sequences v,
// out = RN(A u - theta u - sigma w) / gamma_{j-1}, j >= 1 (w unused for j = 1).
template <class V>
struct MpkSeqV {  // V: the stored type of the sequence (FP64, or FP32 for an FP32 basis)
  const V* u;  // rho_{j-1}(A) v
  const V* w;  // rho_{j-2}(A) v  (j >= 2, Chebyshev)
  V* out;      // rho_j(A) v
};
using MpkSeq = MpkSeqV<double>;
using MpkSeq32 = MpkSeqV<float>;
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
// The same norms from the CSR arrays themselves (no SELL copy, one row per
// lane): rpart gets sum (b - A x)_i^2, bpart (if not NULL) sum b_i^2, in
// csr_residual_nparts(n) dd partials each.
int csr_residual_nparts(int n);
hipError_t launch_csr_residual(const int32_t* rowptr, const int32_t* col, const double* val,
                               int n, const double* b, const double* x, double* rpart,
                               double* bpart, hipStream_t st);

// Sum dd partials (pairs) of `count` independent reductions, each with
// nparts parts stored at part[(k * nparts + q) * 2]; out[k] = RN(sum).
// If sqrt_div_by != NULL: out[k] = sqrt(sum) / *sqrt_div_by... see kernels.
// out[0] = sqrt(RN(sum of the dd partials)).
hipError_t launch_finalize_sqrt(const double* part, int nparts, double* out, hipStream_t st);
hipError_t launch_finalize(const double* part, int nparts, int count, double* out,
                           hipStream_t st);

// The d basis columns of a block in G's order [P_0..P_s, R_0..R_{s-1}]
// (block 0: P only): P_0 at p0, R_0 at r0, P_j (j >= 1) at Y + j ld and R_j
// at Y + (rcol + j) ld.  Addresses are computed from the index, so a kernel
// never loads a column pointer from memory.
struct ColPtr {
  const double* p0;
  const double* r0;
  const double* Y;
  int64_t ld;
  int rcol, s;
  __device__ __forceinline__ const double* at(int a) const {
    if (a == 0) return p0;
    if (a <= s) return Y + (int64_t)a * ld;
    if (a == s + 1) return r0;
    return Y + (int64_t)(rcol + a - s - 1) * ld;
  }
};

// Gram matrix G = Y^T Y of d <= 2 SSCG_S_LIMIT + 1 columns, in the stated
// order (reading R9 for Gram matrices): the rows, zero-padded to a multiple
// of GRAM_GROUP, fall into groups of GRAM_GROUP consecutive rows; a group's
// partial of entry (a, b) is the chain of IEEE fused multiply-adds
// s <- fma(y_ra, y_rb, s) over its rows in order from +0; the partials of the
// groups, zero-padded to the next power of two, are added by pairwise
// summation (left half + right half, recursively).  launch_gram writes the
// partials, part[q * ng + g] for the upper-triangle entry q (row-major,
// a <= b) and group g < ng = gram_ngroups(n); launch_gram_finalize sums them
// into both triangles of G (d x d).  stop may be NULL.
constexpr int GRAM_GROUP = 1024;
__host__ __device__ inline int gram_ngroups(int n) { return (n + GRAM_GROUP - 1) / GRAM_GROUP; }
hipError_t launch_gram(const ColPtr& cols, int n, int d, double* part, Gate g, hipStream_t st);
hipError_t launch_gram_finalize(const double* part, int ng, int d, double* G, const int* stop,
                                hipStream_t st);

// Coordinate solve.  stop may be NULL.
hipError_t launch_kappa(const double* G, int d, int s, int first, sscg_block_info* info,
                        const int* stop, hipStream_t st);
// The coordinate recurrence; with stop != NULL a block that cannot take a
// single step (BREAKDOWN) sets *stop = 3.
// done, if given, is signalled when the kernel completes (by its own launch:
// no separate event record on the stream).
hipError_t launch_inner(const double* G, const sscg_block_params& prm, double* coef,
                        sscg_block_info* info, int* stop, hipStream_t st,
                        hipEvent_t done = nullptr);
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
// *out = max of the n ints width[] (the most nonzeros in a row of a SELL matrix).
hipError_t launch_max_width(const int32_t* width, int n, int32_t* out, hipStream_t st);
hipError_t launch_splitmix_vec(double* out, int n, uint64_t seed, hipStream_t st);
hipError_t launch_lanczos_step(const DevMat& A, const double* v, const double* vprev,
                               const double* beta_prev, double* w, double* part, int* nparts,
                               hipStream_t st);
hipError_t launch_axpy_dot(double* w, const double* v, const double* alpha, double* part,
                           int* nparts, int n, hipStream_t st);
hipError_t launch_div_vec(const double* w, const double* beta, int n, double* out,
                          hipStream_t st);
hipError_t launch_dot_parts(const double* x, const double* y, int n, double* part, int* nparts,
                            hipStream_t st);
hipError_t launch_tridiag_eig(const double* alpha, const double* beta, int k, double* lmin,
                              double* lmax, hipStream_t st);
hipError_t launch_newton_shifts(const double* alpha, const double* beta, int k, int m, double* out,
                                hipStream_t st);

// ---------------------------------------------------------------- batches
//
// A batch solves independent systems side by side.  System q owns rows
// [row0, row0 + npad) of one block-diagonal SELL-64 matrix, npad = n rounded
// up to a multiple of 256 (padding rows are empty and their vector entries
// stay 0), so every 256-row block, Gram chunk and slice belongs to one
// system.  All per-system decisions live in device tables, so the launches of
// one outer block are the same for every block and can be replayed as a
// graph.
constexpr int BATCH_ROWS = 256;                                  // rows per block
constexpr int BATCH_GSZ = (2 * SSCG_S_LIMIT + 1) * (2 * SSCG_S_LIMIT + 1);  // G per system
constexpr int BATCH_CSZ = 3 * (2 * SSCG_S_LIMIT + 1);          // coefficients per system

struct BatchSys {
  int32_t done;        // 1: finished; every later kernel skips the system
  int32_t status;      // SSCG_* once done
  int32_t first;       // the next block is the system's block 0
  int32_t m;           // inner iterations so far
  int32_t s_prev;      // s_k of the previous block
  int32_t blocks;      // blocks committed
  int32_t s_bar;       // s_bar of the current block
  int32_t row0, n;     // first row in the batch layout; rows
  int32_t blk0, blk1;  // 256-row blocks [blk0, blk1)
  int32_t ch0, ch1;    // Gram chunks [ch0, ch1)
  int32_t il;          // 1: two-sequence passes gather (P, R) pairs (scattered columns)
  int32_t vt;          // 1: passes read value tables and 16-bit offsets (all slices fit)
  int32_t sd;          // 1: passes read the slice-diagonal form (all slices fit; not il)
  int32_t p32;         // 1: the current block's basis is FP32 (SSCG_PREC_VARIABLE)
  double tol;          // target relative residual
  double eps_star;     // tol * ||b||
  double b2;           // ||b||^2
  double relres;       // latest true relative residual (relres0 before block 0)
  double lmin, lmax;   // Chebyshev interval of the system
  BasisPrm bp;         // basis parameters derived from it
};

struct BatchHist {  // one committed block of one system
  int32_t s_bar, s_built, s_tilde, s_k;
  int32_t fp32, pad_;  // 1: its basis was FP32
  double relres_true;  // true relative residual of the iterate after the block
};

struct BatchChunk {  // Gram work item: rows [r0, r1) of system sys, one GRAM_GROUP-row group
  int32_t sys, r0, r1, pad_;
};

struct BatchCfg {
  int32_t nsys, S, cap, nblk, nchunks;  // systems, passes per block, history rows, blocks, chunks
  int32_t mode, s_max, s0, f, fixed_s, inner_check, basis, max_iters;
  int64_t ld;                 // column stride of Y
  double c;                   // c_{k,j}
  double* Y;                  // columns P_0..P_S at 0..S, R_0..R_{S-1} at S+1..2S
  float* Y32;                 // the same columns of FP32 blocks (SSCG_PREC_VARIABLE), or NULL
  int32_t vprec;              // 1: each block picks its basis precision (k_batch_plan)
  double* x;                  // iterates, batch layout
  const double* b;
  BatchSys* sys;
  sscg_block_params* prm;     // this block's parameters per system
  sscg_block_info* info;
  double* G;                  // BATCH_GSZ per system
  double* coef;               // BATCH_CSZ per system
  BatchHist* hist;            // nsys * cap
  const int32_t* blk_sys;     // system of each 256-row block (-1: none)
  const BatchChunk* chunks;   // Gram work items, grouped by system
  double* rpart;              // dd partial per 256-row block (residual of x)
  double* bpart;              // dd partial per 256-row block (||b||^2, set-up)
  double* gpart;              // Gram partials: pair * nchunks + chunk
  int32_t* active;            // [0] systems not done (after each block), [1] blocks and
                              // [2] chunks of those systems (lengths of ablk / achk)
  int32_t* ablk;              // 256-row blocks of the systems not done, by system
  int32_t* achk;              // Gram chunks of the systems not done, by system
  int32_t* loff;              // per system: its first entry in ablk, in achk
  int32_t gblk, gchk;         // grids of the row launches: blocks (one per workgroup) and
                              // chunks (one per wavefront) covered at once
  int32_t kbt, gw, mch;       // launch shapes (no bits depend on them): threads per kappa
                              // problem (64, 128, 192, 256), wavefronts per Gram workgroup
                              // (1, 2, 4), matrix-powers load chunk (2, 4, 8); 0: 128, 4, 4
  double2* T[2];              // (P_j, R_j) pairs for the gathers of pass j + 1 (T[j & 1])
  const int32_t* inv;         // inv[row0 + r]: position of row r of the system (row order)
};

// The row launches of a batched block (matrix powers, Gram, recovery) stride
// over the lists of the systems not done with the grid the captured graph
// was given (BatchCfg::gblk, gchk: blocks / chunks covered at once), so
// finished systems and empty pool rows cost no work beyond that grid.
inline int batch_grid(int units) { return units < 1 ? 1 : units; }

// P_j / R_j column of a batch (global row index applies on top).
__host__ __device__ inline double* batch_col(const BatchCfg& c, int col) {
  return c.Y + (int64_t)col * c.ld;
}

// The d columns of a batched block in G's order: P_0..P_s at 0..s, R_0.. at
// S+1.. (s: the system's built steps, S: the batch's column layout).
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

// The same columns of an FP32 block (Y32, read widened to FP64).
struct BatchCols32 {
  const float* Y;
  int64_t ld;
  int s, S;
  __device__ __forceinline__ const float* at(int a) const {
    return Y + (int64_t)(a <= s ? a : S + 1 + (a - s - 1)) * ld;
  }
};

__device__ __forceinline__ BatchCols32 batch_cols32(const BatchCfg& c, int s) {
  return BatchCols32{c.Y32, c.ld, s, c.S};
}

hipError_t launch_sell_widths_n(const int32_t* rowptr, int n, int nslices, int32_t* width,
                                hipStream_t st);
hipError_t launch_sell_fill_off(const int32_t* rowptr, const int32_t* col, const double* val,
                                int n, int nslices, const int64_t* off, const int32_t* width,
                                int col_off, int32_t* scol, double* sval, hipStream_t st);
// Row order of a batched system (positions [0, npad) at row0 of the batch):
// perm[row0 + p] = original row at position p (-1: padding), inv[row0 + r] =
// row0 + position of row r; rows sorted by length within windows where that
// shrinks the SELL-64 padding.
hipError_t launch_row_order(const int32_t* rowptr, int n, int npad, int row0, int32_t* perm,
                            int32_t* inv, hipStream_t st);
// SELL-64 of a batched system in that order (perm: the system's positions).
hipError_t launch_sell_widths_perm(const int32_t* rowptr, const int32_t* perm, int nslices,
                                   int32_t* width, hipStream_t st);
// cnt[0] += stored entries, cnt[1] += those whose column, across the 64 rows
// of their slice, spans 256 or more positions (a scattered gather).
hipError_t launch_sell_fill_perm(const int32_t* rowptr, const int32_t* col, const double* val,
                                 const int32_t* perm, const int32_t* inv, int nslices,
                                 const int64_t* off, const int32_t* width, int row0,
                                 int32_t* scol, double* sval, unsigned long long* cnt,
                                 hipStream_t st);
// sys[q].il = 1 when more than a quarter of system q's entries are scattered
// (cnt[2q], cnt[2q + 1] from launch_sell_fill_perm), q in [q0, q0 + count).
hipError_t launch_set_il(BatchSys* sys, const unsigned long long* cnt, int q0, int count,
                         hipStream_t st);
// 16-bit column offsets and value tables of the batched matrix's slices
// [sl0, sl0 + count) (blk_sys must be set for them); cnt[q] gains one for
// each slice of system q that fits neither.  Then sys[q].vt = (cnt[q] == 0)
// for q in [q0, q0 + count).
hipError_t launch_sell_forms_batch(const int32_t* scol, const double* val, const int64_t* off,
                                   const int32_t* width, int sl0, int count,
                                   const int32_t* blk_sys, int16_t* col16, double* vtab,
                                   uint8_t* vidx, int32_t* cnt, hipStream_t st);
hipError_t launch_set_vt(BatchSys* sys, const int32_t* cnt, int q0, int count, hipStream_t st);
// Slice-diagonal form of one batched system's slices [slice0, slice0 + nsl)
// (perm: the system's positions -> rows, rowptr: its CSR); *cnt gains one per
// slice that does not fit.  Then sys[q].sd = (cnt[q] == 0) (and il = 0 then).
hipError_t launch_sell_sdia_sys(const int32_t* rowptr, const int32_t* perm, int slice0, int nsl,
                                const int32_t* scol, const double* sval, const int64_t* off,
                                const int32_t* width, int32_t* sd_nd, int32_t* sd_delta,
                                double* sd_tab, uint16_t* sd_code, int32_t* cnt, hipStream_t st);
hipError_t launch_set_sd(BatchSys* sys, const int32_t* cnt, int q0, int count, hipStream_t st);
// dst[p] = src[perm[p]] (0 for padding) and dst[perm[p]] = src[p], p < npad.
hipError_t launch_gather_perm(const double* src, const int32_t* perm, int npad, double* dst,
                              hipStream_t st);
hipError_t launch_scatter_perm(const double* src, const int32_t* perm, int npad, double* dst,
                               hipStream_t st);
// Batched pass j; with two sequences the gathers read the pairs tg and the
// outputs' pairs go to tw (if not NULL).
// Batched pass over the blocks listed in ablk[0, *nl) (grid: gblk workgroups
// striding over the list); chunk: entries of a row whose loads are issued
// together (2, 4 or 8; no bits depend on it).  Systems in an FP32 block read
// and write the Y32 sequences f0, f1 instead of s0, s1.
hipError_t launch_mpk_batch(const DevMat& A, int j, int cheb, int nrhs, MpkSeq s0, MpkSeq s1,
                            MpkSeq32 f0, MpkSeq32 f1, const BatchSys* sys,
                            const int32_t* blk_sys, const int32_t* ablk, const int32_t* nl,
                            int gblk, int chunk, const MpkResidual& res, const double2* tg,
                            double2* tw, hipStream_t st);
// t[i] = (a[i], b[i]), i < n.
hipError_t launch_pair(const double* a, const double* b, int64_t n, double2* t, hipStream_t st);
// Set-up from the residual of x_1 (rpart) and ||b||^2 (bpart): relres0, eps*;
// systems with b = 0 or relres0 <= tol are done before block 0.
hipError_t launch_batch_init(const BatchCfg& c, hipStream_t st);
// The same for systems [q0, q0 + count) only.
hipError_t launch_batch_init_range(const BatchCfg& c, int q0, int count, hipStream_t st);
// Sizes of this block per system (s_bar, rank guard) into prm.
hipError_t launch_batch_plan(const BatchCfg& c, hipStream_t st);
// Residual of each system's starting iterate; convergence / iteration cap.
hipError_t launch_batch_res_finalize(const BatchCfg& c, hipStream_t st);
// Gram of every unfinished system's block (its chunks are its GRAM_GROUP-row
// groups, counted from its first row), then each system's G.
hipError_t launch_gram_batch(const BatchCfg& c, hipStream_t st);
hipError_t launch_gram_finalize_batch(const BatchCfg& c, hipStream_t st);
hipError_t launch_kappa_batch(const BatchCfg& c, hipStream_t st);
// Coordinate solve and commit of the block (history, m, s_prev, breakdown).
hipError_t launch_inner_batch(const BatchCfg& c, hipStream_t st);
hipError_t launch_recover_batch(const BatchCfg& c, hipStream_t st);
hipError_t launch_batch_count(const BatchCfg& c, hipStream_t st);

// ---------------------------------------------------------------- mixed precision
//
// The FP32 basis of an inner solve: P_0..P_s at columns 0..s, R_0..R_{s-1} at
// columns rcol..rcol+s-1 of a float buffer with column stride ld.
struct Cols32 {
  const float* Y;
  int64_t ld;
  int s, rcol;
  __host__ __device__ __forceinline__ const float* at(int a) const {
    return Y + (int64_t)(a <= s ? a : rcol + (a - s - 1)) * ld;
  }
};
// out = RN32((sum_k a32_ik u_k computed exactly term by term and summed in
// FP64) - theta u_i - sigma w_i) / gamma), FP64 in between.
hipError_t launch_mpk32_pass(const DevMat& A, const float* val32, int j, BasisPrm bp, int nrhs,
                             MpkSeq32 s0, MpkSeq32 s1, hipStream_t st);
// Gram of d FP32 columns widened to FP64, in the order of launch_gram (the
// products of FP32 values are exact in FP64); same partial layout and
// finalize.
hipError_t launch_gram32(const Cols32& cols, int n, int d, double* part, hipStream_t st);
// dx += Y x' (FP64), r = RN32(Y r'), p = RN32(Y p') (r, p may alias columns).
hipError_t launch_recover32(const Cols32& cols, int n, int d, const double* coef, double* dx,
                            float* r, float* p, hipStream_t st);
hipError_t launch_cast_f32(const double* in, int64_t n, float* out, hipStream_t st);
hipError_t launch_add(double* x, const double* d, int n, hipStream_t st);  // x += d
