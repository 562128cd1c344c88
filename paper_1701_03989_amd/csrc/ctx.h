// Host-side context of libsscg and the helpers shared by api.hip (context,
// per-stage entry points) and solve.hip (the outer block loop).
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace sscg_host {

constexpr int NFAM = 4;  // timing families: mpk, gram, recover, small
constexpr int RING = 8;  // per-block records in flight (device ring, pinned host copy)
constexpr size_t RAN_CAP = 16384;  // timed launches per collection that can carry a ran flag

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

// Grow b to at least `bytes` (waits for the device before freeing).
hipError_t ensure(Buf& b, size_t bytes);

template <class T>
T* as(Buf& b) {
  return reinterpret_cast<T*>(b.p);
}

// Workspace of sscg_batch_solve (kept between calls, grown on demand).
struct BatchWs {
  Buf width, off, scol, sval, flag;  // block-diagonal SELL-64 matrix
  Buf Y, x, b;                       // basis columns, iterates, right-hand sides
  Buf Y32;                           // FP32 basis columns (SSCG_PREC_VARIABLE)
  Buf sys, prm, info, G, coef, hist, blk_sys, chunks, rpart, bpart, gpart, active;
  Buf perm, inv;                     // row order of every system (position <-> row)
  Buf T;                             // (P_j, R_j) pairs for the gathers (two N-row halves)
  Buf ilcnt;                         // per system: stored and scattered SELL entries
  Buf scol16, svidx, svtab, vtcnt;   // compact forms; per system: slices that miss them
  Buf sd_nd, sd_delta, sd_tab, sd_code, sdcnt;  // slice-diagonal form; per system: misses
  Buf ablk, achk, loff;                         // lists of the systems not done
};

// One timed interval on a stream: a single launch, or a group of launches
// enqueued back to back (the passes of one matrix-powers build), each with
// its bytes and, when gated, a ran flag of its own (ran[ran0 + i]).
struct EvRec {
  hipEvent_t a, b;
  int fam;
  double bytes;                  // ungated interval: its bytes, one launch
  int nsub;                      // gated launches in the interval
  size_t ran0;                   // first ran flag of the interval
  double sbytes[SSCG_S_LIMIT];   // bytes of each gated launch
};

}  // namespace sscg_host

struct sscg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;  // the caller's stream (main)
  hipStream_t side = nullptr;    // second stream: speculative blocks' validation
  std::string err;
  // matrix copy
  sscg_host::Buf width, off, scol, sval, scale;
  sscg_host::Buf scol16;  // 16-bit column offsets of the SELL copy (when they fit)
  sscg_host::Buf svidx, svtab;  // value indices and per-slice value tables (when few values)
  sscg_host::Buf sd_nd, sd_delta, sd_tab, sd_code;  // slice-diagonal form (stencils)
  sscg_host::Buf sd_vk;  // per slice: the value code of each distance, if one per distance
  int forms = SSCG_FMT_COL16 | SSCG_FMT_VTAB | SSCG_FMT_SDIA | SSCG_FMT_SDPAIR |
              SSCG_FMT_SDVAL;  // allowed
  // solver workspace
  sscg_host::Buf Y, part, rpart, G, coef, info, scal, xw, bw, x1, lz, lzab, ctl;
  sscg_block_info* hinfo = nullptr;  // pinned, RING entries
  double* hscal = nullptr;            // pinned
  // per ring slot: inner loop done (S1), validation done (S2)
  hipEvent_t evI[sscg_host::RING], evV[sscg_host::RING];
  bool events_made = false;
  // timing
  unsigned timing = 0;  // bit f: time kernel family f
  int64_t launches[sscg_host::NFAM] = {0, 0, 0, 0};
  double ms[sscg_host::NFAM] = {0, 0, 0, 0};
  double bytes[sscg_host::NFAM] = {0, 0, 0, 0};
  std::vector<sscg_host::EvRec> ev;
  size_t ev_used = 0;
  size_t ran_used = 0;  // ran flags handed out since the last collection
  sscg_host::Buf ran;  // int[RAN_CAP] device flags of gated timed launches (zero between uses)
  std::vector<int> hran;
  sscg_host::BatchWs batch;
  int32_t* hactive = nullptr;  // pinned
  int64_t sell_total = 0;      // SELL-64 entries of the last matrix copy
  double mat_bytes = 0.0;      // bytes of it one matrix-powers pass reads (mpk_matrix_bytes)
  // mixed precision: FP32 values of the SELL copy, FP32 basis, FP64 correction and residual
  sscg_host::Buf sval32, Y32, dx, r64;
  sscg_host::Buf xu, upart;  // equilibrated mixed solves: unscaled iterate, its residual partials
  void* scratch = nullptr;   // device address of the static scratch array on this device
  // launch-shape tuning of batches (sscg_set_batch_tuning, sscg_batch_tuning)
  int tune_mode = 1;                 // 1: time the candidates once per batch shape; 0: fixed
  int fixed_kbt = 128, fixed_gw = 4, fixed_mch = 4;  // the shapes of mode 0
  struct TuneEntry {
    int64_t rows;
    int nsys, S, kbt, gw, mch;
  };
  std::vector<TuneEntry> tuned;  // choices per batch shape (rows, systems, s_max)
  int last_kbt = 0, last_gw = 0, last_mch = 0;  // the shapes the last batch ran with
  double last_kappa_us[4] = {0, 0, 0, 0};       // its timings (NaN: not timed)
  double last_gram_us[3] = {0, 0, 0}, last_mpk_us[3] = {0, 0, 0};
};

namespace sscg_host {

int fail(sscg_ctx* c, int code, const char* fmt, ...);

#define HIPCHK(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return ::sscg_host::fail(ctx, e_ == hipErrorOutOfMemory ? SSCG_ERR_OOM : SSCG_ERR_HIP,   \
                               "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                               __LINE__);                                                      \
  } while (0)

int set_device(sscg_ctx* ctx);
// event pair around one launch when its family is timed (slot NO_EVENT otherwise)
constexpr size_t NO_EVENT = ~(size_t)0;
hipError_t ev_begin(sscg_ctx* c, int fam, double bytes, hipStream_t st, size_t* slot);
hipError_t ev_end(sscg_ctx* c, size_t slot, hipStream_t st);
// The ran flag of a timed launch (NULL if the slot is not timed): only launches
// whose first workgroup ran are counted by the statistics.  ev_ran: the
// slot's single launch (its bytes from ev_begin); ev_sub: one more launch of
// a group timed as one interval (up to SSCG_S_LIMIT per slot).
int* ev_ran(sscg_ctx* c, size_t slot);
int* ev_sub(sscg_ctx* c, size_t slot, double bytes);
hipError_t ev_collect(sscg_ctx* c);
hipError_t ev_drop(sscg_ctx* c);

int check_csr(sscg_ctx* ctx, const sscg_csr* A);
int build_mat(sscg_ctx* ctx, const sscg_csr* A, int equilibrate, DevMat* M);
int ensure_parts(sscg_ctx* ctx, int n, int count);
int validate_opts(sscg_ctx* ctx, const sscg_opts* o);
int spectral_bounds_dev(sscg_ctx* ctx, const DevMat& M, int steps, uint64_t seed, double* lmin,
                        double* lmax);
// Basis and c_{k,j} parameters of a solve on M: the Chebyshev interval and
// the Newton shifts (given or estimated), and for the c_{k,j} of Section 4.1
// N_A, kappa(A) and ||A|| (given, else from the spectral estimate).
struct MethodSetup {
  BasisPrm bp;
  double lmin, lmax;
  double shifts[SSCG_S_LIMIT];
  int c_mode, n_a, s_max;
  double kappa_a, norm_a;
  void fill(sscg_block_params& prm) const {
    prm.c_mode = c_mode;
    prm.n_a = n_a;
    prm.s_max = s_max;
    prm.pad_ = 0;
    prm.kappa_a = kappa_a;
    prm.norm_a = norm_a;
    for (int i = 0; i < SSCG_S_LIMIT; ++i) prm.shifts[i] = shifts[i];
  }
};
int method_setup(sscg_ctx* ctx, const DevMat& M, const sscg_opts& o, MethodSetup* ms);
// sscg_solve with SSCG_PREC_VARIABLE (a batch of one system).
int solve_variable(sscg_ctx* ctx, const sscg_csr* A, const double* b, double* x,
                   const sscg_opts& o, sscg_result* res);
// m Newton shifts (host output) from an m-step Lanczos run on M.
int newton_shifts_dev(sscg_ctx* ctx, const DevMat& M, int m, uint64_t seed, double* shifts);
// Most nonzeros in a row of M (from the SELL widths).
int max_row_nnz_dev(sscg_ctx* ctx, const DevMat& M, int* n_a);

// Basis columns of an s-step block: P_0 and R_0 at p0 / r0, P_j (j >= 1) at
// Y + j*ldy, R_j (j >= 1) at Y + (rcol + j)*ldy.
struct BasisCols {
  const double* p0;
  const double* r0;
  double* Y;
  int64_t ldy;
  int rcol;
  double* P(int j) const { return j == 0 ? const_cast<double*>(p0) : Y + (int64_t)j * ldy; }
  double* R(int j) const {
    return j == 0 ? const_cast<double*>(r0) : Y + (int64_t)(rcol + j) * ldy;
  }
};
ColPtr colptr_of(const BasisCols& bc, int s, int first);

// The test of the block's starting iterate on its fused residual: after the
// first pass, relres_in = ||res|| / sqrt(*b2) into info and *stop set at
// tol, so that a converged block's remaining passes stand down.
struct ResCheck {
  const double* b2 = nullptr;  // null: no test inside the passes
  int nparts = 0;
  double tol = 0.0;
  sscg_block_info* info = nullptr;
  int* stop = nullptr;  // the solve's stop flag (the passes' gate)
};
// The s passes of the matrix powers kernel of one block (res: fused residual
// of the block's start, may be {NULL}); stop may be NULL.
int mpk_passes(sscg_ctx* ctx, const DevMat& M, int s, int first, BasisPrm bp, const BasisCols& bc,
               double mat_bytes, const int* stop, const MpkResidual& res,
               const ResCheck& chk = ResCheck{});
// Bytes of A one matrix-powers pass reads in the form it dispatches on: per
// stored SELL-64 entry 3 (one-byte value index, 16-bit column offset), 10
// (value, 16-bit offset) or 12 (value, 32-bit index), plus per slice its
// offset, width and (value tables) its 4-entry table.
double mpk_matrix_bytes(const DevMat& M, int64_t stored);
// Gram of the block's basis into G (device, d x d).
int gram_into(sscg_ctx* ctx, const ColPtr& cols, int n, int d, double* G, const int* stop);

// One outer block of a batch for every unfinished system (capturable).
int batch_enqueue_block(sscg_ctx* ctx, const DevMat& M, const BatchCfg& c, hipStream_t st);

// Graphs of one outer block (batch_enqueue_block) whose row launches have
// grids of 1/4^k of the full lists (k = 0, 1, ...; down to about 256 blocks),
// so that a replay launches about as many workgroups as the systems not done
// have blocks (the launches stride over the lists, so any grid is correct).
struct BlockGraphs {
  std::vector<hipGraph_t> g;
  std::vector<hipGraphExec_t> e;
  std::vector<int> gblk, gchk;
  BlockGraphs() = default;
  BlockGraphs(const BlockGraphs&) = delete;
  BlockGraphs& operator=(const BlockGraphs&) = delete;
  ~BlockGraphs() { clear(); }
  void clear();
  int capture(sscg_ctx* ctx, const DevMat& M, const BatchCfg& c, hipStream_t st);
  // the smallest grids that cover nb blocks and nc chunks
  size_t pick_index(int64_t nb, int64_t nc) const;
  hipGraphExec_t pick(int64_t nb, int64_t nc) const;
};

// Look up the device address of the static scratch array of
// sscg_gram_noalloc on ctx's device (current), once per device; sets
// ctx->scratch.
int scratch_setup(sscg_ctx* ctx);

// sscg_solve with opts->precision = SSCG_PREC_MIXED (arguments checked).
int solve_mixed(sscg_ctx* ctx, const sscg_csr* A, const double* b, double* x, const sscg_opts& o,
                sscg_result* res);
// The FP32 copy of the values of the current SELL matrix (after build_mat).
int build_val32(sscg_ctx* ctx, float** val32);

}  // namespace sscg_host
