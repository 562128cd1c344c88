// sscg_batch_solve: independent systems advanced together, one outer block
// (Algorithm 4, or 2) at a time for all of them.
//
// Layout: system q owns rows [row0_q, row0_q + npad_q) of one block-diagonal
// SELL-64 matrix and of every batch vector, npad_q = n_q rounded up to a
// multiple of 256, so that each 256-row block (one workgroup of the streaming
// kernels), each Gram chunk and each slice belongs to one system.  Padding
// rows are empty and their vector entries stay zero, so they add nothing to
// any sum.  Within a system the rows are in the order of launch_row_order
// (sorted by length in windows where that shrinks the SELL padding); b and
// x are permuted on the way in and out.  Every per-system decision (s_bar_k, the rank guard, s~_k, s_k,
// convergence, the iteration cap) is taken on the device from the system
// table, so one outer block is the same sequence of launches for every block:
// it is captured once as a HIP graph and replayed until no system is left.
// The per-system arithmetic is the single-system path's, kernel for kernel,
// so a system's result does not depend on the rest of the batch.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ctx.h"

using namespace sscg_host;

namespace {

constexpr int CHUNK_ROWS = 1024;  // rows per Gram work item
constexpr int GROUP = 4;          // blocks replayed between checks of the active count
constexpr int KBT_CAND[4] = {64, 128, 192, 256};  // threads per kappa problem
constexpr int GW_CAND[3] = {1, 2, 4};             // wavefronts per Gram workgroup
constexpr int MCH_CAND[3] = {2, 4, 8};            // matrix-powers load chunk
constexpr int TUNE_REPS = 3;                      // timed runs per candidate (the fastest counts)

// The launch shapes of a batch, timed on its live state after its first
// GROUP blocks: every candidate of the next block's first matrix-powers pass,
// kappa and Gram launches is run TUNE_REPS times on the current iterates,
// Gram matrices and basis (their outputs, P_1, R_1, the residual partials,
// the pairs of pass 2, kappa values and Gram partials, are recomputed by the
// next block before anything reads them, and no bits depend on the shapes),
// and the fastest of each is kept in c.  gblk, gchk: the grids the next
// block will use.
int tune_shapes(sscg_ctx* ctx, const DevMat& M, BatchCfg& c, int gblk, int gchk,
                hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    HIPCHK(e);
  }
  BatchCfg t = c;
  t.gblk = gblk;
  t.gchk = gchk;
  // pass 1 of the next block, as batch_enqueue_block launches it
  const int rb = c.S + 1;
  const MpkSeq sp{batch_col(c, 0), nullptr, batch_col(c, 1)};
  const MpkSeq sr{batch_col(c, rb), nullptr, batch_col(c, rb + 1)};
  const MpkResidual res{c.x, c.b, c.rpart};
  MpkSeq32 fp{nullptr, nullptr, nullptr}, fr{nullptr, nullptr, nullptr};
  if (c.Y32) {
    fp = MpkSeq32{c.Y32, nullptr, c.Y32 + c.ld};
    fr = MpkSeq32{c.Y32 + (int64_t)rb * c.ld, nullptr, c.Y32 + (int64_t)(rb + 1) * c.ld};
  }
  auto pass1 = [&]() {
    return launch_mpk_batch(M, 1, c.basis == SSCG_BASIS_CHEBYSHEV, c.S >= 2 ? 2 : 1, sp, sr, fp,
                            fr, c.sys, c.blk_sys, c.ablk, c.active + 1, gblk, t.mch, res,
                            c.T[0], c.S >= 3 ? c.T[1] : nullptr, st);
  };
  auto timed = [&](int what, double* us) -> hipError_t {
    double best = INFINITY;
    for (int r = 0; r < TUNE_REPS; ++r) {
      hipError_t x = hipEventRecord(e0, st);
      if (x == hipSuccess)
        x = what == 0 ? pass1() : (what == 1 ? launch_kappa_batch(t, st) : launch_gram_batch(t, st));
      if (x == hipSuccess) x = hipEventRecord(e1, st);
      if (x == hipSuccess) x = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
      if (x != hipSuccess) return x;
      best = std::min(best, 1e3 * (double)ms);
    }
    *us = best;
    return hipSuccess;
  };
  e = hipSuccess;
  int kbt = c.kbt, gw = c.gw, mch = c.mch;
  double bk = INFINITY, bg = INFINITY, bm = INFINITY;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) {
    t.mch = MCH_CAND[i];
    e = timed(0, &ctx->last_mpk_us[i]);
    if (e == hipSuccess && ctx->last_mpk_us[i] < bm) {
      bm = ctx->last_mpk_us[i];
      mch = MCH_CAND[i];
    }
  }
  t.mch = mch;
  if (c.mode == SSCG_MODE_ADAPTIVE)
    for (int i = 0; i < 4 && e == hipSuccess; ++i) {
      t.kbt = KBT_CAND[i];
      e = timed(1, &ctx->last_kappa_us[i]);
      if (e == hipSuccess && ctx->last_kappa_us[i] < bk) {
        bk = ctx->last_kappa_us[i];
        kbt = KBT_CAND[i];
      }
    }
  t.kbt = kbt;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) {
    t.gw = GW_CAND[i];
    e = timed(2, &ctx->last_gram_us[i]);
    if (e == hipSuccess && ctx->last_gram_us[i] < bg) {
      bg = ctx->last_gram_us[i];
      gw = GW_CAND[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(e);
  c.kbt = kbt;
  c.gw = gw;
  c.mch = mch;
  return SSCG_OK;
}

}  // namespace

void sscg_host::BlockGraphs::clear() {
  for (hipGraphExec_t x : e)
    if (x) (void)hipGraphExecDestroy(x);
  for (hipGraph_t x : g)
    if (x) (void)hipGraphDestroy(x);
  e.clear();
  g.clear();
  gblk.clear();
  gchk.clear();
}

int sscg_host::BlockGraphs::capture(sscg_ctx* ctx, const DevMat& M, const BatchCfg& c0,
                                    hipStream_t st) {
  clear();
  int64_t nb = c0.nblk, nc = c0.nchunks;
  for (;;) {
    BatchCfg c = c0;
    c.gblk = (int)nb;
    c.gchk = (int)nc;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = batch_enqueue_block(ctx, M, c, st);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(st, &graph);
    if (graph) g.push_back(graph);
    if (rc) return rc;
    HIPCHK(ce);
    hipGraphExec_t x = nullptr;
    HIPCHK(hipGraphInstantiate(&x, graph, nullptr, nullptr, 0));
    e.push_back(x);
    gblk.push_back((int)nb);
    gchk.push_back((int)nc);
    if (nb <= 1024) break;
    nb = (nb + 3) / 4;
    nc = (nc + 3) / 4;
  }
  return SSCG_OK;
}

size_t sscg_host::BlockGraphs::pick_index(int64_t nb, int64_t nc) const {
  size_t k = e.size() - 1;
  while (k > 0 && (gblk[k] < nb || gchk[k] < nc)) --k;
  return k;
}

hipGraphExec_t sscg_host::BlockGraphs::pick(int64_t nb, int64_t nc) const {
  return e[pick_index(nb, nc)];
}

extern "C" int sscg_set_batch_tuning(sscg_ctx* ctx, int mode, int kappa_threads, int gram_waves,
                                     int mpk_chunk) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  if (mode != 0 && mode != 1) return fail(ctx, SSCG_ERR_ARG, "tuning mode must be 0 or 1");
  if (mode == 0) {
    const int kbt = kappa_threads ? kappa_threads : 128, gw = gram_waves ? gram_waves : 4;
    if (kbt != 64 && kbt != 128 && kbt != 192 && kbt != 256)
      return fail(ctx, SSCG_ERR_ARG, "kappa threads must be 64, 128, 192 or 256");
    if (gw != 1 && gw != 2 && gw != 4)
      return fail(ctx, SSCG_ERR_ARG, "Gram wavefronts must be 1, 2 or 4");
    const int mch = mpk_chunk ? mpk_chunk : 4;
    if (mch != 2 && mch != 4 && mch != 8)
      return fail(ctx, SSCG_ERR_ARG, "matrix-powers load chunk must be 2, 4 or 8");
    ctx->fixed_kbt = kbt;
    ctx->fixed_gw = gw;
    ctx->fixed_mch = mch;
  }
  ctx->tune_mode = mode;
  ctx->tuned.clear();
  return SSCG_OK;
}

extern "C" int sscg_batch_tuning(sscg_ctx* ctx, int32_t* kappa_threads, int32_t* gram_waves,
                                 int32_t* mpk_chunk, double* kappa_us, double* gram_us,
                                 double* mpk_us) {
  if (!ctx) return SSCG_ERR_ARG;
  if (kappa_threads) *kappa_threads = ctx->last_kbt;
  if (gram_waves) *gram_waves = ctx->last_gw;
  if (mpk_chunk) *mpk_chunk = ctx->last_mch;
  if (mpk_us)
    for (int i = 0; i < 3; ++i) mpk_us[i] = ctx->last_mpk_us[i];
  if (kappa_us)
    for (int i = 0; i < 4; ++i) kappa_us[i] = ctx->last_kappa_us[i];
  if (gram_us)
    for (int i = 0; i < 3; ++i) gram_us[i] = ctx->last_gram_us[i];
  return SSCG_OK;
}

// One outer block for every unfinished system (enqueued on st; capturable).
int sscg_host::batch_enqueue_block(sscg_ctx* ctx, const DevMat& M, const BatchCfg& c,
                                   hipStream_t st) {
  HIPCHK(launch_batch_plan(c, st));
  const int cheb = c.basis == SSCG_BASIS_CHEBYSHEV;
  auto col32 = [&](int col) { return c.Y32 ? c.Y32 + (int64_t)col * c.ld : nullptr; };
  for (int j = 1; j <= c.S; ++j) {
    MpkSeq sp{batch_col(c, j - 1), j >= 2 ? batch_col(c, j - 2) : nullptr, batch_col(c, j)};
    const int rb = c.S + 1;  // R_j at column rb + j
    MpkSeq sr{batch_col(c, rb + j - 1), j >= 2 ? batch_col(c, rb + j - 2) : nullptr,
              batch_col(c, rb + j)};
    MpkSeq32 fp{col32(j - 1), j >= 2 ? col32(j - 2) : nullptr, col32(j)};
    MpkSeq32 fr{col32(rb + j - 1), j >= 2 ? col32(rb + j - 2) : nullptr, col32(rb + j)};
    const int nrhs = j <= c.S - 1 ? 2 : 1;
    MpkResidual res{};
    if (j == 1) res = MpkResidual{c.x, c.b, c.rpart};
    // two-sequence passes gather (P_{j-1}, R_{j-1}) pairs from T[(j-1) & 1] and
    // leave theirs in T[j & 1] when the next pass gathers pairs too
    double2* tw = j + 1 <= c.S - 1 ? c.T[j & 1] : nullptr;
    HIPCHK(launch_mpk_batch(M, j, cheb, nrhs, sp, sr, fp, fr, c.sys, c.blk_sys, c.ablk,
                            c.active + 1, c.gblk, c.mch, res, c.T[(j - 1) & 1], tw,
                            st));
    if (j == 1) HIPCHK(launch_batch_res_finalize(c, st));
  }
  HIPCHK(launch_gram_batch(c, st));
  HIPCHK(launch_gram_finalize_batch(c, st));
  if (c.mode == SSCG_MODE_ADAPTIVE) HIPCHK(launch_kappa_batch(c, st));
  HIPCHK(launch_inner_batch(c, st));
  HIPCHK(launch_recover_batch(c, st));
  HIPCHK(launch_batch_count(c, st));
  return SSCG_OK;
}

extern "C" int sscg_batch_solve(sscg_ctx* ctx, const sscg_batch* B, const sscg_opts* opts,
                                sscg_batch_result* res) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = validate_opts(ctx, opts))) return rc;
  const sscg_opts& o = *opts;
  if (!B || B->nsys < 1 || !B->A || !B->b || !B->x)
    return fail(ctx, SSCG_ERR_ARG, "batch: nsys >= 1 and the A, b, x arrays are required");
  if (o.mode == SSCG_MODE_SCHEDULE)
    return fail(ctx, SSCG_ERR_ARG, "batch: MODE_SCHEDULE is not supported");
  if (o.equilibrate) return fail(ctx, SSCG_ERR_ARG, "batch: equilibration is not supported");
  if (o.basis == SSCG_BASIS_NEWTON || o.c_mode != SSCG_C_CONST)
    return fail(ctx, SSCG_ERR_ARG, "batch: the Newton basis and the theoretical c are not supported");
  if (o.precision == SSCG_PREC_MIXED)
    return fail(ctx, SSCG_ERR_ARG, "batch: SSCG_PREC_MIXED is not supported (SSCG_PREC_VARIABLE is)");
  const int nsys = B->nsys;
  const bool cheb = o.basis == SSCG_BASIS_CHEBYSHEV;
  if (cheb && (!B->lambda_min || !B->lambda_max))
    return fail(ctx, SSCG_ERR_ARG, "batch: the Chebyshev basis needs per-system intervals");
  for (int q = 0; q < nsys; ++q) {
    if ((rc = check_csr(ctx, &B->A[q]))) return rc;
    if (!B->b[q] || !B->x[q]) return fail(ctx, SSCG_ERR_ARG, "batch: b[%d] or x[%d] is NULL", q, q);
    if (cheb && !(B->lambda_max[q] > B->lambda_min[q]))
      return fail(ctx, SSCG_ERR_ARG, "batch: need lambda_max > lambda_min (system %d)", q);
    if (B->tol && !(B->tol[q] > 0.0)) return fail(ctx, SSCG_ERR_ARG, "batch: tol[%d] <= 0", q);
  }

  // ---- layout
  std::vector<BatchSys> hs(nsys);
  std::vector<BatchChunk> hc;
  int64_t rows = 0;
  for (int q = 0; q < nsys; ++q) {
    const int n = B->A[q].n;
    const int64_t npad = std::max<int64_t>(BATCH_ROWS, ((int64_t)n + BATCH_ROWS - 1) / BATCH_ROWS *
                                                           BATCH_ROWS);
    BatchSys& s = hs[q];
    memset(&s, 0, sizeof s);
    s.row0 = (int32_t)rows;
    s.n = n;
    s.blk0 = (int32_t)(rows / BATCH_ROWS);
    s.blk1 = (int32_t)((rows + npad) / BATCH_ROWS);
    s.ch0 = (int32_t)hc.size();
    for (int64_t r = rows; r < rows + npad; r += CHUNK_ROWS)
      hc.push_back(BatchChunk{q, (int32_t)r, (int32_t)std::min(r + CHUNK_ROWS, rows + npad), 0});
    s.ch1 = (int32_t)hc.size();
    s.tol = B->tol ? B->tol[q] : o.tol;
    s.lmin = cheb ? B->lambda_min[q] : 0.0;
    s.lmax = cheb ? B->lambda_max[q] : 1.0;
    rows += npad;
  }
  if (rows > INT32_MAX / 2) return fail(ctx, SSCG_ERR_ARG, "batch: %lld rows are too many",
                                        (long long)rows);
  const int N = (int)rows;
  const int nblk = N / BATCH_ROWS, nslices = N / SSCG_WAVE, nchunks = (int)hc.size();
  std::vector<int32_t> hblk(nblk);
  for (int q = 0; q < nsys; ++q)
    for (int k = hs[q].blk0; k < hs[q].blk1; ++k) hblk[k] = q;
  const int S = o.mode == SSCG_MODE_FIXED ? o.fixed_s : o.s_max;
  const int ncols = 2 * S + 1;  // P_0..P_S, R_0..R_{S-1}
  const int cap = std::max(1, std::min(o.max_iters + 2, res && res->cap > 0 ? res->cap : 1));
  const int dmax = 2 * S + 1, npairs = dmax * (dmax + 1) / 2;

  // ---- workspace (nothing is reallocated once blocks run)
  BatchWs& w = ctx->batch;
  hipStream_t st = ctx->side;
  HIPCHK(hipStreamSynchronize(ctx->stream));  // the caller's A, b, x are ready
  HIPCHK(ensure(w.width, sizeof(int32_t) * (nslices + 1)));
  HIPCHK(ensure(w.off, sizeof(int64_t) * (nslices + 1)));
  HIPCHK(ensure(w.flag, sizeof(int32_t) * 4));
  HIPCHK(ensure(w.Y, sizeof(double) * (size_t)N * ncols));
  const bool vprec = o.precision == SSCG_PREC_VARIABLE;
  if (vprec) HIPCHK(ensure(w.Y32, sizeof(float) * (size_t)N * ncols));
  HIPCHK(ensure(w.x, sizeof(double) * (size_t)N));
  HIPCHK(ensure(w.b, sizeof(double) * (size_t)N));
  HIPCHK(ensure(w.sys, sizeof(BatchSys) * nsys));
  HIPCHK(ensure(w.prm, sizeof(sscg_block_params) * nsys));
  HIPCHK(ensure(w.info, sizeof(sscg_block_info) * nsys));
  HIPCHK(ensure(w.G, sizeof(double) * (size_t)BATCH_GSZ * nsys));
  HIPCHK(ensure(w.coef, sizeof(double) * (size_t)BATCH_CSZ * nsys));
  HIPCHK(ensure(w.hist, sizeof(BatchHist) * (size_t)cap * nsys));
  HIPCHK(ensure(w.blk_sys, sizeof(int32_t) * nblk));
  HIPCHK(ensure(w.chunks, sizeof(BatchChunk) * nchunks));
  HIPCHK(ensure(w.rpart, sizeof(double) * 2 * (size_t)nblk));
  HIPCHK(ensure(w.bpart, sizeof(double) * 2 * (size_t)nblk));
  HIPCHK(ensure(w.gpart, sizeof(double) * 2 * (size_t)npairs * nchunks));
  HIPCHK(ensure(w.active, sizeof(int32_t) * 4));
  HIPCHK(ensure(w.ablk, sizeof(int32_t) * nblk));
  HIPCHK(ensure(w.achk, sizeof(int32_t) * nchunks));
  HIPCHK(ensure(w.loff, sizeof(int32_t) * 2 * nsys));
  HIPCHK(ensure(w.perm, sizeof(int32_t) * (size_t)N));
  HIPCHK(ensure(w.T, sizeof(double2) * 2 * (size_t)N));
  HIPCHK(ensure(w.ilcnt, sizeof(unsigned long long) * 2 * nsys));
  unsigned long long* ilcnt = as<unsigned long long>(w.ilcnt);
  HIPCHK(ensure(w.inv, sizeof(int32_t) * (size_t)N));
  int32_t* perm = as<int32_t>(w.perm);
  int32_t* inv = as<int32_t>(w.inv);

  // ---- block-diagonal SELL-64 copy (structure checked per system)
  int32_t* width = as<int32_t>(w.width);
  int64_t* off = as<int64_t>(w.off);
  int32_t* flag = as<int32_t>(w.flag);
  HIPCHK(hipMemsetAsync(width, 0, sizeof(int32_t) * (nslices + 1), st));
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  for (int q = 0; q < nsys; ++q) {
    const sscg_csr& A = B->A[q];
    const int npad = (hs[q].blk1 - hs[q].blk0) * BATCH_ROWS;
    HIPCHK(launch_check_csr(A.rowptr, A.col, A.n, A.nnz, flag, st));
    HIPCHK(launch_row_order(A.rowptr, A.n, npad, hs[q].row0, perm, inv, st));
    HIPCHK(launch_sell_widths_perm(A.rowptr, perm + hs[q].row0, npad / SSCG_WAVE,
                                   width + hs[q].row0 / SSCG_WAVE, st));
  }
  HIPCHK(launch_scan_offsets(width, nslices, off, st));
  int64_t total = 0;
  int32_t bad = 0;
  HIPCHK(hipMemcpyAsync(&total, off + nslices, sizeof total, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad)
    return fail(ctx, SSCG_ERR_ARG,
                "batch: invalid CSR (rowptr not non-decreasing or a column index outside [0, n))");
  HIPCHK(hipMemsetAsync(ilcnt, 0, sizeof(unsigned long long) * 2 * nsys, st));
  HIPCHK(ensure(w.scol, sizeof(int32_t) * std::max<int64_t>(total, 1)));
  HIPCHK(ensure(w.sval, sizeof(double) * std::max<int64_t>(total, 1)));
  for (int q = 0; q < nsys; ++q) {
    const sscg_csr& A = B->A[q];
    const int npad = (hs[q].blk1 - hs[q].blk0) * BATCH_ROWS;
    HIPCHK(launch_sell_fill_perm(A.rowptr, A.col, A.val, perm + hs[q].row0, inv,
                                 npad / SSCG_WAVE, off + hs[q].row0 / SSCG_WAVE,
                                 width + hs[q].row0 / SSCG_WAVE, hs[q].row0, as<int32_t>(w.scol),
                                 as<double>(w.sval), ilcnt + 2 * q, st));
  }
  DevMat M;
  M.n = N;
  M.nslices = nslices;
  M.off = off;
  M.width = width;
  M.col = as<int32_t>(w.scol);
  M.val = as<double>(w.sval);

  // ---- vectors, tables, set-up residual r_1 = b - A x_1 (into P_0)
  BatchCfg c;
  memset(&c, 0, sizeof c);
  c.nsys = nsys;
  c.S = S;
  c.cap = cap;
  c.nblk = nblk;
  c.nchunks = nchunks;
  c.mode = o.mode;
  c.s_max = o.s_max;
  c.s0 = o.s0_bar > 0 ? o.s0_bar : o.s_max;
  c.f = o.f > 0 ? o.f : o.s_max;
  c.fixed_s = o.fixed_s;
  c.inner_check = o.inner_check;
  c.basis = o.basis;
  c.max_iters = o.max_iters;
  c.ld = N;
  c.c = o.c;
  c.Y = as<double>(w.Y);
  c.Y32 = vprec ? as<float>(w.Y32) : nullptr;
  c.vprec = vprec ? 1 : 0;
  c.x = as<double>(w.x);
  c.b = as<double>(w.b);
  c.sys = as<BatchSys>(w.sys);
  c.prm = as<sscg_block_params>(w.prm);
  c.info = as<sscg_block_info>(w.info);
  c.G = as<double>(w.G);
  c.coef = as<double>(w.coef);
  c.hist = as<BatchHist>(w.hist);
  c.blk_sys = as<int32_t>(w.blk_sys);
  c.chunks = as<BatchChunk>(w.chunks);
  c.rpart = as<double>(w.rpart);
  c.bpart = as<double>(w.bpart);
  c.gpart = as<double>(w.gpart);
  c.active = as<int32_t>(w.active);
  c.ablk = as<int32_t>(w.ablk);
  c.achk = as<int32_t>(w.achk);
  c.loff = as<int32_t>(w.loff);
  c.gblk = nblk;
  c.gchk = nchunks;
  c.T[0] = as<double2>(w.T);
  c.inv = as<int32_t>(w.inv);
  c.T[1] = c.T[0] + N;
  HIPCHK(hipMemsetAsync(c.Y, 0, sizeof(double) * (size_t)N * ncols, st));
  HIPCHK(hipMemsetAsync(c.x, 0, sizeof(double) * (size_t)N, st));
  HIPCHK(hipMemsetAsync(as<double>(w.b), 0, sizeof(double) * (size_t)N, st));
  for (int q = 0; q < nsys; ++q) {  // into the systems' row order
    const int npad = (hs[q].blk1 - hs[q].blk0) * BATCH_ROWS;
    HIPCHK(launch_gather_perm(B->x[q], perm + hs[q].row0, npad, c.x + hs[q].row0, st));
    HIPCHK(launch_gather_perm(B->b[q], perm + hs[q].row0, npad, as<double>(w.b) + hs[q].row0, st));
  }
  HIPCHK(hipMemcpyAsync(c.sys, hs.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, st));
  HIPCHK(launch_set_il(c.sys, ilcnt, 0, nsys, st));
  HIPCHK(hipMemcpyAsync(as<int32_t>(w.blk_sys), hblk.data(), sizeof(int32_t) * nblk,
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(as<BatchChunk>(w.chunks), hc.data(), sizeof(BatchChunk) * nchunks,
                        hipMemcpyHostToDevice, st));
  // 16-bit offsets and value tables, read by the systems all of whose slices fit them
  HIPCHK(ensure(w.scol16, sizeof(int16_t) * std::max<int64_t>(total, 1)));
  HIPCHK(ensure(w.svidx, std::max<int64_t>(total, 1)));
  HIPCHK(ensure(w.svtab, sizeof(double) * VTAB * (size_t)nslices));
  HIPCHK(ensure(w.vtcnt, sizeof(int32_t) * nsys));
  int32_t* vtcnt = as<int32_t>(w.vtcnt);
  HIPCHK(hipMemsetAsync(vtcnt, 0, sizeof(int32_t) * nsys, st));
  HIPCHK(launch_sell_forms_batch(M.col, M.val, off, width, 0, nslices, c.blk_sys,
                                 as<int16_t>(w.scol16), as<double>(w.svtab),
                                 as<uint8_t>(w.svidx), vtcnt, st));
  if ((ctx->forms & SSCG_FMT_COL16) && (ctx->forms & SSCG_FMT_VTAB))
    HIPCHK(launch_set_vt(c.sys, vtcnt, 0, nsys, st));
  M.col16 = as<int16_t>(w.scol16);
  M.vidx = as<uint8_t>(w.svidx);
  M.vtab = as<double>(w.svtab);
  // slice-diagonal form, read by the systems all of whose slices fit it
  HIPCHK(ensure(w.sd_nd, sizeof(int32_t) * (size_t)nslices));
  HIPCHK(ensure(w.sd_delta, sizeof(int32_t) * SD_DIAG * (size_t)nslices));
  HIPCHK(ensure(w.sd_tab, sizeof(double) * 4 * (size_t)nslices));
  HIPCHK(ensure(w.sd_code, sizeof(uint16_t) * (size_t)N));
  HIPCHK(ensure(w.sdcnt, sizeof(int32_t) * nsys));
  int32_t* sdcnt = as<int32_t>(w.sdcnt);
  HIPCHK(hipMemsetAsync(sdcnt, 0, sizeof(int32_t) * nsys, st));
  for (int q = 0; q < nsys && (ctx->forms & SSCG_FMT_SDIA); ++q) {
    const int npad = (hs[q].blk1 - hs[q].blk0) * BATCH_ROWS;
    HIPCHK(launch_sell_sdia_sys(B->A[q].rowptr, perm + hs[q].row0, hs[q].row0 / SSCG_WAVE,
                                npad / SSCG_WAVE, M.col, M.val, off, width,
                                as<int32_t>(w.sd_nd), as<int32_t>(w.sd_delta),
                                as<double>(w.sd_tab), as<uint16_t>(w.sd_code), sdcnt + q, st));
  }
  if (ctx->forms & SSCG_FMT_SDIA) HIPCHK(launch_set_sd(c.sys, sdcnt, 0, nsys, st));
  M.sd_nd = as<int32_t>(w.sd_nd);
  M.sd_delta = as<int32_t>(w.sd_delta);
  M.sd_tab = as<double>(w.sd_tab);
  M.sd_code = as<uint16_t>(w.sd_code);
  HIPCHK(hipMemsetAsync(c.hist, 0, sizeof(BatchHist) * (size_t)cap * nsys, st));
  int np = 0;
  HIPCHK(launch_residual(M, c.b, c.x, batch_col(c, 0), c.rpart, c.bpart, &np, st));
  if (np != nblk) return fail(ctx, SSCG_ERR_HIP, "batch: residual partials %d != blocks %d", np, nblk);
  HIPCHK(launch_pair(batch_col(c, 0), batch_col(c, c.S + 1), N, c.T[0], st));
  HIPCHK(launch_batch_init(c, st));
  HIPCHK(launch_batch_count(c, st));

  // ---- one outer block as a graph (grids in steps of 4), replayed; the
  // lists only shrink, so the grids picked after a check cover them until
  // the next one
  // launch shapes: fixed, a choice made before for this batch shape, or
  // timed after the first GROUP blocks
  for (int i = 0; i < 4; ++i) ctx->last_kappa_us[i] = NAN;
  for (int i = 0; i < 3; ++i) ctx->last_gram_us[i] = ctx->last_mpk_us[i] = NAN;
  bool tune = false;
  if (ctx->tune_mode == 0) {
    c.kbt = ctx->fixed_kbt;
    c.gw = ctx->fixed_gw;
    c.mch = ctx->fixed_mch;
  } else {
    c.kbt = 128;
    c.gw = 4;
    c.mch = 4;
    tune = true;
    for (const auto& t : ctx->tuned)
      if (t.rows == N && t.nsys == nsys && t.S == S) {
        c.kbt = t.kbt;
        c.gw = t.gw;
        c.mch = t.mch;
        tune = false;
      }
  }
  BlockGraphs gg;
  if ((rc = gg.capture(ctx, M, c, st))) return rc;
  // every replay adds >= 1 iteration to each unfinished system or finishes it
  const int64_t limit = (int64_t)o.max_iters + 2;
  int launches = 0;
  HIPCHK(hipMemcpyAsync(ctx->hactive, c.active, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  while (ctx->hactive[0] > 0 && launches < limit) {
    if (tune && launches >= GROUP) {
      tune = false;
      const size_t k = gg.pick_index(ctx->hactive[1], ctx->hactive[2]);
      if ((rc = tune_shapes(ctx, M, c, gg.gblk[k], gg.gchk[k], st))) return rc;
      ctx->tuned.push_back(sscg_ctx::TuneEntry{N, nsys, S, c.kbt, c.gw, c.mch});
      if ((rc = gg.capture(ctx, M, c, st))) return rc;
    }
    const int g = (int)std::min<int64_t>(GROUP, limit - launches);
    hipGraphExec_t ge = gg.pick(ctx->hactive[1], ctx->hactive[2]);
    for (int i = 0; i < g; ++i) HIPCHK(hipGraphLaunch(ge, st));
    launches += g;
    HIPCHK(hipMemcpyAsync(ctx->hactive, c.active, sizeof(int32_t) * 3, hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
  }
  ctx->last_kbt = c.kbt;
  ctx->last_gw = c.gw;
  ctx->last_mch = c.mch;

  // ---- results
  std::vector<BatchHist> hh((size_t)cap * nsys);
  HIPCHK(hipMemcpyAsync(hs.data(), c.sys, sizeof(BatchSys) * nsys, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hh.data(), c.hist, sizeof(BatchHist) * hh.size(), hipMemcpyDeviceToHost,
                        st));
  HIPCHK(hipStreamSynchronize(st));
  int worst = SSCG_OK;
  for (int q = 0; q < nsys; ++q) {
    const BatchSys& s = hs[q];
    if (s.b2 == 0.0)
      HIPCHK(launch_fill(B->x[q], s.n, 0.0, st));
    else
      HIPCHK(launch_scatter_perm(c.x + s.row0, perm + s.row0, (s.blk1 - s.blk0) * BATCH_ROWS,
                                 B->x[q], st));
    const int status = s.done ? s.status : SSCG_NOT_CONVERGED;
    worst = std::max(worst, status);
    if (!res) continue;
    if (res->status) res->status[q] = status;
    if (res->blocks) res->blocks[q] = s.blocks;
    if (res->iters) res->iters[q] = s.m;
    if (res->relres) res->relres[q] = s.relres;
    if (res->cap > 0)
      for (int k = 0; k < res->cap; ++k) {
        const bool in = k < cap && k < s.blocks + (s.status == SSCG_BREAKDOWN ? 1 : 0);
        const BatchHist* h = in ? &hh[(size_t)q * cap + k] : nullptr;
        if (res->s_k) res->s_k[(size_t)q * res->cap + k] = h ? h->s_k : 0;
        if (res->s_tilde) res->s_tilde[(size_t)q * res->cap + k] = h ? h->s_tilde : 0;
        if (res->relres_true) res->relres_true[(size_t)q * res->cap + k] = h ? h->relres_true : NAN;
        if (res->fp32) res->fp32[(size_t)q * res->cap + k] = h ? h->fp32 : 0;
      }
  }
  HIPCHK(hipStreamSynchronize(st));
  if (res) {
    res->graph_launches = launches;
    res->rows = N;
  }
  return worst;
}
