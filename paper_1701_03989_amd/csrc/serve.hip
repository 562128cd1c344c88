// sscg_server: continuous batching of independent solves on one GPU.
//
// The server owns fixed pools laid out like a batch (csrc/batch.hip): a row
// pool (basis columns, iterates, right-hand sides; allocated in units of one
// 1024-row Gram chunk) and an nnz pool (SELL-64 values and column indices).
// One outer block over the whole pool is captured once as a HIP graph; a pool
// block that belongs to no admitted system has system -1 and its workgroups
// return at once, so admitting and retiring systems only rewrites tables and
// pool regions, never the graph.  The row launches of the block stride over
// device-side lists of the blocks of the systems not done (k_batch_count, at
// the end of every block and after admissions), so their cost follows the
// admitted rows, not the pool's size or where in it the systems sit.  A step: wait for the previous block's
// system table, retire the systems it finished (copy x out, free their
// ranges), admit queued requests first come first served while a slot and
// room in both pools are free (matrix copy, set-up residual, table entries),
// then replay the graph for one more block.
//
// Up to PIPE replays are in flight: a step launches the next block before it
// has seen the system table of the last one, so the device never waits for
// the host's retire/admit work.  A replay of a system that is already done
// changes nothing (every batched kernel skips done systems), so a retirement
// seen one block late costs only that block's empty workgroups; a slot's
// table copies older than its admission are ignored.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "ctx.h"

using namespace sscg_host;

namespace {

constexpr int64_t ROW_UNIT = 1024;  // row allocation unit: one Gram chunk
constexpr int PIPE = 2;             // outer blocks in flight

// First-fit allocator of ranges in [0, size).
struct RangeAlloc {
  std::map<int64_t, int64_t> free_;  // start -> length
  void init(int64_t size) {
    free_.clear();
    if (size > 0) free_[0] = size;
  }
  int64_t alloc(int64_t len) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= len) {
        const int64_t s = it->first, l = it->second;
        free_.erase(it);
        if (l > len) free_[s + len] = l - len;
        return s;
      }
    return -1;
  }
  void release(int64_t s, int64_t len) {
    if (len <= 0) return;
    auto it = free_.emplace(s, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Req {
  sscg_csr A;
  const double* b;
  double* x;
  double tol, lmin, lmax;
  int state = 0;  // 0 queued, 1 running, 2 done
  int slot = -1;
  int64_t row0 = 0, npad = 0, nz0 = 0, nzlen = 0;
  int status = SSCG_OK, blocks = 0, iters = 0;
  double relres = NAN;
  std::vector<BatchHist> hist;  // per-block history, copied out at retirement
};

}  // namespace

struct sscg_server {
  sscg_ctx* ctx = nullptr;
  sscg_opts o;
  hipStream_t st = nullptr;
  int S = 0, slots = 0, cap = 0;
  int64_t rows = 0, nnz = 0;
  BatchWs w;
  BatchCfg c;
  DevMat M;
  BlockGraphs graphs;
  RangeAlloc ra, na;
  std::vector<int> free_slots;
  std::vector<int64_t> slot_req;
  std::deque<int64_t> queue;
  std::unordered_map<int64_t, Req> reqs;
  BatchSys* hsys = nullptr;  // pinned copies of the system table after replays k % PIPE
  int64_t* hscan = nullptr;  // pinned scratch
  hipEvent_t ev[PIPE] = {};     // after the system table copy of replay k % PIPE
  hipEvent_t ev_ret = nullptr;  // after the x copies of the last retirements
  int64_t launched = 0, seen = 0;  // replays launched; replays whose table was read
  std::vector<int64_t> adm_at;     // per slot: the first replay its request takes part in
  int64_t st_rows_active = 0;      // sum over replays of the admitted rows
  int64_t next_id = 1;
  int running = 0;
  std::vector<int32_t> hblk;  // staging for block -> system entries
  std::vector<BatchSys> hnew;
};

namespace {

void server_free(sscg_server* s) {
  if (!s) return;
  if (s->st) (void)hipStreamSynchronize(s->st);
  s->graphs.clear();
  BatchWs& w = s->w;
  Buf* bufs[] = {&w.width, &w.off,  &w.scol, &w.sval, &w.flag, &w.Y,       &w.x,
                 &w.b,     &w.sys,  &w.prm,  &w.info, &w.G,    &w.coef,    &w.hist,
                 &w.blk_sys, &w.chunks, &w.rpart, &w.bpart, &w.gpart, &w.active,
                 &w.perm,  &w.inv,  &w.T,    &w.ilcnt, &w.scol16, &w.svidx, &w.svtab,
                 &w.vtcnt, &w.sd_nd, &w.sd_delta, &w.sd_tab, &w.sd_code, &w.sdcnt,
                 &w.ablk,  &w.achk, &w.loff, &w.Y32};
  for (Buf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (s->hsys) (void)hipHostFree(s->hsys);
  if (s->hscan) (void)hipHostFree(s->hscan);
  for (hipEvent_t e : s->ev)
    if (e) (void)hipEventDestroy(e);
  if (s->ev_ret) (void)hipEventDestroy(s->ev_ret);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

// Copy x out and free the ranges of the system in `slot` (it is done; y: its
// table entry).
int retire(sscg_server* s, int slot, const BatchSys& y) {
  sscg_ctx* ctx = s->ctx;
  Req& r = s->reqs[s->slot_req[slot]];
  if (y.b2 == 0.0)
    HIPCHK(launch_fill(r.x, r.A.n, 0.0, s->st));
  else
    HIPCHK(launch_scatter_perm(s->c.x + r.row0, as<int32_t>(s->w.perm) + r.row0, (int)r.npad, r.x,
                               s->st));
  // its pool blocks belong to no system any more
  HIPCHK(hipMemsetAsync(as<int32_t>(s->w.blk_sys) + r.row0 / BATCH_ROWS, 0xFF,
                        sizeof(int32_t) * (r.npad / BATCH_ROWS), s->st));
  r.status = y.status;
  r.blocks = y.blocks;
  r.iters = y.m;
  r.relres = y.relres;
  r.state = 2;
  // the block history (complete once the step's closing synchronization is done)
  r.hist.resize(std::min(y.blocks, s->cap));
  if (!r.hist.empty())
    HIPCHK(hipMemcpyAsync(r.hist.data(), s->c.hist + (size_t)slot * s->cap,
                          sizeof(BatchHist) * r.hist.size(), hipMemcpyDeviceToHost, s->st));
  s->ra.release(r.row0 / ROW_UNIT, r.npad / ROW_UNIT);
  s->na.release(r.nz0, r.nzlen);
  s->slot_req[slot] = 0;
  s->free_slots.push_back(slot);
  --s->running;
  return SSCG_OK;
}

// Admit the request at the head of the queue if it fits: 1 admitted, 0 not
// now (no slot or no room), or a negative error.
int admit(sscg_server* s, int64_t id) {
  sscg_ctx* ctx = s->ctx;
  Req& r = s->reqs[id];
  if (s->free_slots.empty()) return 0;
  const int64_t u = s->ra.alloc(r.npad / ROW_UNIT);
  if (u < 0) return 0;
  const int64_t row0 = u * ROW_UNIT;
  const int ns = (int)(r.npad / SSCG_WAVE);
  const int64_t slice0 = row0 / SSCG_WAVE;
  BatchCfg& c = s->c;
  int32_t* width = as<int32_t>(s->w.width) + slice0;
  int64_t* off = as<int64_t>(s->w.off) + slice0;
  int32_t* flag = as<int32_t>(s->w.flag);
  // structure check and SELL widths, then the request's SELL size
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), s->st));
  int32_t* perm = as<int32_t>(s->w.perm);
  int32_t* inv = as<int32_t>(s->w.inv);
  HIPCHK(launch_check_csr(r.A.rowptr, r.A.col, r.A.n, r.A.nnz, flag, s->st));
  HIPCHK(launch_row_order(r.A.rowptr, r.A.n, (int)r.npad, (int)row0, perm, inv, s->st));
  HIPCHK(launch_sell_widths_perm(r.A.rowptr, perm + row0, ns, width, s->st));
  HIPCHK(launch_scan_offsets_base(width, ns, 0, off, as<int64_t>(s->w.flag) + 1, s->st));
  HIPCHK(hipMemcpyAsync(s->hscan, flag, sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  const int32_t bad = ((const int32_t*)s->hscan)[0];
  const int64_t total = s->hscan[1];
  if (bad) {  // malformed matrix: the request ends without running
    s->ra.release(u, r.npad / ROW_UNIT);
    r.state = 2;
    r.status = SSCG_ERR_ARG;
    return 1;
  }
  const int64_t nz0 = total > 0 ? s->na.alloc(total) : 0;
  if (nz0 < 0) {
    s->ra.release(u, r.npad / ROW_UNIT);
    return 0;
  }
  const int slot = s->free_slots.back();
  s->free_slots.pop_back();
  r.slot = slot;
  s->adm_at[slot] = s->launched;
  r.row0 = row0;
  r.nz0 = nz0;
  r.nzlen = total;
  // the request's SELL-64 rows at [nz0, nz0 + total) of the nnz pool
  HIPCHK(launch_scan_offsets_base(width, ns, nz0, off, as<int64_t>(s->w.flag) + 1, s->st));
  unsigned long long* ilcnt = as<unsigned long long>(s->w.ilcnt);
  HIPCHK(hipMemsetAsync(ilcnt + 2 * slot, 0, sizeof(unsigned long long) * 2, s->st));
  HIPCHK(launch_sell_fill_perm(r.A.rowptr, r.A.col, r.A.val, perm + row0, inv, ns, off, width,
                               (int)row0, as<int32_t>(s->w.scol), as<double>(s->w.sval),
                               ilcnt + 2 * slot, s->st));
  // iterate, right-hand side, basis columns of its rows
  const size_t vb = sizeof(double) * (size_t)r.npad;
  HIPCHK(hipMemsetAsync(c.x + row0, 0, vb, s->st));
  HIPCHK(hipMemsetAsync(as<double>(s->w.b) + row0, 0, vb, s->st));
  for (int col = 0; col < 2 * s->S + 1; ++col)
    HIPCHK(hipMemsetAsync(batch_col(c, col) + row0, 0, vb, s->st));
  HIPCHK(launch_gather_perm(r.x, perm + row0, (int)r.npad, c.x + row0, s->st));
  HIPCHK(launch_gather_perm(r.b, perm + row0, (int)r.npad, as<double>(s->w.b) + row0, s->st));
  // system table entry and block ownership
  const int blk0 = (int)(row0 / BATCH_ROWS), nb = (int)(r.npad / BATCH_ROWS);
  BatchSys& y = s->hnew[slot];
  memset(&y, 0, sizeof y);
  y.row0 = (int32_t)row0;
  y.n = r.A.n;
  y.blk0 = blk0;
  y.blk1 = blk0 + nb;
  y.ch0 = (int32_t)(row0 / ROW_UNIT);
  y.ch1 = (int32_t)((row0 + r.npad) / ROW_UNIT);
  y.tol = r.tol;
  y.lmin = r.lmin;
  y.lmax = r.lmax;
  HIPCHK(hipMemcpyAsync(c.sys + slot, &y, sizeof y, hipMemcpyHostToDevice, s->st));
  HIPCHK(launch_set_il(c.sys, ilcnt, slot, 1, s->st));
  s->hblk.assign(nb, slot);
  HIPCHK(hipMemcpyAsync(as<int32_t>(s->w.blk_sys) + blk0, s->hblk.data(), sizeof(int32_t) * nb,
                        hipMemcpyHostToDevice, s->st));
  // 16-bit offsets and value tables of its slices, read if all of them fit
  int32_t* vtcnt = as<int32_t>(s->w.vtcnt);
  HIPCHK(hipMemsetAsync(vtcnt + slot, 0, sizeof(int32_t), s->st));
  HIPCHK(launch_sell_forms_batch(as<int32_t>(s->w.scol), as<double>(s->w.sval),
                                 as<int64_t>(s->w.off), as<int32_t>(s->w.width), (int)slice0, ns,
                                 as<int32_t>(s->w.blk_sys), as<int16_t>(s->w.scol16),
                                 as<double>(s->w.svtab), as<uint8_t>(s->w.svidx), vtcnt, s->st));
  if ((ctx->forms & SSCG_FMT_COL16) && (ctx->forms & SSCG_FMT_VTAB))
    HIPCHK(launch_set_vt(c.sys, vtcnt, slot, 1, s->st));
  // its slice-diagonal form, read (in place of the above and the pairs) if
  // all of its slices fit
  int32_t* sdcnt = as<int32_t>(s->w.sdcnt);
  HIPCHK(hipMemsetAsync(sdcnt + slot, 0, sizeof(int32_t), s->st));
  if (ctx->forms & SSCG_FMT_SDIA) HIPCHK(launch_sell_sdia_sys(r.A.rowptr, perm + row0, (int)slice0, ns, as<int32_t>(s->w.scol),
                              as<double>(s->w.sval), as<int64_t>(s->w.off),
                              as<int32_t>(s->w.width), as<int32_t>(s->w.sd_nd),
                              as<int32_t>(s->w.sd_delta), as<double>(s->w.sd_tab),
                              as<uint16_t>(s->w.sd_code), sdcnt + slot, s->st));
  if (ctx->forms & SSCG_FMT_SDIA) HIPCHK(launch_set_sd(c.sys, sdcnt, slot, 1, s->st));
  HIPCHK(hipMemsetAsync(c.hist + (size_t)slot * s->cap, 0, sizeof(BatchHist) * s->cap, s->st));
  // r_1 = b - A x_1 into P_0 over the request's slices, then its set-up
  DevMat V = s->M;
  V.n = (int32_t)r.npad;
  V.nslices = ns;
  V.off = off;
  V.width = width;
  int np = 0;
  HIPCHK(launch_residual(V, as<double>(s->w.b) + row0, c.x, batch_col(c, 0) + row0,
                         c.rpart + (size_t)2 * blk0, c.bpart + (size_t)2 * blk0, &np, s->st));
  HIPCHK(launch_pair(batch_col(c, 0) + row0, batch_col(c, s->S + 1) + row0, r.npad,
                     c.T[0] + row0, s->st));
  HIPCHK(launch_batch_init_range(c, slot, 1, s->st));
  // staging buffers must outlive the copies
  HIPCHK(hipStreamSynchronize(s->st));
  s->slot_req[slot] = id;
  r.state = 1;
  ++s->running;
  return 1;
}

}  // namespace

extern "C" int sscg_server_create(sscg_ctx* ctx, const sscg_opts* opts, int64_t pool_rows,
                                  int64_t pool_nnz, int32_t slots, sscg_server** out) {
  if (!ctx || !out) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = validate_opts(ctx, opts))) return rc;
  if (opts->mode == SSCG_MODE_SCHEDULE || opts->equilibrate)
    return fail(ctx, SSCG_ERR_ARG, "server: MODE_SCHEDULE and equilibration are not supported");
  if (opts->basis == SSCG_BASIS_NEWTON || opts->c_mode != SSCG_C_CONST)
    return fail(ctx, SSCG_ERR_ARG, "server: the Newton basis and the theoretical c are not supported");
  if (opts->precision == SSCG_PREC_MIXED)
    return fail(ctx, SSCG_ERR_ARG, "server: SSCG_PREC_MIXED is not supported (SSCG_PREC_VARIABLE is)");
  if (slots < 1 || slots > 65536) return fail(ctx, SSCG_ERR_ARG, "server: bad slot count %d", slots);
  const int64_t rows = (std::max<int64_t>(pool_rows, 1) + ROW_UNIT - 1) / ROW_UNIT * ROW_UNIT;
  if (rows > INT32_MAX / 2) return fail(ctx, SSCG_ERR_ARG, "server: pool_rows too large");
  if (pool_nnz < 1) return fail(ctx, SSCG_ERR_ARG, "server: pool_nnz must be >= 1");
  sscg_server* s = new sscg_server;
  s->ctx = ctx;
  s->o = *opts;
  s->slots = slots;
  s->rows = rows;
  s->nnz = pool_nnz;
  s->S = opts->mode == SSCG_MODE_FIXED ? opts->fixed_s : opts->s_max;
  s->cap = std::min(opts->max_iters + 2, 4096);
  const int N = (int)rows, nslices = N / SSCG_WAVE, nblk = N / BATCH_ROWS;
  const int nchunks = (int)(rows / ROW_UNIT);
  const int ncols = 2 * s->S + 1, dmax = ncols, npairs = dmax * (dmax + 1) / 2;
  BatchWs& w = s->w;
  auto bad = [&](hipError_t e) {
    fail(ctx, e == hipErrorOutOfMemory ? SSCG_ERR_OOM : SSCG_ERR_HIP, "server: %s",
         hipGetErrorString(e));
    server_free(s);
    return e == hipErrorOutOfMemory ? SSCG_ERR_OOM : SSCG_ERR_HIP;
  };
  hipError_t e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
  for (hipEvent_t& v : s->ev)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&v, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_ret, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->hsys, sizeof(BatchSys) * slots * PIPE);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->hscan, sizeof(int64_t) * 4);
  const std::pair<Buf*, size_t> sizes[] = {
      {&w.width, sizeof(int32_t) * (nslices + 1)}, {&w.off, sizeof(int64_t) * (nslices + 1)},
      {&w.scol, sizeof(int32_t) * pool_nnz},       {&w.sval, sizeof(double) * pool_nnz},
      {&w.flag, sizeof(int64_t) * 4},              {&w.Y, sizeof(double) * (size_t)N * ncols},
      {&w.x, sizeof(double) * (size_t)N},          {&w.b, sizeof(double) * (size_t)N},
      {&w.sys, sizeof(BatchSys) * slots},          {&w.prm, sizeof(sscg_block_params) * slots},
      {&w.info, sizeof(sscg_block_info) * slots},  {&w.G, sizeof(double) * BATCH_GSZ * slots},
      {&w.coef, sizeof(double) * BATCH_CSZ * slots},
      {&w.hist, sizeof(BatchHist) * (size_t)s->cap * slots},
      {&w.blk_sys, sizeof(int32_t) * nblk},        {&w.chunks, sizeof(BatchChunk) * nchunks},
      {&w.rpart, sizeof(double) * 2 * (size_t)nblk}, {&w.bpart, sizeof(double) * 2 * (size_t)nblk},
      {&w.gpart, sizeof(double) * 2 * (size_t)npairs * nchunks},
      {&w.active, sizeof(int32_t) * 4},
      {&w.perm, sizeof(int32_t) * (size_t)N},      {&w.inv, sizeof(int32_t) * (size_t)N},
      {&w.T, sizeof(double2) * 2 * (size_t)N},
      {&w.ilcnt, sizeof(unsigned long long) * 2 * (size_t)slots},
      {&w.scol16, sizeof(int16_t) * pool_nnz},     {&w.svidx, sizeof(uint8_t) * pool_nnz},
      {&w.svtab, sizeof(double) * VTAB * (size_t)nslices},
      {&w.vtcnt, sizeof(int32_t) * (size_t)slots},
      {&w.sd_nd, sizeof(int32_t) * (size_t)nslices},
      {&w.sd_delta, sizeof(int32_t) * SD_DIAG * (size_t)nslices},
      {&w.sd_tab, sizeof(double) * 4 * (size_t)nslices},
      {&w.sd_code, sizeof(uint16_t) * (size_t)N},
      {&w.sdcnt, sizeof(int32_t) * (size_t)slots},
      {&w.ablk, sizeof(int32_t) * (size_t)nblk},   {&w.achk, sizeof(int32_t) * (size_t)nchunks},
      {&w.Y32, opts->precision == SSCG_PREC_VARIABLE ? sizeof(float) * (size_t)N * ncols : 0},
      {&w.loff, sizeof(int32_t) * 2 * (size_t)slots}};
  for (const auto& p : sizes)
    if (e == hipSuccess) e = ensure(*p.first, p.second);
  if (e != hipSuccess) return bad(e);
  // empty pool: every block owned by no system, every slot done
  std::vector<BatchSys> hs(slots);
  for (auto& y : hs) {
    memset(&y, 0, sizeof y);
    y.done = 1;
  }
  std::vector<BatchChunk> hc(nchunks);
  for (int k = 0; k < nchunks; ++k)
    hc[k] = BatchChunk{0, (int32_t)(k * ROW_UNIT), (int32_t)((k + 1) * ROW_UNIT), 0};
  e = hipMemsetAsync(w.width.p, 0, w.width.cap, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(w.off.p, 0, w.off.cap, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(w.blk_sys.p, 0xFF, sizeof(int32_t) * nblk, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(w.Y.p, 0, w.Y.cap, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(w.x.p, 0, w.x.cap, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(w.b.p, 0, w.b.cap, s->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(w.sys.p, hs.data(), sizeof(BatchSys) * slots, hipMemcpyHostToDevice, s->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(w.chunks.p, hc.data(), sizeof(BatchChunk) * nchunks, hipMemcpyHostToDevice,
                       s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return bad(e);
  BatchCfg& c = s->c;
  memset(&c, 0, sizeof c);
  c.nsys = slots;
  c.S = s->S;
  c.cap = s->cap;
  c.nblk = nblk;
  c.nchunks = nchunks;
  c.mode = opts->mode;
  c.s_max = opts->s_max;
  c.s0 = opts->s0_bar > 0 ? opts->s0_bar : opts->s_max;
  c.f = opts->f > 0 ? opts->f : opts->s_max;
  c.fixed_s = opts->fixed_s;
  c.inner_check = opts->inner_check;
  c.basis = opts->basis;
  c.max_iters = opts->max_iters;
  c.ld = N;
  c.c = opts->c;
  c.Y = as<double>(w.Y);
  c.Y32 = opts->precision == SSCG_PREC_VARIABLE ? as<float>(w.Y32) : nullptr;
  c.vprec = opts->precision == SSCG_PREC_VARIABLE ? 1 : 0;
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
  s->M.n = N;
  s->M.nslices = nslices;
  s->M.off = as<int64_t>(w.off);
  s->M.width = as<int32_t>(w.width);
  s->M.col = as<int32_t>(w.scol);
  s->M.val = as<double>(w.sval);
  s->M.col16 = as<int16_t>(w.scol16);
  s->M.vidx = as<uint8_t>(w.svidx);
  s->M.vtab = as<double>(w.svtab);
  s->M.sd_nd = as<int32_t>(w.sd_nd);
  s->M.sd_delta = as<int32_t>(w.sd_delta);
  s->M.sd_tab = as<double>(w.sd_tab);
  s->M.sd_code = as<uint16_t>(w.sd_code);
  // one outer block over the whole pool, captured once per grid size (empty
  // lists: no system yet)
  e = launch_batch_count(c, s->st);
  if (e != hipSuccess) return bad(e);
  if ((rc = s->graphs.capture(ctx, s->M, c, s->st))) {
    server_free(s);
    return rc;
  }
  s->ra.init(rows / ROW_UNIT);
  s->na.init(pool_nnz);
  s->slot_req.assign(slots, 0);
  s->adm_at.assign(slots, 0);
  s->hnew.resize(slots);
  for (int q = slots - 1; q >= 0; --q) s->free_slots.push_back(q);
  *out = s;
  return SSCG_OK;
}

extern "C" void sscg_server_destroy(sscg_server* s) {
  if (s) (void)hipSetDevice(s->ctx->device);
  server_free(s);
}

extern "C" int sscg_server_submit(sscg_server* s, const sscg_csr* A, const double* b, double* x,
                                  double tol, double lambda_min, double lambda_max, int64_t* id) {
  if (!s) return SSCG_ERR_ARG;
  sscg_ctx* ctx = s->ctx;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  if (!b || !x) return fail(ctx, SSCG_ERR_ARG, "server: b and x must not be NULL");
  const bool cheb = s->o.basis == SSCG_BASIS_CHEBYSHEV;
  if (cheb && !(lambda_max > lambda_min))
    return fail(ctx, SSCG_ERR_ARG, "server: need lambda_max > lambda_min");
  Req r;
  r.A = *A;
  r.b = b;
  r.x = x;
  r.tol = tol > 0.0 ? tol : s->o.tol;
  r.lmin = cheb ? lambda_min : 0.0;
  r.lmax = cheb ? lambda_max : 1.0;
  r.npad = ((int64_t)std::max(A->n, 1) + ROW_UNIT - 1) / ROW_UNIT * ROW_UNIT;
  if (r.npad > s->rows || A->nnz > s->nnz)
    return fail(ctx, SSCG_ERR_ARG, "server: a system of %d rows / %lld nonzeros never fits the pools",
                A->n, (long long)A->nnz);
  const int64_t k = s->next_id++;
  s->reqs.emplace(k, r);
  s->queue.push_back(k);
  if (id) *id = k;
  return SSCG_OK;
}

extern "C" int sscg_server_step(sscg_server* s, int32_t* running, int32_t* queued,
                                int32_t* retired) {
  if (!s) return SSCG_ERR_ARG;
  sscg_ctx* ctx = s->ctx;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  int nret = 0;
  // systems the oldest replay in flight finished (read once PIPE are in
  // flight, or when nothing runs any more)
  if (s->launched - s->seen == PIPE || (s->running == 0 && s->launched > s->seen)) {
    const int64_t k = s->seen++;
    HIPCHK(hipEventSynchronize(s->ev[k % PIPE]));
    const BatchSys* snap = s->hsys + (size_t)(k % PIPE) * s->slots;
    for (int q = 0; q < s->slots; ++q)
      if (s->slot_req[q] && k >= s->adm_at[q] && snap[q].done) {
        if ((rc = retire(s, q, snap[q]))) return rc;
        ++nret;
      }
    if (nret) HIPCHK(hipEventRecord(s->ev_ret, s->st));
  }
  // first come, first served while the head fits
  int nadm = 0;
  while (!s->queue.empty()) {
    rc = admit(s, s->queue.front());
    if (rc < 0) return rc;
    nadm += rc;
    if (rc == 0 && s->running == 0) {  // empty pools and still no room: it never fits
      Req& r = s->reqs[s->queue.front()];
      r.state = 2;
      r.status = SSCG_ERR_OOM;
      rc = 1;
    }
    if (rc == 0) break;
    s->queue.pop_front();
  }
  // systems finished at set-up (b = 0 or x_1 converged) are retired by the next step
  // the lists of the next block take in the admitted systems
  if (nadm) HIPCHK(launch_batch_count(s->c, s->st));
  if (s->running > 0) {
    int64_t act = 0;
    for (int q = 0; q < s->slots; ++q)
      if (s->slot_req[q]) act += s->reqs[s->slot_req[q]].npad;
    const int b = (int)(s->launched % PIPE);
    HIPCHK(hipGraphLaunch(s->graphs.pick(act / BATCH_ROWS, act / ROW_UNIT), s->st));
    HIPCHK(hipMemcpyAsync(s->hsys + (size_t)b * s->slots, s->c.sys, sizeof(BatchSys) * s->slots,
                          hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipEventRecord(s->ev[b], s->st));
    ++s->launched;
    s->st_rows_active += act;
  }
  // the retired systems' x copies are complete when this returns
  if (nret) HIPCHK(hipEventSynchronize(s->ev_ret));
  if (running) *running = s->running;
  if (queued) *queued = (int32_t)s->queue.size();
  if (retired) *retired = nret;
  return SSCG_OK;
}

extern "C" int sscg_server_poll(sscg_server* s, int64_t id, int32_t* state, int32_t* status,
                                int32_t* blocks, int32_t* iters, double* relres) {
  if (!s) return SSCG_ERR_ARG;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(s->ctx, SSCG_ERR_ARG, "server: unknown request %lld",
                                       (long long)id);
  const Req& r = it->second;
  if (state) *state = r.state;
  if (status) *status = r.status;
  if (blocks) *blocks = r.blocks;
  if (iters) *iters = r.iters;
  if (relres) *relres = r.relres;
  return SSCG_OK;
}

extern "C" int sscg_server_stats(sscg_server* s, int64_t* replays, int64_t* rows_active) {
  if (!s) return SSCG_ERR_ARG;
  if (replays) *replays = s->launched;
  if (rows_active) *rows_active = s->st_rows_active;
  return SSCG_OK;
}

extern "C" int sscg_server_history(sscg_server* s, int64_t id, int32_t cap, int32_t* s_k,
                                   int32_t* s_tilde, double* relres_true, int32_t* fp32,
                                   int32_t* rows) {
  if (!s) return SSCG_ERR_ARG;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(s->ctx, SSCG_ERR_ARG, "server: unknown request %lld",
                                       (long long)id);
  const Req& r = it->second;
  if (r.state != 2) return fail(s->ctx, SSCG_ERR_ARG, "server: request %lld is not done",
                                (long long)id);
  const int nrec = std::min<int>((int)r.hist.size(), std::max(cap, 0));
  for (int k = 0; k < nrec; ++k) {
    if (s_k) s_k[k] = r.hist[k].s_k;
    if (s_tilde) s_tilde[k] = r.hist[k].s_tilde;
    if (relres_true) relres_true[k] = r.hist[k].relres_true;
    if (fp32) fp32[k] = r.hist[k].fp32;
  }
  if (rows) *rows = nrec;
  return SSCG_OK;
}
