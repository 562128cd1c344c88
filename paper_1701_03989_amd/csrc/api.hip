// C ABI of libsscg: context, workspace, validation, the per-stage entry
// points and the helpers the solver shares with them.  All arithmetic of the
// method runs in the kernels of spmv.hip, dense.hip and small.hip; the host
// only sizes launches and moves a few scalars.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "ctx.h"

namespace {
thread_local std::string g_create_err;
}

namespace sscg_host {

hipError_t ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return hipSuccess;
  if (b.p) {
    // queued kernels may still use the old buffer
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    (void)hipFree(b.p);
  }
  b.p = nullptr;
  b.cap = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e == hipSuccess) b.cap = bytes;
  return e;
}

int fail(sscg_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

int set_device(sscg_ctx* ctx) {
  HIPCHK(hipSetDevice(ctx->device));
  return SSCG_OK;
}

hipError_t ev_begin(sscg_ctx* c, int fam, double bytes, hipStream_t st, size_t* slot) {
  *slot = NO_EVENT;
  if (!((c->timing >> fam) & 1u)) return hipSuccess;
  if (c->ev_used == c->ev.size()) {
    EvRec r;
    hipError_t e = hipEventCreate(&r.a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&r.b);
    if (e != hipSuccess) return e;
    c->ev.push_back(r);
  }
  *slot = c->ev_used++;
  EvRec& r = c->ev[*slot];
  r.fam = fam;
  r.bytes = bytes;
  r.nsub = 0;
  r.ran0 = 0;
  return hipEventRecord(r.a, st);
}

hipError_t ev_end(sscg_ctx* c, size_t slot, hipStream_t st) {
  if (slot == NO_EVENT) return hipSuccess;
  return hipEventRecord(c->ev[slot].b, st);
}

int* ev_sub(sscg_ctx* c, size_t slot, double bytes) {
  if (slot == NO_EVENT || !c->ran.p) return nullptr;
  EvRec& r = c->ev[slot];
  // a group's flags are consecutive: taken when its first launch registers
  if (r.nsub == 0) r.ran0 = c->ran_used;
  if (r.nsub >= SSCG_S_LIMIT || r.ran0 + r.nsub >= RAN_CAP || r.ran0 + r.nsub != c->ran_used)
    return nullptr;  // out of flags: the launch is timed without one
  r.sbytes[r.nsub] = bytes;
  r.nsub += 1;
  return as<int>(c->ran) + c->ran_used++;
}

int* ev_ran(sscg_ctx* c, size_t slot) {
  if (slot == NO_EVENT) return nullptr;
  int* f = ev_sub(c, slot, c->ev[slot].bytes);
  if (f) c->ev[slot].bytes = 0.0;  // now carried by the gated launch
  return f;
}

// Forget recorded intervals without counting them; their ran flags are
// cleared (on the stream, ahead of any later launch that may set them).
hipError_t ev_drop(sscg_ctx* c) {
  hipError_t e = hipSuccess;
  const size_t nr = std::min(c->ran_used, RAN_CAP);
  if (c->ran.p && nr) e = hipMemsetAsync(c->ran.p, 0, sizeof(int) * nr, c->stream);
  c->ev_used = 0;
  c->ran_used = 0;
  return e;
}

// Accumulate the recorded intervals (the streams must have passed them).
// Gated launches that stood down are left out: they moved none of their
// bytes; an interval none of whose launches ran is left out entirely.
hipError_t ev_collect(sscg_ctx* c) {
  const size_t nr = std::min(c->ran_used, RAN_CAP);
  if (c->ran.p && nr) {
    c->hran.assign(nr, 0);
    hipError_t e = hipMemcpy(c->hran.data(), c->ran.p, sizeof(int) * nr, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(c->ran.p, 0, sizeof(int) * nr);
    if (e != hipSuccess) return e;
  }
  for (size_t i = 0; i < c->ev_used; ++i) {
    const EvRec& r = c->ev[i];
    int launches = r.nsub == 0 ? 1 : 0;
    double bytes = r.bytes;
    for (int k = 0; k < r.nsub; ++k)
      if (c->hran[r.ran0 + k]) {
        launches += 1;
        bytes += r.sbytes[k];
      }
    if (launches == 0) continue;
    float t = 0.f;
    hipError_t e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return e;
    c->launches[r.fam] += launches;
    c->ms[r.fam] += t;
    c->bytes[r.fam] += bytes;
  }
  c->ev_used = 0;
  c->ran_used = 0;
  return hipSuccess;
}

int check_csr(sscg_ctx* ctx, const sscg_csr* A) {
  if (!A) return fail(ctx, SSCG_ERR_ARG, "A is NULL");
  if (A->n < 1 || A->n > INT32_MAX - 4095)
    return fail(ctx, SSCG_ERR_ARG, "n = %d outside [1, 2^31 - 4096]", A->n);
  if (A->nnz < 0 || A->nnz > INT32_MAX)
    return fail(ctx, SSCG_ERR_ARG, "nnz = %lld outside [0, 2^31) (rowptr is 32-bit)",
                (long long)A->nnz);
  if (!A->rowptr || (A->nnz > 0 && (!A->col || !A->val)))
    return fail(ctx, SSCG_ERR_ARG, "CSR arrays must not be NULL");
  int32_t ends[2] = {-1, -1};
  HIPCHK(hipMemcpyAsync(&ends[0], A->rowptr, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(&ends[1], A->rowptr + A->n, sizeof(int32_t), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ends[0] != 0 || ends[1] != A->nnz)
    return fail(ctx, SSCG_ERR_ARG, "rowptr[0] = %d, rowptr[n] = %d (nnz = %lld)", ends[0], ends[1],
                (long long)A->nnz);
  return SSCG_OK;
}

// CSR -> SELL-64 copy (optionally equilibrated), after a structural check.
int build_mat(sscg_ctx* ctx, const sscg_csr* A, int equilibrate, DevMat* M) {
  const int n = A->n;
  const int nslices = (n + SSCG_WAVE - 1) / SSCG_WAVE;
  HIPCHK(ensure(ctx->width, sizeof(int32_t) * (nslices + 8)));
  HIPCHK(ensure(ctx->off, sizeof(int64_t) * (nslices + 1)));
  // every later kernel gathers through col[]
  int32_t* flag = as<int32_t>(ctx->width) + nslices;
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
  HIPCHK(launch_check_csr(A->rowptr, A->col, n, A->nnz, flag, ctx->stream));
  int32_t bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (bad)
    return fail(ctx, SSCG_ERR_ARG,
                "invalid CSR: rowptr not non-decreasing or a column index outside [0, n)");
  HIPCHK(launch_sell_widths(A->rowptr, n, as<int32_t>(ctx->width), ctx->stream));
  HIPCHK(launch_scan_offsets(as<int32_t>(ctx->width), nslices, as<int64_t>(ctx->off), ctx->stream));
  int64_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, as<int64_t>(ctx->off) + nslices, sizeof total,
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(ensure(ctx->scol, sizeof(int32_t) * total));
  HIPCHK(ensure(ctx->sval, sizeof(double) * total));
  ctx->sell_total = total;
  const double* scale = nullptr;
  if (equilibrate) {
    HIPCHK(ensure(ctx->scale, sizeof(double) * n));
    HIPCHK(launch_row_scale(A->rowptr, A->val, n, as<double>(ctx->scale), ctx->stream));
    scale = as<double>(ctx->scale);
  }
  HIPCHK(launch_sell_fill(A->rowptr, A->col, A->val, n, scale, as<int64_t>(ctx->off),
                          as<int32_t>(ctx->width),
                          as<int32_t>(ctx->scol), as<double>(ctx->sval), ctx->stream));
  // 16-bit column offsets for the matrix-powers pass when every one fits
  HIPCHK(ensure(ctx->scol16, sizeof(int16_t) * total));
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
  HIPCHK(launch_sell_compact(as<int32_t>(ctx->scol), n, as<int64_t>(ctx->off),
                             as<int32_t>(ctx->width), as<int16_t>(ctx->scol16), flag,
                             ctx->stream));
  // value indices when every slice holds few distinct values (stencils)
  HIPCHK(ensure(ctx->svidx, std::max<int64_t>(total, 1)));
  HIPCHK(ensure(ctx->svtab, sizeof(double) * VTAB * std::max(nslices, 1)));
  HIPCHK(hipMemsetAsync(flag + 1, 0, sizeof(int32_t), ctx->stream));
  HIPCHK(launch_sell_vidx(as<double>(ctx->sval), as<int64_t>(ctx->off), as<int32_t>(ctx->width),
                          nslices, as<double>(ctx->svtab), as<uint8_t>(ctx->svidx), flag + 1,
                          ctx->stream));
  // slice-diagonal form when every slice has few distances and values (stencils)
  HIPCHK(ensure(ctx->sd_nd, sizeof(int32_t) * std::max(nslices, 1)));
  HIPCHK(ensure(ctx->sd_delta, sizeof(int32_t) * SD_DIAG * std::max(nslices, 1)));
  HIPCHK(ensure(ctx->sd_tab, sizeof(double) * 4 * std::max(nslices, 1)));
  HIPCHK(ensure(ctx->sd_code, sizeof(uint16_t) * SSCG_WAVE * std::max(nslices, 1)));
  HIPCHK(hipMemsetAsync(flag + 2, 0, sizeof(int32_t), ctx->stream));
  HIPCHK(launch_sell_sdia(A->rowptr, n, as<int32_t>(ctx->scol), as<double>(ctx->sval),
                          as<int64_t>(ctx->off), as<int32_t>(ctx->width), nslices,
                          as<int32_t>(ctx->sd_nd), as<int32_t>(ctx->sd_delta),
                          as<double>(ctx->sd_tab), as<uint16_t>(ctx->sd_code), flag + 2,
                          ctx->stream));
  // whether consecutive slices share their slice-diagonal tables
  HIPCHK(hipMemsetAsync(flag + 3, 0, sizeof(int32_t), ctx->stream));
  HIPCHK(launch_sd_pairs(as<int32_t>(ctx->sd_nd), as<int32_t>(ctx->sd_delta),
                         as<double>(ctx->sd_tab), nslices, flag + 3, ctx->stream));
  // whether each distance of a slice has one value
  HIPCHK(ensure(ctx->sd_vk, sizeof(uint32_t) * std::max(nslices, 1)));
  HIPCHK(hipMemsetAsync(flag + 4, 0, 2 * sizeof(int32_t), ctx->stream));
  HIPCHK(launch_sd_values(as<int32_t>(ctx->sd_nd), as<uint16_t>(ctx->sd_code), nslices,
                          as<uint32_t>(ctx->sd_vk), flag + 4, ctx->stream));
  int32_t fl[6] = {1, 1, 1, 1, 1, 1};
  HIPCHK(hipMemcpyAsync(fl, flag, sizeof fl, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // forms the caller allowed (sscg_set_forms); tables only with 16-bit offsets
  const int32_t wide = fl[0] || !(ctx->forms & SSCG_FMT_COL16);
  const int32_t many = fl[1] || !(ctx->forms & SSCG_FMT_VTAB);
  const int32_t nosd = fl[2] || !(ctx->forms & SSCG_FMT_SDIA);
  M->n = n;
  M->nslices = nslices;
  M->off = as<int64_t>(ctx->off);
  M->width = as<int32_t>(ctx->width);
  M->col = as<int32_t>(ctx->scol);
  M->val = as<double>(ctx->sval);
  M->col16 = wide ? nullptr : as<int16_t>(ctx->scol16);
  M->vidx = many ? nullptr : as<uint8_t>(ctx->svidx);
  M->vtab = many ? nullptr : as<double>(ctx->svtab);
  M->sd_nd = nosd ? nullptr : as<int32_t>(ctx->sd_nd);
  M->sd_delta = nosd ? nullptr : as<int32_t>(ctx->sd_delta);
  M->sd_tab = nosd ? nullptr : as<double>(ctx->sd_tab);
  M->sd_code = nosd ? nullptr : as<uint16_t>(ctx->sd_code);
  M->sd_vk = !nosd && fl[4] == 0 && (ctx->forms & SSCG_FMT_SDVAL) ? as<uint32_t>(ctx->sd_vk)
                                                                   : nullptr;
  // pairs of slices also agree on the per-distance values when those are used
  M->sd_pair = !nosd && fl[3] == 0 && (!M->sd_vk || fl[5] == 0) &&
                       (ctx->forms & SSCG_FMT_SDPAIR) && n >= 2
                   ? 1
                   : 0;
  ctx->mat_bytes = mpk_matrix_bytes(*M, total);
  return SSCG_OK;
}

double mpk_matrix_bytes(const DevMat& M, int64_t stored) {
  // slice-diagonal: a 16-bit code word per row, per slice its count,
  // distances and 4-entry table
  if (M.sd_code) return 2.0 * SSCG_WAVE * M.nslices + (4.0 + 4.0 * SD_DIAG + 32.0) * M.nslices;
  // the other forms: value tables only with 16-bit offsets
  const bool c16 = M.col16 != nullptr, vt = c16 && M.vidx != nullptr;
  const double per_entry = vt ? 1.0 + 2.0 : (c16 ? 8.0 + 2.0 : 8.0 + 4.0);
  const double per_slice = 8.0 + 4.0 + (vt ? 8.0 * VTAB : 0.0);  // off, width, table
  return per_entry * (double)stored + per_slice * (double)M.nslices;
}

ColPtr colptr_of(const BasisCols& bc, int s, int first) {
  (void)first;  // block 0 has d = s + 1 columns: the R columns are never addressed
  return ColPtr{bc.p0, bc.r0, bc.Y, bc.ldy, bc.rcol, s};
}

int mpk_passes(sscg_ctx* ctx, const DevMat& M, int s, int first, BasisPrm bp, const BasisCols& bc,
               double mat_bytes, const int* stop, const MpkResidual& res, const ResCheck& chk) {
  const int n = M.n;
  // the s passes run back to back: one timed interval, a ran flag per pass
  // (two intervals around the residual test when it runs between them)
  size_t slot = 0;
  HIPCHK(ev_begin(ctx, 0, 0.0, ctx->stream, &slot));
  for (int j = 1; j <= s; ++j) {
    if (j == 2 && res.x && chk.b2) {
      HIPCHK(ev_end(ctx, slot, ctx->stream));
      HIPCHK(launch_res_finalize(res.part, chk.nparts, chk.b2, chk.tol, chk.info, chk.stop,
                                 ctx->stream));
      HIPCHK(ev_begin(ctx, 0, 0.0, ctx->stream, &slot));
    }
    MpkSeq sp{bc.P(j - 1), j >= 2 ? bc.P(j - 2) : nullptr, bc.P(j)};
    MpkSeq sr{nullptr, nullptr, nullptr};
    int nrhs = 1;
    if (!first && j <= s - 1) {
      sr = MpkSeq{bc.R(j - 1), j >= 2 ? bc.R(j - 2) : nullptr, bc.R(j)};
      nrhs = 2;
    }
    const bool withres = j == 1 && res.x;
    double vec = 2.0 * nrhs + ((bp.cheb && j >= 2) ? nrhs : 0) + (withres ? 2 : 0);
    double bytes = mat_bytes + 8.0 * n * vec;
    HIPCHK(launch_mpk_pass(M, j, bp, nrhs, sp, sr, Gate{stop, ev_sub(ctx, slot, bytes)},
                           withres ? res : MpkResidual{}, ctx->stream));
  }
  HIPCHK(ev_end(ctx, slot, ctx->stream));
  if (s == 1 && res.x && chk.b2)  // no second pass to place the test before
    HIPCHK(launch_res_finalize(res.part, chk.nparts, chk.b2, chk.tol, chk.info, chk.stop,
                               ctx->stream));
  return SSCG_OK;
}

int gram_into(sscg_ctx* ctx, const ColPtr& cols, int n, int d, double* G, const int* stop) {
  const int ng = gram_ngroups(n);
  HIPCHK(ensure(ctx->part, sizeof(double) * (size_t)ng * (d * (d + 1) / 2)));
  size_t slot = 0;
  HIPCHK(ev_begin(ctx, 1, 8.0 * n * d, ctx->stream, &slot));
  HIPCHK(launch_gram(cols, n, d, as<double>(ctx->part), Gate{stop, ev_ran(ctx, slot)},
                     ctx->stream));
  HIPCHK(ev_end(ctx, slot, ctx->stream));
  HIPCHK(launch_gram_finalize(as<double>(ctx->part), ng, d, G, stop, ctx->stream));
  return SSCG_OK;
}

int ensure_parts(sscg_ctx* ctx, int n, int count) {
  int np = residual_nparts(n);
  int np2 = (n + 255) / 256;
  if (np2 > np) np = np2;
  HIPCHK(ensure(ctx->part, sizeof(double) * 2 * (size_t)np * count));
  return SSCG_OK;
}

// `steps` Lanczos steps on M from the SplitMix64 start vector: alpha_j and
// beta_j stay in ctx->lzab (al, be); *k = steps, or fewer if some beta_j = 0
// (invariant subspace: the run ends there).
int lanczos_dev(sscg_ctx* ctx, const DevMat& M, int steps, uint64_t seed, int* k) {
  const int n = M.n;
  int rc = ensure_parts(ctx, n, 1);
  if (rc) return rc;
  HIPCHK(ensure(ctx->lz, sizeof(double) * 3 * (size_t)n));
  HIPCHK(ensure(ctx->lzab, sizeof(double) * (2 * 64 + 8 + SSCG_S_LIMIT)));
  double* v = as<double>(ctx->lz);
  double* vp = v + n;
  double* w = vp + n;
  double* al = as<double>(ctx->lzab);
  double* be = al + 64;
  double* sc = be + 64;  // [0]: ||u||
  double* part = as<double>(ctx->part);
  int np = 0;
  hipStream_t st = ctx->stream;
  HIPCHK(launch_splitmix_vec(w, n, seed, st));
  HIPCHK(launch_dot_parts(w, w, n, part, &np, st));
  HIPCHK(launch_finalize_sqrt(part, np, sc, st));
  HIPCHK(launch_div_vec(w, sc, n, v, st));
  bool have_prev = false;
  for (int j = 0; j < steps; ++j) {
    HIPCHK(launch_lanczos_step(M, v, have_prev ? vp : nullptr, have_prev ? be + j - 1 : nullptr, w,
                               part, &np, st));
    HIPCHK(launch_finalize(part, np, 1, al + j, st));
    HIPCHK(launch_axpy_dot(w, v, al + j, part, &np, n, st));
    HIPCHK(launch_finalize_sqrt(part, np, be + j, st));
    if (j < steps - 1) {
      HIPCHK(launch_div_vec(w, be + j, n, vp, st));  // vp <- w / beta (the new v)
      double* t = v;
      v = vp;
      vp = t;
      have_prev = true;
    }
  }
  double hb[64];
  HIPCHK(hipMemcpyAsync(hb, be, sizeof(double) * steps, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *k = steps;
  for (int j = 0; j < steps - 1; ++j)
    if (hb[j] == 0.0) {
      *k = j + 1;
      break;
    }
  return SSCG_OK;
}

int spectral_bounds_dev(sscg_ctx* ctx, const DevMat& M, int steps, uint64_t seed, double* lmin,
                        double* lmax) {
  if (steps < 1) steps = 1;
  if (steps > 2 * SSCG_S_LIMIT + 1) steps = 2 * SSCG_S_LIMIT + 1;
  int k = 0;
  int rc = lanczos_dev(ctx, M, steps, seed, &k);
  if (rc) return rc;
  double* al = as<double>(ctx->lzab);
  double* be = al + 64;
  double* sc = be + 64;  // [1]: Gershgorin, [2], [3]: Ritz extremes
  double* part = as<double>(ctx->part);
  int np = 0;
  hipStream_t st = ctx->stream;
  HIPCHK(launch_gershgorin(M, part, &np, st));
  HIPCHK(launch_max_finalize(part, np, sc + 1, st));
  HIPCHK(launch_tridiag_eig(al, be, k, sc + 2, sc + 3, st));
  double out[4];
  HIPCHK(hipMemcpyAsync(out, sc, sizeof out, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *lmax = out[1];
  *lmin = out[2];
  return SSCG_OK;
}

int newton_shifts_dev(sscg_ctx* ctx, const DevMat& M, int m, uint64_t seed, double* shifts) {
  int k = 0;
  int rc = lanczos_dev(ctx, M, m, seed, &k);
  if (rc) return rc;
  double* al = as<double>(ctx->lzab);
  double* be = al + 64;
  double* sc = be + 64 + 8;  // m shifts
  HIPCHK(launch_newton_shifts(al, be, k, m, sc, ctx->stream));
  HIPCHK(hipMemcpyAsync(shifts, sc, sizeof(double) * m, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < m; ++i)
    if (!isfinite(shifts[i])) return fail(ctx, SSCG_ERR_HIP, "Newton shift estimate failed");
  return SSCG_OK;
}

int max_row_nnz_dev(sscg_ctx* ctx, const DevMat& M, int* n_a) {
  int32_t* out = as<int32_t>(ctx->width) + M.nslices + 1;
  HIPCHK(launch_max_width(M.width, M.nslices, out, ctx->stream));
  HIPCHK(hipMemcpyAsync(n_a, out, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return SSCG_OK;
}

int method_setup(sscg_ctx* ctx, const DevMat& M, const sscg_opts& o, MethodSetup* ms) {
  int rc = 0;
  ms->lmin = o.lambda_min;
  ms->lmax = o.lambda_max;
  ms->bp = make_basis(o.basis, 0.0, 1.0);
  for (int i = 0; i < SSCG_S_LIMIT; ++i) ms->shifts[i] = 0.0;
  if (o.basis == SSCG_BASIS_CHEBYSHEV) {
    if (isnan(ms->lmin)) {
      if ((rc = spectral_bounds_dev(ctx, M, o.lanczos_steps, o.lanczos_seed, &ms->lmin,
                                    &ms->lmax)))
        return rc;
      if (!(ms->lmax > ms->lmin)) return fail(ctx, SSCG_ERR_HIP, "spectral estimate failed");
    }
    ms->bp = make_basis(o.basis, ms->lmin, ms->lmax);
  }
  if (o.basis == SSCG_BASIS_NEWTON) {
    if (o.shifts) {
      for (int i = 0; i < o.s_max; ++i) ms->shifts[i] = o.shifts[i];
    } else if ((rc = newton_shifts_dev(ctx, M, o.s_max, o.lanczos_seed, ms->shifts))) {
      return rc;
    }
    ms->bp = make_basis(o.basis, 0.0, 1.0, ms->shifts);
  }
  ms->c_mode = o.c_mode;
  ms->n_a = 0;
  ms->s_max = o.s_max;
  ms->kappa_a = o.kappa_a;
  ms->norm_a = o.norm_a;
  if (o.c_mode == SSCG_C_THEORY) {
    if ((rc = max_row_nnz_dev(ctx, M, &ms->n_a))) return rc;
    if (isnan(ms->kappa_a) || isnan(ms->norm_a)) {
      double lo = ms->lmin, hi = ms->lmax;
      if (isnan(lo) &&
          (rc = spectral_bounds_dev(ctx, M, o.lanczos_steps, o.lanczos_seed, &lo, &hi)))
        return rc;
      if (!(lo > 0.0 && hi >= lo)) return fail(ctx, SSCG_ERR_HIP, "spectral estimate failed");
      if (isnan(ms->kappa_a)) ms->kappa_a = hi / lo;
      if (isnan(ms->norm_a)) ms->norm_a = hi;
    }
  }
  return SSCG_OK;
}

int validate_opts(sscg_ctx* ctx, const sscg_opts* o) {
  if (!o) return fail(ctx, SSCG_ERR_ARG, "opts is NULL");
  if (o->mode < 0 || o->mode > 2) return fail(ctx, SSCG_ERR_ARG, "bad mode %d", o->mode);
  if (o->basis < 0 || o->basis > 2) return fail(ctx, SSCG_ERR_ARG, "bad basis %d", o->basis);
  if (!(o->tol > 0.0)) return fail(ctx, SSCG_ERR_ARG, "tol must be > 0");
  if (o->s_max < 1 || o->s_max > SSCG_S_LIMIT)
    return fail(ctx, SSCG_ERR_ARG, "s_max = %d outside [1, %d]", o->s_max, SSCG_S_LIMIT);
  if (o->s0_bar < 0 || o->s0_bar > o->s_max) return fail(ctx, SSCG_ERR_ARG, "bad s0_bar");
  if (o->f < 0) return fail(ctx, SSCG_ERR_ARG, "bad f");
  if (o->mode == SSCG_MODE_FIXED && (o->fixed_s < 1 || o->fixed_s > o->s_max))
    return fail(ctx, SSCG_ERR_ARG, "fixed_s = %d outside [1, s_max]", o->fixed_s);
  if (o->mode == SSCG_MODE_SCHEDULE) {
    if (!o->schedule || o->schedule_len < 1) return fail(ctx, SSCG_ERR_ARG, "empty schedule");
    for (int i = 0; i < o->schedule_len; ++i)
      if (o->schedule[i] < 1 || o->schedule[i] > o->s_max)
        return fail(ctx, SSCG_ERR_ARG, "schedule[%d] = %d outside [1, s_max]", i, o->schedule[i]);
  }
  if (!(o->c > 0.0)) return fail(ctx, SSCG_ERR_ARG, "c must be > 0");
  if (o->basis == SSCG_BASIS_CHEBYSHEV) {
    bool nan_lo = isnan(o->lambda_min), nan_hi = isnan(o->lambda_max);
    if (nan_lo != nan_hi) return fail(ctx, SSCG_ERR_ARG, "give both Chebyshev bounds or neither");
    if (!nan_lo && !(o->lambda_max > o->lambda_min))
      return fail(ctx, SSCG_ERR_ARG, "need lambda_max > lambda_min");
  }
  if (o->max_iters < 1) return fail(ctx, SSCG_ERR_ARG, "max_iters must be >= 1");
  if (o->basis == SSCG_BASIS_NEWTON && o->shifts)
    for (int i = 0; i < o->s_max; ++i)
      if (!isfinite(o->shifts[i])) return fail(ctx, SSCG_ERR_ARG, "shifts[%d] not finite", i);
  if (o->c_mode < 0 || o->c_mode > 1) return fail(ctx, SSCG_ERR_ARG, "bad c_mode %d", o->c_mode);
  if (o->c_mode == SSCG_C_THEORY &&
      ((!isnan(o->kappa_a) && !(o->kappa_a >= 1.0 && isfinite(o->kappa_a))) ||
       (!isnan(o->norm_a) && !(o->norm_a > 0.0 && isfinite(o->norm_a)))))
    return fail(ctx, SSCG_ERR_ARG, "theoretical c needs kappa_a >= 1 and norm_a > 0 (or NaN)");
  if (o->precision < 0 || o->precision > 2)
    return fail(ctx, SSCG_ERR_ARG, "bad precision %d", o->precision);
  if (o->precision == SSCG_PREC_VARIABLE &&
      (o->mode != SSCG_MODE_ADAPTIVE || o->c_mode != SSCG_C_CONST))
    return fail(ctx, SSCG_ERR_ARG, "variable precision needs the adaptive mode and a constant c");
  if (o->precision == SSCG_PREC_MIXED && (o->max_outer < 1 || !(o->inner_tol > 0.0) ||
                                           !(o->inner_tol < 1.0)))
    return fail(ctx, SSCG_ERR_ARG, "mixed precision needs max_outer >= 1 and 0 < inner_tol < 1");
  return SSCG_OK;
}

}  // namespace sscg_host

using namespace sscg_host;

// ====================================================================== ABI

extern "C" {

void sscg_opts_default(sscg_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->mode = SSCG_MODE_ADAPTIVE;
  o->basis = SSCG_BASIS_MONOMIAL;
  o->tol = 1e-10;
  o->s_max = 8;
  o->s0_bar = 0;
  o->f = 0;
  o->fixed_s = 4;
  o->c = 1.0;
  o->lambda_min = NAN;
  o->lambda_max = NAN;
  o->lanczos_steps = 30;
  o->lanczos_seed = 0;
  o->equilibrate = 0;
  o->inner_check = 1;
  o->max_iters = 100000;
  o->c_mode = SSCG_C_CONST;
  o->kappa_a = NAN;
  o->norm_a = NAN;
  o->shifts = nullptr;
  o->precision = SSCG_PREC_FP64;
  o->max_outer = 30;
  o->inner_tol = 1e-5;
}

int sscg_create(sscg_ctx** out, int device, void* stream) {
  if (!out) {
    g_create_err = "out is NULL";
    return SSCG_ERR_ARG;
  }
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev) {
    g_create_err = "no HIP device " + std::to_string(device);
    return SSCG_ERR_ARG;
  }
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    g_create_err = hipGetErrorString(e);
    return SSCG_ERR_HIP;
  }
  sscg_ctx* c = new sscg_ctx;
  c->device = device;
  c->stream = (hipStream_t)stream;
  bool ok = hipHostMalloc((void**)&c->hinfo, sizeof(sscg_block_info) * RING) == hipSuccess &&
            hipHostMalloc((void**)&c->hscal, sizeof(double) * 16) == hipSuccess &&
            hipHostMalloc((void**)&c->hactive, sizeof(int32_t) * 4) == hipSuccess &&
            hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < RING; ++i)
    ok = hipEventCreateWithFlags(&c->evI[i], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->evV[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    g_create_err = "context allocation failed";
    sscg_destroy(c);
    return SSCG_ERR_OOM;
  }
  c->events_made = true;
  if (scratch_setup(c) != SSCG_OK) {
    g_create_err = c->err;
    sscg_destroy(c);
    return SSCG_ERR_HIP;
  }
  *out = c;
  return SSCG_OK;
}

void sscg_destroy(sscg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->side) (void)hipStreamSynchronize(c->side);
  Buf* bufs[] = {&c->width, &c->off, &c->scol, &c->sval, &c->scale, &c->Y,    &c->part,
                 &c->rpart, &c->G,   &c->coef, &c->info, &c->scal,  &c->xw,   &c->bw,
                 &c->x1,    &c->lz,  &c->lzab, &c->ctl,  &c->ran,   &c->scol16, &c->svidx, &c->svtab,
                 &c->sval32, &c->Y32, &c->dx,  &c->r64, &c->xu, &c->upart,
                 &c->sd_nd, &c->sd_delta, &c->sd_tab, &c->sd_code, &c->sd_vk};
  for (Buf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  BatchWs& w = c->batch;
  Buf* bbufs[] = {&w.width, &w.off,  &w.scol, &w.sval, &w.flag,    &w.Y,      &w.x,     &w.b,
                  &w.sys,   &w.prm,  &w.info, &w.G,    &w.coef,    &w.hist,   &w.blk_sys,
                  &w.chunks, &w.rpart, &w.bpart, &w.gpart, &w.active, &w.perm, &w.inv, &w.T, &w.ilcnt,
                  &w.scol16, &w.svidx, &w.svtab, &w.vtcnt, &w.sd_nd, &w.sd_delta, &w.sd_tab,
                  &w.sd_code, &w.sdcnt, &w.ablk, &w.achk, &w.loff, &w.Y32};
  for (Buf* b : bbufs)
    if (b->p) (void)hipFree(b->p);
  for (auto& r : c->ev) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (c->events_made)
    for (int i = 0; i < RING; ++i) {
      (void)hipEventDestroy(c->evI[i]);
      (void)hipEventDestroy(c->evV[i]);
    }
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->hinfo) (void)hipHostFree(c->hinfo);
  if (c->hscal) (void)hipHostFree(c->hscal);
  if (c->hactive) (void)hipHostFree(c->hactive);
  delete c;
}

const char* sscg_last_error(const sscg_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

int sscg_set_timing(sscg_ctx* ctx, int families) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->timing = (unsigned)families & ((1u << NFAM) - 1);
  if (ctx->timing && !ctx->ran.p) {
    int rc = set_device(ctx);
    if (rc) return rc;
    HIPCHK(ensure(ctx->ran, sizeof(int) * RAN_CAP));
    HIPCHK(hipMemset(ctx->ran.p, 0, sizeof(int) * RAN_CAP));
  }
  for (int f = 0; f < NFAM; ++f) {
    ctx->launches[f] = 0;
    ctx->ms[f] = 0;
    ctx->bytes[f] = 0;
  }
  HIPCHK(ev_drop(ctx));
  return SSCG_OK;
}

int sscg_kernel_stats(sscg_ctx* ctx, int family, int64_t* launches, double* ms, double* bytes) {
  if (!ctx || family < 0 || family >= NFAM) return SSCG_ERR_ARG;
  if (ctx->ev_used) {  // events of per-stage calls not yet collected
    int rc = set_device(ctx);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->side));
    HIPCHK(ev_collect(ctx));
  }
  if (launches) *launches = ctx->launches[family];
  if (ms) *ms = ctx->ms[family];
  if (bytes) *bytes = ctx->bytes[family];
  return SSCG_OK;
}

int sscg_residual(sscg_ctx* ctx, const sscg_csr* A, const double* b, const double* x, double* r,
                  double* out2) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  if (!b || !x || !out2) return fail(ctx, SSCG_ERR_ARG, "b, x and out2 must not be NULL");
  DevMat M;
  if ((rc = build_mat(ctx, A, 0, &M))) return rc;
  if ((rc = ensure_parts(ctx, A->n, 2))) return rc;
  int np = residual_nparts(A->n);
  double* part = as<double>(ctx->part);
  HIPCHK(launch_residual(M, b, x, r, part, part + 2 * (size_t)np, &np, ctx->stream));
  HIPCHK(launch_finalize(part, np, 2, out2, ctx->stream));
  return SSCG_OK;
}

int sscg_spectral_bounds(sscg_ctx* ctx, const sscg_csr* A, int steps, uint64_t seed,
                         double* lambda_min, double* lambda_max) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  if (!lambda_min || !lambda_max) return fail(ctx, SSCG_ERR_ARG, "NULL output");
  if (steps < 1 || steps > 2 * SSCG_S_LIMIT + 1)
    return fail(ctx, SSCG_ERR_ARG, "steps = %d outside [1, %d]", steps, 2 * SSCG_S_LIMIT + 1);
  DevMat M;
  if ((rc = build_mat(ctx, A, 0, &M))) return rc;
  return spectral_bounds_dev(ctx, M, steps, seed, lambda_min, lambda_max);
}

int sscg_matrix_format(sscg_ctx* ctx, const sscg_csr* A, int* format, int64_t* stored) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  DevMat M;
  if ((rc = build_mat(ctx, A, 0, &M))) return rc;
  // the forms the matrix-powers pass dispatches on: tables only with 16-bit offsets
  const int f = (M.col16 ? SSCG_FMT_COL16 : 0) | (M.col16 && M.vidx ? SSCG_FMT_VTAB : 0) |
                (M.sd_code ? SSCG_FMT_SDIA : 0) | (M.sd_code && M.sd_pair ? SSCG_FMT_SDPAIR : 0) |
                (M.sd_code && M.sd_vk ? SSCG_FMT_SDVAL : 0);
  if (format) *format = f;
  if (stored) *stored = ctx->sell_total;
  return SSCG_OK;
}

int sscg_set_forms(sscg_ctx* ctx, int forms) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  if (forms & ~(SSCG_FMT_COL16 | SSCG_FMT_VTAB | SSCG_FMT_SDIA | SSCG_FMT_SDPAIR | SSCG_FMT_SDVAL))
    return fail(ctx, SSCG_ERR_ARG,
                "forms = %d: bits SSCG_FMT_COL16 | VTAB | SDIA | SDPAIR | SDVAL only", forms);
  ctx->forms = forms;
  return SSCG_OK;
}

int sscg_newton_shifts(sscg_ctx* ctx, const sscg_csr* A, int m, uint64_t seed, double* shifts) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  if (!shifts) return fail(ctx, SSCG_ERR_ARG, "NULL output");
  if (m < 1 || m > SSCG_S_LIMIT)
    return fail(ctx, SSCG_ERR_ARG, "m = %d outside [1, %d]", m, SSCG_S_LIMIT);
  DevMat M;
  if ((rc = build_mat(ctx, A, 0, &M))) return rc;
  return newton_shifts_dev(ctx, M, m, seed, shifts);
}

int sscg_mpk_newton(sscg_ctx* ctx, const sscg_csr* A, int s, int first, const double* shifts,
                    double* Y, int64_t ldy, int rcol) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  if (s < 1 || s > SSCG_S_LIMIT)
    return fail(ctx, SSCG_ERR_ARG, "s = %d outside [1, %d]", s, SSCG_S_LIMIT);
  if (!Y || ldy < A->n) return fail(ctx, SSCG_ERR_ARG, "Y NULL or ldy < n");
  if (!first && rcol < s + 1) return fail(ctx, SSCG_ERR_ARG, "rcol must be >= s+1");
  if (!shifts) return fail(ctx, SSCG_ERR_ARG, "shifts is NULL");
  double th[SSCG_S_LIMIT];
  for (int i = 0; i < s; ++i) {
    th[i] = shifts[i];
    if (!isfinite(th[i])) return fail(ctx, SSCG_ERR_ARG, "shifts[%d] not finite", i);
  }
  DevMat M;
  if ((rc = build_mat(ctx, A, 0, &M))) return rc;
  BasisCols bc{Y, Y + (int64_t)rcol * ldy, Y, ldy, rcol};
  return mpk_passes(ctx, M, s, first ? 1 : 0, make_basis(SSCG_BASIS_NEWTON, 0.0, 1.0, th), bc,
                    ctx->mat_bytes, nullptr, MpkResidual{});
}

int sscg_mpk(sscg_ctx* ctx, const sscg_csr* A, int s, int first, int basis, double lambda_min,
             double lambda_max, double* Y, int64_t ldy, int rcol) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  if (s < 1 || s > SSCG_S_LIMIT)
    return fail(ctx, SSCG_ERR_ARG, "s = %d outside [1, %d]", s, SSCG_S_LIMIT);
  if (!Y || ldy < A->n) return fail(ctx, SSCG_ERR_ARG, "Y NULL or ldy < n");
  if (!first && rcol < s + 1) return fail(ctx, SSCG_ERR_ARG, "rcol must be >= s+1");
  if (basis != SSCG_BASIS_MONOMIAL && basis != SSCG_BASIS_CHEBYSHEV)
    return fail(ctx, SSCG_ERR_ARG, "basis %d: monomial or Chebyshev (Newton: sscg_mpk_newton)",
                basis);
  if (basis == SSCG_BASIS_CHEBYSHEV && !(lambda_max > lambda_min))
    return fail(ctx, SSCG_ERR_ARG, "need lambda_max > lambda_min");
  DevMat M;
  if ((rc = build_mat(ctx, A, 0, &M))) return rc;
  BasisCols bc{Y, Y + (int64_t)rcol * ldy, Y, ldy, rcol};
  return mpk_passes(ctx, M, s, first ? 1 : 0, make_basis(basis, lambda_min, lambda_max), bc,
                    ctx->mat_bytes, nullptr, MpkResidual{});
}

int sscg_gram(sscg_ctx* ctx, int n, int s, int first, const double* Y, int64_t ldy, int rcol,
              double* G) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if (n < 1 || s < 1 || s > SSCG_S_LIMIT || !Y || !G || ldy < n)
    return fail(ctx, SSCG_ERR_ARG, "bad Gram arguments");
  if (!first && rcol < s + 1) return fail(ctx, SSCG_ERR_ARG, "rcol must be >= s+1");
  double* Yw = const_cast<double*>(Y);
  BasisCols bc{Y, Y + (int64_t)rcol * ldy, Yw, ldy, rcol};
  const int f = first ? 1 : 0;
  return gram_into(ctx, colptr_of(bc, s, f), n, f ? s + 1 : 2 * s + 1, G, nullptr);
}

int sscg_small_solve(sscg_ctx* ctx, const double* G, const sscg_block_params* prm, double* coef,
                     sscg_block_info* info) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if (!G || !prm || !coef || !info) return fail(ctx, SSCG_ERR_ARG, "NULL argument");
  if (prm->s < 1 || prm->s > SSCG_S_LIMIT) return fail(ctx, SSCG_ERR_ARG, "bad s");
  if (!prm->adaptive && (prm->iters < 1 || prm->iters > prm->s))
    return fail(ctx, SSCG_ERR_ARG, "iters must be in [1, s]");
  if (prm->basis < 0 || prm->basis > 2) return fail(ctx, SSCG_ERR_ARG, "bad basis");
  if (prm->adaptive && !(prm->eps_star > 0.0))
    return fail(ctx, SSCG_ERR_ARG, "need eps_star > 0");
  if (prm->adaptive && prm->c_mode == SSCG_C_CONST && !(prm->c > 0.0))
    return fail(ctx, SSCG_ERR_ARG, "need c > 0");
  if (prm->adaptive && prm->c_mode == SSCG_C_THEORY &&
      !(prm->kappa_a >= 1.0 && prm->norm_a > 0.0 && prm->n_a >= 0 && prm->s_max >= 1))
    return fail(ctx, SSCG_ERR_ARG, "theoretical c needs kappa_a >= 1, norm_a > 0, n_a, s_max");
  if (prm->c_mode < 0 || prm->c_mode > 1) return fail(ctx, SSCG_ERR_ARG, "bad c_mode");
  int d = prm->first ? prm->s + 1 : 2 * prm->s + 1;
  if (prm->adaptive) HIPCHK(launch_kappa(G, d, prm->s, prm->first, info, nullptr, ctx->stream));
  HIPCHK(launch_inner(G, *prm, coef, info, nullptr, ctx->stream));
  return SSCG_OK;
}

int sscg_recover(sscg_ctx* ctx, int n, int s, int first, const double* Y, int64_t ldy, int rcol,
                 const double* coef, double* x, double* r, double* p) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if (n < 1 || s < 1 || s > SSCG_S_LIMIT || !Y || !coef || !x || !r || !p || ldy < n)
    return fail(ctx, SSCG_ERR_ARG, "bad recovery arguments");
  if (!first && rcol < s + 1) return fail(ctx, SSCG_ERR_ARG, "rcol must be >= s+1");
  double* Yw = const_cast<double*>(Y);
  BasisCols bc{Y, Y + (int64_t)rcol * ldy, Yw, ldy, rcol};
  const int f = first ? 1 : 0;
  HIPCHK(launch_recover(colptr_of(bc, s, f), n, f ? s + 1 : 2 * s + 1, coef, x, x, r, p,
                        Gate{nullptr, nullptr}, ctx->stream));
  return SSCG_OK;
}

}  // extern "C"
