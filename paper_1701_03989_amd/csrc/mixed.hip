// Mixed precision sscg_solve: FP64 iterative refinement around adaptive s-step
// CG solves whose matrix powers and basis are FP32.
//
//   r_j = b - A x_j              FP64 matrix, every row sum rounded once
//   A d_j ~= r_j                 Algorithm 4 on the FP32 copy of A: basis in
//                                FP32, Gram / kappa / coefficient recurrence in
//                                FP64, eqs. condy and check with the FP32 unit
//                                round-off 2^-24 and eps* = inner_tol * ||r_j||
//   x_{j+1} = x_j + d_j          FP64 (d_j accumulated in FP64 by the recovery)
//
// until ||r_j|| / ||b|| <= tol.  With equilibration the refinement runs on the
// scaled system but this test is made on the caller's system: x = D^-1/2 x~
// and ||b - A x|| / ||b|| from the caller's CSR arrays.  The inner solve stops
// when its updated residual estimate (r'^T G r')^(1/2) falls to inner_tol * ||r_j||, or makes no
// step.  Bandwidth per inner pass: 8 bytes per stored entry (FP32 value, int32
// index) and 4 per vector element, against 12 and 8 in FP64.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ctx.h"

using namespace sscg_host;

namespace {
constexpr double EPS32 = 0x1p-24;  // unit round-off of the FP32 basis
}

int sscg_host::build_val32(sscg_ctx* ctx, float** val32) {
  HIPCHK(ensure(ctx->sval32, sizeof(float) * std::max<int64_t>(ctx->sell_total, 1)));
  HIPCHK(launch_cast_f32(as<double>(ctx->sval), ctx->sell_total, as<float>(ctx->sval32),
                         ctx->stream));
  *val32 = as<float>(ctx->sval32);
  return SSCG_OK;
}

int sscg_host::solve_mixed(sscg_ctx* ctx, const sscg_csr* A, const double* b, double* x,
                           const sscg_opts& o, sscg_result* res) {
  if (o.mode == SSCG_MODE_SCHEDULE)
    return fail(ctx, SSCG_ERR_ARG, "mixed precision: MODE_SCHEDULE is not supported");
  const int n = A->n;
  hipStream_t st = ctx->stream;
  int rc;
  DevMat M;
  if ((rc = build_mat(ctx, A, o.equilibrate, &M))) return rc;
  float* val32 = nullptr;
  if ((rc = build_val32(ctx, &val32))) return rc;

  const int S = o.mode == SSCG_MODE_FIXED ? o.fixed_s : o.s_max;
  const int64_t ld = ((int64_t)n + 63) / 64 * 64;
  const int rcol = S + 1;
  const int dmax = 2 * S + 1;
  HIPCHK(ensure(ctx->Y32, sizeof(float) * ld * (2 * S + 1)));
  HIPCHK(ensure(ctx->dx, sizeof(double) * n));
  HIPCHK(ensure(ctx->r64, sizeof(double) * n));
  HIPCHK(ensure(ctx->G, sizeof(double) * dmax * dmax));
  HIPCHK(ensure(ctx->coef, sizeof(double) * 3 * dmax));
  HIPCHK(ensure(ctx->info, sizeof(sscg_block_info)));
  HIPCHK(ensure(ctx->scal, sizeof(double) * 16));
  if ((rc = ensure_parts(ctx, n, 2))) return rc;
  const int npg = gram_ngroups(n);
  HIPCHK(ensure(ctx->rpart, sizeof(double) * (size_t)npg * (dmax * (dmax + 1) / 2)));
  float* Y = as<float>(ctx->Y32);
  float* P0 = Y;
  float* R0 = Y + (int64_t)rcol * ld;
  double* dx = as<double>(ctx->dx);
  double* r = as<double>(ctx->r64);
  double* G = as<double>(ctx->G);
  double* coef = as<double>(ctx->coef);
  double* scal = as<double>(ctx->scal);  // [0] r2 [1] b2 (solved system) [2] r2 [3] b2 (caller's)
  double* part = as<double>(ctx->part);
  double* gpart = as<double>(ctx->rpart);
  sscg_block_info* info = as<sscg_block_info>(ctx->info);
  // equilibration (Section 5): solve the scaled system, unscale at the end
  const double* b_in = b;
  double* x_out = x;
  if (o.equilibrate) {
    HIPCHK(ensure(ctx->bw, sizeof(double) * n));
    HIPCHK(ensure(ctx->xw, sizeof(double) * n));
    HIPCHK(launch_scale_vec(b_in, as<double>(ctx->scale), 1, n, as<double>(ctx->bw), st));
    HIPCHK(launch_scale_vec(x_out, as<double>(ctx->scale), 0, n, as<double>(ctx->xw), st));
    b = as<double>(ctx->bw);
    x = as<double>(ctx->xw);
  }

  // equilibrated: the unscaled iterate and its residual on the caller's system
  double* xu = nullptr;
  double* upart = nullptr;
  const int unp = csr_residual_nparts(n);
  if (o.equilibrate) {
    HIPCHK(ensure(ctx->xu, sizeof(double) * n));
    HIPCHK(ensure(ctx->upart, sizeof(double) * 4 * (size_t)unp));
    xu = as<double>(ctx->xu);
    upart = as<double>(ctx->upart);
  }

  sscg_result dummy;
  memset(&dummy, 0, sizeof dummy);
  sscg_result& R = res ? *res : dummy;
  R.blocks = 0;
  R.iters = 0;
  R.basis_vectors = 0;
  R.wasted_vectors = 0;
  R.spec_blocks = 0;
  R.spec_rejected = 0;

  // basis and c_{k,j} parameters of A (estimated in FP64 where not given)
  MethodSetup ms;
  if ((rc = method_setup(ctx, M, o, &ms))) return rc;
  const BasisPrm bp = ms.bp;
  const double lmin = ms.lmin, lmax = ms.lmax;
  R.lambda_min = lmin;
  R.lambda_max = lmax;
  const bool adaptive = o.mode == SSCG_MODE_ADAPTIVE;
  const int s0 = o.s0_bar > 0 ? o.s0_bar : o.s_max;
  const int f = o.f > 0 ? o.f : o.s_max;
  double b2 = 0.0;
  int status = SSCG_NOT_CONVERGED;

  for (int outer = 0;; ++outer) {
    // r_j = b - A x_j and its norm (||b|| on the first pass)
    int np = residual_nparts(n);
    HIPCHK(launch_residual(M, b, x, r, part, outer == 0 ? part + 2 * (size_t)np : nullptr, &np,
                           st));
    HIPCHK(launch_finalize(part, np, outer == 0 ? 2 : 1, scal, st));
    if (o.equilibrate) {  // ||b - A x||^2 and ||b||^2 of the caller's system
      HIPCHK(launch_scale_vec(x, as<double>(ctx->scale), 1, n, xu, st));
      HIPCHK(launch_csr_residual(A->rowptr, A->col, A->val, n, b_in, xu, upart,
                                 upart + 2 * (size_t)unp, st));
      HIPCHK(launch_finalize(upart, unp, 2, scal + 2, st));
    }
    HIPCHK(hipMemcpyAsync(ctx->hscal, scal, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double r2 = ctx->hscal[0];
    if (outer == 0) {
      b2 = ctx->hscal[1];
      if (b2 == 0.0) {  // x = 0 solves A x = 0
        HIPCHK(launch_fill(x, n, 0.0, st));
        R.relres0 = R.relres = 0.0;
        status = SSCG_OK;
        break;
      }
    }
    const double rel = o.equilibrate ? sqrt(ctx->hscal[2]) / sqrt(ctx->hscal[3])
                                     : sqrt(r2) / sqrt(b2);
    if (outer == 0) R.relres0 = rel;
    else if (R.blocks >= 1 && R.blocks - 1 < R.cap && R.relres_true)
      R.relres_true[R.blocks - 1] = rel;
    R.relres = rel;
    if (rel <= o.tol) {
      status = SSCG_OK;
      break;
    }
    if (!isfinite(rel)) {
      status = SSCG_BREAKDOWN;
      break;
    }
    if (outer >= o.max_outer || R.iters >= o.max_iters) break;

    // inner solve of A d = r_j in the FP32 basis
    const double eps_in = o.inner_tol * sqrt(r2);
    HIPCHK(launch_fill(dx, n, 0.0, st));
    HIPCHK(hipMemsetAsync(Y, 0, sizeof(float) * ld * (2 * S + 1), st));
    HIPCHK(launch_cast_f32(r, n, P0, st));
    int m = 0, s_prev = 0, progress = 0;
    for (int k = 0; R.iters < o.max_iters; ++k) {
      const int first = k == 0;
      int s_bar, s;
      if (o.mode == SSCG_MODE_FIXED) {
        s_bar = s = o.fixed_s;
      } else if (first) {
        s_bar = s = s0;
      } else {
        s_bar = std::min(s_prev + f, o.s_max);
        s = std::min(s_bar, std::max(m, 1));
      }
      const int d = first ? s + 1 : 2 * s + 1;
      for (int j = 1; j <= s; ++j) {
        MpkSeq32 sp{Y + (int64_t)(j - 1) * ld, j >= 2 ? Y + (int64_t)(j - 2) * ld : nullptr,
                    Y + (int64_t)j * ld};
        MpkSeq32 sr{nullptr, nullptr, nullptr};
        int nrhs = 1;
        if (!first && j <= s - 1) {
          sr = MpkSeq32{R0 + (int64_t)(j - 1) * ld, j >= 2 ? R0 + (int64_t)(j - 2) * ld : nullptr,
                        R0 + (int64_t)j * ld};
          nrhs = 2;
        }
        HIPCHK(launch_mpk32_pass(M, val32, j, bp, nrhs, sp, sr, st));
      }
      const Cols32 cols{Y, ld, s, rcol};
      HIPCHK(launch_gram32(cols, n, d, gpart, st));
      HIPCHK(launch_gram_finalize(gpart, npg, d, G, nullptr, st));
      sscg_block_params prm;
      prm.s = s;
      prm.first = first;
      prm.adaptive = adaptive;
      prm.iters = s;
      prm.inner_check = o.inner_check;
      prm.basis = o.basis;
      prm.lambda_min = lmin;
      prm.lambda_max = lmax;
      prm.eps_star = eps_in;
      prm.c = o.c;
      prm.unit_roundoff = EPS32;
      ms.fill(prm);
      if (adaptive) HIPCHK(launch_kappa(G, d, s, first, info, nullptr, st));
      HIPCHK(launch_inner(G, prm, coef, info, nullptr, st));
      HIPCHK(launch_recover32(cols, n, d, coef, dx, R0, P0, st));
      HIPCHK(hipMemcpyAsync(ctx->hinfo, info, sizeof(sscg_block_info), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const sscg_block_info& I = ctx->hinfo[0];
      const int kb = R.blocks;
      if (kb < R.cap) {
        if (R.s_bar) R.s_bar[kb] = s_bar;
        if (R.s_built) R.s_built[kb] = s;
        if (R.s_tilde) R.s_tilde[kb] = I.s_tilde;
        if (R.s_k) R.s_k[kb] = I.s_k;
        if (R.gamma) R.gamma[kb] = adaptive ? I.gamma : NAN;
        if (R.thr) R.thr[kb] = adaptive ? I.thr : NAN;
        if (R.res_updated) R.res_updated[kb] = sqrt(std::max(0.0, I.rr));
        if (R.relres_true) R.relres_true[kb] = NAN;
        if (R.kappa)
          for (int i = 0; i < o.s_max; ++i)
            R.kappa[(int64_t)kb * o.s_max + i] = (adaptive && i < s) ? I.kappa[i] : NAN;
      }
      R.blocks += 1;
      R.basis_vectors += first ? s : 2 * s - 1;
      R.wasted_vectors += (int64_t)(s - I.s_k) * (first ? 1 : 2);
      if (I.s_k == 0) break;
      progress += I.s_k;
      R.iters += I.s_k;
      m += I.s_k;
      s_prev = I.s_k;
      if (I.rr <= eps_in * eps_in) break;
    }
    if (progress == 0) {  // the inner solve could not take a step
      status = SSCG_BREAKDOWN;
      break;
    }
    HIPCHK(launch_add(x, dx, n, st));
  }
  if (o.equilibrate) HIPCHK(launch_scale_vec(x, as<double>(ctx->scale), 1, n, x_out, st));
  HIPCHK(hipStreamSynchronize(st));
  R.status = status;
  return status;
}

extern "C" int sscg_mpk32(sscg_ctx* ctx, const sscg_csr* A, int s, int first, int basis,
                          double lambda_min, double lambda_max, float* Y, int64_t ldy, int rcol) {
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
    return fail(ctx, SSCG_ERR_ARG, "basis %d: monomial or Chebyshev", basis);
  if (basis == SSCG_BASIS_CHEBYSHEV && !(lambda_max > lambda_min))
    return fail(ctx, SSCG_ERR_ARG, "need lambda_max > lambda_min");
  DevMat M;
  if ((rc = build_mat(ctx, A, 0, &M))) return rc;
  float* val32 = nullptr;
  if ((rc = build_val32(ctx, &val32))) return rc;
  const BasisPrm bp = make_basis(basis, lambda_min, lambda_max);
  float* R0 = Y + (int64_t)rcol * ldy;
  for (int j = 1; j <= s; ++j) {
    MpkSeq32 sp{Y + (int64_t)(j - 1) * ldy, j >= 2 ? Y + (int64_t)(j - 2) * ldy : nullptr,
                Y + (int64_t)j * ldy};
    MpkSeq32 sr{nullptr, nullptr, nullptr};
    int nrhs = 1;
    if (!first && j <= s - 1) {
      sr = MpkSeq32{R0 + (int64_t)(j - 1) * ldy, j >= 2 ? R0 + (int64_t)(j - 2) * ldy : nullptr,
                    R0 + (int64_t)j * ldy};
      nrhs = 2;
    }
    HIPCHK(launch_mpk32_pass(M, val32, j, bp, nrhs, sp, sr, ctx->stream));
  }
  return SSCG_OK;
}

extern "C" int sscg_gram32(sscg_ctx* ctx, int n, int s, int first, const float* Y, int64_t ldy,
                           int rcol, double* G) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if (n < 1 || s < 1 || s > SSCG_S_LIMIT || !Y || !G || ldy < n)
    return fail(ctx, SSCG_ERR_ARG, "bad Gram arguments");
  if (!first && rcol < s + 1) return fail(ctx, SSCG_ERR_ARG, "rcol must be >= s+1");
  const int d = first ? s + 1 : 2 * s + 1;
  const int np = gram_ngroups(n);
  HIPCHK(ensure(ctx->part, sizeof(double) * (size_t)np * (d * (d + 1) / 2)));
  const Cols32 cols{Y, ldy, s, rcol};
  HIPCHK(launch_gram32(cols, n, d, as<double>(ctx->part), ctx->stream));
  HIPCHK(launch_gram_finalize(as<double>(ctx->part), np, d, G, nullptr, ctx->stream));
  return SSCG_OK;
}
