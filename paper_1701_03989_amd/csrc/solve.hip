// sscg_solve: the outer block loop of Algorithms 2-4 on the device.
//
// Every block k runs on the context's stream S1: the s matrix-powers passes
// (the first one also forms the true residual of the block's starting
// iterate x_k), the Gram matrix, the coordinate solve and the recovery
// x_{k+1} = x_k + Y x', r = Y r', p = Y p'.  The inputs x_k, p_k, r_k and the
// Gram matrix of block k live in set k mod NSET of rotating buffers: block
// k's recovery overwrites the set of block k - 3, whose validation the host
// has always seen complete by then (at most LOOKAHEAD - 1 = 2 blocks are
// pending when a block is enqueued), so block k's inputs survive until it
// is accepted without any wait between the streams.
//
// The host enqueues blocks ahead without waiting, steered by a device flag
// that stops every later kernel (converged, breakdown, or a rejected
// speculation).  In Algorithm 4 the host must know s_k before it can size the
// next block, except in the steady state where the previous block took all
// its s steps: then block k is run speculatively with s~ = s and no break,
// and the exact decisions (kappa of every sub-Gram, eq. condy, eq. check) are
// taken concurrently on a second stream S2 and compared; if they would have
// stopped short, block k is redone from its saved inputs the ordinary way.
// Both routes compute the same numbers, so the result does not depend on
// whether a block was speculative.
#include <math.h>
#include <string.h>

#include <deque>

#include "ctx.h"

using namespace sscg_host;

namespace {

constexpr int LOOKAHEAD = 3;  // blocks enqueued but not yet examined by the host
constexpr int NSET = LOOKAHEAD + 1;  // rotating sets of block inputs (x, p, r, G)

__global__ void k_eps_star(const double* b2, double tol, double* out) {
  if (threadIdx.x == 0) out[0] = tol * sqrt(b2[0]);
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

struct Pending {
  int k, s_bar, s, first, spec, ahead;
};

}  // namespace

// SSCG_PREC_VARIABLE: the blocks pick their basis precision on the device
// (the batched path's plan), so the solve runs as a batch of one system; the
// Chebyshev interval is estimated first when not given.  The per-block
// outputs the batched path does not record (s_bar, s_built, gamma, thr,
// res_updated, kappa) are NaN / 0.
int sscg_host::solve_variable(sscg_ctx* ctx, const sscg_csr* A, const double* b, double* x,
                              const sscg_opts& o, sscg_result* res) {
  if (o.equilibrate)
    return fail(ctx, SSCG_ERR_ARG, "variable precision: equilibration is not supported");
  double lmin = o.lambda_min, lmax = o.lambda_max;
  if (o.basis == SSCG_BASIS_CHEBYSHEV && !(lmax > lmin)) {
    DevMat M;
    int rc = build_mat(ctx, A, 0, &M);
    if (rc) return rc;
    MethodSetup ms;
    if ((rc = method_setup(ctx, M, o, &ms))) return rc;
    lmin = ms.lmin;
    lmax = ms.lmax;
  }
  const double* bs[1] = {b};
  double* xs[1] = {x};
  sscg_batch B;
  memset(&B, 0, sizeof B);
  B.nsys = 1;
  B.A = A;
  B.b = bs;
  B.x = xs;
  B.lambda_min = &lmin;
  B.lambda_max = &lmax;
  int32_t st = 0, bl = 0, it = 0;
  double rel = NAN;
  sscg_batch_result br;
  memset(&br, 0, sizeof br);
  br.cap = res ? res->cap : 0;
  br.status = &st;
  br.blocks = &bl;
  br.iters = &it;
  br.relres = &rel;
  if (res) {
    br.s_k = res->s_k;
    br.s_tilde = res->s_tilde;
    br.relres_true = res->relres_true;
    br.fp32 = res->fp32;
  }
  const int rc = sscg_batch_solve(ctx, &B, &o, &br);
  if (rc < 0) return rc;
  if (res) {
    sscg_result& R = *res;
    R.blocks = bl;
    R.iters = it;
    R.status = st;
    R.relres0 = NAN;
    R.relres = rel;
    R.lambda_min = lmin;
    R.lambda_max = lmax;
    R.basis_vectors = R.wasted_vectors = 0;
    R.spec_blocks = R.spec_rejected = 0;
    for (int k = 0; k < std::min(R.cap, bl); ++k) {
      if (R.s_bar) R.s_bar[k] = 0;
      if (R.s_built) R.s_built[k] = 0;
      if (R.gamma) R.gamma[k] = NAN;
      if (R.thr) R.thr[k] = NAN;
      if (R.res_updated) R.res_updated[k] = NAN;
      if (R.kappa)
        for (int i = 0; i < o.s_max; ++i) R.kappa[(int64_t)k * o.s_max + i] = NAN;
    }
  }
  return st;
}

extern "C" int sscg_solve(sscg_ctx* ctx, const sscg_csr* A, const double* b, double* x,
                          const sscg_opts* opts, sscg_result* res) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if ((rc = validate_opts(ctx, opts))) return rc;
  if ((rc = check_csr(ctx, A))) return rc;
  if (!b || !x) return fail(ctx, SSCG_ERR_ARG, "b and x must not be NULL");
  if (opts->precision == SSCG_PREC_MIXED) return solve_mixed(ctx, A, b, x, *opts, res);
  if (opts->precision == SSCG_PREC_VARIABLE) return solve_variable(ctx, A, b, x, *opts, res);
  const sscg_opts& o = *opts;
  const int n = A->n;
  hipStream_t S1 = ctx->stream, S2 = ctx->side;
  HIPCHK(ev_drop(ctx));

  DevMat M;
  if ((rc = build_mat(ctx, A, o.equilibrate, &M))) return rc;

  // ---- workspace (sized once: nothing may be reallocated while blocks run)
  const int64_t ld = ((int64_t)n + 63) / 64 * 64;
  const int rcol = o.s_max + 1;
  const int ncols = 2 * o.s_max + 1 + 2 * (NSET - 1);  // P_0.., R_0.., P_0/R_0 of the other sets
  const int dmax = 2 * o.s_max + 1;
  const size_t gsz = (size_t)(2 * SSCG_S_LIMIT + 1) * (2 * SSCG_S_LIMIT + 1);
  HIPCHK(ensure(ctx->Y, sizeof(double) * ld * ncols));
  HIPCHK(ensure(ctx->x1, sizeof(double) * n * (NSET - 1)));
  HIPCHK(ensure(ctx->G, sizeof(double) * NSET * gsz));
  HIPCHK(ensure(ctx->coef, sizeof(double) * 3 * (2 * SSCG_S_LIMIT + 1)));
  HIPCHK(ensure(ctx->info, sizeof(sscg_block_info) * RING));
  HIPCHK(ensure(ctx->scal, sizeof(double) * 16));
  HIPCHK(ensure(ctx->ctl, sizeof(int) * 4));
  if ((rc = ensure_parts(ctx, n, 2))) return rc;
  HIPCHK(ensure(ctx->part, std::max(ctx->part.cap, sizeof(double) * (size_t)gram_ngroups(n) *
                                                        (dmax * (dmax + 1) / 2))));
  const int np_res = residual_nparts(n);
  HIPCHK(ensure(ctx->rpart, sizeof(double) * 2 * (size_t)np_res));
  const double* bw = b;
  double* X[NSET];
  X[0] = x;
  for (int q = 1; q < NSET; ++q) X[q] = as<double>(ctx->x1) + (size_t)(q - 1) * n;
  if (o.equilibrate) {
    HIPCHK(ensure(ctx->bw, sizeof(double) * n));
    HIPCHK(ensure(ctx->xw, sizeof(double) * n));
    HIPCHK(launch_scale_vec(b, as<double>(ctx->scale), 1, n, as<double>(ctx->bw), S1));
    HIPCHK(launch_scale_vec(x, as<double>(ctx->scale), 0, n, as<double>(ctx->xw), S1));
    bw = as<double>(ctx->bw);
    X[0] = as<double>(ctx->xw);
  }
  double* Y = as<double>(ctx->Y);
  auto ycol = [&](int c) { return Y + (int64_t)c * ld; };
  double *P0[NSET], *R0[NSET];
  P0[0] = ycol(0);
  R0[0] = ycol(rcol);
  for (int q = 1; q < NSET; ++q) {
    P0[q] = ycol(2 * o.s_max + 2 * q - 1);
    R0[q] = ycol(2 * o.s_max + 2 * q);
  }
  double* Gbuf = as<double>(ctx->G);
  double* coef = as<double>(ctx->coef);
  double* scal = as<double>(ctx->scal);  // [0] r2 [1] b2 [2] relres [3] eps*
  sscg_block_info* dinfo = as<sscg_block_info>(ctx->info);
  int* stop = as<int>(ctx->ctl);

  // ---- r_1 = b - A x_1 into P_0; ||b||, eps*, relres_0
  double* part = as<double>(ctx->part);
  int np = np_res;
  HIPCHK(launch_residual(M, bw, X[0], P0[0], part, part + 2 * (size_t)np, &np, S1));
  HIPCHK(launch_finalize(part, np, 2, scal, S1));
  HIPCHK(launch_relres(scal, scal + 1, scal + 2, S1));
  hipLaunchKernelGGL(k_eps_star, dim3(1), dim3(64), 0, S1, scal + 1, o.tol, scal + 3);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, S1, stop, 0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(ctx->hscal, scal, sizeof(double) * 4, hipMemcpyDeviceToHost, S1));
  HIPCHK(hipStreamSynchronize(S1));
  const double b2 = ctx->hscal[1];
  const double eps_star = ctx->hscal[3];
  const double relres0 = ctx->hscal[2];

  sscg_result dummy;
  memset(&dummy, 0, sizeof dummy);
  sscg_result& R = res ? *res : dummy;
  R.blocks = 0;
  R.iters = 0;
  R.basis_vectors = 0;
  R.wasted_vectors = 0;
  R.spec_blocks = 0;
  R.spec_rejected = 0;
  R.lambda_min = o.lambda_min;
  R.lambda_max = o.lambda_max;
  R.relres0 = relres0;
  R.relres = relres0;

  // copy the answer (set `par`) to the caller's x, undoing the scaling
  auto finish = [&](int status, int par) -> int {
    hipError_t e = hipStreamSynchronize(S1);
    if (e == hipSuccess) e = hipStreamSynchronize(S2);
    if (e == hipSuccess && ctx->timing) e = ev_collect(ctx);
    if (e == hipSuccess && par != 0) e = launch_copy(X[par], n, X[0], S1);
    if (e == hipSuccess && o.equilibrate)
      e = launch_scale_vec(X[0], as<double>(ctx->scale), 1, n, x, S1);
    if (e == hipSuccess) e = hipStreamSynchronize(S1);
    if (e != hipSuccess) return fail(ctx, SSCG_ERR_HIP, "%s", hipGetErrorString(e));
    R.status = status;
    return status;
  };

  if (b2 == 0.0) {  // x = 0 solves A x = 0 exactly
    HIPCHK(launch_fill(X[0], n, 0.0, S1));
    R.relres0 = 0.0;
    R.relres = 0.0;
    return finish(SSCG_OK, 0);
  }
  if (relres0 <= o.tol) return finish(SSCG_OK, 0);

  MethodSetup ms;
  if ((rc = method_setup(ctx, M, o, &ms))) return rc;
  const BasisPrm bp = ms.bp;
  const double lmin = ms.lmin, lmax = ms.lmax;
  R.lambda_min = lmin;
  R.lambda_max = lmax;
  const bool adaptive = o.mode == SSCG_MODE_ADAPTIVE;
  const int s0 = o.s0_bar > 0 ? o.s0_bar : o.s_max;
  const int f = o.f > 0 ? o.f : o.s_max;

  // (s_bar, s) of block k given the previous block's steps and m
  auto sizes = [&](int k, int s_prev, int m, int* s_bar, int* s) {
    if (o.mode == SSCG_MODE_FIXED) {
      *s_bar = *s = o.fixed_s;
    } else if (o.mode == SSCG_MODE_SCHEDULE) {
      *s_bar = *s = o.schedule[k < o.schedule_len ? k : o.schedule_len - 1];
    } else if (k == 0) {
      *s_bar = *s = s0;
    } else {
      *s_bar = s_prev + f < o.s_max ? s_prev + f : o.s_max;
      const int mm = m > 1 ? m : 1;
      *s = *s_bar < mm ? *s_bar : mm;  // rank guard: i <= m
    }
  };

  auto enqueue = [&](const Pending& P) -> int {
    const int k = P.k, s = P.s, first = P.first, par = k % NSET, nxt = (k + 1) % NSET;
    const int slot = k % RING;
    sscg_block_info* info = dinfo + slot;
    const int d = first ? s + 1 : 2 * s + 1;
    BasisCols bc{P0[par], R0[par], Y, ld, rcol};
    MpkResidual rres{};
    if (!first) rres = MpkResidual{X[par], bw, as<double>(ctx->rpart)};
    ResCheck chk{};
    if (!first) chk = ResCheck{scal + 1, np_res, o.tol, info, stop};
    int rc2 = mpk_passes(ctx, M, s, first, bp, bc, ctx->mat_bytes, stop, rres, chk);
    if (rc2) return rc2;
    const ColPtr cols = colptr_of(bc, s, first);
    double* Gk = Gbuf + (size_t)par * gsz;
    if ((rc2 = gram_into(ctx, cols, n, d, Gk, stop))) return rc2;
    sscg_block_params prm;
    prm.s = s;
    prm.first = first;
    prm.adaptive = adaptive && !P.spec;
    prm.iters = s;
    prm.inner_check = o.inner_check;
    prm.basis = o.basis;
    prm.lambda_min = lmin;
    prm.lambda_max = lmax;
    prm.eps_star = eps_star;
    prm.c = o.c;
    prm.unit_roundoff = 0.0;
    ms.fill(prm);
    size_t slot_t = 0;
    if (!P.spec) {
      HIPCHK(ev_begin(ctx, 3, 0.0, S1, &slot_t));
      if (prm.adaptive) HIPCHK(launch_kappa(Gk, d, s, first, info, stop, S1));
      HIPCHK(launch_inner(Gk, prm, coef, info, stop, S1));
      HIPCHK(ev_end(ctx, slot_t, S1));
      HIPCHK(hipMemcpyAsync(ctx->hinfo + slot, info, sizeof(sscg_block_info),
                            hipMemcpyDeviceToHost, S1));
      HIPCHK(hipEventRecord(ctx->evV[slot], S1));
    } else {
      HIPCHK(ev_begin(ctx, 3, 0.0, S1, &slot_t));
      // one event for both side-stream kernels, signalled by the coordinate
      // solve's own launch: a separate event record costs the launch stream
      // several microseconds, and kappa has a whole block's time to finish
      // before the next recovery waits for it
      HIPCHK(launch_inner(Gk, prm, coef, info, stop, S1, ctx->evI[slot]));
      HIPCHK(ev_end(ctx, slot_t, S1));
      // exact decisions on the side stream (they run even after a stop so
      // that a rejected speculation is always reported)
      HIPCHK(hipStreamWaitEvent(S2, ctx->evI[slot], 0));
      HIPCHK(ev_begin(ctx, 3, 0.0, S2, &slot_t));
      HIPCHK(launch_kappa(Gk, d, s, first, info, nullptr, S2));
      HIPCHK(ev_end(ctx, slot_t, S2));
      sscg_block_params pv = prm;
      pv.adaptive = 1;
      HIPCHK(launch_validate(Gk, pv, info, stop, S2));
      HIPCHK(hipMemcpyAsync(ctx->hinfo + slot, info, sizeof(sscg_block_info),
                            hipMemcpyDeviceToHost, S2));
      HIPCHK(hipEventRecord(ctx->evV[slot], S2));
    }
    HIPCHK(ev_begin(ctx, 2, 8.0 * n * (d + 4), S1, &slot_t));
    HIPCHK(launch_recover(cols, n, d, coef, X[par], X[nxt], R0[nxt], P0[nxt],
                          Gate{stop, ev_ran(ctx, slot_t)}, S1));
    HIPCHK(ev_end(ctx, slot_t, S1));
    return SSCG_OK;
  };

  // ---- the block loop
  std::deque<Pending> pend;
  int m = 0, s_prev = 0;           // committed
  bool last_full = false;          // the last committed block took all s steps
  int m_pred = 0, s_prev_pred = 0;  // including pending blocks (assumed full)
  int k_next = 0;
  int no_spec_k = -1;              // a block redone after a rejected speculation
  for (;;) {
    // enqueue while allowed
    while ((int)pend.size() < LOOKAHEAD && (pend.empty() || pend.back().ahead) &&
           m_pred < o.max_iters) {
      Pending P;
      P.k = k_next;
      P.first = k_next == 0;
      sizes(k_next, s_prev_pred, m_pred, &P.s_bar, &P.s);
      const bool prev_full = pend.empty() ? last_full : true;
      P.spec = adaptive && !P.first && prev_full && P.s == P.s_bar && k_next != no_spec_k;
      P.ahead = adaptive ? P.spec : 1;
      if ((rc = enqueue(P))) return rc;
      pend.push_back(P);
      m_pred += P.s;
      s_prev_pred = P.s;
      ++k_next;
    }
    if (pend.empty()) break;
    // examine the oldest pending block
    const Pending P = pend.front();
    const int slot = P.k % RING;
    HIPCHK(hipEventSynchronize(ctx->evV[slot]));
    const sscg_block_info I = ctx->hinfo[slot];
    if (!P.first) {  // true residual of the block's starting iterate x_k
      const double rel = I.relres_in;
      if (P.k - 1 < R.cap && R.relres_true) R.relres_true[P.k - 1] = rel;
      R.relres = rel;
      if (rel <= o.tol) return finish(SSCG_OK, P.k % NSET);
      if (!isfinite(rel)) return finish(SSCG_BREAKDOWN, P.k % NSET);
    }
    if (P.spec) ++R.spec_blocks;
    if (P.spec && I.spec == 2) {  // rejected: redo block k the ordinary way
      ++R.spec_rejected;
      HIPCHK(hipStreamSynchronize(S1));
      HIPCHK(hipStreamSynchronize(S2));
      hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, S1, stop, 0);
      HIPCHK(hipGetLastError());
      pend.clear();
      k_next = P.k;
      m_pred = m;
      s_prev_pred = s_prev;
      no_spec_k = P.k;
      continue;
    }
    pend.pop_front();
    const int s_k = I.s_k;
    if (P.k < R.cap) {
      if (R.s_bar) R.s_bar[P.k] = P.s_bar;
      if (R.s_built) R.s_built[P.k] = P.s;
      if (R.s_tilde) R.s_tilde[P.k] = I.s_tilde;
      if (R.s_k) R.s_k[P.k] = s_k;
      if (R.gamma) R.gamma[P.k] = adaptive ? I.gamma : NAN;
      if (R.thr) R.thr[P.k] = adaptive ? I.thr : NAN;
      if (R.res_updated) R.res_updated[P.k] = sqrt((0.0 > I.rr) ? 0.0 : I.rr);
      if (R.kappa)
        for (int i = 0; i < o.s_max; ++i)
          R.kappa[(int64_t)P.k * o.s_max + i] = (adaptive && i < P.s) ? I.kappa[i] : NAN;
    }
    R.basis_vectors += P.first ? P.s : 2 * P.s - 1;
    if (s_k == 0) return finish(SSCG_BREAKDOWN, P.k % NSET);
    R.wasted_vectors += (int64_t)(P.s - s_k) * (P.first ? 1 : 2);
    m += s_k;
    s_prev = s_k;
    last_full = s_k == P.s;
    R.blocks = P.k + 1;
    R.iters = m;
    if (m >= o.max_iters) {
      // no block after this one was enqueued (the host assumed full blocks):
      // the true residual of x_{k+1} decides the status
      HIPCHK(hipStreamSynchronize(S1));
      HIPCHK(hipStreamSynchronize(S2));
      const int par = (P.k + 1) % NSET;
      int np2 = np_res;
      HIPCHK(launch_residual(M, bw, X[par], nullptr, part, nullptr, &np2, S1));
      HIPCHK(launch_finalize(part, np2, 1, scal, S1));
      HIPCHK(launch_relres(scal, scal + 1, scal + 2, S1));
      HIPCHK(hipMemcpyAsync(ctx->hscal + 2, scal + 2, sizeof(double), hipMemcpyDeviceToHost, S1));
      HIPCHK(hipStreamSynchronize(S1));
      const double rel = ctx->hscal[2];
      if (P.k < R.cap && R.relres_true) R.relres_true[P.k] = rel;
      R.relres = rel;
      return finish(rel <= o.tol ? SSCG_OK : (isfinite(rel) ? SSCG_NOT_CONVERGED : SSCG_BREAKDOWN),
                    par);
    }
    if (pend.empty()) {  // a non-speculative block: the next sizes use its actual s_k
      m_pred = m;
      s_prev_pred = s_prev;
    }
  }
  return fail(ctx, SSCG_ERR_HIP, "block loop ended without a result");
}
