// The coordinate problem of one outer block (Algorithm 4 from "Determine s~"
// to the end of the inner loop), solved in LDS by single workgroups.
//
// k_kappa: kappa(G_i) = lambda_max / lambda_min of every candidate sub-Gram
//   G_i (Section 4.2), one workgroup per i, by two-sided cyclic
//   Jacobi with the parallel round-robin ordering (Golub & Van Loan, Sec.
//   8.5).  The operation sequence is fixed (skip rule, rotation formulas,
//   column-then-row application, mirroring of the upper triangle, exact
//   update of the rotated 2x2 blocks), so equal inputs give equal bits.
// k_inner: s~ by eq. condy, B by eq. AVVB, the coordinate recurrence with the
//   break of eq. check; one wave, lane a owns coordinate a.
#include <hip/hip_ext.h>

#include "common.h"

namespace {

constexpr int MAXK = 2 * SSCG_S_LIMIT + 1;  // largest sub-Gram dimension
constexpr int LDK = MAXK;                  // odd row stride: column walks hit distinct banks
constexpr double EPS = 0x1p-53;            // unit round-off (Section 5)
constexpr double EPS32 = 0x1p-24;          // unit round-off of an FP32 basis
constexpr int MAX_SWEEPS = 40;

// Index of sub-basis column a (of G_i) in the full Gram matrix of s steps.
__device__ __forceinline__ int sub_index(int a, int i, int s, int first) {
  if (first || a <= i) return a;
  return s + 1 + (a - i - 1);
}

// Round-robin position of slot i at step t (m even).
__device__ __forceinline__ int rr_pos(int i, int t, int m) {
  const int x = i - 1 + t;  // below 2 (m - 1) for 0 < i < m and 0 <= t < m - 1
  return i == 0 ? 0 : 1 + (x >= m - 1 ? x - (m - 1) : x);
}

#ifndef SSCG_JT
#define SSCG_JT 192
#endif
constexpr int JT = SSCG_JT;  // threads of a single Jacobi problem (latency)

// LDS of one Jacobi eigenvalue problem: the matrix before and after a step,
// and the rotations of two steps (those of step g + 1 are formed while step g
// is applied, so that a step costs one barrier).
struct JacobiLds {
  double A[2][MAXK * LDK];          // the matrix, row-major, both triangles kept equal
  double ws[2][MAXK], wo[2][MAXK];  // weights of index i: new_i = ws*old_i + wo*old_partner
  double fd[2][MAXK];               // exact diagonal of a rotated index after the step
  int pt[2][MAXK];                  // partner of index i in the step, -1 if not rotated
  int nrot[2];                      // rotations in the step
};

// Entry (r, c), r <= c, of the matrix after one step (rotation tables ws, wo,
// fd, pt) from the matrix A before it: B = A J by columns, then the rows of
// J^T B; a rotated pair keeps the closed form of its diagonal entries and a
// zero off-diagonal entry.  Every thread that needs an entry computes it by
// this one sequence of operations, so the result does not depend on which
// thread (or how many threads) did the work.  The loads are issued in two
// rounds (the tables and a_rc, then the partners' entries) and the cases are
// selected at the end; table values of an index that is not rotated are
// loaded but never used.
__device__ __forceinline__ double step_entry(const double* A, const double* ws, const double* wo,
                                             const double* fd, const int* pt, int r, int c) {
  const int pc = pt[c], pr = pt[r];
  const double wsc = ws[c], woc = wo[c], wsr = ws[r], wor = wo[r], fdc = fd[c];
  const double arc = A[r * LDK + c];
  const int pcc = pc >= 0 ? pc : c, prr = pr >= 0 ? pr : r;
  double arp = A[r * LDK + pcc], apc = A[prr * LDK + c], app = A[prr * LDK + pcc];
  // keep the second round of loads unconditional (not sunk into the cases,
  // which would serialise them); the empty statement changes no value
  asm volatile("" : "+v"(arp), "+v"(apc), "+v"(app));
  const double br = pc >= 0 ? wsc * arc + woc * arp : arc;  // B = A J, row r
  const double bp = pc >= 0 ? wsc * apc + woc * app : apc;  // B = A J, row pr
  const double v = pr >= 0 ? wsr * br + wor * bp : br;
  return (r == c && pc >= 0) ? fdc : (pr == c ? 0.0 : v);
}

// Diagonal entry (i, i) after one step: step_entry(.., i, i), which reduces
// to the closed form of a rotated index and to a_ii otherwise.
__device__ __forceinline__ double step_diag(const double* A, const double* fd, const int* pt,
                                            int i) {
  const int pi = pt[i];
  const double f = fd[i], a = A[i * LDK + i];
  return pi >= 0 ? f : a;
}

// Rotation of the pair (p, q) from a_pp, a_qq, a_pq at the start of the step
// (the symmetric 2x2 Schur decomposition); false when the skip rule holds.
// The rotation is formed alongside the skip test (unused when skipped).
__device__ __forceinline__ bool pair_rotation(double app, double aqq, double apq, double& cs,
                                              double& sn, double& tt) {
  const double thr = EPS * (sqrt(fabs(app)) * sqrt(fabs(aqq)));
  const double tau = (aqq - app) / (2.0 * apq);
  const double sg = tau >= 0.0 ? 1.0 : -1.0;
  tt = fabs(tau) > 1e150 ? 0.5 / tau : sg / (fabs(tau) + sqrt(1.0 + tau * tau));
  cs = 1.0 / sqrt(1.0 + tt * tt);
  sn = tt * cs;
  return fabs(apq) > thr;
}

// Rotations of round-robin step nst (into table slot ^ 1, with their count)
// from the matrix after the step of table slot applied to L.A[cur].  Lane rl
// (rl >= 0: the last m/2 threads of the NT) forms pair rl.
template <int NT>
__device__ __forceinline__ void form_rotations(JacobiLds& L, int cur, int slot, int k, int m,
                                               int nst, int rl) {
  bool rot = false;
  const int o = slot ^ 1;
  if (rl >= 0) {
    const int a = rr_pos(rl, nst, m), b = rr_pos(m - 1 - rl, nst, m);
    const int p = min(a, b), q = max(a, b);
    if (q < k) {
      const double* A = L.A[cur];
      const double app = step_diag(A, L.fd[slot], L.pt[slot], p);
      const double aqq = step_diag(A, L.fd[slot], L.pt[slot], q);
      const double apq = step_entry(A, L.ws[slot], L.wo[slot], L.fd[slot], L.pt[slot], p, q);
      double cs, sn, tt;
      if (pair_rotation(app, aqq, apq, cs, sn, tt)) {
        L.ws[o][p] = cs; L.wo[o][p] = -sn; L.pt[o][p] = q;
        L.ws[o][q] = cs; L.wo[o][q] = sn; L.pt[o][q] = p;
        L.fd[o][p] = app - tt * apq;
        L.fd[o][q] = aqq + tt * apq;
        rot = true;
      } else {
        L.pt[o][p] = -1; L.pt[o][q] = -1;
      }
    } else if (p < k) {
      L.pt[o][p] = -1;
    }
  }
  if ((int)threadIdx.x >= NT - SSCG_WAVE) {  // the wavefront of the rotation lanes
    const int n = __popcll(__ballot(rot));
    if ((int)threadIdx.x == NT - 1) L.nrot[o] = n;
  }
}

// Eigenvalues of the k x k symmetric matrix in L.A[0] (k <= MAXK) by cyclic
// Jacobi on NT threads (a multiple of the wavefront); returns the copy of
// L.A that holds the result.  The first NA threads (all NT for one
// wavefront, else all but the last wavefront) apply the upper-triangle
// entries t, t + NA, ... (row by row) of each step; the last m/2 threads form
// the next step's rotations from the entries they need, so with more than
// one wavefront the rotations and the application of a step overlap.
template <int NT>
__device__ int jacobi(JacobiLds& L, int k) {
  constexpr int NA = NT == SSCG_WAVE ? NT : NT - SSCG_WAVE;
  constexpr int EPT = (MAXK * (MAXK + 1) / 2 + NA - 1) / NA;
  const int t = threadIdx.x;
  const int m = (k & 1) ? k + 1 : k;
  const int ne = k * (k + 1) / 2;
  const int rl = t - (NT - m / 2);
  int er[EPT], ec[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    int e = t + NA * j, r = 0;
    if (t < NA && e < ne) {
      while (e >= k - r) {
        e -= k - r;
        ++r;
      }
      er[j] = r;
      ec[j] = r + e;
    } else {
      er[j] = -1;
      ec[j] = 0;
    }
  }
  for (int i = t; i < MAXK; i += NT) L.pt[1][i] = -1;  // table 1: a step without rotations
  if (t == 0) L.nrot[1] = 0;
  __syncthreads();
  form_rotations<NT>(L, 0, 1, k, m, 0, rl);
  __syncthreads();
  int cur = 0, slot = 0;
  for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
    int rotated = 0;
    for (int st = 0; st < m - 1; ++st) {
      const int nr = L.nrot[slot];
      rotated += nr;
      if (t < NA && nr) {
        const double* A = L.A[cur];
        double* An = L.A[cur ^ 1];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          if (er[j] >= 0) {
            const double v =
                step_entry(A, L.ws[slot], L.wo[slot], L.fd[slot], L.pt[slot], er[j], ec[j]);
            An[er[j] * LDK + ec[j]] = v;
            An[ec[j] * LDK + er[j]] = v;
          }
        }
      }
      form_rotations<NT>(L, cur, slot, k, m, st + 1 < m - 1 ? st + 1 : 0, rl);
      if (nr) cur ^= 1;
      slot ^= 1;
      __syncthreads();
    }
    if (rotated == 0) break;
  }
  return cur;
}

__device__ double kappa_from_diag(const double* A, int k) {
  double lmin = A[0], lmax = A[0];
  bool nan = lmin != lmin;
  for (int a = 1; a < k; ++a) {
    double v = A[a * LDK + a];
    if (v != v) nan = true;
    lmin = v < lmin ? v : lmin;
    lmax = v > lmax ? v : lmax;
  }
  if (nan || !(lmin > 0.0) || isinf(lmax)) return __builtin_inf();
  return lmax / lmin;
}

// kappa(G_i) of the s-step Gram matrix G (d x d) into info->kappa[i-1]
// by jacobi on the NT threads of the workgroup.
template <int NT>
__device__ void kappa_body(JacobiLds& L, const double* __restrict__ G, int d, int s, int first,
                           int i, sscg_block_info* info) {
  int k = first ? i + 1 : 2 * i + 1;
  if (threadIdx.x < k) {
    int b = threadIdx.x;
    int gb = sub_index(b, i, s, first);
    for (int a = 0; a < k; ++a) L.A[0][a * LDK + b] = G[sub_index(a, i, s, first) * d + gb];
  }
  __syncthreads();
  const int cur = jacobi<NT>(L, k);
  if (threadIdx.x == 0) info->kappa[i - 1] = kappa_from_diag(L.A[cur], k);
}

// grid = s workgroups; workgroup i-1 computes kappa(G_i).
__global__ __launch_bounds__(JT) void k_kappa(const double* __restrict__ G, int d, int s,
                                              int first, sscg_block_info* info,
                                              const int* __restrict__ stop) {
  __shared__ JacobiLds L;
  if (stop && *stop) return;
  kappa_body<JT>(L, G, d, s, first, blockIdx.x + 1, info);
}

// Eigenvalue extremes of the Lanczos tridiagonal matrix (k <= MAXK).
__global__ __launch_bounds__(JT) void k_tridiag_eig(const double* __restrict__ alpha,
                                                           const double* __restrict__ beta, int k,
                                                           double* lmin, double* lmax) {
  __shared__ JacobiLds L;
  if (threadIdx.x < k) {
    int b = threadIdx.x;
    for (int a = 0; a < k; ++a) {
      double v = 0.0;
      if (a == b) v = alpha[a];
      else if (b == a + 1) v = beta[a];
      else if (a == b + 1) v = beta[b];
      L.A[0][a * LDK + b] = v;
    }
  }
  __syncthreads();
  const int cur = k > 1 ? jacobi<JT>(L, k) : 0;
  if (threadIdx.x == 0) {
    const double* D = L.A[cur];
    double lo = D[0], hi = D[0];
    for (int a = 1; a < k; ++a) {
      double v = D[a * LDK + a];
      lo = v < lo ? v : lo;
      hi = v > hi ? v : hi;
    }
    *lmin = lo;
    *lmax = hi;
  }
}

// Shifts of the Newton basis from the Lanczos tridiagonal matrix (k <= MAXK):
// all its eigenvalues, ascending, then in Leja order (largest modulus first;
// then the point maximising the product of distances to the points already
// chosen, multiplied in the order of choice; ties to the earlier point);
// out[i] = z[i mod k], i < m.
__global__ __launch_bounds__(JT) void k_newton_shifts(const double* __restrict__ alpha,
                                                      const double* __restrict__ beta, int k,
                                                      int m, double* __restrict__ out) {
  __shared__ JacobiLds L;
  if (threadIdx.x < k) {
    int b = threadIdx.x;
    for (int a = 0; a < k; ++a) {
      double v = 0.0;
      if (a == b) v = alpha[a];
      else if (b == a + 1) v = beta[a];
      else if (a == b + 1) v = beta[b];
      L.A[0][a * LDK + b] = v;
    }
  }
  __syncthreads();
  const int cur = k > 1 ? jacobi<JT>(L, k) : 0;
  if (threadIdx.x != 0) return;
  double* z = L.ws[0];  // k values, ascending
  for (int a = 0; a < k; ++a) {
    const double v = L.A[cur][a * LDK + a];
    int p = a;
    while (p > 0 && z[p - 1] > v) {
      z[p] = z[p - 1];
      --p;
    }
    z[p] = v;
  }
  int* ord = L.pt[0];
  double* used = L.fd[0];  // 1: already chosen
  for (int a = 0; a < k; ++a) used[a] = 0.0;
  int best = 0;
  for (int a = 1; a < k; ++a)
    if (fabs(z[a]) > fabs(z[best])) best = a;
  ord[0] = best;
  used[best] = 1.0;
  for (int t = 1; t < k; ++t) {
    best = -1;
    double bs = 0.0;
    for (int a = 0; a < k; ++a) {
      if (used[a] != 0.0) continue;
      double prod = 1.0;
      for (int u = 0; u < t; ++u) prod = prod * fabs(z[a] - z[ord[u]]);
      if (best < 0 || prod > bs) {
        best = a;
        bs = prod;
      }
    }
    ord[t] = best;
    used[best] = 1.0;
  }
  for (int i = 0; i < m; ++i) out[i] = z[ord[i % k]];
}

// ---------------------------------------------------------------- inner loop

// Coefficients of the three-term recurrence (eq. polybasiscg); th: the
// Newton shifts (read only for the Newton basis, i < s).
__device__ __forceinline__ double rec_theta(const BasisPrm& bp, const double* th, int i) {
  return bp.cheb ? bp.c0 : (bp.newton ? th[i] : 0.0);
}
__device__ __forceinline__ double rec_gamma(const BasisPrm& bp, int i) {
  return bp.cheb ? (i == 0 ? bp.h : bp.h2) : 1.0;
}
__device__ __forceinline__ double rec_sigma(const BasisPrm& bp) { return bp.cheb ? bp.h2 : 0.0; }

// (B v)_a for the s-step basis of s steps (first: P block only), R12 layout.
__device__ __forceinline__ double bmul(const double* v, int a, int s, int first, BasisPrm bp,
                                       const double* th) {
  // block offset, local index and block length
  int off = 0, len = s + 1;
  if (!first && a > s) {
    off = s + 1;
    len = s;
  }
  int j = a - off;
  dd acc = dd_zero();
  // B[a][a-1] = gamma_{j-1}: column j-1 is not the block's last
  if (j >= 1) dd_add_prod(acc, rec_gamma(bp, j - 1), v[a - 1]);
  // B[a][a] = theta_j if column j is not the last
  if (j < len - 1) dd_add_prod(acc, rec_theta(bp, th, j), v[a]);
  // B[a][a+1] = sigma_j if column j+1 is not the last
  if (j + 1 < len - 1) dd_add_prod(acc, rec_sigma(bp), v[a + 1]);
  return dd_round(acc);
}

// sqrt(||B||_1 ||B||_inf) >= ||B||_2 for the B of s steps (eq. AVVB): the
// largest column and row sums of |B|, each summed in index order.
__device__ double b_norm_bound(int s, int first, const BasisPrm& bp, const double* th) {
  double n1 = 0.0, ni = 0.0;
  for (int blk = 0; blk < (first ? 1 : 2); ++blk) {
    const int len = blk == 0 ? s + 1 : s;
    for (int j = 0; j < len; ++j) {
      double c = 0.0, r = 0.0;
      if (j < len - 1) {  // column j: sigma_{j-1}, theta_j, gamma_j (the last column is zero)
        if (j >= 1) c = c + fabs(rec_sigma(bp));
        c = c + fabs(rec_theta(bp, th, j));
        c = c + fabs(rec_gamma(bp, j));
      }
      if (j >= 1) r = r + fabs(rec_gamma(bp, j - 1));  // row j: gamma_{j-1}, theta_j, sigma_j
      if (j < len - 1) r = r + fabs(rec_theta(bp, th, j));
      if (j + 1 < len - 1) r = r + fabs(rec_sigma(bp));
      n1 = c > n1 ? c : n1;
      ni = r > ni ? r : ni;
    }
  }
  return sqrt(n1 * ni);
}

// c_{k,j} of eqs. condy and check: the given constant, or the bound of
// Section 4.1, 6 N_k j kappa(A) with N_k = 7 + 2 N_A + 14 ||B_k|| / ||A||,
// evaluated in this order with every operation rounded on its own.
__device__ __forceinline__ double c_kj(const sscg_block_params& prm, double bnorm, int j) {
  if (prm.c_mode != SSCG_C_THEORY) return prm.c;
  {
#pragma clang fp contract(off)
    const double tau = bnorm / prm.norm_a;
    const double nk = (7.0 + 2.0 * (double)prm.n_a) + 14.0 * tau;
    return ((6.0 * nk) * (double)j) * prm.kappa_a;
  }
}

struct InnerLds {
  double G[MAXK][LDK];
  double v[MAXK + 1];
  double w[MAXK + 1];
  double ps[SSCG_WAVE], pe[SSCG_WAVE];  // per-lane dd partials of the row sums
  double th[SSCG_S_LIMIT];               // Newton shifts
};

// CR dot of lane-owned values over the wave (lanes >= d hold zeros).
__device__ __forceinline__ double wave_dot(double x, double y) {
  dd a = dd_zero();
  dd_add_prod(a, x, y);
  a = dd_wave_reduce(a);
  return dd_round(a);
}

// Lane a (< d) returns RN((G v)_a), v in L.v.  Each row sum is split over
// P = 64 / d lanes (short dependent chains on a single wave), whose dd
// partials are merged in lane order through LDS.
__device__ __forceinline__ double gmul(InnerLds& L, int d) {
  const int l = threadIdx.x;
  const int P = SSCG_WAVE / d;
  const int ch = (d + P - 1) / P;
  const int row = l / P, part = l - row * P;
  dd acc = dd_zero();
  if (row < d) {
    const int b0 = part * ch, b1 = min(b0 + ch, d);
    for (int b = b0; b < b1; ++b) dd_add_prod(acc, L.G[row][b], L.v[b]);
  }
  L.ps[l] = acc.s;
  L.pe[l] = acc.e;
  __syncthreads();
  double gv = 0.0;
  if (l < d) {
    dd t{L.ps[l * P], L.pe[l * P]};
    for (int q = 1; q < P; ++q) dd_merge(t, dd{L.ps[l * P + q], L.pe[l * P + q]});
    gv = dd_round(t);
  }
  __syncthreads();
  return gv;
}

// v^T G v, with v held one value per lane.
__device__ __forceinline__ double quad(InnerLds& L, double va, int d) {
  int a = threadIdx.x;
  L.v[a < MAXK ? a : MAXK] = a < d ? va : 0.0;
  __syncthreads();
  double gv = gmul(L, d);
  return wave_dot(a < d ? va : 0.0, gv);
}

// The coordinate solve of one block (one wave).  With stop != NULL a block
// that cannot take a single step sets *stop = 3.
__device__ void inner_body(InnerLds& L, const double* __restrict__ Gfull,
                           const sscg_block_params& prm, double* __restrict__ coef,
                           sscg_block_info* info, int* stop) {
  const int a = threadIdx.x;
  const double ueps = prm.unit_roundoff > 0.0 ? prm.unit_roundoff : EPS;  // of the basis
  const int s = prm.s, first = prm.first;
  const int dfull = first ? s + 1 : 2 * s + 1;
  BasisPrm bp = make_basis(prm.basis, prm.lambda_min, prm.lambda_max);
  if (a < SSCG_S_LIMIT) L.th[a] = prm.shifts[a];
  __syncthreads();
  // ||B|| bound of the built basis (c_{k,j} of Section 4.1 only)
  const double bnorm = prm.c_mode == SSCG_C_THEORY ? b_norm_bound(s, first, bp, L.th) : 0.0;

  double gam = __builtin_nan(""), thr = __builtin_nan(""), rnorm = __builtin_nan("");
  int st;
  if (prm.adaptive) {
    int r0 = first ? 0 : s + 1;
    rnorm = sqrt(Gfull[r0 * dfull + r0]);
    thr = prm.eps_star / ((c_kj(prm, bnorm, prm.s_max) * ueps) * rnorm);
    st = 1;
    for (int i = 1; i <= s; ++i) {
      if (sqrt(info->kappa[i - 1]) <= thr) st = i;
      else break;
    }
    gam = sqrt(info->kappa[st - 1]);
  } else {
    st = prm.iters;
  }
  const int d = first ? st + 1 : 2 * st + 1;
  for (int e = a; e < d * d; e += SSCG_WAVE) {
    int x = e / d, y = e - x * d;
    L.G[x][y] = Gfull[sub_index(x, st, s, first) * dfull + sub_index(y, st, s, first)];
  }
  __syncthreads();

  // coordinates of lane a
  double p = a == 0 ? 1.0 : 0.0;
  double r = a == (first ? 0 : st + 1) ? 1.0 : 0.0;
  double x = 0.0;
  double rr = quad(L, r, d);
  int s_k = 0, status = SSCG_OK;
  for (int j = 1; j <= st; ++j) {
    // B p
    L.w[a < MAXK ? a : MAXK] = a < d ? p : 0.0;
    __syncthreads();
    double bpv = a < d ? bmul(L.w, a, st, first, bp, L.th) : 0.0;
    __syncthreads();
    // p . G (B p)
    L.v[a < MAXK ? a : MAXK] = a < d ? bpv : 0.0;
    __syncthreads();
    double gbp = gmul(L, d);
    double den = wave_dot(a < d ? p : 0.0, gbp);
    if (den == 0.0 || !(den > 0.0) || isinf(den)) {
      status = j == 1 ? SSCG_BREAKDOWN : SSCG_OK;
      break;
    }
    double alpha = rr / den;
    if (isinf(alpha) || alpha != alpha) {
      status = j == 1 ? SSCG_BREAKDOWN : SSCG_OK;
      break;
    }
    s_k = j;
    double q = alpha * p;
    x = x + q;
    L.w[a < MAXK ? a : MAXK] = a < d ? q : 0.0;
    __syncthreads();
    double bq = a < d ? bmul(L.w, a, st, first, bp, L.th) : 0.0;
    __syncthreads();
    r = r - bq;
    double rr1 = quad(L, r, d);
    double beta = rr1 / rr;
    p = r + beta * p;
    if (a == 0) {
      info->alpha[j - 1] = alpha;
      info->beta[j - 1] = beta;
      info->rr_trace[j - 1] = rr1;
    }
    rr = rr1;
    if (prm.adaptive && prm.inner_check) {
      double m0 = (0.0 > rr1) ? 0.0 : rr1;
      double rhs = prm.eps_star / ((c_kj(prm, bnorm, j) * ueps) * sqrt(m0));
      if (gam >= rhs) break;
    }
  }
  // coefficients in the full basis order, zeros elsewhere
  for (int e = a; e < 3 * dfull; e += SSCG_WAVE) coef[e] = 0.0;
  __syncthreads();
  if (a < d) {
    int fa = sub_index(a, st, s, first);
    coef[fa] = x;
    coef[dfull + fa] = r;
    coef[2 * dfull + fa] = p;
  }
  if (a == 0) {
    info->s_tilde = st;
    info->s_k = s_k;
    info->status = status;
    info->d = dfull;
    info->gamma = gam;
    info->thr = thr;
    info->rnorm = rnorm;
    info->rr = rr;
    info->spec = 0;
    if (stop && s_k == 0) *stop = 3;  // no step possible: later kernels stand down
  }
}

__global__ __launch_bounds__(SSCG_WAVE) void k_inner(const double* __restrict__ Gfull,
                                                     sscg_block_params prm,
                                                     double* __restrict__ coef,
                                                     sscg_block_info* info, int* stop) {
  __shared__ InnerLds L;
  if (stop && *stop) return;
  inner_body(L, Gfull, prm, coef, info, stop);
}

// Decisions of a block that ran speculatively (s~ = s, no break): eq. condy
// from the kappa list (same prefix rule and operations as k_inner), then
// eq. check at every iteration before the last from the recorded
// r'^T G r'.  If either would have stopped short of s iterations, or the run
// itself ended early, the speculation is rejected (*stop = 2).  It runs even
// when the solve has already been stopped, so that a later block's result is
// never accepted on top of an unchecked speculation.
__global__ void k_validate(const double* __restrict__ Gfull, sscg_block_params prm,
                           sscg_block_info* info, int* stop) {
  __shared__ double th[SSCG_S_LIMIT];
  if (threadIdx.x < SSCG_S_LIMIT) th[threadIdx.x] = prm.shifts[threadIdx.x];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double ueps = prm.unit_roundoff > 0.0 ? prm.unit_roundoff : EPS;
  const int s = prm.s, first = prm.first;
  const BasisPrm bp = make_basis(prm.basis, prm.lambda_min, prm.lambda_max);
  const double bnorm = prm.c_mode == SSCG_C_THEORY ? b_norm_bound(s, first, bp, th) : 0.0;
  const int dfull = first ? s + 1 : 2 * s + 1;
  const int r0 = first ? 0 : s + 1;
  const double rnorm = sqrt(Gfull[r0 * dfull + r0]);
  const double thr = prm.eps_star / ((c_kj(prm, bnorm, prm.s_max) * ueps) * rnorm);
  int st = 1;
  for (int i = 1; i <= s; ++i) {
    if (sqrt(info->kappa[i - 1]) <= thr) st = i;
    else break;
  }
  const double gam = sqrt(info->kappa[st - 1]);
  bool ok = st == s && info->s_k == s;
  if (ok && prm.inner_check) {
    for (int j = 1; j < s; ++j) {
      const double rr1 = info->rr_trace[j - 1];
      const double m0 = (0.0 > rr1) ? 0.0 : rr1;
      const double rhs = prm.eps_star / ((c_kj(prm, bnorm, j) * ueps) * sqrt(m0));
      if (gam >= rhs) {
        ok = false;
        break;
      }
    }
  }
  info->s_tilde = st;
  info->gamma = gam;
  info->thr = thr;
  info->rnorm = rnorm;
  info->spec = ok ? 1 : 2;
  if (!ok) *stop = 2;
}


// ---------------------------------------------------------------- batches

// Sizes of this block per system: s_bar_k (Alg. 4), the rank guard, and the
// coordinate-solve parameters.
__global__ void k_batch_plan(BatchCfg c) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= c.nsys) return;
  BatchSys& sy = c.sys[q];
  if (sy.done) return;
  int s_bar, s;
  if (c.mode == SSCG_MODE_FIXED) {
    s_bar = s = c.fixed_s;
  } else if (sy.first) {
    s_bar = s = c.s0;
  } else {
    s_bar = min(sy.s_prev + c.f, c.s_max);
    s = min(s_bar, max(sy.m, 1));
  }
  s = min(s, c.S);
  sy.s_bar = s_bar;
  // basis precision of the block (SSCG_PREC_VARIABLE): FP32 when the bound of
  // eq. fb, rearranged for the unit round-off (Section 6's closing remark),
  // admits 2^-24 with the previous block's gamma and the updated residual
  // norm the block starts from; block 0 is FP64
  sy.p32 = 0;
  if (c.vprec && !sy.first) {
    const sscg_block_info& I = c.info[q];
    const double rr = I.rr < 0.0 ? 0.0 : I.rr;  // NaN stays NaN (then FP64)
    sy.p32 = ((EPS32 * c.c) * I.gamma) * sqrt(rr) <= sy.eps_star ? 1 : 0;
  }
  sscg_block_params prm = {};
  prm.s = s;
  prm.first = sy.first;
  prm.adaptive = c.mode == SSCG_MODE_ADAPTIVE ? 1 : 0;
  prm.iters = s;
  prm.inner_check = c.inner_check;
  prm.basis = c.basis;
  prm.lambda_min = sy.lmin;
  prm.lambda_max = sy.lmax;
  prm.eps_star = sy.eps_star;
  prm.c = c.c;
  prm.unit_roundoff = sy.p32 ? EPS32 : 0.0;
  c.prm[q] = prm;
}

// grid (s_max, systems): kappa(G_i) of system blockIdx.y, i = blockIdx.x + 1, on
// NT threads each (BatchCfg::kbt; the bits do not depend on NT).
template <int NT>
__global__ __launch_bounds__(NT) void k_kappa_batch(BatchCfg c) {
  __shared__ JacobiLds L;
  const int q = blockIdx.y, i = blockIdx.x + 1;
  if (c.sys[q].done) return;
  const sscg_block_params prm = c.prm[q];
  if (!prm.adaptive || i > prm.s) return;
  const int d = prm.first ? prm.s + 1 : 2 * prm.s + 1;
  kappa_body<NT>(L, c.G + (int64_t)q * BATCH_GSZ, d, prm.s, prm.first, i, c.info + q);
}

// Coordinate solve of system blockIdx.x, then the block's commit.
__global__ __launch_bounds__(SSCG_WAVE) void k_inner_batch(BatchCfg c) {
  __shared__ InnerLds L;
  const int q = blockIdx.x;
  BatchSys& sy = c.sys[q];
  if (sy.done) return;
  const sscg_block_params& prm = c.prm[q];
  sscg_block_info* info = c.info + q;
  inner_body(L, c.G + (int64_t)q * BATCH_GSZ, prm, c.coef + (int64_t)q * BATCH_CSZ, info,
             nullptr);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int s_k = info->s_k;
    if (sy.blocks < c.cap) {
      BatchHist& h = c.hist[(int64_t)q * c.cap + sy.blocks];
      h.s_bar = sy.s_bar;
      h.s_built = prm.s;
      h.s_tilde = info->s_tilde;
      h.s_k = s_k;
      h.fp32 = sy.p32;
      h.relres_true = __builtin_nan("");
    }
    if (s_k == 0) {  // no step possible: x stays, the system stops
      sy.done = 1;
      sy.status = SSCG_BREAKDOWN;
    } else {
      sy.m += s_k;
      sy.s_prev = s_k;
      sy.blocks += 1;
      sy.first = 0;
    }
  }
}

}  // namespace

hipError_t launch_kappa(const double* G, int d, int s, int first, sscg_block_info* info,
                        const int* stop, hipStream_t st) {
  hipLaunchKernelGGL(k_kappa, dim3(s), dim3(JT), 0, st, G, d, s, first, info, stop);
  return hipGetLastError();
}

hipError_t launch_inner(const double* G, const sscg_block_params& prm, double* coef,
                        sscg_block_info* info, int* stop, hipStream_t st, hipEvent_t done) {
  if (done)
    hipExtLaunchKernelGGL(k_inner, dim3(1), dim3(SSCG_WAVE), 0, st, nullptr, done, 0, G, prm,
                          coef, info, stop);
  else
    hipLaunchKernelGGL(k_inner, dim3(1), dim3(SSCG_WAVE), 0, st, G, prm, coef, info, stop);
  return hipGetLastError();
}

hipError_t launch_validate(const double* G, const sscg_block_params& prm, sscg_block_info* info,
                           int* stop, hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(1), dim3(SSCG_WAVE), 0, st, G, prm, info, stop);
  return hipGetLastError();
}

hipError_t launch_tridiag_eig(const double* alpha, const double* beta, int k, double* lmin,
                              double* lmax, hipStream_t st) {
  hipLaunchKernelGGL(k_tridiag_eig, dim3(1), dim3(JT), 0, st, alpha, beta, k, lmin, lmax);
  return hipGetLastError();
}

hipError_t launch_newton_shifts(const double* alpha, const double* beta, int k, int m, double* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_newton_shifts, dim3(1), dim3(JT), 0, st, alpha, beta, k, m, out);
  return hipGetLastError();
}

hipError_t launch_batch_plan(const BatchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_plan, dim3((c.nsys + 63) / 64), dim3(64), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_kappa_batch(const BatchCfg& c, hipStream_t st) {
  const dim3 grid(c.S, c.nsys);
  switch (c.kbt) {
    case 64: hipLaunchKernelGGL(k_kappa_batch<64>, grid, dim3(64), 0, st, c); break;
    case 192: hipLaunchKernelGGL(k_kappa_batch<192>, grid, dim3(192), 0, st, c); break;
    case 256: hipLaunchKernelGGL(k_kappa_batch<256>, grid, dim3(256), 0, st, c); break;
    default: hipLaunchKernelGGL(k_kappa_batch<128>, grid, dim3(128), 0, st, c); break;
  }
  return hipGetLastError();
}

hipError_t launch_inner_batch(const BatchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_inner_batch, dim3(c.nsys), dim3(SSCG_WAVE), 0, st, c);
  return hipGetLastError();
}
