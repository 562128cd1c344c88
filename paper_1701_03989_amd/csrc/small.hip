// The coordinate problem of one outer block (Algorithm 4 from "Determine s~"
// to the end of the inner loop), solved in LDS by single wavefronts.
//
// k_kappa: kappa(G_i) = lambda_max / lambda_min of every candidate sub-Gram
//   G_i (Section 4.2), one workgroup (one wave) per i, by two-sided cyclic
//   Jacobi with the parallel round-robin ordering (Golub & Van Loan, Sec.
//   8.5).  The operation sequence is fixed (skip rule, rotation formulas,
//   column-then-row application, mirroring of the upper triangle, exact
//   update of the rotated 2x2 blocks), so equal inputs give equal bits.
// k_inner: s~ by eq. condy, B by eq. AVVB, the coordinate recurrence with the
//   break of eq. check; one wave, lane a owns coordinate a.
#include "common.h"

namespace {

constexpr int MAXK = 2 * SSCG_S_LIMIT + 1;  // largest sub-Gram dimension
constexpr int LDK = MAXK + 1;
constexpr double EPS = 0x1p-53;            // unit round-off (Section 5)
constexpr int MAX_SWEEPS = 40;

// Index of sub-basis column a (of G_i) in the full Gram matrix of s steps.
__device__ __forceinline__ int sub_index(int a, int i, int s, int first) {
  if (first || a <= i) return a;
  return s + 1 + (a - i - 1);
}

// Round-robin position of index `pos_i` at step t (m even).
__device__ __forceinline__ int rr_pos(int i, int t, int m) {
  return i == 0 ? 0 : 1 + ((i - 1 + t) % (m - 1));
}

// Eigenvalues of the k x k symmetric matrix in A (LDS, leading dim LDK) by
// cyclic Jacobi; on return the diagonal holds them.  Called by all 64 lanes.
__device__ void jacobi(double (*A)[LDK], double (*B)[LDK], int k, double* wself, double* wother,
                       int* partner, double* rt, double* rapp, double* raqq, double* rapq,
                       int* rp, int* rq, int* nrot) {
  const int lane = threadIdx.x;
  const int m = (k & 1) ? k + 1 : k;
  for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
    int rotated = 0;
    for (int t = 0; t < m - 1; ++t) {
      // rotation parameters, one lane per pair
      if (lane < MAXK) {
        partner[lane] = -1;
      }
      __syncthreads();
      if (lane == 0) *nrot = 0;
      __syncthreads();
      if (lane < m / 2) {
        int a = rr_pos(lane, t, m), b = rr_pos(m - 1 - lane, t, m);
        int p = min(a, b), q = max(a, b);
        int slot = lane;
        rp[slot] = -1;
        if (q < k) {
          double app = A[p][p], aqq = A[q][q], apq = A[p][q];
          double thr = EPS * (sqrt(fabs(app)) * sqrt(fabs(aqq)));
          if (fabs(apq) > thr) {
            double tau = (aqq - app) / (2.0 * apq);
            double tt;
            if (fabs(tau) > 1e150) {
              tt = 0.5 / tau;
            } else {
              double sg = tau >= 0.0 ? 1.0 : -1.0;
              tt = sg / (fabs(tau) + sqrt(1.0 + tau * tau));
            }
            double c = 1.0 / sqrt(1.0 + tt * tt);
            double s = tt * c;
            wself[p] = c;
            wother[p] = -s;
            partner[p] = q;
            wself[q] = c;
            wother[q] = s;
            partner[q] = p;
            rt[slot] = tt;
            rapp[slot] = app;
            raqq[slot] = aqq;
            rapq[slot] = apq;
            rp[slot] = p;
            rq[slot] = q;
            atomicAdd(nrot, 1);
          }
        }
      }
      __syncthreads();
      int nr = *nrot;
      if (nr == 0) continue;
      rotated += nr;
      // B = A J (columns)
      for (int e = lane; e < k * k; e += SSCG_WAVE) {
        int r = e / k, c = e - r * k;
        int pc = partner[c];
        B[r][c] = pc >= 0 ? wself[c] * A[r][c] + wother[c] * A[r][pc] : A[r][c];
      }
      __syncthreads();
      // A = J^T B (rows)
      for (int e = lane; e < k * k; e += SSCG_WAVE) {
        int r = e / k, c = e - r * k;
        int pr = partner[r];
        A[r][c] = pr >= 0 ? wself[r] * B[r][c] + wother[r] * B[pr][c] : B[r][c];
      }
      __syncthreads();
      // mirror the upper triangle
      for (int e = lane; e < k * k; e += SSCG_WAVE) {
        int r = e / k, c = e - r * k;
        if (r > c) A[r][c] = A[c][r];
      }
      __syncthreads();
      // exact 2x2 updates of the rotated pairs (start-of-step values)
      if (lane < m / 2 && rp[lane] >= 0) {
        int p = rp[lane], q = rq[lane];
        double tt = rt[lane];
        A[p][p] = rapp[lane] - tt * rapq[lane];
        A[q][q] = raqq[lane] + tt * rapq[lane];
        A[p][q] = 0.0;
        A[q][p] = 0.0;
      }
      __syncthreads();
    }
    if (rotated == 0) break;
  }
}

struct JacobiLds {
  double A[MAXK][LDK];
  double B[MAXK][LDK];
  double wself[MAXK + 1], wother[MAXK + 1];
  int partner[MAXK + 1];
  double rt[MAXK], rapp[MAXK], raqq[MAXK], rapq[MAXK];
  int rp[MAXK], rq[MAXK];
  int nrot;
};

__device__ double kappa_from_diag(double (*A)[LDK], int k) {
  double lmin = A[0][0], lmax = A[0][0];
  bool nan = lmin != lmin;
  for (int a = 1; a < k; ++a) {
    double v = A[a][a];
    if (v != v) nan = true;
    lmin = v < lmin ? v : lmin;
    lmax = v > lmax ? v : lmax;
  }
  if (nan || !(lmin > 0.0) || isinf(lmax)) return __builtin_inf();
  return lmax / lmin;
}

// grid = s workgroups of one wave; workgroup i-1 computes kappa(G_i).
__global__ __launch_bounds__(SSCG_WAVE) void k_kappa(const double* __restrict__ G, int d, int s,
                                                     int first, sscg_block_info* info) {
  __shared__ JacobiLds L;
  int i = blockIdx.x + 1;
  int k = first ? i + 1 : 2 * i + 1;
  for (int e = threadIdx.x; e < k * k; e += SSCG_WAVE) {
    int a = e / k, b = e - a * k;
    L.A[a][b] = G[sub_index(a, i, s, first) * d + sub_index(b, i, s, first)];
  }
  __syncthreads();
  jacobi(L.A, L.B, k, L.wself, L.wother, L.partner, L.rt, L.rapp, L.raqq, L.rapq, L.rp, L.rq,
         &L.nrot);
  if (threadIdx.x == 0) info->kappa[i - 1] = kappa_from_diag(L.A, k);
}

// Eigenvalue extremes of the Lanczos tridiagonal matrix (k <= MAXK).
__global__ __launch_bounds__(SSCG_WAVE) void k_tridiag_eig(const double* __restrict__ alpha,
                                                           const double* __restrict__ beta, int k,
                                                           double* lmin, double* lmax) {
  __shared__ JacobiLds L;
  for (int e = threadIdx.x; e < k * k; e += SSCG_WAVE) {
    int a = e / k, b = e - a * k;
    double v = 0.0;
    if (a == b) v = alpha[a];
    else if (b == a + 1) v = beta[a];
    else if (a == b + 1) v = beta[b];
    L.A[a][b] = v;
  }
  __syncthreads();
  if (k > 1)
    jacobi(L.A, L.B, k, L.wself, L.wother, L.partner, L.rt, L.rapp, L.raqq, L.rapq, L.rp, L.rq,
           &L.nrot);
  if (threadIdx.x == 0) {
    double lo = L.A[0][0], hi = L.A[0][0];
    for (int a = 1; a < k; ++a) {
      lo = L.A[a][a] < lo ? L.A[a][a] : lo;
      hi = L.A[a][a] > hi ? L.A[a][a] : hi;
    }
    *lmin = lo;
    *lmax = hi;
  }
}

// ---------------------------------------------------------------- inner loop

// CR dot of lane-owned values over the wave (lanes >= d hold zeros).
__device__ __forceinline__ double wave_dot(double x, double y) {
  dd a = dd_zero();
  dd_add_prod(a, x, y);
  a = dd_wave_reduce(a);
  return dd_round(a);
}

// (B v)_a for the s-step basis of s steps (first: P block only), R12 layout.
__device__ __forceinline__ double bmul(const double* v, int a, int s, int first, BasisPrm bp) {
  // block offset, local index and block length
  int off = 0, len = s + 1;
  if (!first && a > s) {
    off = s + 1;
    len = s;
  }
  int j = a - off;
  double th = bp.cheb ? bp.c0 : 0.0;
  dd acc = dd_zero();
  // B[a][a-1] = gamma_{j-1}: column j-1 is not the block's last
  if (j >= 1) {
    double g = bp.cheb ? (j - 1 == 0 ? bp.h : bp.h2) : 1.0;
    dd_add_prod(acc, g, v[a - 1]);
  }
  // B[a][a] = theta_j if column j is not the last
  if (j < len - 1) dd_add_prod(acc, th, v[a]);
  // B[a][a+1] = sigma_j if column j+1 is not the last
  if (j + 1 < len - 1) dd_add_prod(acc, bp.cheb ? bp.h2 : 0.0, v[a + 1]);
  return dd_round(acc);
}

struct InnerLds {
  double G[MAXK][LDK];
  double v[MAXK + 1];
  double w[MAXK + 1];
};

// (G v)_a then v . (G v), with v held one value per lane.
__device__ __forceinline__ double quad(InnerLds& L, double va, int d) {
  int a = threadIdx.x;
  if (a < SSCG_WAVE) L.v[a < MAXK ? a : MAXK] = a < d ? va : 0.0;
  __syncthreads();
  double gv = 0.0;
  if (a < d) {
    dd acc = dd_zero();
    for (int b = 0; b < d; ++b) dd_add_prod(acc, L.G[a][b], L.v[b]);
    gv = dd_round(acc);
  }
  __syncthreads();
  return wave_dot(a < d ? va : 0.0, gv);
}

__global__ __launch_bounds__(SSCG_WAVE) void k_inner(const double* __restrict__ Gfull,
                                                     sscg_block_params prm,
                                                     double* __restrict__ coef,
                                                     sscg_block_info* info) {
  __shared__ InnerLds L;
  const int a = threadIdx.x;
  const int s = prm.s, first = prm.first;
  const int dfull = first ? s + 1 : 2 * s + 1;
  BasisPrm bp = make_basis(prm.basis, prm.lambda_min, prm.lambda_max);

  double gam = __builtin_nan(""), thr = __builtin_nan(""), rnorm = __builtin_nan("");
  int st;
  if (prm.adaptive) {
    int r0 = first ? 0 : s + 1;
    rnorm = sqrt(Gfull[r0 * dfull + r0]);
    thr = prm.eps_star / ((prm.c * EPS) * rnorm);
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
    double bpv = a < d ? bmul(L.w, a, st, first, bp) : 0.0;
    __syncthreads();
    // p . G (B p)
    L.v[a < MAXK ? a : MAXK] = a < d ? bpv : 0.0;
    __syncthreads();
    double gbp = 0.0;
    if (a < d) {
      dd acc = dd_zero();
      for (int b = 0; b < d; ++b) dd_add_prod(acc, L.G[a][b], L.v[b]);
      gbp = dd_round(acc);
    }
    __syncthreads();
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
    double bq = a < d ? bmul(L.w, a, st, first, bp) : 0.0;
    __syncthreads();
    r = r - bq;
    double rr1 = quad(L, r, d);
    double beta = rr1 / rr;
    p = r + beta * p;
    if (a == 0) {
      info->alpha[j - 1] = alpha;
      info->beta[j - 1] = beta;
    }
    rr = rr1;
    if (prm.adaptive && prm.inner_check) {
      double m0 = (0.0 > rr1) ? 0.0 : rr1;
      double rhs = prm.eps_star / ((prm.c * EPS) * sqrt(m0));
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
  }
}

}  // namespace

hipError_t launch_kappa(const double* G, int d, int s, int first, sscg_block_info* info,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_kappa, dim3(s), dim3(SSCG_WAVE), 0, st, G, d, s, first, info);
  return hipGetLastError();
}

hipError_t launch_inner(const double* G, const sscg_block_params& prm, double* coef,
                        sscg_block_info* info, hipStream_t st) {
  hipLaunchKernelGGL(k_inner, dim3(1), dim3(SSCG_WAVE), 0, st, G, prm, coef, info);
  return hipGetLastError();
}

hipError_t launch_tridiag_eig(const double* alpha, const double* beta, int k, double* lmin,
                              double* lmax, hipStream_t st) {
  hipLaunchKernelGGL(k_tridiag_eig, dim3(1), dim3(SSCG_WAVE), 0, st, alpha, beta, k, lmin, lmax);
  return hipGetLastError();
}
