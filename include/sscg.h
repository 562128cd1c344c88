/*
 * sscg.h -- C ABI of the adaptive s-step conjugate gradient library
 * (E. Carson, "The adaptive s-step conjugate gradient method", arXiv 1701.03989)
 * for AMD Instinct MI355X (gfx950).  Implementation: libsscg.so, hand-written HIP.
 *
 * Problem (Section 1): solve A x = b for a sparse symmetric positive definite
 * A given in CSR form.  sscg_solve runs Algorithm 4 (adaptive s-step CG), or
 * Algorithm 2 (fixed s) or Algorithm 3 (given schedule of s values), and
 * returns x, the s_k schedule and the residual history.  The per-stage calls
 * run one step of an outer block (Algorithm 4) on caller-provided device
 * buffers.
 *
 * Conventions for every call
 *  - All matrix and vector pointers are DEVICE pointers (hipMalloc'd or torch
 *    tensors' data_ptr()) unless a comment says "host".  The caller owns them;
 *    the library never frees or reallocates caller memory.
 *  - FP64 throughout.  Every row sum, inner product and row-wise linear
 *    combination is rounded once from its exact value (the terms' products
 *    enter exactly), so results do not depend on the order of the terms.
 *  - Work is enqueued on the context's stream.  Per-stage calls return once
 *    their kernels are enqueued; sscg_solve and sscg_spectral_bounds return
 *    after the stream has finished the call's work.
 *  - Return value: SSCG_OK (0), or a positive numerical outcome (x is valid,
 *    the history is complete), or a negative error code, in which case no
 *    caller buffer has been written and sscg_last_error() says why.
 *  - A context is used by one host thread at a time.
 */
#ifndef SSCG_H
#define SSCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
  SSCG_OK = 0,             /* true relative residual <= tol                   */
  SSCG_NOT_CONVERGED = 1,  /* max_iters inner iterations done, tol not reached */
  SSCG_BREAKDOWN = 2,      /* a block could not take one step (p'^T G B p' <= 0
                              or non-finite), or the residual became non-finite */
  SSCG_ERR_ARG = -1,       /* invalid argument (message in sscg_last_error)    */
  SSCG_ERR_HIP = -2,       /* HIP runtime error                               */
  SSCG_ERR_OOM = -3        /* device allocation failed                        */
};

enum { SSCG_MODE_ADAPTIVE = 0, SSCG_MODE_FIXED = 1, SSCG_MODE_SCHEDULE = 2 };
enum { SSCG_BASIS_MONOMIAL = 0, SSCG_BASIS_CHEBYSHEV = 1, SSCG_BASIS_NEWTON = 2 };
/* c_{k,j} of eqs. condy and check: the constant opts->c, or the value the
 * bound of Section 4.1 gives, 6 N_k j kappa(A) with N_k = 7 + 2 N_A +
 * 14 ||B_k|| / ||A|| (N_A: most nonzeros in a row of A; ||B_k|| bounded by
 * sqrt(||B||_1 ||B||_inf) of the block's built basis; eq. condy takes
 * j = s_max). */
enum { SSCG_C_CONST = 0, SSCG_C_THEORY = 1 };

/* Largest s the library accepts: the (2s+1)-dimensional coordinate problem
 * of a block is solved by one wavefront. */
#define SSCG_S_LIMIT 16

/* ---------------------------------------------------------------- types */
typedef struct sscg_ctx sscg_ctx;

/* Sparse SPD matrix in CSR form (device arrays).  rowptr[0] = 0, rowptr
 * non-decreasing, rowptr[n] = nnz; col entries in [0, n).  Only the values
 * are read as given: symmetry and positive definiteness are the caller's
 * promise (a violation shows up as SSCG_BREAKDOWN or SSCG_NOT_CONVERGED).
 * nnz is 64-bit; with the 32-bit rowptr of this form it must stay below 2^31,
 * and 1 <= n <= 2^31 - 4096 (row indices padded to whole slices and pairs of
 * slices stay in the int range); other values are rejected with
 * SSCG_ERR_ARG. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t* rowptr; /* n+1 */
  const int32_t* col;    /* nnz */
  const double* val;     /* nnz */
} sscg_csr;

/* Inputs of Algorithm 4 (its Require line) plus the basis choice. */
typedef struct {
  int32_t mode;          /* SSCG_MODE_*                                          */
  int32_t basis;         /* SSCG_BASIS_* (Sections 2 and 5 name both)            */
  double tol;            /* target relative residual; eps* = tol*||b||_2          */
  int32_t s_max;         /* 1..SSCG_S_LIMIT                                      */
  int32_t s0_bar;        /* initial basis size (0: s_max, as in Section 5)        */
  int32_t f;             /* basis growth limit (0: s_max, as in Section 5)        */
  int32_t fixed_s;       /* MODE_FIXED: s of Algorithm 2                          */
  const int32_t* schedule; /* host; MODE_SCHEDULE: s_0, s_1, ... (the last repeats) */
  int32_t schedule_len;
  double c;              /* constant c_{k,j} of eqs. condy/check (default 1)      */
  double lambda_min;     /* Chebyshev interval; NaN: estimated by                 */
  double lambda_max;     /*   sscg_spectral_bounds (Lanczos / Gershgorin)         */
  int32_t lanczos_steps; /* steps of that estimate (default 30)                   */
  uint64_t lanczos_seed; /* SplitMix64 seed of its start vector (default 0)       */
  int32_t equilibrate;   /* 1: solve D^-1/2 A D^-1/2 (Section 5), D_i = max|a_ij| */
  int32_t inner_check;   /* 1: in-loop break of eq. check (Alg. 4); 0: s_k = s~   */
  int32_t max_iters;     /* cap on total inner iterations                         */
  int32_t c_mode;        /* SSCG_C_CONST (default) or SSCG_C_THEORY               */
  double kappa_a;        /* THEORY: kappa(A) and ||A||_2; NaN: lambda_max/lambda_min */
  double norm_a;         /*   and lambda_max of the spectral estimate              */
  const double* shifts;  /* host; BASIS_NEWTON: s_max shifts theta_0, theta_1, ...;
                            NULL: sscg_newton_shifts(m = s_max, lanczos_seed)     */
  int32_t precision;    /* SSCG_PREC_FP64; SSCG_PREC_MIXED (sscg_solve only): FP64
                            iterative refinement around FP32-basis solves;
                            SSCG_PREC_VARIABLE: the basis precision chosen per
                            outer block                                          */
  int32_t max_outer;     /* MIXED: cap on refinement steps (default 30)          */
  double inner_tol;      /* MIXED: each inner solve reduces its residual by this
                            factor (default 1e-5)                                  */
} sscg_opts;

/* Precision of sscg_solve.  MIXED: x_{j+1} = x_j + d_j, r_j = b - A x_j in FP64,
 * where d_j approximately solves A d = r_j by adaptive s-step CG with the
 * matrix powers and the basis in FP32 (each row sum accumulated in FP64 from
 * exact products and rounded once to FP32), the Gram matrix of the FP32 basis
 * from exact products accumulated in FP64, and the coefficient recurrence,
 * kappa estimates (unit round-off 2^-24 in eqs. condy and check) and d_j in
 * FP64.  Stops when ||r_j|| / ||b|| <= tol, measured on the caller's system
 * A x = b also when equilibrating (the refinement is not part of Algorithm 4,
 * so the scaled-system reading of Section 5 does not apply to its stopping
 * test).  Supported by sscg_solve only.  The result field `iters` counts
 * inner iterations of all refinement steps, `blocks` their outer blocks. */
/* VARIABLE (batches, servers, and sscg_solve as a batch of one system with no
 * equilibration, whose history then leaves s_bar, s_built, gamma, thr,
 * res_updated and kappa unset; adaptive mode, constant c): the
 * mixed-precision method of Section 6's closing remark, which rearranges the
 * residual-gap bound eq. fb into eps_k <= eps* / (c kappa(Y_k) max ||r^||), the
 * largest unit round-off outer loop k may use.  Block k >= 1 stores its basis
 * in FP32 when ((2^-24 c) gamma_{k-1}) ||r^|| <= eps*, with gamma_{k-1} the
 * previous block's estimate of kappa(Y) (eq. yhk1) and ||r^|| = (r'^T G r')^(1/2)
 * the updated residual norm it ended with; block 0 and the others are FP64.
 * In an FP32 block each basis column (P_0 = RN32(p), R_0 = RN32(r) and every
 * matrix-powers output) is the FP64 value rounded once to FP32, computed from
 * the stored FP32 columns with the FP64 matrix; the Gram matrix (exact
 * products of the widened columns), kappa, the coefficient recurrence and the
 * recovery of x, r, p stay FP64, and eqs. condy and check use 2^-24.  No
 * restart: x, r, p carry over between blocks of either precision, and the
 * stopping test is the FP64 true residual as in Algorithm 4. */
enum { SSCG_PREC_FP64 = 0, SSCG_PREC_MIXED = 1, SSCG_PREC_VARIABLE = 2 };

/* Per-solve outputs.  The arrays are HOST memory owned by the caller, each
 * with room for `cap` blocks (any may be NULL); entry k describes outer
 * block k.  Blocks beyond `cap` are still run, only not recorded. */
typedef struct {
  int32_t cap;
  int32_t blocks;        /* outer blocks run (= global synchronizations)          */
  int32_t iters;         /* inner iterations run, m                               */
  int32_t status;        /* same as the return value                              */
  double relres0;        /* ||b - A x_1|| / ||b||                                 */
  double relres;         /* ||b - A x|| / ||b|| of the returned x                  */
  double lambda_min, lambda_max;   /* Chebyshev interval used                      */
  int64_t basis_vectors;           /* matrix-vector products of all bases          */
  int64_t wasted_vectors;          /* of those, products not needed by s_k steps   */
  int32_t* s_bar;        /* s_bar_k of Alg. 4 (s of Alg. 2/3)                      */
  int32_t* s_built;      /* basis steps built, after the rank guard                */
  int32_t* s_tilde;      /* s~_k chosen by eq. condy                               */
  int32_t* s_k;          /* inner iterations performed                            */
  double* gamma;         /* estimate of kappa(Y_{k,s~}) (NaN unless adaptive)       */
  double* thr;           /* right-hand side of eq. condy                           */
  double* res_updated;   /* (r'^T G r')^(1/2) after the block                      */
  double* relres_true;   /* ||b - A x|| / ||b|| after the block                    */
  double* kappa;         /* cap*s_max: kappa(G_{k,i}), i = 1..s_max (NaN if not
                            computed); row k at kappa + k*s_max                    */
  int32_t spec_blocks;   /* blocks run ahead speculatively (s_k = s assumed while
                            the exact s~/break decisions ran alongside)           */
  int32_t spec_rejected; /* of those, blocks redone because the decisions differed */
  int32_t* fp32;         /* 1 where the block's basis was FP32 (SSCG_PREC_VARIABLE)  */
} sscg_result;

/* Device-side record of one block's coordinate solve (sscg_small_solve). */
typedef struct {
  int32_t s_tilde;       /* s~ (eq. condy), or the given iteration count          */
  int32_t s_k;           /* iterations performed                                  */
  int32_t status;        /* SSCG_OK or SSCG_BREAKDOWN                             */
  int32_t d;             /* dimension of the coefficient vectors (2s+1 or s+1)    */
  double gamma;          /* sqrt(kappa(G_{s~})) (adaptive)                        */
  double thr;            /* eps* / (c eps ||r_{m+1}||) (adaptive)                  */
  double rnorm;          /* ||r_{m+1}|| = sqrt(G[R0,R0]) (block 0: G[P0,P0])       */
  double rr;             /* r'^T G r' after the last iteration                    */
  double kappa[SSCG_S_LIMIT];      /* kappa(G_i), i = 1..s (adaptive)              */
  double alpha[SSCG_S_LIMIT];      /* alpha_{m+j}, j = 1..s_k                      */
  double beta[SSCG_S_LIMIT];       /* beta_{m+j}                                   */
  double rr_trace[SSCG_S_LIMIT];   /* r'^T G r' after iteration j = 1..s_k         */
  double relres_in;      /* sscg_solve only: ||b - A x|| / ||b|| of the block's start */
  int32_t spec;          /* sscg_solve only: 0 run directly, 1 speculative and
                            confirmed, 2 speculative and rejected (block redone)  */
  int32_t pad_;
} sscg_block_info;

/* Parameters of one block's coordinate solve. */
typedef struct {
  int32_t s;             /* basis steps built (s_bar after the rank guard)        */
  int32_t first;         /* 1 in block 0: basis is P_0..P_s only                   */
  int32_t adaptive;      /* 1: choose s~ <= s by eq. condy; 0: s~ = iters          */
  int32_t iters;         /* iterations when !adaptive (1 <= iters <= s)            */
  int32_t inner_check;   /* adaptive: break by eq. check                          */
  int32_t basis;         /* SSCG_BASIS_*                                          */
  double lambda_min, lambda_max;   /* Chebyshev interval                           */
  double eps_star;       /* tol * ||b||                                           */
  double c;              /* c_{k,j} (c_mode CONST)                                */
  double unit_roundoff;  /* eps of eqs. condy and check (0: 2^-53)                */
  int32_t c_mode;        /* SSCG_C_CONST or SSCG_C_THEORY                         */
  int32_t n_a;           /* THEORY: most nonzeros in a row of A                   */
  int32_t s_max;         /* THEORY: eq. condy uses c_{k,s_max}                    */
  int32_t pad_;
  double kappa_a, norm_a;          /* THEORY: kappa(A), ||A||_2                    */
  double shifts[SSCG_S_LIMIT];     /* BASIS_NEWTON: theta_0, theta_1, ...          */
} sscg_block_params;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues on `stream` (a
 * hipStream_t; NULL = the null stream).  The context owns its workspace. */
int sscg_create(sscg_ctx** ctx, int device, void* stream);
void sscg_destroy(sscg_ctx* ctx);
/* Message of the last failing call on ctx ("" if none).  Valid until the
 * next call on ctx.  sscg_last_error(NULL) reports sscg_create failures. */
const char* sscg_last_error(const sscg_ctx* ctx);
/* Fill *opts with the defaults of Section 5 (adaptive, monomial, tol 1e-10,
 * s_max 8, s0_bar = f = s_max, c = 1, inner checks on, no equilibration). */
void sscg_opts_default(sscg_opts* opts);

/* ---------------------------------------------------------------- solver */

/* Algorithm 4 (opts->mode = ADAPTIVE), 2 (FIXED) or 3 (SCHEDULE) on A x = b.
 * b: device, n.  x: device, n; x_1 on entry, the solution on return.
 * res: may be NULL.  Block 0 builds the P block only (p_1 = r_1); later
 * blocks build min(s_bar_k, m) steps (m = iterations so far), since a larger
 * basis of the same Krylov space is rank deficient.  The solve stops after the
 * first block whose true relative residual is <= tol. */
int sscg_solve(sscg_ctx* ctx, const sscg_csr* A, const double* b, double* x,
               const sscg_opts* opts, sscg_result* res);

/* ---------------------------------------------------------------- stages */

/* Setup (Algorithm 4, first line): r = b - A x, and on the device
 * out2[0] = ||r||^2, out2[1] = ||b||^2 (device, 2 doubles).  r may be NULL. */
int sscg_residual(sscg_ctx* ctx, const sscg_csr* A, const double* b, const double* x,
                  double* r, double* out2);

/* Chebyshev interval: *lambda_max = max_i sum_j |a_ij| (Gershgorin) and
 * *lambda_min = smallest Ritz value of `steps` Lanczos steps started from the
 * SplitMix64(seed) vector u_i = (z_i >> 11) 2^-52 - 1.  Host outputs. */
int sscg_spectral_bounds(sscg_ctx* ctx, const sscg_csr* A, int steps, uint64_t seed,
                         double* lambda_min, double* lambda_max);
/* Shifts of the Newton basis: the Ritz values of an m-step Lanczos run
 * (m <= SSCG_S_LIMIT, start vector as for sscg_spectral_bounds), eigenvalues of
 * the tridiagonal matrix by the Jacobi method of the kappa estimates, sorted
 * ascending and then Leja ordered (first the largest in modulus, then each
 * maximising the product of distances to those already chosen, ties to the
 * earlier); repeated cyclically if the run ended early.  shifts: host, m. */
int sscg_newton_shifts(sscg_ctx* ctx, const sscg_csr* A, int m, uint64_t seed, double* shifts);

/* The device form of A that the stages build and read (not an operation of the
 * method: for callers that budget memory or bandwidth, or check which form a
 * matrix gets).  A is stored as SELL-64: slices of 64 consecutive rows, each
 * padded with zeros to its longest row; *stored gets the padded entry count.
 * *format gets SSCG_FMT_COL16 when every column index lies within 32767 of its
 * slice's first row: the matrix-powers pass then reads 16-bit offsets instead
 * of 32-bit indices.  It also gets SSCG_FMT_VTAB when, in addition, no slice
 * holds more than four distinct values, padding zeros included and compared
 * bit for bit: the pass then reads a one-byte index per entry into a per-slice
 * table of those values (the same bits, so no result changes).  Host outputs;
 * either may be NULL. */
#define SSCG_FMT_COL16 1
#define SSCG_FMT_VTAB 2
/* SSCG_FMT_SDIA: every slice couples its rows to at most 8 column distances
 * d = col - row and holds at most 3 distinct values (padding excluded), and
 * no row has two entries at one distance (stencils): the matrix-powers pass
 * then reads, per slice, the distances and values, and per row one 16-bit
 * word with a 2-bit value code per distance (2 bytes of A per row), and
 * gathers row i's inputs at i + d without loading an index.  It takes
 * precedence over the other forms; the same bits result. */
#define SSCG_FMT_SDIA 4
/* SSCG_FMT_SDPAIR (with SSCG_FMT_SDIA, n >= 2): for every t, slices 2 t and
 * 2 t + 1 (rows 128 t .. 128 t + 127) have the same distances and the same
 * values, bit for bit, so the pass takes such a pair in one wavefront, two
 * rows per lane, with 16-byte loads.  The same bits result. */
#define SSCG_FMT_SDPAIR 8
/* SSCG_FMT_SDVAL (with SSCG_FMT_SDIA): in every slice, all rows with an
 * entry at a given distance have the same value there (stencils with
 * constant coefficients): the pass then takes each distance's value from
 * scalar registers instead of decoding it per row.  With SSCG_FMT_SDPAIR as
 * well, the two slices of each pair also agree on these values (else the
 * pairs are not used).  The same bits result. */
#define SSCG_FMT_SDVAL 16
int sscg_matrix_format(sscg_ctx* ctx, const sscg_csr* A, int* format, int64_t* stored);
/* Which of the compact forms above the context's later calls may build and
 * read (bit mask of SSCG_FMT_*, default all five; 0 = the stored FP64 values
 * with 32-bit indices).  For timing and testing the forms against each
 * other: every form gives the same bits.  Value tables are only used together
 * with 16-bit offsets.  The pair and per-distance value forms serve the FP64
 * passes of single systems (sscg_solve, sscg_mpk, sscg_mpk_newton); the FP32
 * passes, batches and servers read the slice-diagonal form one slice per
 * wavefront with per-row value codes. */
int sscg_set_forms(sscg_ctx* ctx, int forms);

/* Matrix powers (eqs. cg-krylovbasis, polybasiscg): Y is n x ncol, column-major
 * with leading dimension ldy >= n.  On entry column 0 holds p (P_0) and, unless
 * first, column rcol holds r (R_0).  On return columns 1..s hold
 * P_j = rho_j(A) p and, unless first, columns rcol+1..rcol+s-1 hold
 * R_j = rho_j(A) r, with rho_j from the three-term recurrence of `basis` on
 * [lambda_min, lambda_max] (ignored for the monomial basis).  Needs
 * 1 <= s <= SSCG_S_LIMIT and, unless first, rcol >= s+1. */
int sscg_mpk(sscg_ctx* ctx, const sscg_csr* A, int s, int first, int basis,
             double lambda_min, double lambda_max, double* Y, int64_t ldy, int rcol);

/* sscg_mpk for the Newton basis (Section 2): P_j = (A - theta_{j-1} I) P_{j-1},
 * likewise R_j, each row rounded once.  shifts: host, s values theta_0..
 * theta_{s-1}. */
int sscg_mpk_newton(sscg_ctx* ctx, const sscg_csr* A, int s, int first, const double* shifts,
                    double* Y, int64_t ldy, int rcol);

/* Gram matrix (Section 2, Algorithm 4): G = Y_s^T Y_s of the basis columns
 * [P_0..P_s, R_0..R_{s-1}] (first: [P_0..P_s]) laid out as in sscg_mpk.
 * G: device, d x d with d = 2s+1 (first: s+1), both triangles written. */
int sscg_gram(sscg_ctx* ctx, int n, int s, int first, const double* Y, int64_t ldy, int rcol,
              double* G);

/* sscg_gram for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same G, bit for bit, with the partial sums held in a
 * fixed 8 MiB device array of the library (one per GPU, kept until the
 * process ends, its address looked up by sscg_create) instead of the
 * context's growable workspace.  Allocates nothing; enqueues on the
 * context's stream like sscg_gram.  Limit: d(d+1)/2 * ceil(n / 1024) <= 2^20
 * (d = 2s+1, or s+1 when first; e.g. n <= 4.6 M rows at s = 10, 1.9 M at
 * s = 16); larger calls return SSCG_ERR_ARG.  Arguments as for sscg_gram.
 * Calls on one GPU share the array: calls that overlap in time on that GPU
 * (other streams, other contexts, other threads) race and must be
 * serialised by the caller. */
int sscg_gram_noalloc(sscg_ctx* ctx, int n, int s, int first, const double* Y, int64_t ldy,
                      int rcol, double* G);

/* One block's coordinate solve (Algorithm 4 from "Determine s~" to the end
 * of the inner loop): kappa(G_i) for i = 1..s (Jacobi eigenvalues, when
 * adaptive), s~ by eq. condy, B (eq. AVVB), the inner recurrence with the
 * break of eq. check.  G: device d x d from sscg_gram.  Outputs (device):
 * coef[0:d] = x', coef[d:2d] = r', coef[2d:3d] = p' in the order of G's
 * columns; *info. */
int sscg_small_solve(sscg_ctx* ctx, const double* G, const sscg_block_params* prm,
                     double* coef, sscg_block_info* info);

/* Recovery (eq. coords): x <- x + Y x', r <- Y r', p <- Y p' with Y and the
 * coefficient layout of sscg_gram / sscg_small_solve.  r and p may alias
 * columns of Y (each row is read before it is written). */
int sscg_recover(sscg_ctx* ctx, int n, int s, int first, const double* Y, int64_t ldy, int rcol,
                 const double* coef, double* x, double* r, double* p);

/* The FP32 stages of SSCG_PREC_MIXED (same layouts as sscg_mpk and sscg_gram,
 * float basis).  sscg_mpk32: the s passes on the FP32 copy of A's values,
 * each row sum accumulated in FP64 from the exact products of FP32 values
 * (in the row's CSR order), the three-term correction and the division by
 * gamma in FP64, then rounded once to FP32.  sscg_gram32: G = Y^T Y of the
 * FP32 columns (exact products, FP64 sums; d x d FP64, both triangles). */
int sscg_mpk32(sscg_ctx* ctx, const sscg_csr* A, int s, int first, int basis, double lambda_min,
               double lambda_max, float* Y, int64_t ldy, int rcol);
int sscg_gram32(sscg_ctx* ctx, int n, int s, int first, const float* Y, int64_t ldy, int rcol,
                double* G);

/* ---------------------------------------------------------------- batches */

/* Independent systems A_i x_i = b_i solved side by side, each by the same
 * algorithm as sscg_solve (Algorithm 4, or 2 with opts->mode = FIXED) and to
 * the same numbers: every stage of an outer block runs as one launch over all
 * systems (a block-diagonal layout; each system's s_bar_k, s~_k, s_k, m and
 * convergence are decided on the device), and the launches of one outer
 * block are replayed as a HIP graph until every system has finished.
 * Systems may differ in size, matrix and tolerance.  Not supported in a
 * batch: MODE_SCHEDULE, equilibration, and the Chebyshev interval estimate
 * (intervals are inputs).  All arrays of this struct are HOST arrays of
 * length nsys; the pointers they hold are DEVICE pointers owned by the
 * caller. */
typedef struct {
  int32_t nsys;
  const sscg_csr* A;          /* system matrices                                      */
  const double* const* b;     /* right-hand sides (n_i each)                          */
  double* const* x;           /* x_1 on entry, the solution on return (n_i each)      */
  const double* tol;          /* per-system target relative residual (NULL: opts->tol) */
  const double* lambda_min;   /* Chebyshev intervals (required for BASIS_CHEBYSHEV)   */
  const double* lambda_max;
} sscg_batch;

/* Per-system outputs: HOST arrays owned by the caller (any may be NULL);
 * the per-block arrays hold `cap` rows per system, system i at i*cap. */
typedef struct {
  int32_t cap;
  int32_t* status;        /* [nsys] SSCG_OK / NOT_CONVERGED / BREAKDOWN             */
  int32_t* blocks;        /* [nsys] outer blocks of the system                      */
  int32_t* iters;         /* [nsys] inner iterations m                             */
  double* relres;         /* [nsys] ||b - A x|| / ||b|| of the returned x            */
  int32_t* s_k;           /* [nsys*cap] schedule                                    */
  int32_t* s_tilde;       /* [nsys*cap] s~_k of eq. condy                           */
  double* relres_true;    /* [nsys*cap] true relative residual after each block     */
  int32_t graph_launches; /* outer blocks replayed (all systems together)           */
  int32_t rows;           /* rows of the batch layout (each system padded to 256)    */
  int32_t* fp32;          /* [nsys*cap] 1 where the block's basis was FP32 (VARIABLE) */
} sscg_batch_result;

/* Returns SSCG_OK when every system converged, else the largest positive
 * per-system status; negative codes as for sscg_solve (no x written). */
int sscg_batch_solve(sscg_ctx* ctx, const sscg_batch* batch, const sscg_opts* opts,
                     sscg_batch_result* res);

/* Launch shapes of sscg_batch_solve (a tuner written for this library; no
 * result bit depends on the shapes, only the time does).  Three shapes are
 * tuned: the entries of a row whose loads a matrix-powers pass issues
 * together (2, 4 or 8), the threads of each kappa(G_i) problem (64, 128, 192
 * or 256; the Jacobi sweeps of Section 4.2's condition numbers) and the
 * wavefronts per Gram workgroup (1, 2 or 4; one 1024-row group each).
 * mode 1 (the default): after a batch's first four blocks every candidate of
 * the next block's first pass, kappa and Gram launches is timed three times
 * on the live state and the fastest is kept, once per batch shape (total
 * rows, systems, s_max) and context; later batches of that shape reuse the
 * choice.  mode 0: use kappa_threads, gram_waves and mpk_chunk as given (0:
 * 128, 4 and 4).  Either call clears the remembered choices.  SSCG_ERR_ARG
 * for another mode or shape. */
int sscg_set_batch_tuning(sscg_ctx* ctx, int mode, int kappa_threads, int gram_waves,
                          int mpk_chunk);
/* The shapes the last sscg_batch_solve ran with and, if it timed them, the
 * fastest of three runs of each candidate in microseconds (kappa_us[4] for
 * 64, 128, 192, 256 threads; gram_us[3] for 1, 2, 4 wavefronts; mpk_us[3]
 * for chunks of 2, 4, 8; NaN where not timed).  Any output may be NULL. */
int sscg_batch_tuning(sscg_ctx* ctx, int32_t* kappa_threads, int32_t* gram_waves,
                      int32_t* mpk_chunk, double* kappa_us, double* gram_us, double* mpk_us);

/* ---------------------------------------------------------------- serving */

/* A solve server: continuous batching of independent systems on one GPU.
 * Requests are queued by sscg_server_submit and admitted first come, first
 * served, as soon as a slot and room in the pools are free (admission by
 * device-memory footprint: the request's SELL-64 matrix in the nnz pool and
 * its rows, padded to 1024, in the row pool, which holds the 2 s_max + 3
 * vectors of every row).  Each sscg_server_step runs one outer block for all
 * admitted systems (the same batched launches as sscg_batch_solve, replayed
 * from one HIP graph; its row launches take the admitted systems' rows only,
 * wherever they sit in the pool), retires finished systems (x is
 * copied back to the caller's buffer before the step returns) and admits
 * waiting ones; their work overlaps on the device.  A step returns while its
 * block still runs (at most two blocks are in flight), so a system is seen
 * finished, and retired, one or two steps after the block that finished it.  Each result is the one
 * sscg_solve gives for that system alone.  Options as for batches
 * (MODE_SCHEDULE and equilibration are not supported). */
typedef struct sscg_server sscg_server;

/* pool_rows: rows of all admitted systems together (each padded to 1024);
 * pool_nnz: SELL-64 entries of all admitted matrices; slots: admitted
 * systems at once.  The server owns its device memory and a stream of its
 * own; ctx must outlive it. */
int sscg_server_create(sscg_ctx* ctx, const sscg_opts* opts, int64_t pool_rows, int64_t pool_nnz,
                       int32_t slots, sscg_server** server);
void sscg_server_destroy(sscg_server* server);
/* Queue A x = b (device arrays; b and x must stay valid until the request is
 * done; x holds x_1).  tol <= 0: opts->tol; lambda_min/max: the Chebyshev
 * interval (ignored for the monomial basis).  A request that could never fit
 * the pools is refused (SSCG_ERR_ARG). */
int sscg_server_submit(sscg_server* server, const sscg_csr* A, const double* b, double* x,
                       double tol, double lambda_min, double lambda_max, int64_t* id);
/* One outer block for every admitted system, then retirement and admission.
 * Outputs (may be NULL): systems running, requests waiting, requests retired
 * by this call. */
int sscg_server_step(sscg_server* server, int32_t* running, int32_t* queued, int32_t* retired);
/* state: 0 queued, 1 running, 2 done (x written).  The other outputs are
 * valid once done; status as for sscg_solve (SSCG_ERR_ARG if its matrix was
 * found malformed at admission). */
int sscg_server_poll(sscg_server* server, int64_t id, int32_t* state, int32_t* status,
                     int32_t* blocks, int32_t* iters, double* relres);
/* Per-block history of a finished request (Algorithm 4's s_k schedule, the
 * s~_k of eq. condy, the true relative residual after each block and, with
 * SSCG_PREC_VARIABLE, 1 where the block's basis was FP32): HOST
 * arrays of `cap` entries (any may be NULL); *rows gets the number of entries
 * written, min(cap, blocks, the server's history depth max_iters + 2 capped at
 * 4096).  SSCG_ERR_ARG for an unknown request or one that is not done. */
int sscg_server_history(sscg_server* server, int64_t id, int32_t cap, int32_t* s_k,
                        int32_t* s_tilde, double* relres_true, int32_t* fp32, int32_t* rows);
/* Counters since creation (any output may be NULL): outer-block replays
 * launched, and the sum over replays of the admitted systems' rows (each
 * padded to 1024); rows_active / replays is the mean rows per block. */
int sscg_server_stats(sscg_server* server, int64_t* replays, int64_t* rows_active);

/* ---------------------------------------------------------------- timing */

/* Kernel timing with HIP events on the stream each kernel runs on (off by
 * default).  families is a bit mask over the family ids (0 = matrix powers
 * pass, 1 = Gram, 2 = recovery, 3 = condition estimate / coordinate solve;
 * SSCG_TIME_ALL = all four, 0 = off).  While a family's bit is set,
 * sscg_solve and the per-stage calls record an event pair around each of its
 * launches (each pair costs a little time on the stream, so time only the
 * families you need).  sscg_kernel_stats (which waits for the streams)
 * returns, for one family id, the launches, their summed duration in ms and
 * their summed algorithmic bytes: what each launch must move at least, in the
 * form it reads.  Matrix powers: the stored SELL-64 entries of A at 3 bytes
 * (value tables and 16-bit offsets), 10 (16-bit offsets) or 12, per slice its
 * offset and width (and 4-entry table), plus 8 bytes per vector element read
 * or written (sequences, three-term w, outputs, the fused residual's x and b).
 * Gram: 8 n d.  Recovery: 8 n (d + 4).  Every call resets the counters. */
#define SSCG_TIME_ALL 0xF
int sscg_set_timing(sscg_ctx* ctx, int families);
int sscg_kernel_stats(sscg_ctx* ctx, int family, int64_t* launches, double* ms, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* SSCG_H */
