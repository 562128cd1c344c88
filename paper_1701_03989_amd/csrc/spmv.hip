// Sparse kernels: SELL-64 conversion, the matrix-powers pass, the true
// residual, the Gershgorin bound and the Lanczos step.
//
// Every row sum is accumulated exactly in double-double and rounded once, so
// it equals (up to a vanishingly rare near-tie) the correctly rounded exact
// row sum, independent of the order of the terms.
#include <type_traits>

#include "common.h"

namespace {

constexpr int WG = 256;              // 4 wavefronts
constexpr int SLICES_PER_WG = WG / SSCG_WAVE;

// ---------------------------------------------------------------- SELL-64

__global__ __launch_bounds__(WG) void k_check_csr(const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col, int n,
                                                  int64_t nnz, int32_t* __restrict__ flag) {
  int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  int bad = 0;
  if (t < n) bad |= rowptr[t + 1] < rowptr[t];
  if (t < nnz) bad |= (col[t] < 0) | (col[t] >= n);
  if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(WG) void k_sell_widths(const int32_t* __restrict__ rowptr, int n,
                                                    int nslices, int32_t* __restrict__ width) {
  int slice = blockIdx.x * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  if (slice >= nslices) return;
  int row = slice * SSCG_WAVE + (threadIdx.x & (SSCG_WAVE - 1));
  int len = row < n ? rowptr[row + 1] - rowptr[row] : 0;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) len = max(len, __shfl_xor(len, m, SSCG_WAVE));
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) width[slice] = len;
}

// Exclusive scan of 64*width into off[0..nslices]; one workgroup of 1024.
__global__ __launch_bounds__(1024) void k_scan_offsets(const int32_t* __restrict__ width,
                                                       int nslices, int64_t base0,
                                                       int64_t* __restrict__ off,
                                                       int64_t* __restrict__ end) {
  __shared__ int64_t part[1024];
  int t = threadIdx.x;
  int per = (nslices + 1023) / 1024;
  int lo = min(t * per, nslices), hi = min(lo + per, nslices);
  int64_t s = 0;
  for (int i = lo; i < hi; ++i) s += (int64_t)width[i] * SSCG_WAVE;
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int64_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t base = base0 + part[t] - s;  // exclusive prefix of this thread's chunk
  for (int i = lo; i < hi; ++i) {
    off[i] = base;
    base += (int64_t)width[i] * SSCG_WAVE;
  }
  if (t == 1023) *end = base0 + part[1023];
}

// s_i = 1 / sqrt(max_j |a_ij|) (equilibration, Section 5).
__global__ __launch_bounds__(WG) void k_row_scale(const int32_t* __restrict__ rowptr,
                                                  const double* __restrict__ val, int n,
                                                  double* __restrict__ scale) {
  int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  double m = 0.0;
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) m = fmax(m, fabs(val[k]));
  scale[i] = 1.0 / sqrt(m);
}

// One thread per row (and per padding lane of the last slice).  Value
// (a_ij s_i) s_j when a scale is given.
__global__ __launch_bounds__(WG) void k_sell_fill(const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, int n,
                                                  const double* __restrict__ scale,
                                                  const int64_t* __restrict__ off,
                                                  const int32_t* __restrict__ width, int nslices,
                                                  int col_off, int32_t* __restrict__ scol,
                                                  double* __restrict__ sval) {
  int row = blockIdx.x * WG + threadIdx.x;
  int slice = row / SSCG_WAVE;
  if (slice >= nslices) return;
  int lane = row & (SSCG_WAVE - 1);
  int64_t o = off[slice];
  int w = width[slice];
  int k0 = 0, len = 0;
  double si = 1.0;
  if (row < n) {
    k0 = rowptr[row];
    len = rowptr[row + 1] - k0;
    if (scale) si = scale[row];
  }
  for (int j = 0; j < w; ++j) {
    int64_t dst = o + (int64_t)j * SSCG_WAVE + lane;
    if (j < len) {
      int c = col[k0 + j];
      double v = val[k0 + j];
      if (scale) v = (v * si) * scale[c];
      scol[dst] = c + col_off;
      sval[dst] = v;
    } else {
      scol[dst] = (row < n ? row : 0) + col_off;
      sval[dst] = 0.0;
    }
  }
}

// 16-bit column offsets from each slice's first row (one thread per row).
__global__ __launch_bounds__(WG) void k_sell_compact(const int32_t* __restrict__ scol, int n,
                                                     const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ width,
                                                     int nslices, int16_t* __restrict__ col16,
                                                     int32_t* __restrict__ flag) {
  const int row = blockIdx.x * WG + threadIdx.x;
  const int slice = row / SSCG_WAVE;
  if (slice >= nslices) return;
  const int lane = row & (SSCG_WAVE - 1);
  const int64_t o = off[slice];
  const int w = width[slice];
  const int base = slice * SSCG_WAVE;
  int bad = 0;
  for (int j = 0; j < w; ++j) {
    const int64_t e = o + (int64_t)j * SSCG_WAVE + lane;
    int d = 0;
    if (row < n) {
      d = scol[e] - base;
      bad |= d < -32768 || d > 32767;
    }
    col16[e] = (int16_t)d;
  }
  if (bad) atomicOr(flag, 1);
}

// One entry per lane of a slice's value table build (called by the whole
// wavefront): the distinct stored values in order of first appearance (entry
// j, then lane), compared bit for bit.  Lane l < m holds table entry l in tb.
// Returns this lane's index; once a value finds no room, over is set (the
// same on every lane) and the index is meaningless.
__device__ __forceinline__ int vtab_index(double v, int lane, long long& tb, int& m, bool& over) {
  const long long bits = __double_as_longlong(v);
  int idx = -1;
  for (int i = 0; i < m; ++i)
    if (__shfl(tb, i, SSCG_WAVE) == bits && idx < 0) idx = i;
  for (;;) {  // append the lanes' new values, lowest lane first
    const unsigned long long need = __ballot(idx < 0);
    if (need == 0) break;
    if (m == VTAB) {
      over = true;
      if (idx < 0) idx = 0;
      break;
    }
    const long long nb = __shfl(bits, __ffsll((long long)need) - 1, SSCG_WAVE);
    if (lane == m) tb = nb;
    if (idx < 0 && bits == nb) idx = m;
    ++m;
  }
  return idx;
}

// Value table of each slice (one wavefront per slice) and each entry's index
// into it.  More than VTAB values set *flag.
__global__ __launch_bounds__(WG) void k_sell_vidx(const double* __restrict__ val,
                                                  const int64_t* __restrict__ off,
                                                  const int32_t* __restrict__ width, int nslices,
                                                  double* __restrict__ vtab,
                                                  uint8_t* __restrict__ vidx,
                                                  int32_t* __restrict__ flag) {
  const int slice = blockIdx.x * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  if (slice >= nslices) return;  // whole wavefronts
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  const int64_t o = off[slice] + lane;
  const int w = width[slice];
  long long tb = 0;
  int m = 0;
  bool over = false;
  for (int j = 0; j < w; ++j) {
    const int64_t k = o + (int64_t)j * SSCG_WAVE;
    vidx[k] = (uint8_t)vtab_index(val[k], lane, tb, m, over);
  }
  if (lane < VTAB) vtab[(int64_t)slice * VTAB + lane] = __longlong_as_double(lane < m ? tb : 0);
  if (over && lane == 0) *flag = 1;
}

// The slice-diagonal form (DevMat::sd_*) of one slice, called by its whole
// wavefront: lane = the row at position `row` (absolute), len = its number of
// stored entries (the rest of the slice's width is padding).  The distances
// and values are collected in order of first appearance (entry j, then lane),
// like the value table.  Returns true (on every lane) if the slice does not
// fit the form: more than SD_DIAG distances or SD_VALS values, or a row with
// two entries at one distance.
__device__ __forceinline__ bool sdia_slice(int slice, int row, int len,
                                           const int32_t* __restrict__ scol,
                                           const double* __restrict__ sval,
                                           const int64_t* __restrict__ off,
                                           const int32_t* __restrict__ width,
                                           int32_t* __restrict__ sd_nd,
                                           int32_t* __restrict__ sd_delta,
                                           double* __restrict__ sd_tab,
                                           uint16_t* __restrict__ sd_code) {
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  const int64_t o = off[slice] + lane;
  const int w = width[slice];
  int ds = 0, nd = 0;      // lane k < nd holds distance k
  long long tb = 0;        // lane c < m holds value c (bits)
  int m = 0;
  bool over = false, dup = false;
  unsigned code = 0xFFFFu;  // every distance absent
  for (int j = 0; j < w && !over; ++j) {
    const int64_t e = o + (int64_t)j * SSCG_WAVE;
    const bool real = j < len;
    const int d = real ? scol[e] - row : 0;
    const long long bits = real ? __double_as_longlong(sval[e]) : 0;
    int di = -1, vi = -1;
    for (int i = 0; i < nd; ++i)
      if (__shfl(ds, i, SSCG_WAVE) == d && di < 0) di = i;
    for (int i = 0; i < m; ++i)
      if (__shfl(tb, i, SSCG_WAVE) == bits && vi < 0) vi = i;
    for (;;) {  // new distances, lowest lane first
      const unsigned long long need = __ballot(real && di < 0);
      if (need == 0) break;
      if (nd == SD_DIAG) {
        over = true;
        break;
      }
      const int nb = __shfl(d, __ffsll((long long)need) - 1, SSCG_WAVE);
      if (lane == nd) ds = nb;
      if (real && di < 0 && d == nb) di = nd;
      ++nd;
    }
    for (;;) {  // new values
      const unsigned long long need = __ballot(real && vi < 0);
      if (need == 0 || over) break;
      if (m == SD_VALS) {
        over = true;
        break;
      }
      const long long nb = __shfl(bits, __ffsll((long long)need) - 1, SSCG_WAVE);
      if (lane == m) tb = nb;
      if (real && vi < 0 && bits == nb) vi = m;
      ++m;
    }
    if (real && di >= 0 && vi >= 0) {
      const unsigned sh = 2u * (unsigned)di;
      dup |= ((code >> sh) & 3u) != (unsigned)SD_ABSENT;
      code = (code & ~(3u << sh)) | ((unsigned)vi << sh);
    }
  }
  over |= __ballot(dup) != 0;
  // Canonical order: distances ascending, values by their bits ascending
  // (the codes renumbered to match), so that slices with the same distances
  // and values store the same tables.  (Each row sum is formed in
  // double-double and rounded once: whatever the order of its terms, that is
  // the correctly rounded sum but for vanishingly rare near-ties.)
  int dr = 0, vr = 0;  // lane k < nd: rank of distance k; lane c < m: rank of value c
  for (int i = 0; i < nd; ++i) dr += __shfl(ds, i, SSCG_WAVE) < ds ? 1 : 0;
  for (int i = 0; i < m; ++i)
    vr += (unsigned long long)__shfl(tb, i, SSCG_WAVE) < (unsigned long long)tb ? 1 : 0;
  const int vr0 = __shfl(vr, 0, SSCG_WAVE), vr1 = __shfl(vr, 1, SSCG_WAVE),
            vr2 = __shfl(vr, 2, SSCG_WAVE);
  unsigned sorted = 0xFFFFu;
  for (int k = 0; k < nd; ++k) {
    const unsigned f = (code >> (2 * k)) & 3u;
    const unsigned to = 2u * (unsigned)__shfl(dr, k, SSCG_WAVE);
    if (f != (unsigned)SD_ABSENT) {
      const unsigned nv = (unsigned)(f == 0u ? vr0 : (f == 1u ? vr1 : vr2));
      sorted = (sorted & ~(3u << to)) | (nv << to);
    }
  }
  if (lane < SD_DIAG && lane >= nd) sd_delta[(int64_t)slice * SD_DIAG + lane] = 0;
  if (lane < nd) sd_delta[(int64_t)slice * SD_DIAG + dr] = ds;
  if (lane < 4 && lane >= m) sd_tab[(int64_t)slice * 4 + lane] = 0.0;
  if (lane < m) sd_tab[(int64_t)slice * 4 + vr] = __longlong_as_double(tb);
  if (lane == 0) sd_nd[slice] = nd;
  sd_code[row] = (uint16_t)(over ? code : sorted);
  return over;
}

// Single matrix: *flag = 1 if some slice does not fit (the form is then not
// used for the matrix).
__global__ __launch_bounds__(WG) void k_sell_sdia(const int32_t* __restrict__ rowptr, int n,
                                                  const int32_t* __restrict__ scol,
                                                  const double* __restrict__ sval,
                                                  const int64_t* __restrict__ off,
                                                  const int32_t* __restrict__ width, int nslices,
                                                  int32_t* __restrict__ sd_nd,
                                                  int32_t* __restrict__ sd_delta,
                                                  double* __restrict__ sd_tab,
                                                  uint16_t* __restrict__ sd_code,
                                                  int32_t* __restrict__ flag) {
  const int slice = blockIdx.x * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  if (slice >= nslices) return;  // whole wavefronts
  const int row = slice * SSCG_WAVE + (threadIdx.x & (SSCG_WAVE - 1));
  const int len = row < n ? rowptr[row + 1] - rowptr[row] : 0;
  const bool over = sdia_slice(slice, row, len, scol, sval, off, width, sd_nd, sd_delta, sd_tab,
                               sd_code);
  if (over && (threadIdx.x & (SSCG_WAVE - 1)) == 0) atomicOr(flag, 1);
}

// One batched system's slices [slice0, slice0 + nsl): position p of the
// system holds its row perm[p] (-1: padding); *cnt gains one per slice that
// does not fit.
__global__ __launch_bounds__(WG) void k_sell_sdia_sys(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ perm,
                                                      int slice0, int nsl,
                                                      const int32_t* __restrict__ scol,
                                                      const double* __restrict__ sval,
                                                      const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ width,
                                                      int32_t* __restrict__ sd_nd,
                                                      int32_t* __restrict__ sd_delta,
                                                      double* __restrict__ sd_tab,
                                                      uint16_t* __restrict__ sd_code,
                                                      int32_t* __restrict__ cnt) {
  const int i = blockIdx.x * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  if (i >= nsl) return;  // whole wavefronts
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  const int r = perm[i * SSCG_WAVE + lane];
  const int len = r >= 0 ? rowptr[r + 1] - rowptr[r] : 0;
  const int slice = slice0 + i;
  const bool over = sdia_slice(slice, slice * SSCG_WAVE + lane, len, scol, sval, off, width,
                               sd_nd, sd_delta, sd_tab, sd_code);
  if (over && lane == 0) atomicAdd(cnt, 1);
}

// sys[q].sd = 1 when none of system q's slices missed the slice-diagonal
// form (cnt[q] == 0); such a system's passes read it (and not the pairs).
__global__ void k_set_sd(BatchSys* __restrict__ sys, const int32_t* __restrict__ cnt, int q0,
                         int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int q = q0 + i;
  sys[q].sd = cnt[q] == 0 ? 1 : 0;
  if (sys[q].sd) sys[q].il = 0;
}

// ---------------------------------------------------------------- MPK pass
//
// Pass j of the matrix-powers kernel for one or two sequences (P and R of
// eq. cg-krylovbasis, advanced together so A is streamed once per pass):
//   out_i = RN( sum_k a_ik u_k - theta u_i - sigma w_i ) / gamma.
// One wavefront per 64-row slice, one lane per row.
//
// RES: the pass also forms the true residual of the block's starting iterate
// x, res_i = RN(b_i - (A x)_i), from the same stream of A (x gathered as a
// third sequence), and stores per-workgroup dd partials of sum res_i^2.
// The gate: the pass does nothing once the solve has stopped.
template <int NW = SLICES_PER_WG>
__device__ __forceinline__ void wg_store_partial(dd a, double* part, int slot);

// The rows of one slice (lane = row within it); returns the lane's res_i^2
// contribution when RES.
// IL (two sequences): the gathers of u read the pairs tg[c] = (s0.u[c],
// s1.u[c]), one 16-byte load instead of two 8-byte ones on different cache
// lines (random gathers), and tw, if given, receives the pairs of the outputs.
// CEN (slice-diagonal form): the centre terms take the row's own u from its
// distance-0 gather (k_mpk; in the batched pass's larger kernel the extra
// state cost more than the load it saves).
template <int NRHS, bool CHEB, bool HASW, bool RES, bool C16 = false, bool IL = false,
          bool VI = false, bool SD = false, int CHK = 4, class V = double, bool CEN = false,
          bool UV = false>
__device__ __forceinline__ dd mpk_slice(const DevMat& A, int slice, double theta, double sigma,
                                        double gamma, const MpkSeqV<V>& s0, const MpkSeqV<V>& s1,
                                        const double* __restrict__ xres,
                                        const double* __restrict__ bres,
                                        const double2* __restrict__ tg = nullptr,
                                        double2* __restrict__ tw = nullptr) {
  int lane = threadIdx.x & (SSCG_WAVE - 1);
  int row = slice * SSCG_WAVE + lane;
  dd r2 = dd_zero();
  if (slice < A.nslices) {
    const V* __restrict__ u0 = s0.u;
    const V* __restrict__ u1 = s1.u;
    dd a0 = dd_zero(), a1 = dd_zero(), ax = dd_zero();
    // SD: the row's own u values as gathered at distance 0 (hc: it has that
    // entry), so that the centre terms below need no load of their own
    V c0 = 0, c1 = 0;
    bool hc = false;
    if constexpr (SD) {
      // slice-diagonal form: distances and values of the slice (wave-uniform,
      // scalar registers), one 16-bit code word per row; every gather address
      // is row + distance, so all of a chunk's loads issue at once
      const int us = __builtin_amdgcn_readfirstlane(slice);
      const int nd = A.sd_nd[us];
      int dl[SD_DIAG];
      double tv[SD_VALS];
#pragma unroll
      for (int k = 0; k < SD_DIAG; ++k) dl[k] = A.sd_delta[(int64_t)us * SD_DIAG + k];
#pragma unroll
      for (int i = 0; i < SD_VALS; ++i) tv[i] = A.sd_tab[(int64_t)us * 4 + i];
      // UV: each distance's value, the same for every row that has it
      double vu[SD_DIAG];
      if (UV) {
        const uint32_t vw = A.sd_vk[us];
#pragma unroll
        for (int k = 0; k < SD_DIAG; ++k) {
          const uint32_t c = (vw >> (2 * k)) & 3u;
          vu[k] = c == 0u ? tv[0] : (c == 1u ? tv[1] : tv[2]);
        }
      }
      const unsigned code = A.sd_code[row];
      constexpr int CH = CHK;  // entries whose loads are in flight together
#pragma unroll
      for (int k0 = 0; k0 < SD_DIAG; k0 += CH) {
        if (k0 < nd) {
          double v[CH], g0[CH], g1[CH], gx[CH];
          bool pr[CH];
          int c[CH];
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            const int k = k0 + u;
            const unsigned cd = k < nd ? (code >> (2 * k)) & 3u : (unsigned)SD_ABSENT;
            pr[u] = cd != (unsigned)SD_ABSENT;
            v[u] = UV ? vu[k] : (cd == 0u ? tv[0] : (cd == 1u ? tv[1] : tv[2]));
            c[u] = row + dl[k];
          }
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            if (pr[u]) {
              g0[u] = u0[c[u]];
              if (NRHS == 2) g1[u] = u1[c[u]];
              if (RES) gx[u] = xres[c[u]];
            }
          }
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            if (pr[u]) {
              dd_add_prod(a0, v[u], g0[u]);
              if (NRHS == 2) dd_add_prod(a1, v[u], g1[u]);
              if (RES) dd_add_prod(ax, v[u], gx[u]);
              if (CHEB && CEN && k0 + u < nd && dl[k0 + u] == 0) {  // uniform test
                c0 = g0[u];
                if (NRHS == 2) c1 = g1[u];
                hc = true;
              }
            }
          }
        }
      }
    } else {
    int64_t o = A.off[slice] + lane;
    int w = A.width[slice];
    // VI: the slice's value table (wave-uniform) in scalar registers
    double tv[VTAB];
    if (VI) {
      const int us = __builtin_amdgcn_readfirstlane(slice);
#pragma unroll
      for (int i = 0; i < VTAB; ++i) tv[i] = A.vtab[(int64_t)us * VTAB + i];
    }
    // chunks of CH entries: every load of a chunk is issued before its first
    // use (w is uniform over the wave, so the guards do not diverge)
    constexpr int CH = CHK;  // entries whose loads are in flight together
    for (int j0 = 0; j0 < w; j0 += CH) {
      double v[CH], g0[CH], g1[CH], gx[CH];
      int c[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        int64_t k = o + (int64_t)(j0 + u) * SSCG_WAVE;
        bool in = j0 + u < w;
        if (VI) {
          const int ix = in ? (int)A.vidx[k] : 0;
          double t = tv[VTAB - 1];
#pragma unroll
          for (int i = VTAB - 2; i >= 0; --i) t = ix == i ? tv[i] : t;
          v[u] = in ? t : 0.0;
        }
        else v[u] = in ? A.val[k] : 0.0;
        if (C16) c[u] = in ? slice * SSCG_WAVE + (int)A.col16[k] : 0;
        else c[u] = in ? A.col[k] : 0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        if (j0 + u < w) {
          if (IL && NRHS == 2) {
            const double2 t = tg[c[u]];
            g0[u] = t.x;
            g1[u] = t.y;
          } else {
            g0[u] = u0[c[u]];
            if (NRHS == 2) g1[u] = u1[c[u]];
          }
          if (RES) gx[u] = xres[c[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        if (j0 + u < w) {
          dd_add_prod(a0, v[u], g0[u]);
          if (NRHS == 2) dd_add_prod(a1, v[u], g1[u]);
          if (RES) dd_add_prod(ax, v[u], gx[u]);
        }
      }
    }
    }  // SELL forms
    if (row < A.n) {
      double o0, o1 = 0.0;
      if (CHEB) {
        if (!(SD && CEN && hc)) {
          c0 = u0[row];
          if (NRHS == 2) c1 = u1[row];
        }
        dd_add_prod(a0, -theta, c0);
        if (HASW) dd_add_prod(a0, -sigma, s0.w[row]);
        o0 = dd_round(a0) / gamma;
        if (NRHS == 2) {
          dd_add_prod(a1, -theta, c1);
          if (HASW) dd_add_prod(a1, -sigma, s1.w[row]);
          o1 = dd_round(a1) / gamma;
        }
      } else {
        o0 = dd_round(a0);
        if (NRHS == 2) o1 = dd_round(a1);
      }
      // an FP32 sequence stores the FP64 result rounded once (V = float)
      s0.out[row] = (V)o0;
      if (NRHS == 2) s1.out[row] = (V)o1;
      if (IL && NRHS == 2 && tw) tw[row] = make_double2(o0, o1);
      if (RES) {
        dd_add(ax, -bres[row]);
        double ri = -dd_round(ax);
        dd_add_prod(r2, ri, ri);
      }
    }
  }
  return r2;
}

template <int NRHS, bool CHEB, bool HASW, bool RES, bool C16, bool VI, bool SD, bool UV>
__global__ __launch_bounds__(WG) void k_mpk(DevMat A, double theta, double sigma, double gamma,
                                            MpkSeq s0, MpkSeq s1, Gate gate,
                                            const double* __restrict__ xres,
                                            const double* __restrict__ bres,
                                            double* __restrict__ rpart) {
  if (gate_stopped(gate)) return;
  int nb = (A.nslices + SLICES_PER_WG - 1) / SLICES_PER_WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;  // not workgroup 0 (nb >= 1 and xcd_block(nb) maps 0 to 0)
  const int slice =  // uniform over the wavefront
      __builtin_amdgcn_readfirstlane(lb * SLICES_PER_WG + (int)(threadIdx.x / SSCG_WAVE));
  dd r2 = mpk_slice<NRHS, CHEB, HASW, RES, C16, false, VI, SD, 4, double, SD, UV>(
      A, slice, theta, sigma, gamma, s0, s1, xres, bres);
  if (RES) wg_store_partial(r2, rpart, lb);
  gate_mark_ran(gate);
}

// Two rows' worth of a sequence: 8-byte alignment is all the pair form's
// addresses (row + distance, row even) guarantee.
// (A vector type, so that each access stays one 16-byte instruction.)
typedef double sd2 __attribute__((ext_vector_type(2), aligned(8)));

// The pass in the pair form (DevMat::sd_pair): a wavefront takes the 128 rows
// of slices 2t and 2t + 1, lane l the rows 128 t + 2 l and 128 t + 2 l + 1,
// with the pair's common distances and values in scalar registers.  For each
// distance one 16-byte load brings both rows' u values, so a row costs half
// the memory instructions of the one-row-per-lane form.  Where every row of
// the pair and every neighbour it names lie in [0, n) (the interior), the
// loads of all nd distances are issued unconditionally; a boundary pair loads
// each row's value through a clamped index.  Each row adds its terms in the
// order of its distances with the same dd steps as mpk_slice, so the result
// is the same to the bit.  Workgroups of two wavefronts cover four slices, as
// the k_mpk workgroups do, so the residual partials keep their slots.
template <int NRHS, bool CHEB, bool HASW, bool RES, bool UV>
__global__ __launch_bounds__(2 * SSCG_WAVE) void k_mpk_sdp(DevMat A, double theta, double sigma,
                                                           double gamma, MpkSeq s0, MpkSeq s1,
                                                           Gate gate,
                                                           const double* __restrict__ xres,
                                                           const double* __restrict__ bres,
                                                           double* __restrict__ rpart) {
  static_assert(SLICES_PER_WG == 4, "two wavefronts of two slices each");
  if (gate_stopped(gate)) return;
  const int nb = (A.nslices + SLICES_PER_WG - 1) / SLICES_PER_WG;
  const int lb = xcd_block(nb);
  if (lb >= nb) return;  // not workgroup 0 (nb >= 1 and xcd_block(nb) maps 0 to 0)
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  // the pair of slices (uniform over the wavefront: scalar registers)
  const int t = __builtin_amdgcn_readfirstlane(lb * 2 + (int)(threadIdx.x / SSCG_WAVE));
  const int n = A.n;
  dd r2 = dd_zero();
  if (2 * t < A.nslices) {
    const int us = __builtin_amdgcn_readfirstlane(2 * t);
    const int nd = A.sd_nd[us];
    int dl[SD_DIAG];
    double tv[SD_VALS];
#pragma unroll
    for (int k = 0; k < SD_DIAG; ++k) dl[k] = A.sd_delta[(int64_t)us * SD_DIAG + k];
#pragma unroll
    for (int i = 0; i < SD_VALS; ++i) tv[i] = A.sd_tab[(int64_t)us * 4 + i];
    // UV: the value of each distance, the same for every row that has it
    double vu[SD_DIAG];
    if (UV) {
      const uint32_t vw = A.sd_vk[us];
#pragma unroll
      for (int k = 0; k < SD_DIAG; ++k) {
        const uint32_t c = (vw >> (2 * k)) & 3u;
        vu[k] = c == 0u ? tv[0] : (c == 1u ? tv[1] : tv[2]);
      }
    }
    const int base = t * 2 * SSCG_WAVE;  // first row of the pair
    const int r = base + 2 * lane;
    const unsigned lo = 2u * (unsigned)lane;  // the lane's offset from a uniform base
    // uniform: the lowest and highest distance, and which one is 0
    int dmin = 0, dmax = 0, kc = -1;
#pragma unroll
    for (int k = 0; k < SD_DIAG; ++k)
      if (k < nd) {
        dmin = (k == 0 || dl[k] < dmin) ? dl[k] : dmin;
        dmax = (k == 0 || dl[k] > dmax) ? dl[k] : dmax;
        kc = dl[k] == 0 ? k : kc;
      }
    // (in 64 bits: base + 127 + dmax may exceed the int range for n > 2^30)
    const bool inner = 2 * t + 1 < A.nslices && (int64_t)base + 2 * SSCG_WAVE <= n &&
                       (int64_t)base + dmin >= 0 &&
                       (int64_t)base + 2 * SSCG_WAVE - 1 + dmax <= (int64_t)n - 1;
    // codes of the two rows (padding rows and rows past the last slice: none)
    unsigned ca, cb;
    if (inner) {
      const uint32_t w2 = ((const uint32_t*)(A.sd_code + base))[(unsigned)lane];
      ca = w2 & 0xFFFFu;
      cb = w2 >> 16;
    } else {
      const int lim = A.nslices * SSCG_WAVE;
      ca = r < lim ? A.sd_code[r] : 0xFFFFu;
      cb = r + 1 < lim ? A.sd_code[r + 1] : 0xFFFFu;
    }
    dd a0 = dd_zero(), a1 = dd_zero(), ax = dd_zero();  // row r
    dd b0 = dd_zero(), b1 = dd_zero(), bx = dd_zero();  // row r + 1
    double ca0 = 0, ca1 = 0, cb0 = 0, cb1 = 0;           // centre values from distance 0
    // chunks of 4, 3 and 1 distances (the loads of a chunk are in flight
    // together; larger chunks cost occupancy): a seven-point stencil loads no
    // distance twice.  With the residual's third sequence, chunks of 3, 2, 2
    // and 1 (86 -> 74 VGPRs, its pass 38.6 -> 36.9 us at 128^3).
    auto chunk = [&](auto k0c, auto chc) {
      constexpr int k0 = decltype(k0c)::value, CH = decltype(chc)::value;
      if (k0 < nd) {
        sd2 g0[CH], g1[CH], gx[CH];
        if (inner) {
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            // a uniform base (scalar registers) + 16 bytes per lane
            const int ob = base + (k0 + u < nd ? dl[k0 + u] : 0);
            g0[u] = *(const sd2*)((s0.u + ob) + lo);
            if (NRHS == 2) g1[u] = *(const sd2*)((s1.u + ob) + lo);
            if (RES) gx[u] = *(const sd2*)((xres + ob) + lo);
          }
        } else {
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            const int d = k0 + u < nd ? dl[k0 + u] : 0;
            // clamped in 64 bits (an absent entry's row + distance may leave the int range)
            const int ia = (int)min(max((int64_t)r + d, (int64_t)0), (int64_t)n - 1);
            const int ib = (int)min(max((int64_t)r + 1 + d, (int64_t)0), (int64_t)n - 1);
            g0[u].x = s0.u[ia];
            g0[u].y = s0.u[ib];
            if (NRHS == 2) {
              g1[u].x = s1.u[ia];
              g1[u].y = s1.u[ib];
            }
            if (RES) {
              gx[u].x = xres[ia];
              gx[u].y = xres[ib];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int k = k0 + u;
          const unsigned da = k < nd ? (ca >> (2 * k)) & 3u : (unsigned)SD_ABSENT;
          const unsigned db = k < nd ? (cb >> (2 * k)) & 3u : (unsigned)SD_ABSENT;
          if (da != (unsigned)SD_ABSENT) {
            const double v = UV ? vu[k] : (da == 0u ? tv[0] : (da == 1u ? tv[1] : tv[2]));
            dd_add_prod(a0, v, g0[u].x);
            if (NRHS == 2) dd_add_prod(a1, v, g1[u].x);
            if (RES) dd_add_prod(ax, v, gx[u].x);
          }
          if (db != (unsigned)SD_ABSENT) {
            const double v = UV ? vu[k] : (db == 0u ? tv[0] : (db == 1u ? tv[1] : tv[2]));
            dd_add_prod(b0, v, g0[u].y);
            if (NRHS == 2) dd_add_prod(b1, v, g1[u].y);
            if (RES) dd_add_prod(bx, v, gx[u].y);
          }
          if (CHEB && k == kc) {  // uniform: the distance-0 loads are the rows' own u
            ca0 = g0[u].x;
            cb0 = g0[u].y;
            if (NRHS == 2) {
              ca1 = g1[u].x;
              cb1 = g1[u].y;
            }
          }
        }
            }
    };
    if constexpr (RES) {
      chunk(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{});
      chunk(std::integral_constant<int, 3>{}, std::integral_constant<int, 2>{});
      chunk(std::integral_constant<int, 5>{}, std::integral_constant<int, 2>{});
      chunk(std::integral_constant<int, 7>{}, std::integral_constant<int, 1>{});
    } else {
      chunk(std::integral_constant<int, 0>{}, std::integral_constant<int, 4>{});
      chunk(std::integral_constant<int, 4>{}, std::integral_constant<int, 3>{});
      chunk(std::integral_constant<int, 7>{}, std::integral_constant<int, 1>{});
    }
    if (CHEB && kc < 0) {  // no distance 0 in this pair of slices
      const int ia = min(r, n - 1), ib = min(r + 1, n - 1);
      ca0 = s0.u[ia];
      cb0 = s0.u[ib];
      if (NRHS == 2) {
        ca1 = s1.u[ia];
        cb1 = s1.u[ib];
      }
    }
    // outputs of rows r and r + 1 (both in [0, n) in the interior)
    double oa0, oa1 = 0.0, ob0, ob1 = 0.0;
    if (CHEB) {
      double wa0 = 0, wb0 = 0, wa1 = 0, wb1 = 0;
      if (HASW) {
        if (inner) {
          const sd2 w = *(const sd2*)((s0.w + base) + lo);
          wa0 = w.x;
          wb0 = w.y;
          if (NRHS == 2) {
            const sd2 v = *(const sd2*)((s1.w + base) + lo);
            wa1 = v.x;
            wb1 = v.y;
          }
        } else {
          const int ia = min(r, n - 1), ib = min(r + 1, n - 1);
          wa0 = s0.w[ia];
          wb0 = s0.w[ib];
          if (NRHS == 2) {
            wa1 = s1.w[ia];
            wb1 = s1.w[ib];
          }
        }
      }
      dd_add_prod(a0, -theta, ca0);
      if (HASW) dd_add_prod(a0, -sigma, wa0);
      oa0 = dd_round(a0) / gamma;
      dd_add_prod(b0, -theta, cb0);
      if (HASW) dd_add_prod(b0, -sigma, wb0);
      ob0 = dd_round(b0) / gamma;
      if (NRHS == 2) {
        dd_add_prod(a1, -theta, ca1);
        if (HASW) dd_add_prod(a1, -sigma, wa1);
        oa1 = dd_round(a1) / gamma;
        dd_add_prod(b1, -theta, cb1);
        if (HASW) dd_add_prod(b1, -sigma, wb1);
        ob1 = dd_round(b1) / gamma;
      }
    } else {
      oa0 = dd_round(a0);
      ob0 = dd_round(b0);
      if (NRHS == 2) {
        oa1 = dd_round(a1);
        ob1 = dd_round(b1);
      }
    }
    if (inner) {
      *(sd2*)((s0.out + base) + lo) = sd2{oa0, ob0};
      if (NRHS == 2) *(sd2*)((s1.out + base) + lo) = sd2{oa1, ob1};
    } else {
      if (r < n) {
        s0.out[r] = oa0;
        if (NRHS == 2) s1.out[r] = oa1;
      }
      if (r + 1 < n) {
        s0.out[r + 1] = ob0;
        if (NRHS == 2) s1.out[r + 1] = ob1;
      }
    }
    if (RES) {
      if (r < n) {
        dd_add(ax, -bres[r]);
        const double ri = -dd_round(ax);
        dd_add_prod(r2, ri, ri);
      }
      if (r + 1 < n) {
        dd_add(bx, -bres[r + 1]);
        const double ri = -dd_round(bx);
        dd_add_prod(r2, ri, ri);
      }
    }
  }
  if (RES) wg_store_partial<2>(r2, rpart, lb);
  gate_mark_ran(gate);
}

// Batched pass j over the 256-row blocks listed in ablk[0, *nlist) (those of
// the systems not done when the list was made; a workgroup takes every
// gridDim.x-th entry).  Every block belongs to one system (blk_sys), whose
// basis parameters and state come from the system table; blocks of systems
// finished since are skipped.  A system flagged sd reads
// the slice-diagonal form, one flagged vt the value tables and 16-bit offsets
// of k_sell_forms_batch, one flagged il the (P, R) pairs.
template <int NRHS, bool CHEB, bool RES, int CHK>
__global__ __launch_bounds__(WG) void k_mpk_batch(DevMat A, int j, MpkSeq s0, MpkSeq s1,
                                                  MpkSeq32 f0, MpkSeq32 f1,
                                                  const BatchSys* __restrict__ sys,
                                                  const int32_t* __restrict__ blk_sys,
                                                  const int32_t* __restrict__ ablk,
                                                  const int32_t* __restrict__ nlist,
                                                  const double* __restrict__ xres,
                                                  const double* __restrict__ bres,
                                                  double* __restrict__ rpart,
                                                  const double2* __restrict__ tg,
                                                  double2* __restrict__ tw) {
  const int nl = *nlist;
  for (int li = blockIdx.x; li < nl; li += gridDim.x) {  // uniform over the workgroup
    const int lb = ablk[li];
    const int q = blk_sys[lb];
    if (q < 0 || sys[q].done) continue;
    const bool il = NRHS == 2 && sys[q].il;
    const BasisPrm bp = sys[q].bp;
    const double theta = CHEB ? bp.c0 : 0.0, sigma = CHEB ? bp.h2 : 0.0;
    const double gamma = CHEB ? (j == 1 ? bp.h : bp.h2) : 1.0;
    const int slice =  // uniform over the wavefront
        __builtin_amdgcn_readfirstlane(lb * SLICES_PER_WG + (int)(threadIdx.x / SSCG_WAVE));
    dd r2;
    if (sys[q].p32) {  // FP32 block: Y32 sequences, column gathers (no pairs)
      if (sys[q].sd) {
        if (j >= 2)
          r2 = mpk_slice<NRHS, CHEB, CHEB, RES, false, false, false, true, CHK, float>(
              A, slice, theta, sigma, gamma, f0, f1, xres, bres);
        else
          r2 = mpk_slice<NRHS, CHEB, false, RES, false, false, false, true, CHK, float>(
              A, slice, theta, sigma, gamma, f0, f1, xres, bres);
      } else if (sys[q].vt) {
        if (j >= 2)
          r2 = mpk_slice<NRHS, CHEB, CHEB, RES, true, false, true, false, CHK, float>(
              A, slice, theta, sigma, gamma, f0, f1, xres, bres);
        else
          r2 = mpk_slice<NRHS, CHEB, false, RES, true, false, true, false, CHK, float>(
              A, slice, theta, sigma, gamma, f0, f1, xres, bres);
      } else {
        if (j >= 2)
          r2 = mpk_slice<NRHS, CHEB, CHEB, RES, false, false, false, false, CHK, float>(
              A, slice, theta, sigma, gamma, f0, f1, xres, bres);
        else
          r2 = mpk_slice<NRHS, CHEB, false, RES, false, false, false, false, CHK, float>(
              A, slice, theta, sigma, gamma, f0, f1, xres, bres);
      }
    } else if (sys[q].sd) {  // slice-diagonal form (stencils)
      if (j >= 2)
        r2 = mpk_slice<NRHS, CHEB, CHEB, RES, false, false, false, true, CHK>(A, slice, theta, sigma,
                                                                         gamma, s0, s1, xres, bres);
      else
        r2 = mpk_slice<NRHS, CHEB, false, RES, false, false, false, true, CHK>(A, slice, theta, sigma,
                                                                          gamma, s0, s1, xres,
                                                                          bres);
    } else if (il) {
      if (j >= 2)
        r2 = mpk_slice<NRHS, CHEB, CHEB, RES, false, true, false, false, CHK>(A, slice, theta, sigma, gamma, s0, s1,
                                                           xres, bres, tg, tw);
      else
        r2 = mpk_slice<NRHS, CHEB, false, RES, false, true, false, false, CHK>(A, slice, theta, sigma, gamma, s0, s1,
                                                            xres, bres, tg, tw);
    } else if (sys[q].vt) {  // value tables and 16-bit offsets (k_sell_forms_batch)
      if (j >= 2)
        r2 = mpk_slice<NRHS, CHEB, CHEB, RES, true, false, true, false, CHK>(A, slice, theta, sigma, gamma,
                                                                 s0, s1, xres, bres);
      else
        r2 = mpk_slice<NRHS, CHEB, false, RES, true, false, true, false, CHK>(A, slice, theta, sigma, gamma,
                                                                  s0, s1, xres, bres);
    } else {
      if (j >= 2)
        r2 = mpk_slice<NRHS, CHEB, CHEB, RES, false, false, false, false, CHK>(A, slice, theta, sigma, gamma, s0, s1, xres, bres);
      else
        r2 = mpk_slice<NRHS, CHEB, false, RES, false, false, false, false, CHK>(A, slice, theta, sigma, gamma, s0, s1, xres, bres);
    }
    if (RES) {
      wg_store_partial(r2, rpart, lb);
      __syncthreads();  // the partial's LDS is read before the next block rewrites it
    }
  }
}

// Reduce a per-thread dd over the NW waves of the workgroup and store it as
// partial `slot`.
template <int NW>
__device__ __forceinline__ void wg_store_partial(dd a, double* part, int slot) {
  __shared__ double ls[NW], le[NW];
  a = dd_wave_reduce(a);
  int wv = threadIdx.x / SSCG_WAVE;
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) {
    ls[wv] = a.s;
    le[wv] = a.e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    dd t{ls[0], le[0]};
    for (int q = 1; q < NW; ++q) dd_merge(t, dd{ls[q], le[q]});
    part[2 * slot] = t.s;
    part[2 * slot + 1] = t.e;
  }
}

// res_i = RN(b_i - (A x)_i); partials of sum res_i^2 (and sum b_i^2).
__global__ __launch_bounds__(WG) void k_residual(DevMat A, const double* __restrict__ b,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ r,
                                                 double* __restrict__ rpart,
                                                 double* __restrict__ bpart) {
  int nb = (A.nslices + SLICES_PER_WG - 1) / SLICES_PER_WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  const int slice =  // uniform over the wavefront
      __builtin_amdgcn_readfirstlane(lb * SLICES_PER_WG + (int)(threadIdx.x / SSCG_WAVE));
  int lane = threadIdx.x & (SSCG_WAVE - 1);
  int row = slice * SSCG_WAVE + lane;
  dd r2 = dd_zero(), b2 = dd_zero();
  if (slice < A.nslices) {
    int64_t o = A.off[slice] + lane;
    int w = A.width[slice];
    dd a = dd_zero();
#pragma unroll 4
    for (int j = 0; j < w; ++j) {
      int64_t k = o + (int64_t)j * SSCG_WAVE;
      dd_add_prod(a, A.val[k], x[A.col[k]]);
    }
    if (row < A.n) {
      double bi = b[row];
      dd_add(a, -bi);
      double ri = -dd_round(a);
      if (r) r[row] = ri;
      dd_add_prod(r2, ri, ri);
      dd_add_prod(b2, bi, bi);
    }
  }
  wg_store_partial(r2, rpart, lb);
  if (bpart) {
    __syncthreads();
    wg_store_partial(b2, bpart, lb);
  }
}

// The residual of the caller's CSR matrix itself, one row per lane (no SELL
// copy): per-workgroup dd partials of sum (b_i - (A x)_i)^2 and, if bpart,
// of sum b_i^2, each res_i rounded once from its exact value.
__global__ __launch_bounds__(WG) void k_csr_residual(const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, int n,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ rpart,
                                                     double* __restrict__ bpart) {
  int nb = (n + WG - 1) / WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  int row = lb * WG + threadIdx.x;
  dd r2 = dd_zero(), b2 = dd_zero();
  if (row < n) {
    dd a = dd_zero();
    const int k1 = rowptr[row + 1];
    for (int k = rowptr[row]; k < k1; ++k) dd_add_prod(a, val[k], x[col[k]]);
    double bi = b[row];
    dd_add(a, -bi);
    double ri = -dd_round(a);
    dd_add_prod(r2, ri, ri);
    dd_add_prod(b2, bi, bi);
  }
  wg_store_partial(r2, rpart, lb);
  if (bpart) {
    __syncthreads();
    wg_store_partial(b2, bpart, lb);
  }
}

// Gershgorin: partial maxima of RN(sum_j |a_ij|).
__global__ __launch_bounds__(WG) void k_gershgorin(DevMat A, double* __restrict__ part) {
  __shared__ double lm[SLICES_PER_WG];
  int nb = (A.nslices + SLICES_PER_WG - 1) / SLICES_PER_WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  int slice = lb * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  int lane = threadIdx.x & (SSCG_WAVE - 1);
  int row = slice * SSCG_WAVE + lane;
  double m = 0.0;
  if (slice < A.nslices && row < A.n) {
    int64_t o = A.off[slice] + lane;
    int w = A.width[slice];
    dd a = dd_zero();
    for (int j = 0; j < w; ++j) dd_add(a, fabs(A.val[o + (int64_t)j * SSCG_WAVE]));
    m = dd_round(a);
  }
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) m = fmax(m, __shfl_xor(m, k, SSCG_WAVE));
  if (lane == 0) lm[threadIdx.x / SSCG_WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = lm[0];
    for (int q = 1; q < SLICES_PER_WG; ++q) t = fmax(t, lm[q]);
    part[lb] = t;
  }
}

// Lanczos: w_i = RN((A v)_i - beta_prev vprev_i); partials of w.v.  VI: the
// values come from the slice's value table (same bits), as in the passes;
// SD: the slice-diagonal form (its terms in distance order: every row sum is
// correctly rounded, so the order does not change it).
template <bool C16, bool VI = false, bool SD = false>
__global__ __launch_bounds__(WG) void k_lanczos_spmv(DevMat A, const double* __restrict__ v,
                                                     const double* __restrict__ vprev,
                                                     const double* __restrict__ beta_prev,
                                                     double* __restrict__ w,
                                                     double* __restrict__ part) {
  int nb = (A.nslices + SLICES_PER_WG - 1) / SLICES_PER_WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  const int slice =  // uniform over the wavefront
      __builtin_amdgcn_readfirstlane(lb * SLICES_PER_WG + (int)(threadIdx.x / SSCG_WAVE));
  int lane = threadIdx.x & (SSCG_WAVE - 1);
  int row = slice * SSCG_WAVE + lane;
  dd d = dd_zero();
  if (slice < A.nslices) {
    dd a = dd_zero();
    if constexpr (SD) {
      const int us = __builtin_amdgcn_readfirstlane(slice);
      const int nd = A.sd_nd[us];
      int dl[SD_DIAG];
      double sv[SD_VALS];
#pragma unroll
      for (int k = 0; k < SD_DIAG; ++k) dl[k] = A.sd_delta[(int64_t)us * SD_DIAG + k];
#pragma unroll
      for (int i = 0; i < SD_VALS; ++i) sv[i] = A.sd_tab[(int64_t)us * 4 + i];
      const unsigned code = A.sd_code[row];
      unsigned pm = 0;  // bit k: the row has an entry at distance k
#pragma unroll
      for (int k = 0; k < SD_DIAG; ++k)
        if (k < nd && ((code >> (2 * k)) & 3u) != (unsigned)SD_ABSENT) pm |= 1u << k;
      double g[SD_DIAG];
#pragma unroll
      for (int k = 0; k < SD_DIAG; ++k)
        if (pm & (1u << k)) g[k] = v[row + dl[k]];
#pragma unroll
      for (int k = 0; k < SD_DIAG; ++k) {
        if (pm & (1u << k)) {
          const unsigned cd = (code >> (2 * k)) & 3u;
          dd_add_prod(a, cd == 0u ? sv[0] : (cd == 1u ? sv[1] : sv[2]), g[k]);
        }
      }
    } else {
    int64_t o = A.off[slice] + lane;
    int wd = A.width[slice];
    double tv[VTAB];
    if (VI) {
      const int us = __builtin_amdgcn_readfirstlane(slice);
#pragma unroll
      for (int i = 0; i < VTAB; ++i) tv[i] = A.vtab[(int64_t)us * VTAB + i];
    }
    // chunks of CH entries, every load of a chunk issued before its first use
    // (the terms are added in entry order, as one at a time)
    constexpr int CH = 4;
    for (int j0 = 0; j0 < wd; j0 += CH) {
      double av[CH], g[CH];
      int c[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int64_t k = o + (int64_t)(j0 + u) * SSCG_WAVE;
        const bool in = j0 + u < wd;
        if (VI) {
          const int ix = in ? (int)A.vidx[k] : 0;
          double t = tv[VTAB - 1];
#pragma unroll
          for (int i = VTAB - 2; i >= 0; --i) t = ix == i ? tv[i] : t;
          av[u] = in ? t : 0.0;
        } else {
          av[u] = in ? A.val[k] : 0.0;
        }
        if (C16) c[u] = in ? slice * SSCG_WAVE + (int)A.col16[k] : 0;
        else c[u] = in ? A.col[k] : 0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (j0 + u < wd) g[u] = v[c[u]];
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (j0 + u < wd) dd_add_prod(a, av[u], g[u]);
    }
    }  // SELL forms
    if (row < A.n) {
      if (vprev) dd_add_prod(a, -(*beta_prev), vprev[row]);
      double wi = dd_round(a);
      w[row] = wi;
      dd_add_prod(d, wi, v[row]);
    }
  }
  wg_store_partial(d, part, lb);
}

inline int wg_count(int nslices) { return (nslices + SLICES_PER_WG - 1) / SLICES_PER_WG; }


// ---------------------------------------------------------------- FP32 pass
// VI: the values come from the FP64 value tables rounded to FP32, the same
// bits as val32 (which is the FP64 copy rounded entry by entry).
template <int NRHS, bool CHEB, bool HASW, bool C16, bool VI = false>
__global__ __launch_bounds__(WG) void k_mpk32(DevMat A, const float* __restrict__ val32,
                                              double theta, double sigma, double gamma,
                                              MpkSeq32 s0, MpkSeq32 s1) {
  int nb = (A.nslices + SLICES_PER_WG - 1) / SLICES_PER_WG;
  int lb = xcd_block(nb);
  if (lb >= nb) return;
  const int slice =  // uniform over the wavefront
      __builtin_amdgcn_readfirstlane(lb * SLICES_PER_WG + (int)(threadIdx.x / SSCG_WAVE));
  if (slice >= A.nslices) return;
  int lane = threadIdx.x & (SSCG_WAVE - 1);
  int row = slice * SSCG_WAVE + lane;
  int64_t o = A.off[slice] + lane;
  int w = A.width[slice];
  const float* __restrict__ u0 = s0.u;
  const float* __restrict__ u1 = s1.u;
  double a0 = 0.0, a1 = 0.0;
  float tv[VTAB];
  if (VI) {
    const int us = __builtin_amdgcn_readfirstlane(slice);
#pragma unroll
    for (int i = 0; i < VTAB; ++i) tv[i] = (float)A.vtab[(int64_t)us * VTAB + i];
  }
  constexpr int CH = 4;
  for (int j0 = 0; j0 < w; j0 += CH) {
    float v[CH], g0[CH], g1[CH];
    int c[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      int64_t k = o + (int64_t)(j0 + u) * SSCG_WAVE;
      bool in = j0 + u < w;
      if (VI) {
        const int ix = in ? (int)A.vidx[k] : 0;
        float t = tv[VTAB - 1];
#pragma unroll
        for (int i = VTAB - 2; i >= 0; --i) t = ix == i ? tv[i] : t;
        v[u] = in ? t : 0.0f;
      } else {
        v[u] = in ? val32[k] : 0.0f;
      }
      if (C16) c[u] = in ? slice * SSCG_WAVE + (int)A.col16[k] : 0;
      else c[u] = in ? A.col[k] : 0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (j0 + u < w) {
        g0[u] = u0[c[u]];
        if (NRHS == 2) g1[u] = u1[c[u]];
      }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (j0 + u < w) {  // products of FP32 values are exact in FP64
        a0 = a0 + (double)v[u] * (double)g0[u];
        if (NRHS == 2) a1 = a1 + (double)v[u] * (double)g1[u];
      }
  }
  if (row >= A.n) return;
  if (CHEB) {
    double t0 = a0 - theta * (double)u0[row];
    if (HASW) t0 = t0 - sigma * (double)s0.w[row];
    s0.out[row] = (float)(t0 / gamma);
    if (NRHS == 2) {
      double t1 = a1 - theta * (double)u1[row];
      if (HASW) t1 = t1 - sigma * (double)s1.w[row];
      s1.out[row] = (float)(t1 / gamma);
    }
  } else {
    s0.out[row] = (float)a0;
    if (NRHS == 2) s1.out[row] = (float)a1;
  }
}

// ---------------------------------------------------------------- row order of batched systems
//
// SELL-64 pads every slice to its longest row; for rows of uneven length (a
// random graph's degrees) that stores up to twice the nonzeros.  A batched
// system's rows are therefore ordered within windows of ROW_WIN rows by
// descending length (stable), when that shrinks the window's padded size
// by at least 5 %; otherwise (stencils, whose rows are nearly equal and whose
// natural order keeps the gathers coalesced) the window keeps its order.
// perm[p] = original row at position p (-1: padding), inv[row] = position.
// Every row keeps its entries and their order, and every sum over rows is
// correctly rounded, so the order changes no result.
constexpr int ROW_WIN = 1024;

__device__ __forceinline__ int win_padded(const uint32_t* key) {
  // sum of the 16 slice widths of a window from the length groups in the keys
  __shared__ int wsum[ROW_WIN / SSCG_WAVE];
  const int t = threadIdx.x;
  if (t < ROW_WIN / SSCG_WAVE) {
    int w = 0;
    for (int i = 0; i < SSCG_WAVE; ++i) {
      const uint32_t k = key[t * SSCG_WAVE + i];
      const int g = (int)(k >> 10);
      w = max(w, k == 0xFFFFFFFFu || g >= 255 ? 0 : 254 - g);
    }
    wsum[t] = w;
  }
  __syncthreads();
  int s = 0;
  for (int i = 0; i < ROW_WIN / SSCG_WAVE; ++i) s += wsum[i];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(ROW_WIN / 2) void k_row_order(const int32_t* __restrict__ rowptr,
                                                           int n, int npad, int row0,
                                                           int32_t* __restrict__ perm,
                                                           int32_t* __restrict__ inv) {
  __shared__ uint32_t key[ROW_WIN];
  const int w0 = blockIdx.x * ROW_WIN;
  const int t = threadIdx.x;
  for (int i = t; i < ROW_WIN; i += ROW_WIN / 2) {
    const int r = w0 + i;
    uint32_t k = 0xFFFFFFFFu;  // past the system: last
    if (r < npad) {
      int g = 255;  // padding rows after the system's rows
      if (r < n) g = 254 - min(max(rowptr[r + 1] - rowptr[r], 0), 254);
      k = ((uint32_t)g << 10) | (uint32_t)i;
    }
    key[i] = k;
  }
  __syncthreads();
  const int natural = win_padded(key);
  // bitonic sort, ascending: longer rows first, ties in row order
  for (int k = 2; k <= ROW_WIN; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int i = 2 * t - (t & (j - 1));
      const int l = i + j;
      const uint32_t a = key[i], b = key[l];
      if ((a > b) == ((i & k) == 0)) {
        key[i] = b;
        key[l] = a;
      }
      __syncthreads();
    }
  }
  const bool sorted = (int64_t)win_padded(key) * 20 < (int64_t)natural * 19;
  for (int i = t; i < ROW_WIN && w0 + i < npad; i += ROW_WIN / 2) {
    const int r = w0 + (sorted ? (int)(key[i] & 1023u) : i);
    perm[row0 + w0 + i] = r < n ? r : -1;
    if (r < n) inv[row0 + r] = row0 + w0 + i;
  }
}

__global__ __launch_bounds__(WG) void k_sell_widths_perm(const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ perm,
                                                         int nslices, int32_t* __restrict__ width) {
  int slice = blockIdx.x * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  if (slice >= nslices) return;
  const int row = perm[slice * SSCG_WAVE + (threadIdx.x & (SSCG_WAVE - 1))];
  int len = row >= 0 ? rowptr[row + 1] - rowptr[row] : 0;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) len = max(len, __shfl_xor(len, m, SSCG_WAVE));
  if ((threadIdx.x & (SSCG_WAVE - 1)) == 0) width[slice] = len;
}

// One thread per position; columns become positions (inv, global rows).
__global__ __launch_bounds__(WG) void k_sell_fill_perm(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ inv, const int64_t* __restrict__ off,
    const int32_t* __restrict__ width, int nslices, int row0, int32_t* __restrict__ scol,
    double* __restrict__ sval, unsigned long long* __restrict__ cnt) {
  const int pos = blockIdx.x * WG + threadIdx.x;
  const int slice = pos / SSCG_WAVE;
  if (slice >= nslices) return;  // whole wavefronts (nslices * 64 threads)
  const int lane = pos & (SSCG_WAVE - 1);
  const int64_t o = off[slice];
  const int w = width[slice];
  const int row = perm[pos];
  int k0 = 0, len = 0;
  if (row >= 0) {
    k0 = rowptr[row];
    len = rowptr[row + 1] - k0;
  }
  int scattered = 0;
  for (int j = 0; j < w; ++j) {
    const int64_t dst = o + (int64_t)j * SSCG_WAVE + lane;
    int c;
    if (j < len) {
      c = inv[row0 + col[k0 + j]];
      sval[dst] = val[k0 + j];
    } else {
      c = row0 + pos;
      sval[dst] = 0.0;
    }
    scol[dst] = c;
    int lo = c, hi = c;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      lo = min(lo, __shfl_xor(lo, m, SSCG_WAVE));
      hi = max(hi, __shfl_xor(hi, m, SSCG_WAVE));
    }
    scattered += hi - lo >= 256;
  }
  if (lane == 0) {
    atomicAdd(cnt, (unsigned long long)w * SSCG_WAVE);
    atomicAdd(cnt + 1, (unsigned long long)scattered * SSCG_WAVE);
  }
}

__global__ void k_set_il(BatchSys* __restrict__ sys, const unsigned long long* __restrict__ cnt,
                         int q0, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int q = q0 + i;
  sys[q].il = cnt[2 * q + 1] * 4 > cnt[2 * q] ? 1 : 0;
}

// Compact forms of the batched matrix over slices [sl0, sl0 + count), one
// wavefront per slice: 16-bit column offsets (as k_sell_compact) and the
// value table with one-byte indices (as k_sell_vidx).  A slice with an
// offset beyond 16 bits or more than VTAB values adds one to its system's
// count; k_set_vt then lets a system's passes read the compact forms only if
// none of its slices did.
__global__ __launch_bounds__(WG) void k_sell_forms_batch(
    const int32_t* __restrict__ scol, const double* __restrict__ val,
    const int64_t* __restrict__ off, const int32_t* __restrict__ width, int sl0, int count,
    const int32_t* __restrict__ blk_sys, int16_t* __restrict__ col16, double* __restrict__ vtab,
    uint8_t* __restrict__ vidx, int32_t* __restrict__ cnt) {
  const int i = blockIdx.x * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  if (i >= count) return;  // whole wavefronts
  const int slice = sl0 + i;
  const int q = blk_sys[slice / SLICES_PER_WG];
  if (q < 0) return;
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  const int64_t o = off[slice] + lane;
  const int w = width[slice];
  const int base = slice * SSCG_WAVE;
  long long tb = 0;
  int m = 0;
  bool over = false, far = false;
  for (int j = 0; j < w; ++j) {
    const int64_t k = o + (int64_t)j * SSCG_WAVE;
    const int d = scol[k] - base;
    far |= d < -32768 || d > 32767;
    col16[k] = (int16_t)d;
    vidx[k] = (uint8_t)vtab_index(val[k], lane, tb, m, over);
  }
  if (lane < VTAB) vtab[(int64_t)slice * VTAB + lane] = __longlong_as_double(lane < m ? tb : 0);
  if (__ballot(far || over) != 0 && lane == 0) atomicAdd(cnt + q, 1);
}

__global__ void k_set_vt(BatchSys* __restrict__ sys, const int32_t* __restrict__ cnt, int q0,
                         int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int q = q0 + i;
  sys[q].vt = cnt[q] == 0 ? 1 : 0;
}

// dst[p] = src[perm[p]] (0 for padding), p < npad.
__global__ __launch_bounds__(WG) void k_gather_perm(const double* __restrict__ src,
                                                    const int32_t* __restrict__ perm, int npad,
                                                    double* __restrict__ dst) {
  const int p = blockIdx.x * WG + threadIdx.x;
  if (p >= npad) return;
  const int r = perm[p];
  dst[p] = r >= 0 ? src[r] : 0.0;
}

// dst[perm[p]] = src[p] for the system's rows.
__global__ __launch_bounds__(WG) void k_scatter_perm(const double* __restrict__ src,
                                                     const int32_t* __restrict__ perm, int npad,
                                                     double* __restrict__ dst) {
  const int p = blockIdx.x * WG + threadIdx.x;
  if (p >= npad) return;
  const int r = perm[p];
  if (r >= 0) dst[r] = src[p];
}

// t[i] = (a[i], b[i]), i < n.
__global__ __launch_bounds__(WG) void k_pair(const double* __restrict__ a,
                                             const double* __restrict__ b, int64_t n,
                                             double2* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < n) t[i] = make_double2(a[i], b[i]);
}

__global__ __launch_bounds__(WG) void k_cast_f32(const double* __restrict__ in, int64_t n,
                                                 float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}
}  // namespace

// ---------------------------------------------------------------- launches

hipError_t launch_check_csr(const int32_t* rowptr, const int32_t* col, int n, int64_t nnz,
                            int32_t* flag, hipStream_t st) {
  int64_t m = n > nnz ? n : nnz;
  hipLaunchKernelGGL(k_check_csr, dim3((unsigned)((m + WG - 1) / WG)), dim3(WG), 0, st, rowptr, col,
                     n, nnz, flag);
  return hipGetLastError();
}

hipError_t launch_sell_widths(const int32_t* rowptr, int n, int32_t* width, hipStream_t st) {
  int nslices = (n + SSCG_WAVE - 1) / SSCG_WAVE;
  hipLaunchKernelGGL(k_sell_widths, dim3(wg_count(nslices)), dim3(WG), 0, st, rowptr, n, nslices,
                     width);
  return hipGetLastError();
}

hipError_t launch_scan_offsets(const int32_t* width, int nslices, int64_t* off, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, st, width, nslices, (int64_t)0, off,
                     off + nslices);
  return hipGetLastError();
}

hipError_t launch_scan_offsets_base(const int32_t* width, int nslices, int64_t base, int64_t* off,
                                    int64_t* end, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, st, width, nslices, base, off, end);
  return hipGetLastError();
}

hipError_t launch_row_scale(const int32_t* rowptr, const double* val, int n, double* scale,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_row_scale, dim3((n + WG - 1) / WG), dim3(WG), 0, st, rowptr, val, n, scale);
  return hipGetLastError();
}

hipError_t launch_sell_fill(const int32_t* rowptr, const int32_t* col, const double* val, int n,
                            const double* scale, const int64_t* off, const int32_t* width,
                            int32_t* scol, double* sval, hipStream_t st) {
  int nslices = (n + SSCG_WAVE - 1) / SSCG_WAVE;
  int threads = nslices * SSCG_WAVE;
  hipLaunchKernelGGL(k_sell_fill, dim3((threads + WG - 1) / WG), dim3(WG), 0, st, rowptr, col, val,
                     n, scale, off, width, nslices, 0, scol, sval);
  return hipGetLastError();
}

hipError_t launch_sell_vidx(const double* val, const int64_t* off, const int32_t* width,
                            int nslices, double* vtab, uint8_t* vidx, int32_t* flag,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_sell_vidx, dim3(wg_count(nslices)), dim3(WG), 0, st, val, off, width,
                     nslices, vtab, vidx, flag);
  return hipGetLastError();
}

hipError_t launch_sell_sdia(const int32_t* rowptr, int n, const int32_t* scol, const double* sval,
                            const int64_t* off, const int32_t* width, int nslices, int32_t* sd_nd,
                            int32_t* sd_delta, double* sd_tab, uint16_t* sd_code, int32_t* flag,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_sell_sdia, dim3(wg_count(nslices)), dim3(WG), 0, st, rowptr, n, scol, sval,
                     off, width, nslices, sd_nd, sd_delta, sd_tab, sd_code, flag);
  return hipGetLastError();
}

// *flag = 1 if slices 2t and 2t + 1 differ in their count, distances or
// values (bit patterns) for some t; the tables are stored sorted, so equal
// slices have equal tables.
__global__ __launch_bounds__(WG) void k_sd_pairs(const int32_t* __restrict__ sd_nd,
                                                 const int32_t* __restrict__ sd_delta,
                                                 const double* __restrict__ sd_tab, int nslices,
                                                 int32_t* __restrict__ flag) {
  const int t = blockIdx.x * WG + threadIdx.x;
  const int a = 2 * t, b = 2 * t + 1;
  if (b >= nslices) return;
  bool same = sd_nd[a] == sd_nd[b];
  for (int k = 0; k < SD_DIAG; ++k)
    same = same && sd_delta[(int64_t)a * SD_DIAG + k] == sd_delta[(int64_t)b * SD_DIAG + k];
  for (int i = 0; i < 4; ++i)
    same = same && __double_as_longlong(sd_tab[(int64_t)a * 4 + i]) ==
                       __double_as_longlong(sd_tab[(int64_t)b * 4 + i]);
  if (!same) atomicOr(flag, 1);
}

hipError_t launch_sd_pairs(const int32_t* sd_nd, const int32_t* sd_delta, const double* sd_tab,
                           int nslices, int32_t* flag, hipStream_t st) {
  const int np = (nslices + 1) / 2;
  hipLaunchKernelGGL(k_sd_pairs, dim3((np + WG - 1) / WG), dim3(WG), 0, st, sd_nd, sd_delta,
                     sd_tab, nslices, flag);
  return hipGetLastError();
}

// One wavefront per slice: for each distance k, the value code of the rows
// that have an entry there, if they all have the same one.
__global__ __launch_bounds__(WG) void k_sd_values(const int32_t* __restrict__ sd_nd,
                                                  const uint16_t* __restrict__ sd_code,
                                                  int nslices, uint32_t* __restrict__ sd_vk,
                                                  int32_t* __restrict__ flag) {
  const int t = blockIdx.x * SLICES_PER_WG + threadIdx.x / SSCG_WAVE;
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  if (t >= nslices) return;  // uniform over the wavefront
  const int nd = sd_nd[t];
  const unsigned code = sd_code[(int64_t)t * SSCG_WAVE + lane];
  uint32_t vk = 0;
  bool bad = false;
  for (int k = 0; k < SD_DIAG; ++k) {
    const unsigned ck = k < nd ? (code >> (2 * k)) & 3u : (unsigned)SD_ABSENT;
    const bool pr = ck != (unsigned)SD_ABSENT;
    const unsigned long long m = __ballot(pr);
    const unsigned ref = m ? (unsigned)__shfl((int)ck, __ffsll((long long)m) - 1, SSCG_WAVE)
                           : (unsigned)SD_ABSENT;
    bad = bad || __ballot(pr && ck != ref) != 0ull;
    vk |= ref << (2 * k);
  }
  if (lane == 0) {
    sd_vk[t] = vk;
    if (bad) atomicOr(flag, 1);
  }
}

// *flag = 1 if slices 2t and 2t + 1 differ in their value codes for some t.
__global__ __launch_bounds__(WG) void k_sd_vpairs(const uint32_t* __restrict__ sd_vk, int nslices,
                                                  int32_t* __restrict__ flag) {
  const int t = blockIdx.x * WG + threadIdx.x;
  if (2 * t + 1 < nslices && sd_vk[2 * t] != sd_vk[2 * t + 1]) atomicOr(flag, 1);
}

hipError_t launch_sd_values(const int32_t* sd_nd, const uint16_t* sd_code, int nslices,
                            uint32_t* sd_vk, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_sd_values, dim3(wg_count(nslices)), dim3(WG), 0, st, sd_nd, sd_code,
                     nslices, sd_vk, flag);
  const int np = (nslices + 1) / 2;
  hipLaunchKernelGGL(k_sd_vpairs, dim3((np + WG - 1) / WG), dim3(WG), 0, st, sd_vk, nslices,
                     flag + 1);
  return hipGetLastError();
}

hipError_t launch_sell_sdia_sys(const int32_t* rowptr, const int32_t* perm, int slice0, int nsl,
                                const int32_t* scol, const double* sval, const int64_t* off,
                                const int32_t* width, int32_t* sd_nd, int32_t* sd_delta,
                                double* sd_tab, uint16_t* sd_code, int32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_sell_sdia_sys, dim3(wg_count(nsl)), dim3(WG), 0, st, rowptr, perm, slice0,
                     nsl, scol, sval, off, width, sd_nd, sd_delta, sd_tab, sd_code, cnt);
  return hipGetLastError();
}

hipError_t launch_set_sd(BatchSys* sys, const int32_t* cnt, int q0, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_set_sd, dim3((count + 255) / 256), dim3(256), 0, st, sys, cnt, q0, count);
  return hipGetLastError();
}

hipError_t launch_sell_compact(const int32_t* scol, int n, const int64_t* off,
                               const int32_t* width, int16_t* col16, int32_t* flag,
                               hipStream_t st) {
  int nslices = (n + SSCG_WAVE - 1) / SSCG_WAVE;
  int threads = nslices * SSCG_WAVE;
  hipLaunchKernelGGL(k_sell_compact, dim3((threads + WG - 1) / WG), dim3(WG), 0, st, scol, n, off,
                     width, nslices, col16, flag);
  return hipGetLastError();
}

hipError_t launch_sell_widths_n(const int32_t* rowptr, int n, int nslices, int32_t* width,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_sell_widths, dim3(wg_count(nslices)), dim3(WG), 0, st, rowptr, n, nslices,
                     width);
  return hipGetLastError();
}

hipError_t launch_sell_fill_off(const int32_t* rowptr, const int32_t* col, const double* val,
                                int n, int nslices, const int64_t* off, const int32_t* width,
                                int col_off, int32_t* scol, double* sval, hipStream_t st) {
  int threads = nslices * SSCG_WAVE;
  hipLaunchKernelGGL(k_sell_fill, dim3((threads + WG - 1) / WG), dim3(WG), 0, st, rowptr, col, val,
                     n, (const double*)nullptr, off, width, nslices, col_off, scol, sval);
  return hipGetLastError();
}

hipError_t launch_row_order(const int32_t* rowptr, int n, int npad, int row0, int32_t* perm,
                            int32_t* inv, hipStream_t st) {
  hipLaunchKernelGGL(k_row_order, dim3((npad + ROW_WIN - 1) / ROW_WIN), dim3(ROW_WIN / 2), 0, st,
                     rowptr, n, npad, row0, perm, inv);
  return hipGetLastError();
}

hipError_t launch_sell_widths_perm(const int32_t* rowptr, const int32_t* perm, int nslices,
                                   int32_t* width, hipStream_t st) {
  hipLaunchKernelGGL(k_sell_widths_perm, dim3(wg_count(nslices)), dim3(WG), 0, st, rowptr, perm,
                     nslices, width);
  return hipGetLastError();
}

hipError_t launch_sell_fill_perm(const int32_t* rowptr, const int32_t* col, const double* val,
                                 const int32_t* perm, const int32_t* inv, int nslices,
                                 const int64_t* off, const int32_t* width, int row0,
                                 int32_t* scol, double* sval, unsigned long long* cnt,
                                 hipStream_t st) {
  const int threads = nslices * SSCG_WAVE;
  hipLaunchKernelGGL(k_sell_fill_perm, dim3((threads + WG - 1) / WG), dim3(WG), 0, st, rowptr,
                     col, val, perm, inv, off, width, nslices, row0, scol, sval, cnt);
  return hipGetLastError();
}

hipError_t launch_set_il(BatchSys* sys, const unsigned long long* cnt, int q0, int count,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_set_il, dim3((count + 63) / 64), dim3(64), 0, st, sys, cnt, q0, count);
  return hipGetLastError();
}

hipError_t launch_sell_forms_batch(const int32_t* scol, const double* val, const int64_t* off,
                                   const int32_t* width, int sl0, int count,
                                   const int32_t* blk_sys, int16_t* col16, double* vtab,
                                   uint8_t* vidx, int32_t* cnt, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sell_forms_batch, dim3(wg_count(count)), dim3(WG), 0, st, scol, val, off,
                     width, sl0, count, blk_sys, col16, vtab, vidx, cnt);
  return hipGetLastError();
}

hipError_t launch_set_vt(BatchSys* sys, const int32_t* cnt, int q0, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_set_vt, dim3((count + 63) / 64), dim3(64), 0, st, sys, cnt, q0, count);
  return hipGetLastError();
}

hipError_t launch_gather_perm(const double* src, const int32_t* perm, int npad, double* dst,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_gather_perm, dim3((npad + WG - 1) / WG), dim3(WG), 0, st, src, perm, npad,
                     dst);
  return hipGetLastError();
}

hipError_t launch_scatter_perm(const double* src, const int32_t* perm, int npad, double* dst,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_perm, dim3((npad + WG - 1) / WG), dim3(WG), 0, st, src, perm, npad,
                     dst);
  return hipGetLastError();
}

hipError_t launch_pair(const double* a, const double* b, int64_t n, double2* t, hipStream_t st) {
  hipLaunchKernelGGL(k_pair, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, st, a, b, n, t);
  return hipGetLastError();
}

hipError_t launch_mpk_batch(const DevMat& A, int j, int cheb, int nrhs, MpkSeq s0, MpkSeq s1,
                            MpkSeq32 f0, MpkSeq32 f1, const BatchSys* sys,
                            const int32_t* blk_sys, const int32_t* ablk, const int32_t* nl,
                            int gblk, int chunk, const MpkResidual& res, const double2* tg,
                            double2* tw, hipStream_t st) {
  dim3 grid(batch_grid(gblk));
  const bool r = res.x != nullptr;
#define SSCG_MPK_BATCH(N, C, R)                                                                 \
  do {                                                                                          \
    if (chunk == 2)                                                                             \
      hipLaunchKernelGGL((k_mpk_batch<N, C, R, 2>), grid, dim3(WG), 0, st, A, j, s0, s1, f0, f1, \
                         sys, blk_sys, ablk, nl, res.x, res.b, res.part, tg, tw);               \
    else if (chunk == 8)                                                                        \
      hipLaunchKernelGGL((k_mpk_batch<N, C, R, 8>), grid, dim3(WG), 0, st, A, j, s0, s1, f0, f1, \
                         sys, blk_sys, ablk, nl, res.x, res.b, res.part, tg, tw);               \
    else                                                                                        \
      hipLaunchKernelGGL((k_mpk_batch<N, C, R, 4>), grid, dim3(WG), 0, st, A, j, s0, s1, f0, f1, \
                         sys, blk_sys, ablk, nl, res.x, res.b, res.part, tg, tw);               \
  } while (0)
  if (nrhs == 2) {
    if (cheb) { if (r) SSCG_MPK_BATCH(2, true, true); else SSCG_MPK_BATCH(2, true, false); }
    else { if (r) SSCG_MPK_BATCH(2, false, true); else SSCG_MPK_BATCH(2, false, false); }
  } else {
    if (cheb) { if (r) SSCG_MPK_BATCH(1, true, true); else SSCG_MPK_BATCH(1, true, false); }
    else { if (r) SSCG_MPK_BATCH(1, false, true); else SSCG_MPK_BATCH(1, false, false); }
  }
#undef SSCG_MPK_BATCH
  return hipGetLastError();
}

template <int NRHS, bool CHEB, bool HASW, bool C16, bool VI, bool SD = false, bool UV = false>
void mpk_launch_c(dim3 grid, const DevMat& A, double theta, double sigma, double gamma, MpkSeq s0,
                  MpkSeq s1, Gate g, const MpkResidual& res, hipStream_t st) {
  if (res.x)
    hipLaunchKernelGGL((k_mpk<NRHS, CHEB, HASW, true, C16, VI, SD, UV>), grid, dim3(WG), 0, st, A,
                       theta, sigma, gamma, s0, s1, g, res.x, res.b, res.part);
  else
    hipLaunchKernelGGL((k_mpk<NRHS, CHEB, HASW, false, C16, VI, SD, UV>), grid, dim3(WG), 0, st,
                       A, theta, sigma, gamma, s0, s1, g, nullptr, nullptr, nullptr);
}

template <int NRHS, bool CHEB, bool HASW, bool UV>
void mpk_launch_sdp(dim3 grid, const DevMat& A, double theta, double sigma, double gamma,
                    MpkSeq s0, MpkSeq s1, Gate g, const MpkResidual& res, hipStream_t st) {
  if (res.x)
    hipLaunchKernelGGL((k_mpk_sdp<NRHS, CHEB, HASW, true, UV>), grid, dim3(2 * SSCG_WAVE), 0, st,
                       A, theta, sigma, gamma, s0, s1, g, res.x, res.b, res.part);
  else
    hipLaunchKernelGGL((k_mpk_sdp<NRHS, CHEB, HASW, false, UV>), grid, dim3(2 * SSCG_WAVE), 0, st,
                       A, theta, sigma, gamma, s0, s1, g, nullptr, nullptr, nullptr);
}

// The compact forms the copy has: the slice-diagonal form (in pairs of
// slices where they agree), else 16-bit column offsets, and value indices
// with them.
template <int NRHS, bool CHEB, bool HASW>
void mpk_launch(dim3 grid, const DevMat& A, double theta, double sigma, double gamma, MpkSeq s0,
                MpkSeq s1, Gate g, const MpkResidual& res, hipStream_t st) {
  if (A.sd_code && A.sd_pair) {
    if (A.sd_vk)
      mpk_launch_sdp<NRHS, CHEB, HASW, true>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
    else
      mpk_launch_sdp<NRHS, CHEB, HASW, false>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
  } else if (A.sd_code && A.sd_vk)
    mpk_launch_c<NRHS, CHEB, HASW, false, false, true, true>(grid, A, theta, sigma, gamma, s0, s1,
                                                             g, res, st);
  else if (A.sd_code)
    mpk_launch_c<NRHS, CHEB, HASW, false, false, true>(grid, A, theta, sigma, gamma, s0, s1, g,
                                                       res, st);
  else if (A.col16 && A.vidx)
    mpk_launch_c<NRHS, CHEB, HASW, true, true>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
  else if (A.col16)
    mpk_launch_c<NRHS, CHEB, HASW, true, false>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
  else
    mpk_launch_c<NRHS, CHEB, HASW, false, false>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
}

hipError_t launch_mpk_pass(const DevMat& A, int j, BasisPrm bp, int nrhs, MpkSeq s0, MpkSeq s1,
                           Gate g, const MpkResidual& res, hipStream_t st) {
  dim3 grid(xcd_grid(wg_count(A.nslices)));
  if (bp.newton) {  // (A - theta_{j-1} I) u: the j = 1 form, gamma = 1
    const double th = bp.th[j - 1];
    if (nrhs == 2) mpk_launch<2, true, false>(grid, A, th, 0.0, 1.0, s0, s1, g, res, st);
    else mpk_launch<1, true, false>(grid, A, th, 0.0, 1.0, s0, s1, g, res, st);
    return hipGetLastError();
  }
  if (!bp.cheb) {
    if (nrhs == 2) mpk_launch<2, false, false>(grid, A, 0.0, 0.0, 1.0, s0, s1, g, res, st);
    else mpk_launch<1, false, false>(grid, A, 0.0, 0.0, 1.0, s0, s1, g, res, st);
    return hipGetLastError();
  }
  double theta = bp.c0;
  double gamma = j == 1 ? bp.h : bp.h2;
  double sigma = bp.h2;
  if (j == 1) {
    if (nrhs == 2) mpk_launch<2, true, false>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
    else mpk_launch<1, true, false>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
  } else {
    if (nrhs == 2) mpk_launch<2, true, true>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
    else mpk_launch<1, true, true>(grid, A, theta, sigma, gamma, s0, s1, g, res, st);
  }
  return hipGetLastError();
}

int residual_nparts(int n) {
  int nslices = (n + SSCG_WAVE - 1) / SSCG_WAVE;
  return wg_count(nslices);
}

hipError_t launch_residual(const DevMat& A, const double* b, const double* x, double* r,
                           double* rpart, double* bpart, int* nparts, hipStream_t st) {
  int nb = wg_count(A.nslices);
  *nparts = nb;
  hipLaunchKernelGGL(k_residual, dim3(xcd_grid(nb)), dim3(WG), 0, st, A, b, x, r, rpart, bpart);
  return hipGetLastError();
}

int csr_residual_nparts(int n) { return (n + WG - 1) / WG; }

hipError_t launch_csr_residual(const int32_t* rowptr, const int32_t* col, const double* val,
                               int n, const double* b, const double* x, double* rpart,
                               double* bpart, hipStream_t st) {
  int nb = csr_residual_nparts(n);
  hipLaunchKernelGGL(k_csr_residual, dim3(xcd_grid(nb)), dim3(WG), 0, st, rowptr, col, val, n, b,
                     x, rpart, bpart);
  return hipGetLastError();
}

hipError_t launch_gershgorin(const DevMat& A, double* part, int* nparts, hipStream_t st) {
  int nb = wg_count(A.nslices);
  *nparts = nb;
  hipLaunchKernelGGL(k_gershgorin, dim3(xcd_grid(nb)), dim3(WG), 0, st, A, part);
  return hipGetLastError();
}

hipError_t launch_lanczos_step(const DevMat& A, const double* v, const double* vprev,
                               const double* beta_prev, double* w, double* part, int* nparts,
                               hipStream_t st) {
  int nb = wg_count(A.nslices);
  *nparts = nb;
  if (A.sd_code)
    hipLaunchKernelGGL((k_lanczos_spmv<false, false, true>), dim3(xcd_grid(nb)), dim3(WG), 0, st,
                       A, v, vprev, beta_prev, w, part);
  else if (A.col16 && A.vidx)
    hipLaunchKernelGGL((k_lanczos_spmv<true, true>), dim3(xcd_grid(nb)), dim3(WG), 0, st, A, v,
                       vprev, beta_prev, w, part);
  else if (A.col16)
    hipLaunchKernelGGL(k_lanczos_spmv<true>, dim3(xcd_grid(nb)), dim3(WG), 0, st, A, v, vprev,
                       beta_prev, w, part);
  else
    hipLaunchKernelGGL(k_lanczos_spmv<false>, dim3(xcd_grid(nb)), dim3(WG), 0, st, A, v, vprev,
                       beta_prev, w, part);
  return hipGetLastError();
}

// 16-bit column offsets (6 bytes per stored entry with the FP32 value) when
// the matrix copy has them, and value tables as well (3 bytes) when it has those.
template <int NRHS, bool CHEB, bool HASW>
static void mpk32_launch(const DevMat& A, const float* val32, double th, double sg, double gm,
                         MpkSeq32 s0, MpkSeq32 s1, hipStream_t st) {
  dim3 grid(xcd_grid(wg_count(A.nslices)));
  if (A.col16 && A.vidx)
    hipLaunchKernelGGL((k_mpk32<NRHS, CHEB, HASW, true, true>), grid, dim3(WG), 0, st, A, val32,
                       th, sg, gm, s0, s1);
  else if (A.col16)
    hipLaunchKernelGGL((k_mpk32<NRHS, CHEB, HASW, true>), grid, dim3(WG), 0, st, A, val32, th, sg,
                       gm, s0, s1);
  else
    hipLaunchKernelGGL((k_mpk32<NRHS, CHEB, HASW, false>), grid, dim3(WG), 0, st, A, val32, th,
                       sg, gm, s0, s1);
}

hipError_t launch_mpk32_pass(const DevMat& A, const float* val32, int j, BasisPrm bp, int nrhs,
                             MpkSeq32 s0, MpkSeq32 s1, hipStream_t st) {
  if (bp.newton) {
    const double th = bp.th[j - 1];
    if (nrhs == 2) mpk32_launch<2, true, false>(A, val32, th, 0.0, 1.0, s0, s1, st);
    else mpk32_launch<1, true, false>(A, val32, th, 0.0, 1.0, s0, s1, st);
    return hipGetLastError();
  }
  if (!bp.cheb) {
    if (nrhs == 2) mpk32_launch<2, false, false>(A, val32, 0.0, 0.0, 1.0, s0, s1, st);
    else mpk32_launch<1, false, false>(A, val32, 0.0, 0.0, 1.0, s0, s1, st);
    return hipGetLastError();
  }
  const double gamma = j == 1 ? bp.h : bp.h2;
  if (j == 1) {
    if (nrhs == 2) mpk32_launch<2, true, false>(A, val32, bp.c0, bp.h2, gamma, s0, s1, st);
    else mpk32_launch<1, true, false>(A, val32, bp.c0, bp.h2, gamma, s0, s1, st);
  } else {
    if (nrhs == 2) mpk32_launch<2, true, true>(A, val32, bp.c0, bp.h2, gamma, s0, s1, st);
    else mpk32_launch<1, true, true>(A, val32, bp.c0, bp.h2, gamma, s0, s1, st);
  }
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double* in, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_f32, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, st, in, n, out);
  return hipGetLastError();
}
