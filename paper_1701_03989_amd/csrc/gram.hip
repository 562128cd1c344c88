// Gram matrices G = Y^T Y on the FP64 matrix cores, in the stated order.
//
// The order (the oracle states it for Gram matrices): rows zero-padded to a
// multiple of GRAM_GROUP fall into groups of GRAM_GROUP consecutive rows; the
// partial of entry (a, b) over a group is the chain of IEEE fused
// multiply-adds s <- fma(y_ra, y_rb, s) over its rows in order, from +0; the
// group partials, zero-padded to the next power of two, are added pairwise
// (left half + right half, recursively).
//
// One wavefront per group.  v_mfma_f64_16x16x4f64 (D = A B + C, A 16 x 4,
// B 4 x 16) computes every output as the chain
//   fma(A[i][3], B[3][j], fma(A[i][2], B[2][j], fma(A[i][1], B[1][j],
//       fma(A[i][0], B[0][j], C[i][j]))))
// of IEEE FMAs (checked on MI355X against exact-rational models: every one of
// 379,904 outputs of random adversarial inputs matched this chain and no
// other model tried).  With the contraction index k = four consecutive rows
// and the accumulator chained through the group's rows in order, each output
// element is exactly the group partial above.  Columns come in blocks of 16;
// block pairs (0,0) for d <= 16, two blocks of a split for 17 <= d <= 24
// (below), (0,0) (0,1) (1,1) for d <= 32, six pairs for d <= 48.  Operand layouts: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; element v of the accumulator of lane l is
// D[l / 16 + 4 v][l % 16].
//
// The rows of a group pass through the wavefront's LDS tile (64 rows at a
// time, one row per lane, loaded column by column: each load is 512
// contiguous bytes); the next tile's loads are in flight while the current
// one feeds the matrix cores.
#include <type_traits>

#include "common.h"

namespace {

constexpr int GW = 4;    // wavefronts per workgroup, one group each
constexpr int GTR = 64;  // rows per tile (one per lane)

typedef double gd4 __attribute__((ext_vector_type(4)));

// Row stride of a wavefront's LDS tile (doubles; odd: the lanes' rows fall
// in different banks): 16 NB columns, or for the split blocking (d <= 24)
// columns 0..23 and the zero column SPLIT_ZC.
constexpr int SPLIT_NC = 24, SPLIT_ZC = 24;
template <int NB, bool SPLIT>
__host__ __device__ constexpr int tile_ld() {
  return SPLIT ? SPLIT_ZC + 1 : 16 * NB + 1;
}

__device__ __forceinline__ int pair_index(int a, int b, int d) {
  return a * d - a * (a - 1) / 2 + (b - a);  // row-major upper triangle, a <= b
}

// Row r of the columns is stored at position r (single systems).
struct SameRow {
  __device__ __forceinline__ int64_t operator()(int64_t r) const { return r; }
};

// The partials of one group (rows [r0, r0 + GRAM_GROUP), those >= rend read
// as 0) of the d columns of src, written to part[q * pstride + slot]; row r
// is read at position map(r).  tile: this wavefront's GTR x (16 NB + 1)
// doubles of LDS.  Called by a whole wavefront.
//
// SPLIT (NB = 2, 17 <= d <= 24: the two-sequence blocks of s = 8 .. 11):
// two 16 x 16 blocks instead of the three block pairs (0,0) (0,1) (1,1).
// With m = 32 - d, block A takes the row columns I = (0, .., m-1, 16, .., d-1)
// against the column columns J = (0, .., 15), block B the columns
// (m, .., d-1) (padded with a zero column) against themselves.  A holds the
// entries (a, b) with a < m, b <= 15 and, transposed, every (a, b) with
// a <= 15 < b; B those with m <= a <= b <= 15 and 16 <= a <= b.  Every entry
// is still the chain of one matrix-core FMA per row over the same rows in the
// same order (the product of two doubles does not depend on their order), so
// the bits are those of the general blocking.
template <int NB, class Src, class Map, bool SPLIT = false>
__device__ __forceinline__ void gram_group(const Src& src, int d, int64_t r0, int64_t rend,
                                           const Map& map, double* __restrict__ part,
                                           int64_t pstride, int64_t slot,
                                           double* __restrict__ tile) {
  static_assert(!SPLIT || NB == 2, "the split blocking has two column blocks");
  constexpr int NC = SPLIT ? SPLIT_NC : 16 * NB;  // columns fetched (at most)
  constexpr int LD = tile_ld<NB, SPLIT>();
  constexpr int NP = SPLIT ? 2 : NB * (NB + 1) / 2;
  const int lane = threadIdx.x & (SSCG_WAVE - 1);
  gd4 acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = gd4{0.0, 0.0, 0.0, 0.0};
  // columns d..LD-1 of the tile stay 0 (they only feed outputs that are dropped)
  for (int a = d; a < LD; ++a) tile[lane * LD + a] = 0.0;
  // the stored type of the columns: FP64, or FP32 (widened at the LDS store)
  using T = std::remove_cv_t<std::remove_reference_t<decltype(*src.at(0))>>;
  constexpr bool F32 = std::is_same<T, float>::value;
  T nx[NC];
  bool fin = false;  // the fetched row lies before rend
  // FP32 columns: the loads of a row are unconditional in the lane (a lane
  // condition would put each in a branch of its own, where the widening
  // would wait for it): a row past rend reads position 0 and its values are
  // replaced by 0 only at the LDS store one iteration later, so nothing waits
  // for a load before that store.  FP64 columns: the select is made at the
  // load, which measured faster for them.
  auto fetch = [&](int64_t rb) {
    const int64_t row = rb + lane;
    const bool in = row < rend;
    const int64_t pos = in ? map(row) : 0;
    if constexpr (F32) {
      fin = in;
#pragma unroll
      for (int a = 0; a < NC; ++a)
        if (a < d) nx[a] = src.at(a)[pos];  // d is uniform over the wavefront
    } else {
#pragma unroll
      for (int a = 0; a < NC; ++a) nx[a] = (a < d && in) ? src.at(a)[pos] : 0.0;
    }
  };
  fetch(r0);
  for (int t = 0; t < GRAM_GROUP / GTR; ++t) {
#pragma unroll
    for (int a = 0; a < NC; ++a)
      if (a < d) {
        if constexpr (F32) tile[lane * LD + a] = fin ? (double)nx[a] : 0.0;
        else tile[lane * LD + a] = nx[a];
      }
    // every lane's row is in LDS before any lane reads another's (LDS
    // operations of one wavefront complete in order; this keeps the compiler
    // from moving them across)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (t + 1 < GRAM_GROUP / GTR) fetch(r0 + (int64_t)(t + 1) * GTR);
    const int cc = lane & 15;
    // SPLIT: this lane's column in block A's row set and in block B's set
    // (SPLIT_ZC is a zero column of the tile)
    const int m = 32 - d;
    const int ia = cc < m ? cc : 16 + cc - m;
    const int ib = m + cc < d ? m + cc : SPLIT_ZC;
#pragma unroll
    for (int k4 = 0; k4 < GTR / 4; ++k4) {
      const int rr = 4 * k4 + (lane >> 4);
      if constexpr (SPLIT) {
        const double x0 = tile[rr * LD + cc];
        const double xa = tile[rr * LD + ia], xb = tile[rr * LD + ib];
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, x0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb, xb, acc[1], 0, 0, 0);
      } else {
        double x[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) x[b] = tile[rr * LD + 16 * b + cc];
        int p = 0;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
#pragma unroll
          for (int j = i; j < NB; ++j) {
            acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i], x[j], acc[p], 0, 0, 0);
            ++p;
          }
        }
      }
    }
    // all reads of this tile are done before the next iteration overwrites it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if constexpr (SPLIT) {
    const int m = 32 - d;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = (lane >> 4) + 4 * v, j = lane & 15;
      // block A: row i is column i (i < m) or column 16 + i - m against J
      if (i < m) {
        if (i <= j) part[(int64_t)pair_index(i, j, d) * pstride + slot] = acc[0][v];
      } else {
        part[(int64_t)pair_index(j, 16 + i - m, d) * pstride + slot] = acc[0][v];
      }
      // block B: columns m + i and m + j, less the entries block A holds
      const int a = m + i, b = m + j;
      if (i <= j && b < d && (a >= 16 || b < 16))
        part[(int64_t)pair_index(a, b, d) * pstride + slot] = acc[1][v];
    }
    return;
  }
  int p = 0;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int j = i; j < NB; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * i + (lane >> 4) + 4 * v;
        const int b = 16 * j + (lane & 15);
        if (a <= b && b < d) part[(int64_t)pair_index(a, b, d) * pstride + slot] = acc[p][v];
      }
      ++p;
    }
  }
}

template <int NB, bool SPLIT = false>
__global__ __launch_bounds__(GW * SSCG_WAVE) void k_gram(ColPtr cols, int n, int d,
                                                         double* __restrict__ part, int ng,
                                                         Gate gate) {
  if (gate_closed(gate)) return;
  __shared__ double lds[GW * GTR * tile_ld<NB, SPLIT>()];
  const int w = threadIdx.x / SSCG_WAVE;
  const int64_t g = (int64_t)blockIdx.x * GW + w;
  if (g >= ng) return;  // whole wavefronts; no workgroup barrier below
  const int64_t r0 = g * GRAM_GROUP;
  gram_group<NB, ColPtr, SameRow, SPLIT>(cols, d, r0, min((int64_t)n, r0 + GRAM_GROUP), SameRow{},
                                       part, ng, g, lds + w * GTR * tile_ld<NB, SPLIT>());
}

template <int NB, bool SPLIT = false>
__global__ __launch_bounds__(GW * SSCG_WAVE) void k_gram32(Cols32 cols, int n, int d,
                                                           double* __restrict__ part, int ng) {
  __shared__ double lds[GW * GTR * tile_ld<NB, SPLIT>()];
  const int w = threadIdx.x / SSCG_WAVE;
  const int64_t g = (int64_t)blockIdx.x * GW + w;
  if (g >= ng) return;
  const int64_t r0 = g * GRAM_GROUP;
  gram_group<NB, Cols32, SameRow, SPLIT>(cols, d, r0, min((int64_t)n, r0 + GRAM_GROUP), SameRow{},
                                       part, ng, g, lds + w * GTR * tile_ld<NB, SPLIT>());
}

// A batched system's rows may be stored out of order (sorted by length within
// windows of GRAM_GROUP rows, which are also its Gram groups): row r of the
// system is at position inv[row0 + r].  The Gram takes the rows in the
// system's own order, so its bits do not depend on the storage order.
struct BatchRow {
  const int32_t* inv;
  int64_t row0;
  __device__ __forceinline__ int64_t operator()(int64_t r) const { return inv[row0 + r]; }
};

// Batched: over the chunks listed in achk, wavefront w of workgroup b takes
// entries b W + w, then every gridDim.x W-th after it (W wavefronts per
// workgroup: BatchCfg::gw, which changes no bits); a chunk is one group of
// the system that owns its rows (rows of the system past its n read as 0).
// The partials go to the chunk's own slot, whatever its place in the list.
// P32: the launch for the systems in an FP32 block (the others skip them),
// so that neither column type's code shares the other's registers.
template <int NB, int W, bool P32>
__global__ __launch_bounds__(W * SSCG_WAVE) void k_gram_batch(BatchCfg c) {
  constexpr int TLD = 16 * NB + 1;  // holds every blocking's tile
  __shared__ double lds[W * GTR * TLD];
  const int w = threadIdx.x / SSCG_WAVE;
  const int nl = c.active[2];
  for (int li = blockIdx.x * W + w; li < nl; li += gridDim.x * W) {  // whole wavefronts
    const int ci = c.achk[li];
    const BatchChunk ch = c.chunks[ci];
    const int q = c.blk_sys[ch.r0 / BATCH_ROWS];  // the system that owns the chunk's rows now
    if (q < 0 || c.sys[q].done || (c.sys[q].p32 != 0) != P32) continue;
    const sscg_block_params prm = c.prm[q];
    const int d = prm.first ? prm.s + 1 : 2 * prm.s + 1;
    const int64_t row0 = c.sys[q].row0;
    const int64_t rend = min((int64_t)ch.r1 - row0, (int64_t)c.sys[q].n);  // system-local rows
    double* tile = lds + w * GTR * TLD;
    // the blocking of the chunk's own d (d is uniform over the wavefront)
    auto run = [&](const auto& cols) {
      using S = std::remove_cv_t<std::remove_reference_t<decltype(cols)>>;
      const BatchRow map{c.inv, row0};
      if (NB >= 2 && d <= 16)
        gram_group<1, S, BatchRow>(cols, d, ch.r0 - row0, rend, map, c.gpart, c.nchunks, ci,
                                   tile);
      else if (NB >= 2 && d <= 24)
        gram_group<2, S, BatchRow, true>(cols, d, ch.r0 - row0, rend, map, c.gpart, c.nchunks,
                                         ci, tile);
      else if (NB == 3 && d <= 32)
        gram_group<2, S, BatchRow>(cols, d, ch.r0 - row0, rend, map, c.gpart, c.nchunks, ci,
                                   tile);
      else
        gram_group<NB, S, BatchRow>(cols, d, ch.r0 - row0, rend, map, c.gpart, c.nchunks, ci,
                                    tile);
    };
    if constexpr (P32)  // an FP32 block: its columns widened (exact in FP64)
      run(batch_cols32(c, prm.s));
    else
      run(batch_cols(c, prm.s, prm.first));
  }
}

// ---------------------------------------------------------------- pairwise sums
//
// Pairwise sum of v[0..count) zero-padded to P (a power of two >= count),
// by the NT threads of a workgroup: thread t sums the aligned run
// [t L, (t + 1) L) of L = P / T leaves (T = min(P, NT)) with a binary-counter
// stack (the same tree), then the T run sums are added pairwise in LDS.  The
// tree is the complete binary tree over the P leaves for any power of two
// NT.  Returns the sum on every thread.
constexpr int WG = 256;
constexpr int PW_DEPTH = 24;  // stack levels: runs of up to 2^23 leaves per thread

template <int NT = WG>
__device__ double pairwise_sum(const double* __restrict__ v, int64_t count, int64_t P) {
  static_assert((NT & (NT - 1)) == 0, "a power of two");
  constexpr int WG = NT;
  __shared__ double s[WG];
  __shared__ double stk[WG * PW_DEPTH];
  const int t = threadIdx.x;
  const int64_t T = P < WG ? P : WG;
  const int64_t L = P / T;
  double x = 0.0;
  if (t < T) {
    double* st = stk + t * PW_DEPTH;
    for (int64_t k = 0; k < L; ++k) {
      const int64_t i = t * L + k;
      x = i < count ? v[i] : 0.0;
      int b = 0;
      while ((k >> b) & 1) {
        x = st[b] + x;  // left run + right run
        ++b;
      }
      st[b] = x;
    }
  }
  if (t < T) s[t] = x;  // the last value formed is the run's sum
  __syncthreads();
  for (int64_t h = T / 2; h >= 1; h /= 2) {
    double y = 0.0;
    if (t < h) y = s[2 * t] + s[2 * t + 1];
    __syncthreads();
    if (t < h) s[t] = y;
    __syncthreads();
  }
  return s[0];
}

__host__ __device__ inline int64_t pow2_at_least(int64_t m) {
  int64_t p = 1;
  while (p < m) p <<= 1;
  return p;
}

// Entry blockIdx.x of G (upper triangle, row-major) from its ng partials.
__global__ __launch_bounds__(WG) void k_gram_finalize(const double* __restrict__ part, int ng,
                                                      int d, double* __restrict__ G,
                                                      const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int q = blockIdx.x;
  const double g = pairwise_sum(part + (int64_t)q * ng, ng, pow2_at_least(ng));
  if (threadIdx.x == 0) {
    int a = 0, rem = q;
    while (rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    const int b = a + rem;
    G[a * d + b] = g;
    G[b * d + a] = g;
  }
}

// grid (pairs, systems): entry blockIdx.x of system blockIdx.y, by one
// wavefront (most systems have few chunks; a small workgroup with a small
// stack lets many run on a CU).
constexpr int FB_NT = SSCG_WAVE;
__global__ __launch_bounds__(FB_NT) void k_gram_finalize_batch(BatchCfg c) {
  const int q = blockIdx.y, e = blockIdx.x;
  const BatchSys& sy = c.sys[q];
  if (sy.done) return;
  const sscg_block_params prm = c.prm[q];
  const int d = prm.first ? prm.s + 1 : 2 * prm.s + 1;
  if (e >= d * (d + 1) / 2) return;
  const int ngs = sy.ch1 - sy.ch0;
  const double g = pairwise_sum<FB_NT>(c.gpart + (int64_t)e * c.nchunks + sy.ch0, ngs,
                                       pow2_at_least(ngs));
  if (threadIdx.x == 0) {
    int a = 0, rem = e;
    while (rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    const int b = a + rem;
    double* Gq = c.G + (int64_t)q * BATCH_GSZ;
    Gq[a * d + b] = g;
    Gq[b * d + a] = g;
  }
}

int column_blocks(int d) { return (d + 15) / 16; }

}  // namespace

// ---------------------------------------------------------------- launches

hipError_t launch_gram(const ColPtr& cols, int n, int d, double* part, Gate g, hipStream_t st) {
  const int ng = gram_ngroups(n);
  const dim3 grid((ng + GW - 1) / GW), block(GW * SSCG_WAVE);
  switch (column_blocks(d)) {
    case 1: hipLaunchKernelGGL(k_gram<1>, grid, block, 0, st, cols, n, d, part, ng, g); break;
    case 2:
      if (d <= 24)
        hipLaunchKernelGGL((k_gram<2, true>), grid, block, 0, st, cols, n, d, part, ng, g);
      else
        hipLaunchKernelGGL((k_gram<2, false>), grid, block, 0, st, cols, n, d, part, ng, g);
      break;
    default: hipLaunchKernelGGL(k_gram<3>, grid, block, 0, st, cols, n, d, part, ng, g); break;
  }
  return hipGetLastError();
}

hipError_t launch_gram32(const Cols32& cols, int n, int d, double* part, hipStream_t st) {
  const int ng = gram_ngroups(n);
  const dim3 grid((ng + GW - 1) / GW), block(GW * SSCG_WAVE);
  switch (column_blocks(d)) {
    case 1: hipLaunchKernelGGL(k_gram32<1>, grid, block, 0, st, cols, n, d, part, ng); break;
    case 2:
      if (d <= 24)
        hipLaunchKernelGGL((k_gram32<2, true>), grid, block, 0, st, cols, n, d, part, ng);
      else
        hipLaunchKernelGGL((k_gram32<2, false>), grid, block, 0, st, cols, n, d, part, ng);
      break;
    default: hipLaunchKernelGGL(k_gram32<3>, grid, block, 0, st, cols, n, d, part, ng); break;
  }
  return hipGetLastError();
}

hipError_t launch_gram_finalize(const double* part, int ng, int d, double* G, const int* stop,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_gram_finalize, dim3(d * (d + 1) / 2), dim3(WG), 0, st, part, ng, d, G,
                     stop);
  return hipGetLastError();
}

template <int W, bool P32>
void gram_batch_w(const BatchCfg& c, hipStream_t st) {
  const dim3 grid((batch_grid(c.gchk) + W - 1) / W), block(W * SSCG_WAVE);
  switch (column_blocks(2 * c.S + 1)) {
    case 1: hipLaunchKernelGGL((k_gram_batch<1, W, P32>), grid, block, 0, st, c); break;
    case 2: hipLaunchKernelGGL((k_gram_batch<2, W, P32>), grid, block, 0, st, c); break;
    default: hipLaunchKernelGGL((k_gram_batch<3, W, P32>), grid, block, 0, st, c); break;
  }
}

template <bool P32>
void gram_batch_p(const BatchCfg& c, hipStream_t st) {
  switch (c.gw) {
    case 1: gram_batch_w<1, P32>(c, st); break;
    case 2: gram_batch_w<2, P32>(c, st); break;
    default: gram_batch_w<4, P32>(c, st); break;
  }
}

hipError_t launch_gram_batch(const BatchCfg& c, hipStream_t st) {
  gram_batch_p<false>(c, st);
  if (c.vprec) gram_batch_p<true>(c, st);
  return hipGetLastError();
}

hipError_t launch_gram_finalize_batch(const BatchCfg& c, hipStream_t st) {
  const int dm = 2 * c.S + 1;
  hipLaunchKernelGGL(k_gram_finalize_batch, dim3(dm * (dm + 1) / 2, c.nsys), dim3(FB_NT), 0, st,
                     c);
  return hipGetLastError();
}
