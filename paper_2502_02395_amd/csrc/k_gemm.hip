// Batched variable-size FP64 GEMM on CDNA4 matrix cores and batched block
// copies.
//
// The basis transforms of the ULV sweep (Algorithm 4: U_i^T A_ij V_j, the
// diagonal transform and the Schur update of Eq. 21) are many independent
// small dense products of uneven shape.  Instead of padding them to a common
// size (the paper's choice for its vendor batched calls, Section 4.1), every
// launch takes a work list of items of their own M, N, K, strides and
// transposes; each workgroup computes one tile (64 x 64, 128 x 64 or
// 128 x 128, chosen per list by the autotuner) of one item, found by a binary
// search over the per-item tile prefix.
#include "h2_internal.hpp"

namespace h2 {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int LPAD = 1;

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that
// consecutive logical tiles (the tiles of one item, which share operands) run
// on the same XCD and hit the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// One BM x BN output tile per 256-thread workgroup; the four waves form a 2x2
// grid, each wave accumulating (BM/32) x (BN/32) 16x16 MFMA tiles.  Operand
// tiles of TK (16 or 32) are staged through LDS; the next one is prefetched
// into registers while the current one is multiplied (TK = 32 gives the
// loads the time of twice as many MFMAs, at one wave per SIMD less).  Tiles inside M x N and full K tiles load
// without bounds tests.  TA / TB (transposed operands) are compile-time so
// that every index is plain arithmetic.
template <int BM, int BN, int TK, int TA, int TB>
__device__ __forceinline__ void gemm_f64_body(const GemmDesc* __restrict__ descs,
                                              const int* __restrict__ tmap, int tiles) {
  constexpr int MI = BM / 32, NJ = BN / 32;
  constexpr int QA = BM * TK / 256, QB = BN * TK / 256;  // elements per thread per K tile
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  if (logical >= tiles) return;
  const int2 it = reinterpret_cast<const int2*>(tmap)[logical];
  const GemmDesc d = descs[it.x];
  const int t = it.y;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int m0 = (t % tiles_m) * BM;
  const int n0 = (t / tiles_m) * BN;

  __shared__ double As[TK][BM + LPAD];
  __shared__ double Bs[TK][BN + LPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);

  // this thread's operand elements: A(m, k) and B(k, n) of the tile, the
  // contiguous index fastest
  const int am = TA ? (tid / TK) : (tid % BM);
  const int ak = TA ? (tid % TK) : (tid / BM);
  const int bn = TB ? (tid % BN) : (tid / TK);
  const int bk = TB ? (tid / BN) : (tid % TK);
  constexpr int ASTEP = TA ? 256 / TK : 256 / BM;   // along m (TA) or k (!TA)
  constexpr int BSTEP = TB ? 256 / BN : 256 / TK;   // along k (TB) or n (!TB)

  d4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  double ra[QA], rb[QB];
  const int M = d.M, N = d.N, K = d.K;
  const double* __restrict__ Ap = d.A;
  const double* __restrict__ Bp = d.B;
  const int64_t lda = d.lda, ldb = d.ldb;
  const bool inside = (m0 + BM <= M) && (n0 + BN <= N);

#define H2_LOAD(k0, GUARD)                                                       \
  {                                                                              \
    _Pragma("unroll") for (int q = 0; q < QA; ++q) {                             \
      const int gm = m0 + am + (TA ? ASTEP * q : 0);                             \
      const int gk = (k0) + ak + (TA ? 0 : ASTEP * q);                           \
      ra[q] = (!(GUARD) || (gm < M && gk < K))                                   \
                  ? (TA ? Ap[gk + gm * lda] : Ap[gm + gk * lda]) : 0.0;          \
    }                                                                            \
    _Pragma("unroll") for (int q = 0; q < QB; ++q) {                             \
      const int gn = n0 + bn + (TB ? 0 : BSTEP * q);                             \
      const int gk = (k0) + bk + (TB ? BSTEP * q : 0);                           \
      rb[q] = (!(GUARD) || (gn < N && gk < K))                                   \
                  ? (TB ? Bp[gn + gk * ldb] : Bp[gk + gn * ldb]) : 0.0;          \
    }                                                                            \
  }
#define H2_LOAD_TILE(k0)                                                         \
  {                                                                              \
    if (inside && (k0) + TK <= K) H2_LOAD(k0, false) else H2_LOAD(k0, true)      \
  }

  const int nk = (K + TK - 1) / TK;
  if (nk > 0) H2_LOAD_TILE(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QA; ++q) As[ak + (TA ? 0 : ASTEP * q)][am + (TA ? ASTEP * q : 0)] = ra[q];
#pragma unroll
    for (int q = 0; q < QB; ++q) Bs[bk + (TB ? BSTEP * q : 0)][bn + (TB ? 0 : BSTEP * q)] = rb[q];
    __syncthreads();
    if (kt + 1 < nk) H2_LOAD_TILE((kt + 1) * TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const int c = lane & 15;
      double a[MI], b[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = As[kr][wm + 16 * i + c];
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = Bs[kr][wn + 16 * j + c];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#undef H2_LOAD_TILE
#undef H2_LOAD

  // Accumulator layout of the 16x16x4 f64 MFMA (measured on gfx950): element e
  // of lane l holds row 4*e + l/16, column l%16.
  const int col = lane & 15;
  const int rg = lane >> 4;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wm + 16 * i + 4 * e + rg;
        const int gn = n0 + wn + 16 * j + col;
        if (gm < M && gn < N) {
          double v = d.alpha * acc[i][j][e];
          if (d.beta != 0.0) v += d.beta * d.C[gm + (int64_t)gn * d.ldc];
          d.D[gm + (int64_t)gn * d.ldd] = v;
        }
      }
}

// Two symbols per instantiation with the same body so that profiles separate
// the near-pair basis transforms (the dominant cost) from every other product.
template <int BM, int BN, int TK, int TA, int TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmDesc* __restrict__ descs,
                                                       const int* __restrict__ tmap, int tiles) {
  gemm_f64_body<BM, BN, TK, TA, TB>(descs, tmap, tiles);
}
template <int BM, int BN, int TK, int TA, int TB>
__global__ __launch_bounds__(256) void gemm_f64_pair_kernel(const GemmDesc* __restrict__ descs,
                                                            const int* __restrict__ tmap,
                                                            int tiles) {
  gemm_f64_body<BM, BN, TK, TA, TB>(descs, tmap, tiles);
}

template <int BM, int BN, int TK, int TA, int TB>
static void launch_cfg(const GemmDesc* d_desc, const int* d_tile_map, int tiles, hipStream_t st,
                       int tag) {
  const int grid = (tiles + 7) & ~7;
  if (tag == 1)
    hipLaunchKernelGGL((gemm_f64_pair_kernel<BM, BN, TK, TA, TB>), dim3(grid), dim3(256), 0, st,
                       d_desc, d_tile_map, tiles);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, TK, TA, TB>), dim3(grid), dim3(256), 0, st,
                       d_desc, d_tile_map, tiles);
}

template <int BM, int BN, int TK>
static void launch_t(const GemmDesc* d_desc, const int* d_tile_map, int tiles, hipStream_t st,
                     int tag, int tA, int tB) {
  if (!tA && !tB) launch_cfg<BM, BN, TK, 0, 0>(d_desc, d_tile_map, tiles, st, tag);
  else if (!tA && tB) launch_cfg<BM, BN, TK, 0, 1>(d_desc, d_tile_map, tiles, st, tag);
  else if (tA && !tB) launch_cfg<BM, BN, TK, 1, 0>(d_desc, d_tile_map, tiles, st, tag);
  else launch_cfg<BM, BN, TK, 1, 1>(d_desc, d_tile_map, tiles, st, tag);
}

hipError_t launch_gemm(const GemmDesc* d_desc, const int* d_tile_map, int count,
                       int tiles, hipStream_t st, int tag, int cfg, int tA, int tB) {
  if (count <= 0 || tiles <= 0) return hipSuccess;
  switch (cfg) {
    case 1: launch_t<128, 64, 16>(d_desc, d_tile_map, tiles, st, tag, tA, tB); break;
    case 2: launch_t<128, 128, 16>(d_desc, d_tile_map, tiles, st, tag, tA, tB); break;
    case 3: launch_t<64, 64, 32>(d_desc, d_tile_map, tiles, st, tag, tA, tB); break;
    default: launch_t<64, 64, 16>(d_desc, d_tile_map, tiles, st, tag, tA, tB); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Columns spread over the blockIdx.y workgroups of a descriptor, rows over
// the threads.
__global__ __launch_bounds__(256) void copy_kernel(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.x];
  for (int c = blockIdx.y; c < d.cols; c += gridDim.y)
    for (int r = threadIdx.x; r < d.rows; r += 256) {
      const double v = d.trans ? d.src[c + (int64_t)r * d.lds] : d.src[r + (int64_t)c * d.lds];
      d.dst[r + (int64_t)c * d.ldd] = v;
    }
}

hipError_t launch_copy(const CopyDesc* d_desc, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(count, 8), dim3(256), 0, st, d_desc);
  return hipGetLastError();
}

}  // namespace h2
