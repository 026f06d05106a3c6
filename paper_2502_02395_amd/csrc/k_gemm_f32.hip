// Batched variable-size GEMM with FP32 operands, FP32 MFMA (16x16x4, FP32
// accumulation) and FP32 results: the near-pair basis transforms of the
// precision split (Algorithm 4's U_i^T A_ij V_j, here P_i^T (A_ij P_j)) when
// the handle's gemm_prec is FP32.  The operands live in HBM as FP32 copies, so
// the products move half the bytes of the FP64 path and run on the FP32 matrix
// rate.  Work lists, tile maps and tile shapes are those of the FP64 kernel
// (k_gemm.hip); every K tile is 32 deep.
#include "h2_internal.hpp"

namespace h2 {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int xcd_remap_f32(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// Accumulator layout of the 16x16 FP32-output MFMAs (measured on gfx950):
// element e of lane l holds row 4 * (l / 16) + e, column l % 16.
template <int BM, int BN, int TA, int TB, typename TO>
__device__ __forceinline__ void gemm_f32io_body(const GemmDesc* __restrict__ descs,
                                                const int* __restrict__ tmap, int tiles) {
  constexpr int TK = 32;
  constexpr int MI = BM / 32, NJ = BN / 32;
  constexpr int QA = BM * TK / 256, QB = BN * TK / 256;
  const int logical = xcd_remap_f32(blockIdx.x, gridDim.x);
  if (logical >= tiles) return;
  const int2 it = reinterpret_cast<const int2*>(tmap)[logical];
  const GemmDesc d = descs[it.x];
  const int t = it.y;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int m0 = (t % tiles_m) * BM;
  const int n0 = (t / tiles_m) * BN;

  __shared__ float As[TK][BM + 1];
  __shared__ float Bs[TK][BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
  const int am = TA ? (tid / TK) : (tid % BM);
  const int ak = TA ? (tid % TK) : (tid / BM);
  const int bn = TB ? (tid % BN) : (tid / TK);
  const int bk = TB ? (tid / BN) : (tid % TK);
  constexpr int ASTEP = TA ? 256 / TK : 256 / BM;
  constexpr int BSTEP = TB ? 256 / BN : 256 / TK;

  f4v acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = (f4v){0.f, 0.f, 0.f, 0.f};

  float ra[QA], rb[QB];
  const int M = d.M, N = d.N, K = d.K;
  const float* __restrict__ Ap = reinterpret_cast<const float*>(d.A);
  const float* __restrict__ Bp = reinterpret_cast<const float*>(d.B);
  const int64_t lda = d.lda, ldb = d.ldb;
  const bool inside = (m0 + BM <= M) && (n0 + BN <= N);

#define H2F_LOAD(k0, GUARD)                                                      \
  {                                                                              \
    _Pragma("unroll") for (int q = 0; q < QA; ++q) {                             \
      const int gm = m0 + am + (TA ? ASTEP * q : 0);                             \
      const int gk = (k0) + ak + (TA ? 0 : ASTEP * q);                           \
      ra[q] = (!(GUARD) || (gm < M && gk < K))                                   \
                  ? (TA ? Ap[gk + gm * lda] : Ap[gm + gk * lda]) : 0.f;          \
    }                                                                            \
    _Pragma("unroll") for (int q = 0; q < QB; ++q) {                             \
      const int gn = n0 + bn + (TB ? 0 : BSTEP * q);                             \
      const int gk = (k0) + bk + (TB ? BSTEP * q : 0);                           \
      rb[q] = (!(GUARD) || (gn < N && gk < K))                                   \
                  ? (TB ? Bp[gn + gk * ldb] : Bp[gk + gn * ldb]) : 0.f;          \
    }                                                                            \
  }
#define H2F_LOAD_TILE(k0)                                                        \
  {                                                                              \
    if (inside && (k0) + TK <= K) H2F_LOAD(k0, false) else H2F_LOAD(k0, true)    \
  }

  const int nk = (K + TK - 1) / TK;
  if (nk > 0) H2F_LOAD_TILE(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QA; ++q) As[ak + (TA ? 0 : ASTEP * q)][am + (TA ? ASTEP * q : 0)] = ra[q];
#pragma unroll
    for (int q = 0; q < QB; ++q) Bs[bk + (TB ? BSTEP * q : 0)][bn + (TB ? 0 : BSTEP * q)] = rb[q];
    __syncthreads();
    if (kt + 1 < nk) H2F_LOAD_TILE((kt + 1) * TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const int c = lane & 15;
      float a[MI], b[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = As[kr][wm + 16 * i + c];
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = Bs[kr][wn + 16 * j + c];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#undef H2F_LOAD_TILE
#undef H2F_LOAD

  TO* __restrict__ Dp = reinterpret_cast<TO*>(d.D);
  const float alpha = (float)d.alpha;
  const int col = lane & 15;
  const int rg = 4 * (lane >> 4);
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wm + 16 * i + rg + e;
        const int gn = n0 + wn + 16 * j + col;
        if (gm < M && gn < N) Dp[gm + (int64_t)gn * d.ldd] = (TO)(alpha * acc[i][j][e]);
      }
}

template <int BM, int BN, int TA, int TB>
__global__ __launch_bounds__(256) void gemm_f32io_pair_kernel(const GemmDesc* __restrict__ descs,
                                                              const int* __restrict__ tmap,
                                                              int tiles) {
  gemm_f32io_body<BM, BN, TA, TB, float>(descs, tmap, tiles);
}
template <int BM, int BN, int TA, int TB>
__global__ __launch_bounds__(256) void gemm_f32i64o_kernel(const GemmDesc* __restrict__ descs,
                                                           const int* __restrict__ tmap,
                                                           int tiles) {
  gemm_f32io_body<BM, BN, TA, TB, double>(descs, tmap, tiles);
}

template <int BM, int BN, int TA, int TB>
static void launch_f32io_cfg(const GemmDesc* d, const int* tmap, int tiles, hipStream_t st,
                             bool out64) {
  const int grid = (tiles + 7) & ~7;
  if (out64)
    hipLaunchKernelGGL((gemm_f32i64o_kernel<BM, BN, TA, TB>), dim3(grid), dim3(256), 0, st, d,
                       tmap, tiles);
  else
    hipLaunchKernelGGL((gemm_f32io_pair_kernel<BM, BN, TA, TB>), dim3(grid), dim3(256), 0, st, d,
                       tmap, tiles);
}

template <int BM, int BN>
static void launch_f32io_t(const GemmDesc* d, const int* tmap, int tiles, hipStream_t st, int tA,
                           int tB, bool out64) {
  if (!tA && !tB) launch_f32io_cfg<BM, BN, 0, 0>(d, tmap, tiles, st, out64);
  else if (!tA && tB) launch_f32io_cfg<BM, BN, 0, 1>(d, tmap, tiles, st, out64);
  else if (tA && !tB) launch_f32io_cfg<BM, BN, 1, 0>(d, tmap, tiles, st, out64);
  else launch_f32io_cfg<BM, BN, 1, 1>(d, tmap, tiles, st, out64);
}

hipError_t launch_gemm_f32io(const GemmDesc* d_desc, const int* d_tile_map, int count, int tiles,
                             hipStream_t st, int cfg, int tA, int tB, bool out64) {
  if (count <= 0 || tiles <= 0) return hipSuccess;
  switch (cfg) {
    case 1: launch_f32io_t<128, 64>(d_desc, d_tile_map, tiles, st, tA, tB, out64); break;
    case 2: launch_f32io_t<128, 128>(d_desc, d_tile_map, tiles, st, tA, tB, out64); break;
    default: launch_f32io_t<64, 64>(d_desc, d_tile_map, tiles, st, tA, tB, out64); break;
  }
  return hipGetLastError();
}

// Conversions between the FP64 factors and their FP32 copies, over lists of
// contiguous ranges (blockIdx.x = range, CVT_WG workgroups per range, four
// independent elements per thread and pass).
constexpr int CVT_WG = 8;
template <typename TS, typename TD>
__device__ __forceinline__ void cvt_range(const TS* __restrict__ s, TD* __restrict__ t, int64_t n) {
  for (int64_t i0 = (int64_t)blockIdx.y * 1024 + threadIdx.x; i0 < n; i0 += CVT_WG * 1024) {
    TS v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = i0 + 256 * u < n ? s[i0 + 256 * u] : TS(0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 256 * u < n) t[i0 + 256 * u] = (TD)v[u];
  }
}
__global__ __launch_bounds__(256) void cvt_list_kernel(const ConvDesc* __restrict__ descs) {
  const ConvDesc c = descs[blockIdx.x];
  if (c.to32)
    cvt_range(static_cast<const double*>(c.src), static_cast<float*>(c.dst), c.n);
  else
    cvt_range(static_cast<const float*>(c.src), static_cast<double*>(c.dst), c.n);
}

hipError_t launch_cvt_list(const ConvDesc* d, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(cvt_list_kernel, dim3(count, CVT_WG), dim3(256), 0, st, d);
  return hipGetLastError();
}

// Block copies from an FP32 source (the merge of the FP32 transformed blocks'
// SS parts into the parent's near blocks): FP64 destinations (diagonal parent
// blocks, the root) or FP32 ones (off-diagonal parent blocks, read only by the
// FP32 pair transforms).  The CopyDesc pointers hold float arrays where FP32.
template <typename TD>
__global__ __launch_bounds__(256) void copy_f32_kernel(const CopyDesc* __restrict__ descs) {
  const CopyDesc c = descs[blockIdx.x];
  const float* src = reinterpret_cast<const float*>(c.src);
  TD* dst = reinterpret_cast<TD*>(c.dst);
  for (int q = blockIdx.y; q < c.cols; q += gridDim.y)
    for (int r = threadIdx.x; r < c.rows; r += 256) {
      const float v = c.trans ? src[q + (int64_t)r * c.lds] : src[r + (int64_t)q * c.lds];
      dst[r + (int64_t)q * c.ldd] = (TD)v;
    }
}

hipError_t launch_copy_f32(const CopyDesc* d_desc, int count, hipStream_t st, bool dst32) {
  if (count <= 0) return hipSuccess;
  if (dst32)
    hipLaunchKernelGGL(copy_f32_kernel<float>, dim3(count, 8), dim3(256), 0, st, d_desc);
  else
    hipLaunchKernelGGL(copy_f32_kernel<double>, dim3(count, 8), dim3(256), 0, st, d_desc);
  return hipGetLastError();
}

}  // namespace h2
