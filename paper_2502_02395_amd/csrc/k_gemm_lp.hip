// Batched variable-size GEMM in FP32 on CDNA4 matrix cores for FP64
// operands: read in FP64, rounded to FP32 on their way into LDS, multiplied by
// the FP32 MFMA with FP32 accumulation, written back in FP64.  Same work-list
// format and tile mapping as the FP64 kernel (k_gemm.hip); used for the Schur
// update under every reduced gemm_prec.
#include "h2_internal.hpp"

namespace h2 {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int xcd_remap_lp(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// Accumulator layout of the 16x16 FP32-output MFMAs (measured on gfx950):
// element e of lane l holds row ACC_ROW(e, l), column l % 16.
#define ACC_ROW(e, l) (4 * ((l) >> 4) + (e))

// ---------------------------------------------------------------- FP32 MFMA
template <int TAG, int TA, int TB>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const GemmDesc* __restrict__ descs,
                                                       const int* __restrict__ tmap, int count,
                                                       int tiles) {
  constexpr int TK = 16;
  const int logical = xcd_remap_lp(blockIdx.x, gridDim.x);
  if (logical >= tiles) return;
  const int2 it = reinterpret_cast<const int2*>(tmap)[logical];
  const int item = it.x;
  const GemmDesc d = descs[item];
  const int t = it.y;
  const int tiles_m = (d.M + 63) / 64;
  const int m0 = (t % tiles_m) * 64, n0 = (t / tiles_m) * 64;
  __shared__ float As[TK][65];
  __shared__ float Bs[TK][65];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  float ra[4], rb[4];
  // operand element q of this thread: A(am + ..., ak + ...), B(bk + ..., bn + ...)
  const int am = TA ? (tid >> 4) : (tid & 63), ak = TA ? (tid & 15) : (tid >> 6);
  const int bn = TB ? (tid & 63) : (tid >> 4), bk = TB ? (tid >> 6) : (tid & 15);
  const int M = d.M, N = d.N, K = d.K;
  const int64_t lda = d.lda, ldb = d.ldb;
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gm = m0 + am + (TA ? 16 * q : 0), gk = k0 + ak + (TA ? 0 : 4 * q);
      ra[q] = (gm < M && gk < K) ? (float)(TA ? d.A[gk + gm * lda] : d.A[gm + gk * lda]) : 0.f;
      const int gn = n0 + bn + (TB ? 0 : 16 * q), gk2 = k0 + bk + (TB ? 4 * q : 0);
      rb[q] = (gn < N && gk2 < K) ? (float)(TB ? d.B[gn + gk2 * ldb] : d.B[gk2 + gn * ldb]) : 0.f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[ak + (TA ? 0 : 4 * q)][am + (TA ? 16 * q : 0)] = ra[q];
      Bs[bk + (TB ? 4 * q : 0)][bn + (TB ? 0 : 16 * q)] = rb[q];
    }
  };
  const int nk = (d.K + TK - 1) / TK;
  if (nk > 0) load(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    store();
    __syncthreads();
    if (kt + 1 < nk) load((kt + 1) * TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      const float a0 = As[kr][wm + c], a1 = As[kr][wm + 16 + c];
      const float b0 = Bs[kr][wn + c], b1 = Bs[kr][wn + 16 + c];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  const int col = lane & 15;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wm + 16 * i + ACC_ROW(e, lane);
        const int gn = n0 + wn + 16 * j + col;
        if (gm < d.M && gn < d.N) {
          double v = d.alpha * (double)acc[i][j][e];
          if (d.beta != 0.0) v += d.beta * d.C[gm + (int64_t)gn * d.ldc];
          d.D[gm + (int64_t)gn * d.ldd] = v;
        }
      }
}

template <int TAG, int TA, int TB>
static void launch_lp(const GemmDesc* d, const int* o, int count, int tiles, hipStream_t st) {
  const int grid = (tiles + 7) & ~7;
  hipLaunchKernelGGL((gemm_f32_kernel<TAG, TA, TB>), dim3(grid), dim3(256), 0, st, d, o, count, tiles);
}

template <int TAG>
static void launch_lp_t(const GemmDesc* d, const int* o, int count, int tiles, hipStream_t st,
                        int tA, int tB) {
  if (!tA && !tB) launch_lp<TAG, 0, 0>(d, o, count, tiles, st);
  else if (!tA && tB) launch_lp<TAG, 0, 1>(d, o, count, tiles, st);
  else if (tA && !tB) launch_lp<TAG, 1, 0>(d, o, count, tiles, st);
  else launch_lp<TAG, 1, 1>(d, o, count, tiles, st);
}

hipError_t launch_gemm_lp(const GemmDesc* d_desc, const int* d_tile_map, int count, int tiles,
                          int prec, hipStream_t st, int tag, int tA, int tB) {
  if (count <= 0 || tiles <= 0) return hipSuccess;
  if (prec != H2_PREC_FP32) return launch_gemm(d_desc, d_tile_map, count, tiles, st, tag, 0, tA, tB);
  if (tag == 1) launch_lp_t<1>(d_desc, d_tile_map, count, tiles, st, tA, tB);
  else launch_lp_t<0>(d_desc, d_tile_map, count, tiles, st, tA, tB);
  return hipGetLastError();
}

}  // namespace h2
