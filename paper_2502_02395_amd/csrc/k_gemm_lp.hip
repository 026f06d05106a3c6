// Batched variable-size GEMM in reduced precision on CDNA4 matrix cores:
// operands are read in FP64, rounded to FP32 or BF16 on their way into LDS,
// multiplied by the FP32 or BF16 MFMA with FP32 accumulation, and written back
// in FP64.  Same work-list format and tile mapping as the FP64 kernel
// (k_gemm.hip); used for the basis transforms and the Schur update when the
// handle's gemm_prec asks for it.  Rounding to BF16 is round-to-nearest-even.
#include "h2_internal.hpp"

namespace h2 {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int find_item_lp(const int* off, int count, int t) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int xcd_remap_lp(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ unsigned short to_bf16(double x) {
  const float f = (float)x;
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Accumulator layout of the 16x16 FP32-output MFMAs (measured on gfx950):
// element e of lane l holds row ACC_ROW(e, l), column l % 16.
#define ACC_ROW(e, l) (4 * ((l) >> 4) + (e))

// ---------------------------------------------------------------- FP32 MFMA
template <int TAG>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const GemmDesc* __restrict__ descs,
                                                       const int* __restrict__ toff, int count,
                                                       int tiles) {
  constexpr int TK = 16;
  const int logical = xcd_remap_lp(blockIdx.x, gridDim.x);
  if (logical >= tiles) return;
  const int item = find_item_lp(toff, count, logical);
  const GemmDesc d = descs[item];
  const int t = logical - toff[item];
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
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int m, k;
      if (!d.tA) { m = tid & 63; k = (tid >> 6) + 4 * q; } else { k = tid & 15; m = (tid >> 4) + 16 * q; }
      const int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < d.M && gk < d.K) v = d.tA ? d.A[gk + (int64_t)gm * d.lda] : d.A[gm + (int64_t)gk * d.lda];
      ra[q] = (float)v;
      int n, k2;
      if (!d.tB) { k2 = tid & 15; n = (tid >> 4) + 16 * q; } else { n = tid & 63; k2 = (tid >> 6) + 4 * q; }
      const int gn = n0 + n, gk2 = k0 + k2;
      double w = 0.0;
      if (gn < d.N && gk2 < d.K) w = d.tB ? d.B[gn + (int64_t)gk2 * d.ldb] : d.B[gk2 + (int64_t)gn * d.ldb];
      rb[q] = (float)w;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int m, k;
      if (!d.tA) { m = tid & 63; k = (tid >> 6) + 4 * q; } else { k = tid & 15; m = (tid >> 4) + 16 * q; }
      As[k][m] = ra[q];
      int n, k2;
      if (!d.tB) { k2 = tid & 15; n = (tid >> 4) + 16 * q; } else { n = tid & 63; k2 = (tid >> 6) + 4 * q; }
      Bs[k2][n] = rb[q];
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

// ---------------------------------------------------------------- BF16 MFMA
// Tiles are stored row-major in LDS (k contiguous) so that each lane fetches
// its four consecutive k values of one row with a single 8-byte read.
template <int TAG>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const GemmDesc* __restrict__ descs,
                                                        const int* __restrict__ toff, int count,
                                                        int tiles) {
  constexpr int TK = 32, KP = TK + 4;
  const int logical = xcd_remap_lp(blockIdx.x, gridDim.x);
  if (logical >= tiles) return;
  const int item = find_item_lp(toff, count, logical);
  const GemmDesc d = descs[item];
  const int t = logical - toff[item];
  const int tiles_m = (d.M + 63) / 64;
  const int m0 = (t % tiles_m) * 64, n0 = (t / tiles_m) * 64;
  __shared__ __attribute__((aligned(16))) unsigned short As[64][KP];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[64][KP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  unsigned short ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int m, k;
      if (!d.tA) { m = tid & 63; k = (tid >> 6) + 4 * q; } else { k = tid & 31; m = (tid >> 5) + 8 * q; }
      const int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < d.M && gk < d.K) v = d.tA ? d.A[gk + (int64_t)gm * d.lda] : d.A[gm + (int64_t)gk * d.lda];
      ra[q] = to_bf16(v);
      int n, k2;
      if (!d.tB) { k2 = tid & 31; n = (tid >> 5) + 8 * q; } else { n = tid & 63; k2 = (tid >> 6) + 4 * q; }
      const int gn = n0 + n, gk2 = k0 + k2;
      double w = 0.0;
      if (gn < d.N && gk2 < d.K) w = d.tB ? d.B[gn + (int64_t)gk2 * d.ldb] : d.B[gk2 + (int64_t)gn * d.ldb];
      rb[q] = to_bf16(w);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int m, k;
      if (!d.tA) { m = tid & 63; k = (tid >> 6) + 4 * q; } else { k = tid & 31; m = (tid >> 5) + 8 * q; }
      As[m][k] = ra[q];
      int n, k2;
      if (!d.tB) { k2 = tid & 31; n = (tid >> 5) + 8 * q; } else { n = tid & 63; k2 = (tid >> 6) + 4 * q; }
      Bs[n][k2] = rb[q];
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
    for (int kk = 0; kk < TK; kk += 16) {
      const int c = lane & 15, g = (lane >> 4) * 4;
      const s4 a0 = *reinterpret_cast<const s4*>(&As[wm + c][kk + g]);
      const s4 a1 = *reinterpret_cast<const s4*>(&As[wm + 16 + c][kk + g]);
      const s4 b0 = *reinterpret_cast<const s4*>(&Bs[wn + c][kk + g]);
      const s4 b1 = *reinterpret_cast<const s4*>(&Bs[wn + 16 + c][kk + g]);
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc[1][1], 0, 0, 0);
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

hipError_t launch_gemm_lp(const GemmDesc* d_desc, const int* d_tile_off, int count, int tiles,
                          int prec, hipStream_t st, int tag) {
  if (count <= 0 || tiles <= 0) return hipSuccess;
  const int grid = (tiles + 7) & ~7;
  if (prec == H2_PREC_FP32) {
    if (tag == 1)
      hipLaunchKernelGGL(gemm_f32_kernel<1>, dim3(grid), dim3(256), 0, st, d_desc, d_tile_off, count, tiles);
    else
      hipLaunchKernelGGL(gemm_f32_kernel<0>, dim3(grid), dim3(256), 0, st, d_desc, d_tile_off, count, tiles);
  } else if (prec == H2_PREC_BF16) {
    if (tag == 1)
      hipLaunchKernelGGL(gemm_bf16_kernel<1>, dim3(grid), dim3(256), 0, st, d_desc, d_tile_off, count, tiles);
    else
      hipLaunchKernelGGL(gemm_bf16_kernel<0>, dim3(grid), dim3(256), 0, st, d_desc, d_tile_off, count, tiles);
  } else {
    return launch_gemm(d_desc, d_tile_off, count, tiles, st, tag);
  }
  return hipGetLastError();
}

}  // namespace h2
