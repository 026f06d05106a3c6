// Batched variable-size GEMM on the gfx950 BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation) over the same FP32 operands,
// work lists and tile maps as the FP32 kernel (k_gemm_f32.hip): the near-pair,
// diagonal and far-coupling transforms of the precision split when the
// handle's gemm_prec is BF16 or BF16X3.
//
// Each FP32 operand element x is split on its way into LDS into
// h = bf16(x) and l = bf16(x - h) (round to nearest even both times).
//   TERMS = 1 (BF16):   A B ~ Ah Bh                   (operands to 8 bits)
//   TERMS = 3 (BF16X3): A B ~ Ah Bh + Ah Bl + Al Bh   (the dropped Al Bl and the
//                       rounding of l are each below 2^-18 of |a b|, so every
//                       product keeps about 17 bits; the sums are FP32)
// BF16X3 does three MFMAs per product, at a third of the 2.5 PFLOP/s BF16
// rate: still five times the FP32 matrix rate, with an operand precision
// between BF16 and FP32.
#include "h2_internal.hpp"

namespace h2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Global-address-space views (the pointers arrive through descriptors, which
// would otherwise give flat loads and stores).
typedef const float __attribute__((address_space(1)))* gcf_t;

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// RNE splits of N (4 or 8) values, two per conversion instruction:
// h = bf16(x), and for TERMS = 3 also l = bf16(x - h)
template <int TERMS, int N, typename BV>
__device__ __forceinline__ void split_bf16(const float* x, BV& h, BV& l) {
#pragma unroll
  for (int e = 0; e < N; e += 2) {
    const f2v v = {x[e], x[e + 1]};
    const bf16x2 hv = __builtin_convertvector(v, bf16x2);
    h[e] = hv[0];
    h[e + 1] = hv[1];
    if constexpr (TERMS == 3) {
      const bf16x2 lv = __builtin_convertvector(v - __builtin_convertvector(hv, f2v), bf16x2);
      l[e] = lv[0];
      l[e + 1] = lv[1];
    }
  }
}

__device__ __forceinline__ int xcd_remap_bf(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

constexpr int BF_TK = 32;  // K of one MFMA and of one LDS stage
constexpr int BF_LS = 40;  // LDS row stride in bf16: 80 bytes, 16-byte aligned;
                           // 16 consecutive rows start on 16 distinct 4-bank groups

// Four consecutive floats at a 4-byte-aligned address (the blocks start at
// arbitrary offsets): one 16-byte global access.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// One operand tile of R rows (m of A, n of B) x BF_TK: element (r, k) is
// P[r + k ld] (row-contiguous, RC) or P[k + r ld] (k-contiguous).  Thread
// tid stages NV = BF_TK R / 1024 four-float vectors, each one 16-byte load:
//   RC:  a block of 4 rows x KPT = R / 32 consecutive k (vector e = rows
//        r..r+3 of column k + e), transposed when written to LDS so that
//        each row's KPT k values go together; k groups vary fastest over
//        the lanes;
//   !RC: vector q = four consecutive k from 4 (tid % 8) of row tid / 8 + 32 q.
// The staged vectors keep the load layout (no register shuffles between the
// loads and their use, so the loads stay in flight through the MFMAs).  Edge
// tiles take guarded scalar loads.
template <int R, bool RC>
struct OpTile {
  static constexpr int NV = BF_TK * R / 1024;
  static constexpr int KPT = R / 32;          // RC: k per thread
  static constexpr int NKG = BF_TK / KPT;     // RC: k groups
  __device__ static void load(f4u (&v)[NV], gcf_t P, int64_t ld, int r0, int k0, int rows,
                              int K, bool guard, int tid) {
    typedef const f4u __attribute__((address_space(1)))* gp4;
    if constexpr (RC) {
      const int r = r0 + 4 * (tid / NKG), kb = k0 + KPT * (tid % NKG);
      if (!guard) {
#pragma unroll
        for (int e = 0; e < KPT; ++e) v[e] = *(gp4)(P + r + (int64_t)(kb + e) * ld);
      } else {
#pragma unroll
        for (int e = 0; e < KPT; ++e)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            v[e][c] = (r + c < rows && kb + e < K) ? P[r + c + (int64_t)(kb + e) * ld] : 0.f;
      }
    } else {
      const int kb = k0 + 4 * (tid % 8);
      if (!guard) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = *(gp4)(P + kb + (int64_t)(r0 + tid / 8 + 32 * q) * ld);
      } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const int r = r0 + tid / 8 + 32 * q;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            v[q][e] = (r < rows && kb + e < K) ? P[kb + e + (int64_t)r * ld] : 0.f;
        }
      }
    }
  }
  // split into the high (and low) BF16 planes of the LDS tile [R][BF_LS]
  template <int TERMS>
  __device__ static void store(const f4u (&v)[NV], __bf16* __restrict__ H,
                               __bf16* __restrict__ L, int tid) {
    if constexpr (RC) {
      const int r = 4 * (tid / NKG), kb = KPT * (tid % NKG);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        typedef __bf16 bfk __attribute__((ext_vector_type(KPT)));
        float x[KPT];
#pragma unroll
        for (int e = 0; e < KPT; ++e) x[e] = v[e][c];
        bfk h, l;
        split_bf16<TERMS, KPT>(x, h, l);
        *reinterpret_cast<bfk*>(H + (r + c) * BF_LS + kb) = h;
        if constexpr (TERMS == 3) *reinterpret_cast<bfk*>(L + (r + c) * BF_LS + kb) = l;
      }
    } else {
      const int kb = 4 * (tid % 8);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int r = tid / 8 + 32 * q;
        const float x[4] = {v[q][0], v[q][1], v[q][2], v[q][3]};
        bf16x4 h, l;
        split_bf16<TERMS, 4>(x, h, l);
        *reinterpret_cast<bf16x4*>(H + r * BF_LS + kb) = h;
        if constexpr (TERMS == 3) *reinterpret_cast<bf16x4*>(L + r * BF_LS + kb) = l;
      }
    }
  }
};

// One BM x BN output tile per 256-thread workgroup; the four waves form a 2x2
// grid, each accumulating (BM/32) x (BN/32) 16x16 tiles.  The next K stage is
// loaded into registers while the current one is multiplied.
// MFMA operand layout (16x16x32 BF16): lane l holds row (A) or column (B)
// l % 16 and the eight consecutive k from 8 (l / 16); accumulator element e of
// lane l is row 4 (l / 16) + e, column l % 16.
template <int BM, int BN, int TA, int TB, typename TO, int TERMS>
__device__ __forceinline__ void gemm_bf16s_body(const GemmDesc* __restrict__ descs,
                                                const int* __restrict__ tmap, int tiles) {
  constexpr int MI = BM / 32, NJ = BN / 32;
  using TileA = OpTile<BM, TA == 0>;
  using TileB = OpTile<BN, TB == 1>;
  const int logical = xcd_remap_bf(blockIdx.x, gridDim.x);
  if (logical >= tiles) return;
  const int2 it = reinterpret_cast<const int2*>(tmap)[logical];
  const GemmDesc d = descs[it.x];
  const int t = it.y;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int m0 = (t % tiles_m) * BM;
  const int n0 = (t / tiles_m) * BN;

  __shared__ __attribute__((aligned(16))) __bf16 Ah[BM * BF_LS], Bh[BN * BF_LS];
  __shared__ __attribute__((aligned(16))) __bf16 Al[TERMS == 3 ? BM * BF_LS : 8],
      Bl[TERMS == 3 ? BN * BF_LS : 8];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);

  f4v acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = (f4v){0.f, 0.f, 0.f, 0.f};

  const int M = d.M, N = d.N, K = d.K;
  const gcf_t Ap = (gcf_t) reinterpret_cast<const float*>(d.A);
  const gcf_t Bp = (gcf_t) reinterpret_cast<const float*>(d.B);
  const int64_t lda = d.lda, ldb = d.ldb;
  const bool inside = (m0 + BM <= M) && (n0 + BN <= N);
  f4u ra[TileA::NV], rb[TileB::NV];
  auto load = [&](int k0) {
    const bool g = !(inside && k0 + BF_TK <= K);
    TileA::load(ra, Ap, lda, m0, k0, M, K, g, tid);
    TileB::load(rb, Bp, ldb, n0, k0, N, K, g, tid);
  };

  const int r16 = lane & 15, kb = (lane >> 4) * 8;
  const int nk = (K + BF_TK - 1) / BF_TK;
  if (nk > 0) load(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    TileA::template store<TERMS>(ra, Ah, Al, tid);
    TileB::template store<TERMS>(rb, Bh, Bl, tid);
    __syncthreads();
    if (kt + 1 < nk) load((kt + 1) * BF_TK);
    bf16x8 ah[MI], bh[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
      ah[i] = *reinterpret_cast<const bf16x8*>(Ah + (wm + 16 * i + r16) * BF_LS + kb);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      bh[j] = *reinterpret_cast<const bf16x8*>(Bh + (wn + 16 * j + r16) * BF_LS + kb);
    if constexpr (TERMS == 3) {
      bf16x8 al[MI], bl[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        al[i] = *reinterpret_cast<const bf16x8*>(Al + (wm + 16 * i + r16) * BF_LS + kb);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        bl[j] = *reinterpret_cast<const bf16x8*>(Bl + (wn + 16 * j + r16) * BF_LS + kb);
      // the two small terms first; independent accumulators back to back
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
  }

  TO __attribute__((address_space(1)))* Dp =
      (TO __attribute__((address_space(1)))*)reinterpret_cast<TO*>(d.D);
  const float alpha = (float)d.alpha;
  const int rg = 4 * (lane >> 4);
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int gm = m0 + wm + 16 * i + rg;  // rows gm .. gm + 3 of column gn
      const int gn = n0 + wn + 16 * j + r16;
      if (gn >= N) continue;
      auto* q = Dp + gm + (int64_t)gn * d.ldd;
      if (gm + 3 < M) {
        if constexpr (sizeof(TO) == 4) {
          const f4u o = alpha * acc[i][j];
          *(f4u __attribute__((address_space(1)))*)q = o;
        } else {
          const d2u o0 = {(double)(alpha * acc[i][j][0]), (double)(alpha * acc[i][j][1])};
          const d2u o1 = {(double)(alpha * acc[i][j][2]), (double)(alpha * acc[i][j][3])};
          *(d2u __attribute__((address_space(1)))*)q = o0;
          *(d2u __attribute__((address_space(1)))*)(q + 2) = o1;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (gm + e < M) q[e] = (TO)(alpha * acc[i][j][e]);
      }
    }
}

template <int BM, int BN, int TA, int TB, int TERMS>
__global__ __launch_bounds__(256, 2) void gemm_bf16s_pair_kernel(const GemmDesc* __restrict__ descs,
                                                              const int* __restrict__ tmap,
                                                              int tiles) {
  gemm_bf16s_body<BM, BN, TA, TB, float, TERMS>(descs, tmap, tiles);
}
template <int BM, int BN, int TA, int TB, int TERMS>
__global__ __launch_bounds__(256, 2) void gemm_bf16s_o64_kernel(const GemmDesc* __restrict__ descs,
                                                             const int* __restrict__ tmap,
                                                             int tiles) {
  gemm_bf16s_body<BM, BN, TA, TB, double, TERMS>(descs, tmap, tiles);
}

template <int BM, int BN, int TA, int TB, int TERMS>
static void launch_bf16s_cfg(const GemmDesc* d, const int* tmap, int tiles, hipStream_t st,
                             bool out64) {
  const int grid = (tiles + 7) & ~7;
  if (out64)
    hipLaunchKernelGGL((gemm_bf16s_o64_kernel<BM, BN, TA, TB, TERMS>), dim3(grid), dim3(256), 0,
                       st, d, tmap, tiles);
  else
    hipLaunchKernelGGL((gemm_bf16s_pair_kernel<BM, BN, TA, TB, TERMS>), dim3(grid), dim3(256), 0,
                       st, d, tmap, tiles);
}

template <int BM, int BN, int TERMS>
static void launch_bf16s_t(const GemmDesc* d, const int* tmap, int tiles, hipStream_t st, int tA,
                           int tB, bool out64) {
  if (!tA && !tB) launch_bf16s_cfg<BM, BN, 0, 0, TERMS>(d, tmap, tiles, st, out64);
  else if (!tA && tB) launch_bf16s_cfg<BM, BN, 0, 1, TERMS>(d, tmap, tiles, st, out64);
  else if (tA && !tB) launch_bf16s_cfg<BM, BN, 1, 0, TERMS>(d, tmap, tiles, st, out64);
  else launch_bf16s_cfg<BM, BN, 1, 1, TERMS>(d, tmap, tiles, st, out64);
}

template <int TERMS>
static void launch_bf16s_terms(const GemmDesc* d, const int* tmap, int tiles, hipStream_t st,
                               int cfg, int tA, int tB, bool out64) {
  switch (cfg) {
    case 1: launch_bf16s_t<128, 64, TERMS>(d, tmap, tiles, st, tA, tB, out64); break;
    case 2: launch_bf16s_t<128, 128, TERMS>(d, tmap, tiles, st, tA, tB, out64); break;
    default: launch_bf16s_t<64, 64, TERMS>(d, tmap, tiles, st, tA, tB, out64); break;
  }
}

hipError_t launch_gemm_bf16s(const GemmDesc* d_desc, const int* d_tile_map, int count, int tiles,
                             hipStream_t st, int cfg, int tA, int tB, bool out64, int terms) {
  if (count <= 0 || tiles <= 0) return hipSuccess;
  if (terms == 3) launch_bf16s_terms<3>(d_desc, d_tile_map, tiles, st, cfg, tA, tB, out64);
  else if (terms == 1) launch_bf16s_terms<1>(d_desc, d_tile_map, tiles, st, cfg, tA, tB, out64);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace h2
