// Neighbour gathers of the substitution (Eq. 31 and its transpose) and of
// the H^2 matrix-vector product: block-chunk products into partial slots and
// the per-box reductions (see GatherPlan).
#include "h2_internal.hpp"

namespace h2 {

// ------------------------------------------------------------------ gathers
// The substitution and the matvec stream every stored factor block once per
// sweep: HBM-bound.  One wave owns one 64-row chunk of a block (lane = row),
// keeps sixteen column loads in flight (non-temporal: every block is read
// once per pass), and needs no barrier: workgroups are four independent waves.
constexpr int GNR = 16;  // max right-hand sides per pass

// Sum of v[0..7] over the 64 lanes in 10 exchanges instead of 48: each
// butterfly step halves the number of values a lane carries.  On return,
// lane l holds the total of column (l >> 3) & 7.
__device__ __forceinline__ double reduce8(const double (&v)[8], int lane) {
  const bool h = (lane >> 5) & 1, g = (lane >> 4) & 1, f = (lane >> 3) & 1;
  double w[4], z[2];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double send = h ? v[j] : v[4 + j];
    const double keep = h ? v[4 + j] : v[j];
    w[j] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const double send = g ? w[j] : w[2 + j];
    const double keep = g ? w[2 + j] : w[j];
    z[j] = keep + __shfl_xor(send, 16, 64);
  }
  double q = (f ? z[1] : z[0]) + __shfl_xor(f ? z[0] : z[1], 8, 64);
  q += __shfl_xor(q, 4, 64);
  q += __shfl_xor(q, 2, 64);
  q += __shfl_xor(q, 1, 64);
  return q;
}

// Global-address-space view of a pointer: plain global loads instead of
// flat ones (the pointers arrive through descriptors).
template <typename T>
using gptr_t = const T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gptr_t<T> as_global(const T* p) { return (gptr_t<T>)p; }

// Value of v in lane l (l uniform), through the scalar unit.
__device__ __forceinline__ double bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Rows per lane: a chunk is 64 * RPL rows, lane l owns rows l + 64 t.  FP32
// and BF16 copies take two rows per lane (the transposed sums add both rows
// before the cross-lane reduction).  BF16 elements are held as their 16 bits
// (unsigned short) and widened by a shift.
template <typename T>
constexpr int rows_per_lane() { return sizeof(T) < 8 ? 2 : 1; }
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(unsigned short v) {
  return (double)__uint_as_float((unsigned)v << 16);
}

// One batch of BW columns (8 or 16) starting at column sb (BW loads per row in
// flight); xv[c] holds x_d of the current 64 columns, one per lane, and bo is
// the batch's first column within them.  Rows past the chunk read the
// chunk's last row (always in bounds); their x_t is zero and their direct
// sums are never stored.
template <int NR, int RPL, int BW, bool FULL, typename T>
__device__ __forceinline__ void gchunk_cols(const gptr_t<T> (&col)[RPL], int64_t ld, int sb,
                                            int mc, int lane, int nrhs, const double (&xv)[NR],
                                            int bo, const double (&xt)[RPL][NR],
                                            double (&acc)[RPL][NR], double (&tq)[NR], bool dir,
                                            bool tr, int bi) {
  T bv[RPL][BW];
#pragma unroll
  for (int u = 0; u < BW; ++u)
#pragma unroll
    for (int t = 0; t < RPL; ++t)
      bv[t][u] = (FULL || sb + u < mc) ? __builtin_nontemporal_load(col[t] + (int64_t)u * ld)
                                       : T(0);
  if (dir) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c >= nrhs) break;
#pragma unroll
      for (int u = 0; u < BW; ++u)
        if (FULL || sb + u < mc) {
          const double xu = bcast(xv[c], bo + u);
#pragma unroll
          for (int t = 0; t < RPL; ++t) acc[t][c] += widen(bv[t][u]) * xu;
        }
    }
  }
  if (tr) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c >= nrhs) break;
#pragma unroll
      for (int h = 0; h < BW / 8; ++h) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) s += widen(bv[t][8 * h + u]) * xt[t][c];
          v[u] = s;
        }
        const double q = reduce8(v, lane);
        if ((lane & 7) == bi + h) tq[c] = q;
      }
    }
  }
}

template <int NR, typename T, int RPL, int BW>
__device__ __forceinline__ void gchunk_one(const GChunk& ch, double* __restrict__ P, int nrhs,
                                           int lane) {
  const bool dir = ch.od >= 0, tr = ch.ot >= 0;
  bool live[RPL];
  gptr_t<T> col0[RPL];
  double xt[RPL][NR], acc[RPL][NR];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = lane + 64 * t;
    live[t] = r < ch.nr;
    col0[t] = as_global(static_cast<const T*>(ch.M)) + (live[t] ? r : ch.nr - 1);
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      acc[t][c] = 0.0;
      xt[t][c] = (tr && live[t] && c < nrhs) ? as_global(ch.xt)[r + (int64_t)c * ch.ldxt] : 0.0;
    }
  }
  const int64_t ld = ch.ld;
  for (int s0 = 0; s0 < ch.mc; s0 += 64) {
    const int ns = min(64, ch.mc - s0);
    double tq[NR], xv[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      tq[c] = 0.0;
      xv[c] = (dir && lane < ns && c < nrhs) ? as_global(ch.xd)[s0 + lane + (int64_t)c * ch.ldxd]
                                             : 0.0;
    }
    int b = 0;
    for (; b <= ns - BW; b += BW) {
      gptr_t<T> col[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) col[t] = col0[t] + (int64_t)(s0 + b) * ld;
      gchunk_cols<NR, RPL, BW, true, T>(col, ld, s0 + b, ch.mc, lane, nrhs, xv, b, xt, acc, tq, dir,
                                    tr, b >> 3);
    }
    if (b < ns) {
      gptr_t<T> col[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) col[t] = col0[t] + (int64_t)(s0 + b) * ld;
      gchunk_cols<NR, RPL, BW, false, T>(col, ld, s0 + b, ch.mc, lane, nrhs, xv, b, xt, acc, tq, dir,
                                     tr, b >> 3);
    }
    if (tr) {
      const int cc = 8 * (lane & 7) + (lane >> 3);
      if (cc < ns)
        for (int c = 0; c < nrhs; ++c)
          P[ch.ot * nrhs + (int64_t)c * ch.tlen + ch.tcol + s0 + cc] = tq[c];
    }
  }
  if (dir)
#pragma unroll
    for (int t = 0; t < RPL; ++t)
      if (live[t])
        for (int c = 0; c < nrhs; ++c)
          P[ch.od * nrhs + (int64_t)c * ch.dlen + ch.drow + lane + 64 * t] = acc[t][c];
}

// RMAX: the largest rows-per-lane of the plan the chunks come from; each
// chunk runs the variant of its own row count (wave-uniform).  BW: columns
// per batch; 8 keeps the wide variants at four or more waves per SIMD.
template <int NR, typename T, int RMAX, int BW>
__global__ __launch_bounds__(256) void gchunk_kernel(const GChunk* __restrict__ chunks, int nch,
                                                     double* __restrict__ P, int nrhs) {
  const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (w >= nch) return;
  const GChunk& ch = chunks[w];
  const int rpl = __builtin_amdgcn_readfirstlane(ch.rpl);
  const int lane = threadIdx.x & 63;
  if constexpr (RMAX >= 4) {
    if (rpl >= 4) { gchunk_one<NR, T, 4, BW>(ch, P, nrhs, lane); return; }
    if (rpl == 3) { gchunk_one<NR, T, 3, BW>(ch, P, nrhs, lane); return; }
  }
  if constexpr (RMAX >= 2) {
    if (rpl == 2) { gchunk_one<NR, T, 2, BW>(ch, P, nrhs, lane); return; }
  }
  gchunk_one<NR, T, 1, BW>(ch, P, nrhs, lane);
}

template <int NR>
__global__ __launch_bounds__(256) void greduce_kernel(const GRed* __restrict__ reds,
                                                      const int64_t* __restrict__ offs,
                                                      const double* __restrict__ P, int nrhs) {
  const GRed g = reds[blockIdx.x];
  const int r = blockIdx.y * 256 + threadIdx.x;
  if (r >= g.rows) return;
  double acc[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = 0.0;
  // UN slots in flight per pass; the sum still runs over the slots in order
  constexpr int UN = NR <= 2 ? 8 : NR <= 4 ? 4 : 2;
  for (int q = g.s0; q < g.s1; q += UN) {
    double v[UN][NR];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const bool in = q + u < g.s1;
      const double* p = P + (in ? offs[q + u] : 0) * nrhs + r;
#pragma unroll
      for (int c = 0; c < NR; ++c) v[u][c] = (in && c < nrhs) ? p[(int64_t)c * g.rows] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int c = 0; c < NR; ++c)
        if (q + u < g.s1) acc[c] += v[u][c];
  }
  for (int c = 0; c < nrhs; ++c) {
    const double base = g.base ? g.base[r + (int64_t)c * g.ldbase] : 0.0;
    g.y[r + (int64_t)c * g.ldy] = base + g.alpha * acc[c];
  }
}

template <typename T>
static void launch_gchunks_t(const GChunk* ch, int nch, double* P, int nrhs, hipStream_t st,
                             bool wide) {
  const dim3 grid((nch + 3) / 4), blk(256);
  constexpr int RN = rows_per_lane<T>();
  constexpr int RW = sizeof(T) < 8 ? GATHER_WIDE_RPL32 : GATHER_WIDE_RPL64;
  static_assert(GATHER_WIDE_NR == 2, "wide instantiations below");
  if (wide) {
    if (nrhs == 1) hipLaunchKernelGGL((gchunk_kernel<1, T, RW, 8>), grid, blk, 0, st, ch, nch, P, nrhs);
    else hipLaunchKernelGGL((gchunk_kernel<2, T, RW, 8>), grid, blk, 0, st, ch, nch, P, nrhs);
    return;
  }
  if (nrhs == 1) hipLaunchKernelGGL((gchunk_kernel<1, T, RN, 16>), grid, blk, 0, st, ch, nch, P, nrhs);
  else if (nrhs <= 2) hipLaunchKernelGGL((gchunk_kernel<2, T, RN, 16>), grid, blk, 0, st, ch, nch, P, nrhs);
  else if (nrhs <= 4) hipLaunchKernelGGL((gchunk_kernel<4, T, RN, 16>), grid, blk, 0, st, ch, nch, P, nrhs);
  else if (nrhs <= 8) hipLaunchKernelGGL((gchunk_kernel<8, T, RN, 16>), grid, blk, 0, st, ch, nch, P, nrhs);
  else hipLaunchKernelGGL((gchunk_kernel<16, T, RN, 16>), grid, blk, 0, st, ch, nch, P, nrhs);
}

hipError_t launch_gchunks(const GChunk* ch, int nch, double* P, int nrhs, int esz,
                          hipStream_t st, bool wide) {
  if (nch <= 0) return hipSuccess;
  if (nrhs > GNR || nrhs < 1) return hipErrorInvalidValue;
  if (wide && nrhs > GATHER_WIDE_NR) return hipErrorInvalidValue;
  if (esz == 8) launch_gchunks_t<double>(ch, nch, P, nrhs, st, wide);
  else if (esz == 4) launch_gchunks_t<float>(ch, nch, P, nrhs, st, wide);
  else if (esz == 2) launch_gchunks_t<unsigned short>(ch, nch, P, nrhs, st, wide);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_greduce(const GRed* rd, int nred, int max_rows, const int64_t* offs,
                          const double* P, int nrhs, hipStream_t st) {
  if (nred <= 0 || max_rows <= 0) return hipSuccess;
  if (nrhs > GNR || nrhs < 1) return hipErrorInvalidValue;
  const dim3 grid(nred, (max_rows + 255) / 256), blk(256);
  if (nrhs == 1) hipLaunchKernelGGL(greduce_kernel<1>, grid, blk, 0, st, rd, offs, P, nrhs);
  else if (nrhs <= 2) hipLaunchKernelGGL(greduce_kernel<2>, grid, blk, 0, st, rd, offs, P, nrhs);
  else if (nrhs <= 4) hipLaunchKernelGGL(greduce_kernel<4>, grid, blk, 0, st, rd, offs, P, nrhs);
  else if (nrhs <= 8) hipLaunchKernelGGL(greduce_kernel<8>, grid, blk, 0, st, rd, offs, P, nrhs);
  else hipLaunchKernelGGL(greduce_kernel<16>, grid, blk, 0, st, rd, offs, P, nrhs);
  return hipGetLastError();
}

}  // namespace h2
