// Neighbour gathers of the substitution (Eq. 31 and its transpose) and of
// the H^2 matrix-vector product: block-chunk products into partial slots and
// the per-box reductions (see GatherPlan).
#include "h2_internal.hpp"

namespace h2 {

// ------------------------------------------------------------------ gathers
// The substitution and the matvec stream every stored factor block once per
// sweep: HBM-bound.  One wave owns one 64-row chunk of a block (lane = row),
// keeps eight column loads in flight, and needs no barrier: workgroups are
// four independent waves.
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

template <int NR, bool FULL>
__device__ __forceinline__ void gchunk_cols(const GChunk& ch, int s0, int b, int lane, bool live,
                                            int nrhs, const double (&xt)[NR], double (&acc)[NR],
                                            double (&tq)[NR], bool dir, bool tr) {
  const int sb = s0 + b;
  double bv[8];
  const double* col = ch.M + lane + (int64_t)sb * ch.ld;
#pragma unroll
  for (int u = 0; u < 8; ++u)
    bv[u] = (live && (FULL || sb + u < ch.mc)) ? col[(int64_t)u * ch.ld] : 0.0;
  if (dir) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c >= nrhs) break;
      const double* xd = ch.xd + sb + (int64_t)c * ch.ldxd;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (FULL || sb + u < ch.mc) acc[c] += bv[u] * xd[u];
    }
  }
  if (tr) {
    const int bi = b >> 3;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c >= nrhs) break;
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = bv[u] * xt[c];
      const double q = reduce8(v, lane);
      if ((lane & 7) == bi) tq[c] = q;
    }
  }
}

template <int NR>
__global__ __launch_bounds__(256) void gchunk_kernel(const GChunk* __restrict__ chunks, int nch,
                                                     double* __restrict__ P, int nrhs) {
  const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (w >= nch) return;
  const int lane = threadIdx.x & 63;
  const GChunk ch = chunks[w];
  const bool live = lane < ch.nr;
  const bool dir = ch.od >= 0, tr = ch.ot >= 0;
  double xt[NR], acc[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    acc[c] = 0.0;
    xt[c] = (tr && live && c < nrhs) ? ch.xt[lane + (int64_t)c * ch.ldxt] : 0.0;
  }
  for (int s0 = 0; s0 < ch.mc; s0 += 64) {
    const int ns = min(64, ch.mc - s0);
    double tq[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) tq[c] = 0.0;
    int b = 0;
    for (; b + 8 <= ns; b += 8)
      gchunk_cols<NR, true>(ch, s0, b, lane, live, nrhs, xt, acc, tq, dir, tr);
    if (b < ns) gchunk_cols<NR, false>(ch, s0, b, lane, live, nrhs, xt, acc, tq, dir, tr);
    if (tr) {
      const int cc = 8 * (lane & 7) + (lane >> 3);
      if (cc < ns)
        for (int c = 0; c < nrhs; ++c)
          P[ch.ot * nrhs + (int64_t)c * ch.mc + s0 + cc] = tq[c];
    }
  }
  if (dir && live)
    for (int c = 0; c < nrhs; ++c)
      P[ch.od * nrhs + (int64_t)c * ch.dlen + ch.drow + lane] = acc[c];
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
  for (int q = g.s0; q < g.s1; ++q) {
    const double* p = P + offs[q] * nrhs + r;
#pragma unroll
    for (int c = 0; c < NR; ++c)
      if (c < nrhs) acc[c] += p[(int64_t)c * g.rows];
  }
  for (int c = 0; c < nrhs; ++c) {
    const double base = g.base ? g.base[r + (int64_t)c * g.ldbase] : 0.0;
    g.y[r + (int64_t)c * g.ldy] = base + g.alpha * acc[c];
  }
}

hipError_t launch_gchunks(const GChunk* ch, int nch, double* P, int nrhs, hipStream_t st) {
  if (nch <= 0) return hipSuccess;
  if (nrhs > GNR || nrhs < 1) return hipErrorInvalidValue;
  const dim3 grid((nch + 3) / 4), blk(256);
  if (nrhs == 1) hipLaunchKernelGGL(gchunk_kernel<1>, grid, blk, 0, st, ch, nch, P, nrhs);
  else if (nrhs <= 2) hipLaunchKernelGGL(gchunk_kernel<2>, grid, blk, 0, st, ch, nch, P, nrhs);
  else if (nrhs <= 4) hipLaunchKernelGGL(gchunk_kernel<4>, grid, blk, 0, st, ch, nch, P, nrhs);
  else if (nrhs <= 8) hipLaunchKernelGGL(gchunk_kernel<8>, grid, blk, 0, st, ch, nch, P, nrhs);
  else hipLaunchKernelGGL(gchunk_kernel<16>, grid, blk, 0, st, ch, nch, P, nrhs);
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
