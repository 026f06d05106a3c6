// Neighbour gathers of the substitution (Eq. 31 and its transpose) and of
// the H^2 matrix-vector product: block-chunk products into partial slots and
// the per-box reductions (see GatherPlan).
#include <hip/hip_ext.h>

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

// FP64 chunks with GChunk::vec, one right-hand side: lane (g, q) = (lane >> 5,
// lane & 31) reads rows 2q, 2q+1 of the columns 2u + g of each batch of 2U
// columns with one 16-byte load (8-byte alignment suffices on this part; a
// wave moves two columns of 64 rows per load).  With an odd row count the
// lane of the last row reads that row alone.  Direct sums are reduced over
// the two lane halves at the end, the transposed ones over the 32 lanes of
// each half after every batch; both in a fixed order that does not depend
// on the chunk's address.
typedef double f64x2a8 __attribute__((ext_vector_type(2), aligned(8)));

template <bool TAIL>
__device__ __forceinline__ f64x2a8 load_rows2(const double* p, bool both) {
  if (!TAIL || both)
    return __builtin_nontemporal_load(reinterpret_cast<gptr_t<f64x2a8>>(as_global(p)));
  f64x2a8 v;
  v.x = __builtin_nontemporal_load(as_global(p));
  v.y = 0.0;
  return v;
}

template <int U, bool TAIL>
__device__ __forceinline__ void gv64_body(const GChunk& ch, double* __restrict__ P, int lane) {
  static_assert(U == 16, "32 columns per batch");
  const int q = lane & 31, g = lane >> 5;
  const bool dir = ch.od >= 0, tr = ch.ot >= 0;
  const int nr = ch.nr, mc = ch.mc;
  const int64_t ld = ch.ld;
  const bool live = 2 * q < nr;
  const int qe = live ? q : 0;
  const bool both = 2 * qe + 1 < nr;
  const double* base = static_cast<const double*>(ch.M) + 2 * qe;
  const double xt0 = (tr && 2 * q < nr) ? as_global(ch.xt)[2 * q] : 0.0;
  const double xt1 = (tr && 2 * q + 1 < nr) ? as_global(ch.xt)[2 * q + 1] : 0.0;
  double acc0 = 0.0, acc1 = 0.0;
  for (int s0 = 0; s0 < mc; s0 += 2 * U) {
    const double xv = (dir && lane < 2 * U && s0 + lane < mc) ? as_global(ch.xd)[s0 + lane] : 0.0;
    f64x2a8 d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int cc = min(s0 + 2 * u + g, mc - 1);
      d[u] = load_rows2<TAIL>(base + (int64_t)cc * ld, both);
    }
    if (dir) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double xu = __shfl(xv, 2 * u + g, 64);
        acc0 += d[u].x * xu;
        acc1 += d[u].y * xu;
      }
    }
    if (tr) {
      // sums over the 32 lanes of each half: exchanges at distances 16, 8,
      // 4, 2 halve the values a lane carries, the last one adds the pair
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = d[u].x * xt0 + d[u].y * xt1;
      double a[8], b[4], c[2];
      const bool b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1,
                 b1 = (lane >> 1) & 1;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        a[j] = (b4 ? v[8 + j] : v[j]) + __shfl_xor(b4 ? v[j] : v[8 + j], 16, 64);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = (b3 ? a[4 + j] : a[j]) + __shfl_xor(b3 ? a[j] : a[4 + j], 8, 64);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        c[j] = (b2 ? b[2 + j] : b[j]) + __shfl_xor(b2 ? b[j] : b[2 + j], 4, 64);
      double e = (b1 ? c[1] : c[0]) + __shfl_xor(b1 ? c[0] : c[1], 2, 64);
      e += __shfl_xor(e, 1, 64);
      // lane q holds value (q >> 1): column s0 + 2 (q >> 1) + g
      const int col = s0 + 2 * (q >> 1) + g;
      if ((q & 1) == 0 && col < mc) P[ch.ot + ch.tcol + col] = e;
    }
  }
  if (dir) {
    // rows 2q, 2q+1 summed over the two halves: lane (q, g) keeps row 2q + g
    const double r = (g ? acc1 : acc0) + __shfl_xor(g ? acc0 : acc1, 32, 64);
    if (2 * q + g < nr) P[ch.od + ch.drow + 2 * q + g] = r;
  }
}

__device__ __forceinline__ void gv64_one(const GChunk& ch, double* __restrict__ P, int lane) {
  if (__builtin_amdgcn_readfirstlane(ch.nr) & 1) gv64_body<16, true>(ch, P, lane);
  else gv64_body<16, false>(ch, P, lane);
}

// FP32 chunks with GChunk::vec (128 rows), one right-hand side: lane (g, q) =
// (lane >> 5, lane & 31) reads rows 4q..4q+3 of the columns 2u + g of each
// batch of 2U = 16 columns with one 16-byte load (4-byte alignment suffices on
// this part; a wave moves two columns of 128 rows per load).  The lane of a
// row group that the chunk ends inside reads its rows one by one.  Direct
// sums are reduced over the two lane halves at the end, the transposed ones
// over the 32 lanes of each half after every batch, in a fixed order that
// does not depend on the chunk's address.
typedef float f32x4a4 __attribute__((ext_vector_type(4), aligned(4)));

template <bool TAIL>
__device__ __forceinline__ f32x4a4 load_rows4(const float* p, int valid) {
  if (!TAIL || valid >= 4)
    return __builtin_nontemporal_load(reinterpret_cast<gptr_t<f32x4a4>>(as_global(p)));
  f32x4a4 v;
  v.x = valid > 0 ? __builtin_nontemporal_load(as_global(p)) : 0.f;
  v.y = valid > 1 ? __builtin_nontemporal_load(as_global(p + 1)) : 0.f;
  v.z = valid > 2 ? __builtin_nontemporal_load(as_global(p + 2)) : 0.f;
  v.w = 0.f;
  return v;
}

template <int U, bool TAIL>
__device__ __forceinline__ void gv32_body(const GChunk& ch, double* __restrict__ P, int lane,
                                          int nrhs) {
  static_assert(U == 8, "16 columns per batch");
  const int q = lane & 31, g = lane >> 5;
  const bool dir = ch.od >= 0, tr = ch.ot >= 0;
  const int nr = ch.nr, mc = ch.mc;
  const int64_t ld = ch.ld;
  const bool live = 4 * q < nr;
  const int qe = live ? q : 0;
  const int valid = nr - 4 * qe;  // rows of the group inside the chunk (>= 1)
  const float* base = static_cast<const float*>(ch.M) + 4 * qe;
  double xt[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) xt[t] = (tr && 4 * q + t < nr) ? as_global(ch.xt)[4 * q + t] : 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < mc; s0 += 2 * U) {
    const double xv = (dir && lane < 2 * U && s0 + lane < mc) ? as_global(ch.xd)[s0 + lane] : 0.0;
    f32x4a4 d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int cc = min(s0 + 2 * u + g, mc - 1);
      d[u] = load_rows4<TAIL>(base + (int64_t)cc * ld, valid);
    }
    if (dir && nrhs == 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double xu = __shfl(xv, 2 * u + g, 64);
        acc[0] += (double)d[u].x * xu;
        acc[1] += (double)d[u].y * xu;
        acc[2] += (double)d[u].z * xu;
        acc[3] += (double)d[u].w * xu;
      }
    }
    if (tr && nrhs == 1) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        v[u] = (double)d[u].x * xt[0] + (double)d[u].y * xt[1] + (double)d[u].z * xt[2] +
               (double)d[u].w * xt[3];
      double a[4], b[2];
      const bool b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        a[j] = (b4 ? v[4 + j] : v[j]) + __shfl_xor(b4 ? v[j] : v[4 + j], 16, 64);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = (b3 ? a[2 + j] : a[j]) + __shfl_xor(b3 ? a[j] : a[2 + j], 8, 64);
      double e = (b2 ? b[1] : b[0]) + __shfl_xor(b2 ? b[0] : b[1], 4, 64);
      e += __shfl_xor(e, 2, 64);
      e += __shfl_xor(e, 1, 64);
      // lane q holds value (q >> 2): column s0 + 2 (q >> 2) + g
      const int col = s0 + 2 * (q >> 2) + g;
      if ((q & 3) == 0 && col < mc) P[ch.ot + ch.tcol + col] = e;
    }
  }
  if (dir && nrhs == 1) {
    // rows 4q..4q+3 summed over the two halves: lane (q, g) keeps rows
    // 4q + 2g + {0, 1}
    const double r0 = (g ? acc[2] : acc[0]) + __shfl_xor(g ? acc[0] : acc[2], 32, 64);
    const double r1 = (g ? acc[3] : acc[1]) + __shfl_xor(g ? acc[1] : acc[3], 32, 64);
    const int rr = 4 * q + 2 * g;
    if (rr < nr) P[ch.od + ch.drow + rr] = r0;
    if (rr + 1 < nr) P[ch.od + ch.drow + rr + 1] = r1;
  }
}

__device__ __forceinline__ void gv32_one(const GChunk& ch, double* __restrict__ P, int lane,
                                         int nrhs) {
  if (__builtin_amdgcn_readfirstlane(ch.nr) & 3) gv32_body<8, true>(ch, P, lane, nrhs);
  else gv32_body<8, false>(ch, P, lane, nrhs);
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
  if constexpr (NR == 1 && sizeof(T) == 8 && RMAX == 1) {
    if (__builtin_amdgcn_readfirstlane(ch.vec)) { gv64_one(ch, P, lane); return; }
  }
  if constexpr (NR == 1 && sizeof(T) == 4 && RMAX == 2) {
    // nrhs (1 here) stays a run-time value: the compiler keeps the direct and
    // transposed products apart and needs fewer registers
    if (__builtin_amdgcn_readfirstlane(ch.vec)) { gv32_one(ch, P, lane, nrhs); return; }
  }
  if constexpr (RMAX >= 4) {
    if (rpl >= 4) { gchunk_one<NR, T, 4, BW>(ch, P, nrhs, lane); return; }
    if (rpl == 3) { gchunk_one<NR, T, 3, BW>(ch, P, nrhs, lane); return; }
  }
  if constexpr (RMAX >= 2) {
    if (rpl == 2) { gchunk_one<NR, T, 2, BW>(ch, P, nrhs, lane); return; }
  }
  gchunk_one<NR, T, 1, BW>(ch, P, nrhs, lane);
}

// ------------------------------------------------------ packed BF16 chunks
// Chunks of the packed BF16 copies (GatherPlan::v16): the leading dimension
// is a multiple of 8 elements and every chunk starts on a 16-byte boundary,
// so lane (g, q) = (lane >> 4, lane & 15) reads rows 8q..8q+7 of one column
// with a single 16-byte load, and one load instruction of the wave moves
// four columns of 128 rows (1 KiB).  Columns 4u + g of each batch of 4U
// columns belong to lane group g.  Direct sums (rows) are reduced over the
// four groups at the end of the chunk, transposed sums (columns) over the
// sixteen row groups after each batch; both in a fixed order.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int T>
__device__ __forceinline__ double bf16_at(const u32x4& v) {
  const unsigned w = v[T >> 1];
  return (double)__uint_as_float((T & 1) ? (w & 0xffff0000u) : (w << 16));
}

// Sum of v[0..N) over the 16 lanes of each lane group (lanes with equal
// lane >> 4), halving the values a lane carries at each exchange: on return
// lane q of the group holds the total of value q (N = 16) or of value q >> 1
// (N = 8).
template <int N>
__device__ __forceinline__ double reduce_group16(const double (&v)[N], int lane) {
  static_assert(N == 16 || N == 8, "16 or 8 values");
  constexpr int H = N / 2;
  double a[H];
  const bool b3 = (lane >> 3) & 1;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double send = b3 ? v[j] : v[H + j];
    const double keep = b3 ? v[H + j] : v[j];
    a[j] = keep + __shfl_xor(send, 8, 64);
  }
  constexpr int Q = H / 2;
  double b[Q];
  const bool b2 = (lane >> 2) & 1;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const double send = b2 ? a[j] : a[Q + j];
    const double keep = b2 ? a[Q + j] : a[j];
    b[j] = keep + __shfl_xor(send, 4, 64);
  }
  const bool b1 = (lane >> 1) & 1;
  if constexpr (N == 16) {
    double c[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double send = b1 ? b[j] : b[2 + j];
      const double keep = b1 ? b[2 + j] : b[j];
      c[j] = keep + __shfl_xor(send, 2, 64);
    }
    const bool b0 = lane & 1;
    return (b0 ? c[1] : c[0]) + __shfl_xor(b0 ? c[0] : c[1], 1, 64);
  } else {
    const double c = (b1 ? b[1] : b[0]) + __shfl_xor(b1 ? b[0] : b[1], 2, 64);
    return c + __shfl_xor(c, 1, 64);
  }
}

template <int NR, int U>
__global__ __launch_bounds__(256) void gv16_kernel(const GChunk* __restrict__ chunks, int nch,
                                                   double* __restrict__ P, int nrhs) {
  const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (w >= nch) return;
  const GChunk& ch = chunks[w];
  const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4;
  const bool dir = ch.od >= 0, tr = ch.ot >= 0;
  const int nr = ch.nr, mc = ch.mc;
  const int64_t colb = (int64_t)ch.ld * 2;  // bytes per column
  // row groups past the chunk read group 0 (in bounds); their x_t is zero
  // and their direct sums are never stored
  const bool live = 8 * q < nr;
  const char* base = static_cast<const char*>(ch.M) + 16 * (live ? q : 0);
  double xt[8][NR], acc[8][NR];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      acc[t][c] = 0.0;
      xt[t][c] = (tr && c < nrhs && 8 * q + t < nr)
                     ? as_global(ch.xt)[8 * q + t + (int64_t)c * ch.ldxt]
                     : 0.0;
    }
  for (int s0 = 0; s0 < mc; s0 += 4 * U) {
    double xv[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c)
      xv[c] = (dir && c < nrhs && lane < 4 * U && s0 + lane < mc)
                  ? as_global(ch.xd)[s0 + lane + (int64_t)c * ch.ldxd]
                  : 0.0;
    u32x4 d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // columns past the chunk read its last column; x_d is zero there and
      // their transposed sums are not stored
      const int cc = min(s0 + 4 * u + g, mc - 1);
      d[u] = __builtin_nontemporal_load(
          reinterpret_cast<gptr_t<u32x4>>(as_global(base + (int64_t)cc * colb)));
    }
    if (dir) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        if (c < nrhs) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const double xu = __shfl(xv[c], 4 * u + g, 64);
            acc[0][c] += bf16_at<0>(d[u]) * xu;
            acc[1][c] += bf16_at<1>(d[u]) * xu;
            acc[2][c] += bf16_at<2>(d[u]) * xu;
            acc[3][c] += bf16_at<3>(d[u]) * xu;
            acc[4][c] += bf16_at<4>(d[u]) * xu;
            acc[5][c] += bf16_at<5>(d[u]) * xu;
            acc[6][c] += bf16_at<6>(d[u]) * xu;
            acc[7][c] += bf16_at<7>(d[u]) * xu;
          }
        }
      }
    }
    if (tr) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        if (c < nrhs) {
          double pt[U];
#pragma unroll
          for (int u = 0; u < U; ++u)
            pt[u] = bf16_at<0>(d[u]) * xt[0][c] + bf16_at<1>(d[u]) * xt[1][c] +
                    bf16_at<2>(d[u]) * xt[2][c] + bf16_at<3>(d[u]) * xt[3][c] +
                    bf16_at<4>(d[u]) * xt[4][c] + bf16_at<5>(d[u]) * xt[5][c] +
                    bf16_at<6>(d[u]) * xt[6][c] + bf16_at<7>(d[u]) * xt[7][c];
          const double tot = reduce_group16<U>(pt, lane);
          const int uu = U == 16 ? q : (q >> 1);
          const int col = s0 + 4 * uu + g;
          if (col < mc && (U == 16 || (q & 1) == 0))
            P[ch.ot * nrhs + (int64_t)c * ch.tlen + ch.tcol + col] = tot;
        }
      }
    }
  }
  if (dir) {
    // rows 8q..8q+7 summed over the four lane groups: lane (q, g) keeps rows
    // 8q + 4 (g & 1) + 2 (g >> 1) + {0, 1}
    const bool g0 = g & 1, g1 = (g >> 1) & 1;
    const int r0 = 8 * q + 4 * g0 + 2 * g1;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c < nrhs) {
        double a[4], b[2];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double send = g0 ? acc[j][c] : acc[4 + j][c];
          const double keep = g0 ? acc[4 + j][c] : acc[j][c];
          a[j] = keep + __shfl_xor(send, 16, 64);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double send = g1 ? a[j] : a[2 + j];
          const double keep = g1 ? a[2 + j] : a[j];
          b[j] = keep + __shfl_xor(send, 32, 64);
        }
        double* dst = P + ch.od * nrhs + (int64_t)c * ch.dlen + ch.drow;
        if (r0 < nr) dst[r0] = b[0];
        if (r0 + 1 < nr) dst[r0 + 1] = b[1];
      }
    }
  }
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
                             bool wide, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid((nch + 3) / 4), blk(256);
  constexpr int RN = rows_per_lane<T>();
  constexpr int RW = sizeof(T) < 8 ? GATHER_WIDE_RPL32 : GATHER_WIDE_RPL64;
  static_assert(GATHER_WIDE_NR == 2, "wide instantiations below");
  if (wide) {
    if (nrhs == 1) hipExtLaunchKernelGGL((gchunk_kernel<1, T, RW, 8>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
    else hipExtLaunchKernelGGL((gchunk_kernel<2, T, RW, 8>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
    return;
  }
  if (nrhs == 1) hipExtLaunchKernelGGL((gchunk_kernel<1, T, RN, 16>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
  else if (nrhs <= 2) hipExtLaunchKernelGGL((gchunk_kernel<2, T, RN, 16>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
  else if (nrhs <= 4) hipExtLaunchKernelGGL((gchunk_kernel<4, T, RN, 16>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
  else if (nrhs <= 8) hipExtLaunchKernelGGL((gchunk_kernel<8, T, RN, 16>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
  else hipExtLaunchKernelGGL((gchunk_kernel<16, T, RN, 16>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
}

hipError_t launch_gchunks(const GChunk* ch, int nch, double* P, int nrhs, int esz,
                          hipStream_t st, bool wide, bool v16, hipEvent_t e0, hipEvent_t e1) {
  if (nch <= 0) return hipSuccess;
  if (nrhs > GNR || nrhs < 1) return hipErrorInvalidValue;
  if (wide && nrhs > GATHER_WIDE_NR) return hipErrorInvalidValue;
  if (v16 && esz == 2 && !wide && nrhs <= GV16_NR) {
    static_assert(GV16_NR == 1, "instantiation below");
    const dim3 grid((nch + 3) / 4), blk(256);
    hipExtLaunchKernelGGL((gv16_kernel<1, 16>), grid, blk, 0, st, e0, e1, 0, ch, nch, P, nrhs);
    return hipGetLastError();
  }
  if (esz == 8) launch_gchunks_t<double>(ch, nch, P, nrhs, st, wide, e0, e1);
  else if (esz == 4) launch_gchunks_t<float>(ch, nch, P, nrhs, st, wide, e0, e1);
  else if (esz == 2) launch_gchunks_t<unsigned short>(ch, nch, P, nrhs, st, wide, e0, e1);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_greduce(const GRed* rd, int nred, int max_rows, const int64_t* offs,
                          const double* P, int nrhs, hipStream_t st, hipEvent_t e0,
                          hipEvent_t e1) {
  if (nred <= 0 || max_rows <= 0) return hipSuccess;
  if (nrhs > GNR || nrhs < 1) return hipErrorInvalidValue;
  const dim3 grid(nred, (max_rows + 255) / 256), blk(256);
  if (nrhs == 1) hipExtLaunchKernelGGL(greduce_kernel<1>, grid, blk, 0, st, e0, e1, 0, rd, offs, P, nrhs);
  else if (nrhs <= 2) hipExtLaunchKernelGGL(greduce_kernel<2>, grid, blk, 0, st, e0, e1, 0, rd, offs, P, nrhs);
  else if (nrhs <= 4) hipExtLaunchKernelGGL(greduce_kernel<4>, grid, blk, 0, st, e0, e1, 0, rd, offs, P, nrhs);
  else if (nrhs <= 8) hipExtLaunchKernelGGL(greduce_kernel<8>, grid, blk, 0, st, e0, e1, 0, rd, offs, P, nrhs);
  else hipExtLaunchKernelGGL(greduce_kernel<16>, grid, blk, 0, st, e0, e1, 0, rd, offs, P, nrhs);
  return hipGetLastError();
}

}  // namespace h2
