// Kernel-matrix evaluation, the neighbour gathers of the substitution and of
// the H^2 matrix-vector product, and vector utilities.
#include "h2_internal.hpp"

namespace h2 {

// ---------------------------------------------------------- kernel function
// Eq. 35 / Eq. 36 with the regularisation 1/(r + delta) (value 1/delta on the
// diagonal) and the covariance kernels with a nugget added where the two
// point indices coincide.
__device__ __forceinline__ double kernel_value(const KernelDev& k, double r, bool same) {
  switch (k.id) {
    case 0: return 1.0 / (r + k.delta);
    case 1: return exp(-k.kappa * r) / (r + k.delta);
    case 2: return exp(-(r * r) / (k.ell * k.ell)) + (same ? k.nugget : 0.0);
    default: {
      const double a = 1.7320508075688772 * r / k.ell;
      return (1.0 + a) * exp(-a) + (same ? k.nugget : 0.0);
    }
  }
}

__device__ __forceinline__ int find_item_v(const int* off, int count, int t) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One 64 x 64 output tile per workgroup; thread t owns row t%64 and 16 of the
// columns.
__global__ __launch_bounds__(256) void eval_kernel(const EvalDesc* __restrict__ descs,
                                                   const int* __restrict__ toff, int count,
                                                   const double* __restrict__ X, int dim,
                                                   const KernelDev* __restrict__ kern) {
  const int item = find_item_v(toff, count, blockIdx.x);
  const EvalDesc d = descs[item];
  const int t = blockIdx.x - toff[item];
  const int tiles_r = (d.nr + 63) / 64;
  const int r0 = (t % tiles_r) * 64, c0 = (t / tiles_r) * 64;
  const int r = r0 + (threadIdx.x & 63);
  if (r >= d.nr) return;
  const KernelDev k = kern[d.inst];
  const int64_t pr = d.rows[r];
  double xr[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < dim; ++a) xr[a] = X[pr * dim + a];
  for (int cc = threadIdx.x >> 6; cc < 64; cc += 4) {
    const int c = c0 + cc;
    if (c >= d.nc) break;
    const int64_t pc = d.cols[c];
    double s = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double df = xr[a] - X[pc * dim + a];
      s += df * df;
    }
    d.out[r + (int64_t)c * d.ld] = kernel_value(k, sqrt(s), pr == pc);
  }
}

hipError_t launch_eval(const EvalDesc* d_desc, const int* d_tile_off, int count, int tiles,
                       const double* X, int dim, const KernelDev* kern, hipStream_t st) {
  if (count <= 0 || tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(eval_kernel, dim3(tiles), dim3(256), 0, st, d_desc, d_tile_off, count, X,
                     dim, kern);
  return hipGetLastError();
}

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

// ------------------------------------------------------------ vector utilities
__global__ void gather_rows_kernel(const int64_t* idx, int64_t n, int nrhs, const double* src,
                                   int64_t lds, double* dst, int64_t ldd) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % n, c = e / n;
    dst[r + c * ldd] = src[idx[r] + c * lds];
  }
}

__global__ void scatter_rows_kernel(const int64_t* idx, int64_t n, int nrhs, const double* src,
                                    int64_t lds, double* dst, int64_t ldd) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % n, c = e / n;
    dst[idx[r] + c * ldd] = src[r + c * lds];
  }
}

static int grid_for(int64_t work) {
  int64_t g = (work + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_gather_rows(const int64_t* idx, int64_t n, int nrhs, const double* src,
                              int64_t lds, double* dst, int64_t ldd, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, idx, n, nrhs,
                     src, lds, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const int64_t* idx, int64_t n, int nrhs, const double* src,
                               int64_t lds, double* dst, int64_t ldd, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, idx, n,
                     nrhs, src, lds, dst, ldd);
  return hipGetLastError();
}

// Column partial sums: ws[c*NCH + chunk]; then fold (deterministic order).
constexpr int NCH = 256;

__global__ __launch_bounds__(256) void coldot_partial(const double* a, int64_t lda, const double* b,
                                                      int64_t ldb, int64_t n, double* ws) {
  __shared__ double sh[4];
  const int c = blockIdx.y;
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)NCH * 256)
    s += a[i + c * lda] * b[i + c * ldb];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) ws[c * NCH + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void coldot_fold(const double* ws, int nrhs, double* out) {
  const int c = threadIdx.x;
  if (c >= nrhs) return;
  double s = 0.0;
  for (int q = 0; q < NCH; ++q) s += ws[c * NCH + q];
  out[c] = s;
}

hipError_t launch_coldot(const double* a, int64_t lda, const double* b, int64_t ldb, int64_t n,
                         int nrhs, double* ws, double* out, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(coldot_partial, dim3(NCH, nrhs), dim3(256), 0, st, a, lda, b, ldb, n, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(coldot_fold, dim3(1), dim3(256), 0, st, ws, nrhs, out);
  return hipGetLastError();
}

// z = x + alpha[c] * y  (alpha per column from device memory if alphas != NULL,
// scaled by sgn), all n x nrhs with their own leading dimensions.
__global__ void axpby_kernel(double* z, int64_t ldz, const double* x, int64_t ldx, const double* y,
                             int64_t ldy, int64_t n, int nrhs, const double* alphas,
                             const double* alphas_den, double sgn) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % n, c = e / n;
    double a = sgn;
    if (alphas) a *= alphas[c];
    if (alphas_den) a /= alphas_den[c];
    z[r + c * ldz] = x[r + c * ldx] + a * y[r + c * ldy];
  }
}

hipError_t launch_axpby(double* z, int64_t ldz, const double* x, int64_t ldx, const double* y,
                        int64_t ldy, int64_t n, int nrhs, const double* alphas,
                        const double* alphas_den, double sgn, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, z, ldz, x, ldx, y,
                     ldy, n, nrhs, alphas, alphas_den, sgn);
  return hipGetLastError();
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace h2
