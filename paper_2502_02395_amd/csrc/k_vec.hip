// Kernel-matrix evaluation and vector utilities.
#include <climits>

#include "h2_internal.hpp"

namespace h2 {

// ---------------------------------------------------------- kernel function
// Eq. 35 / Eq. 36 with the regularisation 1/(r + delta) (value 1/delta on the
// diagonal), the covariance kernels with a nugget added where the two point
// indices coincide, and the Yukawa kernel with a drift along the first axis
// (dx0 = x_0 - y_0; its transpose is the same kernel with -beta).
__device__ __forceinline__ double kernel_value(const KernelDev& k, double r, double dx0, bool same) {
  switch (k.id) {
    case 0: return 1.0 / (r + k.delta);
    case 1: return exp(-k.kappa * r) / (r + k.delta);
    case 2: return exp(-(r * r) / (k.ell * k.ell)) + (same ? k.nugget : 0.0);
    case 4: {
      const double q = 1.0 / (r + k.delta);
      return exp(-k.kappa * r) * q * (1.0 + k.beta * dx0 * q) + (same ? k.nugget : 0.0);
    }
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
    double s = 0.0, dx0 = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double df = xr[a] - X[pc * dim + a];
      if (a == 0) dx0 = df;
      s += df * df;
    }
    d.out[r + (int64_t)c * d.ld] = kernel_value(k, sqrt(s), dx0, pr == pc);
  }
}

hipError_t launch_eval(const EvalDesc* d_desc, const int* d_tile_off, int count, int tiles,
                       const double* X, int dim, const KernelDev* kern, hipStream_t st) {
  if (count <= 0 || tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(eval_kernel, dim3(tiles), dim3(256), 0, st, d_desc, d_tile_off, count, X,
                     dim, kern);
  return hipGetLastError();
}

// ------------------------------------------------------------ vector utilities
// Four independent elements per thread and pass (coalesced: element
// i0 + 256 u of the block's 1024).
__global__ __launch_bounds__(256) void cvt_f32_kernel(const double* __restrict__ src,
                                                      float* __restrict__ dst, int64_t n) {
  for (int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x; i0 < n;
       i0 += (int64_t)gridDim.x * 1024) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = i0 + 256 * u < n ? src[i0 + 256 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 256 * u < n) dst[i0 + 256 * u] = (float)v[u];
  }
}

hipError_t launch_cvt_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 1023) / 1024, 65536);
  hipLaunchKernelGGL(cvt_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

// BF16 copies (round to nearest even through FP32), same access pattern.
template <typename TS>
__global__ __launch_bounds__(256) void cvt_bf16_kernel(const TS* __restrict__ src,
                                                       unsigned short* __restrict__ dst,
                                                       int64_t n) {
  for (int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x; i0 < n;
       i0 += (int64_t)gridDim.x * 1024) {
    TS v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = i0 + 256 * u < n ? src[i0 + 256 * u] : TS(0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 256 * u < n) {
        const __bf16 h = (__bf16)(float)v[u];
        dst[i0 + 256 * u] = __builtin_bit_cast(unsigned short, h);
      }
  }
}

hipError_t launch_cvt_bf16(const void* src, int esz_src, unsigned short* dst, int64_t n,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 1023) / 1024, 65536);
  if (esz_src == 8)
    hipLaunchKernelGGL(cvt_bf16_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const double*>(src), dst, n);
  else if (esz_src == 4)
    hipLaunchKernelGGL(cvt_bf16_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const float*>(src), dst, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Packed BF16 copies: one thread per 8-row group over the whole list;
// first[b] is the block of block b's first group (planned on the host), each
// thread steps forward from it to its own.  Groups run column by column (a
// column's top groups, then its bottom groups), so the two parts of a column
// are converted by neighbouring threads and the cache line they share is
// read once.  Each thread converts eight rows (to FP32, then to BF16,
// nearest even) and writes them with one 16-byte store; rows past the
// segment's end up to its leading dimension are written as zeros.
template <typename TS>
__global__ __launch_bounds__(256) void cvt_bf16_blks_kernel(const TS* __restrict__ src,
                                                            const CvtBlk* __restrict__ blks,
                                                            const int* __restrict__ first,
                                                            int count, int64_t groups,
                                                            unsigned short* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= groups) return;
  int sg = first[blockIdx.x];
  while (sg + 1 < count && blks[sg + 1].g0 <= e) ++sg;
  const CvtBlk g = blks[sg];
  // the group's index inside its block: a block has fewer than 2^31 groups
  // (its columns times its 8-row groups), so 32-bit quotients suffice
  int le = (int)(e - g.g0);
  int col, r;
  bool top;
  const int lead = g.c_top * g.gb;  // columns with a bottom part only
  if (le < lead) {
    col = le / g.gb;
    r = le - col * g.gb;
    top = false;
  } else {
    le -= lead;
    const int per = g.gt + g.gb;
    const int q = le / per;
    col = g.c_top + q;
    r = le - q * per;
    top = r < g.gt;
    if (!top) r -= g.gt;
  }
  const int r_lo = top ? 0 : g.split;          // the segment's first source row
  const int r_hi = top ? g.split : g.rows;     // and its end
  const TS* sc = src + g.src_off + (int64_t)col * g.src_ld + r_lo + 8 * r;
  TS x[8];
  if (r_lo + 8 * r + 8 <= r_hi) {
    // a full group: 32 or 64 contiguous bytes, read as 16-byte vectors (the
    // element alignment suffices on this part)
    typedef TS tv __attribute__((ext_vector_type(16 / sizeof(TS)), aligned(sizeof(TS))));
    constexpr int NV = 8 * sizeof(TS) / 16, PV = 16 / sizeof(TS);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const tv y = *reinterpret_cast<const tv*>(sc + PV * v);
#pragma unroll
      for (int t = 0; t < PV; ++t) x[PV * v + t] = y[t];
    }
  } else {
#pragma unroll
    for (int t = 0; t < 8; ++t) x[t] = r_lo + 8 * r + t < r_hi ? sc[t] : TS(0);
  }
  unsigned short h[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const __bf16 b = (__bf16)(float)x[t];
    h[t] = __builtin_bit_cast(unsigned short, b);
  }
  uint4 v;
  v.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
  v.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
  v.z = (unsigned)h[4] | ((unsigned)h[5] << 16);
  v.w = (unsigned)h[6] | ((unsigned)h[7] << 16);
  unsigned short* dc = top ? dst + g.top + (int64_t)(col - g.c_top) * (8 * g.gt)
                           : dst + g.bot + (int64_t)col * (8 * g.gb);
  *reinterpret_cast<uint4*>(dc + 8 * r) = v;
}

hipError_t launch_cvt_bf16_blks(const void* src, int esz_src, const CvtBlk* blks,
                                const int* first, int count, int64_t groups,
                                unsigned short* dst, hipStream_t st) {
  if (count <= 0 || groups <= 0) return hipSuccess;
  if ((groups + 255) / 256 > INT_MAX) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((groups + 255) / 256);
  if (esz_src == 8)
    hipLaunchKernelGGL(cvt_bf16_blks_kernel<double>, dim3(grid), dim3(256), 0, st,
                       static_cast<const double*>(src), blks, first, count, groups, dst);
  else if (esz_src == 4)
    hipLaunchKernelGGL(cvt_bf16_blks_kernel<float>, dim3(grid), dim3(256), 0, st,
                       static_cast<const float*>(src), blks, first, count, groups, dst);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

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
// divided by alphas_den[c] if given, scaled by sgn; a zero numerator or
// denominator gives alpha = 0), all n x nrhs with their own leading dimensions.
__global__ void axpby_kernel(double* z, int64_t ldz, const double* x, int64_t ldx, const double* y,
                             int64_t ldy, int64_t n, int nrhs, const double* alphas,
                             const double* alphas_den, double sgn) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % n, c = e / n;
    double a = sgn;
    if (alphas) a *= alphas[c];
    // a column whose ratio has a zero numerator or denominator (a zero or
    // exactly converged right-hand side in CG) keeps its x, r and p
    if (alphas_den) a = (alphas_den[c] != 0.0 && a != 0.0) ? a / alphas_den[c] : 0.0;
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
