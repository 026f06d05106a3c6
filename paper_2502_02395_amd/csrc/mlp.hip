// Rank-predictor network 8 -> 64 -> 64 -> 1 (ReLU, FP32): inference,
// full-batch MSE gradient and Adam.  Not part of the paper: it predicts the
// rank of each box's interpolative decomposition from box geometry so that
// buffers can be sized before compression.  Gradients are reduced in a fixed
// order (per-block partials, then a serial sum per parameter), so training is
// bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "h2_ctx.hpp"

namespace h2 {

constexpr int NP = 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1;  // 4801
constexpr int OW1 = 0, OB1 = 512, OW2 = 576, OB2 = 4672, OW3 = 4736, OB3 = 4800;
constexpr int SPB = 64;  // samples per block in the gradient kernel

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ w,
                                                          const float* __restrict__ x,
                                                          float* __restrict__ y, int64_t n) {
  __shared__ float W[NP];
  for (int e = threadIdx.x; e < NP; e += 256) W[e] = w[e];
  __syncthreads();
  const int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (s >= n) return;
  float xi[8];
  for (int d = 0; d < 8; ++d) xi[d] = x[s * 8 + d];
  float h1[64];
  for (int a = 0; a < 64; ++a) {
    float z = W[OB1 + a];
    for (int d = 0; d < 8; ++d) z += W[OW1 + a * 8 + d] * xi[d];
    h1[a] = z > 0.f ? z : 0.f;
  }
  float out = W[OB3];
  for (int a = 0; a < 64; ++a) {
    float z = W[OB2 + a];
    for (int c = 0; c < 64; ++c) z += W[OW2 + a * 64 + c] * h1[c];
    out += W[OW3 + a] * (z > 0.f ? z : 0.f);
  }
  y[s] = out;
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ w,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ t, int64_t n,
                                                       float* __restrict__ ws,
                                                       float* __restrict__ wloss) {
  __shared__ float W[NP];
  __shared__ float X[SPB][8];
  __shared__ float H1[SPB][64];
  __shared__ float H2[SPB][64];
  __shared__ float dy[SPB];
  const int tid = threadIdx.x;
  const int64_t s0 = blockIdx.x * (int64_t)SPB;
  for (int e = tid; e < NP; e += 256) W[e] = w[e];
  for (int e = tid; e < SPB * 8; e += 256) {
    const int s = e / 8, d = e % 8;
    X[s][d] = (s0 + s < n) ? x[(s0 + s) * 8 + d] : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < SPB * 64; e += 256) {
    const int s = e / 64, a = e % 64;
    float z = W[OB1 + a];
    for (int d = 0; d < 8; ++d) z += W[OW1 + a * 8 + d] * X[s][d];
    H1[s][a] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < SPB * 64; e += 256) {
    const int s = e / 64, a = e % 64;
    float z = W[OB2 + a];
    for (int c = 0; c < 64; ++c) z += W[OW2 + a * 64 + c] * H1[s][c];
    H2[s][a] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  if (tid < SPB) {
    float yv = W[OB3];
    for (int a = 0; a < 64; ++a) yv += W[OW3 + a] * H2[tid][a];
    const bool valid = s0 + tid < n;
    dy[tid] = valid ? 2.f * (yv - t[s0 + tid]) / (float)n : 0.f;
  }
  __syncthreads();
  if (tid == 0) {
    float l = 0.f;
    for (int s = 0; s < SPB; ++s) {
      if (s0 + s >= n) break;
      float yv = W[OB3];
      for (int a = 0; a < 64; ++a) yv += W[OW3 + a] * H2[s][a];
      const float r = yv - t[s0 + s];
      l += r * r;
    }
    wloss[blockIdx.x] = l;
  }
  float* g = ws + (int64_t)blockIdx.x * NP;
  // W3, b3
  if (tid < 64) {
    float acc = 0.f;
    for (int s = 0; s < SPB; ++s) acc += dy[s] * H2[s][tid];
    g[OW3 + tid] = acc;
  }
  if (tid == 64) {
    float acc = 0.f;
    for (int s = 0; s < SPB; ++s) acc += dy[s];
    g[OB3] = acc;
  }
  __syncthreads();
  // dZ2 (overwrites H2)
  for (int e = tid; e < SPB * 64; e += 256) {
    const int s = e / 64, a = e % 64;
    H2[s][a] = (H2[s][a] > 0.f) ? dy[s] * W[OW3 + a] : 0.f;
  }
  __syncthreads();
  // W2, b2
  for (int e = tid; e < 64 * 64; e += 256) {
    const int a = e / 64, c = e % 64;
    float acc = 0.f;
    for (int s = 0; s < SPB; ++s) acc += H2[s][a] * H1[s][c];
    g[OW2 + e] = acc;
  }
  if (tid < 64) {
    float acc = 0.f;
    for (int s = 0; s < SPB; ++s) acc += H2[s][tid];
    g[OB2 + tid] = acc;
  }
  // dZ1 in registers, then over H1
  float dz[16];
  int q = 0;
  for (int e = tid; e < SPB * 64; e += 256, ++q) {
    const int s = e / 64, c = e % 64;
    float acc = 0.f;
    for (int a = 0; a < 64; ++a) acc += H2[s][a] * W[OW2 + a * 64 + c];
    dz[q] = (H1[s][c] > 0.f) ? acc : 0.f;
  }
  __syncthreads();
  q = 0;
  for (int e = tid; e < SPB * 64; e += 256, ++q) H1[e / 64][e % 64] = dz[q];
  __syncthreads();
  for (int e = tid; e < 64 * 8; e += 256) {
    const int c = e / 8, d = e % 8;
    float acc = 0.f;
    for (int s = 0; s < SPB; ++s) acc += H1[s][c] * X[s][d];
    g[OW1 + e] = acc;
  }
  if (tid < 64) {
    float acc = 0.f;
    for (int s = 0; s < SPB; ++s) acc += H1[s][tid];
    g[OB1 + tid] = acc;
  }
}

__global__ void mlp_reduce_kernel(const float* ws, const float* wloss, int nblk, int64_t n,
                                  float* g, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    float acc = 0.f;
    for (int b = 0; b < nblk; ++b) acc += ws[(int64_t)b * NP + p];
    g[p] = acc;
  }
  if (p == 0 && loss) {
    float l = 0.f;
    for (int b = 0; b < nblk; ++b) l += wloss[b];
    *loss = l / (float)n;
  }
}

__global__ void adam_kernel(float* w, float* m, float* v, const float* g, int np, float b1t,
                            float b2t, float lr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const float gp = g[p];
  const float mp = 0.9f * m[p] + 0.1f * gp;
  const float vp = 0.999f * v[p] + 0.001f * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / (1.f - b1t), vh = vp / (1.f - b2t);
  w[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

hipError_t launch_set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

// Features of box i at level l (instance t), in the order the predictor was
// trained on: level/L, log2(points), log(radius/ell), middle/largest and
// smallest/largest bounding-box side, near boxes (j != i), log2(1 + points of
// the boxes that are not near), -log10(eps).
void box_features_host(const Ctx& c, int t, int l, int i, float* f) {
  const Instance& in = c.ins[t];
  const Tree& tr = in.tree;
  const double sz = (double)(tr.start[l][i + 1] - tr.start[l][i]);
  double ext[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < tr.dim; ++a) ext[a] = tr.extent[l][(size_t)i * tr.dim + a];
  std::sort(ext, ext + 3);
  const double emax = ext[2] > 0 ? ext[2] : 1.0;
  const double ell = (in.kern.id >= 2) ? in.kern.ell : 1.0;
  int nnear = 0;
  double near_pts = 0.0;
  for (auto& pr : tr.near[l])
    if (pr.first == i) {
      ++nnear;
      near_pts += (double)(tr.start[l][pr.second + 1] - tr.start[l][pr.second]);
    }
  const double rad = std::max(tr.radius[l][i], 1e-300);
  f[0] = (float)((double)l / tr.L);
  f[1] = (float)std::log2(sz);
  f[2] = (float)std::log(rad / ell);
  f[3] = (float)(ext[1] / emax);
  f[4] = (float)(ext[0] / emax);
  f[5] = (float)(nnear - 1);
  f[6] = (float)std::log2(1.0 + (double)in.n - near_pts);
  f[7] = (float)(-std::log10(c.prm.eps > 0 ? c.prm.eps : 1e-300));
}

// One full-batch training step with the per-block partials in ws
// (nblk * NP + nblk floats; every entry is written before it is read).
static hipError_t mlp_train_launch(float* w, float* m, float* v, float* g, const float* x,
                                   const float* t, int64_t n, int32_t step, float lr, float* loss,
                                   float* ws, hipStream_t st) {
  const int nblk = (int)((n + SPB - 1) / SPB);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(256), 0, st, w, x, t, n, ws,
                     ws + (size_t)nblk * NP);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, ws,
                     ws + (size_t)nblk * NP, nblk, n, g, loss);
  const float b1t = std::pow(0.9f, (float)step), b2t = std::pow(0.999f, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, w, m, v, g, NP, b1t, b2t,
                     lr);
  return hipGetLastError();
}

}  // namespace h2

using namespace h2;

extern "C" {

h2_status h2_mlp_forward(const float* w, const float* x, float* y, int64_t n, void* stream) {
  if (!w || !x || !y || n < 0) return H2_ERR_ARG;
  if (n == 0) return H2_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, x,
                     y, n);
  return hipGetLastError() == hipSuccess ? H2_OK : H2_ERR_HIP;
}

h2_status h2_mlp_train_step(float* w, float* m, float* v, float* g, const float* x, const float* t,
                            int64_t n, int32_t step, float lr, float* loss, void* stream) {
  if (!w || !m || !v || !g || !x || !t || n < 1 || step < 1) return H2_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nblk = (int)((n + SPB - 1) / SPB);
  float* ws = nullptr;
  if (hipMalloc(&ws, sizeof(float) * ((size_t)nblk * NP + nblk)) != hipSuccess) return H2_ERR_ALLOC;
  const hipError_t e = mlp_train_launch(w, m, v, g, x, t, n, step, lr, loss, ws, st);
  const hipError_t s2 = hipStreamSynchronize(st);
  (void)hipFree(ws);
  return (e == hipSuccess && s2 == hipSuccess) ? H2_OK : H2_ERR_HIP;
}

h2_status h2_box_features(h2_handle h, float* feats, void* stream) {
  if (!h || !h->c || !feats) return H2_ERR_ARG;
  Ctx& c = *h->c;
  std::vector<float> f;
  for (auto& S : c.steps)
    for (int b = 0; b < S.nbox; ++b) {
      float v[8];
      box_features_host(c, S.inst[b], S.lvl[b], S.idx[b], v);
      f.insert(f.end(), v, v + 8);
    }
  if (f.empty()) return H2_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(feats, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
    return H2_ERR_HIP;
  return hipStreamSynchronize(st) == hipSuccess ? H2_OK : H2_ERR_HIP;
}

}  // extern "C"
