// Per-box dense factorizations, one 256-thread workgroup per box:
//   * qr_panel / qr_tbuild / qr_diag -- Householder QR of D_i U_i and the
//                     full square Q_i in compact WY form (basis completion,
//                     first step of each level of the ULV sweep; skeleton
//                     columns first);
//   * cpqr_id      -- column-pivoted Householder QR of M^T for the row
//                     interpolative decomposition of Algorithm 1, rank by the
//                     leading |R_jj| > eps |R_00|, then T = R_11^{-1} R_12;
//   * gauss_seidel -- sweeps that approximate the near-sample solve of the
//                     construction (one thread per right-hand-side column);
//   * panel        -- Cholesky and the inverse of its factor on the 64-wide
//                     diagonal panels of the blocked Cholesky factorizations
//                     (near-sample matrices, redundant blocks and the root;
//                     the rest of each, and the full inverse, are batched
//                     GEMMs).
// Householder vectors follow LAPACK's convention (beta = -sign(alpha)||x||,
// v_0 = 1, tau = (beta - alpha)/beta).
#include "h2_internal.hpp"

namespace h2 {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 256 threads; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// Householder reflector for x = col[j..n) (col has stride 1).  Overwrites
// col[j] with beta and col[j+1..n) with v (v_0 = 1 implicit); returns tau.
__device__ double householder(double* col, int j, int n, double* sh, double* beta_out) {
  double p = 0.0;
  for (int i = j + 1 + (int)threadIdx.x; i < n; i += 256) p += col[i] * col[i];
  const double sigma = block_sum(p, sh);
  const double alpha = col[j];
  double tau = 0.0, beta = alpha;
  if (sigma != 0.0) {
    beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
    tau = (beta - alpha) / beta;
    const double scal = 1.0 / (alpha - beta);
    for (int i = j + 1 + (int)threadIdx.x; i < n; i += 256) col[i] *= scal;
  }
  __syncthreads();
  if (threadIdx.x == 0) col[j] = beta;
  __syncthreads();
  *beta_out = beta;
  return tau;
}

// Apply H = I - tau v v^T (v in vcol[j..n), v_j = 1) to column c[j..n) with a
// single wave; returns nothing.  If norm_out != NULL, also returns the sum of
// squares of c[j+1..n) after the update (for pivoting).
__device__ __forceinline__ double apply_reflector_wave(const double* vcol, double* c, int j,
                                                       int n, double tau, bool want_norm) {
  const int lane = threadIdx.x & 63;
  double w = 0.0;
  for (int i = j + lane; i < n; i += 64) w += (i == j ? 1.0 : vcol[i]) * c[i];
  w = wave_sum(w) * tau;
  double s = 0.0;
  for (int i = j + lane; i < n; i += 64) {
    const double nv = c[i] - w * (i == j ? 1.0 : vcol[i]);
    c[i] = nv;
    if (want_norm && i > j) s += nv * nv;
  }
  return want_norm ? wave_sum(s) : 0.0;
}

// ------------------------------------------------------------------ QR + Q
// Householder QR of W = D_i U_i (m x k) and the full square Q_i in compact
// WY form, Q = H_0 H_1 ... H_{k-1} = I - V T V^T (V unit lower trapezoidal,
// T upper triangular):
//   qr_panel   -- one panel of a blocked right-looking factorization, one
//                 workgroup per box, the panel resident in LDS; writes V
//                 explicitly (tmpA), tau, R (Rf) and U_p = V_p T_p (tmpB);
//                 batched GEMMs apply the panel to the trailing columns;
//   qr_tdiag   -- T from G = V^T V (a batched GEMM writes G into P):
//                 T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j],
//                 on the diagonal 64-blocks; GEMMs fill the blocks above;
//   qr_diag    -- after the GEMMs Q = -V (T V^T): add the identity (k = 0
//                 boxes get Q = I outright).
constexpr int QR_PAN = 6912;  // LDS doubles of one panel (54 KiB: two workgroups per CU)
constexpr int QR_PW = 32;     // widest panel

// One panel of the blocked factorization, one workgroup per box with k > J:
// columns J .. J+w-1 of W (rows J .. m-1, already updated by the previous
// panels) are factored in LDS by unblocked Householder steps.  The kernel
// writes the panel's columns of V (explicitly, all m rows) into tmpA, its
// columns of R into Rf, its tau, and, when trailing columns remain,
// U_p = V_p T_p (rows J .. m-1, ld m) into tmpB, T_p being the panel's WY
// factor.  The trailing update W_t -= V_p (U_p^T W_t) is two batched GEMMs.
__global__ __launch_bounds__(256) void qr_panel_kernel(const BoxDev* __restrict__ boxes, int J,
                                                       int w) {
  __shared__ double pan[QR_PAN];
  __shared__ double Tp[QR_PW * QR_PW], Gp[QR_PW * QR_PW], Xp[QR_PW * QR_PW];
  __shared__ double taup[QR_PW], scalp[QR_PW], betap[QR_PW], wv[QR_PW];
  __shared__ double sh[4];
  const BoxDev b = boxes[blockIdx.x];
  const int m = b.m, k = b.k;
  if (m == 0 || k <= J) return;
  const int wj = min(w, k - J), L = m - J;
  // column stride of the panel in LDS: odd, so that threads reading the
  // same row of different columns hit different banks
  const int LP = L | 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* W = b.W;
  // (column loops over waves, row loops over lanes: no index divisions)
  for (int c = wave; c < wj; c += 4)
    for (int r = lane; r < L; r += 64) pan[c * LP + r] = W[J + r + (int64_t)(J + c) * m];
  __syncthreads();
  // Householder steps, thread-parallel, two barriers per column.  Column jj
  // stays unscaled while later columns are updated (v_r = pan[r, jj] * scal
  // for r > jj, v_jj = 1); its scaling and beta are applied at the end.  The
  // update of column jj+1 also accumulates the squared norm of its rows below
  // the diagonal, the sigma of the next step.
  {
    double part = 0.0;
    for (int r = 1 + threadIdx.x; r < L; r += 256) part += pan[r] * pan[r];
    part = wave_sum(part);
    if (lane == 0) sh[wave] = part;
    __syncthreads();
  }
  for (int jj = 0; jj < wj; ++jj) {
    const double sigma = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    const double alpha = pan[jj * LP + jj];
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (sigma != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const int nc = wj - jj - 1;
    if (nc > 0 && tau != 0.0) {
      // w_c = tau (pan[jj, c] + scal sum_{r > jj} pan[r, jj] pan[r, c]),
      // G threads per column (G a power of two dividing 64)
      int G = 64;
      while (G > 8 && G * nc > 256) G >>= 1;
      const int grp = threadIdx.x / G, sub = threadIdx.x % G;
      double acc = 0.0;
      if (grp < nc) {
        const double* vc = pan + jj * LP;
        const double* xc = pan + (jj + 1 + grp) * LP;
        for (int r = jj + 1 + sub; r < L; r += G) acc += vc[r] * xc[r];
      }
      for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (grp < nc && sub == 0) wv[grp] = tau * (pan[(jj + 1 + grp) * LP + jj] + scal * acc);
    }
    if (threadIdx.x == 0) {
      taup[jj] = tau;
      scalp[jj] = scal;
      betap[jj] = beta;
    }
    __syncthreads();
    double nxt = 0.0;
    if (nc > 0) {
      if (tau != 0.0) {
        for (int ci = wave; ci < nc; ci += 4) {
          const double wc = wv[ci];
          double* xc = pan + (jj + 1 + ci) * LP;
          for (int r = jj + lane; r < L; r += 64) {
            const double v = (r == jj) ? 1.0 : pan[jj * LP + r] * scal;
            const double x = xc[r] - v * wc;
            xc[r] = x;
            if (ci == 0 && r > jj + 1) nxt += x * x;
          }
        }
      } else {
        for (int r = jj + 2 + threadIdx.x; r < L; r += 256)
          nxt += pan[(jj + 1) * LP + r] * pan[(jj + 1) * LP + r];
      }
    }
    nxt = wave_sum(nxt);
    if (lane == 0) sh[wave] = nxt;
    __syncthreads();
  }
  for (int c = wave; c < wj; c += 4) {
    const double sc = scalp[c];
    for (int r = c + lane; r < L; r += 64) {
      if (r > c) pan[c * LP + r] *= sc;
      else pan[c * LP + r] = betap[c];
    }
  }
  __syncthreads();
  // R columns J..J+wj-1 (rows above the panel are final in W), tau
  for (int c = wave; c < wj; c += 4)
    for (int r = lane; r < k; r += 64) {
      double v = 0.0;
      if (r < J) v = W[r + (int64_t)(J + c) * m];
      else if (r <= J + c) v = pan[c * LP + (r - J)];
      b.Rf[r + (int64_t)(J + c) * k] = v;
    }
  if ((int)threadIdx.x < wj) b.tau[J + threadIdx.x] = taup[threadIdx.x];
  __syncthreads();
  // V explicit in the panel: zeros above the diagonal, ones on it
  for (int c = wave; c < wj; c += 4)
    for (int r = lane; r <= c; r += 64) pan[c * LP + r] = (r == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int c = wave; c < wj; c += 4)
    for (int r = lane; r < m; r += 64)
      b.tmpA[r + (int64_t)(J + c) * m] = (r < J) ? 0.0 : pan[c * LP + (r - J)];
  if (J + wj >= k) return;
  // T_p from G_p = V_p^T V_p by recursive doubling: for two adjacent blocks
  // of reflectors, T = [T1, -T1 (V1^T V2) T2; 0, T2].  G_p's strict upper
  // triangle (one thread per entry, rows from the later column's diagonal
  // down) goes to Gp; T_p starts as diag(tau).
  for (int pq = threadIdx.x; pq < wj * wj; pq += 256) {
    const int i = pq % wj, jj = pq / wj;
    double d = 0.0;
    if (i < jj)
      for (int r = jj; r < L; ++r) d += pan[i * LP + r] * pan[jj * LP + r];
    Gp[i + jj * QR_PW] = d;
    Tp[i + jj * QR_PW] = (i == jj) ? taup[i] : 0.0;
  }
  __syncthreads();
  for (int sz = 1; sz < wj; sz <<= 1) {
    // X = G12 T2 into Xp, then T12 = -T1 X, for every pair of blocks of size sz
    const int nblk = (wj + 2 * sz - 1) / (2 * sz);
    for (int e = threadIdx.x; e < nblk * sz * sz; e += 256) {
      const int o = (e / (sz * sz)) * 2 * sz, r = e % sz, c = (e / sz) % sz;
      const int c2 = o + sz + c;
      if (c2 < wj) {
        double acc = 0.0;
        for (int q = 0; q <= c; ++q) acc += Gp[o + r + (o + sz + q) * QR_PW] * Tp[o + sz + q + c2 * QR_PW];
        Xp[o + r + c2 * QR_PW] = acc;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nblk * sz * sz; e += 256) {
      const int o = (e / (sz * sz)) * 2 * sz, r = e % sz, c = (e / sz) % sz;
      const int c2 = o + sz + c;
      if (c2 < wj) {
        double acc = 0.0;
        for (int q = r; q < sz; ++q) acc += Tp[o + r + (o + q) * QR_PW] * Xp[o + q + c2 * QR_PW];
        Tp[o + r + c2 * QR_PW] = -acc;
      }
    }
    __syncthreads();
  }
  // U_p = V_p T_p, rows J..m-1 of tmpB (ld m)
  double* U = b.tmpB + J;
  for (int r = threadIdx.x; r < L; r += 256) {
    for (int c = 0; c < wj; ++c) {
      double acc = 0.0;
      for (int i = 0; i <= c; ++i) acc += pan[i * LP + r] * Tp[i + c * QR_PW];
      U[r + (int64_t)c * m] = acc;
    }
  }
}

// Diagonal 64-blocks of T, one workgroup per (box, block q): with G_qq the
// block of G = V^T V and tau the Householder scalars of its columns,
// T_qq[0:j, j] = -tau_j T_qq[0:j, 0:j] G_qq[0:j, j] and T_qq[j, j] = tau_j.
// T_qq overwrites G_qq; the rows below the block in its columns are zeroed.
// The blocks above the diagonal follow by GEMMs,
// T[0:q0, q] = -(T[0:q0, 0:q0] G[0:q0, q]) T_qq.
__global__ __launch_bounds__(256) void qr_tdiag_kernel(const BoxDev* __restrict__ boxes) {
  __shared__ double t[64 * 65];
  __shared__ double gcol[64];
  const BoxDev b = boxes[blockIdx.x];
  const int k = b.k, q0 = 64 * blockIdx.y;
  if (b.m == 0 || q0 >= k) return;
  const int w = min(64, k - q0);
  double* T = b.P + q0 + (int64_t)q0 * k;  // T_qq, ld k
  for (int e = threadIdx.x; e < w * w; e += 256) {
    const int i = e % w, j = e / w;
    t[i + 65 * j] = T[i + (int64_t)j * k];
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if ((int)threadIdx.x < j) gcol[threadIdx.x] = t[threadIdx.x + 65 * j];
    __syncthreads();
    const double tj = b.tau[q0 + j];
    for (int i = threadIdx.x; i < w; i += 256) {
      double v = (i == j) ? tj : 0.0;
      if (i < j) {
        double acc = 0.0;
        for (int q = i; q < j; ++q) acc += t[i + 65 * q] * gcol[q];
        v = -tj * acc;
      }
      t[i + 65 * j] = v;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < w * w; e += 256) {
    const int i = e % w, j = e / w;
    T[i + (int64_t)j * k] = t[i + 65 * j];
  }
  const int below = k - q0 - w;
  for (int e = threadIdx.x; e < below * w; e += 256) {
    const int i = e % below, j = e / below;
    T[w + i + (int64_t)j * k] = 0.0;
  }
}

__global__ __launch_bounds__(256) void qr_diag_kernel(const BoxDev* __restrict__ boxes) {
  const BoxDev b = boxes[blockIdx.x];
  const int m = b.m;
  if (b.k == 0) {
    for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += 256)
      b.Q[e] = (e % m == e / m) ? 1.0 : 0.0;
  } else {
    for (int i = threadIdx.x; i < m; i += 256) b.Q[i + (int64_t)i * m] += 1.0;
  }
}

// ---------------------------------------------------- register-resident panel
// The same panel with the panel in registers, owned by columns: TPC = 256 / W
// threads hold one column each, thread s of the group the rows s + TPC i
// (i < NR).  Householder step jj: the owners of column jj form the reflector
// (norm and alpha summed over their TPC lanes) and publish v through LDS
// (double-buffered, one barrier per step); every group then forms its
// column's product with v (a TPC-lane sum, no cross-column reduction), which
// is the update coefficient for later columns and, for earlier columns l, the
// z_l = V_l^T v_jj of the forward recurrence T[0:j, j] = -tau_j T[0:j, 0:j] z,
// T[j, j] = tau_j; the z are kept in LDS and T_p is formed after the steps,
// each of its rows by one thread (a row only needs its own earlier entries).
// U_p = V_p T_p goes through LDS in 64-row chunks.  Outputs as
// qr_panel_kernel: V explicit in tmpA, R, tau, U_p.

// Sum over aligned groups of TPC (8 or 16) lanes through DPP lane permutes
// within a row of 16 lanes: quad_perm [1,0,3,2] (xor 1), quad_perm [2,3,0,1]
// (xor 2), row_half_mirror (lane i of 8 <- lane 7 - i: the other quad's sum)
// and, for 16, row_mirror (lane i <- lane 15 - i: the other half's sum).
__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  switch (ctrl_sel) {
    case 0:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 1:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 2:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false);
      break;
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int TPC>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(TPC == 8 || TPC == 16, "lane group");
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  v += dpp_f64(v, 2);
  if constexpr (TPC == 16) v += dpp_f64(v, 3);
  return v;
}

template <int W, int NR>
__global__ __launch_bounds__(256, 2) void qr_panel_reg_kernel(const BoxDev* __restrict__ boxes,
                                                              int J, int w) {
  constexpr int TPC = 256 / W;
  constexpr int RMAX = TPC * NR;      // rows the kernel holds
  constexpr int CH = 64;              // rows per U_p chunk
  __shared__ double vbuf[2][RMAX];   // v, row s + TPC i at i TPC + s (no bank conflicts)
  __shared__ double Zs[W * W];        // z of step c in column c (rows l < c)
  __shared__ double Tp[W * W];        // T_p, column-major
  constexpr int VS = W + 1;          // odd row stride: no bank conflicts
  __shared__ double Vc[CH * VS];      // a chunk of V_p, row-major
  __shared__ double bet[W], tau_s[W];
  const BoxDev b = boxes[blockIdx.x];
  const int m = b.m, k = b.k;
  if (m == 0 || k <= J) return;
  const int wj = min(w, k - J), L = m - J;
  const int tid = threadIdx.x;
  const int col = tid / TPC, s = tid % TPC;
  const double* __restrict__ Wm = b.W;
  // rows s + TPC i of column col (clamped into the panel: rows past L and
  // columns past wj hold copies and are never used or written out)
  double a[NR];
  {
    const double* src = Wm + J + (int64_t)(J + min(col, wj - 1)) * m;
#pragma unroll
    for (int i = 0; i < NR; ++i) a[i] = src[min(s + TPC * i, L - 1)];
  }
  for (int jj = 0; jj < wj; ++jj) {
    const int bb = jj & 1;
    if (col == jj) {
      // four independent accumulators: the FP64 chains are a quarter as long
      double sg4[4] = {0.0, 0.0, 0.0, 0.0}, al = 0.0;
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int r = s + TPC * i;
        if (r > jj && r < L) sg4[i & 3] += a[i] * a[i];
        if (r == jj) al = a[i];
      }
      double sg = group_sum<TPC>((sg4[0] + sg4[1]) + (sg4[2] + sg4[3]));
      al = group_sum<TPC>(al);
      double tau = 0.0, beta = al, scal = 0.0;
      if (sg != 0.0) {
        beta = -copysign(sqrt(al * al + sg), al);
        tau = (beta - al) / beta;
        scal = 1.0 / (al - beta);
      }
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int r = s + TPC * i;
        const double v = (r == jj) ? 1.0 : ((r > jj && r < L) ? a[i] * scal : 0.0);
        vbuf[bb][i * TPC + s] = v;
        if (r > jj) a[i] = v;  // the column becomes V below the diagonal
      }
      if (s == 0) {
        tau_s[jj] = tau;
        bet[jj] = beta;
      }
    }
    __syncthreads();
    if (col != jj) {
      double v[NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) v[i] = vbuf[bb][i * TPC + s];
      double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < NR; ++i) p4[i & 3] += v[i] * a[i];
      const double p = group_sum<TPC>((p4[0] + p4[1]) + (p4[2] + p4[3]));
      if (col > jj) {
        const double wc = tau_s[jj] * p;
#pragma unroll
        for (int i = 0; i < NR; ++i) a[i] -= v[i] * wc;
      } else if (s == 0) {
        Zs[col + jj * W] = p;
      }
    }
  }
  __syncthreads();
  // T_p row tid: T[i][c] = -tau_c sum_{i <= l < c} T[i][l] z_l(c)
  if (tid < wj) {
    double trow[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < c; ++l) acc += (l >= tid) ? trow[l] * Zs[l + c * W] : 0.0;
      const double t = (tid < c) ? -tau_s[c] * acc : (tid == c ? tau_s[c] : 0.0);
      trow[c] = t;
      if (c < wj) Tp[tid + c * W] = t;
    }
  }
  // R column J + col (every row of R: it is used as a full k x k matrix),
  // V explicit in tmpA, tau
  if (col < wj) {
    double* Rc = b.Rf + (int64_t)(J + col) * k;
    for (int r = s; r < J; r += TPC) Rc[r] = Wm[r + (int64_t)(J + col) * m];
    double* V = b.tmpA + (int64_t)(J + col) * m;
    for (int r = s; r < J; r += TPC) V[r] = 0.0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int r = s + TPC * i;
      if (r < k - J) Rc[J + r] = (r < col) ? a[i] : (r == col ? bet[col] : 0.0);
      if (r < L) V[J + r] = (r < col) ? 0.0 : (r == col ? 1.0 : a[i]);
    }
    if (s == 0) b.tau[J + col] = tau_s[col];
  }
  if (J + wj >= k) return;
  __syncthreads();  // T_p complete
  // U_p = V_p T_p, rows J .. m-1 of tmpB (ld m), in chunks of CH rows
  for (int r0 = 0; r0 < L; r0 += CH) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int r = s + TPC * i;
      if (r >= r0 && r < r0 + CH)
        Vc[(r - r0) * VS + col] = (r < col) ? 0.0 : (r == col ? 1.0 : a[i]);
    }
    __syncthreads();
    if (col < wj) {
      double tc[W];
#pragma unroll
      for (int l = 0; l < W; ++l) tc[l] = (l <= col) ? Tp[l + col * W] : 0.0;
      for (int rr = s; rr < CH && r0 + rr < L; rr += TPC) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < W; ++l) acc += Vc[rr * VS + l] * tc[l];
        b.tmpB[J + r0 + rr + (int64_t)col * m] = acc;
      }
    }
    __syncthreads();
  }
}

// Panel width of a level: the register kernel's 32 columns up to 256 rows, 16
// up to 768 rows (the panel held in at most 96 registers per thread); beyond,
// the LDS kernel's (its panel must fit in LDS).
int qr_panel_width(int max_m) {
  if (max_m <= 0) return QR_PW;
  if (max_m <= 256) return 32;
  if (max_m <= 768) return 16;
  return std::max(1, std::min(QR_PW, QR_PAN / (max_m + 1)));  // + 1: odd column stride
}

hipError_t launch_qr_panel(const BoxDev* boxes, int nbox, int max_m, int J, int w,
                           hipStream_t st) {
  if (nbox <= 0) return hipSuccess;
  if (max_m <= 256 && w <= 32)
    hipLaunchKernelGGL((qr_panel_reg_kernel<32, 32>), dim3(nbox), dim3(256), 0, st, boxes, J, w);
  else if (max_m <= 512 && w <= 16)
    hipLaunchKernelGGL((qr_panel_reg_kernel<16, 32>), dim3(nbox), dim3(256), 0, st, boxes, J, w);
  else if (max_m <= 768 && w <= 16)
    hipLaunchKernelGGL((qr_panel_reg_kernel<16, 48>), dim3(nbox), dim3(256), 0, st, boxes, J, w);
  else if (w >= 1 && w <= QR_PW && (int64_t)(max_m + 1) * w <= QR_PAN)
    hipLaunchKernelGGL(qr_panel_kernel, dim3(nbox), dim3(256), 0, st, boxes, J, w);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_qr_tdiag(const BoxDev* boxes, int nbox, int max_k, hipStream_t st) {
  if (nbox <= 0 || max_k <= 0) return hipSuccess;
  hipLaunchKernelGGL(qr_tdiag_kernel, dim3(nbox, (max_k + 63) / 64), dim3(256), 0, st, boxes);
  return hipGetLastError();
}

hipError_t launch_qr_diag(const BoxDev* boxes, int nbox, hipStream_t st) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(qr_diag_kernel, dim3(nbox), dim3(256), 0, st, boxes);
  return hipGetLastError();
}

// ------------------------------------------------------------- pivoted QR ID
constexpr int ID_MMAX = 4096;  // largest m: the column norms and pivots live in LDS

// U (m x k, ld m) from T = R_11^{-1} R_12 stored in rows 0..k-1 of columns
// k..m-1 of X (ld s) and the pivot order piv (LDS or global).
__device__ void write_u(const double* X, int s, int m, int k, const int* piv, double* U) {
  const int nr = m - k;
  for (int64_t e = threadIdx.x; e < (int64_t)m * k; e += 256) U[e] = 0.0;
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += 256) U[piv[t] + (int64_t)t * m] = 1.0;
  for (int64_t e = threadIdx.x; e < (int64_t)nr * k; e += 256) {
    const int q = (int)(e % nr), t = (int)(e / nr);
    U[piv[k + q] + (int64_t)t * m] = X[t + (int64_t)(k + q) * s];
  }
}

__global__ __launch_bounds__(256) void cpqr_id_kernel(const IdDesc* __restrict__ descs, double eps,
                                                      int max_rank, int id_m_lds) {
  // column norms and pivot order, sized by the launch to the level's largest
  // m (12 bytes per column), so that small boxes keep many workgroups per CU
  extern __shared__ double id_lds[];
  __shared__ double sh[4];
  __shared__ double bestv[4];
  __shared__ int besti[4];
  __shared__ int kfinal;
  const IdDesc d = descs[blockIdx.x];
  const int s = d.s, m = d.m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* X = d.X;
  const bool forced = d.skel != nullptr;
  double* norms = id_lds;
  int* piv = reinterpret_cast<int*>(id_lds + id_m_lds);

  for (int c = threadIdx.x; c < m; c += 256) piv[c] = c;
  for (int c = wave; c < m; c += 4) {
    double p = 0.0;
    for (int i = lane; i < s; i += 64) p += X[i + (int64_t)c * s] * X[i + (int64_t)c * s];
    p = wave_sum(p);
    if (lane == 0) norms[c] = p;
  }
  int kmax = s < m ? s : m;
  if (max_rank > 0 && max_rank < kmax) kmax = max_rank;
  if (forced) kmax = d.kforced;
  if (threadIdx.x == 0) kfinal = kmax;
  __syncthreads();

  double r00 = 0.0;
  for (int j = 0; j < kmax; ++j) {
    // ---- choose the pivot column
    int p = -1;
    if (forced) {
      if (threadIdx.x == 0) besti[0] = -1;
      __syncthreads();
      const int want = d.skel[j];
      for (int c = j + threadIdx.x; c < m; c += 256)
        if (piv[c] == want) besti[0] = c;
      __syncthreads();
      p = besti[0];
      if (p < 0) p = j;  // invalid input: keep order (host validates)
    } else {
      double bv = -1.0;
      int bi = m;
      for (int c = j + threadIdx.x; c < m; c += 256) {
        const double v = norms[c];
        if (v > bv || (v == bv && c < bi)) { bv = v; bi = c; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (lane == 0) { bestv[wave] = bv; besti[wave] = bi; }
      __syncthreads();
      bv = bestv[0]; bi = besti[0];
      for (int w = 1; w < 4; ++w)
        if (bestv[w] > bv || (bestv[w] == bv && besti[w] < bi)) { bv = bestv[w]; bi = besti[w]; }
      p = bi;
      __syncthreads();
    }
    if (p != j) {
      for (int i = threadIdx.x; i < s; i += 256) {
        const double t = X[i + (int64_t)j * s];
        X[i + (int64_t)j * s] = X[i + (int64_t)p * s];
        X[i + (int64_t)p * s] = t;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const double tn = norms[j]; norms[j] = norms[p]; norms[p] = tn;
        const int ti = piv[j]; piv[j] = piv[p]; piv[p] = ti;
      }
      __syncthreads();
    }
    // ---- reflector on column j
    double beta;
    const double tau = householder(X + (int64_t)j * s, j, s, sh, &beta);
    if (j == 0) {
      r00 = fabs(beta);
      if (r00 == 0.0) { if (threadIdx.x == 0) kfinal = 0; break; }
    }
    if (!forced && !(fabs(beta) > eps * r00)) {
      if (threadIdx.x == 0) kfinal = j;
      break;
    }
    for (int c = j + 1 + wave; c < m; c += 4) {
      const double nn = (tau != 0.0)
          ? apply_reflector_wave(X + (int64_t)j * s, X + (int64_t)c * s, j, s, tau, true)
          : 0.0;
      if (tau == 0.0) {
        double q = 0.0;
        for (int i = j + 1 + lane; i < s; i += 64) q += X[i + (int64_t)c * s] * X[i + (int64_t)c * s];
        q = wave_sum(q);
        if (lane == 0) norms[c] = q;
      } else if (lane == 0) {
        norms[c] = nn;
      }
    }
    __syncthreads();
  }
  __syncthreads();
  const int k = kfinal;
  const int nr = m - k;
  // ---- T = R11^{-1} R12, in place in rows 0..k-1 of columns k..m-1
  for (int t = k - 1; t >= 0; --t) {
    const double rtt = X[t + (int64_t)t * s];
    for (int c = threadIdx.x; c < nr; c += 256) X[t + (int64_t)(k + c) * s] /= rtt;
    __syncthreads();
    for (int e = threadIdx.x; e < t * nr; e += 256) {
      const int q = e % t, c = e / t;
      X[q + (int64_t)(k + c) * s] -= X[q + (int64_t)t * s] * X[t + (int64_t)(k + c) * s];
    }
    __syncthreads();
  }
  // ---- U (m x k, ld m) if it fits the caller's capacity; otherwise the
  // caller writes it later from X and piv (id_write_u_kernel)
  for (int c = threadIdx.x; c < m; c += 256) d.piv[c] = piv[c];
  if (threadIdx.x == 0) *d.k_out = k;
  if (d.kcap <= 0 || k <= d.kcap) write_u(X, s, m, k, piv, d.U);
}

// U = identity rows at the skeleton, T^T elsewhere, from a finished ID.
__global__ __launch_bounds__(256) void id_write_u_kernel(const IdDesc* __restrict__ descs) {
  const IdDesc d = descs[blockIdx.x];
  write_u(d.X, d.s, d.m, *d.k_out, d.piv, d.U);
}

hipError_t launch_id_write_u(const IdDesc* d_desc, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(id_write_u_kernel, dim3(count), dim3(256), 0, st, d_desc);
  return hipGetLastError();
}

hipError_t launch_cpqr_id(const IdDesc* d_desc, int count, double eps, int max_rank, int max_m,
                          hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (max_m < 1 || max_m > ID_MMAX) return hipErrorInvalidValue;
  const size_t lds = (size_t)max_m * (sizeof(double) + sizeof(int));
  hipLaunchKernelGGL(cpqr_id_kernel, dim3(count), dim3(256), lds, st, d_desc, eps, max_rank, max_m);
  return hipGetLastError();
}

// ------------------------------------------------------------ Gauss-Seidel
// Gauss-Seidel sweeps: the columns of X are independent, so each thread owns
// its columns and walks the rows in order (no barriers).  Row i of A is read
// as column i (A symmetric), the same address for every thread.
__global__ __launch_bounds__(256) void gauss_seidel_kernel(const GsDesc* __restrict__ descs,
                                                           int sweeps, int* fail) {
  const GsDesc d = descs[blockIdx.x];
  const int64_t m = d.m;
  for (int c = threadIdx.x; c < d.m; c += 256) {
    double* w = d.W + c;  // w[j * m]: row j of the iterate
    const double* b = d.B + (int64_t)c * d.ldb;
    for (int i = 0; i < d.n; ++i) w[i * m] = 0.0;
    for (int s = 0; s < sweeps; ++s)
      for (int i = 0; i < d.n; ++i) {
        const double* ai = d.A + (int64_t)i * d.lda;
        // four partial sums (independent loads in flight); the diagonal term
        // is added back instead of skipped
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
        int j = 0;
        for (; j + 4 <= d.n; j += 4) {
          p0 += ai[j] * w[j * m];
          p1 += ai[j + 1] * w[(j + 1) * m];
          p2 += ai[j + 2] * w[(j + 2) * m];
          p3 += ai[j + 3] * w[(j + 3) * m];
        }
        for (; j < d.n; ++j) p0 += ai[j] * w[j * m];
        const double aii = ai[i];
        const double acc = b[i] - ((p0 + p1) + (p2 + p3) - aii * w[i * m]);
        if (!(aii > 0.0)) {
          atomicMin(fail, d.code);
          w[i * m] = 0.0;
        } else {
          w[i * m] = acc / aii;
        }
      }
    double* x = d.X + (int64_t)c * d.ldx;
    for (int i = 0; i < d.n; ++i) x[i] = w[i * m];
  }
}

hipError_t launch_gauss_seidel(const GsDesc* d_desc, int count, int sweeps, int* fail,
                               hipStream_t st) {
  if (count <= 0 || sweeps <= 0) return hipSuccess;
  hipLaunchKernelGGL(gauss_seidel_kernel, dim3(count), dim3(256), 0, st, d_desc, sweeps, fail);
  return hipGetLastError();
}

// ------------------------------------------------------------- 64-wide panels
// Cholesky of an nb x nb diagonal block (nb <= 64) and the inverse of its
// factor, all in LDS.  The block is padded to 64 x 64 with the identity (the
// factor and its inverse are then the identity there too).  Cholesky:
// right-looking, one barrier per column (every thread reads the pivot; column
// j is scaled after the barrier, when step j+1 no longer reads it).  Inverse:
// block recursion X = [X11, 0; -X22 L21 X11, X22] from the 16 x 16 diagonal
// blocks (forward substitution, one thread per column) to 32 and 64.
constexpr int PLD = 65;  // LDS leading dimension (odd: column walks are conflict-free)

// X21 = -X22 (L21 X11) for the two diagonal blocks of size 2h starting at
// rows/columns o = 0 and 2h (h = 16), or the one of size 64 (h = 32).
template <int H>
__device__ __forceinline__ void panel_inv_merge(const double* __restrict__ a, double* __restrict__ x,
                                                double* __restrict__ t) {
  constexpr int NBLK = 64 / (2 * H);
  // T = L21 X11  (H x H per block; X11 lower triangular)
  for (int e = threadIdx.x; e < NBLK * H * H; e += 256) {
    const int blk = e / (H * H), r = e % H, c = (e / H) % H;
    const int o = blk * 2 * H;
    double s = 0.0;
    for (int q = c; q < H; ++q) s += a[(o + H + r) + (o + q) * PLD] * x[(o + q) + (o + c) * PLD];
    t[r + c * H + blk * H * H] = s;
  }
  __syncthreads();
  // X21 = -X22 T  (X22 lower triangular)
  for (int e = threadIdx.x; e < NBLK * H * H; e += 256) {
    const int blk = e / (H * H), r = e % H, c = (e / H) % H;
    const int o = blk * 2 * H;
    double s = 0.0;
    for (int q = 0; q <= r; ++q) s += x[(o + H + r) + (o + H + q) * PLD] * t[q + c * H + blk * H * H];
    x[(o + H + r) + (o + c) * PLD] = -s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void panel_kernel(const PanelDesc* __restrict__ descs, int* fail) {
  __shared__ double a[64 * PLD];
  __shared__ double x[64 * PLD];
  __shared__ double t[32 * 32];
  const PanelDesc d = descs[blockIdx.x];
  const int n = d.nb;
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    a[r + c * PLD] = (r < n && c < n) ? d.A[r + (int64_t)c * d.lda] : (r == c ? 1.0 : 0.0);
    x[r + c * PLD] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < 64; ++j) {
    double djj = a[j + j * PLD];
    if (!(djj > 0.0)) {
      if (tid == 0) atomicMin(fail, d.code);
      djj = 1.0;
    }
    const double rd = 1.0 / djj;
    // a[i, c] -= a[i, j] a[c, j] / a[j, j] for j < c <= i (unscaled column j)
    for (int c = j + 1 + wave; c < 64; c += 4) {
      const double acj = a[c + j * PLD] * rd;
      for (int i = c + lane; i < 64; i += 64) a[i + c * PLD] -= a[i + j * PLD] * acj;
    }
    __syncthreads();
    if (tid >= j && tid < 64) {
      const double sj = sqrt(djj);
      a[tid + j * PLD] = tid == j ? sj : a[tid + j * PLD] / sj;
    }
  }
  __syncthreads();
  // diagonal 16 x 16 blocks of the inverse: thread = column, forward substitution
  if (tid < 64) {
    const int o = tid & ~15, j = tid;
    for (int i = o; i < o + 16; ++i) {
      double s = i == j ? 1.0 : 0.0;
      for (int q = o; q < i; ++q) s -= a[i + q * PLD] * x[q + j * PLD];
      x[i + j * PLD] = s / a[i + i * PLD];
    }
  }
  __syncthreads();
  panel_inv_merge<16>(a, x, t);
  panel_inv_merge<32>(a, x, t);
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, c = e / n;
    d.A[r + (int64_t)c * d.lda] = r >= c ? a[r + c * PLD] : 0.0;
    d.dinv[r + (int64_t)c * d.ldd] = x[r + c * PLD];
  }
}

hipError_t launch_panel(const PanelDesc* d, int count, int* fail, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(panel_kernel, dim3(count), dim3(256), 0, st, d, fail);
  return hipGetLastError();
}

// Inverse of the lower triangle of a (unit diagonal if UNIT) into x, which
// must hold zeros: 16 x 16 diagonal blocks by forward substitution (thread =
// column), then the block recursion of panel_inv_merge.
template <bool UNIT>
__device__ __forceinline__ void panel_inv_lower(const double* __restrict__ a, double* __restrict__ x,
                                                double* __restrict__ t) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int o = tid & ~15, j = tid;
    for (int i = o; i < o + 16; ++i) {
      double s = i == j ? 1.0 : 0.0;
      for (int q = o; q < i; ++q) s -= a[i + q * PLD] * x[q + j * PLD];
      x[i + j * PLD] = UNIT ? s : s / a[i + i * PLD];
    }
  }
  __syncthreads();
  panel_inv_merge<16>(a, x, t);
  panel_inv_merge<32>(a, x, t);
}

// Pivot-free LU of an nb x nb diagonal block (nb <= 64), padded to 64 x 64
// with the identity: right-looking, one barrier per column (the update of
// step j uses the unscaled column j and the pivot's reciprocal; column j is
// scaled after the barrier, when no later step reads it).  A zero or
// non-finite pivot writes the job's code to fail and continues with 1.  Then
// L^{-1} (unit lower) and U^{-1}: the latter as the transpose of the inverse
// of U^T, formed in the lower triangle of a after L has been written out.
__global__ __launch_bounds__(256) void lu_panel_kernel(const PanelDesc* __restrict__ descs,
                                                       int* fail) {
  __shared__ double a[64 * PLD];
  __shared__ double x[64 * PLD];
  __shared__ double t[32 * 32];
  const PanelDesc d = descs[blockIdx.x];
  const int n = d.nb;
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    a[r + c * PLD] = (r < n && c < n) ? d.A[r + (int64_t)c * d.lda] : (r == c ? 1.0 : 0.0);
    x[r + c * PLD] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < 64; ++j) {
    double p = a[j + j * PLD];
    if (!(fabs(p) > 0.0) || !isfinite(p)) {
      if (tid == 0) atomicMin(fail, d.code);
      p = 1.0;
    }
    const double rp = 1.0 / p;
    // a[i, c] -= a[i, j] (a[j, c] / p) for i, c > j
    for (int c = j + 1 + wave; c < 64; c += 4) {
      const double ujc = a[j + c * PLD] * rp;
      const int i = j + 1 + lane;
      if (i < 64) a[i + c * PLD] -= a[i + j * PLD] * ujc;
    }
    __syncthreads();
    if (tid > j && tid < 64) a[tid + j * PLD] *= rp;
  }
  __syncthreads();
  // L and U back in place
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, c = e / n;
    d.A[r + (int64_t)c * d.lda] = a[r + c * PLD];
  }
  panel_inv_lower<true>(a, x, t);
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, c = e / n;
    d.dinv[r + (int64_t)c * d.ldd] = x[r + c * PLD];
  }
  __syncthreads();
  // lower triangle of a <- U^T (diagonal kept), x <- 0
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    if (r > c) a[r + c * PLD] = a[c + r * PLD];
    x[r + c * PLD] = 0.0;
  }
  __syncthreads();
  panel_inv_lower<false>(a, x, t);
  // U^{-1} = ((U^T)^{-1})^T
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, c = e / n;
    d.uinv[r + (int64_t)c * d.ldu] = x[c + r * PLD];
  }
}

hipError_t launch_lu_panel(const PanelDesc* d, int count, int* fail, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(lu_panel_kernel, dim3(count), dim3(256), 0, st, d, fail);
  return hipGetLastError();
}

}  // namespace h2
