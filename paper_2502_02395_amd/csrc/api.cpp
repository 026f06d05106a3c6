// The extern "C" entry points declared in include/h2.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "h2_ctx.hpp"

namespace h2 {
h2_status build_impl(int n_inst, const double* const* pts, const int64_t* ns,
                     const h2_kernel* kerns, const h2_params* prm, const int64_t* const* perms,
                     const int32_t* fixed_ranks, const int32_t* fixed_skel, hipStream_t st,
                     h2_handle* out);
}  // namespace h2

using namespace h2;

#define HIPCHK(x)                                  \
  do {                                             \
    if ((x) != hipSuccess) return H2_ERR_HIP;      \
  } while (0)

static hipStream_t S(void* p) { return static_cast<hipStream_t>(p); }

static double geqrf(double m, double k) { return 2.0 * m * k * k - 2.0 / 3.0 * k * k * k; }
static double orgqr_full(double m, double k) {
  return 4.0 * m * m * k - 4.0 * m * k * k + 4.0 / 3.0 * k * k * k;
}

// The LU variant's counts for one step: per box the same QR and diagonal
// transform, the LU of the redundant block 2 r^3/3, L(s)_ii and U(s)_ii
// (k r^2 each), the Schur update 2 k^2 r and both bases (m r^2 each); per
// ordered near pair i != j the transform 2 m_i m_j (m_i + m_j), L(s)_ij
// (k_i r_j^2), U(s)_ij (r_i^2 k_j) and L(r)_ij (r_i r_j^2, i > j) or U(r)_ij
// (r_i^2 r_j, i < j); per ordered far pair k_i k_j (k_i + k_j).  A solve
// takes the same per-block products as the symmetric path.  Pair counts are
// reported unordered, dense leaf blocks ordered.
static void count_flops_lu(Ctx& c, const Step& S, double& ff, double& fs, double& bytes,
                           int64_t& npairs, int64_t& nfar, int64_t& nnzb, int& maxk, int& maxm) {
  double* ph = c.st.flops_factor_phase;
  for (int b = 0; b < S.nbox; ++b) {
    const double m = S.m[b], k = S.k[b], r = m - k;
    const double qr = geqrf(m, k) + orgqr_full(m, k), lu = 2.0 * r * r * r / 3.0;
    const double vs = 2.0 * k * r * r + 2.0 * k * k * r + 2.0 * m * r * r;
    ff += qr + 4.0 * m * m * m + lu + vs;
    ph[0] += qr;
    ph[1] += 4.0 * m * m * m;
    ph[2] += lu;
    ph[3] += vs;
    c.st.flops_schur += 2.0 * k * k * r;
    fs += 4.0 * m * m + 4.0 * r * r;
    maxk = std::max(maxk, S.k[b]);
    maxm = std::max(maxm, S.m[b]);
    bytes += 16.0 * m * m;  // P and P'
  }
  for (size_t p = 0; p < S.np_i.size(); ++p) {
    const int i = S.np_i[p], j = S.np_j[p];
    const double mi = S.m[i], mj = S.m[j], ki = S.k[i], kj = S.k[j], ri = mi - ki, rj = mj - kj;
    bytes += 8.0 * mi * mj;
    if (S.h == 0) ++nnzb;
    if (i >= j) ++npairs;
    if (i == j) {
      fs += 4.0 * ki * ri;
      continue;
    }
    const double t = 2.0 * mi * mj * (mi + mj);
    const double tri = ki * rj * rj + ri * ri * kj + (i > j ? ri * rj * rj : ri * ri * rj);
    ff += t + tri;
    ph[4] += t + tri;
    c.st.flops_pair_gemm += t;
    fs += 2.0 * ki * rj + 2.0 * ri * kj + 2.0 * ri * rj;
  }
  for (size_t f = 0; f < S.fp_i.size(); ++f) {
    const double ki = S.k[S.fp_i[f]], kj = S.k[S.fp_j[f]];
    ff += ki * kj * (ki + kj);
    ph[5] += ki * kj * (ki + kj);
    if (S.fp_i[f] > S.fp_j[f]) ++nfar;
  }
}

// Canonical algorithmic flop counts (unpadded sizes); see include/h2.h.
static void count_flops(Ctx& c) {
  double ff = 0.0, fs = 0.0, bytes = 0.0;
  double* ph = c.st.flops_factor_phase;
  for (int q = 0; q < 9; ++q) ph[q] = 0.0;
  c.st.flops_schur = 0.0;
  int64_t nboxes = 0, npairs = 0, nfar = 0, nnzb = 0;
  int maxk = 0, maxm = 0;
  c.st.flops_pair_gemm = 0.0;
  c.st.pair_launches = 0;
  for (auto& S : c.steps) {
    if (S.g_pair1.count > 0) c.st.pair_launches += 2;
    nboxes += S.nbox;
    if (c.lu) {
      count_flops_lu(c, S, ff, fs, bytes, npairs, nfar, nnzb, maxk, maxm);
      continue;
    }
    for (int b = 0; b < S.nbox; ++b) {
      const double m = S.m[b], k = S.k[b], r = m - k;
      ff += geqrf(m, k) + orgqr_full(m, k) + 4.0 * m * m * m;
      ff += r * r * r / 3.0 + k * r * r + k * k * r + m * r * r;
      ph[0] += geqrf(m, k) + orgqr_full(m, k);
      ph[1] += 4.0 * m * m * m;
      ph[2] += r * r * r / 3.0;
      ph[3] += k * r * r + k * k * r + m * r * r;
      c.st.flops_schur += k * k * r;
      fs += 4.0 * m * m + 4.0 * r * r;
      maxk = std::max(maxk, S.k[b]);
      maxm = std::max(maxm, S.m[b]);
      bytes += 8.0 * m * m;  // P
    }
    for (size_t p = 0; p < S.np_i.size(); ++p) {
      const int i = S.np_i[p], j = S.np_j[p];
      const double mi = S.m[i], mj = S.m[j], ki = S.k[i], kj = S.k[j], ri = mi - ki, rj = mj - kj;
      bytes += 8.0 * mi * mj;
      ++npairs;
      if (i == j) {
        fs += 4.0 * ki * ri;
        if (S.h == 0) ++nnzb;
        continue;
      }
      if (S.h == 0) nnzb += 2;
      ff += ki * rj * rj + kj * ri * ri;
      ff += 2.0 * mi * mj * (mi + mj) + ri * rj * rj;
      ph[4] += ki * rj * rj + kj * ri * ri + 2.0 * mi * mj * (mi + mj) + ri * rj * rj;
      c.st.flops_pair_gemm += 2.0 * mi * mj * (mi + mj);
      fs += 4.0 * ki * rj + 4.0 * kj * ri + 4.0 * ri * rj;
    }
    for (size_t f = 0; f < S.fp_i.size(); ++f) {
      const double ki = S.k[S.fp_i[f]], kj = S.k[S.fp_j[f]];
      ff += ki * kj * (ki + kj);
      ph[5] += ki * kj * (ki + kj);
      ++nfar;
    }
  }
  for (auto& in : c.ins) {
    const double rc = (c.lu ? 2.0 : 1.0) * (double)in.n0 * in.n0 * in.n0 / 3.0;  // LU / Cholesky
    ff += rc;
    ph[7] += rc;
    fs += 2.0 * (double)in.n0 * in.n0;
    bytes += 8.0 * (double)in.n0 * in.n0;
    if (in.tree.L == 0) ++nnzb;
  }
  c.st.n = c.N;
  c.st.n_inst = c.n_inst;
  c.st.levels = c.H;
  c.st.n_boxes = nboxes;
  c.st.near_pairs = npairs;
  c.st.far_pairs = nfar;
  c.st.leaf_near_blocks = nnzb;
  c.st.max_rank_seen = maxk;
  c.st.max_m_seen = maxm;
  c.st.root_n = c.ins.empty() ? 0 : c.ins[0].n0;
  c.st.flops_factor = ff;
  c.st.flops_solve = fs;
  c.st.bytes_factors = bytes;
  c.st.gather_partials = c.part_len;
}

// ------------------------------------------------- no-allocation solve
// The gather partials of h2_solve_noalloc live in this fixed array instead of
// the handle's lazily grown buffer: every GPU the library runs on holds one
// copy (H2_NOALLOC_PARTIALS doubles, 64 MiB) until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current.  No slot needs clearing between calls: every slot a reduction reads
// is written by its chunk earlier in the same gather.
static __device__ __align__(256) double scratch[H2_NOALLOC_PARTIALS];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[64] = {};

static h2_status noalloc_partials(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return H2_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return H2_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return H2_OK;
}

extern "C" {

const char* h2_status_str(h2_status s) {
  switch (s) {
    case H2_OK: return "ok";
    case H2_ERR_ARG: return "invalid argument";
    case H2_ERR_ALLOC: return "allocation failed";
    case H2_ERR_HIP: return "HIP runtime error";
    case H2_ERR_NOT_SPD: return "Cholesky breakdown (matrix not positive definite)";
    case H2_ERR_STATE: return "call out of order";
    case H2_ERR_NOCONV: return "refinement did not converge";
    case H2_ERR_UNSUPPORTED: return "unsupported size or option";
  }
  return "unknown status";
}

h2_status h2_build(const double* pts, int64_t n, const h2_kernel* kernel, const h2_params* params,
                   const int64_t* perm, void* stream, h2_handle* out) {
  const double* p[1] = {pts};
  const int64_t* q[1] = {perm};
  h2_status s = build_impl(1, p, &n, kernel, params, q, nullptr, nullptr, S(stream), out);
  if (s == H2_OK) count_flops(*(*out)->c);
  return s;
}

h2_status h2_build_batched(int32_t n_inst, const double* const* pts, const int64_t* n,
                           const h2_kernel* kernels, const h2_params* params,
                           const int64_t* const* perms, void* stream, h2_handle* out) {
  h2_status s = build_impl(n_inst, pts, n, kernels, params, perms, nullptr, nullptr, S(stream), out);
  if (s == H2_OK) count_flops(*(*out)->c);
  return s;
}

h2_status h2_build_fixed(const double* pts, int64_t n, const h2_kernel* kernel,
                         const h2_params* params, const int64_t* perm, const int32_t* ranks,
                         const int32_t* skel, void* stream, h2_handle* out) {
  if (!ranks || !skel) return H2_ERR_ARG;
  const double* p[1] = {pts};
  const int64_t* q[1] = {perm};
  h2_status s = build_impl(1, p, &n, kernel, params, q, ranks, skel, S(stream), out);
  if (s == H2_OK) count_flops(*(*out)->c);
  return s;
}

static h2_status ensure_graph_stream(Ctx& c);

h2_status h2_factor(h2_handle h, void* stream) {
  if (!h || !h->c) return H2_ERR_ARG;
  Ctx& c = *h->c;
  if (c.failed) return H2_ERR_STATE;
  hipStream_t st = S(stream);
  const double t0 = now_seconds();
  if (c.prm.use_graph) {
    // The caller's stream may be the null stream, which cannot be captured:
    // capture and replay on a stream of our own (default priority), ordered
    // after and before the caller's work by events.
    h2_status ge = ensure_graph_stream(c);
    if (ge != H2_OK) return ge;
    hipStream_t gs = c.graph_stream;
    HIPCHK(hipEventRecord(c.ev_g0, st));
    HIPCHK(hipStreamWaitEvent(gs, c.ev_g0, 0));
    if (!c.graph) {
      HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      h2_status e = do_factor(c, gs);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(gs, &g);
      if (e != H2_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e;
      }
      HIPCHK(ce);
      c.graph_def = g;
      HIPCHK(hipGraphInstantiate(&c.graph, g, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(c.graph, gs));
    HIPCHK(hipEventRecord(c.ev_g1, gs));
    HIPCHK(hipStreamWaitEvent(st, c.ev_g1, 0));
  } else {
    h2_status e = do_factor(c, st);
    if (e != H2_OK) { c.failed = true; return e; }
  }
  int fail = INT_MAX;
  HIPCHK(hipMemcpyAsync(&fail, c.dFail, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  c.st.t_factor = now_seconds() - t0;
  if (c.prm.timing && !c.prm.use_graph) {
    h2_status e = collect_factor_times(c);
    if (e != H2_OK) return e;
  }
  if (fail != INT_MAX) {
    const int hstep = fail >> 20, b = fail & ((1 << 20) - 1);
    if (hstep == 1023) {
      c.st.fail_level = 0;
      c.st.fail_box = 0;
      c.st.fail_inst = b;
    } else {
      const Step& Sx = c.steps[hstep];
      c.st.fail_level = Sx.lvl[b];
      c.st.fail_box = Sx.idx[b];
      c.st.fail_inst = Sx.inst[b];
    }
    c.failed = true;
    c.factored = false;
    return H2_ERR_NOT_SPD;
  }
  c.factored = true;
  return H2_OK;
}

static h2_status solve_plain(Ctx& c, const double* b, double* x, int nc, hipStream_t st) {
  return do_solve_chunk(c, b, c.N, x, c.N, nc, st);
}

// The capture stream and the events that order it after and before the
// caller's stream (created once per handle).
static h2_status ensure_graph_stream(Ctx& c) {
  if (c.graph_stream) return H2_OK;
  HIPCHK(hipStreamCreateWithFlags(&c.graph_stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c.ev_g0, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c.ev_g1, hipEventDisableTiming));
  return H2_OK;
}

// A substitution (op 0: out = M^{-1} in) or an H^2 product (op 1: out = A in,
// on the FP32 copies if lowp) of nc columns.  With `graphs`, the launch
// sequence is captured once per (op, in, out, nc, lowp, partial buffer) on the
// handle's own stream and replayed there, ordered after and before the
// caller's work by events: a solve's hundreds of short launches then cost one
// graph launch.  The sequences hold no memset and no host synchronization.
static h2_status run_op(Ctx& c, int op, const double* in, double* out, int nc, bool lowp,
                        bool graphs, hipStream_t st) {
  auto direct = [&](hipStream_t s) -> h2_status {
    return op == 0 ? solve_plain(c, in, out, nc, s)
                   : do_matvec_chunk(c, in, c.N, out, c.N, nc, s, lowp);
  };
  if (!graphs) return direct(st);
  h2_status e = ensure_graph_stream(c);
  if (e != H2_OK) return e;
  Ctx::SolveGraph* sg = nullptr;
  for (auto& q : c.sgraphs)
    if (q.op == op && q.in == in && q.out == out && q.nc == nc && q.lowp == lowp &&
        q.part == c.part_cur) {
      sg = &q;
      break;
    }
  hipStream_t gs = c.graph_stream;
  HIPCHK(hipEventRecord(c.ev_g0, st));
  HIPCHK(hipStreamWaitEvent(gs, c.ev_g0, 0));
  if (!sg) {
    Ctx::SolveGraph ng;
    ng.op = op; ng.in = in; ng.out = out; ng.nc = nc; ng.lowp = lowp; ng.part = c.part_cur;
    HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    e = direct(gs);
    const hipError_t ce = hipStreamEndCapture(gs, &ng.g);
    if (e != H2_OK) {
      if (ng.g) (void)hipGraphDestroy(ng.g);
      return e;
    }
    HIPCHK(ce);
    if (hipGraphInstantiate(&ng.exec, ng.g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(ng.g);
      return H2_ERR_HIP;
    }
    c.sgraphs.push_back(ng);
    sg = &c.sgraphs.back();
  }
  HIPCHK(hipGraphLaunch(sg->exec, gs));
  HIPCHK(hipEventRecord(c.ev_g1, gs));
  HIPCHK(hipStreamWaitEvent(st, c.ev_g1, 0));
  return H2_OK;
}

static h2_status colnorms(Ctx& c, const double* a, int nc, double* out, hipStream_t st) {
  HIPCHK(launch_coldot(a, c.N, a, c.N, c.N, nc, c.dWs, out, st));
  return H2_OK;
}

// The solve of h2_solve and h2_solve_noalloc: right-hand sides in chunks of
// at most `chunk` columns, gather partials in c.part_cur (sized by the caller
// for part_len x chunk doubles).  time_gathers: record gather events (the
// event pool is created on first use).
static h2_status solve_impl(Ctx& c, const double* b, double* x, int64_t nrhs, int64_t ld,
                            hipStream_t st, int chunk, bool time_gathers, bool graphs_ok) {
  const double t0 = now_seconds();
  // captured substitutions and products: use_graph, untimed (a graph carries
  // no per-launch events), and a caller that allows the graphs' allocations
  const bool graphs = graphs_ok && c.prm.use_graph && !time_gathers;
  const int maxit = c.prm.ir_max_iter;
  if (time_gathers) {
    if (c.gev.empty()) {
      c.gev.resize(4 * 2048, nullptr);
      for (auto& e : c.gev) HIPCHK(hipEventCreate(&e));
    }
    c.gtime = true;
    c.gev_used = 0;
    c.gbytes.clear();
    c.gkind.clear();
  }
  int iters_total = 0;
  int fp64_mv = 0;
  double worst = 0.0;
  bool noconv = false;
  for (int64_t c0 = 0; c0 < nrhs; c0 += chunk) {
    const int nc = (int)std::min<int64_t>(chunk, nrhs - c0);
    const double* bb = b + c0 * ld;
    double* xx = x + c0 * ld;
    // keep b (x may alias it)
    HIPCHK(launch_axpby(c.w_t, c.N, bb, ld, bb, ld, c.N, nc, nullptr, nullptr, 0.0, st));
    if (maxit <= 0) {
      h2_status e = run_op(c, 0, c.w_t, c.w_x, nc, false, graphs, st);
      if (e != H2_OK) return e;
    } else {
      double* sc = c.dScal;  // [0,16): r.r  [16,32): b.b  [32,48): rz  [48,64): pq  [64,80): rz_new
      double hr[NRHS_MAX], hb[NRHS_MAX];
      h2_status e = colnorms(c, c.w_t, nc, sc + 16, st);
      if (e != H2_OK) return e;
      HIPCHK(hipMemcpyAsync(hb, sc + 16, nc * sizeof(double), hipMemcpyDeviceToHost, st));
      if ((e = run_op(c, 0, c.w_t, c.w_x, nc, false, graphs, st)) != H2_OK) return e;
      // r = b - A x
      if ((e = run_op(c, 1, c.w_x, c.w_q, nc, false, graphs, st)) != H2_OK) return e;
      HIPCHK(launch_axpby(c.w_r, c.N, c.w_t, c.N, c.w_q, c.N, c.N, nc, nullptr, nullptr, -1.0, st));
      const bool pcg = c.prm.use_pcg != 0;
      // PCG on FP32 copies of the near blocks and couplings: its own
      // residual decides when to look at the FP64 operator's
      const bool lowp = pcg && c.prm.matvec_prec == H2_PREC_FP32;
      int restarts = 0;
      ++fp64_mv;
      if (pcg) {
        if ((e = run_op(c, 0, c.w_r, c.w_z, nc, false, graphs, st)) != H2_OK) return e;
        HIPCHK(launch_axpby(c.w_p, c.N, c.w_z, c.N, c.w_z, c.N, c.N, nc, nullptr, nullptr, 0.0, st));
        HIPCHK(launch_coldot(c.w_r, c.N, c.w_z, c.N, c.N, nc, c.dWs, sc + 32, st));
      }
      int it = 0;
      double res = 0.0;
      for (;;) {
        if ((e = colnorms(c, c.w_r, nc, sc, st)) != H2_OK) return e;
        HIPCHK(hipMemcpyAsync(hr, sc, nc * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        res = 0.0;
        for (int q = 0; q < nc; ++q) {
          const double rel = hb[q] > 0 ? std::sqrt(hr[q] / hb[q]) : std::sqrt(hr[q]);
          if (!(rel <= res)) res = rel;  // a NaN column makes res NaN
        }
        if (!std::isfinite(res)) { noconv = true; break; }
        if (res <= c.prm.ir_tol && lowp) {
          // the FP64 operator's residual r = b - A x; restart PCG from it
          // while it is above the target
          if ((e = run_op(c, 1, c.w_x, c.w_q, nc, false, graphs, st)) != H2_OK) return e;
          ++fp64_mv;
          HIPCHK(launch_axpby(c.w_r, c.N, c.w_t, c.N, c.w_q, c.N, c.N, nc, nullptr, nullptr, -1.0, st));
          if ((e = colnorms(c, c.w_r, nc, sc, st)) != H2_OK) return e;
          HIPCHK(hipMemcpyAsync(hr, sc, nc * sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          res = 0.0;
          for (int q = 0; q < nc; ++q) {
            const double rel = hb[q] > 0 ? std::sqrt(hr[q] / hb[q]) : std::sqrt(hr[q]);
            if (!(rel <= res)) res = rel;
          }
          if (!std::isfinite(res)) { noconv = true; break; }
          if (res <= c.prm.ir_tol) break;
          if (restarts >= 8 || it >= maxit) { noconv = true; break; }
          ++restarts;
          if ((e = run_op(c, 0, c.w_r, c.w_z, nc, false, graphs, st)) != H2_OK) return e;
          HIPCHK(launch_axpby(c.w_p, c.N, c.w_z, c.N, c.w_z, c.N, c.N, nc, nullptr, nullptr, 0.0, st));
          HIPCHK(launch_coldot(c.w_r, c.N, c.w_z, c.N, c.N, nc, c.dWs, sc + 32, st));
          continue;
        }
        if (res <= c.prm.ir_tol) break;
        if (it >= maxit) { noconv = true; break; }
        ++it;
        if (!pcg) {
          if ((e = run_op(c, 0, c.w_r, c.w_z, nc, false, graphs, st)) != H2_OK) return e;
          HIPCHK(launch_axpby(c.w_x, c.N, c.w_x, c.N, c.w_z, c.N, c.N, nc, nullptr, nullptr, 1.0, st));
          if ((e = run_op(c, 1, c.w_x, c.w_q, nc, false, graphs, st)) != H2_OK) return e;
          ++fp64_mv;
          HIPCHK(launch_axpby(c.w_r, c.N, c.w_t, c.N, c.w_q, c.N, c.N, nc, nullptr, nullptr, -1.0, st));
        } else {
          if ((e = run_op(c, 1, c.w_p, c.w_q, nc, lowp, graphs, st)) != H2_OK) return e;
          if (!lowp) ++fp64_mv;
          HIPCHK(launch_coldot(c.w_p, c.N, c.w_q, c.N, c.N, nc, c.dWs, sc + 48, st));
          HIPCHK(launch_axpby(c.w_x, c.N, c.w_x, c.N, c.w_p, c.N, c.N, nc, sc + 32, sc + 48, 1.0, st));
          HIPCHK(launch_axpby(c.w_r, c.N, c.w_r, c.N, c.w_q, c.N, c.N, nc, sc + 32, sc + 48, -1.0, st));
          if ((e = run_op(c, 0, c.w_r, c.w_z, nc, false, graphs, st)) != H2_OK) return e;
          HIPCHK(launch_coldot(c.w_r, c.N, c.w_z, c.N, c.N, nc, c.dWs, sc + 64, st));
          HIPCHK(launch_axpby(c.w_p, c.N, c.w_z, c.N, c.w_p, c.N, c.N, nc, sc + 64, sc + 32, 1.0, st));
          HIPCHK(hipMemcpyAsync(sc + 32, sc + 64, nc * sizeof(double), hipMemcpyDeviceToDevice, st));
        }
      }
      iters_total = std::max(iters_total, it);
      if (!(res <= worst)) worst = res;  // keeps a NaN
    }
    HIPCHK(launch_axpby(xx, ld, c.w_x, c.N, c.w_x, c.N, c.N, nc, nullptr, nullptr, 0.0, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  c.st.t_solve = now_seconds() - t0;
  if (c.gtime) {
    c.gtime = false;
    double tt[4] = {0.0, 0.0, 0.0, 0.0}, bb[4] = {0.0, 0.0, 0.0, 0.0};
    int nl[4] = {0, 0, 0, 0};
    for (size_t q = 0; q + 4 <= c.gev_used; q += 4) {
      float ms0 = 0.f, ms1 = 0.f;
      HIPCHK(hipEventElapsedTime(&ms0, c.gev[q], c.gev[q + 1]));
      HIPCHK(hipEventElapsedTime(&ms1, c.gev[q + 2], c.gev[q + 3]));
      const int g = q / 4, kind = c.gkind[g];
      tt[kind] += 1e-3 * ms0; bb[kind] += c.gbytes[2 * g]; ++nl[kind];
      tt[2] += 1e-3 * ms1; bb[2] += c.gbytes[2 * g + 1]; ++nl[2];
    }
    for (int q = 0; q < 3; ++q) {
      c.st.t_gather[q] = tt[q];
      c.st.bytes_gather[q] = bb[q];
      c.st.gather_launches[q] = nl[q];
    }
    c.st.t_gather_mv32 = tt[3];
    c.st.bytes_gather_mv32 = bb[3];
    c.st.gather_launches_mv32 = nl[3];
  }
  c.st.ir_fp64_matvecs = fp64_mv;
  c.st.ir_iters = iters_total;
  c.st.ir_residual = worst;
  return noconv ? H2_ERR_NOCONV : H2_OK;
}

h2_status h2_solve(h2_handle h, const double* b, double* x, int64_t nrhs, int64_t ld, void* stream) {
  if (!h || !h->c || !b || !x) return H2_ERR_ARG;
  Ctx& c = *h->c;
  if (nrhs < 1 || ld < c.N) return H2_ERR_ARG;
  if (!c.factored || c.failed) return H2_ERR_STATE;
  {
    h2_status e = ensure_partials(c, (int)std::min<int64_t>(NRHS_MAX, nrhs));
    if (e != H2_OK) return e;
  }
  c.part_cur = c.dPart;
  return solve_impl(c, b, x, nrhs, ld, S(stream), NRHS_MAX, c.prm.timing != 0, true);
}

h2_status h2_solve_noalloc(h2_handle h, const double* b, double* x, int64_t nrhs, int64_t ld,
                           void* stream) {
  if (!h || !h->c || !b || !x) return H2_ERR_ARG;
  Ctx& c = *h->c;
  if (nrhs < 1 || ld < c.N) return H2_ERR_ARG;
  if (!c.factored || c.failed) return H2_ERR_STATE;
  if (c.part_len > H2_NOALLOC_PARTIALS) return H2_ERR_UNSUPPORTED;
  double* part = nullptr;
  {
    h2_status e = noalloc_partials(&part);
    if (e != H2_OK) return e;
  }
  // as many columns per pass as the fixed array holds (at most NRHS_MAX)
  const int64_t fit = c.part_len > 0 ? H2_NOALLOC_PARTIALS / c.part_len : NRHS_MAX;
  const int chunk = (int)std::min<int64_t>(NRHS_MAX, fit);
  c.part_cur = part;
  return solve_impl(c, b, x, nrhs, ld, S(stream), chunk, false, false);
}

h2_status h2_matvec(h2_handle h, const double* x, double* y, int64_t nrhs, int64_t ld, void* stream) {
  if (!h || !h->c || !x || !y || x == y) return H2_ERR_ARG;
  Ctx& c = *h->c;
  if (nrhs < 1 || ld < c.N) return H2_ERR_ARG;
  hipStream_t st = S(stream);
  {
    h2_status e = ensure_partials(c, (int)std::min<int64_t>(NRHS_MAX, nrhs));
    if (e != H2_OK) return e;
  }
  for (int64_t c0 = 0; c0 < nrhs; c0 += NRHS_MAX) {
    const int nc = (int)std::min<int64_t>(NRHS_MAX, nrhs - c0);
    c.part_cur = c.dPart;
    h2_status e = do_matvec_chunk(c, x + c0 * ld, ld, y + c0 * ld, ld, nc, st);
    if (e != H2_OK) return e;
  }
  HIPCHK(hipStreamSynchronize(st));
  return H2_OK;
}

h2_status h2_stats(h2_handle h, h2_stats_t* out) {
  if (!h || !h->c || !out) return H2_ERR_ARG;
  *out = h->c->st;
  return H2_OK;
}

h2_status h2_get_counts(h2_handle h, int64_t* n_boxes, int64_t* n_skel) {
  if (!h || !h->c) return H2_ERR_ARG;
  int64_t nb = 0, ns = 0;
  for (auto& Sx : h->c->steps) {
    nb += Sx.nbox;
    ns += Sx.sum_k;
  }
  if (n_boxes) *n_boxes = nb;
  if (n_skel) *n_skel = ns;
  return H2_OK;
}

h2_status h2_get_structure(h2_handle h, int64_t* perm, int32_t* ranks, int32_t* ms, int64_t* skel) {
  if (!h || !h->c) return H2_ERR_ARG;
  Ctx& c = *h->c;
  if (perm)
    for (auto& in : c.ins) std::memcpy(perm + in.pbase, in.tree.perm.data(), in.n * sizeof(int64_t));
  int64_t bo = 0, so = 0;
  for (auto& Sx : c.steps) {
    for (int b = 0; b < Sx.nbox; ++b) {
      if (ranks) ranks[bo + b] = Sx.k[b];
      if (ms) ms[bo + b] = Sx.m[b];
    }
    if (skel)
      for (int64_t q = 0; q < Sx.sum_k; ++q) {
        int b = (int)(std::upper_bound(Sx.koff.begin(), Sx.koff.end(), q) - Sx.koff.begin()) - 1;
        skel[so + q] = Sx.SK[q] - c.ins[Sx.inst[b]].pbase;
      }
    bo += Sx.nbox;
    so += Sx.sum_k;
  }
  return H2_OK;
}

h2_status h2_get_pairs(h2_handle h, int32_t level, int32_t far, int32_t* pairs, int64_t* count) {
  if (!h || !h->c || !count) return H2_ERR_ARG;
  const Tree& t = h->c->ins[0].tree;
  if (level < 0 || level > t.L) return H2_ERR_ARG;
  const auto& v = far ? t.far[level] : t.near[level];
  *count = (int64_t)v.size();
  if (pairs)
    for (size_t q = 0; q < v.size(); ++q) {
      pairs[2 * q] = v[q].first;
      pairs[2 * q + 1] = v[q].second;
    }
  return H2_OK;
}

h2_status h2_get_basis(h2_handle h, int32_t inst, int32_t level, int32_t box, double* p,
                       int32_t* m, int32_t* k) {
  if (!h || !h->c || inst < 0 || inst >= h->c->n_inst) return H2_ERR_ARG;
  Ctx& c = *h->c;
  const Tree& t = c.ins[inst].tree;
  if (level < 1 || level > t.L || box < 0 || box >= (1 << level)) return H2_ERR_ARG;
  const Step& Sx = c.steps[t.L - level];
  int b = -1;
  for (int q = 0; q < Sx.nbox; ++q)
    if (Sx.inst[q] == inst && Sx.idx[q] == box) { b = q; break; }
  if (b < 0) return H2_ERR_ARG;
  if (m) *m = Sx.m[b];
  if (k) *k = Sx.k[b];
  if (p && Sx.m[b] > 0) {
    if (!c.factored) return H2_ERR_STATE;
    HIPCHK(hipMemcpy(p, Sx.dP + Sx.qoff[b], sizeof(double) * Sx.m[b] * Sx.m[b],
                     hipMemcpyDeviceToHost));
  }
  return H2_OK;
}

h2_status h2_get_root(h2_handle h, int32_t inst, double* a, int64_t* n0) {
  if (!h || !h->c || inst < 0 || inst >= h->c->n_inst) return H2_ERR_ARG;
  Instance& in = h->c->ins[inst];
  if (n0) *n0 = in.n0;
  if (a && in.n0 > 0) {
    if (!h->c->factored) return H2_ERR_STATE;
    HIPCHK(hipMemcpy(a, in.dRootA, sizeof(double) * in.n0 * in.n0, hipMemcpyDeviceToHost));
  }
  return H2_OK;
}

void h2_destroy(h2_handle h) { delete h; }

}  // extern "C"
