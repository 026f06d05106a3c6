// h2_build: H^2 construction with pre-factorization (Algorithm 1) on the
// device, level by level from the leaves, batched over every box of every
// instance at the same height.  The host keeps the index bookkeeping (tree,
// lists, sample selection, parent active sets); kernel evaluation, the
// near-sample Cholesky solves, the interpolative decompositions, couplings and
// near blocks run in the kernels of k_vec.hip, k_dense.hip and k_gemm.hip.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "h2_ctx.hpp"

namespace h2 {

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

Ctx::~Ctx() {
  if (ev_a) (void)hipEventDestroy(ev_a);
  if (ev_b) (void)hipEventDestroy(ev_b);
  if (graph) (void)hipGraphExecDestroy(graph);
  if (graph_def) (void)hipGraphDestroy(graph_def);
  for (auto& sg : sgraphs) {
    if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
    if (sg.g) (void)hipGraphDestroy(sg.g);
  }
  for (hipEvent_t e : gev) (void)hipEventDestroy(e);
  for (hipEvent_t e : fev) (void)hipEventDestroy(e);
  if (ev_g0) (void)hipEventDestroy(ev_g0);
  if (ev_g1) (void)hipEventDestroy(ev_g1);
  if (graph_stream) (void)hipStreamDestroy(graph_stream);
  if (ua.alloc) (void)hipDeviceSynchronize();
  for (void* p : allocs) dev_free(p);
}

hipError_t run_gemm(const Batch<GemmDesc>& b, hipStream_t st, int tag) {
  if (b.f32io && b.terms)
    return launch_gemm_bf16s(b.d, b.toff, b.count, b.tiles, st, b.cfg, b.tA, b.tB, b.f32io == 2,
                             b.terms);
  if (b.f32io)
    return launch_gemm_f32io(b.d, b.toff, b.count, b.tiles, st, b.cfg, b.tA, b.tB, b.f32io == 2);
  return launch_gemm(b.d, b.toff, b.count, b.tiles, st, tag, b.cfg, b.tA, b.tB);
}
hipError_t run_copy(const Batch<CopyDesc>& b, hipStream_t st) {
  return launch_copy(b.d, b.count, st);
}

#define HIPCHK(x)                                  \
  do {                                             \
    if ((x) != hipSuccess) return H2_ERR_HIP;      \
  } while (0)
#define ALLOCHK(p)                                 \
  do {                                             \
    if (!(p)) return H2_ERR_ALLOC;                 \
  } while (0)

static constexpr int ID_MMAX = 4096;    // cpqr_id_kernel LDS capacity
static constexpr int CHOL_NMAX = 2048;  // near-sample points per box (sc^2 doubles each)

// Temporary device buffer of the build, from the handle's allocator, freed at
// scope exit (after the device has finished with it when the caller's
// allocator may hand the memory out again at once).
struct TmpBuf {
  Ctx& c;
  void* p = nullptr;
  explicit TmpBuf(Ctx& ctx) : c(ctx) {}
  TmpBuf(const TmpBuf&) = delete;
  ~TmpBuf() {
    if (!p) return;
    if (c.ua.alloc) (void)hipDeviceSynchronize();
    c.dev_free(p);
  }
  template <class T> T* get(size_t n) {
    if (n == 0) n = 1;
    p = c.dev_alloc(n * sizeof(T));
    return static_cast<T*>(p);
  }
};

template <class T>
static bool upload_tmp(TmpBuf& tb, T*& dst, const std::vector<T>& v, hipStream_t st) {
  dst = tb.get<T>(v.size());
  if (!dst) return false;
  if (v.empty()) return true;
  return hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st) == hipSuccess;
}

static h2_status run_eval(Ctx& c, const std::vector<EvalDesc>& ev, hipStream_t st) {
  if (ev.empty()) return H2_OK;
  TmpBuf tb1(c), tb2(c);
  EvalDesc* d = nullptr;
  int* t = nullptr;
  auto toff = eval_tiles(ev);
  if (!upload_tmp(tb1, d, ev, st) || !upload_tmp(tb2, t, toff, st)) return H2_ERR_ALLOC;
  HIPCHK(launch_eval(d, t, (int)ev.size(), toff.back(), c.dX, c.dim, c.dKern, st));
  HIPCHK(hipStreamSynchronize(st));
  return H2_OK;
}

static h2_status run_gemm_tmp(Ctx& c, const std::vector<GemmDesc>& g, hipStream_t st);

// Blocked Cholesky of SPD blocks A (n x n, ld n) and the explicit inverse of
// the factor, the near-sample solve of the construction (Section 3.5): per
// 64-wide panel, the diagonal block's Cholesky and inverse in LDS
// (panel_kernel), the rows below it times the inverse's transpose, the
// trailing update; then the block rows of X = L^{-1} from the top,
// X_{p,<p} = -X_pp (L_{p,<p} X_{<p,<p}).  A is overwritten by L (zeros above
// the diagonal of the diagonal blocks); Linv (ld n) must hold zeros on entry
// and receives L^{-1}.  A non-positive pivot writes the job's code to fail.
struct CholJob {
  double* A;
  double* Linv;
  int n, code;
};
static h2_status blocked_chol_inv(Ctx& c, const std::vector<CholJob>& jobs, int* fail,
                                  hipStream_t st) {
  if (jobs.empty()) return H2_OK;
  int nmax = 0;
  std::vector<int64_t> so(jobs.size() + 1, 0);  // panel scratch: 64 n per job
  for (size_t q = 0; q < jobs.size(); ++q) {
    nmax = std::max(nmax, jobs[q].n);
    so[q + 1] = so[q] + 64 * (int64_t)std::max(jobs[q].n, 0);
  }
  TmpBuf tsc(c);
  double* dS = tsc.get<double>(so.back());
  ALLOCHK(dS);
  const int np = (nmax + 63) / 64;
  for (int pi = 0; pi < np; ++pi) {
    const int p0 = 64 * pi;
    std::vector<PanelDesc> pd;
    std::vector<GemmDesc> tr, sy;
    std::vector<CopyDesc> bk;
    for (size_t q = 0; q < jobs.size(); ++q) {
      const CholJob& j = jobs[q];
      const int n = j.n;
      if (n <= p0) continue;
      const int w = std::min(64, n - p0), rows = n - p0 - w;
      double* Dp = j.Linv + p0 + (int64_t)p0 * n;
      pd.push_back({j.A + p0 + (int64_t)p0 * n, n, w, Dp, n, j.code});
      if (rows > 0) {
        double* A21 = j.A + p0 + w + (int64_t)p0 * n;
        double* A22 = A21 + (int64_t)w * n;
        double* TA = dS + so[q];  // rows x w, ld n
        tr.push_back(gd(A21, n, 0, Dp, n, 1, nullptr, 1, TA, n, rows, w, w, 1.0, 0.0));
        sy.push_back(gd(TA, n, 0, TA, n, 1, A22, n, A22, n, rows, rows, w, -1.0, 1.0));
        bk.push_back({TA, A21, rows, w, n, n, 0});
      }
    }
    TmpBuf tp(c), tb(c);
    PanelDesc* dpd = nullptr;
    CopyDesc* dbk = nullptr;
    if (!upload_tmp(tp, dpd, pd, st) || !upload_tmp(tb, dbk, bk, st)) return H2_ERR_ALLOC;
    HIPCHK(launch_panel(dpd, (int)pd.size(), fail, st));
    h2_status e = run_gemm_tmp(c, tr, st);
    if (e == H2_OK) e = run_gemm_tmp(c, sy, st);
    if (e != H2_OK) return e;
    HIPCHK(launch_copy(dbk, (int)bk.size(), st));
    HIPCHK(hipStreamSynchronize(st));
  }
  for (int pi = 1; pi < np; ++pi) {
    const int p0 = 64 * pi;
    std::vector<GemmDesc> i1, i2;
    for (size_t q = 0; q < jobs.size(); ++q) {
      const CholJob& j = jobs[q];
      const int n = j.n;
      if (n <= p0) continue;
      const int w = std::min(64, n - p0);
      double* TA = dS + so[q];  // w x p0, ld 64
      i1.push_back(gd(j.A + p0, n, 0, j.Linv, n, 0, nullptr, 1, TA, 64, w, p0, p0, 1.0, 0.0));
      i2.push_back(gd(j.Linv + p0 + (int64_t)p0 * n, n, 0, TA, 64, 0, nullptr, 1, j.Linv + p0, n,
                      w, p0, w, -1.0, 0.0));
    }
    h2_status e = run_gemm_tmp(c, i1, st);
    if (e == H2_OK) e = run_gemm_tmp(c, i2, st);
    if (e != H2_OK) return e;
  }
  return H2_OK;
}

// Blocked pivot-free LU of the near-sample blocks A (n x n, ld n) for the LU
// variant, with the explicit inverses of both factors: per 64-wide panel the
// diagonal block's LU and the inverses of its factors in LDS
// (lu_panel_kernel), L_21 = A_21 U_pp^{-1}, U_12 = L_pp^{-1} A_12, the trailing
// update A_22 -= L_21 U_12; then the block rows of L^{-1},
// X_{p,<p} = -X_pp (L_{p,<p} X_{<p,<p}), and the block columns of U^{-1},
// Y_{<p,p} = -(Y_{<p,<p} U_{<p,p}) Y_pp.  A is overwritten by L (unit, below
// the diagonal) and U; Linv and Uinv (ld n) must hold zeros on entry.  A zero
// or non-finite pivot writes the job's code to fail.
struct LuJob {
  double* A;
  double* Linv;
  double* Uinv;
  int n, code;
};
static h2_status blocked_lu_inv(Ctx& c, const std::vector<LuJob>& jobs, int* fail,
                                hipStream_t st) {
  if (jobs.empty()) return H2_OK;
  int nmax = 0;
  std::vector<int64_t> so(jobs.size() + 1, 0);  // scratch: 128 n per job
  for (size_t q = 0; q < jobs.size(); ++q) {
    nmax = std::max(nmax, jobs[q].n);
    so[q + 1] = so[q] + 128 * (int64_t)std::max(jobs[q].n, 0);
  }
  TmpBuf tsc(c);
  double* dS = tsc.get<double>(so.back());
  ALLOCHK(dS);
  const int np = (nmax + 63) / 64;
  for (int pi = 0; pi < np; ++pi) {
    const int p0 = 64 * pi;
    std::vector<PanelDesc> pd;
    std::vector<GemmDesc> tr, up;
    std::vector<CopyDesc> bk;
    for (size_t q = 0; q < jobs.size(); ++q) {
      const LuJob& j = jobs[q];
      const int n = j.n;
      if (n <= p0) continue;
      const int w = std::min(64, n - p0), rows = n - p0 - w;
      double* Lp = j.Linv + p0 + (int64_t)p0 * n;
      double* Up = j.Uinv + p0 + (int64_t)p0 * n;
      pd.push_back({j.A + p0 + (int64_t)p0 * n, n, w, Lp, n, j.code, Up, n});
      if (rows > 0) {
        double* A21 = j.A + p0 + w + (int64_t)p0 * n;
        double* A12 = j.A + p0 + (int64_t)(p0 + w) * n;
        double* A22 = A21 + (int64_t)w * n;
        double* S1 = dS + so[q];                    // rows x w, ld n
        double* S2 = dS + so[q] + 64 * (int64_t)n;  // w x rows, ld 64
        tr.push_back(gd(A21, n, 0, Up, n, 0, nullptr, 1, S1, n, rows, w, w, 1.0, 0.0));
        tr.push_back(gd(Lp, n, 0, A12, n, 0, nullptr, 1, S2, 64, w, rows, w, 1.0, 0.0));
        up.push_back(gd(S1, n, 0, S2, 64, 0, A22, n, A22, n, rows, rows, w, -1.0, 1.0));
        bk.push_back({S1, A21, rows, w, n, n, 0});
        bk.push_back({S2, A12, w, rows, 64, n, 0});
      }
    }
    TmpBuf tp(c), tb(c);
    PanelDesc* dpd = nullptr;
    CopyDesc* dbk = nullptr;
    if (!upload_tmp(tp, dpd, pd, st) || !upload_tmp(tb, dbk, bk, st)) return H2_ERR_ALLOC;
    HIPCHK(launch_lu_panel(dpd, (int)pd.size(), fail, st));
    h2_status e = run_gemm_tmp(c, tr, st);
    if (e == H2_OK) e = run_gemm_tmp(c, up, st);
    if (e != H2_OK) return e;
    HIPCHK(launch_copy(dbk, (int)bk.size(), st));
    HIPCHK(hipStreamSynchronize(st));
  }
  for (int pi = 1; pi < np; ++pi) {
    const int p0 = 64 * pi;
    std::vector<GemmDesc> i1, i2;
    for (size_t q = 0; q < jobs.size(); ++q) {
      const LuJob& j = jobs[q];
      const int n = j.n;
      if (n <= p0) continue;
      const int w = std::min(64, n - p0);
      double* T1 = dS + so[q];                    // w x p0, ld 64
      double* T2 = dS + so[q] + 64 * (int64_t)n;  // p0 x w, ld n
      i1.push_back(gd(j.A + p0, n, 0, j.Linv, n, 0, nullptr, 1, T1, 64, w, p0, p0, 1.0, 0.0));
      i1.push_back(gd(j.Uinv, n, 0, j.A + (int64_t)p0 * n, n, 0, nullptr, 1, T2, n, p0, w, p0, 1.0,
                      0.0));
      i2.push_back(gd(j.Linv + p0 + (int64_t)p0 * n, n, 0, T1, 64, 0, nullptr, 1, j.Linv + p0, n,
                      w, p0, w, -1.0, 0.0));
      i2.push_back(gd(T2, n, 0, j.Uinv + p0 + (int64_t)p0 * n, n, 0, nullptr, 1,
                      j.Uinv + (int64_t)p0 * n, n, p0, w, w, -1.0, 0.0));
    }
    h2_status e = run_gemm_tmp(c, i1, st);
    if (e == H2_OK) e = run_gemm_tmp(c, i2, st);
    if (e != H2_OK) return e;
  }
  return H2_OK;
}

static h2_status run_gemm_tmp(Ctx& c, const std::vector<GemmDesc>& g, hipStream_t st) {
  if (g.empty()) return H2_OK;
  TmpBuf tb1(c), tb2(c);
  GemmDesc* d = nullptr;
  int* t = nullptr;
  auto tmap = gemm_tile_map(g, GEMM_BM[0], GEMM_BN[0]);
  if (!upload_tmp(tb1, d, g, st) || !upload_tmp(tb2, t, tmap, st)) return H2_ERR_ALLOC;
  HIPCHK(launch_gemm(d, t, (int)g.size(), (int)(tmap.size() / 2), st, 0, 0, g[0].tA, g[0].tB));
  HIPCHK(hipStreamSynchronize(st));
  return H2_OK;
}

h2_status build_impl(int n_inst, const double* const* pts, const int64_t* ns,
                     const h2_kernel* kerns, const h2_params* prm, const int64_t* const* perms,
                     const int32_t* fixed_ranks, const int32_t* fixed_skel, hipStream_t st,
                     h2_handle* out) {
  if (!out || !prm || !pts || !ns || !kerns || n_inst < 1) return H2_ERR_ARG;
  *out = nullptr;
  if (prm->dim != 2 && prm->dim != 3) return H2_ERR_ARG;
  if (prm->leaf < 2 || !(prm->eps >= 0.0) || !(prm->eta >= 0.0)) return H2_ERR_ARG;
  if (prm->s_far < -1 || prm->s_near < -1 || prm->max_rank < 0) return H2_ERR_ARG;
  if (prm->solve_prec != H2_PREC_FP64 && prm->solve_prec != H2_PREC_FP32 &&
      prm->solve_prec != H2_PREC_BF16)
    return H2_ERR_ARG;
  if (prm->gs_sweeps < 0 || prm->gs_sweeps > 64) return H2_ERR_ARG;
  if (prm->matvec_prec != H2_PREC_FP64 && prm->matvec_prec != H2_PREC_FP32) return H2_ERR_ARG;
  if (prm->gemm_prec != H2_PREC_FP64 && prm->gemm_prec != H2_PREC_FP32 &&
      prm->gemm_prec != H2_PREC_BF16 && prm->gemm_prec != H2_PREC_BF16X3)
    return H2_ERR_ARG;
  for (int t = 0; t < n_inst; ++t) {
    if (!pts[t] || ns[t] < 1) return H2_ERR_ARG;
    for (int64_t q = 0; q < ns[t] * prm->dim; ++q)
      if (!std::isfinite(pts[t][q])) return H2_ERR_ARG;
    const h2_kernel& k = kerns[t];
    if (k.id < 0 || k.id > 4) return H2_ERR_ARG;
    const bool reg = k.id <= 1 || k.id == 4;
    if ((reg && !(k.delta > 0.0)) || (!reg && !(k.ell > 0.0))) return H2_ERR_ARG;
    if (k.nugget < 0.0) return H2_ERR_ARG;
    if (k.id == 4 && !std::isfinite(k.beta)) return H2_ERR_ARG;
  }
  // the LU variant: forced, or any non-symmetric kernel
  bool lu = prm->factor_lu != 0;
  for (int t = 0; t < n_inst; ++t)
    if (kerns[t].id == 4 && kerns[t].beta != 0.0) lu = true;
  if (prm->factor_lu != 0 && prm->factor_lu != 1) return H2_ERR_ARG;
  // the LU variant: any transform precision, FP64 or FP32 substitution
  // copies (the packed BF16 copies follow the symmetric path's storage),
  // stationary refinement with the FP64 operator
  if (lu && (prm->solve_prec == H2_PREC_BF16 || prm->matvec_prec != H2_PREC_FP64 ||
             prm->use_pcg))
    return H2_ERR_ARG;
  if (fixed_ranks && n_inst != 1) return H2_ERR_ARG;
  if (prm->allocator && (!prm->allocator->alloc || !prm->allocator->free)) return H2_ERR_ARG;

  const double t_begin = now_seconds();
  auto ctx = std::make_unique<Ctx>();
  Ctx& c = *ctx;
  // a breakdown keeps the handle (failed state) so that h2_stats can report
  // where it happened
  auto not_spd = [&]() {
    c.failed = true;
    auto* hnd = new h2_ctx;
    hnd->c = std::move(ctx);
    *out = hnd;
    return H2_ERR_NOT_SPD;
  };
  c.prm = *prm;
  if (prm->allocator) c.ua = *prm->allocator;
  c.prm.allocator = nullptr;
  c.n_inst = n_inst;
  c.dim = prm->dim;
  c.lu = lu;
  c.st.lu_variant = lu ? 1 : 0;
  c.ins.resize(n_inst);
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));

  int64_t N = 0;
  for (int t = 0; t < n_inst; ++t) {
    Instance& in = c.ins[t];
    in.n = ns[t];
    in.pbase = N;
    N += ns[t];
    const h2_kernel& k = kerns[t];
    in.kern = KernelDev{k.id, k.delta, k.kappa, k.ell, k.nugget, k.id == 4 ? k.beta : 0.0};
    in.rank.assign(in.n, 0);
    if (perms && perms[t]) {
      std::vector<char> seen(in.n, 0);
      for (int64_t q = 0; q < in.n; ++q) {
        const int64_t v = perms[t][q];
        if (v < 0 || v >= in.n || seen[v]) return H2_ERR_ARG;
        seen[v] = 1;
        in.rank[v] = q;
      }
    } else {
      for (int64_t q = 0; q < in.n; ++q) in.rank[q] = q;
    }
  }
  c.N = N;
  // trees in parallel over instances, each on its share of the threads
  {
    const unsigned tw = std::min<unsigned>(hw, n_inst);
    const int per = (int)std::max(1u, hw / tw);
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    for (unsigned w = 0; w < tw; ++w)
      th.emplace_back([&]() {
        for (int t; (t = next.fetch_add(1)) < n_inst;)
          build_tree(pts[t], c.ins[t].n, c.dim, prm->leaf, prm->eta, c.ins[t].tree, per);
      });
    for (auto& x : th) x.join();
  }
  c.H = 0;
  for (auto& in : c.ins) c.H = std::max(c.H, in.tree.L);

  // points (global ids: pbase + local index), kernels, global tree permutation
  {
    std::vector<double> X((size_t)N * c.dim);
    for (int t = 0; t < n_inst; ++t)
      std::memcpy(&X[(size_t)c.ins[t].pbase * c.dim], pts[t], sizeof(double) * c.ins[t].n * c.dim);
    c.dX = c.alloc<double>(X.size());
    ALLOCHK(c.dX);
    HIPCHK(hipMemcpy(c.dX, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice));
    // entry n_inst + t: the transposed kernel G^T(x, y) = G(y, x) of instance
    // t (the drift kernel with -beta; the symmetric kernels unchanged)
    std::vector<KernelDev> kd(2 * n_inst);
    for (int t = 0; t < n_inst; ++t) {
      kd[t] = c.ins[t].kern;
      kd[n_inst + t] = c.ins[t].kern;
      kd[n_inst + t].beta = -kd[n_inst + t].beta;
    }
    c.dKern = c.alloc<KernelDev>(2 * n_inst);
    ALLOCHK(c.dKern);
    HIPCHK(hipMemcpy(c.dKern, kd.data(), 2 * n_inst * sizeof(KernelDev), hipMemcpyHostToDevice));
    std::vector<int64_t> pg(N);
    for (int t = 0; t < n_inst; ++t)
      for (int64_t q = 0; q < c.ins[t].n; ++q) pg[c.ins[t].pbase + q] = c.ins[t].pbase + c.ins[t].tree.perm[q];
    c.dPermG = c.alloc<int64_t>(N);
    ALLOCHK(c.dPermG);
    HIPCHK(hipMemcpy(c.dPermG, pg.data(), N * sizeof(int64_t), hipMemcpyHostToDevice));
  }
  c.dFail = c.alloc<int>(4);
  c.dWs = c.alloc<double>(256 * NRHS_MAX * 4);
  c.dScal = c.alloc<double>(NRHS_MAX * 8);
  ALLOCHK(c.dFail);
  ALLOCHK(c.dWs);
  ALLOCHK(c.dScal);

  // active sets of the current level per instance (global ids)
  std::vector<std::vector<std::vector<int64_t>>> curB(n_inst);
  for (int t = 0; t < n_inst; ++t) {
    const Tree& tr = c.ins[t].tree;
    const int L = tr.L;
    curB[t].resize((size_t)1 << L);
    for (int i = 0; i < (1 << L); ++i)
      for (int64_t q = tr.start[L][i]; q < tr.start[L][i + 1]; ++q)
        curB[t][i].push_back(c.ins[t].pbase + tr.perm[q]);
  }
  size_t fixed_pos = 0, fixed_box = 0;

  // rank prediction for every box of every level, before any compression:
  // one network launch over the tree geometry
  std::vector<std::vector<float>> pred(c.H);
  if (prm->rank_model) {
    std::vector<float> feats;
    std::vector<int> cnt(c.H, 0);
    for (int h = 0; h < c.H; ++h)
      for (int t = 0; t < n_inst; ++t) {
        const int l = c.ins[t].tree.L - h;
        if (l < 1) continue;
        for (int i = 0; i < (1 << l); ++i) {
          float f[8];
          box_features_host(c, t, l, i, f);
          feats.insert(feats.end(), f, f + 8);
          ++cnt[h];
        }
      }
    const int64_t nb_all = (int64_t)feats.size() / 8;
    TmpBuf tw(c), tfe(c), ty(c);
    float* dw = tw.get<float>(4801);
    float* df = tfe.get<float>(feats.size());
    float* dy = ty.get<float>(nb_all);
    if (!dw || !df || !dy) return H2_ERR_ALLOC;
    HIPCHK(hipMemcpy(dw, prm->rank_model, 4801 * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(df, feats.data(), feats.size() * sizeof(float), hipMemcpyHostToDevice));
    if (h2_mlp_forward(dw, df, dy, nb_all, st) != H2_OK) return H2_ERR_HIP;
    std::vector<float> y(nb_all);
    HIPCHK(hipMemcpyAsync(y.data(), dy, nb_all * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int64_t o = 0;
    for (int h = 0; h < c.H; ++h) {
      pred[h].assign(y.begin() + o, y.begin() + o + cnt[h]);
      o += cnt[h];
    }
  }

  c.steps.resize(c.H);
  for (int h = 0; h < c.H; ++h) {
    Step& S = c.steps[h];
    S.h = h;
    std::vector<int> base(n_inst, -1);
    for (int t = 0; t < n_inst; ++t) {
      const int l = c.ins[t].tree.L - h;
      if (l < 1) continue;
      base[t] = S.nbox;
      for (int i = 0; i < (1 << l); ++i) {
        S.inst.push_back(t);
        S.idx.push_back(i);
        S.lvl.push_back(l);
        S.m.push_back((int)curB[t][i].size());
        ++S.nbox;
      }
    }
    const int nb = S.nbox;
    S.boff.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) S.boff[b + 1] = S.boff[b] + S.m[b];
    S.sum_m = S.boff[nb];
    for (int b = 0; b < nb; ++b)
      if (S.m[b] > ID_MMAX) return H2_ERR_UNSUPPORTED;
    // pairs and per-box near lists
    std::vector<std::vector<int>> near_loc(nb);
    for (int t = 0; t < n_inst; ++t) {
      if (base[t] < 0) continue;
      const int l = c.ins[t].tree.L - h;
      // unordered pairs (i >= j), or every ordered pair for the LU variant
      for (auto& pr : c.ins[t].tree.near[l]) {
        near_loc[base[t] + pr.first].push_back(pr.second);
        if (lu || pr.first >= pr.second) {
          S.np_i.push_back(base[t] + pr.first);
          S.np_j.push_back(base[t] + pr.second);
        }
      }
      for (auto& pr : c.ins[t].tree.far[l])
        if (lu ? pr.first != pr.second : pr.first > pr.second) {
          S.fp_i.push_back(base[t] + pr.first);
          S.fp_j.push_back(base[t] + pr.second);
        }
    }
    S.diag_pair.assign(nb, -1);
    for (size_t p = 0; p < S.np_i.size(); ++p)
      if (S.np_i[p] == S.np_j[p]) S.diag_pair[S.np_i[p]] = (int)p;
    // active ids
    S.B.reserve(S.sum_m);
    for (int b = 0; b < nb; ++b)
      S.B.insert(S.B.end(), curB[S.inst[b]][S.idx[b]].begin(), curB[S.inst[b]][S.idx[b]].end());
    S.dB = c.alloc<int64_t>(S.sum_m);
    ALLOCHK(S.dB);
    HIPCHK(hipMemcpy(S.dB, S.B.data(), S.sum_m * sizeof(int64_t), hipMemcpyHostToDevice));

    // ---- sample selection (host)
    std::vector<std::vector<int64_t>> SF(nb), SC(nb);
    for (int t = 0; t < n_inst; ++t) {
      if (base[t] < 0) continue;
      const int l = c.ins[t].tree.L - h;
      const int nbt = 1 << l;
      std::vector<std::vector<int>> nl(near_loc.begin() + base[t], near_loc.begin() + base[t] + nbt);
      std::vector<std::vector<int64_t>> sf, sc;
      sample_level(curB[t], nl, c.ins[t].rank.data(), c.ins[t].pbase, prm->s_far, prm->s_near, sf,
                   sc, (int)hw);
      for (int i = 0; i < nbt; ++i) {
        SF[base[t] + i] = std::move(sf[i]);
        SC[base[t] + i] = std::move(sc[i]);
      }
    }
    std::vector<int> sf(nb), sc(nb), s(nb);
    std::vector<int64_t> sfo(nb + 1, 0), sco(nb + 1, 0), acco(nb + 1, 0), t1o(nb + 1, 0),
        xo(nb + 1, 0), qo(nb + 1, 0);
    std::vector<int64_t> ids_f, ids_c;
    for (int b = 0; b < nb; ++b) {
      sf[b] = (int)SF[b].size();
      sc[b] = (int)SC[b].size();
      // the LU variant samples both sides: [G^T(S_F, B_i); G(S_F, B_i);
      // A_cc^{-T} G^T(S_C, B_i); A_cc^{-1} G(S_C, B_i)]
      s[b] = lu ? 2 * (sf[b] + sc[b]) : sf[b] + sc[b];
      if (sc[b] > CHOL_NMAX) return H2_ERR_UNSUPPORTED;
      // pre-factorization flops (Section 3.5): chol(A_cc) and two triangular
      // solves with the m columns of G(S_C, B_i), or 2 c^2 m per sweep; the
      // LU variant: LU(A_cc) and two solves on each side, or sweeps on both
      if (sc[b] > 0) {
        const double cc = sc[b], mm = S.m[b];
        if (lu)
          c.st.flops_prefactor += prm->gs_sweeps > 0 ? prm->gs_sweeps * 4.0 * cc * cc * mm
                                                     : 2.0 * cc * cc * cc / 3.0 + 4.0 * cc * cc * mm;
        else
          c.st.flops_prefactor += prm->gs_sweeps > 0 ? prm->gs_sweeps * 2.0 * cc * cc * mm
                                                     : cc * cc * cc / 3.0 + 2.0 * cc * cc * mm;
      }
      sfo[b + 1] = sfo[b] + sf[b];
      sco[b + 1] = sco[b] + sc[b];
      acco[b + 1] = acco[b] + (int64_t)sc[b] * sc[b];
      t1o[b + 1] = t1o[b] + (int64_t)sc[b] * S.m[b];
      xo[b + 1] = xo[b] + (int64_t)s[b] * S.m[b];
      qo[b + 1] = qo[b] + (int64_t)S.m[b] * S.m[b];
      ids_f.insert(ids_f.end(), SF[b].begin(), SF[b].end());
      ids_c.insert(ids_c.end(), SC[b].begin(), SC[b].end());
    }
    S.qoff = qo;
    // forced skeletons for this step
    std::vector<int32_t> fk(nb, 0), fsk;
    if (fixed_ranks) {
      for (int b = 0; b < nb; ++b) {
        const int kk = fixed_ranks[fixed_box + b];
        if (kk < 0 || kk > S.m[b] || kk > s[b]) return H2_ERR_ARG;
        fk[b] = kk;
        std::vector<char> seen(S.m[b], 0);
        for (int q = 0; q < kk; ++q) {
          const int pos = fixed_skel[fixed_pos + q];
          if (pos < 0 || pos >= S.m[b] || seen[pos]) return H2_ERR_ARG;
          seen[pos] = 1;
          fsk.push_back(pos);
        }
        fixed_pos += kk;
      }
      fixed_box += nb;
    }
    TmpBuf tf(c), tc(c), tacc(c), tlc(c), tt1(c), tt2(c), tx(c), tpiv(c), tk(c), tfs(c);
    TmpBuf tuc(c), tt1t(c), tt2t(c);  // the LU variant's second side
    int64_t *dF = nullptr, *dC = nullptr;
    if (!upload_tmp(tf, dF, ids_f, st) || !upload_tmp(tc, dC, ids_c, st)) return H2_ERR_ALLOC;
    double* dAcc = tacc.get<double>(acco[nb]);
    double* dLc = tlc.get<double>(acco[nb]);
    double* dT1 = tt1.get<double>(t1o[nb]);
    double* dT2 = tt2.get<double>(t1o[nb]);
    // LU variant: U^{-1} of A_cc (or A_cc^T for the sweeps), G^T(S_C, B_i) and
    // its partial solve
    double *dUc = nullptr, *dT1t = nullptr, *dT2t = nullptr;
    if (lu) {
      dUc = tuc.get<double>(acco[nb]);
      dT1t = tt1t.get<double>(t1o[nb]);
      dT2t = tt2t.get<double>(t1o[nb]);
      ALLOCHK(dUc); ALLOCHK(dT1t); ALLOCHK(dT2t);
    }
    double* dXid = tx.get<double>(xo[nb]);
    int32_t* dPiv = tpiv.get<int32_t>(S.sum_m);
    int32_t* dK = tk.get<int32_t>(nb);
    int32_t* dFs = nullptr;
    if (fixed_ranks && !upload_tmp(tfs, dFs, fsk, st)) return H2_ERR_ALLOC;
    // U capacity: the predicted rank with a margin, else the full m
    S.kcap.assign(nb, 0);
    std::vector<int64_t> uo(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
      int cap = S.m[b];
      if (prm->rank_model) {
        const double kp = std::max(0.0, std::exp2((double)pred[h][b]) - 1.0);
        const double margin = prm->rank_margin > 0 ? prm->rank_margin : 0.0;
        cap = std::min<int64_t>(S.m[b], (int64_t)std::ceil(kp * (1.0 + margin)) + 4);
      }
      S.kcap[b] = cap;
      uo[b + 1] = uo[b] + (int64_t)S.m[b] * cap;
    }
    S.dU = c.alloc<double>(uo[nb]);
    ALLOCHK(S.dU);
    S.Uptr.assign(nb, nullptr);
    for (int b = 0; b < nb; ++b) S.Uptr[b] = S.dU + uo[b];
    c.st.bytes_basis += 8.0 * (double)uo[nb];
    ALLOCHK(dAcc); ALLOCHK(dLc); ALLOCHK(dT1); ALLOCHK(dT2); ALLOCHK(dXid); ALLOCHK(dPiv); ALLOCHK(dK);

    // ---- kernel blocks: A_cc, G(S_C, B_i), G(S_F, B_i) into the ID matrix
    std::vector<EvalDesc> ev;
    for (int b = 0; b < nb; ++b) {
      const int64_t* Bb = S.dB + S.boff[b];
      const int t = S.inst[b], tt = n_inst + t;  // tt: the transposed kernel
      if (sc[b] > 0) {
        ev.push_back({dC + sco[b], dC + sco[b], dAcc + acco[b], sc[b], sc[b], sc[b], t});
        ev.push_back({dC + sco[b], Bb, dT1 + t1o[b], sc[b], S.m[b], sc[b], t});
        if (lu) {
          ev.push_back({dC + sco[b], Bb, dT1t + t1o[b], sc[b], S.m[b], sc[b], tt});
          // the sweeps read row i of their matrix as column i of its storage:
          // A_cc^T's storage for the solves with A_cc
          if (prm->gs_sweeps > 0)
            ev.push_back({dC + sco[b], dC + sco[b], dUc + acco[b], sc[b], sc[b], sc[b], tt});
        }
      }
      if (sf[b] > 0) {
        if (lu) {
          ev.push_back({dF + sfo[b], Bb, dXid + xo[b], sf[b], S.m[b], s[b], tt});
          ev.push_back({dF + sfo[b], Bb, dXid + xo[b] + sf[b], sf[b], S.m[b], s[b], t});
        } else {
          ev.push_back({dF + sfo[b], Bb, dXid + xo[b], sf[b], S.m[b], s[b], t});
        }
      }
    }
    h2_status e = run_eval(c, ev, st);
    if (e != H2_OK) return e;
    // ---- A_Close^T = A_cc^{-1} G(S_C, B_i) by Gauss-Seidel sweeps ...
    if (prm->gs_sweeps > 0) {
      std::vector<GsDesc> gsd;
      // the row-major iterates reuse the (unused) second product buffer
      for (int b = 0; b < nb; ++b) {
        if (sc[b] == 0) continue;
        if (lu) {
          // A_cc X = G(S_C, B_i) and A_cc^T X = G^T(S_C, B_i)
          double* X = dXid + xo[b] + 2 * sf[b];
          gsd.push_back({dUc + acco[b], dT1 + t1o[b], X + sc[b], dT2 + t1o[b], sc[b], S.m[b],
                         sc[b], sc[b], s[b], b});
          gsd.push_back({dAcc + acco[b], dT1t + t1o[b], X, dT2t + t1o[b], sc[b], S.m[b], sc[b],
                         sc[b], s[b], b});
        } else {
          gsd.push_back({dAcc + acco[b], dT1 + t1o[b], dXid + xo[b] + sf[b], dT2 + t1o[b], sc[b],
                         S.m[b], sc[b], sc[b], s[b], b});
        }
      }
      TmpBuf tgs(c);
      GsDesc* dgs = nullptr;
      if (!upload_tmp(tgs, dgs, gsd, st)) return H2_ERR_ALLOC;
      HIPCHK(launch_set_int(c.dFail, INT_MAX, st));
      HIPCHK(launch_gauss_seidel(dgs, (int)gsd.size(), prm->gs_sweeps, c.dFail, st));
      int fail = INT_MAX;
      HIPCHK(hipMemcpyAsync(&fail, c.dFail, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (fail != INT_MAX) {
        c.st.fail_level = c.ins[S.inst[fail]].tree.L - h;
        c.st.fail_box = S.idx[fail];
        c.st.fail_inst = S.inst[fail];
        return not_spd();
      }
    } else if (lu) {
    // ... or exactly, LU variant: U_c^{-1} (L_c^{-1} G(S_C, B_i)) and
    // L_c^{-T} (U_c^{-T} G^T(S_C, B_i))
      std::vector<LuJob> lj;
      for (int b = 0; b < nb; ++b)
        if (sc[b] > 0) lj.push_back({dAcc + acco[b], dLc + acco[b], dUc + acco[b], sc[b], b});
      const size_t ab = (size_t)std::max<int64_t>(acco[nb], 1) * sizeof(double);
      HIPCHK(hipMemsetAsync(dLc, 0, ab, st));
      HIPCHK(hipMemsetAsync(dUc, 0, ab, st));
      HIPCHK(launch_set_int(c.dFail, INT_MAX, st));
      if ((e = blocked_lu_inv(c, lj, c.dFail, st)) != H2_OK) return e;
      int fail = INT_MAX;
      HIPCHK(hipMemcpyAsync(&fail, c.dFail, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (fail != INT_MAX) {
        c.st.fail_level = c.ins[S.inst[fail]].tree.L - h;
        c.st.fail_box = S.idx[fail];
        c.st.fail_inst = S.inst[fail];
        return not_spd();
      }
      std::vector<GemmDesc> g1, g1t, g2, g2t;
      for (int b = 0; b < nb; ++b) {
        const int n = sc[b], m = S.m[b];
        if (n == 0) continue;
        double* X = dXid + xo[b] + 2 * sf[b];
        g1.push_back(gd(dLc + acco[b], n, 0, dT1 + t1o[b], n, 0, nullptr, 1, dT2 + t1o[b], n, n, m,
                        n, 1.0, 0.0));
        g1t.push_back(gd(dUc + acco[b], n, 1, dT1t + t1o[b], n, 0, nullptr, 1, dT2t + t1o[b], n,
                         n, m, n, 1.0, 0.0));
        g2.push_back(gd(dUc + acco[b], n, 0, dT2 + t1o[b], n, 0, nullptr, 1, X + n, s[b], n, m, n,
                        1.0, 0.0));
        g2t.push_back(gd(dLc + acco[b], n, 1, dT2t + t1o[b], n, 0, nullptr, 1, X, s[b], n, m, n,
                         1.0, 0.0));
      }
      for (auto* g : {&g1, &g1t, &g2, &g2t})
        if ((e = run_gemm_tmp(c, *g, st)) != H2_OK) return e;
    } else {
    // ... or exactly: Lc^{-T} (Lc^{-1} G(S_C, B_i))
      std::vector<CholJob> cj;
      for (int b = 0; b < nb; ++b)
        if (sc[b] > 0) cj.push_back({dAcc + acco[b], dLc + acco[b], sc[b], b});
      HIPCHK(hipMemsetAsync(dLc, 0, (size_t)std::max<int64_t>(acco[nb], 1) * sizeof(double), st));
      HIPCHK(launch_set_int(c.dFail, INT_MAX, st));
      if ((e = blocked_chol_inv(c, cj, c.dFail, st)) != H2_OK) return e;
      int fail = INT_MAX;
      HIPCHK(hipMemcpyAsync(&fail, c.dFail, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (fail != INT_MAX) {
        c.st.fail_level = c.ins[S.inst[fail]].tree.L - h;
        c.st.fail_box = S.idx[fail];
        c.st.fail_inst = S.inst[fail];
        return not_spd();
      }
      std::vector<GemmDesc> g1, g2;
      for (int b = 0; b < nb; ++b) {
        if (sc[b] == 0) continue;
        g1.push_back(gd(dLc + acco[b], sc[b], 0, dT1 + t1o[b], sc[b], 0, nullptr, 1, dT2 + t1o[b],
                        sc[b], sc[b], S.m[b], sc[b], 1.0, 0.0));
        g2.push_back(gd(dLc + acco[b], sc[b], 1, dT2 + t1o[b], sc[b], 0, nullptr, 1,
                        dXid + xo[b] + sf[b], s[b], sc[b], S.m[b], sc[b], 1.0, 0.0));
      }
      if ((e = run_gemm_tmp(c, g1, st)) != H2_OK) return e;
      if ((e = run_gemm_tmp(c, g2, st)) != H2_OK) return e;
    }
    // ---- interpolative decomposition
    {
      std::vector<IdDesc> idd(nb);
      int64_t fsp = 0;
      for (int b = 0; b < nb; ++b) {
        idd[b] = IdDesc{dXid + xo[b], S.Uptr[b], dPiv + S.boff[b], dK + b,
                        fixed_ranks ? dFs + fsp : nullptr, s[b], S.m[b], fk[b], S.kcap[b]};
        fsp += fk[b];
      }
      TmpBuf tid(c);
      IdDesc* did = nullptr;
      if (!upload_tmp(tid, did, idd, st)) return H2_ERR_ALLOC;
      const int max_m = nb > 0 ? *std::max_element(S.m.begin(), S.m.end()) : 1;
      HIPCHK(hipStreamSynchronize(st));
      const double t_id = now_seconds();
      HIPCHK(launch_cpqr_id(did, nb, prm->eps, prm->max_rank, max_m, st));
      S.k.assign(nb, 0);
      std::vector<int32_t> piv(S.sum_m);
      HIPCHK(hipMemcpyAsync(S.k.data(), dK, nb * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(piv.data(), dPiv, S.sum_m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      c.st.t_build_id += now_seconds() - t_id;
      // fallback: ranks above the predicted capacity get a buffer of their own
      {
        std::vector<int> over;
        int64_t extra = 0;
        for (int b = 0; b < nb; ++b)
          if (S.k[b] > S.kcap[b]) { over.push_back(b); extra += (int64_t)S.m[b] * S.k[b]; }
        if (!over.empty()) {
          double* dx = c.alloc<double>(extra);
          ALLOCHK(dx);
          std::vector<IdDesc> od;
          int64_t o = 0;
          for (int b : over) {
            S.Uptr[b] = dx + o;
            o += (int64_t)S.m[b] * S.k[b];
            IdDesc q = idd[b];
            q.U = S.Uptr[b];
            od.push_back(q);
          }
          TmpBuf tod(c);
          IdDesc* dod = nullptr;
          if (!upload_tmp(tod, dod, od, st)) return H2_ERR_ALLOC;
          HIPCHK(launch_id_write_u(dod, (int)od.size(), st));
          HIPCHK(hipStreamSynchronize(st));
          c.st.rank_fallbacks += (int)over.size();
          c.st.bytes_basis += 8.0 * (double)extra;
        }
      }
      S.koff.assign(nb + 1, 0);
      S.roff.assign(nb + 1, 0);
      for (int b = 0; b < nb; ++b) {
        S.koff[b + 1] = S.koff[b] + S.k[b];
        S.roff[b + 1] = S.roff[b] + (S.m[b] - S.k[b]);
        for (int q = 0; q < S.k[b]; ++q) S.SK.push_back(S.B[S.boff[b] + piv[S.boff[b] + q]]);
      }
      S.sum_k = S.koff[nb];
      S.sum_r = S.roff[nb];
      S.dSK = c.alloc<int64_t>(S.sum_k);
      ALLOCHK(S.dSK);
      HIPCHK(hipMemcpy(S.dSK, S.SK.data(), S.sum_k * sizeof(int64_t), hipMemcpyHostToDevice));
    }
    // ---- couplings S_ij = G(SK_i, SK_j) (far, i > j) and leaf near blocks
    {
      const size_t nf = S.fp_i.size();
      S.soff.assign(nf + 1, 0);
      for (size_t f = 0; f < nf; ++f)
        S.soff[f + 1] = S.soff[f] + (int64_t)S.k[S.fp_i[f]] * S.k[S.fp_j[f]];
      S.dS = c.alloc<double>(S.soff[nf]);
      ALLOCHK(S.dS);
      std::vector<EvalDesc> ev2;
      for (size_t f = 0; f < nf; ++f) {
        const int i = S.fp_i[f], j = S.fp_j[f];
        ev2.push_back({S.dSK + S.koff[i], S.dSK + S.koff[j], S.dS + S.soff[f], S.k[i], S.k[j],
                       std::max(1, S.k[i]), S.inst[i]});
      }
      const size_t np = S.np_i.size();
      S.poff.assign(np + 1, 0);
      for (size_t p = 0; p < np; ++p)
        S.poff[p + 1] = S.poff[p] + (int64_t)S.m[S.np_i[p]] * S.m[S.np_j[p]];
      if (h == 0) {
        S.dD = c.alloc<double>(S.poff[np]);
        ALLOCHK(S.dD);
        for (size_t p = 0; p < np; ++p) {
          const int i = S.np_i[p], j = S.np_j[p];
          ev2.push_back({S.dB + S.boff[i], S.dB + S.boff[j], S.dD + S.poff[p], S.m[i], S.m[j],
                         S.m[i], S.inst[i]});
        }
      }
      if ((e = run_eval(c, ev2, st)) != H2_OK) return e;
    }
    // ---- parents' active sets
    for (int t = 0; t < n_inst; ++t) {
      if (base[t] < 0) continue;
      const int l = c.ins[t].tree.L - h;
      std::vector<std::vector<int64_t>> nbp((size_t)1 << (l - 1));
      for (int I = 0; I < (1 << (l - 1)); ++I)
        for (int ch = 0; ch < 2; ++ch) {
          const int b = base[t] + 2 * I + ch;
          nbp[I].insert(nbp[I].end(), S.SK.begin() + S.koff[b], S.SK.begin() + S.koff[b + 1]);
        }
      curB[t] = std::move(nbp);
    }
  }
  // roots
  for (int t = 0; t < n_inst; ++t) {
    Instance& in = c.ins[t];
    in.root_ids = curB[t][0];
    in.n0 = (int)in.root_ids.size();
    if (in.n0 > 65536) return H2_ERR_UNSUPPORTED;
  }
  h2_status e = plan_factor(c, st);
  if (e != H2_OK) return e;
  e = plan_solve(c, st);
  if (e != H2_OK) return e;
  if (hipEventCreate(&c.ev_a) != hipSuccess || hipEventCreate(&c.ev_b) != hipSuccess)
    return H2_ERR_HIP;
  if (!prm->no_autotune) {
    e = autotune(c, st);
    if (e != H2_OK) return e;
  }
  c.st.t_build = now_seconds() - t_begin;
  auto* hnd = new h2_ctx;
  hnd->c = std::move(ctx);
  *out = hnd;
  return H2_OK;
}

// ------------------------------------------------------------- factor plan
// Packed BF16 copies of what the substitution reads (its gathers only):
// for every near pair (i, j) the rows [0, k_i) of F_ij from column k_j on
// (L(s)_ij), and for i != j the rows [k_i, m_i) over every column (L(s)_ji^T
// and L(r)_ij); for every box the whole P_i.  The S x S part of F_ij is not
// copied.  Segments are laid out one after another, each with its row count
// rounded up to 8 as leading dimension (a multiple of 8 elements: every
// segment and column starts on a 16-byte boundary).
static void plan_bf16_copies(Step& S, int64_t& nF, int64_t& nP, std::vector<CvtBlk>& sF,
                             std::vector<CvtBlk>& sP) {
  auto r8 = [](int64_t x) { return (x + 7) / 8 * 8; };
  S.cmF.clear();
  S.cmP.clear();
  int64_t off = 0;
  for (size_t p = 0; p < S.np_i.size(); ++p) {
    const int i = S.np_i[p], j = S.np_j[p];
    const int mi = S.m[i], mj = S.m[j], ki = S.k[i], kj = S.k[j];
    CopyMap cm{S.dF + S.poff[p], mi, mi, mj, ki, kj, -1, 1, -1, 1};
    CvtBlk cb{S.poff[p], -1, -1, 0, mi, mi, ki, kj, mj, 0, 0};
    if (ki > 0 && mj > kj) {
      cm.top = cb.top = off;
      cm.ld_top = r8(ki);
      cb.gt = (int)(cm.ld_top / 8);
      off += cm.ld_top * (mj - kj);
    }
    if (i != j && mi > ki && mj > 0) {
      cm.bot = cb.bot = off;
      cm.ld_bot = r8(mi - ki);
      cb.gb = (int)(cm.ld_bot / 8);
      off += cm.ld_bot * mj;
    }
    S.cmF.push_back(cm);
    if (cb.gt + cb.gb > 0) sF.push_back(cb);
  }
  nF = off;
  off = 0;
  for (int b = 0; b < S.nbox; ++b) {
    const int m = S.m[b];
    CopyMap cm{S.dP + S.qoff[b], m, m, m, m, 0, off, r8(m), -1, 1};
    if (m > 0) sP.push_back({S.qoff[b], off, -1, 0, m, m, m, 0, m, (int)(r8(m) / 8), 0});
    off += cm.ld_top * m;
    S.cmP.push_back(cm);
  }
  nP = off;
  // group prefixes (8 rows of one column per group)
  for (auto* v : {&sF, &sP}) {
    int64_t g = 0;
    for (CvtBlk& x : *v) {
      x.g0 = g;
      g += (int64_t)x.c_top * x.gb + (int64_t)(x.cols - x.c_top) * (x.gt + x.gb);
    }
  }
}

h2_status plan_factor(Ctx& c, hipStream_t st) {
  // FP32 transforms (a reduced gemm_prec); the FP32 copies of the leaf near
  // blocks that PCG's products read under matvec_prec FP32 alone do not
  // select them
  const bool f32t = c.prm.gemm_prec != H2_PREC_FP64;
  // root buffers
  int max_n0 = 0;
  for (auto& in : c.ins) {
    const int n0 = std::max(in.n0, 1);
    in.dRoot = c.alloc<double>((size_t)n0 * n0);
    in.dRootA = c.alloc<double>((size_t)n0 * n0);
    in.dRootX = c.alloc<double>((size_t)n0 * n0);
    in.dRinv = c.alloc<double>((size_t)n0 * n0);
    in.dPan = c.alloc<double>((size_t)n0 * (c.lu ? 128 : 64));
    ALLOCHK(in.dRoot); ALLOCHK(in.dRootA); ALLOCHK(in.dRootX); ALLOCHK(in.dRinv); ALLOCHK(in.dPan);
    // L^{-1}: the panels write the diagonal blocks, the inverse block rows
    // the blocks below them; the blocks above stay zero (U^{-1} likewise)
    HIPCHK(hipMemsetAsync(in.dRootX, 0, (size_t)n0 * n0 * sizeof(double), st));
    if (c.lu) {
      in.dRootUi = c.alloc<double>((size_t)n0 * n0);
      ALLOCHK(in.dRootUi);
      HIPCHK(hipMemsetAsync(in.dRootUi, 0, (size_t)n0 * n0 * sizeof(double), st));
    }
    max_n0 = std::max(max_n0, in.n0);
  }
  // L == 0 instances: the dense kernel block is the whole matrix
  {
    std::vector<EvalDesc> ev;
    std::vector<int64_t> ids;
    std::vector<int64_t> io(c.n_inst + 1, 0);
    for (int t = 0; t < c.n_inst; ++t) {
      if (c.ins[t].tree.L == 0) ids.insert(ids.end(), c.ins[t].root_ids.begin(), c.ins[t].root_ids.end());
      io[t + 1] = ids.size();
    }
    if (!ids.empty()) {
      int64_t* dids = c.alloc<int64_t>(ids.size());
      ALLOCHK(dids);
      HIPCHK(hipMemcpy(dids, ids.data(), ids.size() * sizeof(int64_t), hipMemcpyHostToDevice));
      for (int t = 0; t < c.n_inst; ++t) {
        Instance& in = c.ins[t];
        if (in.tree.L != 0) continue;
        in.dRootOrig = c.alloc<double>((size_t)in.n0 * in.n0);
        ALLOCHK(in.dRootOrig);
        ev.push_back({dids + io[t], dids + io[t], in.dRootOrig, in.n0, in.n0, in.n0, t});
      }
      h2_status e = run_eval(c, ev, st);
      if (e != H2_OK) return e;
    }
  }
  // per-step storage
  for (int h = 0; h < c.H; ++h) {
    Step& S = c.steps[h];
    const int nb = S.nbox;
    S.rkoff.assign(nb + 1, 0);
    S.lioff.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
      const int r = S.m[b] - S.k[b];
      S.rkoff[b + 1] = S.rkoff[b] + (int64_t)S.k[b] * S.k[b];
      S.lioff[b + 1] = S.lioff[b] + (int64_t)r * r;
      if (S.m[b] > QR_MMAX) return H2_ERR_UNSUPPORTED;
    }
    const int64_t q = S.qoff[nb];
    S.dQ = c.alloc<double>(q); S.dP = c.alloc<double>(q); S.dTA = c.alloc<double>(q);
    S.dTB = c.alloc<double>(q); S.dW = c.alloc<double>(q);
    S.dR = c.alloc<double>(S.rkoff[nb]); S.dLi = c.alloc<double>(S.lioff[nb]);
    S.dTau = c.alloc<double>(std::max<int64_t>(S.koff[nb], 1));
    ALLOCHK(S.dQ); ALLOCHK(S.dP); ALLOCHK(S.dTA); ALLOCHK(S.dTB); ALLOCHK(S.dW); ALLOCHK(S.dTau);
    ALLOCHK(S.dR); ALLOCHK(S.dLi);
    if (c.lu) {
      S.dPr = c.alloc<double>(q);
      S.dUi = c.alloc<double>(std::max<int64_t>(S.lioff[nb], 1));
      S.dLUs = c.alloc<double>(std::max<int64_t>(128 * S.roff[nb], 1));
      ALLOCHK(S.dPr); ALLOCHK(S.dUi); ALLOCHK(S.dLUs);
    }
    // near blocks of upper steps (m = k_2I + k_2I+1 is known now)
    const size_t np = S.np_i.size();
    S.poff.assign(np + 1, 0);
    for (size_t p = 0; p < np; ++p) S.poff[p + 1] = S.poff[p] + (int64_t)S.m[S.np_i[p]] * S.m[S.np_j[p]];
    if (h > 0) { S.dD = c.alloc<double>(S.poff[np]); ALLOCHK(S.dD); }
    S.dF = c.alloc<double>(S.poff[np]);
    ALLOCHK(S.dF);
    // FP32 transforms: FP32 near blocks (the off-diagonal parent blocks exist
    // only in FP32), far couplings, R factors, pair and far scratch; else the
    // FP64 scratch.  FP32 copies of F and P whenever the substitution reads
    // FP32.
    const bool f32pair = c.prm.gemm_prec != H2_PREC_FP64;
    if (f32pair) {
      const int64_t ns = std::max<int64_t>(S.soff.back(), 1);
      S.dD32 = c.alloc<float>(std::max<int64_t>(S.poff[np], 1));
      S.dT232 = c.alloc<float>(std::max<int64_t>(S.poff[np], 1));
      S.dR32 = c.alloc<float>(std::max<int64_t>(S.rkoff[nb], 1));
      S.dS32 = c.alloc<float>(ns);
      S.dT332 = c.alloc<float>(ns);
      ALLOCHK(S.dD32); ALLOCHK(S.dT232); ALLOCHK(S.dR32); ALLOCHK(S.dS32); ALLOCHK(S.dT332);
      // the fixed leaf near field and far couplings
      if (h == 0) HIPCHK(launch_cvt_f32(S.dD, S.dD32, S.poff[np], st));
      HIPCHK(launch_cvt_f32(S.dS, S.dS32, S.soff.back(), st));
    } else {
      S.dT2 = c.alloc<double>(S.poff[np]);
      S.dT3 = c.alloc<double>(S.soff.back());
      ALLOCHK(S.dT2); ALLOCHK(S.dT3);
      if (c.prm.matvec_prec == H2_PREC_FP32) {
        // FP32 copies of the operator's stored blocks for PCG's products
        S.dS32 = c.alloc<float>(std::max<int64_t>(S.soff.back(), 1));
        ALLOCHK(S.dS32);
        HIPCHK(launch_cvt_f32(S.dS, S.dS32, S.soff.back(), st));
        if (h == 0) {
          S.dD32 = c.alloc<float>(std::max<int64_t>(S.poff[np], 1));
          ALLOCHK(S.dD32);
          HIPCHK(launch_cvt_f32(S.dD, S.dD32, S.poff[np], st));
        }
      }
    }
    if (f32pair || c.prm.solve_prec == H2_PREC_FP32) {
      S.dF32 = c.alloc<float>(std::max<int64_t>(S.poff[np], 1));
      S.dP32 = c.alloc<float>(std::max<int64_t>(q, 1));
      ALLOCHK(S.dF32); ALLOCHK(S.dP32);
      if (c.lu) {
        S.dPr32 = c.alloc<float>(std::max<int64_t>(q, 1));
        ALLOCHK(S.dPr32);
      }
    }
    if (c.prm.solve_prec == H2_PREC_BF16) {
      int64_t nF = 0, nP = 0;
      std::vector<CvtBlk> sF, sP;
      plan_bf16_copies(S, nF, nP, sF, sP);
      S.dF16 = c.alloc<unsigned short>(std::max<int64_t>(nF, 1));
      S.dP16 = c.alloc<unsigned short>(std::max<int64_t>(nP, 1));
      ALLOCHK(S.dF16); ALLOCHK(S.dP16);
      if (!upload(c, S.cvF16, sF, st) || !upload(c, S.cvP16, sP, st)) return H2_ERR_ALLOC;
      auto total = [](const std::vector<CvtBlk>& v) -> int64_t {
        if (v.empty()) return 0;
        const CvtBlk& x = v.back();
        return x.g0 + (int64_t)x.c_top * x.gb + (int64_t)(x.cols - x.c_top) * (x.gt + x.gb);
      };
      S.cvF16_groups = total(sF);
      S.cvP16_groups = total(sP);
      // the segment of the first group of every 256-group block
      auto firsts = [](const std::vector<CvtBlk>& v, int64_t groups) {
        std::vector<int> f((size_t)((groups + 255) / 256));
        size_t sg = 0;
        for (size_t b = 0; b < f.size(); ++b) {
          const int64_t e = (int64_t)b * 256;
          while (sg + 1 < v.size() && v[sg + 1].g0 <= e) ++sg;
          f[b] = (int)sg;
        }
        return f;
      };
      if (!upload(c, S.cvF16_first, firsts(sF, S.cvF16_groups), st) ||
          !upload(c, S.cvP16_first, firsts(sP, S.cvP16_groups), st))
        return H2_ERR_ALLOC;
    }
  }
  // index of (instance, level-local box) in each step
  auto local = [&](int h, int t, int i) -> int {
    const Step& S = c.steps[h];
    // boxes of an instance are contiguous; find its first box
    int lo = 0, hi = S.nbox - 1, first = -1;
    while (lo <= hi) {  // first b with inst[b] >= t
      const int mid = (lo + hi) / 2;
      if (S.inst[mid] >= t) { first = mid; hi = mid - 1; } else lo = mid + 1;
    }
    return first + i;
  };
  // pair maps
  std::vector<std::unordered_map<int64_t, int>> pmap(c.H);
  for (int h = 0; h < c.H; ++h) {
    const Step& S = c.steps[h];
    for (size_t p = 0; p < S.np_i.size(); ++p)
      pmap[h][(int64_t)S.np_i[p] * S.nbox + S.np_j[p]] = (int)p;
  }
  // parent block of child pair (a, b), a >= b, at step h: pointer, ld; with
  // FP32 transforms an off-diagonal parent block below the root exists only
  // in FP32: then ptr32 is set (else nullptr)
  auto parent_block = [&](int h, int a, int b, double*& ptr, int& ld, float*& ptr32) {
    ptr32 = nullptr;
    const Step& S = c.steps[h];
    const int t = S.inst[a];
    const int l = S.lvl[a];
    const int ia = S.idx[a], ib = S.idx[b];
    const int ro = (ia & 1) ? S.k[a - 1] : 0;
    const int co = (ib & 1) ? S.k[b - 1] : 0;
    if (l == 1) {
      ld = c.ins[t].n0;
      ptr = c.ins[t].dRoot + ro + (int64_t)co * ld;
      return;
    }
    const Step& P = c.steps[h + 1];
    const int pI = local(h + 1, t, ia / 2), pJ = local(h + 1, t, ib / 2);
    const int pp = pmap[h + 1].at((int64_t)pI * P.nbox + pJ);
    ld = P.m[pI];
    ptr = P.dD + P.poff[pp] + ro + (int64_t)co * ld;
    if (f32t && pI != pJ) ptr32 = P.dD32 + P.poff[pp] + ro + (int64_t)co * ld;
  };

  for (int h = 0; h < c.H; ++h) {
    Step& S = c.steps[h];
    const int nb = S.nbox;
    std::vector<GemmDesc> gw, gq1, gq2, gq3, gd1, gd2, gv, gv2, gs, gp1, gp2, gf1, gf2;
    std::vector<CopyDesc> cw, cps, cm;
    std::vector<ConvDesc> cvd;  // FP32 transforms: D_ii -> FP32 above the leaves
    std::vector<BoxDev> qr(nb);
    for (int b = 0; b < nb; ++b) {
      const int m = S.m[b], k = S.k[b], r = m - k;
      double* U = S.Uptr[b];
      double* W = S.dW + S.qoff[b];
      double* Q = S.dQ + S.qoff[b];
      double* P = S.dP + S.qoff[b];
      double* TA = S.dTA + S.qoff[b];
      double* TB = S.dTB + S.qoff[b];
      double* R = S.dR + S.rkoff[b];
      double* Li = S.dLi + S.lioff[b];
      double* Dii = S.dD + S.poff[S.diag_pair[b]];
      double* Fii = S.dF + S.poff[S.diag_pair[b]];
      if (h == 0) {
        if (m * k > 0) cw.push_back({U, W, m, k, m, m, 0});
      } else {
        const Step& C = c.steps[h - 1];
        const int a = local(h - 1, S.inst[b], 2 * S.idx[b]);
        const int ka = C.k[a], kb = C.k[a + 1];
        gw.push_back(gd(C.dR + C.rkoff[a], ka, 0, U, m, 0, nullptr, 1, W, m, ka, k, ka, 1.0, 0.0));
        gw.push_back(gd(C.dR + C.rkoff[a + 1], kb, 0, U + ka, m, 0, nullptr, 1, W + ka, m, kb, k, kb,
                        1.0, 0.0));
      }
      qr[b] = BoxDev{m, k, S.inst[b], Q, P, R, Li, TA, TB, W, S.dTau + S.koff[b]};
      if (m * k > 0) {
        // G = V^T V -> P (k x k); T V^T -> TB (k x m); Q = -V (T V^T)
        gq1.push_back(gd(TA, m, 1, TA, m, 0, nullptr, 1, P, k, k, k, m, 1.0, 0.0));
        gq2.push_back(gd(P, k, 0, TA, m, 1, nullptr, 1, TB, k, k, m, k, 1.0, 0.0));
        gq3.push_back(gd(TA, m, 0, TB, k, 0, nullptr, 1, Q, m, m, m, k, -1.0, 0.0));
      }
      if (f32t) {
        // FP32 transforms: D_ii and Q_i from their FP32 copies (Q32 in the
        // P32 buffer, free until P exists), the product in TA's memory as
        // FP32, F_ii = Q^T (.) in FP64 for the Cholesky of its RR part
        float* D32 = S.dD32 + S.poff[S.diag_pair[b]];
        float* Q32 = S.dP32 + S.qoff[b];
        float* T32 = reinterpret_cast<float*>(TA);
        auto asd = [](float* p) { return reinterpret_cast<double*>(p); };
        gd1.push_back(gd(asd(D32), m, 0, asd(Q32), m, 0, nullptr, 1, asd(T32), m, m, m, m, 1.0, 0.0));
        gd2.push_back(gd(asd(Q32), m, 1, asd(T32), m, 0, nullptr, 1, TB, m, m, m, m, 1.0, 0.0));
        if (h > 0) cvd.push_back({Dii, D32, (int64_t)m * m, 1});
      } else {
        gd1.push_back(gd(Dii, m, 0, Q, m, 0, nullptr, 1, TA, m, m, m, m, 1.0, 0.0));
        gd2.push_back(gd(Q, m, 1, TA, m, 0, nullptr, 1, TB, m, m, m, m, 1.0, 0.0));
      }
      if (m * k > 0) cps.push_back({Q, P, m, k, m, m, 0});
      if (c.lu) {
        // LU variant: P = [Q^S | Q^R L^{-T}], P' = [Q^S | Q^R U^{-1}],
        // L(s)_ii = SR U^{-1}, U(s)_ii = L^{-1} RS, SS -= L(s)_ii U(s)_ii
        double* Pr = S.dPr + S.qoff[b];
        double* Ui = S.dUi + S.lioff[b];
        if (m * k > 0) cps.push_back({Q, Pr, m, k, m, m, 0});
        if (r > 0) {
          gv.push_back(gd(Q + (int64_t)k * m, m, 0, Li, r, 1, nullptr, 1, P + (int64_t)k * m, m, m,
                          r, r, 1.0, 0.0));
          gv2.push_back(gd(Q + (int64_t)k * m, m, 0, Ui, r, 0, nullptr, 1, Pr + (int64_t)k * m, m,
                           m, r, r, 1.0, 0.0));
          if (k > 0) {
            gv2.push_back(gd(TB + (int64_t)k * m, m, 0, Ui, r, 0, nullptr, 1, Fii + (int64_t)k * m,
                             m, k, r, r, 1.0, 0.0));
            gv2.push_back(gd(Li, r, 0, TB + k, m, 0, nullptr, 1, Fii + k, m, r, k, r, 1.0, 0.0));
          }
        }
        if (k > 0)
          gs.push_back(gd(Fii + (int64_t)k * m, m, 0, Fii + k, m, 0, TB, m, Fii, m, k, k, r, -1.0,
                          1.0));
        continue;
      }
      if (r > 0) {
        gv.push_back(gd(Q + (int64_t)k * m, m, 0, Li, r, 1, nullptr, 1, P + (int64_t)k * m, m, m, r,
                        r, 1.0, 0.0));
        if (k > 0)
          gv.push_back(gd(TB + (int64_t)k * m, m, 0, Li, r, 1, nullptr, 1, Fii + (int64_t)k * m, m, k,
                          r, r, 1.0, 0.0));
      }
      if (k > 0)
        gs.push_back(gd(Fii + (int64_t)k * m, m, 0, Fii + (int64_t)k * m, m, 1, TB, m, Fii, m, k, k, r,
                        -1.0, 1.0));
    }
    const bool f32pair = f32t;
    // FP32 arrays travel in the double-typed descriptors (the FP32 kernels
    // read them back as float)
    auto asd = [](float* p) { return reinterpret_cast<double*>(p); };
    std::vector<ConvDesc> cvf;
    for (size_t p = 0; p < S.np_i.size(); ++p) {
      const int i = S.np_i[p], j = S.np_j[p];
      if (i == j) {
        if (f32pair)  // F_ii is formed in FP64; the substitution reads its copy
          cvf.push_back({S.dF + S.poff[p], S.dF32 + S.poff[p], (int64_t)S.m[i] * S.m[i], 1});
        continue;
      }
      const int mi = S.m[i], mj = S.m[j];
      if (f32pair) {
        gp1.push_back(gd(asd(S.dD32 + S.poff[p]), mi, 0,
                         asd((c.lu ? S.dPr32 : S.dP32) + S.qoff[j]), mj, 0, nullptr, 1,
                         asd(S.dT232 + S.poff[p]), mi, mi, mj, mj, 1.0, 0.0));
        gp2.push_back(gd(asd(S.dP32 + S.qoff[i]), mi, 1, asd(S.dT232 + S.poff[p]), mi, 0, nullptr,
                         1, asd(S.dF32 + S.poff[p]), mi, mi, mj, mi, 1.0, 0.0));
      } else {
        // (LU variant: the right basis P'_j on the right)
        gp1.push_back(gd(S.dD + S.poff[p], mi, 0, (c.lu ? S.dPr : S.dP) + S.qoff[j], mj, 0,
                         nullptr, 1, S.dT2 + S.poff[p], mi, mi, mj, mj, 1.0, 0.0));
        gp2.push_back(gd(S.dP + S.qoff[i], mi, 1, S.dT2 + S.poff[p], mi, 0, nullptr, 1,
                         S.dF + S.poff[p], mi, mi, mj, mi, 1.0, 0.0));
      }
    }
    // R_i S_ij for all far partners j of box i at once: the far list is sorted
    // by i, so S_ij1 | S_ij2 | ... (each k_i x k_j, ld k_i) is one k_i x sum k_j
    // matrix, and so is its product
    // (FP32 transforms: R32 S32 -> T3_32; T3_32 R32^T into FP32 off-diagonal
    // parent blocks, or into FP64 ones for siblings and the root)
    std::vector<GemmDesc> gf3;
    for (size_t f = 0; f < S.fp_i.size();) {
      const int i = S.fp_i[f], ki = S.k[i];
      size_t g = f;
      int ncol = 0;
      while (g < S.fp_i.size() && S.fp_i[g] == i) ncol += S.k[S.fp_j[g++]];
      if (f32pair)
        gf1.push_back(gd(asd(S.dR32 + S.rkoff[i]), ki, 0, asd(S.dS32 + S.soff[f]), ki, 0, nullptr,
                         1, asd(S.dT332 + S.soff[f]), ki, ki, ncol, ki, 1.0, 0.0));
      else
        gf1.push_back(gd(S.dR + S.rkoff[i], ki, 0, S.dS + S.soff[f], ki, 0, nullptr, 1,
                         S.dT3 + S.soff[f], ki, ki, ncol, ki, 1.0, 0.0));
      f = g;
    }
    for (size_t f = 0; f < S.fp_i.size(); ++f) {
      const int i = S.fp_i[f], j = S.fp_j[f];
      const int ki = S.k[i], kj = S.k[j];
      double* dst;
      float* dst32;
      int ldp;
      parent_block(h, i, j, dst, ldp, dst32);
      if (!f32pair)
        gf2.push_back(gd(S.dT3 + S.soff[f], ki, 0, S.dR + S.rkoff[j], kj, 1, nullptr, 1, dst, ldp,
                         ki, kj, kj, 1.0, 0.0));
      else if (dst32)
        gf2.push_back(gd(asd(S.dT332 + S.soff[f]), ki, 0, asd(S.dR32 + S.rkoff[j]), kj, 1, nullptr,
                         1, asd(dst32), ldp, ki, kj, kj, 1.0, 0.0));
      else
        gf3.push_back(gd(asd(S.dT332 + S.soff[f]), ki, 0, asd(S.dR32 + S.rkoff[j]), kj, 1, nullptr,
                         1, dst, ldp, ki, kj, kj, 1.0, 0.0));
      const bool sib = (S.idx[i] >> 1) == (S.idx[j] >> 1);
      if (sib && ki * kj > 0 && !c.lu) {  // (the LU variant has both orders)
        // transposed copy inside the parent's diagonal block
        cm.push_back({dst, dst - S.k[j] + (int64_t)S.k[j] * ldp, kj, ki, ldp, ldp, 1});
      }
    }
    // from FP32 transformed blocks into FP64 / FP32 parent blocks
    std::vector<CopyDesc> cm32, cm3232;
    for (size_t p = 0; p < S.np_i.size(); ++p) {
      const int a = S.np_i[p], b = S.np_j[p];
      const int ka = S.k[a], kb = S.k[b];
      if (ka * kb == 0) continue;
      double* dst;
      float* dst32;
      int ldp;
      parent_block(h, a, b, dst, ldp, dst32);
      const bool from32 = f32pair && a != b;
      const double* src = from32 ? asd(S.dF32 + S.poff[p]) : S.dF + S.poff[p];
      if (dst32) {  // off-diagonal parent block (not siblings): no transposed copy
        cm3232.push_back({src, asd(dst32), ka, kb, S.m[a], ldp, 0});
        continue;
      }
      std::vector<CopyDesc>& out = from32 ? cm32 : cm;
      out.push_back({src, dst, ka, kb, S.m[a], ldp, 0});
      if (a != b && (S.idx[a] >> 1) == (S.idx[b] >> 1) && !c.lu) {
        // sibling block (2I+1, 2I): also write (2I, 2I+1) = transpose
        double* base = dst - kb;  // row offset of a is k_b; back to the parent origin row
        out.push_back({src, base + (int64_t)kb * ldp, kb, ka, S.m[a], ldp, 1});
      }
    }
    auto up_g = [&](Batch<GemmDesc>& B, const std::vector<GemmDesc>& v) {
      return upload_gemm(c, B, v, st);
    };
    if (!up_g(S.g_w, gw) || !up_g(S.g_qr1, gq1) || !up_g(S.g_qr2, gq2) || !up_g(S.g_qr3, gq3) ||
        !up_g(S.g_diag1, gd1) || !up_g(S.g_diag2, gd2) || !up_g(S.g_v, gv) || !up_g(S.g_v2, gv2) ||
        !up_g(S.g_schur, gs) || !up_g(S.g_pair1, gp1) || !up_g(S.g_pair2, gp2) ||
        !up_g(S.g_far1, gf1) || !up_g(S.g_far2, gf2) || !up_g(S.g_far3, gf3))
      return H2_ERR_ALLOC;
    if (!upload(c, S.c_w, cw, st) || !upload(c, S.c_ps, cps, st) || !upload(c, S.c_merge, cm, st) ||
        !upload(c, S.c_merge32, cm32, st) || !upload(c, S.c_merge3232, cm3232, st) ||
        !upload(c, S.cv_fii, cvf, st) || !upload(c, S.cv_dii, cvd, st) ||
        !upload(c, S.qr, qr, st))
      return H2_ERR_ALLOC;
    if (f32pair) {
      S.g_pair1.f32io = S.g_pair2.f32io = S.g_far1.f32io = S.g_far2.f32io = S.g_diag1.f32io = 1;
      S.g_far3.f32io = S.g_diag2.f32io = 2;
      // BF16 matrix cores: one term (BF16) or three (BF16X3)
      const int terms = c.prm.gemm_prec == H2_PREC_BF16X3 ? 3 : c.prm.gemm_prec == H2_PREC_BF16 ? 1 : 0;
      for (Batch<GemmDesc>* b : {&S.g_pair1, &S.g_pair2, &S.g_far1, &S.g_far2, &S.g_diag1,
                                 &S.g_far3, &S.g_diag2})
        b->terms = terms;
    }
    // blocked Cholesky + inverse of the RR blocks (A at TB + k + k m, ld m;
    // L^{-1} at Li, ld r; panel scratch in TA)
    int rmax = 0;
    for (int b = 0; b < nb; ++b) rmax = std::max(rmax, S.m[b] - S.k[b]);
    const int npan = (rmax + 63) / 64;
    S.ch_panel.assign(npan, {}); S.ch_trsm.assign(npan, {}); S.ch_syrk.assign(npan, {});
    S.ch_back.assign(npan, {}); S.ch_inv1.assign(npan, {}); S.ch_inv2.assign(npan, {});
    for (int pi = 0; pi < npan; ++pi) {
      const int p0 = 64 * pi;
      std::vector<PanelDesc> pd;
      std::vector<GemmDesc> tr, sy, i1, i2;
      std::vector<CopyDesc> bk;
      for (int b = 0; b < nb; ++b) {
        const int m = S.m[b], k = S.k[b], r = m - k;
        if (r <= p0) continue;
        const int w = std::min(64, r - p0), rows = r - p0 - w;
        double* A = S.dTB + S.qoff[b] + k + (int64_t)k * m;
        double* TA = S.dTA + S.qoff[b];
        double* Li = S.dLi + S.lioff[b];
        double* Dp = Li + p0 + (int64_t)p0 * r;
        if (c.lu) {
          // LU variant: L_21 = A_21 U_pp^{-1}, U_12 = L_pp^{-1} A_12 (into the
          // scratch, then back), A_22 -= L_21 U_12; inverse block rows of
          // L^{-1} and block columns of U^{-1}
          double* Ui = S.dUi + S.lioff[b];
          double* Up = Ui + p0 + (int64_t)p0 * r;
          double* S1 = S.dLUs + 128 * S.roff[b];  // rows x w, ld r / w x p0, ld 64
          double* S2 = S1 + 64 * (int64_t)r;       // w x rows, ld 64 / p0 x w, ld r
          pd.push_back({A + p0 + (int64_t)p0 * m, m, w, Dp, r, h * (1 << 20) + b, Up, r});
          if (rows > 0) {
            double* A21 = A + p0 + w + (int64_t)p0 * m;
            double* A12 = A + p0 + (int64_t)(p0 + w) * m;
            double* A22 = A + p0 + w + (int64_t)(p0 + w) * m;
            tr.push_back(gd(A21, m, 0, Up, r, 0, nullptr, 1, S1, r, rows, w, w, 1.0, 0.0));
            tr.push_back(gd(Dp, r, 0, A12, m, 0, nullptr, 1, S2, 64, w, rows, w, 1.0, 0.0));
            sy.push_back(gd(S1, r, 0, S2, 64, 0, A22, m, A22, m, rows, rows, w, -1.0, 1.0));
            bk.push_back({S1, A21, rows, w, r, m, 0});
            bk.push_back({S2, A12, w, rows, 64, m, 0});
          }
          if (p0 > 0) {
            i1.push_back(gd(A + p0, m, 0, Li, r, 0, nullptr, 1, S1, 64, w, p0, p0, 1.0, 0.0));
            i1.push_back(gd(Ui, r, 0, A + (int64_t)p0 * m, m, 0, nullptr, 1, S2, r, p0, w, p0, 1.0,
                            0.0));
            i2.push_back(gd(Dp, r, 0, S1, 64, 0, nullptr, 1, Li + p0, r, w, p0, w, -1.0, 0.0));
            i2.push_back(gd(S2, r, 0, Up, r, 0, nullptr, 1, Ui + (int64_t)p0 * r, r, p0, w, w, -1.0,
                            0.0));
          }
          continue;
        }
        pd.push_back({A + p0 + (int64_t)p0 * m, m, w, Dp, r, h * (1 << 20) + b});
        if (rows > 0) {
          double* A21 = A + p0 + w + (int64_t)p0 * m;
          double* A22 = A + p0 + w + (int64_t)(p0 + w) * m;
          tr.push_back(gd(A21, m, 0, Dp, r, 1, nullptr, 1, TA, r, rows, w, w, 1.0, 0.0));
          sy.push_back(gd(TA, r, 0, TA, r, 1, A22, m, A22, m, rows, rows, w, -1.0, 1.0));
          bk.push_back({TA, A21, rows, w, r, m, 0});
        }
        if (p0 > 0) {
          i1.push_back(gd(A + p0, m, 0, Li, r, 0, nullptr, 1, TA, 64, w, p0, p0, 1.0, 0.0));
          i2.push_back(gd(Dp, r, 0, TA, 64, 0, nullptr, 1, Li + p0, r, w, p0, w, -1.0, 0.0));
        }
      }
      if (!upload(c, S.ch_panel[pi], pd, st) || !up_g(S.ch_trsm[pi], tr) ||
          !up_g(S.ch_syrk[pi], sy) || !upload(c, S.ch_back[pi], bk, st) ||
          !up_g(S.ch_inv1[pi], i1) || !up_g(S.ch_inv2[pi], i2))
        return H2_ERR_ALLOC;
    }
    S.qr.max_rows = 0;
    S.max_k = 0;
    for (auto& q : qr) {
      S.qr.max_rows = std::max(S.qr.max_rows, q.m);
      if (q.m > 0) S.max_k = std::max(S.max_k, q.k);
    }
    // blocked QR: per panel J..J+w-1, Z = U_p^T W_t (into P, ld w) and
    // W_t -= V_p Z, W_t = rows J.. of the trailing columns
    S.qr_w = qr_panel_width(S.qr.max_rows);
    {
      const int w = S.qr_w, npan = (S.max_k + w - 1) / w;
      S.g_pz.assign(npan, {});
      S.g_pu.assign(npan, {});
      for (int pp = 0; pp < npan; ++pp) {
        const int J = pp * w;
        std::vector<GemmDesc> z, u;
        for (auto& q : qr) {
          if (q.m == 0 || q.k <= J) continue;
          const int m = q.m, wj = std::min(w, q.k - J), L = m - J, N = q.k - J - wj;
          if (N <= 0) continue;
          double* Wt = q.W + J + (int64_t)(J + wj) * m;
          z.push_back(gd(q.tmpB + J, m, 1, Wt, m, 0, nullptr, 1, q.P, wj, wj, N, L, 1.0, 0.0));
          u.push_back(gd(q.tmpA + J + (int64_t)J * m, m, 0, q.P, wj, 0, Wt, m, Wt, m, L, N, wj,
                         -1.0, 1.0));
        }
        if (!up_g(S.g_pz[pp], z) || !up_g(S.g_pu[pp], u)) return H2_ERR_ALLOC;
      }
    }
    // T above its diagonal blocks: Y = T[0:q0,0:q0] G[0:q0,q] (into TB),
    // T[0:q0,q] = -Y T_qq
    const int nqb = (S.max_k + 63) / 64;
    S.g_t1.assign(nqb, {});
    S.g_t2.assign(nqb, {});
    for (int qb = 1; qb < nqb; ++qb) {
      const int q0 = 64 * qb;
      std::vector<GemmDesc> t1, t2;
      for (auto& q : qr) {
        if (q.m == 0 || q.k <= q0) continue;
        const int k = q.k, w = std::min(64, k - q0);
        t1.push_back(gd(q.P, k, 0, q.P + (int64_t)q0 * k, k, 0, nullptr, 1, q.tmpB, q0, q0, w, q0,
                        1.0, 0.0));
        t2.push_back(gd(q.tmpB, q0, 0, q.P + q0 + (int64_t)q0 * k, k, 0, nullptr, 1,
                        q.P + (int64_t)q0 * k, k, q0, w, w, -1.0, 0.0));
      }
      if (!up_g(S.g_t1[qb], t1) || !up_g(S.g_t2[qb], t2)) return H2_ERR_ALLOC;
    }
  }
  // root plan: save, then blocked Cholesky panels
  {
    // L == 0: root <- dense block; all: keep a copy of the assembled root
    std::vector<CopyDesc> sv;
    for (auto& in : c.ins)
      if (in.n0 > 0) {
        if (in.tree.L == 0) {
          sv.push_back({in.dRootOrig, in.dRoot, in.n0, in.n0, in.n0, in.n0, 0});
          sv.push_back({in.dRootOrig, in.dRootA, in.n0, in.n0, in.n0, in.n0, 0});
        } else {
          sv.push_back({in.dRoot, in.dRootA, in.n0, in.n0, in.n0, in.n0, 0});
        }
      }
    if (!upload(c, c.r_save, sv, st)) return H2_ERR_ALLOC;
    const int np = (max_n0 + 63) / 64;
    c.r_panel.resize(np);
    c.r_trsm.resize(np);
    c.r_syrk.resize(np);
    c.r_back.resize(np);
    c.r_inv1.resize(np);
    c.r_inv2.resize(np);
    for (int pi = 0; pi < np; ++pi) {
      const int p = pi * 64;
      std::vector<PanelDesc> pd;
      std::vector<GemmDesc> tr, sy;
      std::vector<CopyDesc> bk;
      for (int t = 0; t < c.n_inst; ++t) {
        Instance& in = c.ins[t];
        const int n = in.n0;
        if (n <= p) continue;
        const int nbk = std::min(64, n - p);
        double* A = in.dRoot;
        double* Xpp = in.dRootX + p + (int64_t)p * n;  // L_pp^{-1}, ld n
        const int rows = n - p - nbk;
        if (c.lu) {
          double* Upp = in.dRootUi + p + (int64_t)p * n;  // U_pp^{-1}, ld n
          pd.push_back({A + p + (int64_t)p * n, n, nbk, Xpp, n, (1023 << 20) + t, Upp, n});
          if (rows > 0) {
            double* A21 = A + (p + nbk) + (int64_t)p * n;
            double* A12 = A + p + (int64_t)(p + nbk) * n;
            double* A22 = A + (p + nbk) + (int64_t)(p + nbk) * n;
            double* S1 = in.dPan;                     // rows x nbk, ld n
            double* S2 = in.dPan + 64 * (int64_t)n;   // nbk x rows, ld 64
            tr.push_back(gd(A21, n, 0, Upp, n, 0, nullptr, 1, S1, n, rows, nbk, nbk, 1.0, 0.0));
            tr.push_back(gd(Xpp, n, 0, A12, n, 0, nullptr, 1, S2, 64, nbk, rows, nbk, 1.0, 0.0));
            sy.push_back(gd(S1, n, 0, S2, 64, 0, A22, n, A22, n, rows, rows, nbk, -1.0, 1.0));
            bk.push_back({S1, A21, rows, nbk, n, n, 0});
            bk.push_back({S2, A12, nbk, rows, 64, n, 0});
          }
          continue;
        }
        pd.push_back({A + p + (int64_t)p * n, n, nbk, Xpp, n, (1023 << 20) + t});
        if (rows > 0) {
          double* A21 = A + (p + nbk) + (int64_t)p * n;
          double* A22 = A + (p + nbk) + (int64_t)(p + nbk) * n;
          tr.push_back(gd(A21, n, 0, Xpp, n, 1, nullptr, 1, in.dPan, n,
                          rows, nbk, nbk, 1.0, 0.0));
          sy.push_back(gd(in.dPan, n, 0, in.dPan, n, 1, A22, n, A22, n, rows, rows, nbk, -1.0, 1.0));
          bk.push_back({in.dPan, A21, rows, nbk, n, n, 0});
        }
      }
      if (!upload(c, c.r_panel[pi], pd, st) || !upload_gemm(c, c.r_trsm[pi], tr, st) ||
          !upload_gemm(c, c.r_syrk[pi], sy, st) || !upload(c, c.r_back[pi], bk, st))
        return H2_ERR_ALLOC;
      // block row p of X = L^{-1}: X_{p,<p} = -X_pp (L_{p,<p} X_{<p,<p})
      // (T in the panel scratch, ld 64), after the whole factorization
      std::vector<GemmDesc> i1, i2;
      for (int t = 0; pi > 0 && t < c.n_inst; ++t) {
        Instance& in = c.ins[t];
        const int n = in.n0;
        if (n <= p) continue;
        const int nbk = std::min(64, n - p);
        i1.push_back(gd(in.dRoot + p, n, 0, in.dRootX, n, 0, nullptr, 1, in.dPan, 64, nbk, p, p,
                        1.0, 0.0));
        i2.push_back(gd(in.dRootX + p + (int64_t)p * n, n, 0, in.dPan, 64, 0, nullptr, 1,
                        in.dRootX + p, n, nbk, p, nbk, -1.0, 0.0));
        if (c.lu) {
          // block column p of U^{-1}: Y_{<p,p} = -(Y_{<p,<p} U_{<p,p}) Y_pp
          double* T2 = in.dPan + 64 * (int64_t)n;  // p x nbk, ld n
          i1.push_back(gd(in.dRootUi, n, 0, in.dRoot + (int64_t)p * n, n, 0, nullptr, 1, T2, n, p,
                          nbk, p, 1.0, 0.0));
          i2.push_back(gd(T2, n, 0, in.dRootUi + p + (int64_t)p * n, n, 0, nullptr, 1,
                          in.dRootUi + (int64_t)p * n, n, p, nbk, nbk, -1.0, 0.0));
        }
      }
      if (!upload_gemm(c, c.r_inv1[pi], i1, st) || !upload_gemm(c, c.r_inv2[pi], i2, st))
        return H2_ERR_ALLOC;
    }
    // root^{-1} = X^T X (LU variant: U^{-1} L^{-1}): the root solve of the
    // substitution is one product
    std::vector<GemmDesc> fl;
    for (auto& in : c.ins)
      if (in.n0 > 0) {
        if (c.lu)
          fl.push_back(gd(in.dRootUi, in.n0, 0, in.dRootX, in.n0, 0, nullptr, 1, in.dRinv, in.n0,
                          in.n0, in.n0, in.n0, 1.0, 0.0));
        else
          fl.push_back(gd(in.dRootX, in.n0, 1, in.dRootX, in.n0, 0, nullptr, 1, in.dRinv, in.n0,
                          in.n0, in.n0, in.n0, 1.0, 0.0));
      }
    if (!upload_gemm(c, c.r_full, fl, st)) return H2_ERR_ALLOC;
  }
  return H2_OK;
}

}  // namespace h2
