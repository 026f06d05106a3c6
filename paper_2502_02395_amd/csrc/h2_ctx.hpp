// The handle behind h2_handle: host structure, device arenas and the
// precomputed work lists of every launch of factor, solve and matvec.
#pragma once

#include <climits>
#include <memory>

#include "h2_internal.hpp"
#include "tree.hpp"

namespace h2 {

// A launch-ready batch of descriptors living in device memory.
template <class T>
struct Batch {
  T* d = nullptr;          // descriptors
  int* toff = nullptr;     // eval: tile prefix (count + 1); GEMM: (item, tile) map of the shape in use
  int count = 0;
  int tiles = 0;
  int max_rows = 0;        // thin / gather: row extent for the grid
  // GEMM batches: (item, tile) maps of every tile shape, and the one in use
  int* toffs[GEMM_NCFG] = {};
  int tiles_c[GEMM_NCFG] = {};
  int cfg = 0;
  int tA = 0, tB = 0;      // transposes shared by every item of the list
  int f32io = 0;           // GEMM list on FP32 operands: 1 FP32 results, 2 FP64 results
  int terms = 0;           // FP32-operand list on the BF16 matrix cores: 1 or 3 terms
                           // (0: FP32 matrix cores)
  void use(int c) { cfg = c; toff = toffs[c]; tiles = tiles_c[c]; }
};

// A planned neighbour gather (see GatherPlan): chunk and reduction
// descriptors, and the algorithmic bytes of one pass with one rhs.
struct GSet {
  Batch<GChunk> ch;
  Batch<GRed> rd;
  Batch<int64_t> offs;
  int max_rows = 0;
  int64_t plen = 0;
  double bytes_ch_mat = 0.0, bytes_ch_vec = 0.0, bytes_rd = 0.0;
};
struct GList {
  GSet n;                                  // chunks of 64 rows (128 for FP32 copies)
  GSet w;                                  // wide chunks (up to 4 rows per lane) for
                                           // nrhs <= GATHER_WIDE_NR
  int esz = 8;                             // bytes per block element: 8, or 4 / 2
                                           // for FP32 / BF16 copies
  bool has_w = false;
  bool v16 = false;                        // n reads packed BF16 copies (GatherPlan::v16)
  int kind = -1;                           // timing class (h2_stats); -1: by esz
  const GSet& pick(int nrhs) const { return has_w && nrhs <= GATHER_WIDE_NR ? w : n; }
};

// One height step h above the leaves: level L_t - h of every instance t with
// L_t - h >= 1.  Boxes are ordered instance-major, box-minor.
struct Step {
  int h = 0;
  int nbox = 0;
  std::vector<int> inst, idx, lvl, m, k;
  std::vector<int64_t> boff;               // prefix of m  (active ids, vectors)
  std::vector<int64_t> koff;               // prefix of k  (skeleton ids, skeleton vectors)
  std::vector<int64_t> roff;               // prefix of r = m - k
  int64_t sum_m = 0, sum_k = 0, sum_r = 0;
  // unordered near pairs (i >= j) and far pairs (i > j), step-local indices
  std::vector<int> np_i, np_j, fp_i, fp_j;
  std::vector<int> diag_pair;              // near-pair index of (b, b)
  std::vector<int64_t> poff;               // near-pair block offsets (m_i m_j prefix)
  std::vector<int64_t> soff;               // far-pair coupling offsets (k_i k_j prefix)
  std::vector<int64_t> qoff, rkoff, lioff; // m^2, k^2, r^2 prefixes
  std::vector<int64_t> voff;               // box offsets in the level vectors
  int64_t vld = 0;                         // their leading dimension
  // host copies of ids
  std::vector<int64_t> B;                  // active ids, sum_m
  std::vector<int64_t> SK;                 // skeleton ids, sum_k
  // device buffers
  int64_t* dB = nullptr;
  int64_t* dSK = nullptr;
  double* dU = nullptr;                    // U arena: box b at U capacity m_b x kcap_b
  std::vector<double*> Uptr;               // U_i (m x k, ld m) of every box
  std::vector<int> kcap;                   // predicted U capacity (columns)
  double* dS = nullptr;                    // couplings at soff
  double* dD = nullptr;                    // input near blocks at poff
  double* dF = nullptr;                    // transformed near blocks at poff
  double* dT2 = nullptr;                   // pair scratch at poff
  double* dT3 = nullptr;                   // far scratch at soff
  double *dQ = nullptr, *dP = nullptr, *dTA = nullptr, *dTB = nullptr;  // at qoff
  double* dW = nullptr;                    // QR workspace at qoff
  double* dTau = nullptr;                  // Householder scalars at koff
  float *dF32 = nullptr, *dP32 = nullptr;  // FP32 copies of F and P for the substitution
  float* dPr32 = nullptr;                  // LU variant: FP32 copy of the right basis P'
  unsigned short *dF16 = nullptr, *dP16 = nullptr;  // packed BF16 copies (solve_prec BF16)
  std::vector<CopyMap> cmF, cmP;           // their layout (sorted by source block)
  Batch<CvtBlk> cvF16, cvP16;              // their conversion blocks
  Batch<int> cvF16_first, cvP16_first;     // segment of each 256-group block
  int64_t cvF16_groups = 0, cvP16_groups = 0;  // their 8-row column groups
  float *dD32 = nullptr, *dT232 = nullptr; // FP32 near blocks and pair scratch (FP32 pairs)
  float *dR32 = nullptr, *dS32 = nullptr, *dT332 = nullptr;  // FP32 R, far couplings, scratch
  Batch<ConvDesc> cv_fii;                  // F_ii -> FP32 (diagonal blocks)
  Batch<ConvDesc> cv_dii;                  // D_ii -> FP32 above the leaves
  Batch<CopyDesc> c_merge32;               // merge from FP32 transformed blocks
  Batch<CopyDesc> c_merge3232;             // FP32 blocks into FP32 parent near blocks
  double* dR = nullptr;                    // at rkoff
  double* dLi = nullptr;                   // at lioff
  // LU variant: right basis P'_i = [Q^S | Q^R U(r)_ii^{-1}] (at qoff), U(r)^{-1}
  // (at lioff), panel scratch (128 r per box, at 128 roff)
  double *dPr = nullptr, *dUi = nullptr, *dLUs = nullptr;
  // factor work lists
  Batch<GemmDesc> g_w;                     // W = D_i U_i (upper steps)
  Batch<GemmDesc> g_qr1, g_qr2, g_qr3;     // compact-WY Q: V^T V, T V^T, -V (T V^T)
  std::vector<Batch<GemmDesc>> g_t1, g_t2; // T blocks above the diagonal, per block column
  int qr_w = 1;                            // QR panel width of this level
  std::vector<Batch<GemmDesc>> g_pz, g_pu; // per panel: Z = U_p^T W_t, W_t -= V_p Z
  int max_k = 0;
  Batch<CopyDesc> c_w;                     // W = U (leaf step)
  Batch<BoxDev> qr;
  Batch<GemmDesc> g_diag1, g_diag2;        // D_ii Q, Q^T (.)
  // blocked Cholesky of the RR blocks and the explicit inverse of the factor,
  // per 64-wide panel: diagonal panel, TRSM, trailing update, write-back;
  // then inverse block rows X_p = -D_p (L_p,<p X_<p)
  std::vector<Batch<PanelDesc>> ch_panel;
  std::vector<Batch<GemmDesc>> ch_trsm, ch_syrk, ch_inv1, ch_inv2;
  std::vector<Batch<CopyDesc>> ch_back;
  Batch<CopyDesc> c_ps;                    // P^S = Q^S
  Batch<GemmDesc> g_v;                     // V = Q^R Linv^T, L(s)_ii
  Batch<GemmDesc> g_v2;                    // LU variant: Q^R U^{-1}, L(s)_ii, U(s)_ii
  Batch<GemmDesc> g_schur;                 // SS_ii -= L(s) L(s)^T
  Batch<GemmDesc> g_pair1, g_pair2;        // D_ij P_j, P_i^T (.)
  Batch<GemmDesc> g_far1, g_far2;          // R_i S_ij, (.) R_j^T into the parent
  Batch<GemmDesc> g_far3;                  // FP32 pairs: (.) R_j^T into FP64 parent blocks
  Batch<CopyDesc> c_merge;
  // solve / matvec work lists (built for NRHS_MAX columns)
  GList t_fwd, t_bwd;                      // P^T b, P [xS; s]
  GList g_yr, g_cs, g_t, g_s;              // neighbour gathers of the substitution
  GList t_up, t_down;                      // U^T x, U y
  // solve vectors (ld = sum_m or sum_r), NRHS_MAX columns
  double *v_in = nullptr, *v_d = nullptr, *v_out = nullptr, *v_yr = nullptr, *v_t = nullptr;
  double *v_xh = nullptr, *v_yh = nullptr;  // matvec skeleton vectors (ld sum_k)
};

struct Instance {
  int64_t n = 0, pbase = 0;                // points, global id base
  KernelDev kern{};
  Tree tree;
  std::vector<int64_t> rank;               // position of each local point in pi
  int n0 = 0;                              // root size
  std::vector<int64_t> root_ids;
  double* dRoot = nullptr;                 // n0 x n0 (factored in place)
  double* dRootA = nullptr;                // copy of the assembled root block
  double* dRootOrig = nullptr;             // L == 0: the dense kernel block
  double* dRootX = nullptr;                // n0 x n0: L^{-1} of the root Cholesky factor
  double* dRinv = nullptr;                 // n0 x n0: root^{-1} = L^{-T} L^{-1}
                                           // (LU variant: U^{-1} L^{-1})
  double* dRootUi = nullptr;               // LU variant: n0 x n0 U^{-1} of the root
  double* dPan = nullptr;                  // n0 x 64 panel scratch
  double* v_root = nullptr;                // n0 x NRHS_MAX
};

constexpr int NRHS_MAX = 16;

struct Ctx {
  h2_params prm{};
  int n_inst = 0;
  int dim = 3;
  int64_t N = 0;
  int H = 0;                               // max levels
  bool lu = false;                         // the LU variant (params.factor_lu)
  std::vector<Instance> ins;
  std::vector<Step> steps;                 // h = 0 .. H-1
  double* dX = nullptr;                    // N x dim points (original order per instance)
  KernelDev* dKern = nullptr;
  int64_t* dPermG = nullptr;               // global tree position -> global id
  int* dFail = nullptr;
  double* dWs = nullptr;                   // reduction workspace
  double* dScal = nullptr;                 // small scalars
  // root work lists (per panel step p)
  std::vector<Batch<PanelDesc>> r_panel;
  std::vector<Batch<GemmDesc>> r_trsm, r_syrk;
  std::vector<Batch<CopyDesc>> r_back;
  Batch<CopyDesc> r_save;
  std::vector<Batch<GemmDesc>> r_inv1, r_inv2;  // block rows of L^{-1}
  Batch<GemmDesc> r_full;                  // root^{-1} = X^T X
  GList g_root;                            // substitution: v_root <- root^{-1} v_root
  bool factored = false;
  bool failed = false;
  h2_stats_t st{};
  std::vector<void*> allocs;               // everything hipMalloc'd
  // tree-ordered input / output vectors (N x NRHS_MAX, ld N); the leaf step
  // and root-only instances read and write them directly
  double *vt_in = nullptr, *vt_out = nullptr;
  Batch<CopyDesc> r_in, r_out;             // root-only instances <-> v_root
  GList t_root;                            // root-only instances: matvec
  GList g_mv32;                            // the same list on FP32 copies of the leaf
                                           // near blocks and couplings (matvec_prec FP32)
  GList g_mv;                              // matvec: couplings y^ = S x^ of every level
                                           // and the leaf near field y = D x
  // refinement vectors (N x NRHS_MAX)
  double *w_x = nullptr, *w_r = nullptr, *w_z = nullptr, *w_p = nullptr, *w_q = nullptr, *w_t = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;  // pair-transform timing
  double pair_flops = 0.0;                 // canonical flops of all pair transforms
  int pair_launches = 0;
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_def = nullptr;
  // captured substitutions and operator products of the solve (use_graph,
  // untimed solves): one per (operation, input, output, columns, precision,
  // partial buffer)
  struct SolveGraph {
    int op;                                // 0 substitution, 1 H^2 product
    const double* in;
    double* out;
    int nc;
    bool lowp;
    const double* part;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<SolveGraph> sgraphs;
  hipStream_t graph_stream = nullptr;      // capture and replay (never the null stream)
  // gather timing (params.timing): per gather four events, the start and end
  // of its chunk launch and of its reduction launch (marked by the launches'
  // own dispatches), and the bytes each timed launch moves
  std::vector<hipEvent_t> fev;             // factor phases: (before, after) pairs
  std::vector<int> fev_phase;
  size_t fev_used = 0;
  std::vector<hipEvent_t> gev;
  size_t gev_used = 0;
  bool gtime = false;
  std::vector<double> gbytes;              // per timed gather: chunks, reduction
  std::vector<int> gkind;                  // per timed gather: 0 FP64 blocks, 1 copies
  double* dPart = nullptr;                 // gather partial products
  int64_t part_len = 0;                    // longest list's partials, one rhs
  int part_nrhs = 0;                       // right-hand sides dPart holds
  double* part_cur = nullptr;              // partials the gathers of the current
                                           // solve / matvec call use (dPart, or the
                                           // no-allocation call's fixed array)
  hipEvent_t ev_g0 = nullptr, ev_g1 = nullptr;  // caller stream <-> graph_stream ordering

  // the caller's device allocator (h2_params.allocator); alloc == NULL means
  // hipMalloc / hipFree
  h2_allocator ua{};

  ~Ctx();
  void* dev_alloc(size_t bytes) {
    if (ua.alloc) return ua.alloc(bytes, ua.user);
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
  void dev_free(void* p) {
    if (ua.alloc) ua.free(p, ua.user);
    else (void)hipFree(p);
  }
  template <class T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    void* p = dev_alloc(count * sizeof(T));
    if (!p) return nullptr;
    allocs.push_back(p);
    return static_cast<T*>(p);
  }
  // the device must have finished with p (callers synchronize first)
  void free_one(void* p) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p) {
        dev_free(p);
        allocs[i] = allocs.back();
        allocs.pop_back();
        return;
      }
  }
};

// Upload a host descriptor vector (and tile prefix for tiled batches).
template <class T>
bool upload(Ctx& c, Batch<T>& b, const std::vector<T>& v, hipStream_t st,
            const std::vector<int>* toff = nullptr) {
  b.count = (int)v.size();
  if (v.empty()) return true;
  b.d = c.alloc<T>(v.size());
  if (!b.d) return false;
  if (hipMemcpyAsync(b.d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess)
    return false;
  if (toff) {
    b.toff = c.alloc<int>(toff->size());
    if (!b.toff) return false;
    if (hipMemcpyAsync(b.toff, toff->data(), toff->size() * sizeof(int), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return false;
    b.tiles = toff->back();
  }
  // the host vectors may die after return: wait for the copies
  return hipStreamSynchronize(st) == hipSuccess;
}


// Upload a GEMM batch with the tile prefix of every tile shape (shape 0 in use).
inline bool upload_gemm(Ctx& c, Batch<GemmDesc>& b, const std::vector<GemmDesc>& v,
                        hipStream_t st);
inline std::vector<int> eval_tiles(const std::vector<EvalDesc>& v) {
  std::vector<int> off(v.size() + 1, 0);
  for (size_t i = 0; i < v.size(); ++i) {
    const int tm = (v[i].nr + 63) / 64, tn = (v[i].nc + 63) / 64;
    off[i + 1] = off[i] + ((v[i].nr > 0 && v[i].nc > 0) ? tm * tn : 0);
  }
  return off;
}

inline GemmDesc gd(const double* A, int lda, int tA, const double* B, int ldb, int tB,
                   const double* C, int ldc, double* D, int ldd, int M, int N, int K,
                   double alpha, double beta) {
  GemmDesc g;
  g.A = A; g.B = B; g.C = C; g.D = D;
  g.M = M; g.N = N; g.K = K;
  g.lda = lda < 1 ? 1 : lda; g.ldb = ldb < 1 ? 1 : ldb;
  g.ldc = ldc < 1 ? 1 : ldc; g.ldd = ldd < 1 ? 1 : ldd;
  g.tA = tA; g.tB = tB; g.alpha = alpha; g.beta = beta;
  return g;
}

hipError_t run_gemm(const Batch<GemmDesc>& b, hipStream_t st, int tag = 0);
// Time every tile shape on every factor GEMM batch and keep the fastest.
h2_status autotune(Ctx& c, hipStream_t st);
hipError_t run_copy(const Batch<CopyDesc>& b, hipStream_t st);
h2_status ensure_partials(Ctx& c, int nrhs);
h2_status collect_factor_times(Ctx& c);

// defined in the orchestration sources
h2_status plan_factor(Ctx& c, hipStream_t st);
h2_status plan_solve(Ctx& c, hipStream_t st);
h2_status do_factor(Ctx& c, hipStream_t st);
h2_status do_solve_chunk(Ctx& c, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs,
                         hipStream_t st);
h2_status do_matvec_chunk(Ctx& c, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs,
                          hipStream_t st, bool lowp = false);
double now_seconds();

hipError_t launch_set_int(int* p, int v, hipStream_t st);
// The eight geometry features of box i at level l of instance t (see mlp.hip).
void box_features_host(const Ctx& c, int t, int l, int i, float* f);

inline bool upload_gemm(Ctx& c, Batch<GemmDesc>& b, const std::vector<GemmDesc>& v,
                        hipStream_t st) {
  if (v.empty()) { b.count = 0; return true; }
  b.tA = v[0].tA;
  b.tB = v[0].tB;
  for (auto& g : v)
    if (g.tA != b.tA || g.tB != b.tB) return false;  // lists are built uniform
  if (!upload(c, b, v, st)) return false;
  for (int q = 0; q < GEMM_NCFG; ++q) {
    const std::vector<int> map = gemm_tile_map(v, GEMM_BM[q], GEMM_BN[q]);
    b.toffs[q] = c.alloc<int>(map.size());
    if (!b.toffs[q]) return false;
    if (!map.empty() &&
        hipMemcpy(b.toffs[q], map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice) !=
            hipSuccess)
      return false;
    b.tiles_c[q] = (int)(map.size() / 2);
  }
  b.use(0);
  return true;
}

}  // namespace h2

struct h2_ctx {
  std::unique_ptr<h2::Ctx> c;
};
