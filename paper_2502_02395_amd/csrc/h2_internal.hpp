// Internal declarations shared by the host orchestration (*.cpp) and the HIP
// kernels (*.hip) of the H^2-ULV library.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/h2.h"

namespace h2 {

// ---------------------------------------------------------------- device types

struct KernelDev {          // kernel function parameters of one instance
  int id;
  double delta, kappa, ell, nugget;
  double beta;              // drift kernel: skew strength (its transpose: -beta)
};

// One item of a batched GEMM:  D = alpha * op(A) op(B) + beta * C
// (column-major; op(A) is M x K, op(B) is K x N; C may alias D).
struct GemmDesc {
  const double* A;
  const double* B;
  const double* C;
  double* D;
  int M, N, K;
  int lda, ldb, ldc, ldd;
  int tA, tB;
  double alpha, beta;
};

// One item of a batched kernel-matrix evaluation: out(r, c) = G(x_rows[r], x_cols[c])
struct EvalDesc {
  const int64_t* rows;      // global point ids
  const int64_t* cols;
  double* out;
  int nr, nc, ld;
  int inst;
};

// One item of a batched block copy: dst = src (or src^T)
struct CopyDesc {
  const double* src;
  double* dst;
  int rows, cols;           // of dst
  int lds, ldd;
  int trans;                // 1: dst(r, c) = src(c, r)
};

// Factor blocks of one box (pointers into the handle's arenas).
struct BoxDev {
  int m, k;                 // active size, rank
  int inst;
  double* Q;                // m x m orthogonal completion
  double* P;                // m x m [Q^S | Q^R L(r)^{-T}]
  double* Rf;               // k x k triangular factor of D_i U_i
  double* Linv;             // r x r inverse Cholesky factor of the RR block
  double* tmpA;             // m x m scratch (the QR's explicit V first)
  double* tmpB;             // m x m transformed diagonal block
  double* W;                // m x k QR input, overwritten
  double* tau;              // k Householder scalars
};

constexpr int QR_MMAX = 6911;  // row limit of the QR panel kernel (m + 1 doubles per panel column)

// ------------------------------------------------------------- launch wrappers
// All wrappers enqueue on `st`; they return hipSuccess or the launch error.

// tag 1 launches the same kernel under the symbol gemm_f64_pair_kernel;
// cfg selects the tile shape: 0 = 64x64, 1 = 128x64, 2 = 128x128 (the tile
// prefix d_tile_off must have been computed for that shape).
// Tile shapes (BM x BN, K staged TK at a time): 64x64x16, 128x64x16,
// 128x128x16, 64x64x32.
constexpr int GEMM_NCFG = 4;
constexpr int GEMM_BM[GEMM_NCFG] = {64, 128, 128, 64};
constexpr int GEMM_BN[GEMM_NCFG] = {64, 64, 128, 64};
// Every item of one launch must have the transposes tA, tB.  d_tile_map holds
// two ints per output tile: the item and the tile's index within the item
// (gemm_tile_map, for the launch's tile shape), so a workgroup finds its work
// with one load.
hipError_t launch_gemm(const GemmDesc* d_desc, const int* d_tile_map, int count,
                       int tiles, hipStream_t st, int tag, int cfg, int tA, int tB);
// Same work lists on FP32 MFMA (prec = H2_PREC_FP32: operands rounded to FP32,
// FP32 accumulation, FP64 in and out, 64 x 64 tiles; any other prec runs the
// FP64 kernel).
hipError_t launch_gemm_lp(const GemmDesc* d_desc, const int* d_tile_map, int count,
                          int tiles, int prec, hipStream_t st, int tag, int tA, int tB);
// FP32 operands (pointers in the descriptors hold float arrays), FP32 MFMA
// with FP32 accumulation, beta = 0, results in FP32 (out64 = false) or FP64;
// the same tile maps and shapes (cfg 3 runs as cfg 0).
hipError_t launch_gemm_f32io(const GemmDesc* d_desc, const int* d_tile_map, int count,
                             int tiles, hipStream_t st, int cfg, int tA, int tB,
                             bool out64 = false);
// The same FP32-operand work lists on the BF16 matrix cores: each operand
// element split into BF16 high and low parts; terms = 1 multiplies the high
// parts only, terms = 3 adds both cross terms (about 17-bit operands); FP32
// accumulation, results in FP32 (out64 = false) or FP64.
hipError_t launch_gemm_bf16s(const GemmDesc* d_desc, const int* d_tile_map, int count, int tiles,
                             hipStream_t st, int cfg, int tA, int tB, bool out64, int terms);
// Host: the (item, tile) map of a work list for BM x BN tiles.
inline std::vector<int> gemm_tile_map(const std::vector<GemmDesc>& v, int BM, int BN) {
  std::vector<int> map;
  for (size_t i = 0; i < v.size(); ++i) {
    if (v[i].M <= 0 || v[i].N <= 0) continue;
    const int nt = ((v[i].M + BM - 1) / BM) * ((v[i].N + BN - 1) / BN);
    for (int t = 0; t < nt; ++t) {
      map.push_back((int)i);
      map.push_back(t);
    }
  }
  return map;
}
hipError_t launch_eval(const EvalDesc* d_desc, const int* d_tile_off, int count,
                       int tiles, const double* X, int dim, const KernelDev* kern,
                       hipStream_t st);
hipError_t launch_copy(const CopyDesc* d_desc, int count, hipStream_t st);
// The same copies with an FP32 source (src holds a float pointer), into FP64
// or (dst32) FP32 destinations.
hipError_t launch_copy_f32(const CopyDesc* d_desc, int count, hipStream_t st,
                           bool dst32 = false);
// Contiguous conversions FP64 -> FP32 (to32) or FP32 -> FP64.
struct ConvDesc {
  const void* src;
  void* dst;
  int64_t n;
  int to32;
};
hipError_t launch_cvt_list(const ConvDesc* d, int count, hipStream_t st);

// QR of W (m x k) with R (k x k) and the full Q (m x m) in compact WY form:
// qr_panel factors one panel (V into tmpA, tau, R, U_p = V_p T_p into tmpB)
// and GEMMs update the trailing columns, panel after panel; a GEMM writes
// G = V^T V into P;
// qr_tdiag turns the diagonal 64-blocks of G into those of T in place and
// GEMMs the blocks above them; GEMMs write Q = -V (T V^T); qr_diag adds the
// identity.  One workgroup per box (per box and block for qr_tdiag).
// Panel width for a level whose largest box has max_m rows (the panel of
// max_m x w doubles must fit in LDS), and one panel J .. J+w-1 of every box.
int qr_panel_width(int max_m);
hipError_t launch_qr_panel(const BoxDev* boxes, int nbox, int max_m, int J, int w,
                           hipStream_t st);
hipError_t launch_qr_tdiag(const BoxDev* boxes, int nbox, int max_k, hipStream_t st);
hipError_t launch_qr_diag(const BoxDev* boxes, int nbox, hipStream_t st);
// Gauss-Seidel approximation of X = A^{-1} B (Section 3.5): A n x n SPD
// (lda), B n x m (ldb), X n x m (ldx), sweeps forward sweeps from X = 0; one
// workgroup per block, one thread per column of X, the iterate held row-major
// in the scratch W (n x m) so that a row's reads are coalesced.  A
// non-positive diagonal reports code through *fail.
struct GsDesc {
  const double* A;
  const double* B;
  double* X;
  double* W;
  int n, m, lda, ldb, ldx;
  int code;
};
hipError_t launch_gauss_seidel(const GsDesc* d_desc, int count, int sweeps, int* fail,
                               hipStream_t st);
// Column-pivoted QR interpolative decomposition of X (s x m, ld s), one box
// per workgroup.  Free mode: rank by eps; forced mode: skel[] given.
struct IdDesc {
  double* X;                // s x m workspace; on exit T = R_11^{-1} R_12 in rows 0..k-1
  double* U;                // output basis m x k (ld m), written only if k <= kcap
  int32_t* piv;             // m pivot positions (output)
  int32_t* k_out;           // rank (output)
  const int32_t* skel;      // forced skeleton positions (NULL = free)
  int s, m, kforced;
  int kcap;                 // U capacity in columns (0 = unlimited)
};
// max_m: the largest m of the list (sizes the LDS; at most 4096).
hipError_t launch_cpqr_id(const IdDesc* d_desc, int count, double eps,
                          int max_rank, int max_m, hipStream_t st);
// Write U for IDs whose rank exceeded the capacity given to cpqr_id.
hipError_t launch_id_write_u(const IdDesc* d_desc, int count, hipStream_t st);


// Neighbour gathers of the substitution and the matvec:
//   y_i = base_i + alpha * sum_nbr op(B_nbr) x_nbr
// with op(B) = B ("direct": B is rows x cols, ld ldB) or B^T ("trans": B is
// cols x rows).  base == NULL means zero; base may alias y.  Lists are given
// per box (GatherBox with neighbour ranges into a GatherNbr array) and are
// planned (plan_gather) into
//   * chunks: one wave per 64-row chunk (128 rows for FP32 or BF16 copies,
//     two rows per lane) and, where the plan asks for segments, per seg-column
//     segment of each stored block M.  The wave reads its part of M once and
//     forms the direct product M x_d for those rows and/or the transposed
//     product M^T x_t over those rows; a block that is used directly by one
//     box and transposed by another is read once for both.  Segments bound
//     the serial column walk of one wave: the few, large blocks of the upper
//     levels otherwise leave a launch with a handful of long waves.  The
//     caller picks them per tree height, so a box gets the same arithmetic
//     in every list and handle (batched or not) it appears in;
//   * partial slots: every product writes its own slot of a partial buffer
//     (slot offsets in units of one right-hand side; with nrhs columns slot
//     s starts at off_s * nrhs, column c at off_s * nrhs + c * len);
//   * reductions: per box, y = base + alpha * (sum of its slots in a fixed
//     order), so results are deterministic.
struct GatherBox {
  double* y;
  const double* base;
  int rows, ldy, ldbase;
  double alpha;
  int d0, d1;               // direct neighbour range
  int t0, t1;               // transposed neighbour range
};
struct GatherNbr {
  const double* B;
  const double* x;
  int ldB, ldx, cols;       // cols: summation length
};
struct GChunk {
  const void* M;            // first row of the chunk (column-major, ld; FP64, FP32 or BF16)
  const double* xd;         // direct x: mc entries per rhs (ld ldxd), or NULL
  const double* xt;         // trans x: this chunk's nr entries per rhs (ld ldxt), or NULL
  int ld, ldxd, ldxt;
  int nr, mc;               // chunk rows (<= 64, <= 128 for copies), columns of M
  int dlen, drow;           // direct slot length and this chunk's first row in it
  int tlen, tcol;           // trans slot length and this chunk's first column in it
  int rpl;                  // rows per lane: nr <= 64 rpl
  int vec;                  // 1: FP64 chunk of <= 64 rows or FP32 chunk of <= 128
                            // rows of a narrow plan: with one right-hand side it
                            // is read two (FP64) or four (FP32) rows per lane
                            // with 16-byte loads (element alignment is enough)
  int64_t od, ot;           // slot offsets (one-rhs units); -1 = no such product
};
struct GRed {
  double* y;
  const double* base;
  int rows, ldy, ldbase;
  double alpha;
  int s0, s1;               // slot range in the offset array
};
// Column segments of the gathers at heights >= GATHER_SEG_FROM above the
// leaves (measured: below that the lists have enough waves and the extra
// direct slots cost more than the shorter waves gain).
constexpr int GATHER_SEG = 128;
constexpr int GATHER_SEG_FROM = 5;
// The per-box lists (P^T b, P d, U^T x, U y: one dense block per box) have
// fewer blocks per wave of work, so they take the segments from height 3
// (measured at h = 3, 4: 30-50 % shorter launches; from height 1 or 2 no
// further gain).
constexpr int GATHER_SEG_THIN_FROM = 3;
constexpr int GATHER_SEG_TOP = 32;       // the top levels: a few blocks each
constexpr int GATHER_SEG_TOP_FROM = 8;
// Wide chunks: a block's rows split evenly into chunks of at most 64 x RPL
// rows (one wave each, up to RPL rows per lane: 4 for FP32 or BF16 copies,
// 2 for FP64 blocks), so that e.g. an FP32 block of 150 rows takes one wave with
// most lanes busy instead of two with most lanes of the second idle; used
// for up to GATHER_WIDE_NR right-hand sides (the per-lane accumulators grow
// with rows x rhs).
// Measured: wide chunks win at heights GATHER_WIDE_FROM..GATHER_WIDE_TO; at
// the leaves (many small blocks) and at the top (few waves) the narrow ones
// with 16 columns per batch do.
constexpr int GATHER_WIDE_RPL32 = 4;
constexpr int GATHER_WIDE_RPL64 = 2;
constexpr int GATHER_WIDE_NR = 2;
constexpr int GATHER_WIDE_FROM = 1;
constexpr int GATHER_WIDE_TO = 6;
// Where the packed BF16 copy of one FP64 block lives.  The block (rows x
// cols, column-major, ld) is kept as up to two segments: its rows
// [0, split) from column top_c0 on (the top segment), and its rows
// [split, rows) over every column (the bottom segment; bot < 0: none).  Each
// segment is column-major with a leading dimension that is a multiple of 8
// elements, starts on a 16-byte boundary, and holds zeros below its rows, so
// that a gather can read eight rows of a column with one 16-byte load.
struct CopyMap {
  const double* src;
  int64_t ld;
  int rows, cols, split, top_c0;
  int64_t top, ld_top;      // element offsets into the copy
  int64_t bot, ld_bot;
};
// One block of a packed copy for the conversion kernel (see CopyMap): source
// element offset (into the FP64 or FP32 arena) and ld; its top segment (rows
// [0, split) of columns [c_top, cols), gt groups of 8 rows per column, at
// top) and its bottom segment (rows [split, rows) of every column, gb groups
// per column, at bot; gb = 0: none).  Its 8-row groups are numbered column by
// column from g0 (a column's top groups, then its bottom groups), so that the
// threads converting the two parts of one column are neighbours.
struct CvtBlk {
  int64_t src_off, top, bot, g0;
  int src_ld, rows, split, c_top, cols, gt, gb;
};
// A range of FP64 blocks with a reduced-precision copy: esz 4 = FP32, esz 2
// = BF16.  Without a map the copy has the same element offsets; with one
// (BF16 only, sorted by src) it is packed as the map says.
struct Rebase {
  const double* base;
  int64_t n;
  const void* copy;
  int esz;
  const std::vector<CopyMap>* map = nullptr;
};
struct GatherPlan {
  int esz = 8;                // bytes per block element: 8 FP64, 4 FP32, 2 BF16 copies
  std::vector<GChunk> chunks;
  std::vector<GRed> reds;
  std::vector<int64_t> offs;  // slot offsets, grouped per box
  int64_t plen = 0;           // partial-buffer length for one rhs
  int max_rows = 0;
  // algorithmic bytes of one pass: blocks (independent of nrhs), and vector
  // and partial traffic per rhs
  double bytes_chunks_mat = 0.0, bytes_chunks_vec = 0.0;
  double bytes_red = 0.0;
  // every chunk reads a packed BF16 copy: 16-byte aligned, ld a multiple of
  // 8, zero rows below the chunk up to the next multiple of 8
  bool v16 = false;
};
// rb non-empty: every block must lie in one of its ranges and is read from
// that range's copy (all ranges of one plan share esz; returns false
// otherwise).  seg > 0: column segments of at
// most seg columns (a multiple of 16).  wide: wide chunks (see above).
bool plan_gather(const std::vector<GatherBox>& B, const std::vector<GatherNbr>& Nv,
                 GatherPlan& out, const std::vector<Rebase>& rb = {}, int seg = 0,
                 bool wide = false);
// wide: the chunks come from a wide plan (nrhs <= GATHER_WIDE_NR required).
// esz: bytes per block element (8, 4 or 2).  v16: the plan's v16 (BF16
// chunks of 128 rows read with 16-byte loads, for one right-hand side;
// more fall back to the two-rows-per-lane kernel, which reads the packed
// copies too).  e0, e1: if set, events that the kernel's own dispatch marks
// at its start and end (its duration without a separate marker on the
// stream); the call must launch (nch > 0).
constexpr int GV16_NR = 1;
hipError_t launch_gchunks(const GChunk* ch, int nch, double* P, int nrhs, int esz,
                          hipStream_t st, bool wide = false, bool v16 = false,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// FP32 copy of n doubles.
hipError_t launch_cvt_f32(const double* src, float* dst, int64_t n, hipStream_t st);
// BF16 copy (round to nearest even) of n doubles (esz_src 8) or floats (4).
hipError_t launch_cvt_bf16(const void* src, int esz_src, unsigned short* dst, int64_t n,
                           hipStream_t st);
// Packed BF16 copy: every block of blks (device, count, g0 ascending) from
// src (FP64 or FP32 arena, esz_src 8 or 4) into dst, zero-padded; groups:
// the total number of 8-row groups; first (device, one per 256 groups): the
// block holding group 256 b.
hipError_t launch_cvt_bf16_blks(const void* src, int esz_src, const CvtBlk* blks,
                                const int* first, int count, int64_t groups,
                                unsigned short* dst, hipStream_t st);
// e0, e1 as for launch_gchunks (nred > 0 and max_rows > 0).
hipError_t launch_greduce(const GRed* rd, int nred, int max_rows, const int64_t* offs,
                          const double* P, int nrhs, hipStream_t st, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);

// Blocked Cholesky panel (nb <= 64; the root and the redundant blocks):
// factor the nb x nb diagonal block in place (L below, zeros above) and write
// the inverse of L (nb x nb, zeros above the diagonal) to dinv.
struct PanelDesc {
  double* A;                // diagonal block pointer
  int lda, nb;
  double* dinv;             // nb x nb inverse of the panel's factor (LU: of L)
  int ldd;                  // leading dimension of dinv
  int code;
  double* uinv;             // LU panels: nb x nb inverse of U (ld ldu)
  int ldu;
};
hipError_t launch_panel(const PanelDesc* d, int count, int* fail, hipStream_t st);
// Pivot-free LU of each nb x nb diagonal block (unit lower L below the
// diagonal, U on and above it, in place) and the inverses of L and U.
hipError_t launch_lu_panel(const PanelDesc* d, int count, int* fail, hipStream_t st);

// Vector permutations: dst[r + c*ldd] = src[idx[r] + c*lds]  (gather)
hipError_t launch_gather_rows(const int64_t* idx, int64_t n, int nrhs,
                              const double* src, int64_t lds, double* dst,
                              int64_t ldd, hipStream_t st);
// dst[idx[r] + c*ldd] = src[r + c*lds]  (scatter)
hipError_t launch_scatter_rows(const int64_t* idx, int64_t n, int nrhs,
                               const double* src, int64_t lds, double* dst,
                               int64_t ldd, hipStream_t st);
// out[c] = sum_i a[i, c] b[i, c] (deterministic two-stage sum; ws holds
// 256 * nrhs doubles)
hipError_t launch_coldot(const double* a, int64_t lda, const double* b, int64_t ldb,
                         int64_t n, int nrhs, double* ws, double* out, hipStream_t st);
// z = x + sgn * (alphas[c] / alphas_den[c]) * y  (NULL alpha arrays mean 1)
hipError_t launch_axpby(double* z, int64_t ldz, const double* x, int64_t ldx,
                        const double* y, int64_t ldy, int64_t n, int nrhs,
                        const double* alphas, const double* alphas_den, double sgn,
                        hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);

// MLP (FP32)
hipError_t launch_mlp_forward(const float* w, const float* x, float* y,
                              int64_t n, hipStream_t st);
hipError_t launch_mlp_grad(const float* w, const float* x, const float* t,
                           int64_t n, float* g, float* loss, hipStream_t st);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, int np,
                       int step, float lr, hipStream_t st);

// ------------------------------------------------------------------- helpers

// A device array of descriptors with its tile prefix (for GEMM / eval).
template <class T>
struct DevBatch {
  T* desc = nullptr;
  int* tile_off = nullptr;
  int count = 0;
  int tiles = 0;
};

}  // namespace h2
