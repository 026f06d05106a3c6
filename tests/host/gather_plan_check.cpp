// Host check of the neighbour-gather planner (plan_gather).  Seeded random
// gather lists are planned, and each plan is evaluated on the host the way
// the chunk and reduction kernels define it: a chunk writes M x_d into rows
// [drow, drow + nr) of its direct slot and M^T x_t into columns
// [tcol, tcol + mc) of its transposed slot; a reduction writes
// base + alpha * (sum of its box's slots).  Blocks and vectors hold small
// integers, so every sum is exact in any order and the result must equal the
// gathers' definition
//     y_i = base_i + alpha_i * sum_nbr op(B_nbr) x_nbr
// bit for bit.  This holds for FP64 blocks, FP32 copies split over two
// ranges, and packed BF16 copies (a top segment of the first rows of the
// later columns and a bottom segment of the remaining rows of every
// column), for narrow and wide plans, with and without column segments, and
// for one to three right-hand sides.
//
// Also checked: every partial-slot entry is written exactly once; every
// block element is read exactly once, including a block used directly by
// one box and transposed by another; chunk shapes and flags; the plan's
// algorithmic byte count; every read lies inside the block's copy, never in
// padding or gaps (which hold NaN); and, for the 16-byte BF16 plans, that
// rows up to the next multiple of 8, which those loads also read, are in
// bounds and finite.  Finally, the inputs the planner must refuse are
// refused.
//
// Prints one line per failure and a summary; exit status 0 when every case
// passes.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "../../paper_2502_02395_amd/csrc/h2_internal.hpp"

using namespace h2;

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                                   \
  do {                                                                     \
    if (!(cond)) {                                                         \
      if (g_fail < 25) {                                                   \
        std::printf("FAIL line %d [%s]: ", __LINE__, g_case);              \
        std::printf(__VA_ARGS__);                                          \
        std::printf("\n");                                                 \
      }                                                                    \
      ++g_fail;                                                            \
    }                                                                      \
  } while (0)
char g_case[160] = "";

const double NaN = std::numeric_limits<double>::quiet_NaN();

struct Rng {
  std::mt19937_64 g;
  explicit Rng(uint64_t s) : g(s) {}
  int uni(int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(g); }
  bool coin(int num, int den) { return uni(0, den - 1) < num; }
};

uint16_t bf16_bits(double v) {  // exact for the small integers used here
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
int r8(int n) { return (n + 7) & ~7; }

enum Mode { F64 = 0, F32 = 1, BF16P = 2 };
const char* mode_name[] = {"fp64", "fp32", "bf16-packed"};

// A stored block of the FP64 arena: rows x cols, column-major with ld, at
// element offset off.  Packed copies: rows [0, split) of columns
// [top_c0, cols) form the top segment, rows [split, rows) of every column
// the bottom segment (either may be absent).
struct Stored {
  int64_t off;
  int ld, rows, cols;
  int split = 0, top_c0 = 0;
  bool has_top = false, has_bot = false;
  bool odd_ld = false;    // segments with ld = r8(rows) + 1: no 16-byte loads
  int64_t ptop = -1, pbot = -1;
};

// One use of a sub-block by a box.
struct Use {
  int box, partner;   // partner: the box whose x it multiplies
  int stored;         // index into the stored blocks
  int r0, c0;         // sub-block origin in the stored block
  bool trans;
  bool merged;        // a transposed use that the planner must read with a
                      // direct use of the same block
};

struct Arrays {
  std::vector<double> arena;          // FP64 blocks, NaN outside them
  std::vector<float> c32a, c32b;      // FP32 copies of [0, half) and [half, n)
  int64_t half = 0;
  std::vector<uint16_t> packed;       // packed BF16 copies
  std::vector<double> xs;             // x of every box, NaN in the padding
};

// Element (r, cc) of a chunk's block as the kernels read it, with the reads
// checked against the arrays the plan may point into.
double chunk_at(const Arrays& A, int esz, const GChunk& ch, int r, int cc) {
  const int64_t e = r + (int64_t)cc * ch.ld;
  if (esz == 8) {
    const double* p = static_cast<const double*>(ch.M);
    const int64_t o = (p - A.arena.data()) + e;
    CHECK(o >= 0 && o < (int64_t)A.arena.size(), "FP64 read outside the arena (%lld)", (long long)o);
    return (o >= 0 && o < (int64_t)A.arena.size()) ? A.arena[o] : NaN;
  }
  if (esz == 4) {
    const float* p = static_cast<const float*>(ch.M);
    for (const std::vector<float>* v : {&A.c32a, &A.c32b}) {
      const int64_t o0 = p - v->data();
      if (o0 >= 0 && o0 < (int64_t)v->size()) {
        CHECK(o0 + e < (int64_t)v->size(), "FP32 read past its copy");
        return o0 + e < (int64_t)v->size() ? (*v)[o0 + e] : NaN;
      }
    }
    CHECK(false, "FP32 chunk outside both copies");
    return NaN;
  }
  const uint16_t* p = static_cast<const uint16_t*>(ch.M);
  const int64_t o = (p - A.packed.data()) + e;
  CHECK(o >= 0 && o < (int64_t)A.packed.size(), "BF16 read outside the packed copy (%lld)",
        (long long)o);
  return (o >= 0 && o < (int64_t)A.packed.size()) ? bf16_value(A.packed[o]) : NaN;
}

double x_at(const Arrays& A, const double* x, int64_t i) {
  const int64_t o = (x - A.xs.data()) + i;
  CHECK(o >= 0 && o < (int64_t)A.xs.size(), "x read outside the x arena");
  return (o >= 0 && o < (int64_t)A.xs.size()) ? A.xs[o] : NaN;
}

bool same(double a, double b) { return a == b || (std::isnan(a) && std::isnan(b)); }

struct CaseCfg {
  uint64_t seed;
  Mode mode;
  int seg;
  bool wide;
  int nrhs;
};

int pick_rows(Rng& R) {
  static const int small[] = {0, 1, 3, 7, 8, 9, 16, 31, 63, 64, 65, 100, 127, 128, 129, 131};
  static const int large[] = {191, 255, 256, 257, 300};
  if (R.coin(1, 8)) return large[R.uni(0, 4)];
  return small[R.uni(0, 15)];
}

void run_case(const CaseCfg& cfg, int64_t* n_chunks_total) {
  std::snprintf(g_case, sizeof g_case, "seed %llu %s seg %d %s nrhs %d",
                (unsigned long long)cfg.seed, mode_name[cfg.mode], cfg.seg,
                cfg.wide ? "wide" : "narrow", cfg.nrhs);
  Rng R(cfg.seed);
  const int nrhs = cfg.nrhs;
  const int nb = R.uni(1, 8);
  std::vector<int> rows(nb);
  for (int& m : rows) m = pick_rows(R);

  // x of every box: rows x nrhs with ld rows + pad, NaN in the padding
  Arrays A;
  std::vector<int64_t> xoff(nb);
  std::vector<int> ldx(nb);
  for (int b = 0; b < nb; ++b) {
    ldx[b] = rows[b] + R.uni(0, 3);
    xoff[b] = (int64_t)A.xs.size();
    A.xs.resize(A.xs.size() + (size_t)ldx[b] * nrhs + 1, NaN);
    for (int c = 0; c < nrhs; ++c)
      for (int r = 0; r < rows[b]; ++r) A.xs[xoff[b] + r + (int64_t)c * ldx[b]] = R.uni(-3, 3);
  }

  // uses, each kind on a stored block of its own: direct only; shared
  // (direct by one box, transposed by another); transposed only; one
  // pointer used in two shapes; used directly twice and transposed once
  std::vector<Stored> st;
  std::vector<Use> uses;
  // packed copies: half the cases keep every block at the start of its
  // segment's first column (all chunks 16-byte aligned), so that a layout
  // with an ld that is not a multiple of 8 alone must turn 16-byte loads off
  const bool aligned_case = R.coin(1, 2);
  const int odd_ld_in = R.coin(1, 2) ? 0 : R.uni(1, 4);   // one in odd_ld_in blocks (0: none)
  auto new_stored = [&](int sr, int sc, int* r0, int* c0) {
    Stored s;
    if (cfg.mode != BF16P) {
      const int top = R.uni(0, 5), left = R.uni(0, 3);
      s.rows = top + sr + R.uni(0, 5);
      s.cols = left + sc + R.uni(0, 3);
      s.ld = s.rows + R.uni(0, 2);
      *r0 = top; *c0 = left;
    } else if (R.coin(1, 2)) {
      // in the bottom segment, at its first row (16-byte aligned) or a few
      // rows further down (not aligned: the plan must not take 16-byte loads)
      const int shift = !aligned_case && R.coin(1, 4) ? R.uni(1, 9) : 0;
      s.split = R.uni(0, 12);
      s.rows = s.split + shift + sr + R.uni(0, 9);
      const int left = aligned_case ? 0 : R.uni(0, 3);
      s.cols = left + sc + R.uni(0, 3);
      s.ld = s.rows + R.uni(0, 2);
      s.has_bot = true;
      s.has_top = s.split > 0 && R.coin(1, 2);
      s.top_c0 = R.uni(0, s.cols);
      *r0 = s.split + shift; *c0 = left;
    } else {
      // in the top segment: rows [0, sr) of columns from top_c0 on
      s.split = sr + R.uni(0, 9);
      s.top_c0 = R.uni(0, 3);
      const int left = s.top_c0 + (aligned_case ? 0 : R.uni(0, 2));
      s.cols = left + sc + R.uni(0, 3);
      s.rows = s.split + (R.coin(1, 2) ? R.uni(1, 6) : 0);
      s.ld = s.rows + R.uni(0, 2);
      s.has_top = true;
      s.has_bot = s.rows > s.split;
      *r0 = 0; *c0 = left;
    }
    s.odd_ld = odd_ld_in > 0 && R.coin(1, odd_ld_in);
    st.push_back(s);
    return (int)st.size() - 1;
  };
  for (int b = 0; b < nb; ++b) {
    const int nuse = R.uni(0, 4);
    for (int u = 0; u < nuse; ++u) {
      const int j = R.uni(0, nb - 1);
      int kind = R.uni(0, 4);
      // kind 3 needs a box p whose rows differ from b's
      int p = -1;
      for (int q = 0; q < nb && kind == 3; ++q)
        if (rows[q] != rows[b] && rows[q] > 0) p = q;
      if (kind == 3 && p < 0) kind = 0;
      // kind 4 needs a second box with b's rows
      int b2 = -1;
      for (int q = 0; q < nb && kind == 4; ++q)
        if (q != b && rows[q] == rows[b]) b2 = q;
      if (kind == 4 && b2 < 0) kind = 1;
      int r0, c0;
      if (kind == 0) {           // direct: rows_b x rows_j
        const int s = new_stored(rows[b], rows[j], &r0, &c0);
        uses.push_back({b, j, s, r0, c0, false, false});
      } else if (kind == 1) {    // shared: rows_b x rows_j, direct by b, transposed by j
        const int s = new_stored(rows[b], rows[j], &r0, &c0);
        uses.push_back({b, j, s, r0, c0, false, false});
        uses.push_back({j, b, s, r0, c0, true, true});
      } else if (kind == 2) {    // transposed only: stored rows_j x rows_b
        const int s = new_stored(rows[j], rows[b], &r0, &c0);
        uses.push_back({b, j, s, r0, c0, true, false});
      } else if (kind == 3) {
        // one pointer, two shapes: b uses rows_b x rows_j directly, j uses
        // rows_p x rows_j transposed; these are two blocks, not one
        const int s = new_stored(std::max(rows[b], rows[p]), rows[j], &r0, &c0);
        uses.push_back({b, j, s, r0, c0, false, false});
        uses.push_back({j, p, s, r0, c0, true, false});
      } else {
        // used directly by b and b2 (same rows) and transposed by j: one of
        // the two direct reads also serves the transposed product
        const int s = new_stored(rows[b], rows[j], &r0, &c0);
        uses.push_back({b, j, s, r0, c0, false, false});
        uses.push_back({b2, j, s, r0, c0, false, false});
        uses.push_back({j, b, s, r0, c0, true, true});
      }
    }
  }

  // the FP64 arena: blocks of integers, NaN in the ld padding and the gaps
  for (Stored& s : st) {
    A.arena.resize(A.arena.size() + R.uni(0, 5), NaN);
    s.off = (int64_t)A.arena.size();
    A.arena.resize(A.arena.size() + (size_t)s.ld * s.cols, NaN);
    for (int c = 0; c < s.cols; ++c)
      for (int r = 0; r < s.rows; ++r) A.arena[s.off + r + (int64_t)c * s.ld] = R.uni(-4, 4);
  }
  A.arena.resize(A.arena.size() + 1, NaN);
  const int64_t n = (int64_t)A.arena.size();

  // copies
  std::vector<Rebase> rb;
  std::vector<CopyMap> maps;
  if (cfg.mode == F32) {
    // two ranges split at a block boundary
    A.half = st.empty() ? n : st[st.size() / 2].off;
    A.c32a.assign(A.arena.begin(), A.arena.begin() + A.half);
    A.c32b.assign(A.arena.begin() + A.half, A.arena.end());
    Rebase a, b;
    a.base = A.arena.data(); a.n = A.half; a.copy = A.c32a.data(); a.esz = 4;
    b.base = A.arena.data() + A.half; b.n = n - A.half; b.copy = A.c32b.data(); b.esz = 4;
    if (A.half > 0) rb.push_back(a);
    if (n - A.half > 0) rb.push_back(b);
  } else if (cfg.mode == BF16P) {
    const uint16_t qnan = 0x7FC0;
    for (Stored& s : st) {
      A.packed.resize(A.packed.size() + 8 * R.uni(0, 2), qnan);
      if (s.has_top) {
        s.ptop = (int64_t)A.packed.size();
        const int ldt = r8(s.split) + (s.odd_ld ? 1 : 0);
        A.packed.resize(A.packed.size() + (size_t)ldt * (s.cols - s.top_c0), qnan);
        for (int c = s.top_c0; c < s.cols; ++c)
          for (int r = 0; r < ldt; ++r)
            A.packed[s.ptop + r + (int64_t)(c - s.top_c0) * ldt] =
                r < s.split ? bf16_bits(A.arena[s.off + r + (int64_t)c * s.ld]) : 0;
        A.packed.resize(r8((int)A.packed.size()), qnan);
      }
      if (s.has_bot) {
        s.pbot = (int64_t)A.packed.size();
        const int ldb = r8(s.rows - s.split) + (s.odd_ld ? 1 : 0);
        A.packed.resize(A.packed.size() + (size_t)ldb * s.cols, qnan);
        for (int c = 0; c < s.cols; ++c)
          for (int r = 0; r < ldb; ++r)
            A.packed[s.pbot + r + (int64_t)c * ldb] =
                s.split + r < s.rows ? bf16_bits(A.arena[s.off + s.split + r + (int64_t)c * s.ld])
                                     : 0;
        A.packed.resize(r8((int)A.packed.size()), qnan);
      }
      CopyMap m;
      m.src = A.arena.data() + s.off;
      m.ld = s.ld; m.rows = s.rows; m.cols = s.cols; m.split = s.split; m.top_c0 = s.top_c0;
      m.top = s.has_top ? s.ptop : -1; m.ld_top = r8(s.split) + (s.odd_ld ? 1 : 0);
      m.bot = s.has_bot ? s.pbot : -1; m.ld_bot = r8(s.rows - s.split) + (s.odd_ld ? 1 : 0);
      maps.push_back(m);
    }
    A.packed.resize(A.packed.size() + 8, qnan);
    Rebase a;
    a.base = A.arena.data(); a.n = n; a.copy = A.packed.data(); a.esz = 2; a.map = &maps;
    rb.push_back(a);
  }

  // boxes and their neighbour ranges; y with padding, base NULL, separate
  // or aliasing y
  std::vector<int> ldy(nb), ldbase(nb), base_kind(nb);
  std::vector<int64_t> yoff(nb), boff(nb);
  std::vector<double> ys, bases;
  std::vector<double> alpha(nb);
  static const double alphas[] = {1.0, -1.0, 0.5, 2.0};
  for (int b = 0; b < nb; ++b) {
    ldy[b] = rows[b] + R.uni(0, 2);
    yoff[b] = (int64_t)ys.size();
    ys.resize(ys.size() + (size_t)ldy[b] * nrhs + 1, -777.0);
    base_kind[b] = R.uni(0, 2);   // 0 none, 1 separate, 2 aliasing y
    alpha[b] = alphas[R.uni(0, 3)];
    if (base_kind[b] == 1) {
      ldbase[b] = rows[b] + R.uni(0, 2);
      boff[b] = (int64_t)bases.size();
      bases.resize(bases.size() + (size_t)ldbase[b] * nrhs + 1, NaN);
      for (int c = 0; c < nrhs; ++c)
        for (int r = 0; r < rows[b]; ++r) bases[boff[b] + r + (int64_t)c * ldbase[b]] = R.uni(-9, 9);
    } else if (base_kind[b] == 2) {
      ldbase[b] = ldy[b];
      for (int c = 0; c < nrhs; ++c)
        for (int r = 0; r < rows[b]; ++r) ys[yoff[b] + r + (int64_t)c * ldy[b]] = R.uni(-9, 9);
    } else {
      ldbase[b] = 1;
    }
  }
  std::vector<GatherBox> B(nb);
  std::vector<GatherNbr> Nv;
  for (int b = 0; b < nb; ++b) {
    GatherBox& g = B[b];
    g.y = ys.data() + yoff[b];
    g.base = base_kind[b] == 0 ? nullptr
             : base_kind[b] == 1 ? bases.data() + boff[b] : g.y;
    g.rows = rows[b]; g.ldy = ldy[b]; g.ldbase = ldbase[b]; g.alpha = alpha[b];
    for (int pass = 0; pass < 2; ++pass) {
      (pass == 0 ? g.d0 : g.t0) = (int)Nv.size();
      for (const Use& u : uses) {
        if (u.box != b || u.trans != (pass == 1)) continue;
        const Stored& s = st[u.stored];
        GatherNbr nbv;
        nbv.B = A.arena.data() + s.off + u.r0 + (int64_t)u.c0 * s.ld;
        nbv.ldB = s.ld;
        nbv.x = A.xs.data() + xoff[u.partner];
        nbv.ldx = ldx[u.partner];
        nbv.cols = rows[u.partner];
        Nv.push_back(nbv);
      }
      (pass == 0 ? g.d1 : g.t1) = (int)Nv.size();
    }
  }

  // the gathers' definition, on a copy of y
  std::vector<double> y_exp = ys;
  for (int b = 0; b < nb; ++b) {
    const GatherBox& g = B[b];
    for (int c = 0; c < nrhs; ++c)
      for (int r = 0; r < g.rows; ++r) {
        double s = 0.0;
        for (int q = g.d0; q < g.d1; ++q)
          for (int k = 0; k < Nv[q].cols; ++k)
            s += Nv[q].B[r + (int64_t)k * Nv[q].ldB] * Nv[q].x[k + (int64_t)c * Nv[q].ldx];
        for (int q = g.t0; q < g.t1; ++q)
          for (int k = 0; k < Nv[q].cols; ++k)
            s += Nv[q].B[k + (int64_t)r * Nv[q].ldB] * Nv[q].x[k + (int64_t)c * Nv[q].ldx];
        const double base = g.base ? g.base[r + (int64_t)c * g.ldbase] : 0.0;
        y_exp[yoff[b] + r + (int64_t)c * ldy[b]] = base + g.alpha * s;
      }
  }

  GatherPlan plan;
  const bool ok = plan_gather(B, Nv, plan, rb, cfg.seg, cfg.wide);
  CHECK(ok, "plan_gather refused a valid list");
  if (!ok) return;
  *n_chunks_total += (int64_t)plan.chunks.size();
  const int esz = cfg.mode == F64 ? 8 : cfg.mode == F32 ? 4 : 2;
  CHECK(plan.esz == esz, "esz %d", plan.esz);

  // the same lists give the same plan
  {
    GatherPlan again;
    plan_gather(B, Nv, again, rb, cfg.seg, cfg.wide);
    bool eq = again.chunks.size() == plan.chunks.size() && again.offs == plan.offs &&
              again.plen == plan.plen;
    for (size_t i = 0; eq && i < plan.chunks.size(); ++i)
      eq = std::memcmp(&again.chunks[i], &plan.chunks[i], sizeof(GChunk)) == 0;
    CHECK(eq, "planning the same lists twice differs");
  }

  // expected element count: each use once, a shared block once for both
  int64_t elems = 0;
  int maxr = 0;
  for (int b = 0; b < nb; ++b) maxr = std::max(maxr, rows[b]);
  for (const Use& u : uses)
    if (!u.merged && rows[u.box] > 0 && rows[u.partner] > 0)
      elems += (int64_t)rows[u.box] * rows[u.partner];
  CHECK(plan.max_rows == maxr, "max_rows %d, expected %d", plan.max_rows, maxr);
  CHECK(plan.bytes_chunks_mat == (double)esz * elems, "bytes_chunks_mat %.0f, expected %.0f",
        plan.bytes_chunks_mat, (double)esz * elems);

  // chunk shapes and flags
  const int crows = cfg.wide ? 64 * (esz < 8 ? GATHER_WIDE_RPL32 : GATHER_WIDE_RPL64)
                             : esz < 8 ? 128 : 64;
  int64_t read = 0;
  bool aligned16 = true;
  for (const GChunk& ch : plan.chunks) {
    CHECK(ch.nr >= 1 && ch.nr <= crows, "chunk rows %d (limit %d)", ch.nr, crows);
    CHECK(ch.mc >= 1 && (cfg.seg == 0 || ch.mc <= cfg.seg), "chunk columns %d (segment %d)", ch.mc,
          cfg.seg);
    CHECK(ch.rpl == (ch.nr + 63) / 64, "rows per lane %d for %d rows", ch.rpl, ch.nr);
    const int vec = (!cfg.wide && ((esz == 8 && ch.nr <= 64) || (esz == 4 && ch.nr <= 128))) ? 1 : 0;
    CHECK(ch.vec == vec, "vec %d, expected %d", ch.vec, vec);
    CHECK(ch.od >= 0 || ch.ot >= 0, "chunk without a product");
    CHECK((ch.od >= 0) == (ch.xd != nullptr) && (ch.ot >= 0) == (ch.xt != nullptr),
          "slot and vector disagree");
    if (ch.od >= 0) CHECK(ch.drow >= 0 && ch.drow + ch.nr <= ch.dlen, "direct rows");
    if (ch.ot >= 0) CHECK(ch.tcol >= 0 && ch.tcol + ch.mc <= ch.tlen, "transposed columns");
    if (ch.od >= 0) {
      // row chunks of a block depend on its height alone: steps of crows
      // (narrow), or the fewest chunks of at most crows rows, split evenly
      // (wide)
      const int m = ch.dlen, nck = (m + crows - 1) / crows;
      bool start_ok = false;
      for (int c = 0; c < nck && !start_ok; ++c) {
        const int a = cfg.wide ? (int)((int64_t)m * c / nck) : c * crows;
        const int e = cfg.wide ? (int)((int64_t)m * (c + 1) / nck) : std::min(m, (c + 1) * crows);
        start_ok = ch.drow == a && ch.nr == e - a;
      }
      CHECK(start_ok, "row chunk [%d, %d) of a block of %d rows", ch.drow, ch.drow + ch.nr, m);
    }
    read += (int64_t)ch.nr * ch.mc;
    if (reinterpret_cast<uintptr_t>(ch.M) % 16 != 0 || ch.ld % 8 != 0) aligned16 = false;
  }
  CHECK(read == elems, "block elements read %lld, expected %lld", (long long)read,
        (long long)elems);
  if (cfg.mode == BF16P && !cfg.wide)
    CHECK(plan.v16 == aligned16, "v16 %d with aligned chunks %d", (int)plan.v16, (int)aligned16);
  else
    CHECK(!plan.v16, "v16 outside narrow packed BF16 plans");

  // the host model of the chunk kernels
  const int64_t plen = plan.plen * nrhs;
  std::vector<double> P((size_t)plen, NaN);
  std::vector<uint8_t> written((size_t)plen, 0);
  auto put = [&](int64_t i, double v) {
    CHECK(i >= 0 && i < plen, "slot index %lld outside %lld", (long long)i, (long long)plen);
    if (i < 0 || i >= plen) return;
    CHECK(!written[i], "slot entry %lld written twice", (long long)i);
    written[i] = 1;
    P[i] = v;
  };
  for (const GChunk& ch : plan.chunks) {
    if (plan.v16)
      for (int cc = 0; cc < ch.mc; ++cc)
        for (int r = ch.nr; r < r8(ch.nr); ++r)
          CHECK(std::isfinite(chunk_at(A, esz, ch, r, cc)), "16-byte load reads a non-finite row");
    for (int c = 0; c < nrhs; ++c) {
      if (ch.od >= 0)
        for (int r = 0; r < ch.nr; ++r) {
          double s = 0.0;
          for (int cc = 0; cc < ch.mc; ++cc)
            s += chunk_at(A, esz, ch, r, cc) * x_at(A, ch.xd, cc + (int64_t)c * ch.ldxd);
          put(ch.od * nrhs + (int64_t)c * ch.dlen + ch.drow + r, s);
        }
      if (ch.ot >= 0)
        for (int cc = 0; cc < ch.mc; ++cc) {
          double s = 0.0;
          for (int r = 0; r < ch.nr; ++r)
            s += chunk_at(A, esz, ch, r, cc) * x_at(A, ch.xt, r + (int64_t)c * ch.ldxt);
          put(ch.ot * nrhs + (int64_t)c * ch.tlen + ch.tcol + cc, s);
        }
    }
  }
  int64_t missing = 0;
  for (uint8_t w : written) missing += w ? 0 : 1;
  CHECK(missing == 0, "%lld slot entries never written", (long long)missing);

  // the host model of the reductions
  CHECK((int)plan.reds.size() == nb, "%d reductions for %d boxes", (int)plan.reds.size(), nb);
  for (const GRed& g : plan.reds) {
    CHECK(g.s0 >= 0 && g.s0 <= g.s1 && g.s1 <= (int)plan.offs.size(), "slot range");
    for (int c = 0; c < nrhs; ++c)
      for (int r = 0; r < g.rows; ++r) {
        double s = 0.0;
        for (int q = g.s0; q < g.s1; ++q) {
          const int64_t i = plan.offs[q] * nrhs + (int64_t)c * g.rows + r;
          CHECK(i >= 0 && i < plen, "reduction reads outside the slots");
          s += (i >= 0 && i < plen) ? P[i] : NaN;
        }
        const double base = g.base ? g.base[r + (int64_t)c * g.ldbase] : 0.0;
        g.y[r + (int64_t)c * g.ldy] = base + g.alpha * s;
      }
  }
  int64_t bad = 0;
  for (size_t i = 0; i < ys.size(); ++i) bad += same(ys[i], y_exp[i]) ? 0 : 1;
  CHECK(bad == 0, "%lld of %zu y entries differ from the definition", (long long)bad, ys.size());
}

// Inputs the planner must refuse.
void refusals() {
  std::snprintf(g_case, sizeof g_case, "refusals");
  std::vector<double> arena(64 * 64, 1.0), x(64, 1.0), y(64, 0.0);
  std::vector<float> c32(arena.size(), 1.0f);
  std::vector<uint16_t> packed(arena.size(), 0);
  std::vector<GatherBox> B(1);
  B[0].y = y.data(); B[0].base = nullptr; B[0].rows = 16; B[0].ldy = 16; B[0].ldbase = 1;
  B[0].alpha = 1.0; B[0].d0 = 0; B[0].d1 = 1; B[0].t0 = 1; B[0].t1 = 1;
  std::vector<GatherNbr> Nv(1);
  Nv[0].B = arena.data() + 64 * 32; Nv[0].x = x.data(); Nv[0].ldB = 64; Nv[0].ldx = 16;
  Nv[0].cols = 16;
  GatherPlan p;
  CHECK(plan_gather(B, Nv, p), "a plain FP64 list");
  CHECK(!plan_gather(B, Nv, p, {}, 8), "a segment width that is not a multiple of 16");
  CHECK(!plan_gather(B, Nv, p, {}, -16), "a negative segment width");
  Rebase lo;
  lo.base = arena.data(); lo.n = 64 * 32; lo.copy = c32.data(); lo.esz = 4;
  CHECK(!plan_gather(B, Nv, p, {lo}), "a block outside every copy range");
  Rebase hi = lo;
  hi.base = arena.data() + 64 * 32; hi.n = 64 * 32; hi.copy = c32.data();
  CHECK(plan_gather(B, Nv, p, {lo, hi}), "a block inside the second range");
  Rebase h8 = hi;
  h8.esz = 8;
  CHECK(!plan_gather(B, Nv, p, {lo, h8}), "an FP64 copy range");
  Rebase h2r = hi;
  h2r.esz = 2;
  CHECK(!plan_gather(B, Nv, p, {lo, h2r}), "copy ranges of different widths");
  std::vector<CopyMap> maps(1);
  CopyMap& m = maps[0];
  m.src = arena.data(); m.ld = 64; m.rows = 64; m.cols = 64; m.split = 20; m.top_c0 = 0;
  m.top = 0; m.ld_top = 24; m.bot = 24 * 64; m.ld_bot = 48;
  Rebase pk;
  pk.base = arena.data(); pk.n = (int64_t)arena.size(); pk.copy = packed.data(); pk.esz = 2;
  pk.map = &maps;
  Rebase pk4 = pk;
  pk4.esz = 4;
  CHECK(!plan_gather(B, Nv, p, {pk4}), "a packed map on FP32 copies");
  // column 32, rows 0..15: inside the top segment
  CHECK(plan_gather(B, Nv, p, {pk}), "a block in the top segment");
  // rows 10..25 cross the split at 20
  Nv[0].B = arena.data() + 64 * 32 + 10;
  CHECK(!plan_gather(B, Nv, p, {pk}), "a block across the segment split");
  // rows 20..35 start the bottom segment
  Nv[0].B = arena.data() + 64 * 32 + 20;
  CHECK(plan_gather(B, Nv, p, {pk}), "a block in the bottom segment");
  CHECK(p.v16, "an aligned block of the bottom segment takes 16-byte loads");
  // without a top segment, rows 0..15 have no copy
  maps[0].top = -1;
  Nv[0].B = arena.data() + 64 * 32;
  CHECK(!plan_gather(B, Nv, p, {pk}), "a block in a missing top segment");
  // rows below the block's last row
  maps[0].top = 0;
  Nv[0].B = arena.data() + 64 * 32 + 50;
  CHECK(!plan_gather(B, Nv, p, {pk}), "a block past the stored rows");
  // a block before the first mapped block
  maps[0].src = arena.data() + 64;
  Nv[0].B = arena.data() + 10;
  CHECK(!plan_gather(B, Nv, p, {pk}), "a block before every mapped block");
}

}  // namespace

int main() {
  refusals();
  int64_t chunks = 0;
  int cases = 0;
  const int segs[] = {0, 16, 32, 128};
  for (uint64_t seed = 1; seed <= 32; ++seed)
    for (int mode = 0; mode < 3; ++mode)
      for (int wide = 0; wide < 2; ++wide) {
        CaseCfg cfg;
        cfg.seed = seed * 1000 + mode * 10 + wide;
        cfg.mode = (Mode)mode;
        cfg.seg = segs[seed % 4];
        cfg.wide = wide != 0;
        cfg.nrhs = 1 + (int)(seed % 3);
        run_case(cfg, &chunks);
        ++cases;
      }
  std::printf("%d cases, %lld chunks, %d failures\n", cases, (long long)chunks, g_fail);
  return g_fail == 0 ? 0 : 1;
}
