// Planner of the neighbour gathers (GatherPlan in h2_internal.hpp): items
// keyed by stored block (a block used directly by one box and transposed by
// another becomes one item), row chunks and column segments, partial slots,
// per-box reductions and the algorithmic bytes of one pass.
#include <algorithm>
#include <climits>
#include <unordered_map>

#include "h2_internal.hpp"

namespace h2 {

bool plan_gather(const std::vector<GatherBox>& B, const std::vector<GatherNbr>& Nv,
                 GatherPlan& out, const std::vector<Rebase>& rb, int seg, bool wide) {
  if (seg < 0 || seg % 16 != 0) return false;
  const int W = seg > 0 ? seg : INT_MAX;
  out = GatherPlan();
  out.esz = rb.empty() ? 8 : rb[0].esz;
  for (const Rebase& r : rb)
    if (r.esz != out.esz || (r.esz != 4 && r.esz != 2)) return false;
  const bool copy = out.esz < 8;
  const double esz = out.esz;
  bool packed = copy;
  for (const Rebase& r : rb) packed = packed && r.map != nullptr;
  if (packed && out.esz != 2) return false;
  // The copy of a sub-block that starts at p and spans `rows` rows, and its
  // leading dimension (*ld); nullptr when p lies in no range, or when a
  // packed copy does not hold those rows in one segment.
  auto to_copy = [&](const double* p, int rows, int64_t* ld) -> const char* {
    for (const Rebase& r : rb) {
      if (!(p >= r.base && p < r.base + r.n)) continue;
      const char* cp = static_cast<const char*>(r.copy);
      if (!r.map) return cp + (p - r.base) * r.esz;
      const std::vector<CopyMap>& mp = *r.map;
      // last block whose source starts at or before p
      auto it = std::upper_bound(mp.begin(), mp.end(), p,
                                 [](const double* a, const CopyMap& b) { return a < b.src; });
      if (it == mp.begin()) return nullptr;
      const CopyMap& b = *(it - 1);
      const int64_t e = p - b.src;
      if (e >= b.ld * b.cols) return nullptr;
      const int64_t row = e % b.ld, col = e / b.ld;
      if (row < b.split) {
        if (b.top < 0 || col < b.top_c0 || row + rows > b.split) return nullptr;
        *ld = b.ld_top;
        return cp + (b.top + (col - b.top_c0) * b.ld_top + row) * r.esz;
      }
      if (b.bot < 0 || row + rows > b.rows) return nullptr;
      *ld = b.ld_bot;
      return cp + (b.bot + col * b.ld_bot + (row - b.split)) * r.esz;
    }
    return nullptr;
  };
  struct Item {
    const double* M;
    int ld, mr, mc;
    int dq = -1, tq = -1;      // neighbour entries using M directly / transposed
    int dbox = -1, tbox = -1;
    int64_t od = -1;           // first of the per-segment direct slots (mr each)
    int64_t ot0 = -1;          // first of the per-row-chunk trans slots (mc each)
  };
  auto nseg_of = [W](int mc) { return mc <= W ? 1 : (mc + W - 1) / W; };
  std::vector<Item> items;
  std::vector<int> item_of_d(Nv.size(), -1), item_of_t(Nv.size(), -1);
  std::unordered_multimap<const double*, int> dir_items;
  for (size_t bx = 0; bx < B.size(); ++bx) {
    const GatherBox& g = B[bx];
    out.max_rows = std::max(out.max_rows, g.rows);
    for (int q = g.d0; q < g.d1; ++q) {
      const GatherNbr& n = Nv[q];
      if (g.rows <= 0 || n.cols <= 0) continue;
      Item it;
      it.M = n.B; it.ld = n.ldB; it.mr = g.rows; it.mc = n.cols;
      it.dq = q; it.dbox = (int)bx;
      item_of_d[q] = (int)items.size();
      dir_items.emplace(n.B, (int)items.size());
      items.push_back(it);
    }
  }
  // a block used transposed by one box and directly by another is read once
  for (size_t bx = 0; bx < B.size(); ++bx) {
    const GatherBox& g = B[bx];
    for (int q = g.t0; q < g.t1; ++q) {
      const GatherNbr& n = Nv[q];
      if (g.rows <= 0 || n.cols <= 0) continue;
      int hit = -1;
      auto range = dir_items.equal_range(n.B);
      for (auto e = range.first; e != range.second; ++e) {
        const Item& it = items[e->second];
        if (it.tq < 0 && it.ld == n.ldB && it.mr == n.cols && it.mc == g.rows) { hit = e->second; break; }
      }
      if (hit < 0) {
        Item it;
        it.M = n.B; it.ld = n.ldB; it.mr = n.cols; it.mc = g.rows;
        hit = (int)items.size();
        items.push_back(it);
      }
      items[hit].tq = q;
      items[hit].tbox = (int)bx;
      item_of_t[q] = hit;
    }
  }
  // Chunks of 64 rows, 128 for FP32 or BF16 copies (one or two rows per
  // lane), or wide: the rows split evenly into the fewest chunks of at most
  // 64 x GATHER_WIDE_RPL32 / GATHER_WIDE_RPL64 rows.  Boundaries depend only on the block's size, so
  // results are reproducible across handles and runs.
  const int crows = wide ? 64 * (copy ? GATHER_WIDE_RPL32 : GATHER_WIDE_RPL64)
                         : copy ? 128 : 64;
  auto chunk_starts = [crows, wide](const Item& it) {
    std::vector<int> r;
    if (wide) {
      const int nck = (it.mr + crows - 1) / crows;
      for (int c = 0; c < nck; ++c) r.push_back((int)((int64_t)it.mr * c / nck));
    } else {
      for (int r0 = 0; r0 < it.mr; r0 += crows) r.push_back(r0);
    }
    r.push_back(it.mr);
    return r;
  };
  // slots, chunks and bytes
  int64_t off = 0;
  std::vector<int> nck_of(items.size());
  for (size_t ii = 0; ii < items.size(); ++ii) {
    Item& it = items[ii];
    const std::vector<int> rs = chunk_starts(it);
    const int nck = (int)rs.size() - 1;
    const int nseg = nseg_of(it.mc);
    nck_of[ii] = nck;
    if (it.dq >= 0) { it.od = off; off += (int64_t)nseg * it.mr; }
    if (it.tq >= 0) { it.ot0 = off; off += (int64_t)nck * it.mc; }
    const GatherNbr* nd = it.dq >= 0 ? &Nv[it.dq] : nullptr;
    const GatherNbr* nt = it.tq >= 0 ? &Nv[it.tq] : nullptr;
    int64_t ldc = it.ld;
    const char* Mc = copy ? to_copy(it.M, it.mr, &ldc) : nullptr;
    if (copy && !Mc) return false;
    for (int c = 0; c < nck; ++c) {
      const int r0 = rs[c];
      for (int sg = 0; sg < nseg; ++sg) {
        const int c0 = sg * std::min(W, it.mc), c1 = std::min(it.mc, c0 + W);
        const int64_t e0 = r0 + (int64_t)c0 * it.ld;
        GChunk ch;
        ch.M = copy ? static_cast<const void*>(Mc + (r0 + (int64_t)c0 * ldc) * out.esz)
                    : static_cast<const void*>(it.M + e0);
        ch.xd = nd ? nd->x + c0 : nullptr;
        ch.xt = nt ? nt->x + r0 : nullptr;
        ch.ld = (int)ldc;
        ch.ldxd = nd ? nd->ldx : 1;
        ch.ldxt = nt ? nt->ldx : 1;
        ch.nr = rs[c + 1] - r0;
        ch.mc = c1 - c0;
        ch.dlen = it.mr;
        ch.drow = r0;
        ch.tlen = it.mc;
        ch.tcol = c0;
        ch.rpl = (ch.nr + 63) / 64;
        ch.vec = (!wide && ((!copy && ch.nr <= 64) || (out.esz == 4 && ch.nr <= 128))) ? 1 : 0;
        ch.od = nd ? it.od + (int64_t)sg * it.mr : -1;
        ch.ot = nt ? it.ot0 + (int64_t)c * it.mc : -1;
        out.chunks.push_back(ch);
      }
    }
    out.bytes_chunks_mat += esz * it.mr * it.mc;
    if (nd) out.bytes_chunks_vec += 8.0 * (it.mc + (double)nseg * it.mr);   // x_d, slots
    if (nt) out.bytes_chunks_vec += 8.0 * (it.mr + (double)nck * it.mc);    // x_t, slots
  }
  out.plen = off;
  // packed BF16: every chunk 16-byte aligned with ld a multiple of 8 and a
  // first row that is a multiple of 8 (rows past the segment are zeros)
  out.v16 = packed && !wide;
  for (const GChunk& ch : out.chunks)
    if (out.v16 && (reinterpret_cast<uintptr_t>(ch.M) % 16 != 0 || ch.ld % 8 != 0 || ch.nr > 128))
      out.v16 = false;
  for (size_t bx = 0; bx < B.size(); ++bx) {
    const GatherBox& g = B[bx];
    GRed r;
    r.y = g.y; r.base = g.base; r.rows = g.rows; r.ldy = g.ldy; r.ldbase = g.ldbase;
    r.alpha = g.alpha;
    r.s0 = (int)out.offs.size();
    for (int q = g.d0; q < g.d1; ++q)
      if (item_of_d[q] >= 0) {
        const Item& it = items[item_of_d[q]];
        for (int sg = 0; sg < nseg_of(it.mc); ++sg) out.offs.push_back(it.od + (int64_t)sg * it.mr);
      }
    for (int q = g.t0; q < g.t1; ++q)
      if (item_of_t[q] >= 0) {
        const Item& it = items[item_of_t[q]];
        for (int c = 0; c < nck_of[item_of_t[q]]; ++c)
          out.offs.push_back(it.ot0 + (int64_t)c * it.mc);
      }
    r.s1 = (int)out.offs.size();
    out.reds.push_back(r);
    out.bytes_red += 8.0 * g.rows * ((r.s1 - r.s0) + 1 + (g.base ? 1 : 0));
  }
  return true;
}

}  // namespace h2
