// Work lists and launch sequences of the factorization (Algorithm 4), the
// parallel substitution (Section 3.7) and the H^2 matrix-vector product.
//
// Substitution in the two-sided basis P_i = [Q_i^S | Q_i^R L(r)_ii^{-T}]:
// the transformed block F_ij = P_i^T A_ij P_j holds, in S-first order,
//   [ SS_ij          L(s)_ij                           ]
//   [ L(s)_ji^T      L(r)_ii^{-1} L(r)_ij  (i > j)      ]
// so with d_i = P_i^T b_i = [c_i^S; z_i], z_i = L(r)_ii^{-1} c_i^R, Eq. 31 reads
//   y_i^R = z_i - sum_{j<i} (L(r)_ii^{-1} L(r)_ij) z_j,
//   c_i^S -= sum_j L(s)_ij y_j^R                        (forward), and
//   t_j   = y_j^R - sum_i L(s)_ij^T x_i^S,
//   s_j   = t_j - sum_{i>j} (L(r)_ii^{-1} L(r)_ij)^T t_i,
//   x_j   = P_j [x_j^S; s_j]                           (backward),
// which is the transpose of Eq. 31 since Q_j^R L(r)_jj^{-T} s_j = Q_j^R x_j^R.
// LU variant (every ordered pair stored): the left basis P_i as above, the
// right basis P'_j = [Q_j^S | Q_j^R U(r)_jj^{-1}], F_ij = P_i^T A_ij P'_j with
// L(s)_ij, U(s)_ij and L(r)_ii^{-1} RR_ij U(r)_jj^{-1}; the same recurrences
// read every block directly (F_ij^SR, F_ji^RS, F_ji^RR where the symmetric
// form reads transposes) and the backward sweep ends with x_j = P'_j [x^S; s].
// Every step is a batched product or neighbour gather, the root solve
// included (a product with the explicit root inverse).
#include <algorithm>
#include <climits>
#include <unordered_map>

#include "h2_ctx.hpp"

namespace h2 {

#define HIPCHK(x)                                  \
  do {                                             \
    if ((x) != hipSuccess) return H2_ERR_HIP;      \
  } while (0)
#define ALLOCHK(p)                                 \
  do {                                             \
    if (!(p)) return H2_ERR_ALLOC;                 \
  } while (0)

static int local_box(const Step& S, int t, int i) {
  int lo = 0, hi = S.nbox - 1, first = -1;
  while (lo <= hi) {
    const int mid = (lo + hi) / 2;
    if (S.inst[mid] >= t) { first = mid; hi = mid - 1; } else lo = mid + 1;
  }
  return first + i;
}

static bool up_gather(Ctx& c, GList& L, const std::vector<GatherBox>& B,
                      const std::vector<GatherNbr>& Nv, hipStream_t st,
                      const std::vector<Rebase>& rb = {}, int seg = 0, bool wide = false);

// Per-box products D = alpha op(A) B + beta C (beta 0, or 1 with C == D) as
// gathers with one neighbour: A direct (tA = 0) or transposed (tA = 1).
static bool up_thin(Ctx& c, GList& L, const std::vector<GemmDesc>& v, hipStream_t st,
                    const std::vector<Rebase>& rb = {}, int seg = 0, bool wide = false) {
  std::vector<GatherBox> B;
  std::vector<GatherNbr> Nv;
  for (const GemmDesc& g : v) {
    if (g.beta != 0.0 && (g.beta != 1.0 || g.C != g.D)) return false;
    const int q = (int)Nv.size();
    Nv.push_back({g.A, g.B, g.lda, g.ldb, g.K});
    GatherBox x{g.D, g.beta != 0.0 ? g.C : nullptr, g.M, g.ldd, g.ldc, g.alpha, q, q, q, q};
    if (g.tA) x.t1 = q + 1; else x.d1 = q + 1;
    B.push_back(x);
  }
  return up_gather(c, L, B, Nv, st, rb, seg, wide);
}

static bool up_gather(Ctx& c, GList& L, const std::vector<GatherBox>& B,
                      const std::vector<GatherNbr>& Nv, hipStream_t st,
                      const std::vector<Rebase>& rb, int seg, bool wide) {
  // packed BF16 copies take the 16-byte-load chunks instead of wide ones
  for (const Rebase& r : rb)
    if (r.map) wide = false;
  auto up_set = [&](GSet& S, bool wide) {
    GatherPlan p;
    if (!plan_gather(B, Nv, p, rb, seg, wide)) return false;
    L.esz = p.esz;
    if (!wide) L.v16 = p.v16;
    S.max_rows = p.max_rows;
    S.plen = p.plen;
    S.bytes_ch_mat = p.bytes_chunks_mat;
    S.bytes_ch_vec = p.bytes_chunks_vec;
    S.bytes_rd = p.bytes_red;
    c.part_len = std::max(c.part_len, p.plen);
    return upload(c, S.ch, p.chunks, st) && upload(c, S.rd, p.reds, st) &&
           upload(c, S.offs, p.offs, st);
  };
  L.has_w = wide;
  return up_set(L.n, false) && (!wide || up_set(L.w, true));
}

// The partial buffer holds the longest list's partial products for nrhs
// columns; it grows (outside any captured region) when more columns come.
h2_status ensure_partials(Ctx& c, int nrhs) {
  if (c.part_len == 0 || nrhs <= c.part_nrhs) return H2_OK;
  if (c.dPart) {
    if (hipDeviceSynchronize() != hipSuccess) return H2_ERR_HIP;
    c.free_one(c.dPart);
    c.dPart = nullptr;
  }
  c.dPart = c.alloc<double>((size_t)c.part_len * nrhs);
  if (!c.dPart) { c.part_nrhs = 0; return H2_ERR_ALLOC; }
  c.part_nrhs = nrhs;
  return H2_OK;
}

// Chunks then reduction; with timing on, each launch marks a start and an
// end event through its own dispatch (no marker between the launches; the
// event pool is sized once, gathers beyond it run untimed).
static hipError_t gather(Ctx& c, const GList& L, int nrhs, hipStream_t st) {
  const bool wide = L.has_w && nrhs <= GATHER_WIDE_NR;
  const GSet& S = L.pick(nrhs);
  if (S.rd.count == 0) return hipSuccess;
  const bool t = c.gtime && c.gev_used + 4 <= c.gev.size();
  hipEvent_t* ev = t ? &c.gev[c.gev_used] : nullptr;
  hipError_t e;
  if (t && S.ch.count == 0) {  // nothing to launch: an empty interval
    if ((e = hipEventRecord(ev[0], st)) != hipSuccess || (e = hipEventRecord(ev[1], st)) != hipSuccess)
      return e;
  }
  if ((e = launch_gchunks(S.ch.d, S.ch.count, c.part_cur, nrhs, L.esz, st, wide,
                          L.v16 && !wide, t ? ev[0] : nullptr, t ? ev[1] : nullptr)) !=
      hipSuccess)
    return e;
  if (t && S.max_rows <= 0) {
    if ((e = hipEventRecord(ev[2], st)) != hipSuccess || (e = hipEventRecord(ev[3], st)) != hipSuccess)
      return e;
  }
  if ((e = launch_greduce(S.rd.d, S.rd.count, S.max_rows, S.offs.d, c.part_cur, nrhs, st,
                          t ? ev[2] : nullptr, t ? ev[3] : nullptr)) != hipSuccess)
    return e;
  if (t) {
    c.gev_used += 4;
    c.gbytes.push_back(S.bytes_ch_mat + S.bytes_ch_vec * nrhs);
    c.gbytes.push_back(S.bytes_rd * nrhs);
    c.gkind.push_back(L.kind >= 0 ? L.kind : L.esz < 8 ? 1 : 0);
  }
  return hipSuccess;
}

h2_status plan_solve(Ctx& c, hipStream_t st) {
  const int NR = NRHS_MAX;
  c.vt_in = c.alloc<double>((size_t)c.N * NR);
  c.vt_out = c.alloc<double>((size_t)c.N * NR);
  c.w_x = c.alloc<double>((size_t)c.N * NR);
  c.w_r = c.alloc<double>((size_t)c.N * NR);
  c.w_z = c.alloc<double>((size_t)c.N * NR);
  c.w_p = c.alloc<double>((size_t)c.N * NR);
  c.w_q = c.alloc<double>((size_t)c.N * NR);
  c.w_t = c.alloc<double>((size_t)c.N * NR);
  ALLOCHK(c.vt_in); ALLOCHK(c.vt_out); ALLOCHK(c.w_x); ALLOCHK(c.w_r);
  ALLOCHK(c.w_z); ALLOCHK(c.w_p); ALLOCHK(c.w_q); ALLOCHK(c.w_t);
  for (auto& in : c.ins) {
    in.v_root = c.alloc<double>((size_t)std::max(in.n0, 1) * NR);
    ALLOCHK(in.v_root);
  }
  // vectors of every step
  for (int h = 0; h < c.H; ++h) {
    Step& S = c.steps[h];
    S.voff.assign(S.nbox, 0);
    if (h == 0) {
      S.vld = c.N;
      for (int b = 0; b < S.nbox; ++b) {
        const Instance& in = c.ins[S.inst[b]];
        S.voff[b] = in.pbase + in.tree.start[in.tree.L][S.idx[b]];
      }
      S.v_in = c.vt_in;
      S.v_out = c.vt_out;
      S.v_d = c.alloc<double>((size_t)c.N * NR);
      ALLOCHK(S.v_d);
    } else {
      S.vld = S.sum_m;
      for (int b = 0; b < S.nbox; ++b) S.voff[b] = S.boff[b];
      S.v_in = c.alloc<double>((size_t)S.sum_m * NR);
      S.v_out = c.alloc<double>((size_t)S.sum_m * NR);
      S.v_d = c.alloc<double>((size_t)S.sum_m * NR);
      ALLOCHK(S.v_in); ALLOCHK(S.v_out); ALLOCHK(S.v_d);
    }
    S.v_yr = c.alloc<double>((size_t)std::max<int64_t>(S.sum_r, 1) * NR);
    S.v_t = c.alloc<double>((size_t)std::max<int64_t>(S.sum_r, 1) * NR);
    S.v_xh = c.alloc<double>((size_t)std::max<int64_t>(S.sum_k, 1) * NR);
    S.v_yh = c.alloc<double>((size_t)std::max<int64_t>(S.sum_k, 1) * NR);
    ALLOCHK(S.v_yr); ALLOCHK(S.v_t); ALLOCHK(S.v_xh); ALLOCHK(S.v_yh);
  }
  // parent vector slice of box b at step h (forward: in, backward: out)
  auto parent_slice = [&](int h, int b, bool out, double*& p, int& ld) {
    const Step& S = c.steps[h];
    const int t = S.inst[b];
    const int off = (S.idx[b] & 1) ? S.k[b - 1] : 0;
    if (S.lvl[b] == 1) {
      Instance& in = c.ins[t];
      p = in.v_root + off;
      ld = std::max(in.n0, 1);
      return;
    }
    const Step& P = c.steps[h + 1];
    const int pb = local_box(P, t, S.idx[b] / 2);
    p = (out ? P.v_out : P.v_in) + P.voff[pb] + off;
    ld = (int)P.vld;
  };

  // the matvec's couplings of every level and the leaf near field are
  // independent of each other: one list, planned after the loop
  std::vector<std::vector<GatherBox>> mv_b(c.H + 1);
  std::vector<std::vector<GatherNbr>> mv_n(c.H + 1);
  for (int h = 0; h < c.H; ++h) {
    Step& S = c.steps[h];
    const int nb = S.nbox;
    const int vld = (int)S.vld;
    const int rld = (int)std::max<int64_t>(S.sum_r, 1);
    const int kld = (int)std::max<int64_t>(S.sum_k, 1);
    // neighbour lists (other, pair) from the unordered near pairs: lower[i]
    // the pairs (i, j < i), upper[j] the same pairs seen from j (read
    // transposed); LU variant (every ordered pair stored): lower[i] the pairs
    // (i, j < i), higher[i] the pairs (i, j > i), all read directly
    std::vector<std::vector<std::pair<int, int>>> lower(nb), upper(nb), higher(nb);
    for (size_t p = 0; p < S.np_i.size(); ++p) {
      const int i = S.np_i[p], j = S.np_j[p];
      if (i == j) continue;
      if (c.lu) {
        (j < i ? lower[i] : higher[i]).push_back({j, (int)p});
      } else {
        lower[i].push_back({j, (int)p});
        upper[j].push_back({i, (int)p});
      }
    }
    std::vector<std::vector<std::pair<int, int>>> flo(nb), fup(nb);
    for (size_t f = 0; f < S.fp_i.size(); ++f) {
      flo[S.fp_i[f]].push_back({S.fp_j[f], (int)f});
      if (!c.lu) fup[S.fp_j[f]].push_back({S.fp_i[f], (int)f});
    }
    auto F = [&](int p) { return S.dF + S.poff[p]; };
    std::vector<GemmDesc> tf, tb, tu, td;
    std::vector<GatherBox> b1, b2, b3, b4, bc, bn;
    std::vector<GatherNbr> n1, n2, n3, n4, nc, nn;
    for (int b = 0; b < nb; ++b) {
      const int m = S.m[b], k = S.k[b], r = m - k;
      const double* P = S.dP + S.qoff[b];
      double* vin = S.v_in + S.voff[b];
      double* vd = S.v_d + S.voff[b];
      double* vout = S.v_out + S.voff[b];
      double* yr = S.v_yr + S.roff[b];
      double* tv = S.v_t + S.roff[b];
      // forward: d = P^T b
      tf.push_back(gd(P, m, 1, vin, vld, 0, nullptr, 1, vd, vld, m, NR, m, 1.0, 0.0));
      // y^R = z - sum_{j<i} Lt_ij z_j
      {
        GatherBox g{yr, vd + k, r, rld, vld, -1.0, (int)n1.size(), 0, 0, 0};
        for (auto& jp : lower[b]) {
          const int j = jp.first;
          n1.push_back({F(jp.second) + k + (int64_t)S.k[j] * m, S.v_d + S.voff[j] + S.k[j], m, vld,
                        S.m[j] - S.k[j]});
        }
        g.d1 = (int)n1.size();
        g.t0 = g.t1 = (int)n1.size();
        if (r > 0) b1.push_back(g);
      }
      // c^S -= sum_j L(s)_ij y_j^R, written into the parent vector
      if (k > 0) {
        double* py;
        int pld;
        parent_slice(h, b, false, py, pld);
        GatherBox g{py, vd, k, pld, vld, -1.0, (int)n2.size(), 0, 0, 0};
        const double* Fii = S.dF + S.poff[S.diag_pair[b]];
        if (r > 0) n2.push_back({Fii + (int64_t)k * m, yr, m, rld, r});
        for (auto& jp : lower[b]) {
          const int j = jp.first, rj = S.m[j] - S.k[j];
          if (rj > 0) n2.push_back({F(jp.second) + (int64_t)S.k[j] * m, S.v_yr + S.roff[j], m, rld, rj});
        }
        for (auto& jp : higher[b]) {  // LU variant: L(s)_ij = F_ij^SR, j > i
          const int j = jp.first, rj = S.m[j] - S.k[j];
          if (rj > 0) n2.push_back({F(jp.second) + (int64_t)S.k[j] * m, S.v_yr + S.roff[j], m, rld, rj});
        }
        g.d1 = (int)n2.size();
        g.t0 = (int)n2.size();
        for (auto& jp : upper[b]) {
          const int j = jp.first, rj = S.m[j] - S.k[j];
          if (rj > 0) n2.push_back({F(jp.second) + S.k[j], S.v_yr + S.roff[j], S.m[j], rld, rj});
        }
        g.t1 = (int)n2.size();
        b2.push_back(g);
      }
      // backward: t_j = y_j^R - sum_i L(s)_ij^T x_i^S  (+ copy x_j^S into d_j)
      {
        double* xs;
        int xld;
        parent_slice(h, b, true, xs, xld);
        if (r > 0) {
          GatherBox g{tv, yr, r, rld, rld, -1.0, (int)n3.size(), 0, 0, 0};
          for (auto& ip : upper[b]) {  // i > j stored as (i, j): direct? no: L(s)_ij^T from F_ij
            (void)ip;
          }
          // direct: i < j, block F_ji (ji stored since j > i): rows k_j.., cols 0..k_i
          for (auto& ip : lower[b]) {
            const int i = ip.first, ki = S.k[i];
            if (ki == 0) continue;
            double* xsi;
            int xldi;
            parent_slice(h, i, true, xsi, xldi);
            n3.push_back({F(ip.second) + k, xsi, m, xldi, ki});
          }
          const double* Fjj = S.dF + S.poff[S.diag_pair[b]];
          if (c.lu) {
            // U(s)_ji = F_ji^RS for i = j and i > j, read directly
            if (k > 0) n3.push_back({Fjj + k, xs, m, xld, k});
            for (auto& ip : higher[b]) {
              const int i = ip.first, ki = S.k[i];
              if (ki == 0) continue;
              double* xsi;
              int xldi;
              parent_slice(h, i, true, xsi, xldi);
              n3.push_back({F(ip.second) + k, xsi, m, xldi, ki});
            }
          }
          g.d1 = (int)n3.size();
          g.t0 = (int)n3.size();
          if (k > 0 && !c.lu) n3.push_back({Fjj + (int64_t)k * m, xs, m, xld, k});
          for (auto& ip : upper[b]) {
            const int i = ip.first, ki = S.k[i];
            if (ki == 0) continue;
            double* xsi;
            int xldi;
            parent_slice(h, i, true, xsi, xldi);
            n3.push_back({F(ip.second) + (int64_t)k * S.m[i], xsi, S.m[i], xldi, ki});
          }
          g.t1 = (int)n3.size();
          b3.push_back(g);
        }
        if (k > 0) {
          GatherBox g{vd, xs, k, vld, xld, 0.0, (int)n3.size(), (int)n3.size(), (int)n3.size(),
                      (int)n3.size()};
          b3.push_back(g);
        }
      }
      // s_j = t_j - sum_{i>j} Lt_ij^T t_i, into d_j[k:]
      if (r > 0) {
        GatherBox g{vd + k, tv, r, vld, rld, -1.0, (int)n4.size(), 0, 0, 0};
        for (auto& ip : higher[b]) {  // LU variant: U(r)_ji read directly from F_ji^RR
          const int i = ip.first, ri = S.m[i] - S.k[i];
          if (ri > 0)
            n4.push_back({F(ip.second) + k + (int64_t)S.k[i] * m, S.v_t + S.roff[i], m, rld, ri});
        }
        g.d1 = g.t0 = (int)n4.size();
        for (auto& ip : upper[b]) {
          const int i = ip.first, ri = S.m[i] - S.k[i];
          if (ri > 0)
            n4.push_back({F(ip.second) + S.k[i] + (int64_t)k * S.m[i], S.v_t + S.roff[i], S.m[i], rld, ri});
        }
        g.t1 = (int)n4.size();
        b4.push_back(g);
      }
      // x_j = P_j d_j (LU variant: the right basis P'_j)
      const double* Pb = c.lu ? S.dPr + S.qoff[b] : P;
      tb.push_back(gd(Pb, m, 0, vd, vld, 0, nullptr, 1, vout, vld, m, NR, m, 1.0, 0.0));

      // ---- matvec: upward U^T x
      const double* U = S.Uptr[b];
      if (k > 0) {
        if (h == 0) {
          tu.push_back(gd(U, m, 1, c.vt_in + S.voff[b], vld, 0, nullptr, 1, S.v_xh + S.koff[b], kld, k,
                          NR, m, 1.0, 0.0));
        } else {
          const Step& C = c.steps[h - 1];
          const int a = local_box(C, S.inst[b], 2 * S.idx[b]);
          tu.push_back(gd(U, m, 1, C.v_xh + C.koff[a], (int)std::max<int64_t>(C.sum_k, 1), 0, nullptr,
                          1, S.v_xh + S.koff[b], kld, k, NR, m, 1.0, 0.0));
        }
      }
      // couplings y^_i = sum_j S_ij x^_j
      if (k > 0) {
        GatherBox g{S.v_yh + S.koff[b], nullptr, k, kld, kld, 1.0, (int)nc.size(), 0, 0, 0};
        for (auto& jf : flo[b]) {
          const int j = jf.first;
          if (S.k[j] > 0) nc.push_back({S.dS + S.soff[jf.second], S.v_xh + S.koff[j], k, kld, S.k[j]});
        }
        g.d1 = (int)nc.size();
        g.t0 = (int)nc.size();
        for (auto& jf : fup[b]) {
          const int j = jf.first;
          if (S.k[j] > 0)
            nc.push_back({S.dS + S.soff[jf.second], S.v_xh + S.koff[j], S.k[j], kld, S.k[j]});
        }
        g.t1 = (int)nc.size();
        bc.push_back(g);
      }
      // downward U y^
      if (h == 0) {
        // y_i = (near field, written first) + U y^
        if (k > 0)
          td.push_back(gd(U, m, 0, S.v_yh + S.koff[b], kld, 0, c.vt_out + S.voff[b], vld,
                          c.vt_out + S.voff[b], vld, m, NR, k, 1.0, 1.0));
        // near field y_i = sum_j D_ij x_j
        GatherBox g{c.vt_out + S.voff[b], nullptr, m, vld, vld, 1.0, (int)nn.size(), 0, 0, 0};
        nn.push_back({S.dD + S.poff[S.diag_pair[b]], c.vt_in + S.voff[b], m, vld, m});
        for (auto& jp : lower[b]) {
          const int j = jp.first;
          nn.push_back({S.dD + S.poff[jp.second], c.vt_in + S.voff[j], m, vld, S.m[j]});
        }
        for (auto& jp : higher[b]) {
          const int j = jp.first;
          nn.push_back({S.dD + S.poff[jp.second], c.vt_in + S.voff[j], m, vld, S.m[j]});
        }
        g.d1 = (int)nn.size();
        g.t0 = (int)nn.size();
        for (auto& jp : upper[b]) {
          const int j = jp.first;
          nn.push_back({S.dD + S.poff[jp.second], c.vt_in + S.voff[j], S.m[j], vld, S.m[j]});
        }
        g.t1 = (int)nn.size();
        bn.push_back(g);
      } else if (k > 0) {
        const Step& C = c.steps[h - 1];
        const int a = local_box(C, S.inst[b], 2 * S.idx[b]);
        double* dst = C.v_yh + C.koff[a];
        const int cld = (int)std::max<int64_t>(C.sum_k, 1);
        td.push_back(gd(U, m, 0, S.v_yh + S.koff[b], kld, 0, dst, cld, dst, cld, m, NR, k, 1.0, 1.0));
      }
    }
    // the substitution may read FP32 or BF16 copies of F and P (a gather
    // list reads one element type); the matvec reads FP64.  Reduced-precision
    // pair transforms leave the off-diagonal F in FP32 only, so they imply at
    // least the FP32 reads.
    std::vector<Rebase> rb;
    if (c.prm.solve_prec == H2_PREC_BF16) {
      rb.push_back({S.dF, S.poff.back(), S.dF16, 2, &S.cmF});
      rb.push_back({S.dP, S.qoff[S.nbox], S.dP16, 2, &S.cmP});
    } else if (c.prm.solve_prec == H2_PREC_FP32 || c.prm.gemm_prec != H2_PREC_FP64) {
      rb.push_back({S.dF, S.poff.back(), S.dF32, 4});
      rb.push_back({S.dP, S.qoff[S.nbox], S.dP32, 4});
      if (c.lu) rb.push_back({S.dPr, S.qoff[S.nbox], S.dPr32, 4});
    }
    const int sg = h >= GATHER_SEG_TOP_FROM ? GATHER_SEG_TOP
                 : h >= GATHER_SEG_FROM     ? GATHER_SEG
                                            : 0;
    const bool wd = h >= GATHER_WIDE_FROM && h <= GATHER_WIDE_TO;
    const std::vector<Rebase> none;
    const int sgt = sg > 0 ? sg : h >= GATHER_SEG_THIN_FROM ? GATHER_SEG : 0;
    if (!up_thin(c, S.t_fwd, tf, st, rb, sgt, wd) || !up_thin(c, S.t_bwd, tb, st, rb, sgt, wd) ||
        !up_thin(c, S.t_up, tu, st, none, sgt, wd) || !up_thin(c, S.t_down, td, st, none, sgt, wd) ||
        !up_gather(c, S.g_yr, b1, n1, st, rb, sg, wd) ||
        !up_gather(c, S.g_cs, b2, n2, st, rb, sg, wd) ||
        !up_gather(c, S.g_t, b3, n3, st, rb, sg, wd) ||
        !up_gather(c, S.g_s, b4, n4, st, rb, sg, wd))
      return H2_ERR_ALLOC;
    mv_b[h + 1] = std::move(bc);
    mv_n[h + 1] = std::move(nc);
    if (h == 0) {
      mv_b[0] = std::move(bn);
      mv_n[0] = std::move(nn);
    }
  }
  {
    // top level first, so that the few long waves of the top levels start
    // at once and run under the leaf lists instead of trailing them
    std::vector<GatherBox> B;
    std::vector<GatherNbr> Nv;
    for (int q = c.H; q >= 0; --q) {
      const int off = (int)Nv.size();
      for (GatherBox g : mv_b[q]) {
        g.d0 += off; g.d1 += off; g.t0 += off; g.t1 += off;
        B.push_back(g);
      }
      Nv.insert(Nv.end(), mv_n[q].begin(), mv_n[q].end());
    }
    if (!up_gather(c, c.g_mv, B, Nv, st)) return H2_ERR_ALLOC;
    if (c.prm.matvec_prec == H2_PREC_FP32) {
      // the same products on the FP32 copies (PCG's inner products)
      std::vector<Rebase> rb32;
      for (const Step& S : c.steps)
        if (S.dS32 && S.soff.back() > 0) rb32.push_back({S.dS, S.soff.back(), S.dS32, 4});
      const Step& S0 = c.steps[0];
      if (S0.dD32 && S0.poff.back() > 0) rb32.push_back({S0.dD, S0.poff.back(), S0.dD32, 4});
      if (!up_gather(c, c.g_mv32, B, Nv, st, rb32)) return H2_ERR_ALLOC;
      c.g_mv32.kind = 3;
    }
  }
  // root solves and root-only instances
  {
    std::vector<CopyDesc> ri, ro;
    std::vector<GemmDesc> tr;
    // v_root <- root^{-1} v_root in place (the chunks read x before the
    // reduction writes y), one neighbour per 64 columns so that the product
    // spreads over many waves
    std::vector<GatherBox> rb;
    std::vector<GatherNbr> rn;
    for (auto& in : c.ins) {
      if (in.n0 == 0) continue;
      GatherBox g{in.v_root, nullptr, in.n0, in.n0, in.n0, 1.0, (int)rn.size(), 0, 0, 0};
      for (int c0 = 0; c0 < in.n0; c0 += 64)
        rn.push_back({in.dRinv + (int64_t)c0 * in.n0, in.v_root + c0, in.n0, in.n0,
                      std::min(64, in.n0 - c0)});
      g.d1 = g.t0 = g.t1 = (int)rn.size();
      rb.push_back(g);
      if (in.tree.L == 0) {
        ri.push_back({c.vt_in + in.pbase, in.v_root, in.n0, NR, (int)c.N, in.n0, 0});
        ro.push_back({in.v_root, c.vt_out + in.pbase, in.n0, NR, in.n0, (int)c.N, 0});
        tr.push_back(gd(in.dRootOrig, in.n0, 0, c.vt_in + in.pbase, (int)c.N, 0, nullptr, 1,
                        c.vt_out + in.pbase, (int)c.N, in.n0, NR, in.n0, 1.0, 0.0));
      }
    }
    if (!up_gather(c, c.g_root, rb, rn, st) || !upload(c, c.r_in, ri, st) ||
        !upload(c, c.r_out, ro, st) || !up_thin(c, c.t_root, tr, st))
      return H2_ERR_ALLOC;
  }
  return ensure_partials(c, 1);
}

// ------------------------------------------------------------------ factor
// Basis transforms and Schur update in the handle's GEMM precision: the
// FP32-operand lists carry their own kernel choice; the Schur update (FP64
// operands) runs on FP32 MFMA under every reduced precision.
static hipError_t run_gemm_p(const Ctx& c, const Batch<GemmDesc>& b, hipStream_t st, int tag = 0) {
  if (c.prm.gemm_prec == H2_PREC_FP64 || b.f32io) return run_gemm(b, st, tag);
  return launch_gemm_lp(b.d, b.toffs[0], b.count, b.tiles_c[0], H2_PREC_FP32, st, tag, b.tA, b.tB);
}

// Autotuner: every factor GEMM work list is timed with every tile shape (one
// warm-up launch, then the best of two timed launches, HIP events on the
// build stream) and the fastest shape is kept.  Running a work list on buffers
// that the first factorization has not yet filled is safe: the kernels have no
// data-dependent control flow and write only the list's own outputs.
h2_status autotune(Ctx& c, hipStream_t st) {
  // reduced precision: only the FP32-operand pair lists have tile shapes
  const bool fp64 = c.prm.gemm_prec == H2_PREC_FP64;
  auto tune = [&](Batch<GemmDesc>& b, int tag) -> h2_status {
    if (b.count == 0 || (!fp64 && !b.f32io)) return H2_OK;
    int best = 0;
    float best_ms = 1e30f;
    for (int q = 0; q < GEMM_NCFG; ++q) {
      b.use(q);
      HIPCHK(run_gemm(b, st, tag));
      float ms_q = 1e30f;
      for (int r = 0; r < 2; ++r) {
        HIPCHK(hipEventRecord(c.ev_a, st));
        HIPCHK(run_gemm(b, st, tag));
        HIPCHK(hipEventRecord(c.ev_b, st));
        HIPCHK(hipEventSynchronize(c.ev_b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c.ev_a, c.ev_b));
        ms_q = std::min(ms_q, ms);
      }
      if (ms_q < best_ms) { best_ms = ms_q; best = q; }
    }
    b.use(best);
    ++c.st.tuned_lists;
    c.st.tuned_cfg_hist[best] += 1;
    return H2_OK;
  };
  for (auto& S : c.steps) {
    for (Batch<GemmDesc>* b : {&S.g_w, &S.g_qr1, &S.g_qr2, &S.g_qr3, &S.g_diag1, &S.g_diag2,
                               &S.g_v, &S.g_schur, &S.g_far1, &S.g_far2, &S.g_far3}) {
      h2_status e = tune(*b, 0);
      if (e != H2_OK) return e;
    }
    for (size_t p = 0; p < S.g_pz.size(); ++p)
      for (Batch<GemmDesc>* b : {&S.g_pz[p], &S.g_pu[p]}) {
        h2_status e = tune(*b, 0);
        if (e != H2_OK) return e;
      }
    for (size_t p = 1; p < S.g_t1.size(); ++p)
      for (Batch<GemmDesc>* b : {&S.g_t1[p], &S.g_t2[p]}) {
        h2_status e = tune(*b, 0);
        if (e != H2_OK) return e;
      }
    for (size_t p = 0; p < S.ch_trsm.size(); ++p)
      for (Batch<GemmDesc>* b : {&S.ch_trsm[p], &S.ch_syrk[p], &S.ch_inv1[p], &S.ch_inv2[p]}) {
        h2_status e = tune(*b, 0);
        if (e != H2_OK) return e;
      }
    for (Batch<GemmDesc>* b : {&S.g_pair1, &S.g_pair2}) {
      h2_status e = tune(*b, 1);
      if (e != H2_OK) return e;
    }
  }
  return H2_OK;
}

// Phases of the factorization timed with params.timing (events from a pool
// in the handle, read after the factorization without stalling it).
enum FactorPhase {
  FP_QR, FP_DIAG, FP_CHOL, FP_VS, FP_PAIR, FP_FAR, FP_MERGE, FP_ROOT, FP_F32, FP_N
};

h2_status do_factor(Ctx& c, hipStream_t st) {
  HIPCHK(launch_set_int(c.dFail, INT_MAX, st));
  const bool f32t = c.prm.gemm_prec != H2_PREC_FP64;  // FP32 transforms
  const bool timing = c.prm.timing != 0 && !c.prm.use_graph;
  if (timing && c.fev.empty()) {
    c.fev.resize(2 * FP_N * (c.H + 2), nullptr);
    for (auto& e : c.fev) HIPCHK(hipEventCreate(&e));
  }
  c.fev_phase.clear();
  size_t ne = 0;
  auto mark = [&](int phase) -> hipError_t {  // event before the phase, event after
    if (!timing || ne + 2 > c.fev.size()) return hipSuccess;
    c.fev_phase.push_back(phase);
    return hipEventRecord(c.fev[ne], st);
  };
  auto done = [&]() -> hipError_t {
    if (!timing || c.fev_phase.size() * 2 != ne + 2) return hipSuccess;
    const hipError_t e = hipEventRecord(c.fev[ne + 1], st);
    ne += 2;
    return e;
  };
  for (int h = 0; h < c.H; ++h) {
    Step& S = c.steps[h];
    HIPCHK(mark(FP_QR));
    if (h == 0) HIPCHK(run_copy(S.c_w, st));
    else HIPCHK(run_gemm(S.g_w, st));
    for (size_t pp = 0; pp < S.g_pz.size(); ++pp) {  // one entry per panel
      HIPCHK(launch_qr_panel(S.qr.d, S.qr.count, S.qr.max_rows, (int)pp * S.qr_w, S.qr_w, st));
      HIPCHK(run_gemm(S.g_pz[pp], st));
      HIPCHK(run_gemm(S.g_pu[pp], st));
    }
    HIPCHK(run_gemm(S.g_qr1, st));
    HIPCHK(launch_qr_tdiag(S.qr.d, S.qr.count, S.max_k, st));
    for (size_t q = 1; q < S.g_t1.size(); ++q) {
      HIPCHK(run_gemm(S.g_t1[q], st));
      HIPCHK(run_gemm(S.g_t2[q], st));
    }
    HIPCHK(run_gemm(S.g_qr2, st));
    HIPCHK(run_gemm(S.g_qr3, st));
    HIPCHK(launch_qr_diag(S.qr.d, S.qr.count, st));
    HIPCHK(done());
    if (f32t) {  // FP32 transforms: Q_i and (above the leaves) D_ii to FP32
      HIPCHK(mark(FP_F32));
      HIPCHK(launch_cvt_f32(S.dQ, S.dP32, S.qoff[S.nbox], st));
      HIPCHK(launch_cvt_list(S.cv_dii.d, S.cv_dii.count, st));
      HIPCHK(done());
    }
    HIPCHK(mark(FP_DIAG));
    HIPCHK(run_gemm_p(c, S.g_diag1, st));
    HIPCHK(run_gemm_p(c, S.g_diag2, st));
    HIPCHK(done());
    HIPCHK(mark(FP_CHOL));
    HIPCHK(launch_fill(S.dLi, S.lioff.back(), 0.0, st));
    if (c.lu) HIPCHK(launch_fill(S.dUi, S.lioff.back(), 0.0, st));
    for (size_t p = 0; p < S.ch_panel.size(); ++p) {
      if (c.lu) HIPCHK(launch_lu_panel(S.ch_panel[p].d, S.ch_panel[p].count, c.dFail, st));
      else HIPCHK(launch_panel(S.ch_panel[p].d, S.ch_panel[p].count, c.dFail, st));
      HIPCHK(run_gemm(S.ch_trsm[p], st));
      HIPCHK(run_gemm(S.ch_syrk[p], st));
      HIPCHK(run_copy(S.ch_back[p], st));
    }
    for (size_t p = 1; p < S.ch_panel.size(); ++p) {
      HIPCHK(run_gemm(S.ch_inv1[p], st));
      HIPCHK(run_gemm(S.ch_inv2[p], st));
    }
    HIPCHK(done());
    HIPCHK(mark(FP_VS));
    HIPCHK(run_copy(S.c_ps, st));
    HIPCHK(run_gemm(S.g_v, st));
    HIPCHK(run_gemm(S.g_v2, st));
    HIPCHK(run_gemm_p(c, S.g_schur, st));
    HIPCHK(done());
    if (f32t) {  // FP32 pair transforms: operands and finished F_ii to FP32
      HIPCHK(mark(FP_F32));
      HIPCHK(launch_cvt_f32(S.dP, S.dP32, S.qoff[S.nbox], st));
      if (c.lu) HIPCHK(launch_cvt_f32(S.dPr, S.dPr32, S.qoff[S.nbox], st));
      HIPCHK(launch_cvt_f32(S.dR, S.dR32, S.rkoff[S.nbox], st));
      HIPCHK(launch_cvt_list(S.cv_fii.d, S.cv_fii.count, st));
      HIPCHK(done());
    }
    HIPCHK(mark(FP_PAIR));
    HIPCHK(run_gemm_p(c, S.g_pair1, st, 1));
    HIPCHK(run_gemm_p(c, S.g_pair2, st, 1));
    HIPCHK(done());
    HIPCHK(mark(FP_FAR));
    HIPCHK(run_gemm_p(c, S.g_far1, st));
    HIPCHK(run_gemm_p(c, S.g_far2, st));
    HIPCHK(run_gemm(S.g_far3, st));
    HIPCHK(done());
    HIPCHK(mark(FP_MERGE));
    HIPCHK(run_copy(S.c_merge, st));
    HIPCHK(launch_copy_f32(S.c_merge32.d, S.c_merge32.count, st));
    HIPCHK(launch_copy_f32(S.c_merge3232.d, S.c_merge3232.count, st, true));
    HIPCHK(done());
  }
  HIPCHK(mark(FP_ROOT));
  HIPCHK(run_copy(c.r_save, st));
  for (size_t p = 0; p < c.r_panel.size(); ++p) {
    if (c.lu) HIPCHK(launch_lu_panel(c.r_panel[p].d, c.r_panel[p].count, c.dFail, st));
    else HIPCHK(launch_panel(c.r_panel[p].d, c.r_panel[p].count, c.dFail, st));
    HIPCHK(run_gemm(c.r_trsm[p], st));
    HIPCHK(run_gemm(c.r_syrk[p], st));
    HIPCHK(run_copy(c.r_back[p], st));
  }
  for (size_t p = 1; p < c.r_inv1.size(); ++p) {
    HIPCHK(run_gemm(c.r_inv1[p], st));
    HIPCHK(run_gemm(c.r_inv2[p], st));
  }
  HIPCHK(run_gemm(c.r_full, st));
  HIPCHK(done());
  if (c.prm.solve_prec == H2_PREC_FP32 && c.prm.gemm_prec == H2_PREC_FP64) {
    HIPCHK(mark(FP_F32));
    for (auto& S : c.steps) {
      HIPCHK(launch_cvt_f32(S.dF, S.dF32, S.poff.back(), st));
      HIPCHK(launch_cvt_f32(S.dP, S.dP32, S.qoff[S.nbox], st));
      if (c.lu) HIPCHK(launch_cvt_f32(S.dPr, S.dPr32, S.qoff[S.nbox], st));
    }
    HIPCHK(done());
  }
  if (c.prm.solve_prec == H2_PREC_BF16) {
    // BF16 copies for the substitution: from the FP32 transforms' results
    // (F_ii converted to FP32 above) or from the FP64 factors
    HIPCHK(mark(FP_F32));
    const bool from32 = c.prm.gemm_prec != H2_PREC_FP64;
    for (auto& S : c.steps) {
      if (from32)
        HIPCHK(launch_cvt_bf16_blks(S.dF32, 4, S.cvF16.d, S.cvF16_first.d, S.cvF16.count, S.cvF16_groups, S.dF16, st));
      else
        HIPCHK(launch_cvt_bf16_blks(S.dF, 8, S.cvF16.d, S.cvF16_first.d, S.cvF16.count, S.cvF16_groups, S.dF16, st));
      HIPCHK(launch_cvt_bf16_blks(S.dP, 8, S.cvP16.d, S.cvP16_first.d, S.cvP16.count, S.cvP16_groups, S.dP16, st));
    }
    HIPCHK(done());
  }
  c.fev_used = ne;
  return H2_OK;
}

// After the factorization has completed: per-phase seconds into the stats.
h2_status collect_factor_times(Ctx& c) {
  for (int q = 0; q < FP_N; ++q) c.st.t_factor_phase[q] = 0.0;
  for (size_t i = 0; 2 * i + 1 < c.fev_used; ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c.fev[2 * i], c.fev[2 * i + 1]));
    c.st.t_factor_phase[c.fev_phase[i]] += 1e-3 * ms;
  }
  c.st.t_pair_gemm = c.st.t_factor_phase[FP_PAIR];
  return H2_OK;
}

// ------------------------------------------------------------------- solve
h2_status do_solve_chunk(Ctx& c, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs,
                         hipStream_t st) {
  HIPCHK(launch_gather_rows(c.dPermG, c.N, nrhs, b, ldb, c.vt_in, c.N, st));
  for (int h = 0; h < c.H; ++h) {
    Step& S = c.steps[h];
    HIPCHK(gather(c, S.t_fwd, nrhs, st));
    HIPCHK(gather(c, S.g_yr, nrhs, st));
    HIPCHK(gather(c, S.g_cs, nrhs, st));
  }
  HIPCHK(run_copy(c.r_in, st));
  HIPCHK(gather(c, c.g_root, nrhs, st));
  HIPCHK(run_copy(c.r_out, st));
  for (int h = c.H - 1; h >= 0; --h) {
    Step& S = c.steps[h];
    HIPCHK(gather(c, S.g_t, nrhs, st));
    HIPCHK(gather(c, S.g_s, nrhs, st));
    HIPCHK(gather(c, S.t_bwd, nrhs, st));
  }
  HIPCHK(launch_scatter_rows(c.dPermG, c.N, nrhs, c.vt_out, c.N, x, ldx, st));
  return H2_OK;
}

h2_status do_matvec_chunk(Ctx& c, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs,
                          hipStream_t st, bool lowp) {
  if (lowp && c.g_mv32.n.rd.count == 0 && c.g_mv.n.rd.count > 0) return H2_ERR_STATE;
  HIPCHK(launch_gather_rows(c.dPermG, c.N, nrhs, x, ldx, c.vt_in, c.N, st));
  for (int h = 0; h < c.H; ++h) HIPCHK(gather(c, c.steps[h].t_up, nrhs, st));
  // couplings of every level, leaf near field
  HIPCHK(gather(c, lowp ? c.g_mv32 : c.g_mv, nrhs, st));
  for (int h = c.H - 1; h >= 0; --h) HIPCHK(gather(c, c.steps[h].t_down, nrhs, st));
  HIPCHK(gather(c, c.t_root, nrhs, st));
  HIPCHK(launch_scatter_rows(c.dPermG, c.N, nrhs, c.vt_out, c.N, y, ldy, st));
  return H2_OK;
}

}  // namespace h2
