// Chains of the canonical half domain for the full evaluation (host code).
//
// The paper's enhanced evaluation (Sec. 3.2) rests on segments overlapping shorter segments:
// both start at (0,0) and the shorter one's pixels are the first pixels of the longer one.  Here
// the same relation is used to share work: a chain is one walked vector v and every vector u
// whose digitised path is, up to a translation, pixels 0..l of v's path (l = n_u, the path of u
// has n_u + 1 pixels).  Counts are translation invariant on a periodic image (Sec. 2.1), so the
// running AND/OR product of v's walk after pixel l is u's product.
//
// Construction, longest vectors first: a vector not yet in a chain is walked (it cannot be a
// prefix of any vector still to come, those being no longer).  At pixel l of the walk the only
// vector whose path can be pixels 0..l is u = p_l itself (taken with dy >= 0).  With the major
// axis of the walk, pixel k has minor coordinate q_k = floor(k s + 1/2), s = m/n, so the slopes
// that digitise to q_0..q_l on 0..l form the interval I_l = intersection over k <= l of
// [(q_k - 1/2)/k, (q_k + 1/2)/k); u's path is pixels 0..l exactly when its own slope q_l / l lies
// in I_l.  The walk keeps I_l as two fractions, so each prefix costs O(1) and the whole
// construction O(sum of walked lengths).
#include <algorithm>
#include <cstdlib>
#include <queue>

#include "../../include/lpf.h"
#include "lpf_internal.h"

namespace lpf {

namespace {

// p / q (q > 0) compared as fractions with 64-bit cross products (|p|, q < 2^17 here).
inline bool frac_less(int64_t p1, int64_t q1, int64_t p2, int64_t q2) { return p1 * q2 < p2 * q1; }

}  // namespace

void build_chains(int cx, int cy, ChainSet &out) {
  out.chains.clear();
  out.mems.clear();
  out.walk = 0;
  out.path_pixels = 0;
  // canonical index of (dx, dy): [0,cx] x [0,cy] row by row, then [-cx,-1] x [1,cy]
  const int64_t n1 = (int64_t)(cx + 1) * (cy + 1);
  auto index_of = [&](int dx, int dy) -> int64_t {
    if (dx >= 0) return (int64_t)dy * (cx + 1) + dx;
    return n1 + (int64_t)(dy - 1) * cx + (dx + cx);
  };
  const int64_t nv = n1 + (int64_t)cx * cy;
  // vectors by length, longest first (canonical order within a length)
  const int nmax = std::max(cx, cy);
  std::vector<int64_t> cnt(nmax + 2, 0);
  auto len = [](int dx, int dy) { return std::max(std::abs(dx), dy); };
  for (int dy = 0; dy <= cy; ++dy)
    for (int dx = -cx; dx <= cx; ++dx) {
      if (dy == 0 && dx < 0) continue;
      ++cnt[nmax - len(dx, dy) + 1];
      out.path_pixels += len(dx, dy) + 1;
    }
  for (int i = 1; i <= nmax + 1; ++i) cnt[i] += cnt[i - 1];
  std::vector<int32_t> order(nv);
  for (int dy = 0; dy <= cy; ++dy)
    for (int dx = -cx; dx <= cx; ++dx) {
      if (dy == 0 && dx < 0) continue;
      order[cnt[nmax - len(dx, dy)]++] = (int32_t)index_of(dx, dy);
    }
  auto vec_of = [&](int64_t i, int &dx, int &dy) {
    if (i < n1) {
      dy = (int)(i / (cx + 1));
      dx = (int)(i - (int64_t)dy * (cx + 1));
    } else {
      const int64_t r = i - n1;
      dy = 1 + (int)(r / cx);
      dx = -cx + (int)(r - (int64_t)(dy - 1) * cx);
    }
  };
  std::vector<char> placed(nv, 0);
  for (int32_t v : order) {
    if (placed[v]) continue;
    int dx, dy;
    vec_of(v, dx, dy);
    const int adx = std::abs(dx), n = std::max(adx, dy);
    const bool xm = adx >= dy;
    const int m = xm ? dy : adx;
    const int sx = dx < 0 ? -1 : 1;
    ChainDesc c{};
    c.dx = (int16_t)dx;
    c.dy = (int16_t)dy;
    c.m0 = (int32_t)out.mems.size();
    // I_l = [lo_p / lo_q, hi_p / hi_q), in units of 1/2: bounds (2q - 1) / 2k and (2q + 1) / 2k
    int64_t lo_p = -1, lo_q = 1, hi_p = 1 << 30, hi_q = 1;
    int err = n, q = 0;  // q_k = floor((2km + n) / 2n) by the incremental error term
    for (int k = 0; k < n; ++k) {
      if (k > 0) {
        if (frac_less(lo_p, lo_q, 2 * q - 1, 2 * k)) {
          lo_p = 2 * q - 1;
          lo_q = 2 * k;
        }
        if (frac_less(2 * q + 1, 2 * k, hi_p, hi_q)) {
          hi_p = 2 * q + 1;
          hi_q = 2 * k;
        }
      }
      // u = p_k; its slope q / k (k = 0: the zero vector, a prefix of every path)
      const bool match = k == 0 || (!frac_less(q, k, lo_p, lo_q) && frac_less(q, k, hi_p, hi_q));
      if (match) {
        int ux = xm ? sx * k : sx * q, uy = xm ? q : k;
        if (uy == 0 && ux < 0) ux = -ux;  // a horizontal run: the canonical (k, 0)
        const int64_t u = index_of(ux, uy);
        if (!placed[u]) {
          placed[u] = 1;
          out.mems.push_back(MemDesc{(int32_t)u, (int16_t)ux, (int16_t)uy, k});
        }
      }
      err += 2 * m;
      if (err >= 2 * n) {
        err -= 2 * n;
        ++q;
      }
    }
    placed[v] = 1;
    out.mems.push_back(MemDesc{(int32_t)v, (int16_t)dx, (int16_t)dy, n});
    c.nm = (int32_t)out.mems.size() - c.m0;
    c.lw = n;
    out.chains.push_back(c);
    out.walk += n + 1;
  }
}

void pack_bins(const ChainSet &all, int64_t nb_want, BinPlan &out) {
  // chains with more members than a quarter of a bin's slots are cut into pieces walking the
  // same vector up to their last member (axis and diagonal chains: one member per pixel)
  constexpr int kPiece = kSlotWords / 4;
  std::vector<ChainDesc> pieces;
  pieces.reserve(all.chains.size());
  for (const ChainDesc &cd : all.chains)
    for (int j0 = 0; j0 < cd.nm; j0 += kPiece) {
      ChainDesc pc = cd;
      pc.m0 = cd.m0 + j0;
      pc.nm = std::min(kPiece, cd.nm - j0);
      pc.lw = all.mems[pc.m0 + pc.nm - 1].l;
      pieces.push_back(pc);
    }
  const int64_t nch = (int64_t)pieces.size();
  const int64_t nv = (int64_t)all.mems.size();
  // bins at most half full of members on average, so that the packing has room
  int64_t nb = std::max<int64_t>(nb_want, 2 * ((nv + kSlotWords / 2 - 1) / (kSlotWords / 2)));
  nb = std::max<int64_t>(1, std::min<int64_t>(nb, nch));
  std::vector<int> order(nch);
  std::vector<int64_t> cost(nch);
  for (int64_t i = 0; i < nch; ++i) {
    order[i] = (int)i;
    cost[i] = pieces[i].lw + 1 + 3 * (int64_t)pieces[i].nm;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<std::vector<int>> bins;
  std::vector<int64_t> bload, bmem;
  for (;;) {
    bins.assign(nb, {});
    bload.assign(nb, 0);
    bmem.assign(nb, 0);
    using Item = std::pair<int64_t, int>;  // (load, bin)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int b = 0; b < nb; ++b) heap.push({0, b});
    bool fit = true;
    for (int i : order) {
      // the least loaded bin with room for the piece's members; a bin without room leaves the
      // heap for good (with bins half full on average this drops very few)
      while (!heap.empty() && bmem[heap.top().second] + pieces[i].nm > kSlotWords / 2)
        heap.pop();
      if (heap.empty()) {
        fit = false;
        break;
      }
      Item t = heap.top();
      heap.pop();
      bins[t.second].push_back(i);
      bload[t.second] += cost[i];
      bmem[t.second] += pieces[i].nm;
      heap.push({bload[t.second], t.second});
    }
    if (fit) break;
    nb = std::min<int64_t>(2 * nb, nch);  // one piece per bin always fits
  }
  out.nbins = (int)nb;
  out.chains.clear();
  out.mems.clear();
  out.chains.reserve(nch);
  out.mems.reserve(nv);
  out.off.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    out.off[b] = (int32_t)out.chains.size();
    for (int i : bins[b]) {
      ChainDesc cd = pieces[i];
      const int32_t m0 = (int32_t)out.mems.size();
      for (int j = 0; j < cd.nm; ++j) out.mems.push_back(all.mems[cd.m0 + j]);
      cd.m0 = m0;
      out.chains.push_back(cd);
    }
  }
  out.off[nb] = (int32_t)out.chains.size();
  out.cost = bload;
}

}  // namespace lpf

// Plan statistics for a cutoff (host only, no device): out[0] = |D_c|, out[1] = chains,
// out[2] = pixels walked per start word (sum over chains of the walked length + 1),
// out[3] = M_c (sum over D_c of n + 1, the per-vector walk).
extern "C" lpf_status lpf_chain_stats(int cx, int cy, int64_t *out) {
  if (!out || cx < 0 || cy < 0 || cx > 32767 || cy > 32767) return LPF_E_INVAL;
  if ((int64_t)(cx + 1) * (cy + 1) + (int64_t)cx * cy > ((int64_t)1 << 26)) return LPF_E_UNSUPPORTED;
  lpf::ChainSet cs;
  lpf::build_chains(cx, cy, cs);
  out[0] = (int64_t)cs.mems.size();
  out[1] = (int64_t)cs.chains.size();
  out[2] = cs.walk;
  out[3] = cs.path_pixels;
  return LPF_OK;
}

// Host check of the packed plan for cutoff (cx, cy) with nb_want bins requested (no device):
// every vector of D_c appears exactly once as a member, members of a piece have increasing l
// ending at the piece's walked length, each member's vector is the walked path's pixel l (the
// slope test) and no bin holds more than kSlotWords / 2 members.  out (host, 4 int64): bins,
// pieces, largest members per bin, total walk of the pieces.  Returns LPF_OK when every check
// holds, LPF_E_INVAL on a failed check or a bad argument.
extern "C" lpf_status lpf_plan_check(int cx, int cy, int64_t nb_want, int64_t *out) {
  if (!out || cx < 0 || cy < 0 || cx > 4096 || cy > 4096 || nb_want < 1) return LPF_E_INVAL;
  lpf::ChainSet cs;
  lpf::build_chains(cx, cy, cs);
  lpf::BinPlan bp;
  lpf::pack_bins(cs, nb_want, bp);
  const int64_t nv = (int64_t)(cx + 1) * (cy + 1) + (int64_t)cx * cy;
  std::vector<int> seen(nv, 0);
  int64_t maxmem = 0, walk = 0;
  for (int b = 0; b < bp.nbins; ++b) {
    int64_t mem = 0;
    for (int j = bp.off[b]; j < bp.off[b + 1]; ++j) {
      const lpf::ChainDesc &c = bp.chains[j];
      mem += c.nm;
      walk += c.lw + 1;
      const int adx = std::abs((int)c.dx), n = std::max(adx, (int)c.dy);
      const bool xm = adx >= c.dy;
      const int m = xm ? c.dy : adx;
      int prev = -1;
      for (int t = 0; t < c.nm; ++t) {
        const lpf::MemDesc &md = bp.mems[c.m0 + t];
        if (md.l <= prev || md.l > n || md.idx < 0 || md.idx >= nv) return LPF_E_INVAL;
        prev = md.l;
        ++seen[md.idx];
        // pixel l of the walked path, by the digitisation rule, as a canonical vector
        const int q = n ? (int)((2ll * md.l * m + n) / (2ll * n)) : 0;
        int ux = xm ? md.l : q, uy = xm ? q : md.l;
        if (c.dx < 0) ux = -ux;
        if (uy == 0 && ux < 0) ux = -ux;
        if (ux != md.dx || uy != md.dy || std::max(std::abs(ux), uy) != md.l) return LPF_E_INVAL;
      }
      if (prev != c.lw) return LPF_E_INVAL;
    }
    maxmem = std::max(maxmem, mem);
    if (mem > lpf::kSlotWords / 2) return LPF_E_INVAL;
  }
  for (int64_t i = 0; i < nv; ++i)
    if (seen[i] != 1) return LPF_E_INVAL;
  out[0] = bp.nbins;
  out[1] = (int64_t)bp.chains.size();
  out[2] = maxmem;
  out[3] = walk;
  return LPF_OK;
}
