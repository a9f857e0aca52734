// Host tables of the offset-row interchange delta (Sec. 4 modification operator): vector groups,
// their rows (one per placement block and offset d) and the chunks the launch's workgroups take.
#include <cstdlib>
#include <map>
#include <queue>
#include <stdexcept>

#include "../../include/lpf.h"
#include "lpf_internal.h"

namespace lpf {

namespace {

int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

// One class of vectors: frame, row step, minor sign, major extent n, and the minor extents m
// with their (dx, dy).
struct ClassVecs {
  int frame, sr, ms, n;
  std::vector<int> m;
  std::vector<std::pair<int, int>> v;
};

}  // namespace

DiagGeo diag_geometry(int W, int H, int cx, int cy) {
  DiagGeo g{};
  // largest minor extent: steep vectors |dx| <= min(cx, cy - 1), flat ones dy <= min(cx, cy)
  const int mm0 = std::max(0, std::min(cx, cy - 1)), mm1 = std::min(cx, cy);
  g.B[0] = mm0 + 1;
  g.B[1] = mm1 + 1;
  g.rowoff[0] = cy;
  g.rowoff[1] = cx;
  g.rows[0] = H + 2 * cy;
  g.rows[1] = W + 2 * cx;
  // a window starts at minor bit (coordinate + B + o) >= 0 with o >= -(mm + 1) and is read as
  // the dword pair holding its 32 bits
  g.we[0] = ((W - 1 + 2 * mm0 + 1) >> 5) + 2;
  g.we[1] = ((H - 1 + 2 * mm1 + 1) >> 5) + 2;
  g.off[0] = 0;
  g.off[1] = g.rows[0] * g.we[0];
  g.total = g.off[1] + g.rows[1] * g.we[1];
  for (int f = 0; f < 2; ++f) {
    const int P = f == 0 ? W : H;
    uint32_t pat = 0;
    for (int t = 0; t < 32; t += P) pat |= 1u << t;
    g.pat[f] = pat;
  }
  return g;
}

bool build_diag_table(int cx, int cy, int nchunks, size_t max_bytes, DiagTable &t) {
  std::vector<int16_t> can((size_t)2 * lpf_num_vectors(cx, cy));
  if (lpf_vectors(cx, cy, can.data()) != LPF_OK) return false;
  std::map<std::pair<int, int>, int> index;
  for (size_t i = 0; i < can.size() / 2; ++i) index[{can[2 * i], can[2 * i + 1]}] = (int)i;
  // rows of the whole table: sum over groups of blocks x (2n) (estimate, before building)
  {
    double rows = 0;
    for (int n = 1; n <= std::max(cx, cy); ++n) {
      const double groups = 4.0 * ((n + kDiagG) / kDiagG);
      rows += groups * 2.0 * n * ((n + 32) / 32);
    }
    if (rows * sizeof(DiagRow) > (double)max_bytes) return false;
  }
  std::vector<ClassVecs> classes;
  {
    ClassVecs z{1, 1, 1, 0, {0}, {{0, 0}}};
    classes.push_back(z);  // the zero vector: one placement, no rows
  }
  for (int n = 1; n <= std::max(cx, cy); ++n) {
    if (n <= cx) {
      ClassVecs fp{1, 1, 1, n, {}, {}}, fm{1, -1, 1, n, {}, {}};  // flat, dx > 0 / dx < 0
      for (int m = 0; m <= std::min(n, cy); ++m) {
        fp.m.push_back(m);
        fp.v.push_back({n, m});
        if (m >= 1) {
          fm.m.push_back(m);
          fm.v.push_back({-n, m});
        }
      }
      if (!fp.m.empty()) classes.push_back(fp);
      if (!fm.m.empty()) classes.push_back(fm);
    }
    if (n <= cy) {
      ClassVecs sp{0, 1, 1, n, {}, {}}, sm{0, 1, -1, n, {}, {}};  // steep, dx >= 0 / dx < 0
      for (int m = 0; m <= std::min(n - 1, cx); ++m) {
        sp.m.push_back(m);
        sp.v.push_back({m, n});
        if (m >= 1) {
          sm.m.push_back(m);
          sm.v.push_back({-m, n});
        }
      }
      if (!sp.m.empty()) classes.push_back(sp);
      if (!sm.m.empty()) classes.push_back(sm);
    }
  }
  std::vector<DiagGroup> groups;
  std::vector<std::vector<DiagRow>> grows;
  std::vector<int64_t> cost;
  std::vector<int> ys;
  for (const ClassVecs &c : classes) {
    const int n = c.n;
    for (size_t g0 = 0; g0 < c.m.size(); g0 += kDiagG) {
      const int G = (int)std::min<size_t>(kDiagG, c.m.size() - g0);
      DiagGroup gr{};
      gr.n = n;
      gr.G = G;
      gr.frame = c.frame;
      gr.sr = c.sr;
      gr.nb = (n + 32) / 32;
      if (gr.nb > 8) throw std::runtime_error("diag table: more than 8 placement blocks");
      for (int g = 0; g < kDiagG; ++g) gr.idx[g] = g < G ? index.at(c.v[g0 + g]) : 0;
      // digitised minor coordinate y_k of each vector (eq. (segments))
      ys.assign((size_t)G * (n + 1), 0);
      for (int g = 0; g < G; ++g)
        for (int k = 0; k <= n; ++k)
          ys[(size_t)g * (n + 1) + k] = n ? (int)((2LL * k * c.m[g0 + g] + n) / (2LL * n)) : 0;
      std::vector<DiagRow> rows;
      for (int b = 0; b < gr.nb; ++b) {
        gr.boff[b] = (int32_t)rows.size();
        const int kb0 = 32 * b, kb1 = std::min(32 * b + 31, n);
        for (int d = -kb1; d <= n - kb0; ++d) {
          if (d == 0) continue;
          const int lo = std::max(0, -d - kb0), hi = std::min(kb1 - kb0, n - d - kb0);
          if (lo > hi) continue;
          DiagRow r{};
          r.d = d;
          r.valid = (hi - lo == 31 ? 0xffffffffu : ((1u << (hi - lo + 1)) - 1u)) << lo;
          int lower[kDiagG];
          int omin = 1 << 30;
          for (int g = 0; g < G; ++g) {
            const int m = c.m[g0 + g];
            const int *y = &ys[(size_t)g * (n + 1)];
            const int f = (int)floor_div((int64_t)d * m, n);
            uint32_t hib = 0;
            for (int tt = lo; tt <= hi; ++tt) {
              const int k = kb0 + tt;
              const int delta = y[k + d] - y[k];
              if (delta != f && delta != f + 1) throw std::runtime_error("diag table: offset");
              if (delta == f + 1) hib |= 1u << tt;
            }
            // minor sign +: offsets f, f + 1 at bits j, j + 1; sign -: -f - 1, -f at bits j, j + 1
            lower[g] = c.ms > 0 ? f : -f - 1;
            r.hs[g] = c.ms > 0 ? hib : ~hib;
            omin = std::min(omin, lower[g]);
          }
          r.o = omin;
          for (int g = 0; g < G; ++g) {
            const int j = lower[g] - omin;
            if (j < 0 || j > 30) throw std::runtime_error("diag table: window span");
            r.jp[g / 4] |= (uint32_t)j << (8 * (g % 4));
          }
          rows.push_back(r);
        }
      }
      gr.boff[gr.nb] = (int32_t)rows.size();
      for (int b = gr.nb + 1; b < 9; ++b) gr.boff[b] = gr.boff[gr.nb];
      cost.push_back((int64_t)rows.size() * (10 * G + 24) + 16 * G + 8);
      groups.push_back(gr);
      grows.push_back(std::move(rows));
    }
  }
  // chunks: longest-processing-time-first over the groups
  const int ng = (int)groups.size();
  nchunks = std::max(1, std::min(nchunks, ng));
  std::vector<int> order(ng);
  for (int i = 0; i < ng; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  using Item = std::pair<int64_t, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int b = 0; b < nchunks; ++b) heap.push({0, b});
  std::vector<std::vector<int>> bins(nchunks);
  for (int i : order) {
    Item it = heap.top();
    heap.pop();
    bins[it.second].push_back(i);
    heap.push({it.first + cost[i], it.second});
  }
  t.groups.clear();
  t.rows.clear();
  t.chunk_off.assign(nchunks + 1, 0);
  for (int b = 0; b < nchunks; ++b) {
    t.chunk_off[b] = (int32_t)t.groups.size();
    for (int i : bins[b]) {
      DiagGroup gr = groups[i];
      gr.row0 = (int32_t)t.rows.size();
      t.rows.insert(t.rows.end(), grows[i].begin(), grows[i].end());
      t.groups.push_back(gr);
    }
  }
  t.chunk_off[nchunks] = (int32_t)t.groups.size();
  return t.rows.size() * sizeof(DiagRow) <= max_bytes;
}

}  // namespace lpf
