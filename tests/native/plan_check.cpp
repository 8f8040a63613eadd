// CPU check of the library's host planning (layout, tile lists, blocked
// table copies and seed rows) for many plan shapes.  Built with bounds
// assertions (SHT_CHECK) and sanitizers by tests/test_host_sanitizers.py.
// Invariants checked here: every element of both blocked table copies and of
// the seed rows is written (the buffers start as NaN); every (level, m, row
// or latitude block, column block) appears in a tile list exactly once, and
// nothing else does, for every admissible column blocking and both orders.
#include <cmath>
#include <cstdio>
#include <map>
#include <tuple>
#include <vector>

#include "sht_plan.h"

using namespace sht;

static int g_fail = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++g_fail;                                                           \
    }                                                                     \
  } while (0)

template <typename T>
static void check_tables(const LevelDesc* lev, int nlev, const Layout& Y, int grid, bool otf) {
  std::vector<T> tab(otf ? 0 : Y.tab, (T)NAN), syn(otf ? 0 : Y.tabs, (T)NAN);
  std::vector<double> seeds(otf ? Y.seeds : 0, NAN);
  std::vector<int> j0(Y.nm_total, -1);
  for (int l = 0; l < nlev; ++l) {
    const LevelDesc& L = lev[l];
    std::vector<double> mu(L.J), s(L.J);
    grid_nodes(L.J, grid, mu.data(), s.data());
    fill_table_level<T>(L, mu.data(), s.data(), otf ? nullptr : tab.data(), Y.taboff.data() + L.m_base,
                        otf ? nullptr : syn.data(), Y.taboff_syn.data() + L.m_base, j0.data() + L.m_base,
                        otf ? seeds.data() : nullptr, Y.seedoff.data() + L.m_base);
  }
  for (T v : tab) CHECK(!std::isnan((double)v));
  for (T v : syn) CHECK(!std::isnan((double)v));
  for (double v : seeds) CHECK(!std::isnan(v));
  for (int l = 0; l < nlev; ++l)
    for (int m = 0; m <= lev[l].N; ++m) CHECK(j0[lev[l].m_base + m] >= 0 && j0[lev[l].m_base + m] <= lev[l].Jh);
}

static void check_tiles(int form, const LevelDesc* lev, int nlev, const int* jst, bool analysis, int ncb, int sched) {
  const std::vector<Tile> t = build_tiles(form, nlev, lev, jst, analysis, ncb, sched);
  std::map<std::tuple<int, int, int, int>, int> seen;
  for (const Tile& x : t)
    if (x.level >= 0) seen[std::make_tuple(x.level, x.m, x.rb, x.cb)] += 1;
  const int BN = 16 * ncb;
  size_t expect = 0;
  for (int l = 0; l < nlev; ++l) {
    const LevelDesc& L = lev[l];
    const int ncol = (2 * L.F + BN - 1) / BN;
    for (int m = 0; m <= L.N; ++m) {
      const int nm = L.N - m + 1;
      const int rows = form == SHT_FORM_BF16X6 ? 256 : 128;
      const int nb = analysis ? (nm + rows - 1) / rows : (L.Jh + 127) / 128 - jst[L.m_base + m] / 128;
      const int b0 = analysis ? 0 : jst[L.m_base + m] / 128;
      for (int cb = 0; cb < ncol; ++cb)
        for (int b = b0; b < b0 + nb; ++b) {
          auto it = seen.find(std::make_tuple(l, m, b, cb));
          CHECK(it != seen.end() && it->second == 1);
          ++expect;
        }
    }
  }
  CHECK(seen.size() == expect);
  if (sched == 0) CHECK(t.size() % 8 == 0);
}

struct Case {
  int nlev, form, grid, otf;
  std::vector<int> N, J, I, F;
};

int main() {
  const std::vector<Case> cases = {
      {1, SHT_FORM_FP64, SHT_GRID_CC_POLES, 0, {21}, {43}, {64}, {1}},
      {1, SHT_FORM_FP32, SHT_GRID_FEJER2, 0, {130}, {250}, {300}, {9}},
      {1, SHT_FORM_BF16X6, SHT_GRID_CC_POLES, 0, {100}, {203}, {216}, {5}},
      {1, SHT_FORM_FP32, SHT_GRID_FEJER1, 1, {90}, {183}, {192}, {40}},
      {1, SHT_FORM_FP64, SHT_GRID_GAUSS, 1, {60}, {61}, {128}, {3}},
      {1, SHT_FORM_BF16X6, SHT_GRID_FEJER2, 1, {0}, {1}, {2}, {2}},
      {1, SHT_FORM_FP32, SHT_GRID_CC_POLES, 0, {40}, {20}, {96}, {64}},     // J < 2N+1
      {1, SHT_FORM_FP32, SHT_GRID_FEJER2, 0, {300}, {97}, {800}, {23}},     // ragged column tile
      {3, SHT_FORM_FP32, SHT_GRID_CC_POLES, 0, {64, 128, 33}, {129, 257, 20}, {200, 400, 100}, {3, 2, 5}},
      {3, SHT_FORM_FP64, SHT_GRID_CC_POLES, 1, {32, 64, 128}, {65, 129, 257}, {100, 200, 400}, {32, 32, 32}},
      {2, SHT_FORM_BF16X6, SHT_GRID_FEJER2, 0, {79, 159}, {159, 319}, {240, 480}, {64, 64}},
  };
  int ncase = 0;
  for (const Case& c : cases) {
    for (int FB : {4, 8, 16}) {
      const int ncb = choose_ncb(c.form, c.nlev, c.N.data(), c.J.data(), c.F.data());
      LevelDesc lev[SHT_MAX_LEVELS];
      Layout Y;
      layout_levels(c.nlev, c.N.data(), c.J.data(), c.I.data(), c.F.data(), 16 * ncb, FB, lev, &Y);
      CHECK(Y.taboff.back() == Y.tab && Y.seedoff.back() == Y.seeds);
      if (FB == 8) {
        if (c.form == SHT_FORM_FP64)
          check_tables<double>(lev, c.nlev, Y, c.grid, c.otf != 0);
        else
          check_tables<float>(lev, c.nlev, Y, c.grid, c.otf != 0);
      }
      std::vector<int> jst(Y.nm_total, 0);
      for (int k = 0; k < Y.nm_total; k += 3) jst[k] = 32 * (k % 4);  // some left-out polar blocks
      for (int l = 0; l < c.nlev; ++l)
        for (int m = 0; m <= lev[l].N; ++m) {
          int& j = jst[lev[l].m_base + m];
          if (j > lev[l].Jh) j = lev[l].Jh;
        }
      for (int cb : {1, 2, 4, 5, 8, 10}) {
        bool ok = true;
        for (int l = 0; l < c.nlev; ++l)
          if (lev[l].Cp % (16 * cb)) ok = false;
        if (!ok) continue;
        for (int sched = 0; sched < 2; ++sched)
          for (int dir = 0; dir < 2; ++dir) check_tiles(c.form, lev, c.nlev, jst.data(), dir == 0, cb, sched);
      }
      ++ncase;
    }
  }
  std::printf("plan_check: %d layouts, %d failures\n", ncase, g_fail);
  return g_fail ? 1 : 0;
}
