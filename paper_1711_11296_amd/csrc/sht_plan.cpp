// Host-side layout planning (see sht_plan.h): sizes and offsets, tile lists,
// blocked table copies.  With SHT_CHECK every computed index is asserted to
// lie inside the block it belongs to.

#include "sht_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

namespace sht {

int choose_ncb(int form, int nlev, const int* N, const int* J, const int* F) {
  const int cand64[] = {8, 4, 2, 1};
  const int cand32[] = {10, 8, 5, 4, 2, 1};
  const int* cand = form == SHT_FORM_FP64 ? cand64 : cand32;
  const int nc = form == SHT_FORM_FP64 ? 4 : 6;
  int best = 1;
  double bestc = 1e300;
  for (int k = 0; k < nc; ++k) {
    double c = 0;
    for (int l = 0; l < nlev; ++l) {
      double work = (double)(N[l] + 1) * (N[l] + 2) * ((J[l] + 1) / 2);
      c += work * (double)roundup(2LL * F[l], 16LL * cand[k]);
    }
    if (c < bestc * (1 - 1e-12)) {
      bestc = c;
      best = cand[k];
    }
  }
  return best;
}

void layout_levels(int nlev, const int* Nv, const int* Jv, const int* Iv, const int* Fv, int BN, int FB,
                   LevelDesc* lev, Layout* out) {
  Layout& Y = *out;
  Y = Layout();
  long long moff = 0;
  for (int l = 0; l < nlev; ++l) {
    LevelDesc& L = lev[l];
    std::memset(&L, 0, sizeof(L));
    L.N = Nv[l];
    L.J = Jv[l];
    L.I = Iv[l];
    L.F = Fv[l];
    L.Jh = (L.J + 1) / 2;
    L.Kp = (int)roundup(L.Jh, SHT_K_PAD);
    // a whole number of Legendre column tiles (BN) and of zonal items (2 FB
    // columns each), so that no zonal item writes past the end of a row
    L.Cp = (int)roundup(2LL * L.F, std::lcm(BN, 2 * FB));
    factor_radices(L.I, L.rad, &L.nrad);
    for (int q = 0, ns = 1; q < L.nrad; ns *= L.rad[q], ++q) {
      L.pns[q] = ns;
      L.ptw[q] = L.I / (ns * L.rad[q]);
      L.pmag[q] = ns > 1 ? 0xFFFFFFFFu / (unsigned)ns + 1u : 0u;
    }
    L.nfb = (L.F + FB - 1) / FB;
    while ((1 << L.wsh) < 2 * FB && L.wsh < 4) ++L.wsh;  // W = min(2 FB, 16), a power of two
    L.fft_item0 = (int)Y.items;
    Y.items += (long long)L.Jh * L.nfb;
    L.m_base = (int)moff;
    moff += L.N + 1;
    L.grid_off = Y.grid;
    Y.grid += (long long)L.F * L.J * L.I;
    L.spec_off = Y.spec;
    Y.spec += (long long)L.F * (L.N + 1) * (L.N + 2);
    L.ws_off = Y.ws;
    L.wplane = ws_plane(L.Kp, L.Cp);
    L.spoff = L.Kp == L.Jh ? L.wplane : (long long)L.Jh * L.Cp;
    Y.ws += roundup((long long)(L.N + 1) * 2 * L.wplane, 64);
    for (int m = 0; m <= L.N; ++m) {
      Y.taboff.push_back(Y.tab);
      // analysis copy: rows padded to the row tile of 128
      Y.tab += roundup(L.N - m + 1, 128) * L.Kp;
      Y.taboff_syn.push_back(Y.tabs);
      const int kr2 = 32;  // natural rows per K block
      Y.tabs += (long long)((L.Jh + 127) / 128) * ((L.N - m + kr2) / kr2) * 128 * kr2;
      Y.seedoff.push_back(Y.seeds);
      Y.seeds += 2LL * ((L.N - m + 16) / 16) * L.Kp;
      Y.recoff.push_back(Y.rec);
      Y.rec += 2LL * (L.N - m + 1);
    }
    SHT_ASSERT(L.Cp % BN == 0 && L.Cp % (2 * FB) == 0 && L.Cp >= 2 * L.F && (1 << L.wsh) == std::min(2 * FB, 16));
    SHT_ASSERT(L.Kp % SHT_K_PAD == 0 && L.Kp >= L.Jh);
    // the synthesis planes stay inside the region and off the rows the
    // analysis keeps zero (rows Jh .. Kp of its layout, 2 Cp elements each)
    SHT_ASSERT(L.spoff + (long long)L.Jh * L.Cp <= 2 * L.wplane &&
               (L.Kp == L.Jh || L.spoff + (long long)L.Jh * L.Cp <= 2LL * L.Jh * L.Cp));
  }
  // one sentinel past the last (level, m): block m of a level spans
  // [off[m], off[m + 1])
  Y.taboff.push_back(Y.tab);
  Y.taboff_syn.push_back(Y.tabs);
  Y.seedoff.push_back(Y.seeds);
  Y.recoff.push_back(Y.rec);
  Y.nm_total = (int)moff;
  SHT_ASSERT((long long)Y.taboff.size() == moff + 1 && (long long)Y.recoff.size() == moff + 1);
}

// Split a tile list (in locality order) into 8 contiguous chunks of equal
// cost and deal them so that chunk x runs on XCD x (block id % 8 == x).
static std::vector<Tile> xcd_schedule(const std::vector<Tile>& tiles, const std::vector<double>& cost) {
  const int X = 8;
  double total = 0;
  for (double c : cost) total += c;
  std::vector<std::vector<Tile>> chunk(X);
  double acc = 0;
  int x = 0;
  for (size_t i = 0; i < tiles.size(); ++i) {
    chunk[x].push_back(tiles[i]);
    acc += cost[i];
    while (x < X - 1 && acc >= total * (x + 1) / X) ++x;
  }
  size_t len = 0;
  for (auto& c : chunk) len = std::max(len, c.size());
  std::vector<Tile> out(len * X, Tile{-1, 0, 0, 0});
  for (int xx = 0; xx < X; ++xx)
    for (size_t i = 0; i < chunk[xx].size(); ++i) out[i * X + xx] = chunk[xx][i];
  return out;
}

std::vector<Tile> build_tiles(int form, int nlev, const LevelDesc* lev, const int* jst, bool analysis, int ncb,
                              int sched) {
  const int BN = 16 * ncb;
  std::vector<Tile> t;
  std::vector<double> c;
  for (int l = 0; l < nlev; ++l) {
    const LevelDesc& L = lev[l];
    SHT_ASSERT(L.Cp % BN == 0);
    // column tiles that hold at least one field (the row length may be
    // padded past the last field by more than a tile)
    const int ncol = std::min(L.Cp / BN, (2 * L.F + BN - 1) / BN);
    for (int m = 0; m <= L.N; ++m) {
      const int nm = L.N - m + 1;
      const int j0 = jst[L.m_base + m];  // reduced transform: latitudes below are left out
      SHT_ASSERT(j0 >= 0 && j0 <= L.Jh);
      for (int cb = 0; cb < ncol; ++cb) {
        SHT_ASSERT(cb * BN < 2 * L.F && (cb + 1) * BN <= L.Cp);
        if (analysis) {
          // 128-row tiles; 256 in the split form; K blocks of 32 latitudes
          // (16 in the FP64 form)
          const int rows = form == SHT_FORM_BF16X6 ? 256 : 128;
          const int kb = form == SHT_FORM_FP64 ? 16 : 32;
          for (int rb = 0; rb < (nm + rows - 1) / rows; ++rb) {
            SHT_ASSERT(rb * rows < nm);
            t.push_back(Tile{l, m, rb, cb});
            c.push_back((double)(L.Kp - j0 / kb * kb) * BN);
          }
        } else {
          // 128-latitude tiles; K blocks of 32 natural rows (64 in the
          // split form); tiles wholly below j0 are left out (the zonal
          // synthesis reads those workspace rows as zero)
          const int kr2 = form == SHT_FORM_BF16X6 ? 64 : 32;
          for (int jt = j0 / 128; jt < (L.Jh + 127) / 128; ++jt) {
            SHT_ASSERT(jt * 128 < L.Jh);
            t.push_back(Tile{l, m, jt, cb});
            c.push_back(((double)roundup(nm, kr2) + kr2) * 2 * BN);
          }
        }
      }
    }
  }
  if (sched == 1) return t;
  return xcd_schedule(t, c);
}

// Analysis copy: per m, rows r = n - m padded to 128, blocked in the order
// the analysis kernel streams it: per (128-row tile, KB-column block) one
// contiguous chunk (KB = 32 for float, 16 for double), inside it one run per
// wave (16 rows r = 32 q + 2 i + p), inside that one 64-lane vector after
// the other: vector v of lane (i, g) holds columns 4 (v E + e) + g, e < E =
// 16 bytes / element size.  Synthesis copy: per m, one chunk per
// (128-latitude tile, K block of 32 natural rows), blocked per wave and lane
// vector like the analysis copy (see the loop below).
template <typename T>
void fill_table_level(const LevelDesc& L, const double* mu, const double* sint, T* dst, const long long* off_a,
                      T* dsyn, const long long* off_s, int* j0, double* seeds, const long long* off_seed) {
  const int N = L.N, Jh = L.Jh, Kp = L.Kp;
  int nth = (int)std::thread::hardware_concurrency();
  nth = std::max(1, std::min(nth, 64));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t) {
    pool.emplace_back([=]() {
      std::vector<double> col;
      for (int k = t; k <= N; k += nth) {
        const int m = (k % 2 == 0) ? k / 2 : N - k / 2;
        const int nm = N - m + 1;
        col.assign((size_t)nm * Jh, 0.0);
        alf_column(N, m, Jh, mu, sint, col.data(), Jh);
        if (j0) {
          // reduced transform (Sec. 4.1): first latitude (from the pole) at
          // which some |P~_n^m| reaches 1e-16
          int first = Jh;
          for (int r = 0; r < nm; ++r)
            for (int j = 0; j < first; ++j)
              if (std::fabs(col[(size_t)r * Jh + j]) >= 1e-16) {
                first = j;
                break;
              }
          j0[m] = first;
        }
        if (seeds) {
          // generated P~: rows 16 g and 16 g + 1 of every 16-degree group
          double* sd = seeds + off_seed[m];
          const long long seed_len = off_seed[m + 1] - off_seed[m];
          SHT_ASSERT(seed_len == 2LL * ((nm + 15) / 16) * Kp);
          for (int g = 0; g < (nm + 15) / 16; ++g)
            for (int t2 = 0; t2 < 2; ++t2) {
              const int r = 16 * g + t2;
              for (int j = 0; j < Kp; ++j) {
                const size_t d = (size_t)(2 * g + t2) * Kp + j;
                SHT_ASSERT((long long)d < seed_len);
                sd[d] = (r < nm && j < Jh) ? col[(size_t)r * Jh + j] : 0.0;
              }
            }
        }
        if (!dst) continue;  // generated P~: seed rows only
        T* blk = dst + off_a[m];
        const int R = (int)roundup(nm, 128);
        const long long blk_len = off_a[m + 1] - off_a[m];
        SHT_ASSERT(blk_len == (long long)R * Kp);
        constexpr int KB = sizeof(T) == 4 ? 32 : 16, E = 16 / (int)sizeof(T);
        const int nkbk = Kp / KB;
        for (int r = 0; r < R; ++r)
          for (int j = 0; j < Kp; ++j) {
            const int rt = r / 128, rr = r % 128;
            const int q = rr / 32, i = (rr % 32) / 2, p = rr % 2;
            const int kb = j / KB, jj = j % KB;
            const int g = jj % 4, kk = jj / 4;
            const int v = kk / E, e = kk % E;
            const size_t d = ((size_t)rt * nkbk + kb) * 128 * KB + (size_t)(2 * q + p) * 16 * KB +
                             (size_t)((v * 4 + g) * 16 + i) * E + e;
            SHT_ASSERT((long long)d < blk_len);
            blk[d] = (r < nm && j < Jh) ? (T)col[(size_t)r * Jh + j] : (T)0;
          }
        // synthesis copy: per (128-latitude tile, K block of 2 KR natural
        // rows) one chunk; inside it one run per wave (parity p, quarter q)
        // of 64-lane vectors: vector v of lane (i, g) holds latitude
        // 32 q + 16 (v / (KQ/E)) + i and r' = g KQ + E (v % (KQ/E)) + e
        constexpr int KR = 16, KQs = KR / 4, NVs = 2 * KQs / E;
        const int nkbs = (nm + 2 * KR - 1) / (2 * KR);
        const int JT = (Jh + 127) / 128;
        const size_t chunk = (size_t)128 * 2 * KR;
        T* sb = dsyn + off_s[m];
        const long long syn_len = off_s[m + 1] - off_s[m];
        SHT_ASSERT(syn_len == (long long)JT * nkbs * (long long)chunk);
        for (int jt = 0; jt < JT; ++jt)
          for (int kb = 0; kb < nkbs; ++kb)
            for (int w = 0; w < 8; ++w)
              for (int v = 0; v < NVs; ++v)
                for (int ln = 0; ln < 64; ++ln)
                  for (int e = 0; e < E; ++e) {
                    const int p = w & 1, q = w >> 1, i = ln & 15, g = ln >> 4;
                    const int jb = v / (KQs / E), kk = (v % (KQs / E)) * E + e;
                    const int r = kb * 2 * KR + 2 * (g * KQs + kk) + p;
                    const int j = jt * 128 + 32 * q + 16 * jb + i;
                    const size_t d = ((size_t)jt * nkbs + kb) * chunk + (size_t)w * (chunk / 8) +
                                     (size_t)(v * 64 + ln) * E + e;
                    SHT_ASSERT((long long)d < syn_len);
                    sb[d] = (r < nm && j < Jh) ? (T)col[(size_t)r * Jh + j] : (T)0;
                  }
      }
    });
  }
  for (auto& th : pool) th.join();
}

template void fill_table_level<float>(const LevelDesc&, const double*, const double*, float*, const long long*, float*,
                                      const long long*, int*, double*, const long long*);
template void fill_table_level<double>(const LevelDesc&, const double*, const double*, double*, const long long*,
                                       double*, const long long*, int*, double*, const long long*);

}  // namespace sht
