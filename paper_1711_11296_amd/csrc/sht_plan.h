// Host-side layout planning of the transform library: the per-level sizes
// and offsets of the tables, seed rows and workspace, the tile lists of the
// Legendre kernels, and the filling of the blocked table copies.  Plain C++
// (no HIP), so that it is built into the library and, with bounds
// assertions (SHT_CHECK) and sanitizers, into a CPU check.
#ifndef SHT_PLAN_H_
#define SHT_PLAN_H_

#include <vector>

#include "sht_internal.h"

#ifdef SHT_CHECK
#include <cstdio>
#include <cstdlib>
#define SHT_ASSERT(c)                                                                   \
  do {                                                                                  \
    if (!(c)) {                                                                         \
      std::fprintf(stderr, "SHT_CHECK failed: %s (%s:%d)\n", #c, __FILE__, __LINE__); \
      std::abort();                                                                     \
    }                                                                                   \
  } while (0)
#else
#define SHT_ASSERT(c) ((void)0)
#endif

namespace sht {

inline long long roundup(long long a, long long b) { return (a + b - 1) / b * b; }

// Column blocking shared by all levels: the one that pads the least
// (weighted by the Legendre work), preferring wider tiles on ties.
int choose_ncb(int form, int nlev, const int* N, const int* J, const int* F);

// Offsets of one plan's per-(level, m) blocks and its totals (elements);
// each offset vector has one sentinel entry past the last (level, m).
struct Layout {
  std::vector<long long> taboff;      // analysis table copy
  std::vector<long long> taboff_syn;  // synthesis table copy
  std::vector<long long> seedoff;     // seed rows of generated P~
  std::vector<long long> recoff;      // recurrence coefficients
  long long tab = 0, tabs = 0, seeds = 0, rec = 0;
  long long items = 0;                // zonal work items
  long long grid = 0, spec = 0, ws = 0;
  int nm_total = 0;                   // (level, m) pairs
};

// Fill the level descriptors (sizes, FFT radices, offsets; the device
// pointers stay null) for column tiles of BN columns and zonal items of FB
// fields, and the offsets of every (level, m) block.
void layout_levels(int nlev, const int* N, const int* J, const int* I, const int* F, int BN, int FB,
                   LevelDesc* lev, Layout* out);

// Tile list of one Legendre kernel for column blocking ncb (16*ncb columns
// per tile; every level's workspace row length Cp must be a multiple of it).
// jst: per (level, m) first latitude kept (reduced transform; else 0).
// sched 0: locality order (m, column block, row block) cut into 8 chunks of
// equal cost, chunk x dealt to block ids == x (mod 8), i.e. to XCD x;
// sched 1: the same order dealt round robin.
std::vector<Tile> build_tiles(int form, int nlev, const LevelDesc* lev, const int* jst, bool analysis, int ncb,
                              int sched);

// Fill both blocked copies of one level's table (dst / dsyn may be null:
// then only j0 and seeds are produced) from FP64 columns of P~; j0 (may be
// null): per m the first latitude with some |P~_n^m| >= 1e-16; seeds (may be
// null): rows 16 g and 16 g + 1 of every 16-degree group g, Kp long.  The
// per-m offsets are those of layout_levels.
template <typename T>
void fill_table_level(const LevelDesc& L, const double* mu, const double* sint, T* dst, const long long* off_a,
                      T* dsyn, const long long* off_s, int* j0, double* seeds, const long long* off_seed);

}  // namespace sht

#endif  // SHT_PLAN_H_
