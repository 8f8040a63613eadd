// Internal declarations shared by the host planner, the kernels and the C ABI.
#ifndef SHT_INTERNAL_H_
#define SHT_INTERNAL_H_

#include <cstddef>
#include <cstdint>

#include "../../include/sht.h"

#define SHT_MAX_LEVELS 8
#define SHT_MAX_RADICES 12
#define SHT_MAX_I 4096

// Latitude (contraction) dimension of the table and workspace is padded to a
// multiple of this.
#define SHT_K_PAD 32

namespace sht {

// ---- host planning (sht_host.cpp) ----
bool grid_args_ok(int J, int kind);
void grid_nodes(int J, int kind, double* mu, double* sint);
void grid_weights(int J, int kind, double* w);
void alf_column(int N, int m, int nr, const double* mu, const double* sint,
                double* out, long ld);
void alf_table(int N, int nr, const double* mu, const double* sint,
               double* out, int nthreads);
bool factor_radices(int I, int* rad, int* nrad);

// ---- device-side descriptors ----

// One transform level as the kernels see it.
struct LevelDesc {
  int N, J, I, F;
  int Jh;      // ceil(J/2): folded rows (northern rows incl. equator)
  int Kp;      // Jh padded to SHT_K_PAD
  int Cp;      // workspace row length (columns = 2F padded)
  int nrad;
  int rad[SHT_MAX_RADICES];   // radix of each Stockham pass
  int pns[SHT_MAX_RADICES];   // product of the radices of the earlier passes
  int ptw[SHT_MAX_RADICES];   // twiddle index stride I / (pns * rad)
  unsigned pmag[SHT_MAX_RADICES];  // floor((2^32-1)/pns) + 1 (0 when pns == 1)
  int fft_item0;   // first FFT work item of this level
  int nfb;         // field blocks of the FFT kernels
  int m_base;      // index of (level, m=0) in the per-m offset arrays
  int zk;          // zonal stage, one-launch multi-level kernel: configuration of this level (set at launch)
  int wsh;         // log2 of the analysis workspace column block W = min(2 FB, 16) (ws_col)
  long long grid_off;  // element offset of this level in the grid buffer
  long long spec_off;  // element offset of this level in the spec buffer
  long long ws_off;    // element offset in the workspace
  long long wplane;    // half the workspace elements from one wavenumber's region to the next (ws_plane)
  long long spoff;     // synthesis: offset of the odd-parity plane in a region (wplane, or Jh Cp when Kp > Jh)
  const void* tw;      // I twiddles exp(-2 pi i k / I), complex, data type
  const double* wrow;  // Jh quadrature weights of the northern rows
  const double* murow; // Kp nodes mu_j of the northern rows, zero past Jh (analysis with generated P~)
};

struct FftArgs {
  int nlev;
  int nitems;
  LevelDesc lev[SHT_MAX_LEVELS];
  const void* src;   // grid (analysis) or workspace (synthesis)
  void* dst;         // workspace (analysis) or grid (synthesis)
  // scalars: value *= (use_w ? w_j : 1) * (use_inv_I ? 1/I : 1) * (m ? mscale : 1)
  int use_w;
  int use_inv_I;
  double mscale;
  int tw_lds;        // element offset of the LDS twiddle table (set at launch)
  int fb;            // fields per work item (zonal_fields_per_block)
  int one_launch;    // multi-level plans: one launch over all levels where they allow it
  // per (level, m): first latitude of the Legendre sums (reduced transform;
  // null otherwise); the synthesis leaves whole 128-latitude tiles below it
  // out of the workspace, and the zonal synthesis reads them as zero
  const int* jstart;
};

// One work tile of a Legendre kernel; level < 0 marks an idle slot.
struct Tile {
  int level, m, rb, cb;
};

struct GemmArgs {
  int nlev;
  int ntiles;
  LevelDesc lev[SHT_MAX_LEVELS];
  const Tile* tiles;           // one per workgroup
  const long long* tab_off;    // per (level, m): element offset of the table block
  const void* table;           // P~ table copy (FP64 in the FP64 form, else FP32)
  const int* jstart;           // per (level, m): first latitude of the sums (reduced transform; else 0)
  const void* spec_in;         // synthesis: spectra
  void* spec_out;              // analysis: spectra
  void* ws;                    // workspace
  // analysis with P~ generated in the kernel (FP64): per (level, m) the two
  // seed rows P~_{m+16g}, P~_{m+16g+1} of every 16-degree group g, each Kp
  // long, and the recurrence coefficients (A_r, B_r) of the rows r = n - m,
  // P~_n = A_r mu P~_{n-1} - B_r P~_{n-2}
  const double* seeds;
  const long long* seed_off;
  const double* rec;
  const long long* rec_off;
};

// ---- kernel launchers (sht_fft.hip, sht_legendre.hip) ----
// The stream argument is a hipStream_t.
// Fields per zonal work item: 4 (FP64) or 8, and 16 for large single-level
// FP32-data plans whose fixed-length kernel holds one wavenumber per thread
// (I = 1440 or 480), so that every workspace run is a whole 128-byte line.
// The level's workspace size with that blocking must be below 4 GiB (the
// planner checks and falls back to 8).
int zonal_fields_per_block(int form, int nlev, int N, int J, int I, int F);
// Workspace layout (per level).  The region of wavenumber m starts
// 2 wplane elements after that of m - 1 and holds Kp rows j of 2 Cp
// elements (rows j >= ceil(J/2) stay zero), for the columns
// c = 2 field + {re, im} < Cp of both parities p.  The two directions use
// it differently (each writes and reads its own):
// * synthesis (and forward adjoint): two planes, parity p at p spoff,
//   row j < ceil(J/2) at j Cp, column c; spoff = wplane, or ceil(J/2) Cp
//   when Kp > ceil(J/2), so that these planes never overlap the rows the
//   analysis keeps zero;
// * analysis (and inverse adjoint): row j at 2 j Cp holds both parities in
//   blocks of W = 2^wsh = min(2 FB, 16) columns, [column block][parity][W]
//   (ws_col): the columns of a zonal work item are one block (two for
//   16-field items), so the item's stores for one m are one contiguous run
//   of 4 FB elements (128 bytes for 8 FP32 fields), and each latitude row
//   of a Legendre analysis tile is one run over both parities.
// Offset of (parity, column c) within an analysis row:
constexpr int ws_col(int wsh, int par, int c) {
  return ((c >> wsh) << (wsh + 1)) + (par << wsh) + (c & ((1 << wsh) - 1));
}
// wplane is one parity's share of a region, Kp Cp elements, plus a pad, so
// that the regions of consecutive wavenumbers (one wave's 64 lanes in the
// zonal kernels) do not start at the same offset modulo the large powers of
// two that HBM channels are interleaved by.
constexpr long long kWsPlanePad = 32;  // elements (a multiple of 16; chosen by measurement)
inline long long ws_plane(long long Kp, long long Cp) { return Kp * Cp + kWsPlanePad; }
// The fixed-length zonal kernels address the workspace with 32-bit byte
// offsets from a per-wave base: 64 wavenumbers x 2 wplane must stay below
// 4 GiB (else the runtime-radix kernels run).
inline bool zonal_offsets_fit(long long wplane, long long elem) {
  return 128.0 * (double)wplane * (double)elem < 4294967296.0;
}
// 1 if the one-launch multi-level zonal kernel of this form and direction
// keeps values in scratch memory (register spills), else 0
int zonal_one_launch_spills(int form, bool analysis);
int launch_zonal(int form, bool analysis, const FftArgs& a, int maxN, void* stream);
// gen: generate P~ in the kernels from the plan's seed rows instead of
// reading a table (plan option otf)
int launch_legendre(int form, bool analysis, const GemmArgs& g, int ncb, bool gen, void* stream);
// Transfers between truncations and nested grids (sht_transfer.hip).
int launch_retruncate(int Nin, int Nout, int F, bool dbl, const void* in, void* out, void* stream);
int launch_inject(int Jf, int If, int Jc, int Ic, int F, int rs, int r0, int cs, bool dbl, const void* fine,
                  void* coarse, void* stream);
// Zero units [first16, first16 + len16) (16-byte units) of nplanes planes
// spaced pitch16 units apart, starting at base (16-byte aligned).
int launch_clear_span(void* base, long long nplanes, long long pitch16, long long first16, long long len16,
                      void* stream);
int launch_product(long long n, bool dbl, const void* a, const void* b, void* out, void* stream);
int launch_laplacian(int N, int F, double scale, bool dbl, const void* in, void* out, void* stream);
int launch_residual(long long n, long long n_per, double alpha, bool dbl, const void* x, const void* kappa,
                    const void* y, const void* f, void* r, void* stream);
// Widest column blocking (16-column units) a Legendre kernel of a form takes.
int max_ncb(int form, bool analysis);

}  // namespace sht

#endif  // SHT_INTERNAL_H_
