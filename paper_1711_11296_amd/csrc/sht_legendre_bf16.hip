// Legendre stage in the split-bfloat16 form (the transform, the tile lists
// and the FP32 table layouts are those of sht_legendre.hip): the FP32
// operands are split into three bfloat16 pieces inside the kernels, six
// piece products per term run on the bfloat16 matrix cores, FP32
// accumulation.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "sht_device.h"
#include "sht_internal.h"

namespace sht {

// ---------------------------------------------------------------------------
// Split-bfloat16 form.  An FP32 value x is written as x = x0 + x1 + x2 with
// bfloat16 pieces: x0 = bf16(x), x1 = bf16(x - x0), x2 = x - x0 - x1, each
// rounded to nearest.  The splitting is exact: x - x0 is a multiple of the
// FP32 unit of x below half a bfloat16 unit, so it has at most 16
// significant bits, and the last remainder at most 8, which bfloat16 holds.
// |x1| <= 2^-8 |x| and |x2| <= 2^-16 |x|.  A product a*b is accumulated in
// FP32 from the six piece products whose piece indices sum to at most 2,
// smallest first (a2 b0, a1 b1, a0 b2, a1 b0, a0 b1, a0 b0); every piece
// product is exact in FP32 and the three dropped ones are below 2^-23 |a b|
// together, the size of one FP32 rounding.
//
// Both operands are split in the kernels: the table from its FP32 copies
// (the same arrays the FP32 form reads), the workspace or spectra when they
// are staged in LDS, where they are stored as three bfloat16 planes laid out
// for the matrix-core reads.  Memory traffic is therefore that of the FP32
// form, and the matrix work is 6 bfloat16 steps of 16x16x32 per 8 FP32
// steps of 16x16x4 with each step at 8 times the FP32 rate per cycle.
//
// MFMA: v_mfma_f32_16x16x32_bf16.  Lane l supplies 8 values of row (A) or
// column (B) l%16 in the contraction slots 8*(l/16) .. 8*(l/16)+7; element i
// of its result is row 4*(l/16) + i, column l%16.  Which contraction index
// sits in which slot is free as long as A and B agree; the kernels use the
// assignment the FP32 table copies already have (below).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// three bfloat16 pieces of n floats (n = 4 or 8), rounded to nearest
template <typename F, typename B>
__device__ __forceinline__ void split3(F x, B (&pc)[3]) {
  pc[0] = __builtin_convertvector(x, B);
  const F r = x - __builtin_convertvector(pc[0], F);
  pc[1] = __builtin_convertvector(r, B);
  pc[2] = __builtin_convertvector(r - __builtin_convertvector(pc[1], F), B);
}

// acc += a * b from the pieces of both operands
__device__ __forceinline__ f32x4 mfma6(const bf16x8 (&a)[3], const bf16x8 (&b)[3], f32x4 acc) {
  acc = mfma_bf16(a[2], b[0], acc);
  acc = mfma_bf16(a[1], b[1], acc);
  acc = mfma_bf16(a[0], b[2], acc);
  acc = mfma_bf16(a[1], b[0], acc);
  acc = mfma_bf16(a[0], b[1], acc);
  acc = mfma_bf16(a[0], b[0], acc);
  return acc;
}

// Pieces of the right-hand operand in LDS: [piece][parity][column][PITCH]
// bfloat16, the 32 contraction slots of a column contiguous and padded to
// 80 bytes, so that the 16-byte reads of 8 consecutive columns (one LDS
// cycle) fall on 8 distinct groups of 4 banks.
constexpr int kX6Pitch = 40;

// ---------------------------------------------------------------------------
// analysis: C[n][c] = P[n][j] * B_par(n)[j][c]
// tile = 128 rows r = n - m (both parities) x BN = 16*NCB columns, 4 waves.
// Wave w: parity p = w & 1, row half q = w >> 1; it owns the 32 rows
// r = 64 q + 32 h + 2 i + p (h < 2, two MFMA row blocks) and all NCB column
// blocks; each B read feeds both row blocks.  The contraction runs over
// latitudes in blocks of 32; lane (i, g) holds, in slot 8 g + e (e < 8),
// latitude 4 e + g of the block: exactly the values its run of the FP32
// analysis table copy holds (that copy is blocked for 16-row runs; row
// block h of wave (q, p) is run 4 q + 2 h + p).
// The workspace block (both parities, 32 x BN) is fetched into registers one
// block ahead, split and stored into LDS; one LDS stage per workgroup and
// two workgroups per CU, one in its split/store phase while the other runs
// its matrix steps.
// ---------------------------------------------------------------------------
template <int NCB>
struct X6Analysis {
  static constexpr int BN = 16 * NCB;
  static constexpr int KB = 32;                      // latitudes per block
  static constexpr int PLANE = 2 * BN * kX6Pitch;    // bfloat16 per piece
  static constexpr int TASKS = 2 * BN;               // (parity, column quad, g)
  static constexpr int TR = (TASKS + 255) / 256;     // task rounds per thread
  static constexpr int CS = BN + 1;                  // output staging pitch
  static constexpr size_t lds_bytes() {
    const size_t main = (size_t)3 * PLANE * 2;
    const size_t cst = (size_t)64 * CS * 4;
    return main > cst ? main : cst;
  }
};

template <int NCB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_legendre_analysis_bf16(const GemmArgs g) {
  using S = X6Analysis<NCB>;
  constexpr int BN = S::BN, KB = S::KB, P = kX6Pitch;
  typedef float f4 __attribute__((ext_vector_type(4)));

  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* Bs = reinterpret_cast<__bf16*>(smem_raw);

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int r0 = t.rb * 128;
  const int c0 = t.cb * BN;
  const int Kp = L.Kp;
  const long long Cp = L.Cp;
  const long long plane = (long long)Kp * Cp;
  const float* wsm = static_cast<const float*>(g.ws) + L.ws_off + (2LL * m) * plane + c0;

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int p = w & 1, q = w >> 1;
  const int li = lane & 15, lg = lane >> 4;
  const bool active = r0 + 64 * q + p < nm;
  // run 4 q + p of the table block; row block h adds two runs
  const float* arow = static_cast<const float*>(g.table) + g.tab_off[L.m_base + m] +
                      (long long)t.rb * Kp * 128 + (4 * q + p) * 16 * KB + lane * 4;

  f32x4 acc[2][NCB];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[h][c] = f32x4{0, 0, 0, 0};

  // table: two K blocks ahead in two register sets (loop unrolled by two);
  // [h][v]: vector v holds slots 4 v .. 4 v + 3
  f4 an[2][2][2];
  // workspace: one K block ahead; task u = ((par * BN/4) + cq) * 4 + gg holds
  // latitudes 4 e + gg (e < 8) of columns 4 cq .. 4 cq + 3 of parity par
  f4 bq[S::TR][8];
  auto gload_a = [&](int kb, f4 (&av)[2][2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < 2; ++v)
        av[h][v] = *reinterpret_cast<const f4*>(arow + (long long)kb * 128 * KB + h * 32 * KB + v * 256);
  };
  auto gload_b = [&](int kb) {
#pragma unroll
    for (int i = 0; i < S::TR; ++i) {
      int u = tid + i * 256;
      if (S::TR * 256 != S::TASKS && u >= S::TASKS) u = S::TASKS - 1;  // clamped, not stored
      const int gg = u & 3, cq = (u >> 2) % (BN / 4), par = (u >> 2) / (BN / 4);
      const float* src = wsm + par * plane + (long long)(kb * KB + gg) * Cp + 4 * cq;
#pragma unroll
      for (int e = 0; e < 8; ++e) bq[i][e] = *reinterpret_cast<const f4*>(src + 4LL * e * Cp);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int i = 0; i < S::TR; ++i) {
      const int u = tid + i * 256;
      if (S::TR * 256 == S::TASKS || u < S::TASKS) {
        const int gg = u & 3, cq = (u >> 2) % (BN / 4), par = (u >> 2) / (BN / 4);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const f32x8 x = {bq[i][0][cc], bq[i][1][cc], bq[i][2][cc], bq[i][3][cc],
                           bq[i][4][cc], bq[i][5][cc], bq[i][6][cc], bq[i][7][cc]};
          bf16x8 pc[3];
          split3(x, pc);
#pragma unroll
          for (int k = 0; k < 3; ++k)
            *reinterpret_cast<bf16x8*>(Bs + k * S::PLANE + (par * BN + 4 * cq + cc) * P + 8 * gg) = pc[k];
        }
      }
    }
  };
  auto compute = [&](const f4 (&av)[2][2]) {
    bf16x8 a[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const f32x8 x = {av[h][0][0], av[h][0][1], av[h][0][2], av[h][0][3],
                       av[h][1][0], av[h][1][1], av[h][1][2], av[h][1][3]};
      split3(x, a[h]);
    }
    const __bf16* Bp = Bs + (p * BN + li) * P + 8 * lg;
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      bf16x8 b[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) b[k] = *reinterpret_cast<const bf16x8*>(Bp + k * S::PLANE + c * 16 * P);
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h][c] = mfma6(a[h], b, acc[h][c]);
    }
  };
  const int nkb = Kp / KB;
  // one K block; H = kb & 1 selects the table registers of block kb (and of
  // kb + 2).  Loads past the end are clamped to the last block (never used),
  // which keeps memory operations out of branches.
  auto step = [&](auto hc, int kb) {
    constexpr int H = decltype(hc)::value;
    lds_barrier();  // every wave is done reading the previous block
    lstore();
    gload_b(kb + 1 < nkb ? kb + 1 : nkb - 1);
    lds_barrier();
    f4 ac[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < 2; ++v) ac[h][v] = an[H][h][v];
    gload_a(kb + 2 < nkb ? kb + 2 : nkb - 1, an[H]);
    if (active) compute(ac);
  };

  gload_a(0, an[0]);
  gload_b(0);
  gload_a(nkb > 1 ? 1 : 0, an[1]);
  for (int kb = 0; kb < nkb; kb += 2) {
    step(std::integral_constant<int, 0>{}, kb);
    if (kb + 1 < nkb) step(std::integral_constant<int, 1>{}, kb + 1);
  }

  // stage 64 rows at a time in LDS, then write spec rows contiguously
  float* Cs = reinterpret_cast<float*>(smem_raw);  // [64][CS]
  float* spec = static_cast<float*>(g.spec_out) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long base = spec_idx(N, m, m);
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    __syncthreads();
    if (q == hh) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
          for (int i = 0; i < 4; ++i) Cs[(32 * h + 2 * (4 * lg + i) + p) * S::CS + c * 16 + li] = acc[h][c][i];
    }
    __syncthreads();
    for (int qq = tid; qq < 64 * (BN / 2); qq += 256) {
      const int fl = qq >> 6, rl = qq & 63;
      const int f = (c0 >> 1) + fl;
      const int r = r0 + 64 * hh + rl;
      if (r < nm && f < L.F) {
        float* d = spec + ((long long)f * nc + base + r) * 2;
        d[0] = Cs[rl * S::CS + 2 * fl];
        d[1] = Cs[rl * S::CS + 2 * fl + 1];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// synthesis: S_p[j][c] = sum_{r of parity p} P[r][j] * a[r][c]
// tile = 128 latitudes x BN = 16*NCB columns, both parities, 8 waves.  Wave
// w: parity p = w & 1, latitude quarter q = w >> 1; it owns the 32
// latitudes j = 32 q + 16 jb + i (jb < 2) and all NCB column blocks.  The
// contraction runs over r' (r = 2 r' + p) in blocks of 32 per parity (64
// natural rows, two blocks of the FP32 synthesis table copy); lane (i, g)
// holds in slot 8 g + 4 s + u (s < 2, u < 4) r' = 16 s + 4 g + u of the
// block, which is what its run of table block 2 kb + s holds.
// The spectra of a block (64 rows x BN/2 fields) are fetched into
// registers two blocks ahead, split and stored into the other of two LDS
// stages; one barrier per block.
// ---------------------------------------------------------------------------
template <int NCB>
struct X6Synthesis {
  static constexpr int BN = 16 * NCB;
  static constexpr int PLANE = 2 * BN * kX6Pitch;   // bfloat16 per piece
  static constexpr int STAGE = 3 * PLANE;
  static constexpr int TASKS = 4 * BN;              // (field, g, s): 8 natural rows
  static constexpr int TR = (TASKS + 511) / 512;
  static constexpr int CHUNK = 128 * 32;            // FP32 table block (32 natural rows)
  static constexpr size_t lds_bytes() { return (size_t)2 * STAGE * 2; }
};

template <int NCB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_legendre_synthesis_bf16(const GemmArgs g) {
  using S = X6Synthesis<NCB>;
  constexpr int BN = S::BN, P = kX6Pitch;
  typedef float f4 __attribute__((ext_vector_type(4)));

  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* Bs = reinterpret_cast<__bf16*>(smem_raw);  // [2 stage][3 piece][2 parity][BN][P]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int nkb = (nm + 63) / 64;       // blocks of 64 natural rows
  const int nkb32 = (nm + 31) / 32;     // blocks of the FP32 table copy
  const int jt = t.rb;
  const int c0 = t.cb * BN;
  const long long Cp = L.Cp;
  const float* spec = static_cast<const float*>(g.spec_in) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long sbase = spec_idx(N, m, m);

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int p = w & 1, q = w >> 1;
  const int li = lane & 15, lg = lane >> 4;
  const bool active = jt * 128 + 32 * q < L.Jh;
  const float* arun = static_cast<const float*>(g.table) + g.tab_off[L.m_base + m] +
                      (long long)jt * nkb32 * S::CHUNK + w * (S::CHUNK / 8) + lane * 4;

  f32x4 acc[2][NCB];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[jb][c] = f32x4{0, 0, 0, 0};

  // The tile's spectra as a buffer starting at its first field and wave
  // number: reads past the end of the level's spectra return zero (fields
  // beyond F), rows beyond n = N are masked; offsets stay below 4 GiB.
  const long long sfirst = ((long long)(c0 >> 1) * nc + sbase) * 2;
  const long long sbytes = ((long long)L.F * nc * 2 - sfirst) * 4LL;
  const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(spec + sfirst), (short)0, (int)(unsigned)(sbytes > 0xFFFFFFFFLL ? 0xFFFFFFFFLL : sbytes),
      0x00020000);

  // operands two blocks ahead in two register sets (loop unrolled by two):
  // an[s][jb] = table block 2 kb + s, latitude block jb; task u = (fl, gg, s)
  // with s fastest holds natural rows 32 s + 8 gg .. + 7 (re, im) of field fl
  f4 an[2][2][2], ac[2][2];
  f4 rq[2][S::TR][4];
  auto gload = [&](int kb, f4 (&av)[2][2], f4 (&bq)[S::TR][4]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int k32 = 2 * kb + s < nkb32 ? 2 * kb + s : nkb32 - 1;  // clamped: those rows are masked
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
        av[s][jb] = *reinterpret_cast<const f4*>(arun + (long long)k32 * S::CHUNK + jb * 256);
    }
#pragma unroll
    for (int i = 0; i < S::TR; ++i) {
      const int u = tid + i * 512;  // tasks past the end read zeros, beyond the buffer
      const int s = u & 1, gg = (u >> 1) & 3, fl = u >> 3;
      const int r = kb * 64 + 32 * s + 8 * gg;
      const unsigned off = ((unsigned)fl * (unsigned)nc + (unsigned)r) * 8u;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        bq[i][v] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(srs, (int)(off + 16u * v), 0, 0));
    }
  };
  auto lstore = [&](int stage, const f4 (&bq)[S::TR][4], int kb) {
    __bf16* dst = Bs + stage * S::STAGE;
#pragma unroll
    for (int i = 0; i < S::TR; ++i) {
      const int u = tid + i * 512;
      if (S::TR * 512 == S::TASKS || u < S::TASKS) {
        const int s = u & 1, gg = (u >> 1) & 3, fl = u >> 3;
        const int r = kb * 64 + 32 * s + 8 * gg;
        float x[16];  // natural rows r + k (k < 8), re and im
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) x[4 * v + e] = r + (4 * v + e) / 2 < nm ? bq[i][v][e] : 0.f;
#pragma unroll
        for (int par = 0; par < 2; ++par)
#pragma unroll
          for (int ri = 0; ri < 2; ++ri) {
            // rows r + 2 u' + par, u' < 4: r' = 16 s + 4 gg + u'
            const f4 y = {x[2 * par + ri], x[4 + 2 * par + ri], x[8 + 2 * par + ri], x[12 + 2 * par + ri]};
            bf16x4 pc[3];
            split3(y, pc);
#pragma unroll
            for (int k = 0; k < 3; ++k)
              *reinterpret_cast<bf16x4*>(dst + k * S::PLANE + (par * BN + 2 * fl + ri) * P + 8 * gg + 4 * s) = pc[k];
          }
      }
    }
  };
  auto compute = [&](int stage) {
    bf16x8 a[2][3];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const f32x8 x = {ac[0][jb][0], ac[0][jb][1], ac[0][jb][2], ac[0][jb][3],
                       ac[1][jb][0], ac[1][jb][1], ac[1][jb][2], ac[1][jb][3]};
      split3(x, a[jb]);
    }
    const __bf16* Bp = Bs + stage * S::STAGE + (p * BN + li) * P + 8 * lg;
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      bf16x8 b[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) b[k] = *reinterpret_cast<const bf16x8*>(Bp + k * S::PLANE + c * 16 * P);
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) acc[jb][c] = mfma6(a[jb], b, acc[jb][c]);
    }
  };
  // one K block; H = kb & 1 selects the register set of block kb (and of
  // kb + 2), 1 - H that of block kb + 1
  auto step = [&](auto hc, int kb) {
    constexpr int H = decltype(hc)::value;
    gload(kb + 2 < nkb ? kb + 2 : nkb - 1, an[H], rq[H]);
    if (active) compute(H);
    // after the last block this fills the idle stage with a clamped block
    // (nothing reads it)
    lstore(1 - H, rq[1 - H], kb + 1 < nkb ? kb + 1 : nkb - 1);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) ac[s][jb] = an[1 - H][s][jb];
    lds_barrier();
  };

  gload(0, an[0], rq[0]);
  gload(nkb > 1 ? 1 : 0, an[1], rq[1]);
  lstore(0, rq[0], 0);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) ac[s][jb] = an[0][s][jb];
  __syncthreads();
  for (int kb = 0; kb < nkb; kb += 2) {
    step(std::integral_constant<int, 0>{}, kb);
    if (kb + 1 < nkb) step(std::integral_constant<int, 1>{}, kb + 1);
  }

  if (!active) return;
  const long long plane = (long long)L.Kp * Cp;
  float* ws = static_cast<float*>(g.ws) + L.ws_off + (2LL * m + p) * plane;
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = jt * 128 + 32 * q + 16 * jb + 4 * lg + i;
      if (j < L.Jh) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) ws[(long long)j * Cp + c0 + c * 16 + li] = acc[jb][c][i];
      }
    }
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
template <int NCB>
static hipError_t launch_bf16_ncb(bool analysis, const GemmArgs& g, hipStream_t st) {
  const dim3 grid(g.ntiles);
  if (analysis) {
    const size_t lds = X6Analysis<NCB>::lds_bytes();
    lds_optin<k_legendre_analysis_bf16<NCB>>(lds);
    hipLaunchKernelGGL((k_legendre_analysis_bf16<NCB>), grid, dim3(256), lds, st, g);
  } else {
    const size_t lds = X6Synthesis<NCB>::lds_bytes();
    lds_optin<k_legendre_synthesis_bf16<NCB>>(lds);
    hipLaunchKernelGGL((k_legendre_synthesis_bf16<NCB>), grid, dim3(512), lds, st, g);
  }
  return hipGetLastError();
}

hipError_t launch_legendre_bf16(bool analysis, const GemmArgs& g, int ncb, hipStream_t st) {
  switch (ncb) {
    case 1: return launch_bf16_ncb<1>(analysis, g, st);
    case 2: return launch_bf16_ncb<2>(analysis, g, st);
    case 4: return launch_bf16_ncb<4>(analysis, g, st);
    case 5: return launch_bf16_ncb<5>(analysis, g, st);
    case 8: return launch_bf16_ncb<8>(analysis, g, st);
    case 10: return launch_bf16_ncb<10>(analysis, g, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sht
