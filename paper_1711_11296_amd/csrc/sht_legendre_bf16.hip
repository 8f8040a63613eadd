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

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Three bfloat16 pieces of a pair of floats, rounded to nearest, packed two
// per 32-bit word (low half = first value).  The remainders x - x0 are
// formed by the bfloat16 dot-product instruction as x + (-1) x0 + (-0) x0':
// its products are exact and the sum is representable, so it is exact.
// (The weight pairs are written with -0 rather than +0 so that they stay
// 32-bit literals: (-1, +0) would be encoded as the inline constant -1.0,
// which the instruction does not read as the bfloat16 pair (-1, 0).)
__device__ __forceinline__ unsigned cvt_pk_bf16(float a, float b) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ __forceinline__ void split_pair(float x0, float x1, unsigned (&pc)[3]) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 neg_lo = __builtin_bit_cast(bf16x2, 0x8000BF80u);  // (-1, -0)
  const bf16x2 neg_hi = __builtin_bit_cast(bf16x2, 0xBF808000u);  // (-0, -1)
  pc[0] = cvt_pk_bf16(x0, x1);
  const bf16x2 h = __builtin_bit_cast(bf16x2, pc[0]);
  const float r0 = __builtin_amdgcn_fdot2_f32_bf16(h, neg_lo, x0, false);
  const float r1 = __builtin_amdgcn_fdot2_f32_bf16(h, neg_hi, x1, false);
  pc[1] = cvt_pk_bf16(r0, r1);
  const bf16x2 mm = __builtin_bit_cast(bf16x2, pc[1]);
  pc[2] = cvt_pk_bf16(__builtin_amdgcn_fdot2_f32_bf16(mm, neg_lo, r0, false),
                      __builtin_amdgcn_fdot2_f32_bf16(mm, neg_hi, r1, false));
}
// pieces of n = 4 or 8 floats as bfloat16 vectors (B = bf16x4 or bf16x8)
template <int n, typename B>
__device__ __forceinline__ void split3(const float (&x)[n], B (&pc)[3]) {
  typedef unsigned U __attribute__((ext_vector_type(n / 2)));
  U w[3];
#pragma unroll
  for (int i = 0; i < n / 2; ++i) {
    unsigned t[3];
    split_pair(x[2 * i], x[2 * i + 1], t);
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k][i] = t[k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) pc[k] = __builtin_bit_cast(B, w[k]);
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

// Both kernels step through K blocks with two LDS stages and one barrier
// per block: the matrix cores multiply block kb (table pieces in registers,
// right-hand pieces in LDS stage kb & 1); then the wave splits block kb + 1,
// fetched one block earlier (table values into its registers, right-hand
// values into the other LDS stage); block kb + 2 is in flight meanwhile.
// The split work is a list of units: unit u < 8 splits one pair of table
// values, the others one pair of right-hand values and, after the second
// pair of a column, store its three 8-byte pieces.  Threads without a
// right-hand task (when the block has fewer tasks than threads) store into
// the padding slots 32..39 of a column, which no matrix step reads.  Waves
// without rows (latitudes) in the tile run the same steps without the
// products: the choice is made once, outside the loop, so that the loop
// body has no branches (the accumulators then stay in their registers).
// ---------------------------------------------------------------------------
// analysis: C[n][c] = P[n][j] * B_par(n)[j][c]
// tile = 256 rows r = n - m (two 128-row blocks of the table copy, both
// parities) x BN = 16*NCB columns, 8 waves.  Wave w: row block th = w >> 2,
// quarter q = (w >> 1) & 1, parity p = w & 1; it owns the 32 rows
// r = 128 th + 64 q + 32 h + 2 i + p (h < 2, two MFMA row blocks) and all
// NCB column blocks, so that each B read feeds both row blocks.  The
// contraction runs over latitudes in blocks of 32; lane (i, g) holds, in
// slot 8 g + e (e < 8), latitude 4 e + g of the block: exactly the values
// its run of the FP32 analysis table copy holds (that copy is blocked for
// 16-row runs; row block h of wave (q, p) is run 4 q + 2 h + p).  A second
// 128-row block past the end of the rows is not read: its waves fetch the
// first block's runs again (no extra memory traffic) and skip the
// products.  Right-hand task u (eh fastest, then gg, cq, par) holds
// latitudes 4 e + gg (e = 4 eh .. 4 eh + 3) of columns 4 cq .. 4 cq + 3 of
// parity par; its pieces go to slots 8 gg + 4 eh .. + 3.
// ---------------------------------------------------------------------------
template <int NCB>
struct X6Analysis {
  static constexpr int NT = 512;                     // threads (8 waves)
  static constexpr int BN = 16 * NCB;
  static constexpr int KB = 32;                      // latitudes per block
  static constexpr int PLANE = 2 * BN * kX6Pitch;    // bfloat16 per piece
  static constexpr int STAGE = 3 * PLANE;
  static constexpr int TASKS = 4 * BN;               // (parity, column quad, g, half)
  static constexpr int TR = (TASKS + 511) / 512;     // task rounds per thread
  static constexpr int CS = BN + 1;                  // output staging pitch
  static constexpr int PS = 256 * KB;                // GEN: generated block, FP32
  static constexpr size_t lds_bytes(bool gen) {
    const size_t main = (size_t)2 * STAGE * 2 + (gen ? (size_t)PS * 4 : 0);
    const size_t cst = (size_t)64 * CS * 4;
    return main > cst ? main : cst;
  }
};

// Swizzle of the generated analysis block [256 rows][32 latitudes] (FP32):
// element (row, lat) at row * 32 + (lat ^ x6_swz(row)).
__device__ __forceinline__ int x6_swz(int row) { return 2 * ((row >> 1) & 15); }

// GEN: the FP32 table values are generated in the kernel instead (the
// three-term recurrence of Sec. 4.1 in FP64 from the plan's seed rows,
// rounded once to FP32, so that the pieces equal those of the table path):
// per K block thread t produces the 16 rows of group t / 32 of the tile at
// latitude t % 32 into an LDS block; after a barrier each wave reads and
// splits its values, and a second barrier guards the block against the
// next block's writes.
template <int NCB, bool GEN>
__global__ __launch_bounds__(X6Analysis<NCB>::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_legendre_analysis_bf16(const GemmArgs g) {
  using S = X6Analysis<NCB>;
  constexpr int BN = S::BN, KB = S::KB, P = kX6Pitch, TR = S::TR;
  typedef float f4 __attribute__((ext_vector_type(4)));

  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* Bs = reinterpret_cast<__bf16*>(smem_raw);  // [2 stage][3 piece][2 parity][BN][P]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int r0 = t.rb * 256;
  const int c0 = t.cb * BN;
  const int Kp = L.Kp;
  const long long Cp = L.Cp;
  const long long plane = L.wplane;
  const float* wsm = static_cast<const float*>(g.ws) + L.ws_off + (2LL * m) * plane;  // region m

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int th = w >> 2, q = (w >> 1) & 1, p = w & 1;
  const int li = lane & 15, lg = lane >> 4;
  const bool active = r0 + 128 * th + 64 * q + p < nm;
  const int nrb = (nm + 127) / 128;
  const int rbt = 2 * t.rb + th < nrb ? 2 * t.rb + th : nrb - 1;
  // run 4 q + p of the table block; row block h adds two runs
  const float* arow = GEN ? nullptr
                          : static_cast<const float*>(g.table) + g.tab_off[L.m_base + m] +
                                (long long)rbt * Kp * 128 + (4 * q + p) * 16 * KB + lane * 4;
  float* Ps = reinterpret_cast<float*>(Bs + 2 * S::STAGE);  // GEN: [256 rows][32 latitudes], swizzled
  // lanes 0..31 of wave w generate group 2 w, lanes 32..63 group 2 w + 1
  // (rows 16 ggrp .. + 15 of the tile) at latitude glat; the coefficients of
  // both groups are held in their half of the wave for the whole tile
  const int ggrp = tid >> 5, glat = tid & 31;
  const int gi = t.rb * 16 + ggrp;
  const bool gon = GEN && 16 * gi < nm;
  const double* gseed = GEN ? g.seeds + g.seed_off[L.m_base + m] + (gon ? 2LL * gi * Kp : 0LL) : nullptr;
  double gcA = 0.0, gcB = 0.0;
  if constexpr (GEN) gen_coef(g.rec + g.rec_off[L.m_base + m], 16 * gi, nm, lane, gcA, gcB);
  double gmu[2] = {0.0, 0.0}, gx0[2] = {0.0, 0.0}, gx1[2] = {0.0, 0.0};
  auto gen_fetch = [&](int kb, int set) __attribute__((always_inline)) {
    if constexpr (GEN) {
      if (gon) {
        const int j = kb * KB + glat;
        gmu[set] = L.murow[j];
        gx0[set] = gseed[j];
        gx1[set] = gseed[Kp + j];  // zero row when 16 gi + 1 = n_m
      }
    }
  };
  auto gen_store = [&](int set) __attribute__((always_inline)) {
    if constexpr (GEN) {
      gen_rows16<true>(gcA, gcB, 16 * gi, nm, gmu[set], gx0[set], gx1[set], [&](int s2, double x) {
        const int row = 16 * ggrp + s2;
        Ps[row * 32 + (glat ^ x6_swz(row))] = (float)x;
      });
    }
  };
  // right-hand tasks: source offset (latitude 0 of the block) and LDS offset
  const float* bsrc[TR];
  int boff[TR];
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const int u = tid + i * 512;
    const bool valid = TR * 512 == S::TASKS || u < S::TASKS;
    const int uc = valid ? u : S::TASKS - 1;  // loads clamped to a real task
    const int eh = uc & 1, gg = (uc >> 1) & 3, cq = (uc >> 3) % (BN / 4), par = (uc >> 3) / (BN / 4);
    bsrc[i] = wsm + (long long)(16 * eh + gg) * 2 * Cp + ws_col(L.wsh, par, c0 + 4 * cq);
    boff[i] = valid ? (par * BN + 4 * cq) * P + 8 * gg + 4 * eh : 32;
  }

  f32x4 acc[2][NCB];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[h][c] = f32x4{0, 0, 0, 0};

  f4 araw[2][2][2];    // [set][h][v]: vector v holds slots 4 v .. 4 v + 3
  f4 braw[2][TR][4];   // [set][round][e]
  bf16x8 acur[2][3];   // pieces of the table block being multiplied

  auto gload = [&](int kb, int set) __attribute__((always_inline)) {
    if constexpr (!GEN) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int v = 0; v < 2; ++v)
          araw[set][h][v] = *reinterpret_cast<const f4*>(arow + (long long)kb * 128 * KB + h * 32 * KB + v * 256);
    }
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        braw[set][i][e] = *reinterpret_cast<const f4*>(bsrc[i] + (long long)(kb * KB + 4 * e) * 2 * Cp);
  };
  auto split_a = [&](int set) __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float x[8] = {araw[set][h][0][0], araw[set][h][0][1], araw[set][h][0][2], araw[set][h][0][3],
                          araw[set][h][1][0], araw[set][h][1][1], araw[set][h][1][2], araw[set][h][1][3]};
      split3(x, acur[h]);
    }
  };
  // GEN: the wave's values of the generated block, split (slot 8 g + e holds
  // latitude 4 e + g)
  auto gen_split_a = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rr = 128 * th + 64 * q + 32 * h + 2 * li + p;
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = Ps[rr * 32 + ((4 * e + lg) ^ x6_swz(rr))];
      split3(x, acur[h]);
    }
  };
  auto split_b = [&](int set, int stage) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const float x[4] = {braw[set][i][0][cc], braw[set][i][1][cc], braw[set][i][2][cc], braw[set][i][3][cc]};
        bf16x4 pc[3];
        split3(x, pc);
#pragma unroll
        for (int k = 0; k < 3; ++k)
          *reinterpret_cast<bf16x4*>(Bs + stage * S::STAGE + k * S::PLANE + boff[i] + cc * P) = pc[k];
      }
  };
  auto compute = [&](int stage) __attribute__((always_inline)) {
    const __bf16* Bp = Bs + stage * S::STAGE + (p * BN + li) * P + 8 * lg;
    // column blocks in pairs: the six piece products of each term go to one
    // accumulator smallest first, and the four accumulators of a pair (two
    // row blocks by two column blocks) take turns, so that four independent
    // chains keep the bfloat16 matrix pipe busy
#pragma unroll
    for (int c = 0; c < NCB; c += 2) {
      constexpr int CC = 2;
      bf16x8 bb[CC][3];
#pragma unroll
      for (int cc = 0; cc < CC; ++cc)
        if (c + cc < NCB)
#pragma unroll
          for (int k = 0; k < 3; ++k)
            bb[cc][k] = *reinterpret_cast<const bf16x8*>(Bp + k * S::PLANE + (c + cc) * 16 * P);
#pragma unroll
      for (int pr = 0; pr < 6; ++pr) {
        constexpr int ia[6] = {2, 1, 0, 1, 0, 0}, ib[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
        for (int cc = 0; cc < CC; ++cc)
          if (c + cc < NCB)
#pragma unroll
            for (int h = 0; h < 2; ++h) acc[h][c + cc] = mfma_bf16(acur[h][ia[pr]], bb[cc][ib[pr]], acc[h][c + cc]);
      }
    }
  };
  const int nkb = Kp / KB;
  // one K block: raw set 1 - H holds block kb + 1, block kb + 2 goes to set
  // H (clamped past the end: never used, keeps memory operations out of
  // branches)
  auto step = [&](auto act, auto hc, int kb) __attribute__((always_inline)) {
    constexpr bool ACT = decltype(act)::value;
    constexpr int H = decltype(hc)::value;
    gen_fetch(kb + 2 < nkb ? kb + 2 : nkb - 1, H);
    gload(kb + 2 < nkb ? kb + 2 : nkb - 1, H);
    // keep the loads ahead of the block's work (the scheduler would sink
    // them towards their distant uses)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (ACT) {
      compute(H);
      if constexpr (!GEN) split_a(1 - H);
    }
    gen_store(1 - H);  // block kb + 1 (clamped after the last: nothing reads it)
    split_b(1 - H, 1 - H);
    lds_barrier();
    if constexpr (GEN) {
      if constexpr (ACT) gen_split_a();
      lds_barrier();
    }
  };
  // pairs of blocks with a branch-free body, then an odd last block
  // reduced transform: the blocks before kb0 hold only latitudes where
  // every |P~_n^m| < 1e-16 (kb0 = 0 otherwise)
  const int kb0 = min(g.jstart[L.m_base + m] / KB, nkb - 1);
  auto run = [&](auto act) __attribute__((always_inline)) {
    int kb = kb0;
    for (; kb + 1 < nkb; kb += 2) {
      step(act, std::integral_constant<int, 0>{}, kb);
      step(act, std::integral_constant<int, 1>{}, kb + 1);
    }
    if (kb < nkb) step(act, std::integral_constant<int, 0>{}, kb);
  };

  gload(kb0, 0);
  gload(kb0 + 1 < nkb ? kb0 + 1 : nkb - 1, 1);
  if constexpr (GEN) {
    gen_fetch(kb0, 0);
    gen_store(0);
    gen_fetch(kb0 + 1 < nkb ? kb0 + 1 : nkb - 1, 1);
  } else {
    split_a(0);
  }
  split_b(0, 0);
  __syncthreads();
  if constexpr (GEN) {
    if (active) gen_split_a();
    __syncthreads();
  }
  if (active)
    run(std::true_type{});
  else
    run(std::false_type{});

  // stage 64 rows at a time in LDS, then write spec rows contiguously
  float* Cs = reinterpret_cast<float*>(smem_raw);  // [64][CS]
  float* spec = static_cast<float*>(g.spec_out) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long base = spec_idx(N, m, m);
#pragma unroll
  for (int hh = 0; hh < 4; ++hh) {
    if (r0 + 64 * hh >= nm) break;  // uniform across the workgroup
    __syncthreads();
    if ((w >> 1) == hh) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
          for (int i = 0; i < 4; ++i) Cs[(32 * h + 2 * (4 * lg + i) + p) * S::CS + c * 16 + li] = acc[h][c][i];
    }
    __syncthreads();
    for (int qq = tid; qq < 64 * (BN / 2); qq += 512) {
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
// Right-hand task u = (fl, gg, s) holds natural rows 32 s + 8 gg .. + 7
// (re, im) of field fl of the block.  Lane order s, gg, fl bit 1, fl bit 0,
// ...: the 16 lanes of one LDS write cycle cover fields fl and fl + 2,
// whose columns are 80 words apart, so their 8-byte pieces fill all 32
// banks once.
// ---------------------------------------------------------------------------
template <int NCB>
struct X6Synthesis {
  static constexpr int NT = 512;                    // threads (8 waves)
  static constexpr int BN = 16 * NCB;
  static constexpr int PLANE = 2 * BN * kX6Pitch;   // bfloat16 per piece
  static constexpr int STAGE = 3 * PLANE;
  static constexpr int TASKS = 4 * BN;              // (field, g, s): 8 natural rows
  static constexpr int TR = (TASKS + 511) / 512;
  static constexpr int CHUNK = 128 * 32;            // FP32 table block (32 natural rows)
  static constexpr int GP = 130;                    // GEN: pitch of the generated block [64 rows][128 latitudes]
  static constexpr size_t lds_bytes(bool gen) { return (size_t)2 * STAGE * 2 + (gen ? (size_t)64 * GP * 4 : 0); }
};

// GEN: the FP32 table values are generated in the kernel (as in the
// analysis): per block of 64 natural rows wave w produces the 16 rows of
// group w >> 1 at the latitudes 64 (w & 1) + lane of the tile into an LDS
// block [row][GP].
template <int NCB, bool GEN>
__global__ __launch_bounds__(X6Synthesis<NCB>::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_legendre_synthesis_bf16(const GemmArgs g) {
  using S = X6Synthesis<NCB>;
  constexpr int BN = S::BN, P = kX6Pitch, TR = S::TR;
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
  const float* arun = GEN ? nullptr
                          : static_cast<const float*>(g.table) + g.tab_off[L.m_base + m] +
                                (long long)jt * nkb32 * S::CHUNK + w * (S::CHUNK / 8) + lane * 4;
  float* Ps = reinterpret_cast<float*>(Bs + 2 * S::STAGE);  // GEN: [64 rows][GP]
  // wave w generates group w >> 1 of each block (uniform across the wave)
  // at latitude 64 (w & 1) + lane of the tile; the group's recurrence
  // coefficients are fetched into lanes with its seed values
  const int gsub = w >> 1, glat = 64 * (w & 1) + lane;
  const int gj = jt * 128 + glat;
  const bool gjin = GEN && gj < L.Kp;
  const double* gseeds = GEN ? g.seeds + g.seed_off[L.m_base + m] : nullptr;
  const double* grec = GEN ? g.rec + g.rec_off[L.m_base + m] : nullptr;
  const double gmu = gjin ? L.murow[gj] : 0.0;
  double gx0[2] = {0.0, 0.0}, gx1[2] = {0.0, 0.0}, gcA[2] = {0.0, 0.0}, gcB[2] = {0.0, 0.0};
  auto gen_fetch = [&](int kb, int set) __attribute__((always_inline)) {
    if constexpr (GEN) {
      const int gi = 4 * kb + gsub;
      gen_coef(grec, 16 * gi, nm, lane, gcA[set], gcB[set]);
      if (gjin && 16 * gi < nm) {
        gx0[set] = gseeds[2LL * gi * L.Kp + gj];
        gx1[set] = gseeds[(2LL * gi + 1) * L.Kp + gj];  // zero row when 16 gi + 1 = n_m
      }
    }
  };
  auto gen_store = [&](int kb, int set) __attribute__((always_inline)) {
    if constexpr (GEN) {
      const int gi = 4 * kb + gsub;
      gen_rows16<false>(gcA[set], gcB[set], 16 * gi, gjin ? nm : 0, gmu, gx0[set], gx1[set],
                        [&](int s2, double x) { Ps[(16 * gsub + s2) * S::GP + glat] = (float)x; });
    }
  };

  // The tile's spectra as a buffer starting at its first field and wave
  // number: reads past the end of the level's spectra return zero (fields
  // beyond F), rows beyond n = N are masked; offsets stay below 4 GiB.
  const long long sfirst = ((long long)(c0 >> 1) * nc + sbase) * 2;
  long long sbytes = ((long long)L.F * nc * 2 - sfirst) * 4LL;
  if (sbytes < 0) sbytes = 0;  // a tile past the last field (all its reads are zeros)
  const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(spec + sfirst), (short)0, (int)(unsigned)(sbytes > 0xFFFFFFFFLL ? 0xFFFFFFFFLL : sbytes),
      0x00020000);

  // right-hand tasks: first natural row within a block, byte offset of
  // field fl's row 0, LDS offset
  int brow[TR], boff[TR];
  unsigned bsrc[TR];
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const int u = tid + i * 512;
    const bool valid = TR * 512 == S::TASKS || u < S::TASKS;
    const int s = u & 1, gg = (u >> 1) & 3;
    const int fl = (((u >> 3) & 1) << 1) | ((u >> 4) & 1) | ((u >> 5) << 2);
    brow[i] = 32 * s + 8 * gg;
    bsrc[i] = (unsigned)fl * (unsigned)nc * 8u;  // tasks past the end read zeros or other fields; not stored
    boff[i] = valid ? 2 * fl * P + 8 * gg + 4 * s : 32;
  }

  f32x4 acc[2][NCB];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[jb][c] = f32x4{0, 0, 0, 0};

  f4 araw[2][2][2];    // [set][s][jb]: table block 2 kb + s, latitude block jb
  f4 braw[2][TR][4];   // [set][round][v]: rows r + 2 v, r + 2 v + 1 (re, im)
  bf16x8 acur[2][3];

  auto gload = [&](int kb, int set) __attribute__((always_inline)) {
    if constexpr (!GEN) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int k32 = 2 * kb + s < nkb32 ? 2 * kb + s : nkb32 - 1;  // clamped: those rows are masked
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
          araw[set][s][jb] = *reinterpret_cast<const f4*>(arun + (long long)k32 * S::CHUNK + jb * 256);
      }
    }
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const unsigned off = bsrc[i] + (unsigned)(kb * 64 + brow[i]) * 8u;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        braw[set][i][v] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(srs, (int)(off + 16u * v), 0, 0));
    }
  };
  auto split_a = [&](int set) __attribute__((always_inline)) {
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const float x[8] = {araw[set][0][jb][0], araw[set][0][jb][1], araw[set][0][jb][2], araw[set][0][jb][3],
                          araw[set][1][jb][0], araw[set][1][jb][1], araw[set][1][jb][2], araw[set][1][jb][3]};
      split3(x, acur[jb]);
    }
  };
  // GEN: the wave's values of the generated block, split (slot 8 g + 4 s + u
  // holds r' = 16 s + 4 g + u, natural row 2 r' + p)
  auto gen_split_a = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      float x[8];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          x[4 * s2 + u] = Ps[(32 * s2 + 8 * lg + 2 * u + p) * S::GP + 32 * q + 16 * jb + li];
      split3(x, acur[jb]);
    }
  };
  // block kb of raw set `set` into LDS stage `stage`
  auto split_b = [&](int set, int stage, int kb) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const int r = kb * 64 + brow[i];
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
          // rows r + 2 u + par, u < 4: r' = 16 s + 4 gg + u
          float y[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) y[u] = r + 2 * u + par < nm ? braw[set][i][u][2 * par + ri] : 0.f;
          bf16x4 pc[3];
          split3(y, pc);
#pragma unroll
          for (int k = 0; k < 3; ++k)
            *reinterpret_cast<bf16x4*>(Bs + stage * S::STAGE + k * S::PLANE + boff[i] + (par * BN + ri) * P) = pc[k];
        }
    }
  };
  auto compute = [&](int stage) __attribute__((always_inline)) {
    const __bf16* Bp = Bs + stage * S::STAGE + (p * BN + li) * P + 8 * lg;
    // column blocks in pairs, four independent accumulator chains (as in
    // the analysis)
#pragma unroll
    for (int c = 0; c < NCB; c += 2) {
      constexpr int CC = 2;
      bf16x8 bb[CC][3];
#pragma unroll
      for (int cc = 0; cc < CC; ++cc)
        if (c + cc < NCB)
#pragma unroll
          for (int k = 0; k < 3; ++k)
            bb[cc][k] = *reinterpret_cast<const bf16x8*>(Bp + k * S::PLANE + (c + cc) * 16 * P);
#pragma unroll
      for (int pr = 0; pr < 6; ++pr) {
        constexpr int ia[6] = {2, 1, 0, 1, 0, 0}, ib[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
        for (int cc = 0; cc < CC; ++cc)
          if (c + cc < NCB)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
              acc[jb][c + cc] = mfma_bf16(acur[jb][ia[pr]], bb[cc][ib[pr]], acc[jb][c + cc]);
      }
    }
  };
  auto step = [&](auto act, auto hc, int kb) __attribute__((always_inline)) {
    constexpr bool ACT = decltype(act)::value;
    constexpr int H = decltype(hc)::value;
    const int kn = kb + 1 < nkb ? kb + 1 : nkb - 1;
    gen_fetch(kb + 2 < nkb ? kb + 2 : nkb - 1, H);
    gload(kb + 2 < nkb ? kb + 2 : nkb - 1, H);
    // keep the loads ahead of the block's work (the scheduler would sink
    // them towards their distant uses)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (ACT) {
      compute(H);
      if constexpr (!GEN) split_a(1 - H);
    }
    gen_store(kn, 1 - H);
    split_b(1 - H, 1 - H, kn);
    lds_barrier();
    if constexpr (GEN) {
      if constexpr (ACT) gen_split_a();
      lds_barrier();
    }
  };
  // pairs of blocks with a branch-free body, then an odd last block
  auto run = [&](auto act) __attribute__((always_inline)) {
    int kb = 0;
    for (; kb + 1 < nkb; kb += 2) {
      step(act, std::integral_constant<int, 0>{}, kb);
      step(act, std::integral_constant<int, 1>{}, kb + 1);
    }
    if (kb < nkb) step(act, std::integral_constant<int, 0>{}, kb);
  };

  // reduced transform: a tile whose latitudes all lie below the first one
  // kept for this m writes zeros (uniform across the workgroup)
  if (jt * 128 + 128 > g.jstart[L.m_base + m]) {
    gload(0, 0);
    gload(nkb > 1 ? 1 : 0, 1);
    if constexpr (GEN) {
      gen_fetch(0, 0);
      gen_store(0, 0);
      gen_fetch(nkb > 1 ? 1 : 0, 1);
    } else {
      split_a(0);
    }
    split_b(0, 0, 0);
    __syncthreads();
    if constexpr (GEN) {
      if (active) gen_split_a();
      __syncthreads();
    }
    if (active)
      run(std::true_type{});
    else
      run(std::false_type{});
  }

  if (!active) return;
  const long long plane = L.wplane;
  float* ws = static_cast<float*>(g.ws) + L.ws_off + (2LL * m) * plane + p * L.spoff;
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
template <int NCB, bool GEN>
static hipError_t launch_bf16_ncb(bool analysis, const GemmArgs& g, hipStream_t st) {
  const dim3 grid(g.ntiles);
  if (analysis) {
    const size_t lds = X6Analysis<NCB>::lds_bytes(GEN);
    lds_optin<k_legendre_analysis_bf16<NCB, GEN>>(lds);
    hipLaunchKernelGGL((k_legendre_analysis_bf16<NCB, GEN>), grid, dim3(X6Analysis<NCB>::NT), lds, st, g);
  } else {
    const size_t lds = X6Synthesis<NCB>::lds_bytes(GEN);
    lds_optin<k_legendre_synthesis_bf16<NCB, GEN>>(lds);
    hipLaunchKernelGGL((k_legendre_synthesis_bf16<NCB, GEN>), grid, dim3(X6Synthesis<NCB>::NT), lds, st, g);
  }
  return hipGetLastError();
}

template <bool GEN>
static hipError_t launch_bf16_gen(bool analysis, const GemmArgs& g, int ncb, hipStream_t st) {
  switch (ncb) {
    case 1: return launch_bf16_ncb<1, GEN>(analysis, g, st);
    case 2: return launch_bf16_ncb<2, GEN>(analysis, g, st);
    case 4: return launch_bf16_ncb<4, GEN>(analysis, g, st);
    case 5: return launch_bf16_ncb<5, GEN>(analysis, g, st);
    case 8: return launch_bf16_ncb<8, GEN>(analysis, g, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_legendre_bf16(bool analysis, const GemmArgs& g, int ncb, bool gen, hipStream_t st) {
  return gen ? launch_bf16_gen<true>(analysis, g, ncb, st) : launch_bf16_gen<false>(analysis, g, ncb, st);
}

}  // namespace sht
