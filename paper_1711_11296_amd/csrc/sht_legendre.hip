// Meridional (Legendre) stage of the transform pair on the matrix cores.
//
// Analysis, Sec. 3.1 eq. cc-quad with the parity fold of App. B (eqs. B3,
// B4): for every zonal wavenumber m,
//     a_n^m = sum_{j < ceil(J/2)} P~_n^m(mu_j) * (S^m_j if n-m even, A^m_j if odd)
// where S and A already carry the quadrature weight.  With all fields side
// by side this is, per m and parity, a dense product
//     C[n][c] = P[n][j] * B_par[j][c],  c = 2*field + {re, im},
// which the kernels run on MFMA (v_mfma_f32_16x16x4_f32 for FP32 data,
// v_mfma_f64_16x16x4_f64 for FP64 data).
//
// Synthesis, Sec. 2 eq. iLT split by parity (App. B): per m,
//     S^m_j = sum_{n-m even} P~_n^m(mu_j) a_n^m,  A^m_j = sum_{n-m odd} ...
// i.e. the same table read transposed.
//
// Table layout: two copies per (level, m), each blocked in the order its
// kernel streams it (analysis: rows r = n - m padded to 128 by Kp columns j;
// synthesis: 128-latitude tiles by blocks of 32 natural rows; zero padding;
// see the kernels below).  The split-bfloat16 kernels read the same FP32
// copies.  Workspace layouts: see ws_col and ws_plane (the analysis reads
// rows of both parities interleaved in column blocks, the synthesis writes
// one plane per parity).
//
// Work decomposition: a host-built list gives one tile per workgroup; it is
// ordered so that the tiles of one m, which share the same right-hand
// operand, land on the same XCD (workgroups are dealt to the 8 XCDs round
// robin), and so that every XCD gets the same amount of work.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "sht_device.h"
#include "sht_internal.h"

namespace sht {

// ---------------------------------------------------------------------------
// analysis: C[n][c] = P[n][j] * B_par(n)[j][c]
// tile = 128 consecutive rows r = n - m (both parities) x BN = 16*NCB
// columns, 8 waves.  Wave w: parity p = w & 1, row quarter q = w >> 1; it
// owns the 16 rows r = 32 q + 2 i + p (one MFMA row block) and all NCB
// column blocks.
// The contraction runs over j in blocks of KB.  Lane (i, g) of a wave
// supplies the k values j = 4 kk + g (kk < KB/4) of its row.  The analysis
// copy of the table is blocked per (128-row tile, KB columns) and, inside a
// block, per wave and per 64-lane vector, so that each wave streams its
// operands with fully contiguous 1 KiB loads straight into registers.
// The right-hand operand (both parities of the workspace block) goes through
// LDS in two stages: block kb+1 is fetched into registers while the matrix
// cores work on block kb and stored into the other stage afterwards, so one
// barrier per block suffices.
// ---------------------------------------------------------------------------
template <typename T, int NCB, bool GEN = false>
struct AnalysisShape {
  static constexpr int E = 16 / (int)sizeof(T);        // scalars per 16 bytes
  // contraction block; generated P~ in FP64 also takes 32 latitudes (there
  // is no table layout to match, and a block's recurrence and two barriers
  // then serve twice the products)
  static constexpr int KB = (sizeof(T) == 4 || GEN) ? 32 : 16;
  static constexpr int KQ = KB / 4;                    // k values per lane and block
  static constexpr int BN = 16 * NCB;
  // With an even number of column blocks the right-hand operand goes from
  // memory to LDS directly (global_load_lds, 64 x 16 bytes per instruction,
  // contiguous in LDS), in rows 2 k + parity of BN elements (one
  // instruction fills both parities of one or more latitudes, contiguous in
  // the workspace) whose 16-column blocks are swapped in pairs for odd k
  // (column c sits at c ^ 16): the lane groups g = 0, 1 that one LDS cycle
  // serves read latitudes k of different parity and so hit different bank
  // halves.  Otherwise it is staged through registers into rows
  // parity KB + k padded to a pitch of 16 mod 32 words.
  static constexpr bool DMA = NCB % 2 == 0;
  static constexpr int BS = DMA ? BN : BN + (sizeof(T) == 4 ? 16 : 2);
  static constexpr int STAGE = 2 * KB * BS;            // elements of one stage
  static constexpr int BV = 2 * KB * BN / E;           // 16-byte vectors per block
  static constexpr int NB = (BV + 511) / 512;
  static constexpr int CS = BN + 1;                    // staging pitch of the output
  static constexpr int PS = 128 * KB;                  // generated P~ of one block (GEN)
  static constexpr size_t lds_bytes(bool gen) {
    const size_t main = (size_t)(2 * STAGE + (gen ? PS : 0)) * sizeof(T);
    const size_t cst = (size_t)64 * CS * sizeof(T);
    return main > cst ? main : cst;
  }
};

// Swizzle of the generated analysis block [128 rows][KB latitudes]: element
// (row, lat) sits at row * KB + (lat ^ gen_swz(row)), so that the 32
// latitudes one store instruction writes and the rows 2 i + p of one read
// instruction fall on distinct banks.
template <int KB>
__device__ __forceinline__ int gen_swz(int row) {
  return (2 * ((row >> 1) & 15)) & (KB - 1);
}

// GEN: the table operand is generated in the kernel (see gen_rows16): per K
// block, wave w produces the 16 rows of group w of the tile (lane l <
// KB at latitude l) into an LDS block, and after a barrier each wave reads
// its rows' values from it into the registers the table path fills from
// memory.
// The seed values of block kb + 2 are fetched while block kb is multiplied;
// the generated block is written after the products (its previous contents
// were read into registers before the last barrier), read after the next
// barrier, and a second barrier guards it against the next block's writes.
template <typename T, int NCB, bool GEN>
// (The FP64 generated kernel with 8 column blocks fills the LDS, one
// workgroup per compute unit: it takes the registers of two waves per SIMD.)
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && GEN && NCB > 4 ? 2 : 4))) void k_legendre_analysis(const GemmArgs g) {
  typedef typename Acc<T>::type AccT;
  typedef typename V16<T>::type V;
  using S = AnalysisShape<T, NCB, GEN>;
  constexpr int E = S::E, KB = S::KB, KQ = S::KQ, BN = S::BN, BS = S::BS;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Bs = reinterpret_cast<T*>(smem_raw);          // [2 stage][2 parity][KB][BS]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int r0 = t.rb * 128;
  const int c0 = t.cb * BN;
  const int Kp = L.Kp;
  const long long Cp = L.Cp;
  const long long plane = L.wplane;
  const T* wsm = static_cast<const T*>(g.ws) + L.ws_off + (2LL * m) * plane;  // region m

  const int tid = threadIdx.x;
  // wave-uniform values live in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int p = w & 1, q = w >> 1;
  const int li = lane & 15, lg = lane >> 4;
  const bool active = r0 + 32 * q + p < nm;
  // this wave's run of the blocked table (see the table layout above)
  const T* arow = GEN ? nullptr
                      : static_cast<const T*>(g.table) + g.tab_off[L.m_base + m] + (long long)t.rb * Kp * 128 +
                            w * 16 * KB + lane * E;
  T* Ps = Bs + 2 * S::STAGE;  // GEN: [128 rows][KB latitudes], swizzled (gen_swz)
  // GEN: wave w generates group w (rows 16 w .. 16 w + 15 of the tile), lane
  // l at latitude l % KB of each block (lanes l and l + KB compute and
  // store the same values, which keeps the code free of branches); the
  // group's recurrence coefficients are held in lanes for the whole tile
  const int ggrp = w, glat = lane & (KB - 1);
  const int gi = t.rb * 8 + ggrp;
  const bool gon = GEN && 16 * gi < nm;  // uniform across the wave
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
        gx1[set] = gseed[Kp + j];  // (a zero row when 16 gi + 1 = n_m: the seed rows are padded)
      }
    }
  };
  auto gen_store = [&](int set) __attribute__((always_inline)) {
    if constexpr (GEN) {
      gen_rows16<false>(gcA, gcB, 16 * gi, nm, gmu[set], gx0[set], gx1[set], [&](int s2, double x) {
        const int row = 16 * ggrp + s2;
        Ps[row * KB + (glat ^ gen_swz<KB>(row))] = (T)x;
      });
    }
  };
  T areg[KQ];
  auto gen_read = [&]() __attribute__((always_inline)) {
    const int rr = 32 * q + 2 * li + p;
#pragma unroll
    for (int kk = 0; kk < KQ; ++kk) areg[kk] = Ps[rr * KB + ((4 * kk + lg) ^ gen_swz<KB>(rr))];
  };

  AccT acc[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) acc[c] = AccT{0, 0, 0, 0};

  // The table operand is fetched two K blocks ahead into two register sets
  // used in turn (loop unrolled by two); the workspace operand one block
  // ahead (LDS stages).
  V an[2][KQ / E], ac[KQ / E];
  V rb[S::DMA ? 1 : S::NB];
  // (issued unconditionally, also by waves without rows in this tile and
  // for blocks past the end, clamped: with straight-line loads the wait
  // counts cover exactly the block that is consumed)
  auto gload_a = [&](int kb, V (&av)[KQ / E]) {
#pragma unroll
    for (int v = 0; v < KQ / E; ++v) av[v] = *reinterpret_cast<const V*>(arow + kb * 128 * KB + v * 64 * E);
  };
  auto gload_b = [&](int kb) {
    if constexpr (S::DMA) return;
#pragma unroll
    for (int i = 0; i < S::NB; ++i) {
      const int qq = tid + i * 512;
      if (S::NB * 512 == S::BV || qq < S::BV) {
        const int par = qq / (KB * BN / E);
        const int rem = qq - par * (KB * BN / E);
        const int row = rem / (BN / E), cv = rem % (BN / E);
        rb[i] = *reinterpret_cast<const V*>(wsm + (long long)(kb * KB + row) * 2 * Cp +
                                            ws_col(L.wsh, par, c0 + cv * E));
      }
    }
  };
  auto lstore = [&](int stage) {
    if constexpr (S::DMA) return;
    T* dst = Bs + stage * S::STAGE;
#pragma unroll
    for (int i = 0; i < S::NB; ++i) {
      const int qq = tid + i * 512;
      if (S::NB * 512 == S::BV || qq < S::BV) {
        const int par = qq / (KB * BN / E);
        const int rem = qq - par * (KB * BN / E);
        const int row = rem / (BN / E), cv = rem % (BN / E);
        *reinterpret_cast<V*>(dst + (par * KB + row) * BS + cv * E) = rb[i];
      }
    }
  };
  // memory -> LDS without registers: instruction i of wave w fills the
  // 1 KiB chunk number i*8 + w of the stage; lane l takes its 16-byte piece
  // (row 2 k + parity, physical column) and fetches the logical column under
  // the swizzle.  The lane's byte offsets within a K block are fixed for the
  // tile (32-bit, from the block's uniform base).
  unsigned dofs[S::DMA ? S::NB : 1];
  if constexpr (S::DMA) {
    static_assert(S::BV % 512 == 0, "whole chunks per wave");
#pragma unroll
    for (int i = 0; i < S::NB; ++i) {
      const int u = (i * 8 + w) * 64 + lane;
      const int rr = u / (BN / E), col = (u - rr * (BN / E)) * E;
      const int k = rr >> 1, par = rr & 1;
      dofs[i] = (unsigned)(k * 2 * (int)Cp + ws_col(L.wsh, par, c0 + (col ^ ((k & 1) << 4)))) * (unsigned)sizeof(T);
    }
  }
  auto dma = [&](int kb, int stage) {
    if constexpr (S::DMA) {
      T* dst = Bs + stage * S::STAGE;
      const char* src = reinterpret_cast<const char*>(wsm + (long long)kb * KB * 2 * Cp);
#pragma unroll
      for (int i = 0; i < S::NB; ++i) load_to_lds16(src + dofs[i], dst + (i * 8 + w) * 64 * E);
    }
  };
  // Wait for this wave's LDS fills: they were issued before the two table
  // loads of the block after next, which may stay in flight (vector memory
  // operations of a wave complete in issue order).
  auto wait_fills = [&]() {
    if constexpr (S::DMA) {
      static_assert(GEN || KQ / E == 2, "two table loads per block");
      if constexpr (GEN)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // nothing else is worth keeping in flight
      else
        asm volatile("s_waitcnt vmcnt(2)" ::: "memory");
    }
  };
  auto compute = [&](int stage) {
    T a[KQ];
    if constexpr (GEN) {
#pragma unroll
      for (int kk = 0; kk < KQ; ++kk) a[kk] = areg[kk];
    } else {
#pragma unroll
      for (int v = 0; v < KQ / E; ++v)
#pragma unroll
        for (int e = 0; e < E; ++e) a[v * E + e] = ac[v][e];
    }
    // LDS row of (parity p, latitude k): 2 k + p (DMA) or p KB + k
    constexpr int RK = S::DMA ? 2 : 1, RP = S::DMA ? 1 : KB;
    const T* Bp = Bs + stage * S::STAGE + (p * RP + lg * RK) * BS + li;
    // swizzled column-block offsets (latitudes g + 4 kk have the parity of g)
    const int sw = (S::DMA && (lg & 1)) ? 16 : 0;
#pragma unroll
    for (int kk = 0; kk < KQ; ++kk) {
      T bv[NCB];
#pragma unroll
      for (int c = 0; c < NCB; ++c) bv[c] = Bp[4 * kk * RK * BS + c * 16 + ((c & 1) ? -sw : sw)];
#pragma unroll
      for (int c = 0; c < NCB; ++c) acc[c] = mfma16(a[kk], bv[c], acc[c]);
    }
    // B reads run two k-steps ahead (paired reads of two columns)
    constexpr int RD = (NCB + 1) / 2;
    mfma_lds_pipeline<2 * RD, (KQ - 2) * RD, (NCB + RD - 1) / RD, 2 * NCB>();
  };
  const int nkb = Kp / KB;
  // one K block; H = kb & 1 selects the table registers of block kb (and of
  // kb + 2), 1 - H those of block kb + 1
  auto step = [&](auto hc, int kb) {
    constexpr int H = decltype(hc)::value;
    // after the last block the idle stage receives a clamped block that
    // nothing reads, which keeps the loop free of branches around memory
    // operations
    const int kn = kb + 1 < nkb ? kb + 1 : nkb - 1;
    gen_fetch(kb + 2 < nkb ? kb + 2 : nkb - 1, H);
    dma(kn, 1 - H);
    gload_b(kn);
    asm volatile("" ::: "memory");  // the table loads below are issued after the fills
    if constexpr (!GEN) gload_a(kb + 2 < nkb ? kb + 2 : nkb - 1, an[H]);
    if (active) compute(H);
    gen_store(1 - H);  // block kb + 1 (clamped after the last: nothing reads it)
    lstore(1 - H);
    wait_fills();
    if constexpr (!GEN) {
#pragma unroll
      for (int v = 0; v < KQ / E; ++v) ac[v] = an[1 - H][v];
    }
    lds_barrier();
    if constexpr (GEN) {
      gen_read();
      lds_barrier();
    }
  };

  // reduced transform: the blocks before kb0 hold only latitudes where
  // every |P~_n^m| < 1e-16 (kb0 = 0 otherwise)
  const int kb0 = min(g.jstart[L.m_base + m] / KB, nkb - 1);
  dma(kb0, 0);
  gload_b(kb0);
  asm volatile("" ::: "memory");
  if constexpr (GEN) {
    gen_fetch(kb0, 0);
    gen_store(0);
    gen_fetch(kb0 + 1 < nkb ? kb0 + 1 : nkb - 1, 1);
  } else {
    gload_a(kb0, an[0]);
    gload_a(kb0 + 1 < nkb ? kb0 + 1 : nkb - 1, an[1]);
  }
  lstore(0);
  wait_fills();
  if constexpr (!GEN) {
#pragma unroll
    for (int v = 0; v < KQ / E; ++v) ac[v] = an[0][v];
  }
  __syncthreads();
  if constexpr (GEN) {
    gen_read();
    __syncthreads();
  }
  for (int kb = kb0; kb < nkb; kb += 2) {
    step(std::integral_constant<int, 0>{}, kb);
    if (kb + 1 < nkb) step(std::integral_constant<int, 1>{}, kb + 1);
  }

  // stage 64 rows at a time in LDS, then write spec rows contiguously
  T* Cs = Bs;  // [64][CS]
  T* spec = static_cast<T*>(g.spec_out) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long base = spec_idx(N, m, m);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if ((q >> 1) == h) {
#pragma unroll
      for (int c = 0; c < NCB; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rl = 32 * (q & 1) + 2 * out_row<T>(lg, i) + p;
          Cs[rl * S::CS + c * 16 + li] = acc[c][i];
        }
    }
    __syncthreads();
    for (int qq = tid; qq < 64 * (BN / 2); qq += 512) {
      const int fl = qq >> 6, rl = qq & 63;
      const int f = (c0 >> 1) + fl;
      const int r = r0 + 64 * h + rl;
      if (r < nm && f < L.F) {
        T* d = spec + ((long long)f * nc + base + r) * 2;
        d[0] = Cs[rl * S::CS + 2 * fl];
        d[1] = Cs[rl * S::CS + 2 * fl + 1];
      }
    }
    if (h == 0) __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// synthesis: S_p[j][c] = sum_{r of parity p} P[r][j] * a[r][c]
// tile = 128 latitudes j x BN = 16*NCB columns, both parities, 8 waves.
// Wave w: parity p = w & 1, latitude quarter q = w >> 1; it owns the 32
// latitudes j = 32 q + 16 jb + i (jb < 2, two MFMA row blocks) and all NCB
// column blocks.  The contraction runs over r' (r = 2 r' + p) in blocks of
// KR per parity; lane (i, g) supplies r' = g KR/4 + kk (kk < KR/4).
// The table operand comes straight from memory into registers: the
// synthesis copy is blocked per (m, 128-latitude tile, K block), inside a
// block per wave and per 64-lane vector (vector v of lane (i, g) holds
// latitude block jb = v / (KQ/E) and r' = g KQ + E (v % (KQ/E)) + e).
// The spectral operand goes through LDS in two stages, transposed to
// [parity][column][r'] so that each lane reads its KR/4 values of a column
// as 16-byte vectors; one barrier per block.
// ---------------------------------------------------------------------------
template <typename T, int NCB>
struct SynthesisShape {
  static constexpr int E = 16 / (int)sizeof(T);
  static constexpr int KR = 16;                         // r' per parity and block
  static constexpr int KQ = KR / 4;                    // r' per lane and block
  static constexpr int BN = 16 * NCB;
  static constexpr int PITCH = KR + 16 / (int)sizeof(T);  // 16-byte pad: 4 mod 32 words
  static constexpr int STAGE = 2 * BN * PITCH;
  static constexpr int NV = 2 * KQ / E;                // table vectors per lane and block
  static constexpr int QUADS = (BN / 2) * (KR / 2);    // 4 natural rows of one field
  static constexpr int NQ = (QUADS + 511) / 512;
  static constexpr int CHUNK = 128 * 2 * KR;           // table elements per block
  static constexpr int GP = 130;                       // GEN: pitch of the generated block [2 KR rows][128 latitudes]
  static constexpr size_t lds_bytes(bool gen) { return (size_t)(2 * STAGE + (gen ? 2 * KR * GP : 0)) * sizeof(T); }
};

// GEN: the table operand is generated in the kernel (see gen_rows16): per K
// block of 2 KR natural rows (two 16-degree groups), waves 0..3 produce the
// 16 rows of one group for 64 latitudes of the tile each into an LDS block
// [row][latitude] (pitch 130: the reads of one instruction, 16 latitudes by
// 4 rows, fall on distinct banks); barriers as in the analysis.
template <typename T, int NCB, bool GEN>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) void k_legendre_synthesis(const GemmArgs g) {
  typedef typename Acc<T>::type AccT;
  typedef typename V16<T>::type V;
  using S = SynthesisShape<T, NCB>;
  constexpr int E = S::E, KR = S::KR, KQ = S::KQ, BN = S::BN, PITCH = S::PITCH;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Bs = reinterpret_cast<T*>(smem_raw);  // [2 stage][2 parity][BN][PITCH]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int nkb = (nm + 2 * KR - 1) / (2 * KR);
  const int jt = t.rb;
  const int c0 = t.cb * BN;
  const long long Cp = L.Cp;
  const T* spec = static_cast<const T*>(g.spec_in) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long sbase = spec_idx(N, m, m);

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int p = w & 1, q = w >> 1;
  const int li = lane & 15, lg = lane >> 4;
  const bool active = jt * 128 + 32 * q < L.Jh;
  const T* arun = GEN ? nullptr
                      : static_cast<const T*>(g.table) + g.tab_off[L.m_base + m] + (long long)jt * nkb * S::CHUNK +
                            w * (S::CHUNK / 8) + lane * E;
  T* Ps = Bs + 2 * S::STAGE;  // GEN: [2 KR rows][GP]
  // GEN: waves 0..3 generate; wave w takes group gsub = w >> 1 of each block
  // (rows 16 gsub .. + 15 of the block, uniform across the wave) at
  // latitude glat = 64 (w & 1) + lane of the tile; the group's recurrence
  // coefficients are fetched into lanes with its seed values
  const int gsub = w >> 1, glat = 64 * (w & 1) + lane;
  const int gj = jt * 128 + glat;
  const bool gthr = GEN && w < 4;  // uniform across the wave
  const bool gjin = gthr && gj < L.Kp;
  const double* gseeds = GEN ? g.seeds + g.seed_off[L.m_base + m] : nullptr;
  const double* grec = GEN ? g.rec + g.rec_off[L.m_base + m] : nullptr;
  const double gmu = (GEN && gjin) ? L.murow[gj] : 0.0;
  double gx0[2] = {0.0, 0.0}, gx1[2] = {0.0, 0.0}, gcA[2] = {0.0, 0.0}, gcB[2] = {0.0, 0.0};
  auto gen_fetch = [&](int kb, int set) __attribute__((always_inline)) {
    if constexpr (GEN) {
      const int gi = 2 * kb + gsub;
      if (gthr) gen_coef(grec, 16 * gi, nm, lane, gcA[set], gcB[set]);
      if (gjin && 16 * gi < nm) {
        gx0[set] = gseeds[2LL * gi * L.Kp + gj];
        gx1[set] = gseeds[(2LL * gi + 1) * L.Kp + gj];  // zero row when 16 gi + 1 = n_m
      }
    }
  };
  auto gen_store = [&](int kb, int set) __attribute__((always_inline)) {
    if constexpr (GEN) {
      if (gthr) {
        const int gi = 2 * kb + gsub;
        gen_rows16<false>(gcA[set], gcB[set], 16 * gi, gjin ? nm : 0, gmu, gx0[set], gx1[set],
                          [&](int s2, double x) { Ps[(16 * gsub + s2) * S::GP + glat] = (T)x; });
      }
    }
  };
  T areg[2][KQ];
  auto gen_read = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int kk = 0; kk < KQ; ++kk) areg[jb][kk] = Ps[(2 * (lg * KQ + kk) + p) * S::GP + 32 * q + 16 * jb + li];
  };

  AccT acc[2][NCB];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[jb][c] = AccT{0, 0, 0, 0};

  constexpr int QV = 8 / E;  // vectors per quad: 4 rows (re, im) of one field
  // Operands are fetched two K blocks ahead into two register sets used in
  // turn (the loop is unrolled by two so that the set is a compile-time
  // choice): block kb + 2 is requested while block kb is multiplied, and
  // block kb + 1, requested one block earlier, goes to LDS afterwards.
  V an[2][S::NV], ac[S::NV];
  V rq[2][S::NQ][QV];
  // The tile's spectra as a buffer starting at its first field and wave
  // number: reads past the end of the level's spectra return zero (fields
  // beyond F), rows beyond n = N are masked; offsets stay below 4 GiB (at
  // most 16 NCB fields of at most (N+1)(N+2)/2 rows).
  const long long sfirst = ((long long)(c0 >> 1) * nc + sbase) * 2;
  long long sbytes = ((long long)L.F * nc * 2 - sfirst) * (long long)sizeof(T);
  if (sbytes < 0) sbytes = 0;  // a tile past the last field (all its reads are zeros)
  const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<T*>(spec + sfirst), (short)0, (int)(unsigned)(sbytes > 0xFFFFFFFFLL ? 0xFFFFFFFFLL : sbytes),
      0x00020000);
  // Quad task qq: field fl, quad rp (natural rows 4 rp .. 4 rp + 3 of the
  // block).  In the FP32 form the lanes of a half-wave take 4 quads of 8
  // fields, so that the 8-byte stores of one instruction (column 2 fl + ri,
  // pitch 20 words) cover all 64 LDS banks once; otherwise quads vary
  // fastest.
  auto quad_of = [&](int qq, int& fl, int& rp) __attribute__((always_inline)) {
    if constexpr (sizeof(T) == 4 && KR / 2 == 8) {
      rp = (qq & 3) | (((qq >> 5) & 1) << 2);
      fl = ((qq >> 2) & 7) | ((qq >> 6) << 3);
    } else {
      fl = qq / (KR / 2);
      rp = qq % (KR / 2);
    }
  };
  // (issued unconditionally, also by waves without latitudes in this tile
  // and for blocks past the end, clamped: with straight-line loads the
  // compiler's wait counts cover exactly the block that is consumed)
  auto gload = [&](int kb, V (&av)[S::NV], V (&bq)[S::NQ][QV]) {
    if constexpr (!GEN) {
#pragma unroll
      for (int v = 0; v < S::NV; ++v)
        av[v] = *reinterpret_cast<const V*>(arun + (long long)kb * S::CHUNK + v * 64 * E);
    }
#pragma unroll
    for (int i = 0; i < S::NQ; ++i) {
      const int qq = tid + i * 512;
      int fl, rp;
      quad_of(qq, fl, rp);
      const int r = kb * 2 * KR + 4 * rp;  // first natural row of the quad
      const unsigned off = ((unsigned)fl * (unsigned)nc + (unsigned)r) * 2u * (unsigned)sizeof(T);
      // vector u holds natural rows r + u E/2 .. r + (u+1) E/2 - 1; rows
      // beyond n = N are masked when the quad is stored to LDS
#pragma unroll
      for (int u = 0; u < QV; ++u)
        bq[i][u] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(srs, (int)(off + 16u * u), 0, 0));
    }
  };
  auto lstore = [&](int stage, const V (&bq)[S::NQ][QV], int kb) {
    T* dst = Bs + stage * S::STAGE;
#pragma unroll
    for (int i = 0; i < S::NQ; ++i) {
      const int qq = tid + i * 512;
      if (S::NQ * 512 == S::QUADS || qq < S::QUADS) {
        int fl, rp;
        quad_of(qq, fl, rp);
        const int r = kb * 2 * KR + 4 * rp;
        T x[8];
#pragma unroll
        for (int u = 0; u < QV; ++u)
#pragma unroll
          for (int e = 0; e < E; ++e) x[u * E + e] = r + (u * E + e) / 2 < nm ? bq[i][u][e] : (T)0;
        // x = re, im of natural rows r, r+1, r+2, r+3: parity par, r' = 2 rp + h
#pragma unroll
        for (int par = 0; par < 2; ++par)
#pragma unroll
          for (int ri = 0; ri < 2; ++ri) {
            typedef T T2 __attribute__((ext_vector_type(2)));
            *reinterpret_cast<T2*>(dst + (par * BN + 2 * fl + ri) * PITCH + 2 * rp) =
                T2{x[2 * par + ri], x[4 + 2 * par + ri]};
          }
      }
    }
  };
  auto compute = [&](int stage) {
    T a[2][KQ];
    if constexpr (GEN) {
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int kk = 0; kk < KQ; ++kk) a[jb][kk] = areg[jb][kk];
    } else {
#pragma unroll
      for (int v = 0; v < S::NV; ++v)
#pragma unroll
        for (int e = 0; e < E; ++e) a[v / (KQ / E)][(v % (KQ / E)) * E + e] = ac[v][e];
    }
    const T* Bp = Bs + stage * S::STAGE + (p * BN + li) * PITCH + lg * KQ;
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      T bv[KQ];
#pragma unroll
      for (int v = 0; v < KQ / E; ++v) {
        const V x = *reinterpret_cast<const V*>(Bp + c * 16 * PITCH + v * E);
#pragma unroll
        for (int e = 0; e < E; ++e) bv[v * E + e] = x[e];
      }
#pragma unroll
      for (int kk = 0; kk < KQ; ++kk)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) acc[jb][c] = mfma16(a[jb][kk], bv[kk], acc[jb][c]);
    }
    // the reads of a column block are issued two column blocks ahead
    constexpr int RDC = KQ / E;
    mfma_lds_pipeline<2 * RDC, (NCB - 2) * RDC, (2 * KQ + RDC - 1) / RDC, 4 * KQ>();
  };
  // one K block; H = kb & 1 selects the register set of block kb (and of
  // kb + 2), 1 - H that of block kb + 1
  auto step = [&](auto hc, int kb) {
    constexpr int H = decltype(hc)::value;
    gen_fetch(kb + 2 < nkb ? kb + 2 : nkb - 1, H);
    gload(kb + 2 < nkb ? kb + 2 : nkb - 1, an[H], rq[H]);
    if (active) compute(H);
    // after the last block this fills the idle stage with a clamped block
    // (nothing reads it), which keeps the loop free of branches around
    // memory operations
    lstore(1 - H, rq[1 - H], kb + 1 < nkb ? kb + 1 : nkb - 1);
    gen_store(kb + 1 < nkb ? kb + 1 : nkb - 1, 1 - H);
    if constexpr (!GEN) {
#pragma unroll
      for (int v = 0; v < S::NV; ++v) ac[v] = an[1 - H][v];
    }
    lds_barrier();
    if constexpr (GEN) {
      gen_read();
      lds_barrier();
    }
  };

  // reduced transform: a tile whose latitudes all lie below the first one
  // kept for this m writes zeros (uniform across the workgroup)
  if (jt * 128 + 128 > g.jstart[L.m_base + m]) {
    gload(0, an[0], rq[0]);
    gload(nkb > 1 ? 1 : 0, an[1], rq[1]);
    lstore(0, rq[0], 0);
    if constexpr (GEN) {
      gen_fetch(0, 0);
      gen_store(0, 0);
      gen_fetch(nkb > 1 ? 1 : 0, 1);
    } else {
#pragma unroll
      for (int v = 0; v < S::NV; ++v) ac[v] = an[0][v];
    }
    __syncthreads();
    if constexpr (GEN) {
      gen_read();
      __syncthreads();
    }
    for (int kb = 0; kb < nkb; kb += 2) {
      step(std::integral_constant<int, 0>{}, kb);
      if (kb + 1 < nkb) step(std::integral_constant<int, 1>{}, kb + 1);
    }
  }

  if (!active) return;
  const long long plane = L.wplane;
  T* ws = static_cast<T*>(g.ws) + L.ws_off + (2LL * m) * plane + p * L.spoff;
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = jt * 128 + 32 * q + 16 * jb + out_row<T>(lg, i);
      if (j < L.Jh) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) ws[(long long)j * Cp + c0 + c * 16 + li] = acc[jb][c][i];
      }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
static size_t lds_analysis(int ncb, bool gen) {
  switch (ncb) {
    case 1: return gen ? AnalysisShape<T, 1, true>::lds_bytes(true) : AnalysisShape<T, 1>::lds_bytes(false);
    case 2: return gen ? AnalysisShape<T, 2, true>::lds_bytes(true) : AnalysisShape<T, 2>::lds_bytes(false);
    case 4: return gen ? AnalysisShape<T, 4, true>::lds_bytes(true) : AnalysisShape<T, 4>::lds_bytes(false);
    case 5: return gen ? AnalysisShape<T, 5, true>::lds_bytes(true) : AnalysisShape<T, 5>::lds_bytes(false);
    case 8: return gen ? AnalysisShape<T, 8, true>::lds_bytes(true) : AnalysisShape<T, 8>::lds_bytes(false);
    default: return gen ? AnalysisShape<T, 10, true>::lds_bytes(true) : AnalysisShape<T, 10>::lds_bytes(false);
  }
}

template <typename T>
static size_t lds_synthesis(int ncb, bool gen) {
  switch (ncb) {
    case 1: return SynthesisShape<T, 1>::lds_bytes(gen);
    case 2: return SynthesisShape<T, 2>::lds_bytes(gen);
    case 4: return SynthesisShape<T, 4>::lds_bytes(gen);
    case 5: return SynthesisShape<T, 5>::lds_bytes(gen);
    case 8: return SynthesisShape<T, 8>::lds_bytes(gen);
    default: return SynthesisShape<T, 8>::lds_bytes(gen);
  }
}

constexpr int kMaxSynthesisNcb = 8;

template <typename T, int NCB, bool GEN>
static hipError_t launch_ncb(bool analysis, const GemmArgs& g, hipStream_t st) {
  const dim3 grid(g.ntiles), block(512);
  if constexpr (sizeof(T) == 8 && NCB > 8) return hipErrorInvalidValue;  // FP64 takes at most 8
  else if (analysis) {
    const size_t lds = lds_analysis<T>(NCB, GEN);
    lds_optin<k_legendre_analysis<T, NCB, GEN>>(lds);
    hipLaunchKernelGGL((k_legendre_analysis<T, NCB, GEN>), grid, block, lds, st, g);
  } else {
    // wider synthesis tiles do not fit the register file
    if constexpr (NCB > kMaxSynthesisNcb) return hipErrorInvalidValue;
    else {
      const size_t lds = lds_synthesis<T>(NCB, GEN);
      lds_optin<k_legendre_synthesis<T, NCB, GEN>>(lds);
      hipLaunchKernelGGL((k_legendre_synthesis<T, NCB, GEN>), grid, block, lds, st, g);
    }
  }
  return hipGetLastError();
}

template <typename T, bool GEN>
static hipError_t launch_legendre_t(bool analysis, const GemmArgs& g, int ncb, hipStream_t st) {
  switch (ncb) {
    case 1: return launch_ncb<T, 1, GEN>(analysis, g, st);
    case 2: return launch_ncb<T, 2, GEN>(analysis, g, st);
    case 4: return launch_ncb<T, 4, GEN>(analysis, g, st);
    case 5: return launch_ncb<T, 5, GEN>(analysis, g, st);
    case 8: return launch_ncb<T, 8, GEN>(analysis, g, st);
    case 10: return launch_ncb<T, 10, GEN>(analysis, g, st);
    default: return hipErrorInvalidValue;
  }
}

int max_ncb(int form, bool analysis) {
  if (form == SHT_FORM_BF16X6) return 8;  // wider split-form tiles do not fit the register file
  if (form == SHT_FORM_FP64) return 8;
  return analysis ? 10 : kMaxSynthesisNcb;
}

int launch_legendre(int form, bool analysis, const GemmArgs& g, int ncb, bool gen, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (g.ntiles <= 0) return (int)hipSuccess;
  if (form == SHT_FORM_BF16X6) return (int)launch_legendre_bf16(analysis, g, ncb, gen, st);
  if (form == SHT_FORM_FP64)
    return (int)(gen ? launch_legendre_t<double, true>(analysis, g, ncb, st)
                     : launch_legendre_t<double, false>(analysis, g, ncb, st));
  return (int)(gen ? launch_legendre_t<float, true>(analysis, g, ncb, st)
                   : launch_legendre_t<float, false>(analysis, g, ncb, st));
}

}  // namespace sht
