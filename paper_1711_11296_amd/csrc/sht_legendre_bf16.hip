// Legendre stage in the split-bfloat16 form (see sht_legendre.hip for the
// transform and the data layouts): operands carried as three bfloat16
// pieces, six piece products per term on the bfloat16 matrix cores, FP32
// accumulation.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "sht_device.h"
#include "sht_internal.h"

namespace sht {

// ---------------------------------------------------------------------------
// Split-bfloat16 form: every operand x is carried as three bfloat16 pieces
// x = x0 + x1 + x2 (8 significant bits each).  The product of two operands
// is accumulated in FP32 from the six piece products whose piece indices sum
// to at most 2 (x0 y0, x0 y1, x1 y0, x0 y2, x1 y1, x2 y0), smallest first;
// the three dropped products are below 2^-24 relative.  Table pieces are
// split from FP64 on the host; the right-hand operand (FP32) is split in the
// kernel by truncation, which is exact: x - x0 and (x - x0) - x1 are
// representable, and the remainder has at most 8 significant bits.
// MFMA: v_mfma_f32_16x16x32_bf16 (lane l supplies 8 consecutive k values
// 8*(l/16) + e of row/column l%16; result layout as for the FP32 16x16x4).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Split 8 floats into three bfloat16x8 pieces (exact, by truncation).
__device__ __forceinline__ void split3x8(const float (&x)[8], bf16x8& h, bf16x8& m, bf16x8& l) {
  unsigned uh[8], um[8], ul[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const unsigned u = __float_as_uint(x[e]);
    const float fh = __uint_as_float(u & 0xFFFF0000u);
    const float r = x[e] - fh;
    const unsigned ur = __float_as_uint(r);
    const float fm = __uint_as_float(ur & 0xFFFF0000u);
    const float r2 = r - fm;
    uh[e] = u;
    um[e] = ur;
    ul[e] = __float_as_uint(r2);
  }
  u32x4 ph, pm, pl;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ph[q] = (uh[2 * q] >> 16) | (uh[2 * q + 1] & 0xFFFF0000u);
    pm[q] = (um[2 * q] >> 16) | (um[2 * q + 1] & 0xFFFF0000u);
    pl[q] = (ul[2 * q] >> 16) | (ul[2 * q + 1] & 0xFFFF0000u);
  }
  h = __builtin_bit_cast(bf16x8, ph);
  m = __builtin_bit_cast(bf16x8, pm);
  l = __builtin_bit_cast(bf16x8, pl);
}

// acc += a * b with a = (a0, a1, a2) and b = (b0, b1, b2) split operands
__device__ __forceinline__ f32x4 mfma6(const bf16x8 (&a)[3], bf16x8 b0, bf16x8 b1, bf16x8 b2,
                                       f32x4 acc) {
  acc = mfma_bf16(a[2], b0, acc);
  acc = mfma_bf16(a[1], b1, acc);
  acc = mfma_bf16(a[0], b2, acc);
  acc = mfma_bf16(a[1], b0, acc);
  acc = mfma_bf16(a[0], b1, acc);
  acc = mfma_bf16(a[0], b0, acc);
  return acc;
}

// Analysis in the split form.  Same tiling as the FP32 kernel (64 rows x
// 16*NCB columns, waves (parity, column half)); the contraction advances 32
// latitudes per block, one 16x16x32 step per piece product.
template <int NCB>
__global__ __launch_bounds__(256) void k_legendre_analysis_bf16(const GemmArgs g) {
  typedef typename V16<float>::type V;
  constexpr int KB = 32;
  constexpr int BN = 16 * NCB;
  constexpr int HC = (NCB + 1) / 2;
  constexpr int AS = 40;                   // bf16 per LDS row of A (5 x 16 bytes)
  constexpr int BS = BN + 2;               // conflict-free B reads
  constexpr int NA = 3 * 64 * KB / 8 / 256;
  constexpr int NB = 2 * KB * BN / 4 / 256;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned short* As = reinterpret_cast<unsigned short*>(smem_raw);   // [3][2][32][AS]
  float* Bs = reinterpret_cast<float*>(smem_raw + 3 * 64 * AS * 2);   // [2][KB][BS]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int r0 = t.rb * 64;
  const int c0 = t.cb * BN;
  const int Kp = L.Kp;
  const long long Cp = L.Cp;
  const unsigned short* tab = static_cast<const unsigned short*>(g.table) + g.tab_off[L.m_base + m] +
                              (long long)r0 * Kp;
  const long long plane = (long long)Kp * Cp;
  const float* wsm = static_cast<const float*>(g.ws) + L.ws_off + (2LL * m) * plane + c0;

  const int tid = threadIdx.x;
  // wave-uniform values live in scalar registers, so the per-wave choices
  // below are scalar branches around whole K-blocks
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int p = w & 1, ch = w >> 1;
  const int li = lane & 15, lg = lane >> 4;
  const int nrb = (r0 + 32 + p) < nm ? 2 : ((r0 + p) < nm ? 1 : 0);  // active row blocks
  const bool full_cols = ch == 0;  // HC column blocks, else NCB - HC

  f32x4 acc[2][HC];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < HC; ++c) acc[a][c] = f32x4{0, 0, 0, 0};

  u32x4 ra[NA];
  V rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + i * 256;
      const int pc = q / 256, rem = q % 256;
      const int row = rem / 4, cv = rem % 4;
      ra[i] = *reinterpret_cast<const u32x4*>(tab + pc * g.table_plane + (long long)row * Kp + k0 + cv * 8);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + i * 256;
      const int par = q / (KB * BN / 4);
      const int rem = q - par * (KB * BN / 4);
      const int row = rem / (BN / 4), cv = rem % (BN / 4);
      rb[i] = *reinterpret_cast<const V*>(wsm + par * plane + (long long)(k0 + row) * Cp + cv * 4);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + i * 256;
      const int pc = q / 256, rem = q % 256;
      const int row = rem / 4, cv = rem % 4;
      *reinterpret_cast<u32x4*>(As + ((pc * 2 + (row & 1)) * 32 + (row >> 1)) * AS + cv * 8) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + i * 256;
      const int par = q / (KB * BN / 4);
      const int rem = q - par * (KB * BN / 4);
      const int row = rem / (BN / 4), cv = rem % (BN / 4);
      lds_store8<float>(Bs + (par * KB + row) * BS + cv * 4, rb[i]);
    }
  };

  const int nkb = Kp / KB;
  auto kloop = [&](auto nrc, auto ncc) {
    constexpr int NR = decltype(nrc)::value, NC = decltype(ncc)::value;
    gload(0);
    lstore();
    __syncthreads();
    for (int kb = 0; kb < nkb; ++kb) {
      if (kb + 1 < nkb) gload((kb + 1) * KB);
      if constexpr (NR > 0 && NC > 0) {
        bf16x8 av[NR][3];
#pragma unroll
        for (int rb2 = 0; rb2 < NR; ++rb2)
#pragma unroll
          for (int pc = 0; pc < 3; ++pc)
            av[rb2][pc] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const u32x4*>(As + ((pc * 2 + p) * 32 + 16 * rb2 + li) * AS + 8 * lg));
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int cb = ch * HC + c;
          float bv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) bv[e] = Bs[(p * KB + 8 * lg + e) * BS + cb * 16 + li];
          bf16x8 b0, b1, b2;
          split3x8(bv, b0, b1, b2);
#pragma unroll
          for (int r = 0; r < NR; ++r) acc[r][c] = mfma6(av[r], b0, b1, b2, acc[r][c]);
        }
      }
      __syncthreads();
      if (kb + 1 < nkb) {
        lstore();
        __syncthreads();
      }
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using CH = std::integral_constant<int, HC>;
  using CL = std::integral_constant<int, NCB - HC>;
  if (nrb == 0) {
    kloop(I0{}, CH{});
  } else if (full_cols || 2 * HC == NCB) {
    if (nrb == 2)
      kloop(I2{}, CH{});
    else
      kloop(I1{}, CH{});
  } else {
    if (nrb == 2)
      kloop(I2{}, CL{});
    else
      kloop(I1{}, CL{});
  }

  constexpr int CS = BN + 1;
  float* Cs = reinterpret_cast<float*>(smem_raw);  // [64][CS]
#pragma unroll
  for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
    for (int c = 0; c < HC; ++c) {
      const int cb = ch * HC + c;
      if (cb < NCB) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rl = 2 * (16 * rb2 + 4 * lg + i) + p;
          Cs[rl * CS + cb * 16 + li] = acc[rb2][c][i];
        }
      }
    }
  __syncthreads();
  float* spec = static_cast<float*>(g.spec_out) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long base = spec_idx(N, m, m) + r0;
  for (int q = tid; q < 64 * (BN / 2); q += 256) {
    const int fl = q >> 6, rl = q & 63;
    const int f = (c0 >> 1) + fl;
    if (r0 + rl < nm && f < L.F) {
      float* d = spec + ((long long)f * nc + base + rl) * 2;
      d[0] = Cs[rl * CS + 2 * fl];
      d[1] = Cs[rl * CS + 2 * fl + 1];
    }
  }
}

// Synthesis in the split form: tile 64 j x 16*NCB columns, contraction over
// natural rows in blocks of 64 (32 per parity, one 16x16x32 step).  The
// table comes from its split synthesis copy, blocked per (m, 64-row j block,
// 64-row r block) as [piece plane][parity][64 j][32 r'].
template <int NCB>
__global__ __launch_bounds__(256) void k_legendre_synthesis_bf16(const GemmArgs g) {
  constexpr int BN = 16 * NCB;
  constexpr int HC = (NCB + 1) / 2;
  constexpr int KH = 32;                  // table rows per parity and block
  constexpr int AS = 40;                  // bf16 per LDS row (5 x 16 bytes)
  constexpr int BS = BN + 2;
  constexpr int NA = 3 * 2 * 64 * KH / 8 / 256;
  constexpr int NB = (BN / 2) * KH / 256 > 0 ? (BN / 2) * KH / 256 : 1;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned short* At = reinterpret_cast<unsigned short*>(smem_raw);    // [3][2][64][AS]
  float* Bs = reinterpret_cast<float*>(smem_raw + 3 * 2 * 64 * AS * 2);  // [2][KH][BS]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int nkb = (nm + 63) / 64;
  const int jb = t.rb;
  const int c0 = t.cb * BN;
  const long long Cp = L.Cp;
  const unsigned short* tab = static_cast<const unsigned short*>(g.table) + g.tab_off[L.m_base + m] +
                              (long long)jb * nkb * 4096;
  const float* spec = static_cast<const float*>(g.spec_in) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long sbase = spec_idx(N, m, m);

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int p = w & 1, ch = w >> 1;
  const int li = lane & 15, lg = lane >> 4;
  const bool full_cols = ch == 0;  // HC column blocks, else NCB - HC

  f32x4 acc[4][HC];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < HC; ++c) acc[a][c] = f32x4{0, 0, 0, 0};

  u32x4 ra[NA];
  float rs[NB][4];
  auto gload = [&](int kb) {
    const unsigned short* blk = tab + (long long)kb * 4096;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + i * 256;
      const int pc = q / 512, rem = q % 512;
      ra[i] = *reinterpret_cast<const u32x4*>(blk + pc * g.table_plane + rem * 8);
    }
    const int rb0 = kb * 64;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + i * 256;
      const int fl = q / KH, rp = q % KH;
      const int f = (c0 >> 1) + fl;
      const int r = rb0 + 2 * rp;
      rs[i][0] = rs[i][1] = rs[i][2] = rs[i][3] = 0.f;
      if (fl < BN / 2 && f < L.F) {
        const float* sp = spec + ((long long)f * nc + sbase + r) * 2;
        if (r < nm) {
          rs[i][0] = sp[0];
          rs[i][1] = sp[1];
        }
        if (r + 1 < nm) {
          rs[i][2] = sp[2];
          rs[i][3] = sp[3];
        }
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + i * 256;
      const int pc = q / 512, rem = q % 512;
      const int e0 = rem * 8;
      const int pj = e0 / KH, kv = e0 % KH;   // (parity*64 + j), r'
      *reinterpret_cast<u32x4*>(At + (pc * 128 + pj) * AS + kv) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + i * 256;
      const int fl = q / KH, rp = q % KH;
      if (fl < BN / 2) {
        float* d0 = Bs + rp * BS + 2 * fl;
        float* d1 = Bs + (KH + rp) * BS + 2 * fl;
        d0[0] = rs[i][0];
        d0[1] = rs[i][1];
        d1[0] = rs[i][2];
        d1[1] = rs[i][3];
      }
    }
  };

  auto kloop = [&](auto ncc) {
    constexpr int NC = decltype(ncc)::value;
    gload(0);
    lstore();
    __syncthreads();
    for (int kb = 0; kb < nkb; ++kb) {
      if (kb + 1 < nkb) gload(kb + 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int cb = ch * HC + c;
        float bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = Bs[(p * KH + 8 * lg + e) * BS + cb * 16 + li];
        bf16x8 b0, b1, b2;
        split3x8(bv, b0, b1, b2);
#pragma unroll
        for (int jr = 0; jr < 4; ++jr) {
          bf16x8 av[3];
#pragma unroll
          for (int pc = 0; pc < 3; ++pc)
            av[pc] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const u32x4*>(At + (pc * 128 + p * 64 + 16 * jr + li) * AS + 8 * lg));
          acc[jr][c] = mfma6(av, b0, b1, b2, acc[jr][c]);
        }
      }
      __syncthreads();
      if (kb + 1 < nkb) {
        lstore();
        __syncthreads();
      }
    }
  };
  if (full_cols || 2 * HC == NCB)
    kloop(std::integral_constant<int, HC>{});
  else
    kloop(std::integral_constant<int, NCB - HC>{});

  const long long plane = (long long)L.Kp * Cp;
  float* ws = static_cast<float*>(g.ws) + L.ws_off + (2LL * m + p) * plane;
#pragma unroll
  for (int jr = 0; jr < 4; ++jr)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = jb * 64 + 16 * jr + 4 * lg + i;
      if (j < L.Jh) {
#pragma unroll
        for (int c = 0; c < HC; ++c) {
          const int cb = ch * HC + c;
          if (cb < NCB) ws[(long long)j * Cp + c0 + cb * 16 + li] = acc[jr][c][i];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static size_t lds_analysis_bf16(int ncb) {
  const int BN = 16 * ncb;
  size_t stage = (size_t)3 * 64 * 40 * 2 + (size_t)2 * 32 * (BN + 2) * 4;
  size_t cst = (size_t)64 * (BN + 1) * 4;
  return stage > cst ? stage : cst;
}

static size_t lds_synthesis_bf16(int ncb) {
  const int BN = 16 * ncb;
  return (size_t)3 * 2 * 64 * 40 * 2 + (size_t)2 * 32 * (BN + 2) * 4;
}

hipError_t launch_legendre_bf16(bool analysis, const GemmArgs& g, int ncb, hipStream_t st) {
  const dim3 grid(g.ntiles), block(256);
#define SHT_BLAUNCH(NCB_)                                                        \
  case NCB_:                                                                    \
    if (analysis) {                                                             \
      lds_optin<k_legendre_analysis_bf16<NCB_>>(lds_analysis_bf16(NCB_));      \
      hipLaunchKernelGGL((k_legendre_analysis_bf16<NCB_>), grid, block,        \
                         lds_analysis_bf16(NCB_), st, g);                       \
    } else {                                                                    \
      lds_optin<k_legendre_synthesis_bf16<NCB_>>(lds_synthesis_bf16(NCB_));    \
      hipLaunchKernelGGL((k_legendre_synthesis_bf16<NCB_>), grid, block,       \
                         lds_synthesis_bf16(NCB_), st, g);                      \
    }                                                                           \
    break;
  switch (ncb) {
    SHT_BLAUNCH(1)
    SHT_BLAUNCH(2)
    SHT_BLAUNCH(4)
    SHT_BLAUNCH(5)
    SHT_BLAUNCH(8)
    SHT_BLAUNCH(10)
    default:
      return hipErrorInvalidValue;
  }
#undef SHT_BLAUNCH
  return hipGetLastError();
}

}  // namespace sht
