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
// Table layout: per (level, m) a block of R_m = roundup(N-m+1, 64) rows
// (row r = n - m, zero padding) by Kp columns (j, zero padding), row-major.
// Workspace layout: ws[m][parity][j][c] (see the zonal stage).
//
// Work decomposition: a host-built list gives one tile per workgroup; it is
// ordered so that the tiles of one m, which share the same right-hand
// operand, land on the same XCD (workgroups are dealt to the 8 XCDs round
// robin), and so that every XCD gets the same amount of work.

#include <hip/hip_runtime.h>

#include "sht_internal.h"

namespace sht {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<float> {
  typedef f32x4 type;
};
template <>
struct Acc<double> {
  typedef f64x4 type;
};

// 16x16x4 outer-product step: lane l supplies A[l%16][k] and B[k][l%16]
// for k = l/16 (any k labelling works as long as A and B agree).  Element i
// of lane l's result is C[out_row(l/16, i)][l%16]: rows 4*(l/16) + i for
// the FP32 instruction, (l/16) + 4*i for the FP64 one (measured lane layout).
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ int out_row(int lg, int i) {
  return sizeof(T) == 8 ? lg + 4 * i : 4 * lg + i;
}

__device__ __forceinline__ long long spec_idx(int N, int m, int n) {
  return (long long)m * (2 * N + 3 - m) / 2 + (n - m);
}

template <typename T>
struct V16;
template <>
struct V16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct V16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

// ---------------------------------------------------------------------------
// analysis: C[n][c] = P[n][j] * B_par(n)[j][c]
// tile = 64 consecutive rows n - m (both parities) x BN = 16*NCB columns.
// wave w: parity p = w & 1, half h = w >> 1; its 16 rows are
//   r = 32 h + 2 i + p, i = 0..15 (local to the tile).
// ---------------------------------------------------------------------------
template <typename T, int NCB>
__global__ __launch_bounds__(256) void k_legendre_analysis(const GemmArgs g) {
  typedef typename Acc<T>::type AccT;
  typedef typename V16<T>::type V;
  constexpr int E = 16 / (int)sizeof(T);           // scalars per 16 bytes
  constexpr int KB = sizeof(T) == 4 ? 32 : 16;    // contraction block
  constexpr int KQ = KB / 4;                       // k-steps per block
  constexpr int BN = 16 * NCB;
  constexpr int AS = KB + E;                       // LDS row stride of A
  constexpr int BS = BN + E;                       // LDS row stride of B

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);          // [64][AS]
  T* Bs = As + 64 * AS;                            // [2][KB][BS]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int r0 = t.rb * 64;
  const int c0 = t.cb * BN;
  const int Kp = L.Kp;
  const long long Cp = L.Cp;
  const T* tab = static_cast<const T*>(g.table) + g.tab_off[L.m_base + m] + (long long)r0 * Kp;
  const T* wsm = static_cast<const T*>(g.ws) + L.ws_off + (2LL * m) * Kp * Cp;
  const long long plane = (long long)Kp * Cp;

  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int p = w & 1, h = w >> 1;
  const int li = lane & 15, lg = lane >> 4;
  const int arow = 32 * h + 2 * li + p;            // this lane's A row
  const bool active = (r0 + 32 * h + p) < nm;

  AccT acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = AccT{0, 0, 0, 0};

  for (int k0 = 0; k0 < Kp; k0 += KB) {
    // A block: 64 rows x KB
    for (int q = tid; q < 64 * KB / E; q += 256) {
      const int row = q / (KB / E), cv = q % (KB / E);
      const V v = *reinterpret_cast<const V*>(tab + (long long)row * Kp + k0 + cv * E);
      *reinterpret_cast<V*>(As + row * AS + cv * E) = v;
    }
    // B blocks: 2 parities x KB rows x BN columns
    for (int q = tid; q < 2 * KB * BN / E; q += 256) {
      const int par = q / (KB * BN / E);
      const int rem = q - par * (KB * BN / E);
      const int row = rem / (BN / E), cv = rem % (BN / E);
      const V v = *reinterpret_cast<const V*>(wsm + par * plane + (long long)(k0 + row) * Cp + c0 + cv * E);
      *reinterpret_cast<V*>(Bs + (par * KB + row) * BS + cv * E) = v;
    }
    __syncthreads();
    if (active) {
      const T* Ap = As + arow * AS + lg * KQ;       // k = lg*KQ + kk
      const T* Bp = Bs + (p * KB + lg * KQ) * BS + li;
#pragma unroll
      for (int kk = 0; kk < KQ; ++kk) {
        const T a = Ap[kk];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma16(a, Bp[kk * BS + cb * 16], acc[cb]);
      }
    }
    __syncthreads();
  }

  // stage the 64 x BN tile in LDS, then write spec rows contiguously
  T* Cs = As;  // [64][BN]
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rl = 32 * h + 2 * out_row<T>(lg, i) + p;
      Cs[rl * BN + cb * 16 + li] = acc[cb][i];
    }
  __syncthreads();
  T* spec = static_cast<T*>(g.spec_out) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long base = spec_idx(N, m, m) + r0;
  for (int q = tid; q < 64 * (BN / 2); q += 256) {
    const int fl = q >> 6, rl = q & 63;
    const int f = (c0 >> 1) + fl;
    if (r0 + rl < nm && f < L.F) {
      T* d = spec + ((long long)f * nc + base + rl) * 2;
      d[0] = Cs[rl * BN + 2 * fl];
      d[1] = Cs[rl * BN + 2 * fl + 1];
    }
  }
}

// ---------------------------------------------------------------------------
// synthesis: S_p[j][c] = sum_{r of parity p} P[r][j] * a[r][c]
// tile = 32 rows j x BN columns, both parities.
// wave w: output parity p = w & 1, rows j = 32 jb + 16 h + (0..15), h = w >> 1.
// contraction over natural rows r = n - m in blocks of 32 (16 per parity).
// ---------------------------------------------------------------------------
template <typename T, int NCB>
__global__ __launch_bounds__(256) void k_legendre_synthesis(const GemmArgs g) {
  typedef typename Acc<T>::type AccT;
  typedef typename V16<T>::type V;
  constexpr int E = 16 / (int)sizeof(T);
  constexpr int BN = 16 * NCB;
  constexpr int KR = 32;            // natural rows per block
  constexpr int KH = KR / 2;        // rows per parity
  constexpr int AS = KH + E;        // LDS stride of the transposed table
  constexpr int BS = BN + E;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* At = reinterpret_cast<T*>(smem_raw);     // [2][32 j][AS]
  T* Bs = At + 2 * 32 * AS;                   // [2][KH][BS]

  const Tile t = g.tiles[blockIdx.x];
  if (t.level < 0) return;
  const LevelDesc& L = g.lev[t.level];
  const int N = L.N, m = t.m;
  const int nm = N - m + 1;
  const int j0 = t.rb * 32;
  const int c0 = t.cb * BN;
  const int Kp = L.Kp;
  const long long Cp = L.Cp;
  const T* tab = static_cast<const T*>(g.table) + g.tab_off[L.m_base + m];
  const T* spec = static_cast<const T*>(g.spec_in) + L.spec_off;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long sbase = spec_idx(N, m, m);

  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int p = w & 1, h = w >> 1;
  const int li = lane & 15, lg = lane >> 4;

  AccT acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = AccT{0, 0, 0, 0};

  for (int rb0 = 0; rb0 < nm; rb0 += KR) {
    // table block rows rb0..rb0+31 (padded rows are zero), columns j0..j0+31,
    // stored transposed and split by parity: At[r&1][j][r>>1]
    for (int q = tid; q < KR * 32 / E; q += 256) {
      const int r = q / (32 / E), jv = q % (32 / E);
      const V v = *reinterpret_cast<const V*>(tab + (long long)(rb0 + r) * Kp + j0 + jv * E);
#pragma unroll
      for (int e = 0; e < E; ++e) At[((r & 1) * 32 + jv * E + e) * AS + (r >> 1)] = v[e];
    }
    // spectra rows rb0..rb0+31, columns c0..c0+BN: pairs (re, im) of field f
    for (int q = tid; q < KR * (BN / 2); q += 256) {
      const int fl = q / KR, r = q % KR;
      const int f = (c0 >> 1) + fl;
      T re = (T)0, im = (T)0;
      if (rb0 + r < nm && f < L.F) {
        const T* s = spec + ((long long)f * nc + sbase + rb0 + r) * 2;
        re = s[0];
        im = s[1];
      }
      T* d = Bs + ((r & 1) * KH + (r >> 1)) * BS + 2 * fl;
      d[0] = re;
      d[1] = im;
    }
    __syncthreads();
    {
      const T* Ap = At + (p * 32 + 16 * h + li) * AS + lg * 4;   // k = lg*4 + kk
      const T* Bp = Bs + (p * KH + lg * 4) * BS + li;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const T a = Ap[kk];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma16(a, Bp[kk * BS + cb * 16], acc[cb]);
      }
    }
    __syncthreads();
  }

  T* ws = static_cast<T*>(g.ws) + L.ws_off + (2LL * m + p) * Kp * Cp;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = j0 + 16 * h + out_row<T>(lg, i);
    if (j < L.Jh) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) ws[(long long)j * Cp + c0 + cb * 16 + li] = acc[cb][i];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
static size_t lds_analysis(int ncb) {
  const int E = 16 / (int)sizeof(T);
  const int KB = sizeof(T) == 4 ? 32 : 16;
  const int BN = 16 * ncb;
  size_t stage = (size_t)(64 * (KB + E) + 2 * KB * (BN + E)) * sizeof(T);
  size_t cst = (size_t)64 * BN * sizeof(T);
  return stage > cst ? stage : cst;
}

template <typename T>
static size_t lds_synthesis(int ncb) {
  const int E = 16 / (int)sizeof(T);
  const int BN = 16 * ncb;
  return (size_t)(2 * 32 * (16 + E) + 2 * 16 * (BN + E)) * sizeof(T);
}

template <typename T>
static hipError_t launch_legendre_t(bool analysis, const GemmArgs& g, int ncb,
                                    hipStream_t st) {
  const dim3 grid(g.ntiles), block(256);
#define SHT_LLAUNCH(NCB_)                                                        \
  case NCB_:                                                                    \
    if (analysis)                                                               \
      hipLaunchKernelGGL((k_legendre_analysis<T, NCB_>), grid, block,          \
                         lds_analysis<T>(NCB_), st, g);                         \
    else                                                                        \
      hipLaunchKernelGGL((k_legendre_synthesis<T, NCB_>), grid, block,         \
                         lds_synthesis<T>(NCB_), st, g);                        \
    break;
  switch (ncb) {
    SHT_LLAUNCH(1)
    SHT_LLAUNCH(2)
    SHT_LLAUNCH(4)
    SHT_LLAUNCH(8)
    SHT_LLAUNCH(10)
    default:
      return hipErrorInvalidValue;
  }
#undef SHT_LLAUNCH
  return hipGetLastError();
}

int launch_legendre(int form, bool analysis, const GemmArgs& g, int ncb,
                    void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (form == SHT_FORM_FP64) return (int)launch_legendre_t<double>(analysis, g, ncb, st);
  return (int)launch_legendre_t<float>(analysis, g, ncb, st);
}

size_t legendre_lds_bytes(int form, bool analysis, int ncb) {
  if (form == SHT_FORM_FP64)
    return analysis ? lds_analysis<double>(ncb) : lds_synthesis<double>(ncb);
  return analysis ? lds_analysis<float>(ncb) : lds_synthesis<float>(ncb);
}

}  // namespace sht
