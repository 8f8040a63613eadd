// Zonal (longitude) stage of the transform pair, with the equatorial parity
// fold of App. B fused in.
//
// Analysis, Sec. 2 (discretised zonal integral, 1/I convention): for the
// mirror pair of rows (j, J-1-j) the kernel forms z = x_north + i x_south,
// runs one complex FFT of length I in LDS (Stockham, radices 2/3/4/5), and
// separates the two real spectra:
//   X_north^m = (Z^m + conj Z^{I-m}) / 2,  X_south^m = (Z^m - conj Z^{I-m}) / 2i.
// It then writes the symmetric and antisymmetric parts of App. B (eqs. B3,
// B4), already multiplied by the quadrature weight:
//   S^m_j = w_j (X_north^m + X_south^m),  A^m_j = w_j (X_north^m - X_south^m);
// the equator row (odd J) gives S = w X_eq and A = 0.
//
// Synthesis: the reverse.  From S and A (the Legendre sums of Sec. 2,
// eq. iLT, split by parity) the kernel rebuilds X_north = S + A and
// X_south = S - A, packs Z^m = X_north^m + i X_south^m and its Hermitian
// partner at I-m, and one inverse FFT yields both rows:
//   x(lambda_i) = Re X^0 + 2 sum_{m>=1} Re(X^m e^{i m lambda_i}).
//
// Work decomposition: one workgroup per (mirror row pair, block of FB
// fields).  The FB fields go through the LDS buffer one after the other and
// the wavenumbers m <= N of all FB fields are kept in registers, so that each
// workspace access is a contiguous run of 2*FB values (64 bytes) per (m,
// parity, row) instead of one isolated complex value; the analysis stores
// both parities of a row as one run of 4*FB values (ws_col).
//
// Workspace layout (per level): see ws_col and ws_plane; the analysis and
// the synthesis lay it out differently.

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "sht_internal.h"

namespace sht {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}

template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}

// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  return {a.y, -a.x};
}

// In-register DFT of length R with the forward sign exp(-2 pi i t k / R).
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename T>
struct Dft<T, 3> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T h = (T)0.5;
    const T s = (T)0.86602540378443864676372317075293618;  // sin(2 pi / 3)
    cx<T> a = v[0], b = v[1], c = v[2];
    cx<T> sbc = cadd(b, c);
    cx<T> dbc = csub(b, c);
    cx<T> t1 = {a.x - h * sbc.x, a.y - h * sbc.y};
    // -i s (b - c)
    cx<T> t2 = {s * dbc.y, -s * dbc.x};
    v[0] = cadd(a, sbc);
    v[1] = cadd(t1, t2);
    v[2] = csub(t1, t2);
  }
};

template <typename T>
struct Dft<T, 4> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
    cx<T> s0 = cadd(a, c), d0 = csub(a, c);
    cx<T> s1 = cadd(b, d), d1 = mul_mi(csub(b, d));
    v[0] = cadd(s0, s1);
    v[2] = csub(s0, s1);
    v[1] = cadd(d0, d1);
    v[3] = csub(d0, d1);
  }
};

template <typename T>
struct Dft<T, 8> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T r = (T)0.70710678118654752440084436210484904;  // 1/sqrt(2)
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4>::run(e);
    Dft<T, 4>::run(o);
    // o_k *= exp(-2 pi i k / 8)
    const cx<T> o1 = {r * (o[1].x + o[1].y), r * (o[1].y - o[1].x)};
    const cx<T> o2 = {o[2].y, -o[2].x};
    const cx<T> o3 = {r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <typename T>
struct Dft<T, 5> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T c1 = (T)0.30901699437494742410229341718281906;   // cos(2 pi/5)
    const T c2 = (T)-0.80901699437494742410229341718281906;  // cos(4 pi/5)
    const T s1 = (T)0.95105651629515357211643933337938214;   // sin(2 pi/5)
    const T s2 = (T)0.58778525229247312916870595463907277;   // sin(4 pi/5)
    cx<T> x0 = v[0];
    cx<T> p1 = cadd(v[1], v[4]), q1 = csub(v[1], v[4]);
    cx<T> p2 = cadd(v[2], v[3]), q2 = csub(v[2], v[3]);
    cx<T> r1 = {x0.x + c1 * p1.x + c2 * p2.x, x0.y + c1 * p1.y + c2 * p2.y};
    cx<T> r2 = {x0.x + c2 * p1.x + c1 * p2.x, x0.y + c2 * p1.y + c1 * p2.y};
    // i1 = s1 q1 + s2 q2, i2 = s2 q1 - s1 q2; y1 = r1 - i*i1, y4 = r1 + i*i1,
    // y2 = r2 - i*i2, y3 = r2 + i*i2
    cx<T> i1 = {s1 * q1.x + s2 * q2.x, s1 * q1.y + s2 * q2.y};
    cx<T> i2 = {s2 * q1.x - s1 * q2.x, s2 * q1.y - s1 * q2.y};
    v[0] = {x0.x + p1.x + p2.x, x0.y + p1.y + p2.y};
    v[1] = {r1.x + i1.y, r1.y - i1.x};
    v[4] = {r1.x - i1.y, r1.y + i1.x};
    v[2] = {r2.x + i2.y, r2.y - i2.x};
    v[3] = {r2.x - i2.y, r2.y + i2.x};
  }
};

// ---------------------------------------------------------------------------
// Composite in-register DFTs, R = R1 * R2 (Cooley-Tukey): R2 DFTs of length
// R1 over the inputs n = R2 n1 + n2, the internal twiddles
// exp(-2 pi i n2 k1 / R), then R1 DFTs of length R2; output index
// k = k1 + R1 k2.  The twiddles are compile-time constants.
// ---------------------------------------------------------------------------
constexpr double kTwoPi = 6.283185307179586476925286766559005768;

// sin(x) for |x| <= pi/2 by its Taylor series (accurate to double rounding)
constexpr double csin_small(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

// sin(2 pi e / R) and cos(2 pi e / R) with exact integer range reduction
constexpr double csin2pi(int e, int R) {
  e %= R;
  if (e < 0) e += R;
  // reduce to the first half turn by symmetry: sin(2 pi - x) = -sin(x)
  if (2 * e > R) return -csin2pi(R - e, R);
  // x = 2 pi e / R in [0, pi]; sin(x) = sin(pi - x)
  if (4 * e > R) return csin_small(kTwoPi * (double)(R - 2 * e) / (2.0 * R));
  return csin_small(kTwoPi * (double)e / (double)R);
}

constexpr double ccos2pi(int e, int R) { return csin2pi(4 * e + R, 4 * R); }

// Calls f(integral_constant<int, i>) for i = 0..N-1, so that f can form
// constant expressions from i.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <typename T, int R1, int R2>
struct DftCT {
  static constexpr int R = R1 * R2;
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> y[R2][R1];
    static_for<R2>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      cx<T> t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
      Dft<T, R1>::run(t);
      static_for<R1>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        if constexpr (n2 == 0 || k1 == 0) {
          y[n2][k1] = t[k1];
        } else {
          constexpr T c = (T)ccos2pi(n2 * k1, R), sn = (T)-csin2pi(n2 * k1, R);
          y[n2][k1] = cx<T>{t[k1].x * c - t[k1].y * sn, t[k1].x * sn + t[k1].y * c};
        }
      });
    });
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cx<T> t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2][k1];
      Dft<T, R2>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
};

template <typename T>
struct Dft<T, 6> : DftCT<T, 3, 2> {};
template <typename T>
struct Dft<T, 9> : DftCT<T, 3, 3> {};
template <typename T>
struct Dft<T, 10> : DftCT<T, 5, 2> {};
template <typename T>
struct Dft<T, 12> : DftCT<T, 4, 3> {};
template <typename T>
struct Dft<T, 15> : DftCT<T, 5, 3> {};
template <typename T>
struct Dft<T, 16> : DftCT<T, 4, 4> {};
template <typename T>
struct Dft<T, 20> : DftCT<T, 5, 4> {};

// LDS position of element i of the FFT buffers (dense).
__device__ __forceinline__ int lp(int i) { return i; }

// q = floor(j / d) for 0 <= j < 2^13 and 2 <= d <= 4096, with
// magic = floor((2^32 - 1) / d) + 1 (exhaustively checked over that range).
__device__ __forceinline__ int fastdiv(int j, unsigned magic) {
  return (int)__umulhi((unsigned)j, magic);
}

// One Stockham pass of radix R over FC sequences of length I that lie one
// after the other in LDS, in place: every thread first loads and transforms
// all its butterflies, then (after a barrier) stores them.  Ns is the product
// of the radices of the earlier passes.  A thread owns butterfly position j
// in all FC sequences, so the index arithmetic and the twiddles are shared by
// the FC transforms.  With q = floor(j / Ns) and k = j - q Ns the inputs are
// j + t I/R and the outputs q Ns R + k + t Ns = j R - k (R-1) + t Ns.
template <typename T, int NT, int FC, int MAXI, int R>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int I, int Ns, int twstep,
                                              unsigned magic, const cx<T>* __restrict__ tw) {
  constexpr int BPT = (MAXI / R + NT - 1) / NT;
  const int nb = twstep * Ns;  // I / R
  cx<T> v[BPT][FC][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < nb) {
      cx<T> w[R];
      if (Ns > 1) {
        const int k = j - fastdiv(j, magic) * Ns;
        const int step = k * twstep;
        int idx = step;
#pragma unroll
        for (int t = 1; t < R; ++t) {
          w[t] = tw[idx];
          idx += step;
        }
      }
#pragma unroll
      for (int f = 0; f < FC; ++f) {
        const int src = f * I + j;
#pragma unroll
        for (int t = 0; t < R; ++t) v[b][f][t] = buf[lp(src + t * nb)];
        if (Ns > 1) {
#pragma unroll
          for (int t = 1; t < R; ++t) v[b][f][t] = cmul(v[b][f][t], w[t]);
        }
        Dft<T, R>::run(v[b][f]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + b * NT;
    if (j < nb) {
      int out = j * R;
      if (Ns > 1) out -= (j - fastdiv(j, magic) * Ns) * (R - 1);
#pragma unroll
      for (int f = 0; f < FC; ++f) {
        const int dst = f * I + out;
#pragma unroll
        for (int t = 0; t < R; ++t) buf[lp(dst + t * Ns)] = v[b][f][t];
      }
    }
  }
  __syncthreads();
}

// Forward complex FFTs (sign -) of the FC sequences in buf, natural order in
// and out.  Every thread of the block must call it.
template <typename T, int NT, int FC, int MAXI>
__device__ __forceinline__ void fft_lds(cx<T>* buf, const LevelDesc& L, const cx<T>* tw) {
  for (int p = 0; p < L.nrad; ++p) {
    const int R = L.rad[p], Ns = L.pns[p], tws = L.ptw[p];
    const unsigned mg = L.pmag[p];
    if (R == 8)
      stockham_pass<T, NT, FC, MAXI, 8>(buf, L.I, Ns, tws, mg, tw);
    else if (R == 4)
      stockham_pass<T, NT, FC, MAXI, 4>(buf, L.I, Ns, tws, mg, tw);
    else if (R == 2)
      stockham_pass<T, NT, FC, MAXI, 2>(buf, L.I, Ns, tws, mg, tw);
    else if (R == 3)
      stockham_pass<T, NT, FC, MAXI, 3>(buf, L.I, Ns, tws, mg, tw);
    else
      stockham_pass<T, NT, FC, MAXI, 5>(buf, L.I, Ns, tws, mg, tw);
  }
}

__device__ __forceinline__ int level_of(const FftArgs& a, int item) {
  int l = 0;
  while (l + 1 < a.nlev && item >= a.lev[l + 1].fft_item0) ++l;
  return l;
}

// One past the last work item (slot) of level l.
__device__ __forceinline__ int level_end(const FftArgs& a, int l) {
  return l + 1 < a.nlev ? a.lev[l + 1].fft_item0 : a.nitems;
}

// Store/load FB complex values (2*FB scalars, 64 bytes) starting at a
// 64-byte aligned address, as 16-byte vector accesses.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <typename T, int FB>
__device__ __forceinline__ void store_run(T* dst, const cx<T> (&v)[FB]) {
  static_assert(2 * FB <= 16, "one analysis workspace column block");
  typedef typename Vec16<T>::type V;
  constexpr int E = 16 / sizeof(T);  // scalars per vector
  V* d = reinterpret_cast<V*>(dst);
#pragma unroll
  for (int k = 0; k < 2 * FB / E; ++k) {
    V o;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = k * E + e;
      o[e] = (q & 1) ? v[q >> 1].y : v[q >> 1].x;
    }
    d[k] = o;
  }
}

template <typename T, int FB>
__device__ __forceinline__ void load_run(const T* src, cx<T> (&v)[FB]) {
  typedef typename Vec16<T>::type V;
  constexpr int E = 16 / sizeof(T);
  const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
  for (int k = 0; k < 2 * FB / E; ++k) {
    const V o = s[k];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = k * E + e;
      if (q & 1)
        v[q >> 1].y = o[e];
      else
        v[q >> 1].x = o[e];
    }
  }
}

// The workspace run of one (wavenumber, parity, latitude pair, field block)
// is 2 FB values = 64 bytes, and the thread of wavenumber m holds the whole
// run; consecutive lanes hold consecutive m, whose runs are a plane apart.
// Before storing, the four lanes of each quad exchange 16-byte pieces so
// that lane j holds piece j of the four runs of its quad; a 16-byte store
// instruction then covers 16 whole runs instead of touching 64 cache lines.
constexpr int kQuadXor1 = 0xB1;  // DPP quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;  // DPP quad_perm [2,3,0,1]

// 4x4 transpose of 16-byte pieces across a quad; its own inverse.  Every
// lane of the quad must take part.
__device__ __forceinline__ void quad_transpose(int (&x)[4][4]) {
  const int j = threadIdx.x & 3;
  const bool h1 = (j & 1) != 0, h2 = (j & 2) != 0;
#pragma unroll
  for (int p = 0; p < 4; p += 2)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int v = h1 ? x[p][d] : x[p + 1][d];
      const int r = __builtin_amdgcn_update_dpp(0, v, kQuadXor1, 0xF, 0xF, false);
      if (h1)
        x[p][d] = r;
      else
        x[p + 1][d] = r;
    }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int v = h2 ? x[p][d] : x[p + 2][d];
      const int r = __builtin_amdgcn_update_dpp(0, v, kQuadXor2, 0xF, 0xF, false);
      if (h2)
        x[p][d] = r;
      else
        x[p + 2][d] = r;
    }
}

// Store the runs v of the quad's four wavenumbers m - j .. m - j + 3
// (j = lane in quad) at dst(m') = base + (2 m') * plane; runs with m' > N
// are skipped.  All lanes of the quad must call it.  base is uniform and the
// 64 lanes of a wave hold consecutive wavenumbers: each address is a
// uniform 64-bit base at the wave's first wavenumber plus a 32-bit per-lane
// byte offset of fewer than 128 planes (zonal_offsets_fit).  A run of 2 FB
// values is 64 or 128 bytes; a 128-byte run goes as two 64-byte halves.
template <typename T, int FB>
__device__ __forceinline__ void store_runs_quad(T* base, long long plane, int m, int N,
                                                const cx<T> (&v)[FB]) {
  constexpr int HALVES = 2 * FB * (int)sizeof(T) / 64;
  static_assert(HALVES * 64 == 2 * FB * (int)sizeof(T) && HALVES <= 2, "64- or 128-byte runs");
  const int lane = threadIdx.x & 63, j = lane & 3;
  const long long step64 = 2 * plane * (long long)sizeof(T);
  const int mw = __builtin_amdgcn_readfirstlane(m - lane);  // the wave's first wavenumber
  char* b = reinterpret_cast<char*>(base) + (long long)mw * step64;
  const unsigned step = (unsigned)step64;
#pragma unroll
  for (int hf = 0; hf < HALVES; ++hf) {
    int x[4][4];
    __builtin_memcpy(x, reinterpret_cast<const char*>(v) + 64 * hf, 64);
    quad_transpose(x);
    unsigned off = (unsigned)(lane - j) * step + 16u * (unsigned)j + 64u * (unsigned)hf;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mr = m - j + r;
      if (mr <= N) {
        typedef int i32x4 __attribute__((ext_vector_type(4)));
        *reinterpret_cast<i32x4*>(b + off) = i32x4{x[r][0], x[r][1], x[r][2], x[r][3]};
      }
      off += step;
    }
  }
}

// Work item = (level, mirror row pair jp, block fb of FB fields).
struct Item {
  int l, jp, fb, js;
  bool eq;
};

// Workgroup b runs on XCD b mod 8 and walks the slots b, b + G, ...
// (G = gridDim.x, a multiple of 8 on a full device).  The slots of a level
// are a contiguous range; within it, local slot i is mapped to the level's
// list position x R' + k (x = i mod 8, k = i / 8, R' the length of the
// x-th eighth of the level's list): the workgroups of one XCD work through
// one contiguous eighth of every level, so the field blocks of one latitude
// pair run on one XCD at about the same time and fill whole workspace lines
// in its L2, and every XCD gets the same share of each level.  The map is a
// permutation of [0, n).
__device__ __forceinline__ int xcd_map(int i, int n) {
  const int x = i & 7, k = i >> 3;
  const int R = n >> 3, rem = n & 7;
  return x * R + (x < rem ? x : rem) + k;
}

__device__ __forceinline__ Item decode_item(const FftArgs& a, int slot) {
  Item it;
  it.l = level_of(a, slot);
  const LevelDesc& L = a.lev[it.l];
  const int local = xcd_map(slot - L.fft_item0, level_end(a, it.l) - L.fft_item0);
  it.jp = local / L.nfb;
  it.fb = local - it.jp * L.nfb;
  it.eq = (L.J & 1) && (it.jp == (L.J >> 1));
  it.js = L.J - 1 - it.jp;
  return it;
}

template <typename T>
__device__ __forceinline__ T row_scale(const FftArgs& a, const LevelDesc& L, int jp) {
  T r = (T)1;
  if (a.use_w) r = (T)L.wrow[jp];
  if (a.use_inv_I) r = (T)((double)r / (double)L.I);
  return r;
}

// ---------------------------------------------------------------------------
// analysis: grid [F][J][I] -> workspace S/A
// Persistent workgroups walk the work items with a stride of gridDim.x.
// FB fields per item, FC of them transformed together; the rows of the next
// FC fields (of this item, or the first FC of the next item) are prefetched
// into registers while the current ones are transformed, so loads, FFTs and
// the stores of the previous item overlap.  Twiddles are staged in LDS when
// TWL is set (reloaded when the level changes).
// ---------------------------------------------------------------------------
// The slots item, item + G, ... below `end` (any levels); returns the first
// slot past them.  Every thread of the workgroup calls it alike.
template <typename T, int NT, int FB, int FC, int MS, int MAXI, bool TWL>
__device__ __forceinline__ int zonal_analysis_run(const FftArgs& a, int item, int end, unsigned char* smem_raw) {
  constexpr int NRD = FB / FC;
  constexpr int LPT = (MAXI + NT - 1) / NT;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const T* grid0 = static_cast<const T*>(a.src);
  T* ws0 = static_cast<T*>(a.dst);
  const T msc = (T)a.mscale;

  T pn[FC][LPT], ps[FC][LPT];
  auto load_rows = [&](int item, int rd) __attribute__((always_inline)) {
    const Item it = decode_item(a, item);
    const LevelDesc& L = a.lev[it.l];
    const T* grid = grid0 + L.grid_off;
#pragma unroll
    for (int fc = 0; fc < FC; ++fc) {
      const int f = it.fb * FB + rd * FC + fc;
      const bool valid = f < L.F;
      const T* rn = grid + ((long long)f * L.J + it.jp) * L.I;
      const T* rs = grid + ((long long)f * L.J + it.js) * L.I;
#pragma unroll
      for (int e = 0; e < LPT; ++e) {
        const int i = threadIdx.x + e * NT;
        pn[fc][e] = (valid && i < L.I) ? rn[i] : (T)0;
        ps[fc][e] = (valid && !it.eq && i < L.I) ? rs[i] : (T)0;
      }
    }
  };

  if (item >= end) return item;
  int lcur = -1;
  const cx<T>* tw = nullptr;
  load_rows(item, 0);
  for (; item < end; item += gridDim.x) {
    const Item it = decode_item(a, item);
    const LevelDesc& L = a.lev[it.l];
    const int I = L.I, N = L.N;
    if (it.l != lcur) {
      if (TWL) {
        __syncthreads();  // the previous level's twiddles are no longer read
        cx<T>* twl = buf + a.tw_lds;
        const cx<T>* twg = static_cast<const cx<T>*>(L.tw);
        for (int i = threadIdx.x; i < I; i += NT) twl[i] = twg[i];
        tw = twl;
      } else {
        tw = static_cast<const cx<T>*>(L.tw);
      }
      lcur = it.l;
    }
    const T rscale = row_scale<T>(a, L, it.jp);
    const int next = item + (int)gridDim.x;

    cx<T> stS[MS][FB], stA[MS][FB];
#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {
#pragma unroll
      for (int fc = 0; fc < FC; ++fc)
#pragma unroll
        for (int e = 0; e < LPT; ++e) {
          const int i = threadIdx.x + e * NT;
          if (i < I) buf[lp(fc * I + i)] = cx<T>{pn[fc][e], ps[fc][e]};
        }
      __syncthreads();
      if (rd + 1 < NRD)
        load_rows(item, rd + 1);
      else if (next < end)
        load_rows(next, 0);
      fft_lds<T, NT, FC, MAXI>(buf, L, tw);
#pragma unroll
      for (int s = 0; s < MS; ++s) {
        const int m = threadIdx.x + s * NT;
#pragma unroll
        for (int fc = 0; fc < FC; ++fc) {
          cx<T> S = {(T)0, (T)0}, A = {(T)0, (T)0};
          if (m <= N) {
            const cx<T> P = buf[lp(fc * I + m)];
            cx<T> Q = buf[lp(fc * I + (m == 0 ? 0 : I - m))];
            Q.y = -Q.y;  // conj Z^{I-m}
            const T h = (T)0.5;
            const cx<T> Xn = {h * (P.x + Q.x), h * (P.y + Q.y)};
            const cx<T> Xs = {h * (P.y - Q.y), -h * (P.x - Q.x)};
            const T sc = m == 0 ? rscale : rscale * msc;
            S = cx<T>{sc * (Xn.x + Xs.x), sc * (Xn.y + Xs.y)};
            A = cx<T>{sc * (Xn.x - Xs.x), sc * (Xn.y - Xs.y)};
            if (m == 0) {
              S.y = (T)0;
              A.y = (T)0;
            }
            if (it.eq) A = cx<T>{(T)0, (T)0};
          }
          stS[s][rd * FC + fc] = S;
          stA[s][rd * FC + fc] = A;
        }
      }
      __syncthreads();
    }

    T* ws = ws0 + L.ws_off;
    const long long Cp = L.Cp;
    const long long plane = L.wplane;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int m = threadIdx.x + s * NT;
      if (m <= N) {
        // the item's column block (ws_col): even run, then odd run
        T* dS = ws + (2LL * m) * plane + (long long)it.jp * 2 * Cp + 4 * it.fb * FB;
        store_run<T, FB>(dS, stS[s]);
        store_run<T, FB>(dS + 2 * FB, stA[s]);
      }
    }
  }
  return item;
}

template <typename T, int NT, int FB, int FC, int MS, int MAXI, bool TWL>
__global__ __launch_bounds__(NT) void k_zonal_analysis(const FftArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  zonal_analysis_run<T, NT, FB, FC, MS, MAXI, TWL>(a, blockIdx.x, a.nitems, smem_raw);
}

// ---------------------------------------------------------------------------
// synthesis: workspace S/A -> grid [F][J][I]
// Persistent like the analysis; the workspace runs of the next item are
// loaded as soon as the last round of the current item has filled its
// buffers, so they overlap that round's FFT and row stores.
// ---------------------------------------------------------------------------
template <typename T, int NT, int FB, int FC, int MS, int MAXI, bool TWL>
__device__ __forceinline__ int zonal_synthesis_run(const FftArgs& a, int item, int end, unsigned char* smem_raw) {
  constexpr int NRD = FB / FC;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const T* ws0 = static_cast<const T*>(a.src);
  T* grid0 = static_cast<T*>(a.dst);
  const T msc = (T)a.mscale;

  cx<T> stS[MS][FB], stA[MS][FB];
  auto load_ws = [&](int item) __attribute__((always_inline)) {
    const Item it = decode_item(a, item);
    const LevelDesc& L = a.lev[it.l];
    const T* ws = ws0 + L.ws_off;
    const long long Cp = L.Cp;
    const long long plane = L.wplane;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int m = threadIdx.x + s * NT;
      // rows below the first 128-latitude tile the Legendre synthesis
      // computes for this m (reduced transform) are zero
      if (m <= L.N && (!a.jstart || it.jp >= (a.jstart[L.m_base + m] & ~127))) {
        const T* sS = ws + (2LL * m) * plane + (long long)it.jp * Cp + 2 * it.fb * FB;
        load_run<T, FB>(sS, stS[s]);
        load_run<T, FB>(sS + L.spoff, stA[s]);
      } else {
#pragma unroll
        for (int q = 0; q < FB; ++q) stS[s][q] = stA[s][q] = cx<T>{(T)0, (T)0};
      }
    }
  };

  if (item >= end) return item;
  int lcur = -1;
  const cx<T>* tw = nullptr;
  load_ws(item);
  for (; item < end; item += gridDim.x) {
    const Item it = decode_item(a, item);
    const LevelDesc& L = a.lev[it.l];
    const int I = L.I, J = L.J, N = L.N;
    if (it.l != lcur) {
      if (TWL) {
        __syncthreads();
        cx<T>* twl = buf + a.tw_lds;
        const cx<T>* twg = static_cast<const cx<T>*>(L.tw);
        for (int i = threadIdx.x; i < I; i += NT) twl[i] = twg[i];
        tw = twl;
      } else {
        tw = static_cast<const cx<T>*>(L.tw);
      }
      lcur = it.l;
    }
    const T rscale = row_scale<T>(a, L, it.jp);
    const int next = item + (int)gridDim.x;
    T* grid = grid0 + L.grid_off;

#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {
#pragma unroll
      for (int fc = 0; fc < FC; ++fc) {
        const int bf = fc * I;
        // zero the bins no thread fills: N < i < I-N
        for (int i = N + 1 + threadIdx.x; i < I - N; i += NT) buf[lp(bf + i)] = cx<T>{(T)0, (T)0};
#pragma unroll
        for (int s = 0; s < MS; ++s) {
          const int m = threadIdx.x + s * NT;
          if (m <= N) {
            const cx<T> S = stS[s][rd * FC + fc], A = stA[s][rd * FC + fc];
            const T sc = m == 0 ? (T)1 : msc;
            cx<T> Xn = {sc * (S.x + A.x), sc * (S.y + A.y)};
            cx<T> Xs = {sc * (S.x - A.x), sc * (S.y - A.y)};
            if (m == 0) {
              Xn.y = (T)0;
              Xs.y = (T)0;
            }
            // the buffer holds conj(Z): the forward FFT of conj(Z) is the
            // conjugate of the inverse transform of Z, with
            // Z^m = Xn + i Xs and Z^{I-m} = conj(Xn) + i conj(Xs)
            buf[lp(bf + m)] = cx<T>{Xn.x - Xs.y, -(Xn.y + Xs.x)};
            if (m > 0) buf[lp(bf + I - m)] = cx<T>{Xn.x + Xs.y, Xn.y - Xs.x};
          }
        }
      }
      __syncthreads();
      if (rd + 1 == NRD && next < end) load_ws(next);
      fft_lds<T, NT, FC, MAXI>(buf, L, tw);
#pragma unroll
      for (int fc = 0; fc < FC; ++fc) {
        const int f = it.fb * FB + rd * FC + fc;
        if (f < L.F) {
          const int bf = fc * I;
          T* rn = grid + ((long long)f * J + it.jp) * I;
          T* rs = grid + ((long long)f * J + it.js) * I;
          for (int i = threadIdx.x; i < I; i += NT) {
            const cx<T> y = buf[lp(bf + i)];
            rn[i] = rscale * y.x;
            if (!it.eq) rs[i] = -rscale * y.y;
          }
        }
      }
      __syncthreads();
    }
  }
  return item;
}

template <typename T, int NT, int FB, int FC, int MS, int MAXI, bool TWL>
__global__ __launch_bounds__(NT) void k_zonal_synthesis(const FftArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  zonal_synthesis_run<T, NT, FB, FC, MS, MAXI, TWL>(a, blockIdx.x, a.nitems, smem_raw);
}

// ---------------------------------------------------------------------------
// Fixed-length transforms: I = 16 R2 R3 in three passes with compile-time
// radices, twiddle strides and index arithmetic.
//
// The FC sequences of a round lie in LDS with a field stride of IP = 17 I/16
// complex values.  The output of the radix-16 first pass (Ns = 1, element
// 16 j + t of the natural order) is stored at the padded position 17 j + t,
// so that the 64 lanes of a wave, which own consecutive j, hit distinct
// banks; the second pass reads that padded order (its inputs j + t I/R2 sit
// at j + j/16 + t (17/16)(I/R2), since I/R2 is a multiple of 16) and writes
// the natural order; the third pass reads and writes the natural order.
// The twiddles of passes two and three are staged in LDS as [t-1][k]
// (k = butterfly position within its Ns-block), so that consecutive lanes
// read consecutive entries.
//
// Analysis loads the grid rows straight into the registers of the first
// pass (thread of butterfly j loads elements j + t I/16 of both rows, which
// is coalesced across the lanes); synthesis stores the last pass straight to
// the grid rows (element j + t Ns3 of each of the two rows).
// ---------------------------------------------------------------------------
template <int I_, int R2_, int R3_>
struct Plan3 {
  static constexpr int I = I_, R1 = 16, R2 = R2_, R3 = R3_;
  static_assert(R1 * R2 * R3 == I, "radices must multiply to I");
  static constexpr int nb1 = I / R1, nb2 = I / R2, nb3 = I / R3;
  static constexpr int Ns2 = R1, Ns3 = R1 * R2;
  static_assert(nb3 == Ns3, "last pass");
  static_assert(I % 16 == 0 && nb2 % 16 == 0, "padded layout");
  static constexpr int IP = I + I / 16;        // padded field stride
  static constexpr int S2P = nb2 + nb2 / 16;   // padded stride of pass-2 inputs
  static constexpr int tw2 = 0, tw3 = (R2 - 1) * Ns2, ntw = tw3 + (R3 - 1) * Ns3;
};

template <typename T, class P, int NT, int FC>
struct Fft3 {
  static constexpr int S1 = (FC * P::nb1 + NT - 1) / NT;
  static constexpr int S2 = (FC * P::nb2 + NT - 1) / NT;
  static constexpr int S3 = (FC * P::nb3 + NT - 1) / NT;

  // twiddles of passes two and three from the table exp(-2 pi i e / I)
  static __device__ void stage_twiddles(cx<T>* twl, const cx<T>* __restrict__ twg) {
    for (int x = threadIdx.x; x < P::ntw; x += NT) {
      int e;
      if (x < P::tw3) {
        const int t = x / P::Ns2 + 1, k = x - (t - 1) * P::Ns2;
        e = t * k * P::R3;
      } else {
        const int y = x - P::tw3;
        const int t = y / P::Ns3 + 1, k = y - (t - 1) * P::Ns3;
        e = t * k;
      }
      twl[x] = twg[e];
    }
  }

  // first pass on values already in registers (v[s] = inputs j + t nb1 of
  // slot s); results stored in the padded order
  static __device__ __forceinline__ void pass1_store(cx<T> (&v)[S1][16], cx<T>* buf) {
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int u = threadIdx.x + s * NT;
      if (u < FC * P::nb1) {
        const int f = u / P::nb1, j = u - f * P::nb1;
        Dft<T, 16>::run(v[s]);
        cx<T>* d = buf + f * P::IP + 17 * j;
#pragma unroll
        for (int t = 0; t < 16; ++t) d[t] = v[s][t];
      }
    }
  }

  // first pass from the natural order in LDS (in place, padded result)
  static __device__ __forceinline__ void pass1_lds(cx<T>* buf) {
    cx<T> v[S1][16];
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int u = threadIdx.x + s * NT;
      if (u < FC * P::nb1) {
        const int f = u / P::nb1, j = u - f * P::nb1;
        const cx<T>* src = buf + f * P::IP + j;
#pragma unroll
        for (int t = 0; t < 16; ++t) v[s][t] = src[t * P::nb1];
      }
    }
    __syncthreads();
    pass1_store(v, buf);
    __syncthreads();
  }

  // second pass: padded order in, natural order out (in place)
  static __device__ __forceinline__ void pass2(cx<T>* buf, const cx<T>* twl) {
    constexpr int R = P::R2;
    cx<T> v[S2][R];
#pragma unroll
    for (int s = 0; s < S2; ++s) {
      const int u = threadIdx.x + s * NT;
      if (u < FC * P::nb2) {
        const int f = u / P::nb2, j = u - f * P::nb2;
        const cx<T>* src = buf + f * P::IP + j + (j >> 4);
#pragma unroll
        for (int t = 0; t < R; ++t) v[s][t] = src[t * P::S2P];
        const cx<T>* w = twl + P::tw2 + (j & 15);
#pragma unroll
        for (int t = 1; t < R; ++t) v[s][t] = cmul(v[s][t], w[(t - 1) * P::Ns2]);
        Dft<T, R>::run(v[s]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S2; ++s) {
      const int u = threadIdx.x + s * NT;
      if (u < FC * P::nb2) {
        const int f = u / P::nb2, j = u - f * P::nb2;
        cx<T>* d = buf + f * P::IP + (j >> 4) * (16 * R) + (j & 15);
#pragma unroll
        for (int t = 0; t < R; ++t) d[t * 16] = v[s][t];
      }
    }
    __syncthreads();
  }

  // third pass into registers: v[s][t] is element j + t Ns3 of field f,
  // (f, j) = slot s of this thread
  static __device__ __forceinline__ void pass3_regs(cx<T> (&v)[S3][P::R3], const cx<T>* buf,
                                                    const cx<T>* twl) {
    constexpr int R = P::R3;
#pragma unroll
    for (int s = 0; s < S3; ++s) {
      const int u = threadIdx.x + s * NT;
      if (u < FC * P::nb3) {
        const int f = u / P::nb3, j = u - f * P::nb3;
        const cx<T>* src = buf + f * P::IP + j;
#pragma unroll
        for (int t = 0; t < R; ++t) v[s][t] = src[t * P::nb3];
        const cx<T>* w = twl + P::tw3 + j;
#pragma unroll
        for (int t = 1; t < R; ++t) v[s][t] = cmul(v[s][t], w[(t - 1) * P::Ns3]);
        Dft<T, R>::run(v[s]);
      }
    }
  }
};

// The slots item, item + G, ... of level l (item is one of them); returns
// the first slot past the level.  Every thread of the workgroup calls it
// alike.
template <typename T, class P, int NT, int FB, int FC, int MS>
__device__ __forceinline__ int zonal_analysis_run_p3(const FftArgs& a, int l, int item, unsigned char* smem_raw) {
  using F3 = Fft3<T, P, NT, FC>;
  constexpr int NRD = FB / FC, I = P::I;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* twl = buf + FC * P::IP;
  const LevelDesc& L = a.lev[l];
  const int s0 = L.fft_item0, end = level_end(a, l), n = end - s0;
  const T* grid = static_cast<const T*>(a.src) + L.grid_off;
  T* ws = static_cast<T*>(a.dst) + L.ws_off;
  const T msc = (T)a.mscale;
  const int N = L.N, J = L.J;

  if (item >= end) return item;
  F3::stage_twiddles(twl, static_cast<const cx<T>*>(L.tw));

  cx<T> v1[F3::S1][16];
  auto load_rows = [&](int slot, int rd) __attribute__((always_inline)) {
    const int itm = xcd_map(slot - s0, n);
    const int jp = itm / L.nfb, fb = itm - jp * L.nfb;
    const bool eq = (J & 1) && (jp == (J >> 1));
#pragma unroll
    for (int s = 0; s < F3::S1; ++s) {
      const int u = threadIdx.x + s * NT;
      if (u < FC * P::nb1) {
        const int f = u / P::nb1, j = u - f * P::nb1;
        const int fld = fb * FB + rd * FC + f;
        const bool valid = fld < L.F;
        const T* rn = grid + ((long long)fld * J + jp) * I + j;
        const T* rs = grid + ((long long)fld * J + (J - 1 - jp)) * I + j;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          v1[s][t].x = valid ? rn[t * P::nb1] : (T)0;
          v1[s][t].y = (valid && !eq) ? rs[t * P::nb1] : (T)0;
        }
      }
    }
  };

  load_rows(item, 0);
  for (; item < end; item += gridDim.x) {
    const int itm = xcd_map(item - s0, n);
    const int jp = itm / L.nfb, fb = itm - jp * L.nfb;
    const bool eq = (J & 1) && (jp == (J >> 1));
    const T rscale = row_scale<T>(a, L, jp);
    const int next = item + (int)gridDim.x;

    cx<T> stS[MS][FB], stA[MS][FB];
#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {
      F3::pass1_store(v1, buf);
      __syncthreads();
      if (rd + 1 < NRD)
        load_rows(item, rd + 1);
      else if (next < end)
        load_rows(next, 0);
      F3::pass2(buf, twl);
      {
        cx<T> v3[F3::S3][P::R3];
        F3::pass3_regs(v3, buf, twl);
        __syncthreads();
        // only the bins m <= N and I - m (m <= N) are used by the fold
#pragma unroll
        for (int s = 0; s < F3::S3; ++s) {
          const int u = threadIdx.x + s * NT;
          if (u < FC * P::nb3) {
            const int f = u / P::nb3, j = u - f * P::nb3;
            cx<T>* d = buf + f * P::IP + j;
#pragma unroll
            for (int t = 0; t < P::R3; ++t) {
              const int pos = j + t * P::Ns3;
              if (pos <= N || pos >= I - N) d[t * P::Ns3] = v3[s][t];
            }
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int s = 0; s < MS; ++s) {
        const int m = threadIdx.x + s * NT;
#pragma unroll
        for (int fc = 0; fc < FC; ++fc) {
          cx<T> S = {(T)0, (T)0}, A = {(T)0, (T)0};
          if (m <= N) {
            const cx<T> Pm = buf[fc * P::IP + m];
            cx<T> Q = buf[fc * P::IP + (m == 0 ? 0 : I - m)];
            Q.y = -Q.y;  // conj Z^{I-m}
            const T h = (T)0.5;
            const cx<T> Xn = {h * (Pm.x + Q.x), h * (Pm.y + Q.y)};
            const cx<T> Xs = {h * (Pm.y - Q.y), -h * (Pm.x - Q.x)};
            const T sc = m == 0 ? rscale : rscale * msc;
            S = cx<T>{sc * (Xn.x + Xs.x), sc * (Xn.y + Xs.y)};
            A = cx<T>{sc * (Xn.x - Xs.x), sc * (Xn.y - Xs.y)};
            if (m == 0) {
              S.y = (T)0;
              A.y = (T)0;
            }
            if (eq) A = cx<T>{(T)0, (T)0};
          }
          stS[s][rd * FC + fc] = S;
          stA[s][rd * FC + fc] = A;
        }
      }
      __syncthreads();
    }

    const long long Cp = L.Cp;
    const long long plane = L.wplane;
    // the item's column blocks of W = min(2 FB, 16) columns (ws_col): the
    // even run at the start of each, the odd one W elements later; a
    // 16-field item's two blocks are written in address order (even and odd
    // piece of the first block, then of the second), one 128-byte line after
    // the other
    constexpr int WB = 2 * FB < 16 ? 2 * FB : 16;
    T* wrow = ws + (long long)jp * 2 * Cp + 4 * fb * FB;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int m = threadIdx.x + s * NT;
      if constexpr (2 * FB == WB) {
        store_runs_quad<T, FB>(wrow, plane, m, N, stS[s]);
        store_runs_quad<T, FB>(wrow + WB, plane, m, N, stA[s]);
      } else {
        static_assert(2 * FB == 2 * WB, "one or two column blocks per item");
        typedef const cx<T>(&Half)[FB / 2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          store_runs_quad<T, FB / 2>(wrow + 2 * WB * h, plane, m, N,
                                     reinterpret_cast<Half>(stS[s][h * (FB / 2)]));
          store_runs_quad<T, FB / 2>(wrow + 2 * WB * h + WB, plane, m, N,
                                     reinterpret_cast<Half>(stA[s][h * (FB / 2)]));
        }
      }
    }
  }
  return item;
}

template <typename T, class P, int NT, int FB, int FC, int MS>
__global__ __launch_bounds__(NT) void k_zonal_analysis_p3(const FftArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  zonal_analysis_run_p3<T, P, NT, FB, FC, MS>(a, 0, blockIdx.x, smem_raw);
}

template <typename T, class P, int NT, int FB, int FC, int MS>
__device__ __forceinline__ int zonal_synthesis_run_p3(const FftArgs& a, int l, int item, unsigned char* smem_raw) {
  using F3 = Fft3<T, P, NT, FC>;
  constexpr int NRD = FB / FC, I = P::I;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* twl = buf + FC * P::IP;
  const LevelDesc& L = a.lev[l];
  const int s0 = L.fft_item0, end = level_end(a, l), n = end - s0;
  const T* ws = static_cast<const T*>(a.src) + L.ws_off;
  T* grid = static_cast<T*>(a.dst) + L.grid_off;
  const T msc = (T)a.mscale;
  const int N = L.N, J = L.J;
  const long long Cp = L.Cp;
  const long long plane = L.wplane;

  cx<T> stS[MS][FB], stA[MS][FB];
  auto load_ws = [&](int slot) __attribute__((always_inline)) {
    const int itm = xcd_map(slot - s0, n);
    const int jp = itm / L.nfb, fb = itm - jp * L.nfb;
    // the runs of the wave's 64 consecutive wavenumbers: a uniform base at
    // its first wavenumber plus 32-bit lane offsets (zonal_offsets_fit)
    const int lane = threadIdx.x & 63;
    const unsigned lstep = (unsigned)(2 * plane * (long long)sizeof(T));
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int m = threadIdx.x + s * NT;
      // rows below the first 128-latitude tile the Legendre synthesis
      // computes for this m (reduced transform) are zero
      if (m <= N && (!a.jstart || jp >= (a.jstart[L.m_base + m] & ~127))) {
        const int mw = __builtin_amdgcn_readfirstlane(m - lane);
        const char* wb = reinterpret_cast<const char*>(ws + (2LL * mw) * plane + (long long)jp * Cp + 2 * fb * FB);
        const T* sS = reinterpret_cast<const T*>(wb + (unsigned)lane * lstep);
        load_run<T, FB>(sS, stS[s]);
        load_run<T, FB>(sS + L.spoff, stA[s]);
      } else {
#pragma unroll
        for (int q = 0; q < FB; ++q) stS[s][q] = stA[s][q] = cx<T>{(T)0, (T)0};
      }
    }
  };

  if (item >= end) return item;
  F3::stage_twiddles(twl, static_cast<const cx<T>*>(L.tw));
  load_ws(item);
  for (; item < end; item += gridDim.x) {
    const int itm = xcd_map(item - s0, n);
    const int jp = itm / L.nfb, fb = itm - jp * L.nfb;
    const bool eq = (J & 1) && (jp == (J >> 1));
    const T rscale = row_scale<T>(a, L, jp);
    const int next = item + (int)gridDim.x;

#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {
#pragma unroll
      for (int fc = 0; fc < FC; ++fc) {
        cx<T>* bf = buf + fc * P::IP;
        // zero the bins no thread fills: N < i < I-N
        for (int i = N + 1 + threadIdx.x; i < I - N; i += NT) bf[i] = cx<T>{(T)0, (T)0};
#pragma unroll
        for (int s = 0; s < MS; ++s) {
          const int m = threadIdx.x + s * NT;
          if (m <= N) {
            const cx<T> S = stS[s][rd * FC + fc], A = stA[s][rd * FC + fc];
            const T sc = m == 0 ? (T)1 : msc;
            cx<T> Xn = {sc * (S.x + A.x), sc * (S.y + A.y)};
            cx<T> Xs = {sc * (S.x - A.x), sc * (S.y - A.y)};
            if (m == 0) {
              Xn.y = (T)0;
              Xs.y = (T)0;
            }
            // conj(Z) with Z^m = Xn + i Xs and Z^{I-m} = conj(Xn) + i conj(Xs);
            // the forward FFT of conj(Z) is the conjugate of the inverse one
            bf[m] = cx<T>{Xn.x - Xs.y, -(Xn.y + Xs.x)};
            if (m > 0) bf[I - m] = cx<T>{Xn.x + Xs.y, Xn.y - Xs.x};
          }
        }
      }
      __syncthreads();
      if (rd + 1 == NRD && next < end) load_ws(next);
      F3::pass1_lds(buf);
      F3::pass2(buf, twl);
      cx<T> v3[F3::S3][P::R3];
      F3::pass3_regs(v3, buf, twl);
#pragma unroll
      for (int s = 0; s < F3::S3; ++s) {
        const int u = threadIdx.x + s * NT;
        if (u < FC * P::nb3) {
          const int f = u / P::nb3, j = u - f * P::nb3;
          const int fld = fb * FB + rd * FC + f;
          if (fld < L.F) {
            T* rn = grid + ((long long)fld * J + jp) * I + j;
            T* rs = grid + ((long long)fld * J + (J - 1 - jp)) * I + j;
#pragma unroll
            for (int t = 0; t < P::R3; ++t) rn[t * P::Ns3] = rscale * v3[s][t].x;
            if (!eq) {
#pragma unroll
              for (int t = 0; t < P::R3; ++t) rs[t * P::Ns3] = -rscale * v3[s][t].y;
            }
          }
        }
      }
      __syncthreads();  // the next round refills the buffer
    }
  }
  return item;
}

template <typename T, class P, int NT, int FB, int FC, int MS>
__global__ __launch_bounds__(NT) void k_zonal_synthesis_p3(const FftArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  zonal_synthesis_run_p3<T, P, NT, FB, FC, MS>(a, 0, blockIdx.x, smem_raw);
}


// ---------------------------------------------------------------------------
// Multi-level plans in one launch.  A configuration says how a level runs:
// with a compile-time three-pass plan (ZP3) or with runtime radices (ZRt).
// The persistent workgroups of k_zonal_levels walk their slots in increasing
// order, which visits the levels one after the other, each as a contiguous
// run of slots (every level's items are spread over all XCDs, see xcd_map);
// a run is handed to the level's configuration (LevelDesc::zk), and the LDS
// is reused by the next run after a barrier.  One launch therefore covers
// every level, with no idle tail between levels.
// ---------------------------------------------------------------------------
template <class P, int FC, int MS>
struct ZP3 {
  template <typename T>
  static constexpr size_t lds() {
    return (size_t)(FC * P::IP + P::ntw) * sizeof(cx<T>);
  }
  template <typename T, int NT, int FB, bool ANA>
  static __device__ __forceinline__ int run(const FftArgs& a, int l, int item, unsigned char* smem) {
    if constexpr (ANA)
      return zonal_analysis_run_p3<T, P, NT, FB, FC, MS>(a, l, item, smem);
    else
      return zonal_synthesis_run_p3<T, P, NT, FB, FC, MS>(a, l, item, smem);
  }
};

// runtime radices, twiddles staged in LDS at FftArgs::tw_lds
template <int FC, int MS, int MAXI>
struct ZRt {
  static constexpr int fc = FC, maxi = MAXI, ms = MS;
  template <typename T, int NT, int FB, bool ANA>
  static __device__ __forceinline__ int run(const FftArgs& a, int l, int item, unsigned char* smem) {
    if constexpr (ANA)
      return zonal_analysis_run<T, NT, FB, FC, MS, MAXI, true>(a, item, level_end(a, l), smem);
    else
      return zonal_synthesis_run<T, NT, FB, FC, MS, MAXI, true>(a, item, level_end(a, l), smem);
  }
};

template <typename T, int NT, int FB, bool ANA, class C, class... Cs>
__device__ __forceinline__ int zonal_run_cfg(const FftArgs& a, int k, int l, int item, unsigned char* smem) {
  if (k == 0) return C::template run<T, NT, FB, ANA>(a, l, item, smem);
  if constexpr (sizeof...(Cs) > 0)
    return zonal_run_cfg<T, NT, FB, ANA, Cs...>(a, k - 1, l, item, smem);
  else
    return level_end(a, l);  // (not reached: the launcher gives every level a configuration)
}

template <typename T, int NT, int FB, bool ANA, class... Cs>
__global__ __launch_bounds__(NT) void k_zonal_levels(const FftArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int item = blockIdx.x;
  while (item < a.nitems) {
    const int l = level_of(a, item);
    item = zonal_run_cfg<T, NT, FB, ANA, Cs...>(a, a.lev[l].zk, l, item, smem_raw);
    __syncthreads();  // the next level's run refills the LDS
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// LDS per workgroup on gfx950 is 160 KiB; above 64 KiB a kernel has to opt in.
constexpr size_t kMaxLds = 160 * 1024;

template <auto Kernel>
static void lds_optin(size_t bytes) {
  static size_t done = 0;  // one flag per kernel instantiation
  if (bytes > 65536 && bytes > done) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    done = bytes;
  }
}

static int g_num_cu = 0;

template <typename T, int NT, int FB, int FC, int MS, int MAXI>
static hipError_t launch_cfg(bool analysis, const FftArgs& a, int maxI, hipStream_t st) {
  // FC padded buffers sized for the largest level, then the twiddles
  FftArgs a2 = a;
  const int belems = (FC * maxI + 1) & ~1;
  a2.tw_lds = belems;
  const size_t buf = (size_t)belems * sizeof(cx<T>);
  const size_t twb = (size_t)maxI * sizeof(cx<T>);
  const bool twl = buf + twb <= kMaxLds;
  const size_t lds = buf + (twl ? twb : 0);
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        g_num_cu <= 0)
      g_num_cu = 256;
  }
  // persistent workgroups: as many as fit on the device at once
  int per_cu = (int)(kMaxLds / lds);
  const int by_waves = 2048 / NT;
  per_cu = per_cu < by_waves ? per_cu : by_waves;
  per_cu = per_cu < 1 ? 1 : per_cu;
  int nwg = g_num_cu * per_cu;
  nwg = nwg < a.nitems ? nwg : a.nitems;
  const dim3 grid(nwg), block(NT);
  if (analysis) {
    if (twl) {
      lds_optin<k_zonal_analysis<T, NT, FB, FC, MS, MAXI, true>>(lds);
      hipLaunchKernelGGL((k_zonal_analysis<T, NT, FB, FC, MS, MAXI, true>), grid, block, lds, st, a2);
    } else {
      lds_optin<k_zonal_analysis<T, NT, FB, FC, MS, MAXI, false>>(lds);
      hipLaunchKernelGGL((k_zonal_analysis<T, NT, FB, FC, MS, MAXI, false>), grid, block, lds, st, a2);
    }
  } else {
    if (twl) {
      lds_optin<k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, true>>(lds);
      hipLaunchKernelGGL((k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, true>), grid, block, lds, st, a2);
    } else {
      lds_optin<k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, false>>(lds);
      hipLaunchKernelGGL((k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, false>), grid, block, lds, st, a2);
    }
  }
  return hipGetLastError();
}

template <typename T, class P, int NT, int FB, int FC, int MS>
static hipError_t launch_p3_ms(bool analysis, const FftArgs& a, hipStream_t st) {
  const size_t lds = (size_t)(FC * P::IP + P::ntw) * sizeof(cx<T>);
  int per_cu = (int)(kMaxLds / lds);
  const int by_waves = 2048 / NT;
  per_cu = per_cu < by_waves ? per_cu : by_waves;
  per_cu = per_cu < 1 ? 1 : per_cu;
  int nwg = g_num_cu * per_cu;
  nwg = nwg < a.nitems ? nwg : a.nitems;
  const dim3 grid(nwg), block(NT);
  if (analysis) {
    lds_optin<k_zonal_analysis_p3<T, P, NT, FB, FC, MS>>(lds);
    hipLaunchKernelGGL((k_zonal_analysis_p3<T, P, NT, FB, FC, MS>), grid, block, lds, st, a);
  } else {
    lds_optin<k_zonal_synthesis_p3<T, P, NT, FB, FC, MS>>(lds);
    hipLaunchKernelGGL((k_zonal_synthesis_p3<T, P, NT, FB, FC, MS>), grid, block, lds, st, a);
  }
  return hipGetLastError();
}

template <typename T, class P, int NT, int FB, int FC>
static hipError_t launch_p3(bool analysis, const FftArgs& a, int maxN, hipStream_t st) {
  static_assert(FB % FC == 0, "field rounds");
  constexpr int MSMAX = ((P::I + 1) / 2 + NT - 1) / NT;  // N + 1 <= (I + 1) / 2
  static_assert(MSMAX <= 3, "wavenumbers per thread");
  const int nm = maxN + 1;
  if constexpr (MSMAX >= 3)
    if (nm > 2 * NT) return launch_p3_ms<T, P, NT, FB, FC, 3>(analysis, a, st);
  if constexpr (MSMAX >= 2)
    if (nm > NT) return launch_p3_ms<T, P, NT, FB, FC, 2>(analysis, a, st);
  return launch_p3_ms<T, P, NT, FB, FC, 1>(analysis, a, st);
}

// Single-level plans whose I has a compile-time three-pass plan.
template <typename T, int FB>
static bool launch_fixed(bool analysis, const FftArgs& a, int maxN, hipStream_t st, hipError_t* err) {
  if (a.nlev != 1) return false;
  // the fixed-length kernels address the workspace with 32-bit offsets
  // from a per-wave base
  const LevelDesc& L = a.lev[0];
  if (!zonal_offsets_fit(L.wplane, sizeof(T))) return false;
  constexpr bool dbl = sizeof(T) == 8;
  switch (a.lev[0].I) {
    case 2880:
      if constexpr (FB > 8) return false;  // several wavenumbers per thread: 8 fields at most
      else {
        // two fields per round (four spill registers and ~5 % more time with
        // four); 512 threads: 768- and 1024-thread workgroups (one per CU,
        // more waves) spill and measured 10-50 % slower at T959
        *err = launch_p3<T, Plan3<2880, 12, 15>, 512, FB, 2>(analysis, a, maxN, st);
        return true;
      }
    case 1440:
      *err = launch_p3<T, Plan3<1440, 9, 10>, 512, FB, dbl ? 2 : 4>(analysis, a, maxN, st);
      return true;
    case 480:
      *err = launch_p3<T, Plan3<480, 6, 5>, 256, FB, dbl ? 4 : 8>(analysis, a, maxN, st);
      return true;
    case 1920:
      if constexpr (FB > 8) return false;
      else {
        *err = launch_p3<T, Plan3<1920, 12, 10>, 512, FB, dbl ? 2 : 4>(analysis, a, maxN, st);
        return true;
      }
    case 960:
      if constexpr (FB > 8) return false;
      else {
        *err = launch_p3<T, Plan3<960, 6, 10>, 512, FB, dbl ? 2 : 4>(analysis, a, maxN, st);
        return true;
      }
    case 1600:
      if constexpr (FB > 8) return false;
      else {
        *err = launch_p3<T, Plan3<1600, 10, 10>, 512, FB, dbl ? 2 : 4>(analysis, a, maxN, st);
        return true;
      }
    case 800:
      if constexpr (FB > 8) return false;
      else {
        *err = launch_p3<T, Plan3<800, 5, 10>, 256, FB, 4>(analysis, a, maxN, st);
        return true;
      }
    case 400:
      if constexpr (FB > 8) return false;
      else {
        *err = launch_p3<T, Plan3<400, 5, 5>, 256, FB, dbl ? 4 : 8>(analysis, a, maxN, st);
        return true;
      }
    default:
      return false;
  }
}

// compute units of the current device (persistent grids are sized by it)
static void ensure_num_cu() {
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        g_num_cu <= 0)
      g_num_cu = 256;
  }
}

template <typename T, int FB, int FC>
static hipError_t launch_generic(bool analysis, const FftArgs& a, int maxN, hipStream_t st) {
  int maxI = 0;
  for (int l = 0; l < a.nlev; ++l) maxI = a.lev[l].I > maxI ? a.lev[l].I : maxI;
  const int nm = maxN + 1;
  if (maxI <= 1024 && nm <= 512) {
    if (nm <= 256) return launch_cfg<T, 256, FB, FC, 1, 1024>(analysis, a, maxI, st);
    return launch_cfg<T, 256, FB, FC, 2, 1024>(analysis, a, maxI, st);
  }
  if (maxI <= 2048 && nm <= 1024) {
    if (nm <= 512) return launch_cfg<T, 512, FB, FC, 1, 2048>(analysis, a, maxI, st);
    return launch_cfg<T, 512, FB, FC, 2, 2048>(analysis, a, maxI, st);
  }
  // one 512-thread workgroup per CU: 256 registers per lane, no spilling
  if (nm <= 512) return launch_cfg<T, 512, FB, FC, 1, 4096>(analysis, a, maxI, st);
  if (nm <= 1024) return launch_cfg<T, 512, FB, FC, 2, 4096>(analysis, a, maxI, st);
  if (nm <= 1536) return launch_cfg<T, 512, FB, FC, 3, 4096>(analysis, a, maxI, st);
  return launch_cfg<T, 512, FB, FC, 4, 4096>(analysis, a, maxI, st);
}

// The configurations of the one-launch kernel for one element type (zk =
// index into C1600, C800, C400, CRt) and its two instantiations.
template <typename T>
struct ZLevels {
  static constexpr bool dbl = sizeof(T) == 8;
  static constexpr int NT = 512;
  using C1600 = ZP3<Plan3<1600, 10, 10>, dbl ? 2 : 4, 2>;
  using C800 = ZP3<Plan3<800, 5, 10>, 4, 1>;
  using C400 = ZP3<Plan3<400, 5, 5>, dbl ? 4 : 8, 1>;
  using CRt = ZRt<dbl ? 1 : 4, 1, 1024>;
  template <int FB, bool ANA>
  static constexpr auto kernel() {
    return &k_zonal_levels<T, NT, FB, ANA, C1600, C800, C400, CRt>;
  }
};

// Multi-level plans whose levels all have I = 1600, 800 or 400 (three-pass
// plans) or I <= 1024 (runtime radices), and at least two launches' worth of
// lengths: one launch of k_zonal_levels.  Returns false (nothing launched)
// for other plans.
template <typename T, int FB>
static bool launch_levels_one(bool analysis, const FftArgs& a, hipStream_t st, hipError_t* err) {
  constexpr int NT = ZLevels<T>::NT;
  using C1600 = typename ZLevels<T>::C1600;
  using C800 = typename ZLevels<T>::C800;
  using C400 = typename ZLevels<T>::C400;
  using CRt = typename ZLevels<T>::CRt;
  if (a.nlev < 2 || a.fb != FB) return false;
  FftArgs b = a;
  size_t lds = 0;
  int maxIrt = 0, kinds = 0;
  for (int l = 0; l < a.nlev; ++l) {
    const LevelDesc& L = a.lev[l];
    int k;
    size_t need = 0;
    if (L.I == 1600 || L.I == 800 || L.I == 400) {
      // the three-pass kernels address the workspace with 32-bit offsets
      // from a per-wave base
      if (!zonal_offsets_fit(L.wplane, sizeof(T))) return false;
      k = L.I == 1600 ? 0 : L.I == 800 ? 1 : 2;
      need = k == 0 ? C1600::template lds<T>() : k == 1 ? C800::template lds<T>() : C400::template lds<T>();
    } else {
      if (L.I > CRt::maxi || L.N + 1 > CRt::ms * NT) return false;
      k = 3;
      maxIrt = L.I > maxIrt ? L.I : maxIrt;
    }
    kinds |= 1 << k;
    b.lev[l].zk = k;
    lds = need > lds ? need : lds;
  }
  // one runtime-radix launch or one length alone gains nothing
  if (__builtin_popcount(kinds) < 2) return false;
  if (maxIrt) {
    b.tw_lds = (CRt::fc * maxIrt + 1) & ~1;
    const size_t rt = (size_t)(b.tw_lds + maxIrt) * sizeof(cx<T>);
    lds = rt > lds ? rt : lds;
  }
  int per_cu = (int)(kMaxLds / lds);
  const int by_waves = 2048 / NT;
  per_cu = per_cu < by_waves ? per_cu : by_waves;
  per_cu = per_cu < 1 ? 1 : per_cu;
  int nwg = g_num_cu * per_cu;
  nwg = nwg < a.nitems ? nwg : a.nitems;
  const dim3 grid(nwg), block(NT);
  if (analysis) {
    constexpr auto K = ZLevels<T>::template kernel<FB, true>();
    lds_optin<K>(lds);
    hipLaunchKernelGGL(K, grid, block, lds, st, b);
  } else {
    constexpr auto K = ZLevels<T>::template kernel<FB, false>();
    lds_optin<K>(lds);
    hipLaunchKernelGGL(K, grid, block, lds, st, b);
  }
  *err = hipGetLastError();
  return true;
}

// Multi-level plans: one launch of k_zonal_levels where every level fits
// it (and FftArgs::one_launch asks for it); otherwise each level whose I has a compile-time three-pass plan gets
// a launch of its own (one level per argument block, its items renumbered
// from 0), and the other levels share one launch of the runtime-radix
// kernel.  All launches go to the same stream, and the levels
// write disjoint parts of the output.
template <typename T, int FB, int FC>
static hipError_t launch_levels(bool analysis, const FftArgs& a, hipStream_t st) {
  hipError_t e1 = hipSuccess;
  if (a.one_launch && launch_levels_one<T, FB>(analysis, a, st, &e1)) return e1;
  FftArgs rest = a;
  rest.nlev = 0;
  rest.nitems = 0;
  int rest_maxN = 0;
  for (int l = 0; l < a.nlev; ++l) {
    FftArgs one = a;
    one.nlev = 1;
    one.lev[0] = a.lev[l];
    one.lev[0].fft_item0 = 0;
    one.nitems = a.lev[l].Jh * a.lev[l].nfb;
    hipError_t e = hipSuccess;
    if (launch_fixed<T, FB>(analysis, one, a.lev[l].N, st, &e)) {
      if (e != hipSuccess) return e;
      continue;
    }
    rest.lev[rest.nlev] = a.lev[l];
    rest.lev[rest.nlev].fft_item0 = rest.nitems;
    rest.nitems += one.nitems;
    rest.nlev += 1;
    rest_maxN = a.lev[l].N > rest_maxN ? a.lev[l].N : rest_maxN;
  }
  if (rest.nlev == 0) return hipSuccess;
  return launch_generic<T, FB, FC>(analysis, rest, rest_maxN, st);
}

template <typename T, int FB, int FC>
static hipError_t launch_zonal_t(bool analysis, const FftArgs& a, int maxN, hipStream_t st) {
  ensure_num_cu();
  if (a.nlev > 1) return launch_levels<T, FB, FC>(analysis, a, st);
  hipError_t err = hipSuccess;
  if (launch_fixed<T, FB>(analysis, a, maxN, st, &err)) return err;
  return launch_generic<T, FB, FC>(analysis, a, maxN, st);
}

int zonal_one_launch_spills(int form, bool analysis) {
  const void* k = nullptr;
  if (form == SHT_FORM_FP64)
    k = analysis ? reinterpret_cast<const void*>(ZLevels<double>::kernel<4, true>())
                 : reinterpret_cast<const void*>(ZLevels<double>::kernel<4, false>());
  else
    k = analysis ? reinterpret_cast<const void*>(ZLevels<float>::kernel<8, true>())
                 : reinterpret_cast<const void*>(ZLevels<float>::kernel<8, false>());
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, k) != hipSuccess) return 1;
  return fa.localSizeBytes > 0 ? 1 : 0;
}

int zonal_fields_per_block(int form, int nlev, int N, int J, int I, int F) {
  if (form == SHT_FORM_FP64) return 4;
  // wide items halve the item count: only where plenty remain for 256 CUs
  const long long items16 = (long long)((J + 1) / 2) * ((F + 15) / 16);
  if (nlev == 1 && items16 >= 4096 && ((I == 1440 && N + 1 <= 512) || (I == 480 && N + 1 <= 256))) return 16;
  return 8;
}

int launch_zonal(int form, bool analysis, const FftArgs& a, int maxN, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the kernels' item width must match every level's analysis column block
  const int fb = form == SHT_FORM_FP64 ? 4 : (a.fb == 16 ? 16 : 8);
  for (int l = 0; l < a.nlev; ++l)
    if ((1 << a.lev[l].wsh) != (2 * fb < 16 ? 2 * fb : 16)) return (int)hipErrorInvalidValue;
  if (form == SHT_FORM_FP64) return (int)launch_zonal_t<double, 4, 1>(analysis, a, maxN, st);
  if (a.fb == 16) {
    ensure_num_cu();
    hipError_t err = hipErrorInvalidValue;
    if (!launch_fixed<float, 16>(analysis, a, maxN, st, &err)) return (int)hipErrorInvalidValue;
    return (int)err;
  }
  return (int)launch_zonal_t<float, 8, 4>(analysis, a, maxN, st);
}

}  // namespace sht
