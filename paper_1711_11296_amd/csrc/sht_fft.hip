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
// parity, row) instead of one isolated complex value.
//
// Workspace layout (per level): ws[m][parity][j][c], j < Kp (rows >= ceil(J/2)
// stay zero), c = 2*field + {re, im} < Cp.

#include <hip/hip_runtime.h>

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

// q = floor(j / d) for 0 <= j < 2^13 and 2 <= d <= 4096, with
// magic = floor((2^32 - 1) / d) + 1 (exhaustively checked over that range).
__device__ __forceinline__ int fastdiv(int j, unsigned magic) {
  return (int)__umulhi((unsigned)j, magic);
}

// One Stockham pass of radix R over FC sequences of length I that lie one
// after the other in LDS, in place: every thread first loads and transforms
// all its butterflies, then (after a barrier) stores them.  Ns is the product
// of the radices of the earlier passes.  Butterfly u covers sequence
// f = u / (I/R) (FC is 1 or 2) and position j = u mod (I/R).
template <typename T, int NT, int FC, int MAXI, int R>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int I, int Ns, int twstep,
                                              unsigned magic, const cx<T>* __restrict__ tw) {
  constexpr int BPT = (FC * MAXI / R + NT - 1) / NT;
  const int nb = twstep * Ns;  // I / R
  const int tot = FC * nb;
  cx<T> v[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int u = threadIdx.x + b * NT;
    if (u < tot) {
      const int f = (FC == 2 && u >= nb) ? 1 : 0;
      const int j = u - f * nb;
      const cx<T>* src = buf + f * I + j;
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = src[t * nb];
      if (Ns > 1) {
        const int k = j - fastdiv(j, magic) * Ns;
#pragma unroll
        for (int t = 1; t < R; ++t) v[b][t] = cmul(v[b][t], tw[t * k * twstep]);
      }
      Dft<T, R>::run(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int u = threadIdx.x + b * NT;
    if (u < tot) {
      const int f = (FC == 2 && u >= nb) ? 1 : 0;
      const int j = u - f * nb;
      int q = j, k = 0;
      if (Ns > 1) {
        q = fastdiv(j, magic);
        k = j - q * Ns;
      }
      cx<T>* dst = buf + f * I + q * Ns * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) dst[t * Ns] = v[b][t];
    }
  }
  __syncthreads();
}

// Forward complex FFTs (sign -) of the FC sequences in buf, natural order in
// and out.  Every thread of the block must call it.
template <typename T, int NT, int FC, int MAXI>
__device__ void fft_lds(cx<T>* buf, const LevelDesc& L, const cx<T>* tw) {
  for (int p = 0; p < L.nrad; ++p) {
    const int R = L.rad[p], Ns = L.pns[p], tws = L.ptw[p];
    const unsigned mg = L.pmag[p];
    if (R == 4)
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

// ---------------------------------------------------------------------------
// analysis: grid [F][J][I] -> workspace S/A
// FB fields per workgroup, FC of them transformed together; the rows of the
// next FC fields are prefetched into registers while the current ones are
// transformed.  Twiddles are staged in LDS when TWL is set.
// ---------------------------------------------------------------------------
template <typename T, int NT, int FB, int FC, int MS, int MAXI, bool TWL>
__global__ __launch_bounds__(NT) void k_zonal_analysis(const FftArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int item = blockIdx.x;
  if (item >= a.nitems) return;
  const int l = level_of(a, item);
  const LevelDesc& L = a.lev[l];
  const int local = item - L.fft_item0;
  const int jp = local / L.nfb;
  const int fb = local - jp * L.nfb;
  const int I = L.I, J = L.J, N = L.N;
  const bool eq = (J & 1) && (jp == (J >> 1));
  const int js = J - 1 - jp;
  const T* grid = static_cast<const T*>(a.src) + L.grid_off;
  T* ws = static_cast<T*>(a.dst) + L.ws_off;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const cx<T>* tw = static_cast<const cx<T>*>(L.tw);
  if (TWL) {
    cx<T>* twl = buf + FC * I;
    for (int i = threadIdx.x; i < I; i += NT) twl[i] = tw[i];
    tw = twl;
  }

  T rscale = (T)1;
  if (a.use_w) rscale = (T)L.wrow[jp];
  if (a.use_inv_I) rscale = (T)((double)rscale / (double)I);
  const T msc = (T)a.mscale;

  constexpr int LPT = (MAXI + NT - 1) / NT;
  T pn[FC][LPT], ps[FC][LPT];
  auto load_rows = [&](int rd) {
#pragma unroll
    for (int fc = 0; fc < FC; ++fc) {
      const int f = fb * FB + rd * FC + fc;
      const bool valid = f < L.F;
      const T* rn = grid + ((long long)f * J + jp) * I;
      const T* rs = grid + ((long long)f * J + js) * I;
#pragma unroll
      for (int e = 0; e < LPT; ++e) {
        const int i = threadIdx.x + e * NT;
        pn[fc][e] = (valid && i < I) ? rn[i] : (T)0;
        ps[fc][e] = (valid && !eq && i < I) ? rs[i] : (T)0;
      }
    }
  };

  cx<T> stS[MS][FB], stA[MS][FB];
  load_rows(0);
#pragma unroll
  for (int rd = 0; rd < FB / FC; ++rd) {
#pragma unroll
    for (int fc = 0; fc < FC; ++fc)
#pragma unroll
      for (int e = 0; e < LPT; ++e) {
        const int i = threadIdx.x + e * NT;
        if (i < I) buf[fc * I + i] = cx<T>{pn[fc][e], ps[fc][e]};
      }
    __syncthreads();
    if (rd + 1 < FB / FC) load_rows(rd + 1);
    fft_lds<T, NT, FC, MAXI>(buf, L, tw);
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int m = threadIdx.x + s * NT;
#pragma unroll
      for (int fc = 0; fc < FC; ++fc) {
        cx<T> S = {(T)0, (T)0}, A = {(T)0, (T)0};
        if (m <= N) {
          const cx<T> P = buf[fc * I + m];
          cx<T> Q = buf[fc * I + (m == 0 ? 0 : I - m)];
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
          if (eq) A = cx<T>{(T)0, (T)0};
        }
        stS[s][rd * FC + fc] = S;
        stA[s][rd * FC + fc] = A;
      }
    }
    __syncthreads();
  }

  const long long Cp = L.Cp;
  const long long plane = (long long)L.Kp * Cp;
#pragma unroll
  for (int s = 0; s < MS; ++s) {
    const int m = threadIdx.x + s * NT;
    if (m <= N) {
      T* dS = ws + (2LL * m) * plane + (long long)jp * Cp + 2 * fb * FB;
      store_run<T, FB>(dS, stS[s]);
      store_run<T, FB>(dS + plane, stA[s]);
    }
  }
}

// ---------------------------------------------------------------------------
// synthesis: workspace S/A -> grid [F][J][I]
// ---------------------------------------------------------------------------
template <typename T, int NT, int FB, int FC, int MS, int MAXI, bool TWL>
__global__ __launch_bounds__(NT) void k_zonal_synthesis(const FftArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int item = blockIdx.x;
  if (item >= a.nitems) return;
  const int l = level_of(a, item);
  const LevelDesc& L = a.lev[l];
  const int local = item - L.fft_item0;
  const int jp = local / L.nfb;
  const int fb = local - jp * L.nfb;
  const int I = L.I, J = L.J, N = L.N;
  const bool eq = (J & 1) && (jp == (J >> 1));
  const int js = J - 1 - jp;
  const T* ws = static_cast<const T*>(a.src) + L.ws_off;
  T* grid = static_cast<T*>(a.dst) + L.grid_off;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const cx<T>* tw = static_cast<const cx<T>*>(L.tw);
  if (TWL) {
    cx<T>* twl = buf + FC * I;
    for (int i = threadIdx.x; i < I; i += NT) twl[i] = tw[i];
    tw = twl;
  }

  T rscale = (T)1;
  if (a.use_w) rscale = (T)L.wrow[jp];
  if (a.use_inv_I) rscale = (T)((double)rscale / (double)I);
  const T msc = (T)a.mscale;

  const long long Cp = L.Cp;
  const long long plane = (long long)L.Kp * Cp;
  cx<T> stS[MS][FB], stA[MS][FB];
#pragma unroll
  for (int s = 0; s < MS; ++s) {
    const int m = threadIdx.x + s * NT;
    if (m <= N) {
      const T* sS = ws + (2LL * m) * plane + (long long)jp * Cp + 2 * fb * FB;
      load_run<T, FB>(sS, stS[s]);
      load_run<T, FB>(sS + plane, stA[s]);
    } else {
#pragma unroll
      for (int q = 0; q < FB; ++q) stS[s][q] = stA[s][q] = cx<T>{(T)0, (T)0};
    }
  }

#pragma unroll
  for (int rd = 0; rd < FB / FC; ++rd) {
#pragma unroll
    for (int fc = 0; fc < FC; ++fc) {
      cx<T>* bf = buf + fc * I;
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
          // the buffer holds conj(Z): the forward FFT of conj(Z) is the
          // conjugate of the inverse transform of Z, with
          // Z^m = Xn + i Xs and Z^{I-m} = conj(Xn) + i conj(Xs)
          bf[m] = cx<T>{Xn.x - Xs.y, -(Xn.y + Xs.x)};
          if (m > 0) bf[I - m] = cx<T>{Xn.x + Xs.y, Xn.y - Xs.x};
        }
      }
    }
    __syncthreads();
    fft_lds<T, NT, FC, MAXI>(buf, L, tw);
#pragma unroll
    for (int fc = 0; fc < FC; ++fc) {
      const int f = fb * FB + rd * FC + fc;
      if (f < L.F) {
        const cx<T>* bf = buf + fc * I;
        T* rn = grid + ((long long)f * J + jp) * I;
        T* rs = grid + ((long long)f * J + js) * I;
        for (int i = threadIdx.x; i < I; i += NT) {
          const cx<T> y = bf[i];
          rn[i] = rscale * y.x;
          if (!eq) rs[i] = -rscale * y.y;
        }
      }
    }
    __syncthreads();
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

template <typename T, int NT, int FB, int FC, int MS, int MAXI>
static hipError_t launch_cfg(bool analysis, const FftArgs& a, int maxI, hipStream_t st) {
  const size_t buf = (size_t)FC * maxI * sizeof(cx<T>);
  const size_t twb = (size_t)maxI * sizeof(cx<T>);
  const bool twl = buf + twb <= kMaxLds;
  const size_t lds = buf + (twl ? twb : 0);
  const dim3 grid(a.nitems), block(NT);
  if (analysis) {
    if (twl) {
      lds_optin<k_zonal_analysis<T, NT, FB, FC, MS, MAXI, true>>(lds);
      hipLaunchKernelGGL((k_zonal_analysis<T, NT, FB, FC, MS, MAXI, true>), grid, block, lds, st, a);
    } else {
      lds_optin<k_zonal_analysis<T, NT, FB, FC, MS, MAXI, false>>(lds);
      hipLaunchKernelGGL((k_zonal_analysis<T, NT, FB, FC, MS, MAXI, false>), grid, block, lds, st, a);
    }
  } else {
    if (twl) {
      lds_optin<k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, true>>(lds);
      hipLaunchKernelGGL((k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, true>), grid, block, lds, st, a);
    } else {
      lds_optin<k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, false>>(lds);
      hipLaunchKernelGGL((k_zonal_synthesis<T, NT, FB, FC, MS, MAXI, false>), grid, block, lds, st, a);
    }
  }
  return hipGetLastError();
}

template <typename T, int FB, int FC>
static hipError_t launch_zonal_t(bool analysis, const FftArgs& a, int maxN, hipStream_t st) {
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
  if (nm <= 1024) return launch_cfg<T, 1024, FB, FC, 1, 4096>(analysis, a, maxI, st);
  return launch_cfg<T, 1024, FB, FC, 2, 4096>(analysis, a, maxI, st);
}

int zonal_fields_per_block(int form) { return form == SHT_FORM_FP64 ? 4 : 8; }

int launch_zonal(int form, bool analysis, const FftArgs& a, int maxN, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (form == SHT_FORM_FP64) return (int)launch_zonal_t<double, 4, 1>(analysis, a, maxN, st);
  return (int)launch_zonal_t<float, 8, 2>(analysis, a, maxN, st);
}

}  // namespace sht
