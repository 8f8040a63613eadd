// Transfers between truncations and between nested grids, the building
// blocks of the two-grid cycle of App. C: spectral restriction and
// prolongation are a re-truncation of the triangular spectrum (coefficients
// with n above the target truncation dropped, those above the source
// truncation set to zero); grid restriction is injection, the nested rows
// and columns of the finer grid (Sec. 3.2).  Also the pointwise product of
// grids, the nonlinear terms whose aliasing Sec. 4.2 measures, and the two
// pieces of the residual of the elliptic problem of App. C with a
// variable-coefficient Laplacian: the spectral Laplacian (Y_n^m is an
// eigenfunction with eigenvalue -n(n+1) on the unit sphere) and the fused
// grid update r = x - alpha * kappa * y - f.  All are bound by HBM bandwidth.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "sht_internal.h"

namespace sht {

// One block per (field, wavenumber m) run of the output triangle; threads
// over n.  Complex pairs move as one 8- or 16-byte element.
template <typename T>
__global__ __launch_bounds__(256) void k_retruncate(int Nin, int Nout, int F, const T* in, T* out) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  const int m = blockIdx.x, f = blockIdx.y;
  const long long ncin = (long long)(Nin + 1) * (Nin + 2) / 2;
  const long long ncout = (long long)(Nout + 1) * (Nout + 2) / 2;
  const long long bo = (long long)f * ncout + (long long)m * (2 * Nout + 3 - m) / 2 - m;
  const long long bi = (long long)f * ncin + (long long)m * (2 * Nin + 3 - m) / 2 - m;
  const T2* src = reinterpret_cast<const T2*>(in);
  T2* dst = reinterpret_cast<T2*>(out);
  for (int n = m + (int)threadIdx.x; n <= Nout; n += 256)
    dst[bo + n] = (m <= Nin && n <= Nin) ? src[bi + n] : T2{(T)0, (T)0};
}

// One block row per (field, coarse row); threads over coarse columns.
template <typename T>
__global__ __launch_bounds__(256) void k_inject(int Jf, int If, int Jc, int Ic, int rs, int r0, int cs,
                                                const T* fine, T* coarse) {
  const int jc = blockIdx.x, f = blockIdx.y;
  const T* src = fine + ((long long)f * Jf + (long long)r0 + (long long)rs * jc) * If;
  T* dst = coarse + ((long long)f * Jc + jc) * Ic;
  for (int i = threadIdx.x; i < Ic; i += 256) dst[i] = src[(long long)cs * i];
}

// Zero a span of 16-byte units in each of nplanes equally spaced planes:
// units [first, first + len) of plane p start at base + p * pitch.  Used to
// clear the padding rows of a workspace that other calls share.
__global__ __launch_bounds__(256) void k_clear_span(uint4* base, long long nplanes, long long pitch, long long first,
                                                    long long len) {
  const long long total = nplanes * len;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
    const long long p = i / len, k = i - p * len;
    base[p * pitch + first + k] = uint4{0u, 0u, 0u, 0u};
  }
}

// out = a * b elementwise, four elements per thread (n a multiple of 4
// handled by the vector body, the tail by the first threads)
template <typename T>
__global__ __launch_bounds__(256) void k_product(long long n, const T* a, const T* b, T* out) {
  typedef T T4 __attribute__((ext_vector_type(4)));
  const long long n4 = n / 4;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n4; i += (long long)gridDim.x * 256) {
    const T4 x = reinterpret_cast<const T4*>(a)[i], y = reinterpret_cast<const T4*>(b)[i];
    reinterpret_cast<T4*>(out)[i] = x * y;
  }
  const long long t = 4 * n4 + blockIdx.x * 256LL + threadIdx.x;
  if (blockIdx.x == 0 && t < n) out[t] = a[t] * b[t];
}

// out(m, n) = c_n * in(m, n), c_n = -scale * n (n + 1) rounded once to T;
// one block per (field, wavenumber m), threads over n.
template <typename T>
__global__ __launch_bounds__(256) void k_laplacian(int N, double scale, const T* in, T* out) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  const int m = blockIdx.x, f = blockIdx.y;
  const long long nc = (long long)(N + 1) * (N + 2) / 2;
  const long long b = (long long)f * nc + (long long)m * (2 * N + 3 - m) / 2 - m;
  const T2* src = reinterpret_cast<const T2*>(in);
  T2* dst = reinterpret_cast<T2*>(out);
  for (int n = m + (int)threadIdx.x; n <= N; n += 256) {
    const T c = (T)(-scale * ((double)n * (double)(n + 1)));
    const T2 v = src[b + n];
    dst[b + n] = T2{c * v.x, c * v.y};
  }
}

// r = x - alpha * kappa * y - f elementwise, kappa (one grid of n_per
// values) shared by the nf fields; blocks over (chunk of a field, field),
// 16-byte vectors when n_per is a multiple of the vector length, so kappa
// is indexed without a division and read from L2 after the first field
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_residual(long long n_per, long long nf, T alpha, const T* x, const T* kappa,
                                                  const T* y, const T* f, T* r) {
  constexpr int E = VEC ? 16 / (int)sizeof(T) : 1;
  typedef T TV __attribute__((ext_vector_type(E)));
  const long long nv = n_per / E;
  for (long long fl = blockIdx.y; fl < nf; fl += gridDim.y) {
    const long long off = fl * nv;
    const TV* xv = reinterpret_cast<const TV*>(x) + off;
    const TV* yv = reinterpret_cast<const TV*>(y) + off;
    const TV* fv = reinterpret_cast<const TV*>(f) + off;
    TV* rv = reinterpret_cast<TV*>(r) + off;
    const TV* kv = reinterpret_cast<const TV*>(kappa);
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < nv; i += (long long)gridDim.x * 256)
      rv[i] = xv[i] - alpha * kv[i] * yv[i] - fv[i];
  }
}

int launch_laplacian(int N, int F, double scale, bool dbl, const void* in, void* out, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid(N + 1, F), block(256);
  if (dbl)
    hipLaunchKernelGGL(k_laplacian<double>, grid, block, 0, st, N, scale, static_cast<const double*>(in),
                       static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_laplacian<float>, grid, block, 0, st, N, scale, static_cast<const float*>(in),
                       static_cast<float*>(out));
  return (int)hipGetLastError();
}

int launch_residual(long long n, long long n_per, double alpha, bool dbl, const void* x, const void* kappa,
                    const void* y, const void* f, void* r, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long nf = n / n_per;
  const int E = dbl ? 2 : 4;
  // 16-byte vectors where every field starts 16-byte aligned; else scalars
  // (element-aligned slices of a larger buffer, e.g. one level of a
  // multi-level plan's grids)
  auto a16 = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  const bool vec = n_per % E == 0 && a16(x) && a16(kappa) && a16(y) && a16(f) && a16(r);
  long long bx = (n_per / (vec ? E : 1) + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 4096 ? 4096 : bx);
  const long long by = nf > 65535 ? 65535 : nf;
  const dim3 grid((unsigned)bx, (unsigned)by), block(256);
  if (dbl) {
    const double* a[4] = {static_cast<const double*>(x), static_cast<const double*>(kappa),
                          static_cast<const double*>(y), static_cast<const double*>(f)};
    if (vec)
      hipLaunchKernelGGL((k_residual<double, true>), grid, block, 0, st, n_per, nf, alpha, a[0], a[1], a[2], a[3],
                         static_cast<double*>(r));
    else
      hipLaunchKernelGGL((k_residual<double, false>), grid, block, 0, st, n_per, nf, alpha, a[0], a[1], a[2], a[3],
                         static_cast<double*>(r));
  } else {
    const float* a[4] = {static_cast<const float*>(x), static_cast<const float*>(kappa),
                         static_cast<const float*>(y), static_cast<const float*>(f)};
    if (vec)
      hipLaunchKernelGGL((k_residual<float, true>), grid, block, 0, st, n_per, nf, (float)alpha, a[0], a[1], a[2],
                         a[3], static_cast<float*>(r));
    else
      hipLaunchKernelGGL((k_residual<float, false>), grid, block, 0, st, n_per, nf, (float)alpha, a[0], a[1], a[2],
                         a[3], static_cast<float*>(r));
  }
  return (int)hipGetLastError();
}

int launch_clear_span(void* base, long long nplanes, long long pitch16, long long first16, long long len16,
                      void* stream) {
  const long long total = nplanes * len16;
  if (total <= 0) return (int)hipSuccess;
  const long long blocks = std::min<long long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_clear_span, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<uint4*>(base), nplanes, pitch16, first16, len16);
  return (int)hipGetLastError();
}

int launch_product(long long n, bool dbl, const void* a, const void* b, void* out, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  long long blocks = (n / 4 + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
  if (dbl)
    hipLaunchKernelGGL(k_product<double>, dim3((unsigned)blocks), dim3(256), 0, st, n, static_cast<const double*>(a),
                       static_cast<const double*>(b), static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_product<float>, dim3((unsigned)blocks), dim3(256), 0, st, n, static_cast<const float*>(a),
                       static_cast<const float*>(b), static_cast<float*>(out));
  return (int)hipGetLastError();
}

int launch_retruncate(int Nin, int Nout, int F, bool dbl, const void* in, void* out, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid(Nout + 1, F), block(256);
  if (dbl)
    hipLaunchKernelGGL(k_retruncate<double>, grid, block, 0, st, Nin, Nout, F, static_cast<const double*>(in),
                       static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_retruncate<float>, grid, block, 0, st, Nin, Nout, F, static_cast<const float*>(in),
                       static_cast<float*>(out));
  return (int)hipGetLastError();
}

int launch_inject(int Jf, int If, int Jc, int Ic, int F, int rs, int r0, int cs, bool dbl, const void* fine,
                  void* coarse, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid(Jc, F), block(256);
  if (dbl)
    hipLaunchKernelGGL(k_inject<double>, grid, block, 0, st, Jf, If, Jc, Ic, rs, r0, cs,
                       static_cast<const double*>(fine), static_cast<double*>(coarse));
  else
    hipLaunchKernelGGL(k_inject<float>, grid, block, 0, st, Jf, If, Jc, Ic, rs, r0, cs,
                       static_cast<const float*>(fine), static_cast<float*>(coarse));
  return (int)hipGetLastError();
}

}  // namespace sht
