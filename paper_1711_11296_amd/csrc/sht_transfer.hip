// Transfers between truncations and between nested grids, the building
// blocks of the two-grid cycle of App. C: spectral restriction and
// prolongation are a re-truncation of the triangular spectrum (coefficients
// with n above the target truncation dropped, those above the source
// truncation set to zero); grid restriction is injection, the nested rows
// and columns of the finer grid (Sec. 3.2).  Also the pointwise product of
// grids, the nonlinear terms whose aliasing Sec. 4.2 measures.  All are
// bound by HBM bandwidth.

#include <hip/hip_runtime.h>

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
