// Device-side helpers shared by the Legendre kernels (FP32/FP64 and split
// bfloat16 forms): matrix-core steps and their lane layouts, LDS transfer and
// barrier primitives, scheduling hints.
#ifndef SHT_DEVICE_H_
#define SHT_DEVICE_H_

#include <hip/hip_runtime.h>

#include <type_traits>

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

// One 16-byte piece per lane from global memory straight into LDS
// (global_load_lds_dwordx4): the wave's 64 pieces land contiguously at
// lds_base, lane l at byte 16 l; lds_base must be uniform across the wave.
// Completion is awaited with s_waitcnt vmcnt.
__device__ __forceinline__ void load_to_lds16(const void* src, void* lds_base) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
#endif
}

// Workgroup barrier for LDS hand-offs only: waits for this wave's LDS
// operations, not for its outstanding global loads (which __syncthreads'
// fence would also drain, defeating loads issued blocks ahead).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Instruction-order hint for a K-block body (scheduling groups of the
// compiler, no effect on results): PRE LDS reads first, then ROUNDS times
// PER MFMAs followed by one LDS read, then TAIL MFMAs.  It keeps the LDS
// reads of a k-step ahead of the MFMAs that consume them, which the default
// schedule (each read right before its first use) does not.
template <int PRE, int ROUNDS, int PER, int TAIL>
__device__ __forceinline__ void mfma_lds_pipeline() {
#pragma unroll
  for (int i = 0; i < PRE; ++i) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
  for (int i = 0; i < ROUNDS; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  if constexpr (TAIL > 0) __builtin_amdgcn_sched_group_barrier(0x008, TAIL, 0);
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

// 16-byte vector store into LDS at an address that is only 8-byte aligned.
template <typename T>
__device__ __forceinline__ void lds_store8(T* dst, const typename V16<T>::type& v) {
  if constexpr (sizeof(T) == 4) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    reinterpret_cast<f2*>(dst)[0] = f2{v[0], v[1]};
    reinterpret_cast<f2*>(dst)[1] = f2{v[2], v[3]};
  } else {
    *reinterpret_cast<typename V16<T>::type*>(dst) = v;
  }
}

template <auto Kernel>
static void lds_optin(size_t bytes) {
  static size_t done = 0;  // one flag per kernel instantiation
  if (bytes > 65536 && bytes > done) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    done = bytes;
  }
}

// Generated P~ (plan option otf), shared by both directions and all forms:
// the rows r = n - m of a block are produced by the three-term recurrence of
// Sec. 4.1, P~_r = A_r mu P~_{r-1} - B_r P~_{r-2}, in FP64 from the two
// stored seed rows of each 16-degree group (rows 16 gi and 16 gi + 1 of
// every latitude), one latitude per lane, and rounded once to the element
// type.  The coefficients of a group sit in lanes (gen_coef) and are
// broadcast per step (v_readlane), so the recurrence waits on no memory; a
// row at or beyond n_m has zero coefficients and therefore comes out zero,
// and so does every later row of the group.

// Lane l of a wave holds (A_r, B_r) of row r = r0 + 2 + (l % 32) of its
// group, for l % 32 < 14 and r < nm (zero otherwise); with TWO the lanes
// 32..63 belong to a second group (r0 is the lane's own group's first row).
__device__ __forceinline__ void gen_coef(const double* rec, int r0, int nm, int lane, double& cA, double& cB) {
  const int r = r0 + 2 + (lane & 31);
  const bool ok = (lane & 31) < 14 && r < nm;
  cA = ok ? rec[2 * r] : 0.0;
  cB = ok ? rec[2 * r + 1] : 0.0;
}

template <bool TWO>
__device__ __forceinline__ double gen_bcast(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  const unsigned long long b0 = ((unsigned long long)(unsigned)__builtin_amdgcn_readlane(hi, l) << 32) |
                                (unsigned)__builtin_amdgcn_readlane(lo, l);
  if constexpr (!TWO) {
    return __builtin_bit_cast(double, b0);
  } else {
    const unsigned long long b1 = ((unsigned long long)(unsigned)__builtin_amdgcn_readlane(hi, l + 32) << 32) |
                                  (unsigned)__builtin_amdgcn_readlane(lo, l + 32);
    return __builtin_bit_cast(double, (__lane_id() < 32) ? b0 : b1);
  }
}

// The 16 rows r0 .. r0 + 15 at one latitude: st(s, value) receives row r0 + s.
template <bool TWO, class Store>
__device__ __forceinline__ void gen_rows16(double cA, double cB, int r0, int nm, double mu, double x0, double x1,
                                           Store st) {
  x0 = r0 < nm ? x0 : 0.0;
  x1 = r0 + 1 < nm ? x1 : 0.0;
  st(0, x0);
  st(1, x1);
#pragma unroll
  for (int s = 2; s < 16; ++s) {
    const double x2 = gen_bcast<TWO>(cA, s - 2) * mu * x1 - gen_bcast<TWO>(cB, s - 2) * x0;
    st(s, x2);
    x0 = x1;
    x1 = x2;
  }
}

// Split-bfloat16 Legendre kernels (sht_legendre_bf16.hip).
hipError_t launch_legendre_bf16(bool analysis, const GemmArgs& g, int ncb, bool gen, hipStream_t st);

}  // namespace sht

#endif  // SHT_DEVICE_H_
