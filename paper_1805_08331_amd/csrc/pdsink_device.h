// Device-side building blocks shared by the pdsink kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdsink {

constexpr int WG = 256;             // threads per workgroup (4 wave64)
constexpr int NWAVE = WG / 64;
constexpr int NEG = -(1 << 24);     // log2 scale of an empty row/column: every entry built from it underflows to 0
constexpr int BIG = (1 << 24);
constexpr int QNONE = -(1 << 30);   // "cell not in the support" marker for the per-cell log2 estimates

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// x * 2^e, exact while the result is a normal float; |e| clamped so the
// hardware sees a sane shift (results beyond it are 0 or inf anyway).
__device__ __forceinline__ float ldx(float x, int e) {
  e = e < -400 ? -400 : (e > 400 ? 400 : e);
  return __builtin_amdgcn_ldexpf(x, e);
}
__device__ __forceinline__ double ldxd(double x, int e) {
  e = e < -3000 ? -3000 : (e > 3000 ? 3000 : e);
  return __builtin_amdgcn_ldexp(x, e);
}
// floor(log2 x) for finite x > 0 (exact: the exponent field).
__device__ __forceinline__ int ilog2f(float x) { return __builtin_amdgcn_frexp_expf(x) - 1; }

// Wait for the last MFMA of a K-loop to retire before its accumulators are
// read.  Measured on gfx950: with only the compiler-inserted wait states, the
// ds_write of the last accumulator register of v_mfma_f32_32x32x2_f32 read a
// value that lacked the final MFMA's contribution.  The scheduling barriers
// keep the MFMA before, and every consumer after, the explicit wait.
__device__ __forceinline__ void mfma_drain() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 15\n\ts_nop 15\n\ts_nop 15\n\ts_nop 15" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// Sum over a workgroup of NW waves, same fixed order on every call (deterministic).
template <int NW = NWAVE>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll 4
  for (int w = 0; w < NW; ++w) t += red[w];
  return t;
}
template <int NW = NWAVE>
__device__ __forceinline__ int block_max(int v, int* red) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = red[0];
#pragma unroll 4
  for (int w = 1; w < NW; ++w) t = max(t, red[w]);
  return t;
}

// A positive value s * 2^e kept as (exponent, double mantissa) so that sums of
// terms whose magnitudes span far beyond the double range stay exact in shape.
struct ESum {
  int e;
  double s;
};
__device__ __forceinline__ ESum esum_add(ESum a, ESum b) {
  if (a.s == 0.0) return b;
  if (b.s == 0.0) return a;
  const int e = max(a.e, b.e);
  return ESum{e, ldxd(a.s, a.e - e) + ldxd(b.s, b.e - e)};
}
// Sum over the wave: the largest exponent first, then one scaled sum, so the
// shuffles carry plain doubles.  (A zero term has exponent NEG and vanishes.)
__device__ __forceinline__ ESum wave_esum(ESum v) {
  int e = v.s != 0.0 ? v.e : -(1 << 24);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e = max(e, __shfl_xor(e, o));
  double x = v.s != 0.0 ? ldxd(v.s, v.e - e) : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return ESum{e, x};
}
template <int NW = NWAVE>
__device__ __forceinline__ ESum block_esum(ESum v, int* rede, double* reds) {
  v = wave_esum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    rede[threadIdx.x >> 6] = v.e;
    reds[threadIdx.x >> 6] = v.s;
  }
  __syncthreads();
  ESum t{rede[0], reds[0]};
#pragma unroll 2
  for (int w = 1; w < NW; ++w) t = esum_add(t, ESum{rede[w], reds[w]});
  return t;
}

}  // namespace pdsink
