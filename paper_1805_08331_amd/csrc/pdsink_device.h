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

// Completion record of one pair, for callers that pick up each result while
// the launch that computes it still runs (same layout as pdsink_done in the
// C header): the outputs first, then the tag, stored with release ordering
// at system scope, so that a host thread which reads the tag and then the
// other fields sees their final values.
struct DoneRec {
  double cost;
  float err;
  int status;
  int it[2];
  unsigned tag;
  unsigned reserved;
};
static_assert(sizeof(DoneRec) == 32, "pdsink_done layout");

__device__ __forceinline__ void post_done(DoneRec* done, unsigned tag, long long q, double cost, int it_lp, int it_hp,
                                          float err, int st) {
  DoneRec* r = done + q;
  r->cost = cost;
  r->err = err;
  r->status = st;
  r->it[0] = it_lp;
  r->it[1] = it_hp;
  __hip_atomic_store(&r->tag, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

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

// Cross-lane steps without LDS traffic: DPP moves within rows of 16 lanes
// (quad swaps, rotations, mirrors) and the gfx950 permlane swaps between
// rows (lanes l and l ^ 16) and halves (l and l ^ 32).  Each reduction leaves
// its result in every lane.
constexpr int DPP_QXOR1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int DPP_QXOR2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int DPP_ROR4 = 0x124;     // row_ror:4
constexpr int DPP_ROR8 = 0x128;     // row_ror:8
constexpr int DPP_HMIRROR = 0x141;  // row_half_mirror: lane 7 - i within 8
constexpr int DPP_MIRROR = 0x140;   // row_mirror: lane 15 - i within 16

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL)), hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
// The two values of lanes l and l ^ 16 (SWAP = 16) or l and l ^ 32 (SWAP = 32).
template <int SWAP>
__device__ __forceinline__ void swap_i(int v, int& a, int& b) {
  if constexpr (SWAP == 16) {
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    a = (int)p[0];
    b = (int)p[1];
  } else {
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    a = (int)p[0];
    b = (int)p[1];
  }
}
template <int SWAP>
__device__ __forceinline__ void swap_d(double v, double& a, double& b) {
  const long long x = __double_as_longlong(v);
  int la, lb, ha, hb;
  swap_i<SWAP>((int)(x & 0xffffffffLL), la, lb);
  swap_i<SWAP>((int)(x >> 32), ha, hb);
  a = __longlong_as_double(((long long)(unsigned)ha << 32) | (unsigned)la);
  b = __longlong_as_double(((long long)(unsigned)hb << 32) | (unsigned)lb);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<DPP_QXOR1>(v);
  v += dpp_d<DPP_QXOR2>(v);
  v += dpp_d<DPP_ROR4>(v);
  v += dpp_d<DPP_ROR8>(v);
  double a, b;
  swap_d<16>(v, a, b);
  v = a + b;
  swap_d<32>(v, a, b);
  return a + b;
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<DPP_QXOR1>(v);
  v += dpp_f<DPP_QXOR2>(v);
  v += dpp_f<DPP_ROR4>(v);
  v += dpp_f<DPP_ROR8>(v);
  int a, b;
  swap_i<16>(__float_as_int(v), a, b);
  v = __int_as_float(a) + __int_as_float(b);
  swap_i<32>(__float_as_int(v), a, b);
  return __int_as_float(a) + __int_as_float(b);
}
__device__ __forceinline__ int wave_sum(int v) {
  v += dpp_i<DPP_QXOR1>(v);
  v += dpp_i<DPP_QXOR2>(v);
  v += dpp_i<DPP_ROR4>(v);
  v += dpp_i<DPP_ROR8>(v);
  int a, b;
  swap_i<16>(v, a, b);
  v = a + b;
  swap_i<32>(v, a, b);
  return a + b;
}
__device__ __forceinline__ int wave_max(int v) {
  v = max(v, dpp_i<DPP_QXOR1>(v));
  v = max(v, dpp_i<DPP_QXOR2>(v));
  v = max(v, dpp_i<DPP_ROR4>(v));
  v = max(v, dpp_i<DPP_ROR8>(v));
  int a, b;
  swap_i<16>(v, a, b);
  v = max(a, b);
  swap_i<32>(v, a, b);
  return max(a, b);
}
__device__ __forceinline__ int wave_min(int v) {
  v = min(v, dpp_i<DPP_QXOR1>(v));
  v = min(v, dpp_i<DPP_QXOR2>(v));
  v = min(v, dpp_i<DPP_ROR4>(v));
  v = min(v, dpp_i<DPP_ROR8>(v));
  int a, b;
  swap_i<16>(v, a, b);
  v = min(a, b);
  swap_i<32>(v, a, b);
  return min(a, b);
}
__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, dpp_d<DPP_QXOR1>(v));
  v = fmin(v, dpp_d<DPP_QXOR2>(v));
  v = fmin(v, dpp_d<DPP_ROR4>(v));
  v = fmin(v, dpp_d<DPP_ROR8>(v));
  double a, b;
  swap_d<16>(v, a, b);
  v = fmin(a, b);
  swap_d<32>(v, a, b);
  return fmin(a, b);
}
// Maximum over aligned groups of N consecutive lanes (N = 4, 8, 16, 32), in
// every lane of the group.
template <int N>
__device__ __forceinline__ int group_max(int v) {
  static_assert(N == 4 || N == 8 || N == 16 || N == 32, "group size");
  v = max(v, dpp_i<DPP_QXOR1>(v));
  v = max(v, dpp_i<DPP_QXOR2>(v));
  if constexpr (N >= 8) v = max(v, dpp_i<DPP_HMIRROR>(v));
  if constexpr (N >= 16) v = max(v, dpp_i<DPP_MIRROR>(v));
  if constexpr (N >= 32) {
    int a, b;
    swap_i<16>(v, a, b);
    v = max(a, b);
  }
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
__device__ __forceinline__ double block_min(double v, double* red) {
  v = wave_min(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = red[0];
#pragma unroll 4
  for (int w = 1; w < NW; ++w) t = fmin(t, red[w]);
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
  const int e = wave_max(v.s != 0.0 ? v.e : -(1 << 24));
  return ESum{e, wave_sum(v.s != 0.0 ? ldxd(v.s, v.e - e) : 0.0)};
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
