// Resident-kernel variant of the per-pair Sinkhorn solve (Algorithm 1 of
// Lacombe, Cuturi, Oudot, NeurIPS 2018) for grids up to 100 x 100 on the
// 128-padded layout, supports on or above the diagonal and up to 512 cells
// per side.  Same iteration, stopping rule, representation and cost as the
// general kernel of sinkhorn_pair.h; what differs is how often the
// per-pair scaffolding around the two contractions of Proposition 2 is
// rebuilt, and where it lives.
//
// Sticky scales.  A scaling vector y is stored as 2^(P_i + Q_j) * residual.
// After an update the new y is first expressed in y's previous scales; the
// row/column refit runs only when that residual spans more than SPAN octaves
// (or y has no scales yet).  Between refits the scales of both sides are
// fixed, so the absorbed 1-D kernels of both K applications (K v with v's
// scales, K u with u's) do not change: all four are kept in LDS as BF16 and
// rebuilt, with their max-plus normalisers, only after a refit of their side.
// Over a solve of a few hundred iterations a side is refit a handful of
// times, mostly in the first tens of iterations.
//
// Layout (BF16 phase).  Four kernels of d rows x KD columns (KD = d rounded
// up to the MFMA depth 16), then two slots that alternate between half steps:
// the input residual X (d + 1 rows, the last one zero for padded tile rows)
// is read by contraction 1, whose output T^T goes to the other slot; the
// result W of contraction 2 is stored packed (upper triangle, column j holds
// rows 0 .. j) over the dead X; the update writes the new residual into
// the slot that held T^T, which the next half step reads as its X.  A half
// step without refit, rebuild or suspect needs four workgroup barriers.
// The FP32 phase (refinement, the FP32 form and the cost) computes kernel
// entries on the fly and lays X, T and W out over the same bytes.
#pragma once

#include "sinkhorn_pair.h"

namespace pdsink {

constexpr int FAST_DMAX = 100;                  // largest grid of the variant
constexpr int RESIDENT_AUTO_DMIN = 65;          // smallest grid it runs by default with FP32 contractions
constexpr int FAST_KD = 112;                    // FAST_DMAX rounded up to 16
constexpr int FAST_LDB = FAST_KD + 8;           // BF16 row stride at most (16-byte aligned rows)
constexpr int FAST_MAXSUSP = 128;               // suspects handled per half step
constexpr int FAST_SPAN = 44;                   // residual span (octaves) kept without a refit
// Margin (octaves) between the bound on what the contractions drop and a
// trusted value: the FP32 unit roundoff for FP32 contractions; in the BF16
// phase 2^-10, already below the rounding of the BF16 operands (2^-8 relative
// per entry), since the FP32 refinement decides the result.
constexpr int FAST_MARGIN_BF16 = 10;

struct FastLayout {
  // BF16 phase
  static constexpr int KBYTES = FAST_DMAX * FAST_LDB * 2;               // one kernel
  static constexpr int SLOT = (FAST_DMAX + 2) * FAST_LDB * 2;           // X / T^T / packed W + staging
  static constexpr int K1V = 0, K2V = KBYTES, K1U = 2 * KBYTES, K2U = 3 * KBYTES;
  static constexpr int S0 = 4 * KBYTES, S1 = S0 + SLOT;
  static constexpr int BIG = S1 + SLOT;
  // packed W (columns padded to multiples of 4 rows, 4 (a+1)(2a+b) floats
  // before column j = 4a + b) and a 16-byte dummy slot per lane after it
  static constexpr int WP = (4 * (FAST_DMAX / 4 + 1) * (2 * (FAST_DMAX / 4) + FAST_DMAX % 4) + 4 * 64) * 4;
  // FP32 phase: X [d + 1][KD + 1], T [KD][129], W packed + staging
  static constexpr int LTF = 128 + 1;
  static constexpr int FA = 0;
  static constexpr int FB = ((FAST_DMAX + 1) * (FAST_KD + 1) * 4 + 15) & ~15;
  static constexpr int FC = FB + ((FAST_KD * LTF * 4 + 15) & ~15);
  static_assert(WP <= SLOT, "packed W in one slot");
  static_assert(FC + WP <= BIG, "FP32 layout within the BF16 one");
};

struct FastSmem {
  alignas(16) char big[FastLayout::BIG];
  alignas(16) int tge[256];
  int tgde[256], tkb[256];
  float tgm[256], tgdm[256], tc1[256], tcd[256];
  alignas(16) int Pu[128];
  alignas(16) int Qu[128];
  alignas(16) int Pv[128];
  alignas(16) int Qv[128];
  alignas(16) int Ru[128];
  alignas(16) int Su[128];
  alignas(16) int Rv[128];
  alignas(16) int Sv[128];
  // refit extrema; between refits the same bytes hold the staging of x's
  // support list for the exact path (pass A to the suspects) and the terms
  // of <y, k_Delta> (final pass to the next half step's contraction 2)
  alignas(16) int fit[2][4][128];
  int sflag, nsusp;
  double red[PNW], reds[PNW], redf[PNW];
  int rede[PNW], redi[PNW], redm[PNW];
  // per-wave partial results of an update pass: error sum, flags, span
  struct alignas(16) Rec {
    double eg;
    int flags;
    int span;
  } rec[PNW], rec2[PNW];
  int susp_cell[FAST_MAXSUSP], susp_e[FAST_MAXSUSP];
  float susp_m[FAST_MAXSUSP];
};
static_assert(sizeof(FastSmem) <= 160 * 1024, "one workgroup's LDS");

// Kernel headroom (octaves) for an input whose residual may span +-span
// octaves.  A contraction sums at most 2^14 products of two kernel entries
// (each at most 2^H) and one residual entry, so its values stay below
// 2^(2H + span + 14); 2H + span <= 113 keeps them below 2^127.  The larger
// the headroom, the smaller the part of each kernel row lost to the flush
// below 2^-126, and the fewer cells need the exact evaluation.
__device__ __forceinline__ int fast_headroom(int span) { return max(0, min(HEAD, (113 - span) >> 1)); }

// Index of cell (i, j), i <= j, in the packed upper triangle stored by
// columns, each padded to a multiple of 4 rows (so that 4 consecutive rows
// starting at a multiple of 4 form one aligned 16-byte group): column j =
// 4a + b starts at sum_{j' < j} 4 ceil((j' + 1) / 4) = 4 (a + 1)(2a + b).
__device__ __forceinline__ int wcol(int j) { return 4 * ((j >> 2) + 1) * (2 * (j >> 2) + (j & 3)); }
__device__ __forceinline__ int widx(int i, int j) { return wcol(j) + i; }

// Per-side state beyond the support list.
struct FSide {
  int ex;        // diagonal entry mx * 2^ex
  double mx;
  int mres;      // residual span of the last update (octaves)
  int H;         // headroom of the side's kernels
  int span;      // refit when a new residual spans more than this
  bool fitted;   // the side has scales
  bool rs;       // R, S of the side's scales are current
  bool kern;     // the BF16 kernels of the side's scales are current
  int rs_gen;    // bumped whenever R, S of the side are recomputed
  int sc_gen;    // bumped whenever the side's scales are refit
};

// Per-thread constants of the update of one support entry of y from x, fixed
// between refits: tagged with the generations of x's normalisers and y's scales.
struct FCache {
  int shp;       // P_y(i) + Q_y(j) + R_x(i) + S_x(j): log2 of y's scale over K x's
  int e0;        // ge_Delta(j - i) - R_x(i) - S_x(j): the diagonal-bin term's exponent
  float gdm;     // its mantissa
  int edot;      // P_y(i) + Q_y(j) + ge_Delta(j - i): exponent of y_ij k_Delta,ij
  int rs_tag, sc_tag;
};

// Phase cycle counters (library built with PDSINK_PROFILE=1 only): cycles
// between workgroup barriers accumulated per phase, events counted, summed
// over pairs into g_phase by thread 0 at the end of each solve.
#ifndef PDSINK_PROFILE
#define PDSINK_PROFILE 0
#endif
enum FPhase {
  PH_SETUP, PH_SCALES, PH_BUILD, PH_C1, PH_C2, PH_PASSA, PH_SUSPECT, PH_REFIT, PH_FINAL, PH_COST,
  PH_N_HALF, PH_N_REFIT, PH_N_BUILD, PH_N_SCALES, PH_N_SUSPECT, PH_N_PAIRS, PH_COUNT
};
#if PDSINK_PROFILE
__device__ unsigned long long g_phase[PH_COUNT];
#endif
struct FProf {
#if PDSINK_PROFILE
  unsigned long long acc[PH_COUNT];
  unsigned long long last;
  __device__ void init() {
    for (int k = 0; k < PH_COUNT; ++k) acc[k] = 0;
    last = __builtin_readcyclecounter();
  }
  __device__ void mark(int k) {
    const unsigned long long now = __builtin_readcyclecounter();
    acc[k] += now - last;
    last = now;
  }
  __device__ void count(int k) { acc[k] += 1; }
  __device__ void commit() {
    if (threadIdx.x == 0)
      for (int k = 0; k < PH_COUNT; ++k) atomicAdd(&g_phase[k], acc[k]);
  }
#else
  __device__ void init() {}
  __device__ void mark(int) {}
  __device__ void count(int) {}
  __device__ void commit() {}
#endif
};

// Support list of a histogram (staged in `stage`: cell [cap] then value [cap]).
__device__ __forceinline__ double f_build_support(FastSmem& s, const float* __restrict__ h, int d, SupList<1>& sp,
                                                  bool& too_big, bool& lower, char* stage) {
  constexpr int D = 128;
  int* scell = reinterpret_cast<int*>(stage);
  float* sval = reinterpret_cast<float*>(stage + PWGS * 4);
  const int n = d * d;
  const int per = (n + PWGS - 1) / PWGS;
  const int c0 = threadIdx.x * per, c1 = min(c0 + per, n);
  int cnt = 0, low = 0;
  double mass = 0.0;
  for (int c = c0; c < c1; ++c) {
    const float v = h[c];
    if (v > 0.0f) {
      ++cnt;
      mass += v;
      low |= (c % d) < (c / d);
    }
  }
  lower = __syncthreads_or(low);
  int total;
  int off = block_scan(cnt, s.redi, total);
  mass = block_sum<PNW>(mass, s.red);
  too_big = total > PWGS;
  if (!too_big) {
    for (int c = c0; c < c1; ++c) {
      const float v = h[c];
      if (v > 0.0f) {
        scell[off] = (c / d) * D + (c % d);
        sval[off] = v;
        ++off;
      }
    }
  }
  __syncthreads();
  const bool ok = !too_big && (int)threadIdx.x < total;
  sp.set_entry(0, ok ? scell[threadIdx.x] : -1, ok ? sval[threadIdx.x] : 0.0f);
  __syncthreads();
  return mass;
}

// R_i = max_k (P_k + ge(i - k)) - H (rows i >= d: BIG), S_j likewise from Q:
// the max-plus normalisers of the absorbed kernels (as compute_RS).
__device__ __forceinline__ void f_compute_RS(const FastSmem& s, const int* P, const int* Q, int d, int H, int* R,
                                             int* S) {
  constexpr int D = 128;
  constexpr int NRB = 2 * D / 4, NPART = PWGS / NRB, KPT = D / NPART;
  const int combo = threadIdx.x / NPART, part = threadIdx.x % NPART;
  const bool rows = combo < NRB / 2;
  const int i0 = 4 * (rows ? combo : combo - NRB / 2);
  const int* X = rows ? P : Q;
  const int k0 = part * KPT;
  int b0 = NEG, b1 = NEG, b2 = NEG, b3 = NEG;
  const int start = i0 - k0 + D - 1 - (KPT - 1);
  int xv[KPT], wv[KPT + 4];
#pragma unroll
  for (int t = 0; t < KPT; t += 4) {
    const int4 v = *reinterpret_cast<const int4*>(X + k0 + t);
    xv[t] = v.x;
    xv[t + 1] = v.y;
    xv[t + 2] = v.z;
    xv[t + 3] = v.w;
  }
#pragma unroll
  for (int m = 0; m < KPT + 4; m += 4) {
    const int4 v = *reinterpret_cast<const int4*>(s.tge + start + m);
    wv[m] = v.x;
    wv[m + 1] = v.y;
    wv[m + 2] = v.z;
    wv[m + 3] = v.w;
  }
#pragma unroll
  for (int t = 0; t < KPT; ++t) {
    const int x = xv[t];
    b0 = max(b0, x + wv[KPT - 1 - t]);
    b1 = max(b1, x + wv[KPT - t]);
    b2 = max(b2, x + wv[KPT + 1 - t]);
    b3 = max(b3, x + wv[KPT + 2 - t]);
  }
  b0 = group_max<NPART>(b0);
  b1 = group_max<NPART>(b1);
  b2 = group_max<NPART>(b2);
  b3 = group_max<NPART>(b3);
  if (part == 0) {
    int* out = (rows ? R : S) + i0;
    const int bb[4] = {b0, b1, b2, b3};
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = i0 + r < d ? (bb[r] <= NEG / 2 ? 0 : bb[r] - H) : BIG;
  }
}

// BF16 kernels K1[i][k] = 2^(P_k + g(i-k) - R_i), K2[j][l] from Q and S, rows
// below d and columns below KD (entries of columns k >= d are exact zeros:
// P_k = NEG there), assembled as BF16 bit patterns from the table words
// (see build_kernels_bf16).  X7 holds P then Q clamped and shifted to the
// exponent field (2 x 128 ints).
__device__ __forceinline__ void f_build_bf16(const FastSmem& s, const int* X7, const int* R, const int* S, int d,
                                             int KD, int LDB, __bf16* K1, __bf16* K2) {
  constexpr int D = 128;
  const int nch = KD / 16;
  for (int item = threadIdx.x; item < nch * d; item += PWGS) {
    const int i = item % d, k0 = 16 * (item / d);
    const int* tw = s.tkb + i - k0 + D - 1;
    int wd[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) wd[t] = tw[-t];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int* x7 = X7 + side * 128 + k0;
      const int base7 = (126 - (side == 0 ? R : S)[i]) << 7;
      const int4 xa = *reinterpret_cast<const int4*>(x7), xb = *reinterpret_cast<const int4*>(x7 + 4);
      const int4 xc = *reinterpret_cast<const int4*>(x7 + 8), xd = *reinterpret_cast<const int4*>(x7 + 12);
      const int xs[16] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w,
                          xc.x, xc.y, xc.z, xc.w, xd.x, xd.y, xd.z, xd.w};
      unsigned int pk[8];
#pragma unroll
      for (int t = 0; t < 16; t += 2) {
        const int v0 = min(max(wd[t] + xs[t] + base7, 0), 0x7FFF);
        const int v1 = min(max(wd[t + 1] + xs[t + 1] + base7, 0), 0x7FFF);
        pk[t >> 1] = (unsigned)v0 | ((unsigned)v1 << 16);
      }
      uint4* dst = reinterpret_cast<uint4*>((side == 0 ? K1 : K2) + i * LDB + k0);
      dst[0] = uint4{pk[0], pk[1], pk[2], pk[3]};
      dst[1] = uint4{pk[4], pk[5], pk[6], pk[7]};
    }
  }
}

// Contraction 1 in BF16: T^T[j][k] = sum_l X[k][l] K2[j][l] for the wave's
// column block tj = w mod 4 and row blocks {0, 3} (w < 4) or {1, 2}: eight
// MFMA steps per wave at KD = 112 with the triangle trimmed.  Rows k >= d of
// X read the zero row d; rows j >= d of K2 read row d - 1 (their outputs are
// not stored).  Every operand of the wave's steps is read before the first
// MFMA (NST = KD / 16 steps at most, fixed at compile time), so the matrix
// cores run the two accumulation chains back to back instead of waiting on
// each LDS read.
template <int NST, int TK0, int TK1, bool TRIM>
__device__ __forceinline__ void f_c1_chain(const __bf16* xa0, const __bf16* xa1, const __bf16* kb, floatx16& acc0,
                                           floatx16& acc1) {
  constexpr int S0 = TRIM ? 2 * TK0 : 0;
  constexpr int S1 = TRIM ? (2 * TK1 < NST ? 2 * TK1 : NST) : 0;
  constexpr int PF = 4;   // steps in flight: a rotating register buffer
  bf16x8 a0[PF], a1[PF], b[PF];
  auto load = [&](int st) {
    b[st % PF] = *reinterpret_cast<const bf16x8*>(kb + 16 * st);
    a0[st % PF] = *reinterpret_cast<const bf16x8*>(xa0 + 16 * st);
    if (st >= S1) a1[st % PF] = *reinterpret_cast<const bf16x8*>(xa1 + 16 * st);
  };
#pragma unroll
  for (int st = S0; st < NST && st < S0 + PF; ++st) load(st);
  // the order below is kept: the MFMAs of a step, then the reads of the step
  // PF later into the registers they just consumed
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int st = S0; st < NST; ++st) {
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[st % PF], b[st % PF], acc0, 0, 0, 0);
    if (st >= S1) acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[st % PF], b[st % PF], acc1, 0, 0, 0);
    if (st + PF < NST) load(st + PF);
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int NST>
__device__ __forceinline__ void f_c1_bf16(const __bf16* X, const __bf16* K2, __bf16* Tt, int d, int LDB, bool trim) {
  constexpr int KD = 16 * NST;
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tj = w & 3, tk0 = w < 4 ? 0 : 1, tk1 = w < 4 ? 3 : 2;
  const int j = tj * 32 + lr;
  const int r0 = tk0 * 32 + lr, r1 = tk1 * 32 + lr;
  const __bf16* xa0 = X + (r0 < d ? r0 : d) * LDB + 8 * lk;
  const __bf16* xa1 = X + (r1 < d ? r1 : d) * LDB + 8 * lk;
  const __bf16* kb = K2 + min(j, d - 1) * LDB + 8 * lk;
  floatx16 acc0 = {}, acc1 = {};
  if (w < 4) {
    if (trim) f_c1_chain<NST, 0, 3, true>(xa0, xa1, kb, acc0, acc1);
    else f_c1_chain<NST, 0, 3, false>(xa0, xa1, kb, acc0, acc1);
  } else {
    if (trim) f_c1_chain<NST, 1, 2, true>(xa0, xa1, kb, acc0, acc1);
    else f_c1_chain<NST, 1, 2, false>(xa0, xa1, kb, acc0, acc1);
  }
  // No explicit drain after the BF16 chains: the compiler's wait states
  // before the first reads of the accumulators (s_nop 7 / 11 after
  // v_mfma_f32_32x32x16_bf16) cover them (the FP32 chains keep mfma_drain).
  // Unconditional stores: rows j >= d go to the slot's spare row d + 1, and
  // groups of columns k >= KD to the pad columns KD .. KD + 3 of the row;
  // neither is ever read.  (Selecting the address keeps the epilogue free
  // of branches, which cost more here than the stores they would skip.)
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  __bf16* trow = Tt + (j < d ? j : d + 1) * LDB;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k0 = tk0 * 32 + 8 * q + 4 * lk, k1 = tk1 * 32 + 8 * q + 4 * lk;
    const bf16x4 v0 = {(__bf16)acc0[4 * q], (__bf16)acc0[4 * q + 1], (__bf16)acc0[4 * q + 2], (__bf16)acc0[4 * q + 3]};
    const bf16x4 v1 = {(__bf16)acc1[4 * q], (__bf16)acc1[4 * q + 1], (__bf16)acc1[4 * q + 2], (__bf16)acc1[4 * q + 3]};
    *reinterpret_cast<bf16x4*>(trow + (k0 < KD ? k0 : KD)) = v0;
    *reinterpret_cast<bf16x4*>(trow + (k1 < KD ? k1 : KD)) = v1;
  }
}

// Store of one 32 x 32 accumulator tile (row block ti, column block tj; the
// lane holds column j = 32 tj + (lane mod 32) and rows i0 + 8q + t, q, t in
// 0..3, in registers 4q + t) into the packed upper triangle: each group of 4
// rows is one aligned 16-byte store.  A group whose first row lies on or
// above the diagonal is stored whole (rows past j land in the column's
// padding); other groups, and columns j >= d, go to a dummy slot of the lane.
// The address is selected per lane, with no branch: on gfx950 a branch
// around each store (even one uniform over the wave) made this epilogue
// cost more than the stores themselves.
__device__ __forceinline__ void f_store_w(float* Wp, const floatx16& acc, int ti, int tj, int d) {
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int i0 = ti * 32 + 4 * lk, j = tj * 32 + lr;
  float4* grp = reinterpret_cast<float4*>(Wp + widx(i0, j));
  float4* dummy = reinterpret_cast<float4*>(Wp + wcol(d)) + lane;
  const int lim = j < d ? j - i0 : -1;   // group q (rows i0 + 8q ..) is stored when 8q <= lim
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = {acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
    *(8 * q <= lim ? grp + 2 * q : dummy) = v;
  }
}

// Upper tiles of contraction 2 per wave: waves 0-3 two tiles of one row
// block sharing the K1 operand, waves 4 and 5 one tile each as two chains
// over the halves of k, waves 6 and 7 none.
__device__ __forceinline__ void f_c2_tiles(int w, int& ti, int& tj) {
  if (w < 4) {
    ti = w < 2 ? 0 : w - 1;
    tj = w == 0 ? 0 : (w == 2 ? 1 : 2);
  } else {
    ti = w == 4 ? 1 : 3;
    tj = 3;
  }
}

// Contraction 2 in BF16: W[i][j] = sum_k K1[i][k] T^T[j][k] on the upper
// tiles, stored packed into Wp (which must not alias K1 or T^T).  As in
// contraction 1, every operand is read before the first MFMA.
template <int NST>
__device__ __forceinline__ void f_c2_bf16(const __bf16* K1, const __bf16* Tt, float* Wp, int d, int LDB) {
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= 6) return;
  int ti, tj;
  f_c2_tiles(w, ti, tj);
  const int i = ti * 32 + lr, ja = tj * 32 + lr;
  const __bf16* ka = K1 + min(i, d - 1) * LDB + 8 * lk;
  const __bf16* t0 = Tt + min(ja, d - 1) * LDB + 8 * lk;
  floatx16 acc0 = {}, acc1 = {};
  constexpr int PF = 4;   // steps in flight: a rotating register buffer (as in contraction 1)
  if (w < 4) {
    const __bf16* t1 = Tt + min(ja + 32, d - 1) * LDB + 8 * lk;
    bf16x8 a[PF], b0[PF], b1[PF];
    auto load = [&](int st) {
      a[st % PF] = *reinterpret_cast<const bf16x8*>(ka + 16 * st);
      b0[st % PF] = *reinterpret_cast<const bf16x8*>(t0 + 16 * st);
      b1[st % PF] = *reinterpret_cast<const bf16x8*>(t1 + 16 * st);
    };
#pragma unroll
    for (int st = 0; st < NST && st < PF; ++st) load(st);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[st % PF], b0[st % PF], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[st % PF], b1[st % PF], acc1, 0, 0, 0);
      if (st + PF < NST) load(st + PF);
      __builtin_amdgcn_sched_barrier(0);
    }
    f_store_w(Wp, acc0, ti, tj, d);
    f_store_w(Wp, acc1, ti, tj + 1, d);
  } else {
    // chain a: steps [0, H), chain b: steps [H, NST)
    constexpr int H = (NST + 1) / 2;
    bf16x8 a[NST], b[NST];
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      a[st] = *reinterpret_cast<const bf16x8*>(ka + 16 * st);
      b[st] = *reinterpret_cast<const bf16x8*>(t0 + 16 * st);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < H; ++st) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[st], b[st], acc0, 0, 0, 0);
      if (H + st < NST) acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[H + st], b[H + st], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc0[r] += acc1[r];
    f_store_w(Wp, acc0, ti, tj, d);
  }
}

// FP32 kernel entry 2^(P_k + g(i-k) - Ri) (times c(i-k) when WEIGHTED: the m of
// Proposition 3), built from the exact exponent/mantissa tables.
template <bool WEIGHTED>
__device__ __forceinline__ float f_kentry(const FastSmem& s, int i, int k, const int* P, int Ri) {
  constexpr int D = 128;
  const int idx = i - k + D - 1;
  float v = ldx(s.tgm[idx], P[k] + s.tge[idx] - Ri);
  if (WEIGHTED) v *= s.tc1[idx];
  return v;
}

// Contraction 1 in FP32: T[k][j] = sum_l X[k][l] kt2[j][l] (kt2 from Q and S,
// weighted when WEIGHTED); X [d + 1][LXF] (row d zero), T [KD][LTF].
template <bool WEIGHTED>
__device__ __forceinline__ void f_c1_fp32(const FastSmem& s, const float* X, float* T, const int* Q, const int* S,
                                          int d, int KD, bool trim) {
  constexpr int LTF = FastLayout::LTF;
  const int LXF = KD + 1;
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tj = w & 3, tk0 = w < 4 ? 0 : 1, tk1 = w < 4 ? 3 : 2;
  const int j = tj * 32 + lr, r0 = tk0 * 32 + lr, r1 = tk1 * 32 + lr;
  const int lb0 = trim ? tk0 * 32 : 0, lb1 = min(trim ? tk1 * 32 : 0, KD);
  const float* x0 = X + (r0 < d ? r0 : d) * LXF;
  const float* x1 = X + (r1 < d ? r1 : d) * LXF;
  const int Sj = S[j];
  floatx16 acc0 = {}, acc1 = {};
#pragma unroll 4
  for (int l0 = lb0; l0 < lb1; l0 += 2) {
    const int l = l0 + lk;
    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x0[l], f_kentry<WEIGHTED>(s, j, l, Q, Sj), acc0, 0, 0, 0);
  }
#pragma unroll 4
  for (int l0 = lb1; l0 < KD; l0 += 2) {
    const int l = l0 + lk;
    const float b = f_kentry<WEIGHTED>(s, j, l, Q, Sj);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x0[l], b, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(x1[l], b, acc1, 0, 0, 0);
  }
  mfma_drain();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k0 = tk0 * 32 + 8 * (r >> 2) + 4 * lk + (r & 3), k1 = tk1 * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
    if (k0 < KD) T[k0 * LTF + j] = acc0[r];
    if (k1 < KD) T[k1 * LTF + j] = acc1[r];
  }
}

// Contraction 2 in FP32: W[i][j] = sum_k kt1[i][k] T[k][j] (kt1 from P and R,
// weighted when WEIGHTED) on the upper tiles, stored packed into Wp.
template <bool WEIGHTED>
__device__ __forceinline__ void f_c2_fp32(const FastSmem& s, const float* T, float* Wp, const int* P, const int* R,
                                          int d, int KD) {
  constexpr int LTF = FastLayout::LTF;
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= 6) return;
  int ti, tj;
  f_c2_tiles(w, ti, tj);
  const int ia = ti * 32 + lr, ja = tj * 32 + lr;
  const int Ra = R[ia];
  floatx16 acc0 = {}, acc1 = {};
  if (w < 4) {
    // one kernel entry for both tiles; operands of step k0 + 2 read while step k0 runs
    float a = f_kentry<WEIGHTED>(s, ia, lk, P, Ra), b0 = T[lk * LTF + ja], b1 = T[lk * LTF + ja + 32];
    // (bounded unrolling: fully unrolled at the small grids' depths these
    // loops pushed the whole kernel into scratch spills, 50 to 110 VGPRs)
#pragma unroll 2
    for (int k0 = 0; k0 < KD; k0 += 2) {
      const int kn = (k0 + 2 < KD ? k0 + 2 : 0) + lk;
      const float na = f_kentry<WEIGHTED>(s, ia, kn, P, Ra), nb0 = T[kn * LTF + ja], nb1 = T[kn * LTF + ja + 32];
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc1, 0, 0, 0);
      a = na;
      b0 = nb0;
      b1 = nb1;
    }
    mfma_drain();
    f_store_w(Wp, acc0, ti, tj, d);
    f_store_w(Wp, acc1, ti, tj + 1, d);
  } else {
    const int H2 = KD / 2;
    float a0 = f_kentry<WEIGHTED>(s, ia, lk, P, Ra), b0 = T[lk * LTF + ja];
    float a1 = f_kentry<WEIGHTED>(s, ia, lk + H2, P, Ra), b1 = T[(lk + H2) * LTF + ja];
#pragma unroll 2
    for (int k0 = 0; k0 < H2; k0 += 2) {
      const int kn = (k0 + 2 < H2 ? k0 + 2 : 0) + lk;
      const float na0 = f_kentry<WEIGHTED>(s, ia, kn, P, Ra), nb0 = T[kn * LTF + ja];
      const float na1 = f_kentry<WEIGHTED>(s, ia, kn + H2, P, Ra), nb1 = T[(kn + H2) * LTF + ja];
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc1, 0, 0, 0);
      a0 = na0;
      b0 = nb0;
      a1 = na1;
      b1 = nb1;
    }
    mfma_drain();
#pragma unroll
    for (int r = 0; r < 16; ++r) acc0[r] += acc1[r];
    f_store_w(Wp, acc0, ti, tj, d);
  }
}

// Exact values of (K x) (times C when WEIGHTED) at the suspects [0, ns) of
// s.susp_cell: a sum over x's support with explicit exponents (as
// exact_all): largest term exponent first, then the scaled sum.  x is a
// staged list of PWGS entries (cell, residual; cell < 0 = none) or, when
// `dense`, 1 on every grid cell.  FIN: the value in the natural scale of the
// cell, 2^-(R_i + S_j), plus the diagonal-bin term x_Delta k_Delta; the
// total vanishing sets s.sflag.
template <bool WEIGHTED, bool FIN>
__device__ __forceinline__ void f_exact(FastSmem& s, const int* xcell, const float* xres, bool dense, int d,
                                        const int* Px, const int* Qx, const int* R, const int* S, int ns, int xD_e,
                                        float xD_m) {
  constexpr int D = 128;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  auto finish = [&](int id, int c, int em, float acc) {
    if constexpr (FIN) {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      const ESum g{em - R[i] - S[j], (double)acc};
      const ESum tot = esum_add(g, ESum{xD_e + s.tgde[dl] - R[i] - S[j], (double)(xD_m * s.tgdm[dl])});
      if (tot.s > 0.0) {
        s.susp_e[id] = tot.e;
        s.susp_m[id] = (float)tot.s;
      } else {
        atomicOr(&s.sflag, 1);
        s.susp_e[id] = 0;
        s.susp_m[id] = 1.0f;
      }
    } else {
      s.susp_e[id] = em;
      s.susp_m[id] = acc;
    }
  };
  if (!dense) {
    constexpr int EPL = PWGS / 64;
    int kr[EPL], l[EPL], eb[EPL];
    float xm[EPL];
#pragma unroll
    for (int u = 0; u < EPL; ++u) {
      const int cell = xcell[lane + 64 * u];
      const float x = xres[lane + 64 * u];
      const bool ok = cell >= 0 && x > 0.0f;
      kr[u] = ok ? cell / D : 0;
      l[u] = ok ? cell % D : 0;
      xm[u] = ok ? x : 0.0f;
      eb[u] = ok ? Px[kr[u]] + Qx[l[u]] : QNONE;
    }
    for (int id = wave; id < ns; id += PNW) {
      const int c = s.susp_cell[id];
      const int ti = c / D, tj = c % D;
      int em = QNONE;
#pragma unroll
      for (int u = 0; u < EPL; ++u)
        if (eb[u] != QNONE)
          em = max(em, eb[u] + ilog2f(xm[u]) + s.tge[ti - kr[u] + D - 1] + s.tge[tj - l[u] + D - 1]);
      em = wave_max(em);
      float acc = 0.0f;
#pragma unroll
      for (int u = 0; u < EPL; ++u) {
        if (eb[u] != QNONE) {
          const int i1 = ti - kr[u] + D - 1, i2 = tj - l[u] + D - 1;
          float mm = xm[u] * s.tgm[i1] * s.tgm[i2];
          if (WEIGHTED) mm *= (s.tc1[i1] + s.tc1[i2]);
          acc += ldx(mm, eb[u] + s.tge[i1] + s.tge[i2] - em);
        }
      }
      acc = wave_sum(acc);
      if (lane == 0) finish(id, c, em, acc);
    }
    __syncthreads();
    return;
  }
  // dense x (the all-ones start): four suspects per wave
  constexpr int NT4 = 4;
  const int nx = d * d;
  for (int id0 = wave * NT4; id0 < ns; id0 += PNW * NT4) {
    const int nt = min(NT4, ns - id0);
    int ti[NT4], tj[NT4], em[NT4];
#pragma unroll
    for (int t = 0; t < NT4; ++t) {
      const int c = t < nt ? s.susp_cell[id0 + t] : 0;
      ti[t] = c / D;
      tj[t] = c % D;
      em[t] = QNONE;
    }
    for (int e = lane; e < nx; e += 64) {
      const int kr = e / d, l = e % d;
      const int eb = Px[kr] + Qx[l];
#pragma unroll
      for (int t = 0; t < NT4; ++t) em[t] = max(em[t], eb + s.tge[ti[t] - kr + D - 1] + s.tge[tj[t] - l + D - 1]);
    }
#pragma unroll
    for (int t = 0; t < NT4; ++t) em[t] = wave_max(em[t]);
    float acc[NT4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int e = lane; e < nx; e += 64) {
      const int kr = e / d, l = e % d;
      const int eb = Px[kr] + Qx[l];
#pragma unroll
      for (int t = 0; t < NT4; ++t) {
        const int i1 = ti[t] - kr + D - 1, i2 = tj[t] - l + D - 1;
        float mm = s.tgm[i1] * s.tgm[i2];
        if (WEIGHTED) mm *= (s.tc1[i1] + s.tc1[i2]);
        acc[t] += ldx(mm, eb + s.tge[i1] + s.tge[i2] - em[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < NT4; ++t) acc[t] = wave_sum(acc[t]);
    if (lane == 0) {
#pragma unroll
      for (int t = 0; t < NT4; ++t)
        if (t < nt) finish(id0 + t, ti[t] * D + tj[t], em[t], acc[t]);
    }
  }
  __syncthreads();
}

// Where one half step reads and writes.
struct FBufs {
  float* w;        // packed K x
  void* nx;        // the new residual (zeroed here, then written on y's support)
  char* stage;     // staging of x's support list for the exact path
  bool nx_bf16;    // format of nx
};

__device__ __forceinline__ void f_put_x(void* buf, int cell, float v, bool bf16, int KD) {
  constexpr int D = 128;
  const int i = cell / D, j = cell % D;
  if (bf16) reinterpret_cast<__bf16*>(buf)[i * (KD + 8) + j] = (__bf16)v;
  else reinterpret_cast<float*>(buf)[i * (KD + 1) + j] = v;
}

// Zero the d + 1 rows of an X buffer in either format.
__device__ __forceinline__ void f_zero_x(void* buf, bool bf16, int d, int KD) {
  const int bytes = bf16 ? (d + 1) * (KD + 8) * 2 : (d + 1) * (KD + 1) * 4;
  uint4* p = reinterpret_cast<uint4*>(buf);
  for (int c = threadIdx.x; c < (bytes >> 4); c += PWGS) p[c] = uint4{0u, 0u, 0u, 0u};
  for (int c = (bytes & ~15) + threadIdx.x; c < bytes; c += PWGS) reinterpret_cast<char*>(buf)[c] = 0;
}

// The update y = target / (K x) on y's support (the sticky-scale form of
// y_update).  K x is W (packed, scaled by 2^-(R_i + S_j)) except at the
// suspects.  With `check`, first the marginal error of the previous y and
// the stopping rule.  The new y is expressed in y's current scales when that
// keeps its residual within y.span octaves; otherwise (or when y has no
// scales yet) the scales are refit by two sweeps of row/column centring, and
// y's normalisers and kernels become stale.  Writes the residual to nx and
// returns <y, k_Delta> (grid part) in dot.
__device__ __forceinline__ void f_update(FastSmem& s, const FBufs& b, SupList<1>& ys, int wix, FCache& cc,
                                         bool lp_contract, const SupList<1>& xsup,
                                         bool x_dense, int d, int KD, const FSide& xs, int H, const int* Px,
                                         const int* Qx, const int* R, const int* S, int* Py, int* Qy, FSide& ysd,
                                         bool check, double& err_out, bool& stop_out, int& bad, int& range,
                                         double errD, double m, double tol, double switch_tol, bool& lowp, int t,
                                         int max_iter, FProf& pf) {
  constexpr int D = 128;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float mxf = (float)xs.mx;
  const int thr = H + max(xs.mres, 20) + 14 - 126 + (lp_contract ? FAST_MARGIN_BF16 : SUSP_MARGIN);
  int* xcell = reinterpret_cast<int*>(b.stage);
  float* xres = reinterpret_cast<float*>(b.stage + PWGS * 4);
  const bool fitted = ysd.fitted;

  // Pass A: suspects, error terms of the previous y, candidate residual in
  // y's current scales, staging of x, clearing of the new X.
  ys.set_q(0, QNONE);
  ys.set_qe(0, QNONE);
  const int c = ys.cell(0);
  const float tg = ys.tgt(0);
  int lover = 0, lbad = 0, span = 0;
  float cand = 0.0f;
  double eg = 0.0;
  if (cc.rs_tag != xs.rs_gen || cc.sc_tag != ysd.sc_gen) {
    // x's normalisers or y's scales changed: refresh the entry's constants
    if (c >= 0) {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      cc.shp = Py[i] + Qy[j] + R[i] + S[j];
      cc.e0 = s.tgde[dl] - R[i] - S[j];
      cc.gdm = s.tgdm[dl];
      cc.edot = Py[i] + Qy[j] + s.tgde[dl];
    }
    cc.rs_tag = xs.rs_gen;
    cc.sc_tag = ysd.sc_gen;
  }
  if (c >= 0) {
    const float w = b.w[wix];
    const int E = xs.ex + cc.e0;
    const float Dm = mxf * cc.gdm;
    const int lw = w > 0.0f ? ilog2f(w) : QNONE;
    const int ld = Dm > 0.0f ? E + ilog2f(Dm) : QNONE;
    const int le = max(lw, ld);
    if (le < thr) {
      const int id = atomicAdd(&s.nsusp, 1);
      if (id < FAST_MAXSUSP) {
        s.susp_cell[id] = c;
        ys.set_q(0, QSUSP + id);
      } else {
        lover = 1;
        if (le == QNONE) lbad = 1;
        ys.set_q(0, le == QNONE ? 0 : ilog2f(tg) - le);
        ys.set_qe(0, le == QNONE ? 0 : ilog2f(tg) - le);
      }
    } else {
      const int qk = ilog2f(tg) - le;
      ys.set_q(0, qk);
      ys.set_qe(0, qk);
      const int shp = cc.shp;
      if (check) {
        const double r = (double)ys.res(0);
        const double row = ldxd(r * (double)w, shp) + ldxd(r * (double)Dm, E + shp);
        eg += fabs(row - (double)tg);
      }
      if (fitted) {
        cand = tg / (ldx(w, shp) + ldx(Dm, E + shp));
        span = abs(qk - shp);
      }
    }
  }
  if (!x_dense) {
    const int xc = xsup.cell(0);
    xcell[tid] = xc;
    xres[tid] = xc >= 0 ? xsup.res(0) : 0.0f;
  }
  f_zero_x(b.nx, b.nx_bf16, d, KD);
  {
    const double egw = check ? wave_sum(eg) : 0.0;
    const unsigned long long bb = __ballot(lbad), bo = __ballot(lover);
    const int sw = wave_max(span);
    if (lane == 0) s.rec[wave] = FastSmem::Rec{egw, (bb ? 1 : 0) | (bo ? 2 : 0), sw};
  }
  __syncthreads();
  pf.mark(PH_PASSA);
  const int ns = min(s.nsusp, FAST_MAXSUSP);
  double egs = 0.0;
  int flags = 0, spn = 0;
#pragma unroll
  for (int w = 0; w < PNW; ++w) {
    const FastSmem::Rec r = s.rec[w];
    egs += r.eg;
    flags |= r.flags;
    spn = max(spn, r.span);
  }

  // Suspects: exact values, their error terms, candidates and spans.
  if (ns > 0) {
    f_exact<false, true>(s, xcell, xres, x_dense, d, Px, Qx, R, S, ns, xs.ex, mxf);
    double eg2 = 0.0;
    int sp2 = 0;
    const int qk = ys.q(0);
    if (qk >= QSUSP) {
      const int id = qk - QSUSP;
      const int i = c / D, j = c % D;
      const int se = s.susp_e[id];
      const float sm = s.susp_m[id];
      const int qx = ilog2f(tg) - (se + ilog2f(sm));
      ys.set_qe(0, qx);
      const int shp = cc.shp;
      if (check) eg2 = fabs(ldxd((double)ys.res(0) * (double)sm, se + shp) - (double)tg);
      if (fitted) {
        cand = tg / ldx(sm, se + shp);
        sp2 = abs(qx - shp);
      }
    }
    eg2 = check ? wave_sum(eg2) : 0.0;
    sp2 = wave_max(sp2);
    if (lane == 0) s.rec2[wave] = FastSmem::Rec{eg2, 0, sp2};
    __syncthreads();
#pragma unroll
    for (int w = 0; w < PNW; ++w) {
      const FastSmem::Rec r = s.rec2[w];
      egs += r.eg;
      spn = max(spn, r.span);
    }
    flags |= s.sflag;
    pf.count(PH_N_SUSPECT);
    pf.mark(PH_SUSPECT);
  }

  if (check) {
    err_out = (egs + errD) / m;
    const bool measured_lowp = lowp;   // never stop on an error measured with BF16 contractions
    if (lowp && (err_out <= switch_tol || 2 * t >= max_iter)) lowp = false;
    if ((!measured_lowp && err_out <= tol) || t >= max_iter) {
      stop_out = true;
      if (flags & 1) bad = 1;
      return;
    }
  }
  if (flags & 1) bad = 1;
  if (flags & 2) range |= 2;   // more suspects than the list holds

  const int qe = ys.qe(0);
  int mres;
  if (!fitted || spn > ysd.span) {
    // Refit: two sweeps of row/column centring of the per-cell log2 estimates.
    for (int r = tid; r < D; r += PWGS) {
#pragma unroll
      for (int sw = 0; sw < 2; ++sw) {
        s.fit[sw][0][r] = INT_MIN;
        s.fit[sw][1][r] = INT_MAX;
        s.fit[sw][2][r] = INT_MIN;
        s.fit[sw][3][r] = INT_MAX;
      }
    }
    __syncthreads();
    const int i = c / D, j = c % D;
    const bool has = qe != QNONE;
    if (has) {
      atomicMax(&s.fit[0][0][i], qe);
      atomicMin(&s.fit[0][1][i], qe);
    }
    __syncthreads();
    if (has) {
      const int v = qe - midrange(s.fit[0][0], s.fit[0][1], i);
      atomicMax(&s.fit[0][2][j], v);
      atomicMin(&s.fit[0][3][j], v);
    }
    __syncthreads();
    if (has) {
      const int v = qe - midrange(s.fit[0][2], s.fit[0][3], j);
      atomicMax(&s.fit[1][0][i], v);
      atomicMin(&s.fit[1][1][i], v);
    }
    __syncthreads();
    if (has) {
      const int v = qe - midrange(s.fit[1][0], s.fit[1][1], i);
      atomicMax(&s.fit[1][2][j], v);
      atomicMin(&s.fit[1][3][j], v);
    }
    __syncthreads();
    {
      const int r = PWGS - 1 - tid;   // threads holding no support entry unless the list is full
      if (r < D) {
        Py[r] = s.fit[1][0][r] != INT_MIN ? midrange(s.fit[1][0], s.fit[1][1], r) - R[r] : NEG;
        Qy[r] = s.fit[1][2][r] != INT_MIN ? midrange(s.fit[1][2], s.fit[1][3], r) - S[r] : NEG;
      }
    }
    int mr = 0;
    if (c >= 0) {
      const int dl = j - i + D - 1;
      const int sh = midrange(s.fit[1][0], s.fit[1][1], i) + midrange(s.fit[1][2], s.fit[1][3], j);
      const int qk = ys.q(0);
      if (qk >= QSUSP) {
        const int id = qk - QSUSP;
        cand = tg / ldx(s.susp_m[id], s.susp_e[id] + sh);
      } else {
        const int E = xs.ex + s.tgde[dl] - R[i] - S[j];
        const float Dm = mxf * s.tgdm[dl];
        cand = tg / (ldx(b.w[wix], sh) + ldx(Dm, E + sh));
      }
      mr = abs(qe - sh);
    }
    mr = wave_max(mr);
    if (lane == 0) s.redm[wave] = mr;
    __syncthreads();   // new scales visible; every read of the fit arrays done
    mres = 0;
#pragma unroll
    for (int w = 0; w < PNW; ++w) mres = max(mres, s.redm[w]);
    ++mres;
    ysd.fitted = true;
    ysd.rs = false;
    ysd.kern = false;
    ++ysd.sc_gen;
    // room for the residual to drift before the next refit
    ysd.span = max(FAST_SPAN, mres);
    ysd.H = fast_headroom(ysd.span);
    pf.count(PH_N_REFIT);
    pf.mark(PH_REFIT);
  } else {
    mres = spn + 1;
  }
  ysd.mres = mres;
  if (mres > 100) range |= 1;

  // Final pass: the new residual, and y_ij k_Delta,ij as the thread's term of
  // <y, k_Delta>, which the waves idle in the next half step's contraction 2
  // sum (f_reduce_dot).  Each thread overwrites only its own staging entry.
  int et = NEG;
  float mt = 0.0f;
  if (c >= 0) {
    ys.set_res(0, cand);
    f_put_x(b.nx, c, cand, b.nx_bf16, KD);
    if (cc.sc_tag == ysd.sc_gen) {   // no refit in this update: the cached constants hold
      et = cc.edot;
      mt = cand * cc.gdm;
    } else {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      et = Py[i] + Qy[j] + s.tgde[dl];
      mt = cand * s.tgdm[dl];
    }
  }
  s.fit[0][0][tid] = et;
  reinterpret_cast<float*>(&s.fit[0][0][0])[PWGS + tid] = mt;
  __syncthreads();
  pf.mark(PH_FINAL);
}

// <y, k_Delta> from the terms the last update left in s.fit: waves 6 and 7
// (idle in contraction 2) sum four terms per thread with explicit exponents,
// then one record per wave; every thread combines the two records after the
// next workgroup barrier (f_dot_result).
__device__ __forceinline__ void f_reduce_dot(FastSmem& s) {
  const int tid = threadIdx.x, w = tid >> 6;
  if (w < PNW - 2) return;
  const int* te = &s.fit[0][0][0];
  const float* tm = reinterpret_cast<const float*>(te) + PWGS;
  const int t0 = tid - (PNW - 2) * 64;
  ESum a{NEG, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float mk = tm[t0 + 128 * k];
    if (mk > 0.0f) a = esum_add(a, ESum{te[t0 + 128 * k], (double)mk});
  }
  a = wave_esum(a);
  if ((tid & 63) == 0) {
    s.rede[w] = a.e;
    s.redf[w] = a.s;
  }
}
__device__ __forceinline__ ESum f_dot_result(const FastSmem& s) {
  return esum_add(ESum{s.rede[PNW - 2], s.redf[PNW - 2]}, ESum{s.rede[PNW - 1], s.redf[PNW - 1]});
}

// Operand pointers of the BF16 layout.
__device__ __forceinline__ __bf16* fk(FastSmem& s, int off) { return reinterpret_cast<__bf16*>(s.big + off); }

template <int NST>
__device__ __forceinline__ void fast_solve_pair(const PairParams& prm, FastSmem& s, long long pair) {
  constexpr int D = 128;
  using L = FastLayout;
  const int tid = threadIdx.x;
  const int d = prm.d;
  constexpr int KD = 16 * NST;   // d rounded up to the MFMA depth
  const int LDB = KD + 8;
  FProf pf;
  pf.init();

  for (int x = tid; x < 2 * D; x += PWGS) {
    const bool in = x < 2 * D - 1;
    s.tge[x] = in ? prm.ge[x] : NEG;
    s.tkb[x] = in ? prm.kb[x] : -(1 << 27);
    s.tgm[x] = in ? prm.gm[x] : 0.0f;
    s.tgde[x] = in ? prm.gde[x] : NEG;
    s.tgdm[x] = in ? prm.gdm[x] : 0.0f;
    s.tc1[x] = in ? prm.c1[x] : 0.0f;
    s.tcd[x] = in ? prm.cd[x] : 0.0f;
  }
  const float* __restrict__ A = prm.hist_a + (size_t)prm.ia[pair] * d * d;
  const float* __restrict__ B = prm.hist_b + (size_t)prm.ib[pair] * d * d;
  SupList<1> ua, vb;
  bool big_a, big_b, low_a, low_b;
  const double mA = f_build_support(s, A, d, ua, big_a, low_a, s.big);
  const double mB = f_build_support(s, B, d, vb, big_b, low_b, s.big);
  if (big_a || big_b || low_a || low_b) {
    // lists beyond the registers, or mass below the diagonal: the general kernel
    if (tid == 0) prm.redo[pair] = (unsigned char)(prm.only_redo + 1);
    return;
  }
  if (tid == 0) prm.redo[pair] = (unsigned char)prm.only_redo;
  // packed-W index of each thread's support cells (cells on or above the diagonal)
  int wix_a = 0, wix_b = 0;
  {
    const int ca = ua.cell(0), cb = vb.cell(0);
    if (ca >= 0) wix_a = widx(ca / D, ca % D);
    if (cb >= 0) wix_b = widx(cb / D, cb % D);
  }
  const double aD = mB, bD = mA, m = mA + mB;
  if (m <= 0.0) {
    if (tid == 0) {
      prm.cost[pair] = 0.0;
      prm.iters[2 * pair] = 0;
      prm.iters[2 * pair + 1] = 0;
      prm.err[pair] = 0.0f;
      prm.status[pair] = 0;
      if (prm.done) post_done(prm.done, prm.done_tag, pair, 0.0, 0, 0, 0.0f, 0);
    }
    return;
  }

  bool lowp = prm.precision == 1;
  ESum kv{NEG, 0.0};
  FSide su{0, 0.0, 0, HEAD, FAST_SPAN, false, false, false, 0, 0};
  // v = 1: scales 0, residual 1; full headroom, and the span that headroom
  // allows before v's first refit
  FSide sv{0, 1.0, 0, HEAD, 113 - 2 * HEAD, true, false, false, 0, 0};
  FCache cache_u{0, 0, 0.0f, 0, -1, -1}, cache_v{0, 0, 0.0f, 0, -1, -1};
  // v = 1 on every grid cell and on the diagonal bin, in the X format of the
  // first half step
  int p = 0;                                  // BF16 phase: X in slot p
  void* X0 = lowp ? (void*)(s.big + L::S0) : (void*)(s.big + L::FA);
  f_zero_x(X0, lowp, d, KD);
  for (int r = tid; r < D; r += PWGS) {
    s.Pv[r] = r < d ? 0 : NEG;
    s.Qv[r] = r < d ? 0 : NEG;
    s.Pu[r] = NEG;
    s.Qu[r] = NEG;
  }
  __syncthreads();
  for (int c = tid; c < d * d; c += PWGS) {
    const int i = c / d, j = c % d;
    f_put_x(X0, i * D + j, 1.0f, lowp, KD);
    kv = esum_add(kv, ESum{s.tgde[j - i + D - 1], (double)s.tgdm[j - i + D - 1]});
  }
  vb.set_res(0, 1.0f);
  ua.set_q(0, QNONE);
  kv = esum_add(block_esum<PNW>(kv, s.rede, s.reds), ESum{sv.ex, sv.mx});   // (K v)_Delta
  ESum ku{NEG, 0.0};
  bool v_dense = true;

  int t = 0, it_lp = 0, it_hp = 0, bad = 0, range = 0;
  double err = INFINITY;
  if (tid == 0) {
    s.nsusp = 0;
    s.sflag = 0;
  }
  __syncthreads();
  pf.mark(PH_SETUP);

  // The grid part of <y, k_Delta> of the last update waits, as per-thread
  // terms, for the idle waves of the next half step's contraction 2.
  bool pend = false;

  // One half step: y = target / (K x).  After contraction 2 the diagonal-bin
  // entry of K x is complete: (K v)_Delta before a u-update, (K u)_Delta
  // before a v-update.
  auto half = [&](bool u_update, bool lp_now, bool check, bool& stop) {
    FSide& xd = u_update ? sv : su;
    FSide& yd = u_update ? su : sv;
    SupList<1>& ys = u_update ? ua : vb;
    const SupList<1>& xl = u_update ? vb : ua;
    int* Px = u_update ? s.Pv : s.Pu;
    int* Qx = u_update ? s.Qv : s.Qu;
    int* Rx = u_update ? s.Rv : s.Ru;
    int* Sx = u_update ? s.Sv : s.Su;
    int* Py = u_update ? s.Pu : s.Pv;
    int* Qy = u_update ? s.Qu : s.Qv;
    const bool xdense = u_update && v_dense;
    const int H = xd.H;
    pf.count(PH_N_HALF);
    if (!xd.rs) {
      f_compute_RS(s, Px, Qx, d, H, Rx, Sx);
      xd.rs = true;
      xd.kern = false;
      ++xd.rs_gen;
      __syncthreads();
      pf.count(PH_N_SCALES);
      pf.mark(PH_SCALES);
    }
    FBufs bf;
    if (lp_now) {
      __bf16* K1 = fk(s, u_update ? L::K1V : L::K1U);
      __bf16* K2 = fk(s, u_update ? L::K2V : L::K2U);
      char* sx = s.big + (p ? L::S1 : L::S0);
      char* so = s.big + (p ? L::S0 : L::S1);
      if (!xd.kern) {
        int* X7 = reinterpret_cast<int*>(so);   // free until contraction 1 writes T^T there
        for (int r = tid; r < D; r += PWGS) {
          X7[r] = min(max(Px[r], -(1 << 20)), 1 << 20) << 7;
          X7[128 + r] = min(max(Qx[r], -(1 << 20)), 1 << 20) << 7;
        }
        __syncthreads();
        f_build_bf16(s, X7, Rx, Sx, d, KD, LDB, K1, K2);
        xd.kern = true;
        __syncthreads();
        pf.count(PH_N_BUILD);
        pf.mark(PH_BUILD);
      }
      f_c1_bf16<NST>(reinterpret_cast<const __bf16*>(sx), K2, reinterpret_cast<__bf16*>(so), d, LDB, !xdense);
      __syncthreads();
      pf.mark(PH_C1);
      if (pend) f_reduce_dot(s);
      f_c2_bf16<NST>(K1, reinterpret_cast<const __bf16*>(so), reinterpret_cast<float*>(sx), d, LDB);
      bf.w = reinterpret_cast<float*>(sx);   // over the dead X
      bf.stage = reinterpret_cast<char*>(&s.fit[0][0][0]);
      bf.nx = so;                             // over the dead T^T
      bf.nx_bf16 = true;
    } else {
      float* Xf = reinterpret_cast<float*>(s.big + L::FA);
      float* Tf = reinterpret_cast<float*>(s.big + L::FB);
      float* Wf = reinterpret_cast<float*>(s.big + L::FC);
      f_c1_fp32<false>(s, Xf, Tf, Qx, Sx, d, KD, !xdense);
      __syncthreads();
      pf.mark(PH_C1);
      if (pend) f_reduce_dot(s);
      f_c2_fp32<false>(s, Tf, Wf, Px, Rx, d, KD);
      bf.w = Wf;
      bf.stage = reinterpret_cast<char*>(&s.fit[0][0][0]);
      bf.nx = Xf;
      bf.nx_bf16 = false;
    }
    if (tid == 0) {
      s.nsusp = 0;
      s.sflag = 0;
    }
    __syncthreads();
    pf.mark(PH_C2);
    if (pend) {
      const ESum dp = f_dot_result(s);
      if (u_update) kv = esum_add(dp, ESum{sv.ex, sv.mx});
      else ku = esum_add(dp, ESum{su.ex, su.mx});
      pend = false;
    }
    const double errD = (u_update && check) ? fabs(ldxd(su.mx * kv.s, su.ex + kv.e) - aD) : 0.0;
    double e = 0.0;
    const bool lp_before = lowp;
    // The switch to FP32 is decided by the error check inside a u-update; the
    // update then still writes the new residual in BF16, and it is rewritten
    // here in the FP32 layout (whose X lies over the v-side kernels, unused
    // from now on; the slots holding this update's K x are not touched).
    f_update(s, bf, ys, u_update ? wix_a : wix_b, u_update ? cache_u : cache_v, lp_now, xl, xdense, d, KD, xd, H,
             Px, Qx, Rx, Sx, Py, Qy, yd, check, e, stop, bad, range,
             errD, m, prm.tol, prm.switch_tol, lowp, t, prm.max_iter, pf);
    if (check) err = e;
    pend = !stop;
    if (!stop && lp_before && !lowp) {
      float* Xf = reinterpret_cast<float*>(s.big + L::FA);
      f_zero_x(Xf, false, d, KD);
      __syncthreads();
      const int c = ys.cell(0);
      if (c >= 0) f_put_x(Xf, c, ys.res(0), false, KD);
      __syncthreads();
    }
    // (the update's last barrier orders its writes of the new X before the
    // next contraction reads them)
    if (lp_now) p ^= 1;
  };

  for (;;) {
    // u-update: u = a / K v, after checking the marginal error of (u, v).
    const bool lp_now = lowp;
    bool stop = false;
    half(true, lp_now, t >= 1, stop);   // also completes kv = (K v)_Delta
    if (stop || bad) break;
    if (range & 2) break;
    su.ex = -kv.e;
    su.mx = aD / kv.s;
    // v-update: v = b / K^T u (K is symmetric); completes ku = (K u)_Delta
    bool nostop = false;
    half(false, lowp, false, nostop);
    v_dense = false;
    sv.ex = -ku.e;
    sv.mx = bD / ku.s;
    ++t;
    if (lp_now) ++it_lp;
    else ++it_hp;
    if (bad) break;
    if (range & 2) break;
  }
  if (range & 2) {
    // the LDS suspect list overflowed: the general kernel solves the pair
    if (tid == 0) prm.redo[pair] = (unsigned char)(prm.only_redo + 1);
    return;
  }

  // Transport cost of Proposition 3 for (u_t, v_t), FP32 contractions and FP64
  // sums, with the kernels of (Pv, Qv) (Rv, Sv are current: the last half step
  // applied K to v) and the suspects of that half step recomputed exactly.
  float* Xf = reinterpret_cast<float*>(s.big + L::FA);
  float* Tf = reinterpret_cast<float*>(s.big + L::FB);
  float* Wf = reinterpret_cast<float*>(s.big + L::FC);
  __syncthreads();
  f_zero_x(Xf, false, d, KD);
  __syncthreads();
  if (v_dense) {
    for (int c = tid; c < d * d; c += PWGS) f_put_x(Xf, (c / d) * D + (c % d), 1.0f, false, KD);
  } else {
    const int c = vb.cell(0);
    if (c >= 0) f_put_x(Xf, c, vb.res(0), false, KD);
  }
  __syncthreads();
  double g = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) f_c1_fp32<false>(s, Xf, Tf, s.Qv, s.Sv, d, KD, !v_dense);
    else f_c1_fp32<true>(s, Xf, Tf, s.Qv, s.Sv, d, KD, !v_dense);
    __syncthreads();
    if (pass == 0) f_c2_fp32<true>(s, Tf, Wf, s.Pv, s.Rv, d, KD);
    else f_c2_fp32<false>(s, Tf, Wf, s.Pv, s.Rv, d, KD);
    __syncthreads();
    const int c = ua.cell(0);
    if (c >= 0 && ua.q(0) < QSUSP) {
      const float r = ua.res(0);
      if (r > 0.0f) {
        const int i = c / D, j = c % D;
        g += ldxd((double)r * (double)Wf[wix_a], s.Pu[i] + s.Qu[j] + s.Rv[i] + s.Sv[j]);
      }
    }
    __syncthreads();
  }
  const int ns = bad ? 0 : min(s.nsusp, FAST_MAXSUSP);
  if (ns > 0) {
    int* xcell = &s.fit[0][0][0];
    float* xres = reinterpret_cast<float*>(xcell + PWGS);
    if (!v_dense) {
      const int c = vb.cell(0);
      xcell[tid] = c;
      xres[tid] = c >= 0 ? vb.res(0) : 0.0f;
    }
    __syncthreads();
    f_exact<true, false>(s, xcell, xres, v_dense, d, s.Pv, s.Qv, s.Rv, s.Sv, ns, 0, 0.0f);
    const int qk = ua.q(0);
    if (qk >= QSUSP) {
      const float r = ua.res(0);
      if (r > 0.0f) {
        const int c = ua.cell(0), i = c / D, j = c % D;
        const int id = qk - QSUSP;
        g += ldxd((double)r * (double)s.susp_m[id], s.susp_e[id] + s.Pu[i] + s.Qu[j]);
      }
    }
  }
  {
    const int c = ua.cell(0);
    if (c >= 0) {
      const float r = ua.res(0);
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      if (r > 0.0f)
        g += ldxd(sv.mx * (double)r * (double)s.tgdm[dl] * (double)s.tcd[dl], sv.ex + s.Pu[i] + s.Qu[j] + s.tgde[dl]);
    }
  }
  {
    const int c = vb.cell(0);
    if (c >= 0) {
      const float r = vb.res(0);
      if (!v_dense && r > 0.0f) {
        const int i = c / D, j = c % D, dl = j - i + D - 1;
        g += ldxd(su.mx * (double)r * (double)s.tgdm[dl] * (double)s.tcd[dl], su.ex + s.Pv[i] + s.Qv[j] + s.tgde[dl]);
      }
    }
  }
  const double cost = block_sum<PNW>(g, s.red);
  if (tid == 0) {
    int st = 0;
    if (!(err <= prm.tol)) st |= 1;
    if (bad || !isfinite(cost)) st |= 2;
    if (range) st |= 4;
    prm.cost[pair] = bad ? NAN : cost;
    prm.iters[2 * pair] = it_lp;
    prm.iters[2 * pair + 1] = it_hp;
    prm.err[pair] = (float)err;
    prm.status[pair] = st;
    if (prm.done && !(st & 6)) post_done(prm.done, prm.done_tag, pair, cost, it_lp, it_hp, (float)err, st);
  }
  pf.mark(PH_COST);
  pf.count(PH_N_PAIRS);
  pf.commit();
}

// One workgroup per pair (pair perm[b] when a launch order is given).  NST =
// ceil(d / 16) MFMA steps per contraction: 5, 6 or 7 for the grids 65 .. 100.
template <int NST>
__global__ __launch_bounds__(PWGS) void sinkhorn_fast_kernel(PairParams prm) {
  __shared__ FastSmem s;
  const long long pair = prm.perm ? prm.perm[blockIdx.x] : blockIdx.x;
  fast_solve_pair<NST>(prm, s, pair);
}

constexpr int FAST_DMIN = 65;   // smaller grids take the 64-padded layout of the general kernel

}  // namespace pdsink
