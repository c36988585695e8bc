// Fused per-pair Sinkhorn kernel: Algorithm 1 of Lacombe, Cuturi, Oudot
// (NeurIPS 2018) on the d x d grid plus the diagonal bin.  One workgroup of
// 8 waves per pair; every iterate stays in LDS and registers for the whole
// solve.
//
// Work layout.  The grid is padded to D = 32, 64 or 128 and cut into 32 x 32
// tiles; wave w computes tiles w, w + 8, ... of both contractions of
// Proposition 2 on the matrix cores.  Everything elementwise (the scaling
// update, the marginal error, the diagonal-bin terms, the refit of the
// scales) runs over compact lists of the two histograms' supports: u is zero
// off supp(a) and v off supp(b), so only those cells carry state.  Support
// entry s of a side belongs to thread s mod 512, register slot s / 512.
// The lists are built once per pair with a block prefix scan (deterministic
// order), and the contraction result reaches them through one LDS tile store.
//
// Numerical representation (the paper is silent on stabilisation).  A scaling
// vector x on the grid is stored as x_ij = 2^(P_i + Q_j) * xt_ij with integer
// row/column log2 scales P, Q (int32) and an FP32 residual xt; the diagonal
// entry as m * 2^e.  Because 2^(P_i + Q_j) factors over rows and columns, the
// separable K application of Proposition 2 stays a pair of 1-D contractions:
//   K x (grid) = 2^(R_i + S_j) * (kt1 * Xt * kt2^T)_ij + x_Delta k_Delta,ij
// with per-row/column "absorbed" 1-D kernels
//   kt1[i][k] = 2^(P_k + g(i-k) - R_i),  R_i = max_k (P_k + ge(i-k)) - H,
// g(delta) = -(|delta|/d)^p / gamma * log2(e), and kt2 likewise from Q.  The
// entries are at most 2^H: H octaves of headroom (chosen from the input's
// residual range so nothing overflows) push everything the contractions drop
// far below the natural scale.  Each kernel entry is built exactly as
// ldexp(mantissa(delta), integer exponent) from per-context tables, without
// transcendental instructions.
//
// After each half step the new scaling y = target / (K x) is re-expressed:
// natural scales (-R, -S) plus integer offsets (rho, sigma) from two sweeps of
// row/column centring of the per-cell log2 estimates, which keeps the residual
// within a few tens of octaves (the non-separable part of the potentials).
// This is exact re-representation of the same iterates: only FP32 rounding of
// the contractions and divisions remains.
//
// The two separable normalisations cannot see every four-index product: at a
// few cells all terms of (K x)_ij can still fall out of range.  Cells whose
// normalised value is below the trusted level ("suspects", 2^-40 relative
// error budget) are recomputed exactly, as a sum over the input's support with
// explicit exponents, and those exact values feed the update, the marginal
// error and the transport cost.
#pragma once
#include <climits>

#include "pdsink_device.h"

namespace pdsink {

struct PairParams {
  int d;
  double tol;
  int max_iter;
  int precision;       // 0 = FP32, 1 = BF16 contractions until err <= switch_tol, then FP32
  double switch_tol;
  // per-context tables, index delta + (D - 1), delta in [-(D-1), D-1]
  const int* ge;       // kernel exponent, ceil(g(delta))
  const float* gm;     // kernel mantissa 2^(g - ge) in (0.5, 1]; 0 for |delta| >= d
  const int* gde;      // diagonal-kernel exponent for delta = j - i
  const float* gdm;
  const float* c1;     // (|delta|/d)^p
  const float* cd;     // 2 (|delta|/(2d))^p
  const int* kb;       // BF16 kernel word: (e << 7) | m7 with 2^g = (1 + m7/128) 2^(e - 1), exactly
                       // bf16(gm) 2^ge; -(2^27) for |delta| >= d
  // the batch
  const float* hist_a;
  const float* hist_b;
  const int* ia;
  const int* ib;
  long long n_pairs;
  double* cost;
  int* iters;
  float* err;
  int* status;
  // support-size routing between kernel variants: a launch at level L handles
  // the pairs with redo[q] == L (level 0: every pair, whatever redo holds) and
  // sets redo[q] = L + 1, leaving the outputs alone, for a pair whose support
  // does not fit the variant; else it sets redo[q] = L.
  unsigned char* redo;
  int only_redo;
  // support lists of the global-list variant: list_stride bytes per workgroup
  char* lists;
  size_t list_stride;
  // operand slices (grids beyond 128): GlobalOps<D>::BYTES per workgroup
  char* ops;
  // optional warm start of v (WarmState per pair): read when state_in, and
  // written with the final v
  char* state;
  int state_in;
  // optional gradient terms of Proposition 5, [n_pairs][d * d]: log u + log
  // v_Delta on the cells of supp(a)
  double* gout;
  // optional device flag: when it is set the launch does nothing (the
  // barycenter's outer steps after its stopping test)
  const int* stop;
  // optional per-pair completion records (host-mapped or device memory): a
  // pair whose result is final here (no NONFINITE or RANGE flag, which the
  // log-domain launch takes up) posts it with done_tag
  DoneRec* done;
  unsigned done_tag;
  // optional error-control bounds of section 3 per pair (upper: rounded plan,
  // lower: c-transform dual), with the ground exponent and gamma they need
  double* upper;
  double* lower;
  double gamma;
  double p;
  // optional launch order of the register-list launch: workgroup b solves
  // pair perm[b] (NULL: pair b)
  const int* perm;
};

constexpr int PWGS = 512;      // threads per pair workgroup
constexpr int PNW = PWGS / 64; // its waves
constexpr int MAXSUSP = 256;   // suspects handled per half step
constexpr int QSUSP = 1 << 28; // per-entry marker: entry is suspect number q - QSUSP
constexpr int HEAD = 40;       // kernel headroom octaves for an input residual within 2^20
constexpr int SUSP_MARGIN = 24; // octaves between the dropped-term bound and a trusted value

template <int D>
struct Cfg {
  static constexpr int NT = D / 32;          // tiles per grid dimension
  static constexpr int NTILES = NT * NT;     // waves with a contraction tile
  static constexpr int LDF = D + 1;          // FP32 row stride: rows start in different banks
  static constexpr int LDB = D + 8;          // BF16 row stride: 16-byte aligned rows
  static constexpr int TPR = PWGS / (2 * D); // threads per (side, row) in compute_RS
};

// Operand buffers of the contractions and the support-list staging area:
// in LDS for D <= 128; for larger grids they live in a per-workgroup slice of
// the workspace (GlobalOps) and the LDS part is empty.
template <int D, bool G = (D > 128)>
struct OpsLds {
  using C = Cfg<D>;
  union {
    struct {
      float X[D * C::LDF];    // input residual (A operand of contraction 1)
      float T[D * C::LDF];    // X kt2^T, row-major [k][j]; then the K x tile store
    } f;
    struct {
      __bf16 X[D * C::LDB];
      __bf16 Tt[D * C::LDB];  // X kt2^T, transposed [j][k] (B operand of contraction 2)
      __bf16 K1[D * C::LDB];  // kt1 [i][k]
      __bf16 K2[D * C::LDB];  // kt2 [j][l]
    } b;
    struct {
      int cell[D * D];        // support-list staging at pair start
      float val[D * D];
    } st;
  } u;
};
template <int D>
struct OpsLds<D, true> {};

// Layout of the global operand slice (grids beyond 128): the same buffers as
// the LDS union, plus a K x buffer of its own.
template <int D>
struct GlobalOps {
  using C = Cfg<D>;
  static constexpr size_t F = (size_t)2 * D * C::LDF * 4, B = (size_t)4 * D * C::LDB * 2, S = (size_t)2 * D * D * 4;
  static constexpr size_t UNION = ((F > B ? (F > S ? F : S) : (B > S ? B : S)) + 255) & ~(size_t)255;
  static constexpr size_t W = UNION;                                   // K x buffer, FP32 [D][LDF]
  static constexpr size_t BYTES = (W + (size_t)D * C::LDF * 4 + 255) & ~(size_t)255;
};

template <int D>
struct PairSmem : OpsLds<D> {
  alignas(16) int tge[2 * D];
  int tgde[2 * D], tkb[2 * D];
  float tgm[2 * D], tgdm[2 * D], tc1[2 * D], tcd[2 * D];
  alignas(16) int Pu[D];
  alignas(16) int Qu[D];
  alignas(16) int Pv[D];
  alignas(16) int Qv[D];
  int R[D], S[D];
  // BF16 kernel build: the input scales clamped to +-2^20 and shifted to the
  // exponent field of a BF16 word
  alignas(16) int P7[D];
  alignas(16) int Q7[D];
  // refit extrema: [sweep][row max, row min, column max, column min][D]
  alignas(16) int fit[2][4][D];   // also the FP64 cost tables of the bounds
  int sflag;               // bit 0: a suspect's exact value vanished
  double red[PNW];
  double reds[PNW];
  int rede[PNW];
  int redi[PNW];
  int nsusp;
  int susp_cell[MAXSUSP];
  int susp_e[MAXSUSP];     // value = susp_m * 2^susp_e (natural scale, or absolute for the cost)
  float susp_m[MAXSUSP];
  int* gsusp;              // global-list variant: suspect arrays of capacity D^2 in the workspace
  int xs_cell[PWGS];       // staging of a register support list for the exact path
  float xs_res[PWGS];
  char* gops;              // global operand slice (grids beyond 128)
};

// Operand buffers (LDS union, or the global slice beyond D = 128).
template <int D>
__device__ __forceinline__ float* opXf(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.f.X;
  else return reinterpret_cast<float*>(s.gops);
}
template <int D>
__device__ __forceinline__ float* opTf(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.f.T;
  else return reinterpret_cast<float*>(s.gops) + D * Cfg<D>::LDF;
}
template <int D>
__device__ __forceinline__ __bf16* opXb(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.b.X;
  else return reinterpret_cast<__bf16*>(s.gops);
}
template <int D>
__device__ __forceinline__ __bf16* opTtb(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.b.Tt;
  else return reinterpret_cast<__bf16*>(s.gops) + D * Cfg<D>::LDB;
}
template <int D>
__device__ __forceinline__ __bf16* opK1b(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.b.K1;
  else return reinterpret_cast<__bf16*>(s.gops) + 2 * D * Cfg<D>::LDB;
}
template <int D>
__device__ __forceinline__ __bf16* opK2b(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.b.K2;
  else return reinterpret_cast<__bf16*>(s.gops) + 3 * D * Cfg<D>::LDB;
}
template <int D>
__device__ __forceinline__ int* stCell(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.st.cell;
  else return reinterpret_cast<int*>(s.gops);
}
template <int D>
__device__ __forceinline__ float* stVal(PairSmem<D>& s) {
  if constexpr (D <= 128) return s.u.st.val;
  else return reinterpret_cast<float*>(s.gops) + D * D;
}

// The K x tile buffer: FP32 [D][LDF], after contraction 2.  In LDS it lies
// over storage that is dead by then (T in FP32 mode; Tt and K1 in BF16
// mode); beyond D = 128 it has its own place in the global slice.
template <int D>
__device__ __forceinline__ float* wbuf(PairSmem<D>& s, bool bf16) {
  if constexpr (D <= 128) return bf16 ? reinterpret_cast<float*>(s.u.b.Tt) : s.u.f.T;
  else return reinterpret_cast<float*>(s.gops + GlobalOps<D>::W);
}

// Suspect arrays: in LDS (MAXSUSP entries) for register lists; in the
// workspace slot (D^2 entries: every cell can be one) for global lists.
template <int D, int SPT>
__device__ __forceinline__ int* suspCell(PairSmem<D>& s) {
  if constexpr (SPT > 0) return s.susp_cell;
  else return s.gsusp;
}
template <int D, int SPT>
__device__ __forceinline__ int* suspE(PairSmem<D>& s) {
  if constexpr (SPT > 0) return s.susp_e;
  else return s.gsusp + D * D;
}
template <int D, int SPT>
__device__ __forceinline__ float* suspM(PairSmem<D>& s) {
  if constexpr (SPT > 0) return s.susp_m;
  else return reinterpret_cast<float*>(s.gsusp + 2 * D * D);
}
template <int D, int SPT>
__device__ __forceinline__ constexpr int suspCap() {
  return SPT > 0 ? MAXSUSP : D * D;
}

// Kernel headroom for an input whose residual spans +-mres octaves.
__device__ __forceinline__ int headroom(int mres) { return max(0, min(HEAD, HEAD + 20 - mres)); }

// Prefix sum over the workgroup (deterministic): returns the exclusive prefix
// of v and the total.
__device__ __forceinline__ int block_scan(int v, int* red, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) red[w] = x;
  __syncthreads();
  int before = 0, tot = 0;
  for (int i = 0; i < PNW; ++i) {
    const int r = red[i];
    if (i < w) before += r;
    tot += r;
  }
  total = tot;
  return before + x - v;
}

// R_i = max_k (P_k + ge(i - k)) - H over the input's rows k, and S_j from Q
// likewise; rows i >= d get BIG so that their kernel rows are exactly zero.
// Each thread takes 4 consecutive output rows of one side and a slice of k
// (NPART adjacent lanes share a row block); the 4 table entries it needs
// slide by one position per k, so each k costs one table read.  Rows of an
// empty input (every P_k = NEG) get 0: all their kernel entries vanish anyway.
template <int D>
__device__ __forceinline__ void compute_RS(PairSmem<D>& s, const int* P, const int* Q, int d, int H) {
  constexpr int NRB = 2 * D / 4;         // (side, 4-row block) combinations
  constexpr int NPART = PWGS / NRB;      // lanes per combination
  constexpr int KPT = D / NPART;         // k values per lane
  static_assert(NPART * NRB == PWGS && KPT * NPART == D && NPART <= 64, "compute_RS layout");
  const int combo = threadIdx.x / NPART, part = threadIdx.x % NPART;
  const bool rows = combo < NRB / 2;
  const int i0 = 4 * (rows ? combo : combo - NRB / 2);
  const int* X = rows ? P : Q;
  const int k0 = part * KPT;
  int b0 = NEG, b1 = NEG, b2 = NEG, b3 = NEG;
  if constexpr (KPT % 4 == 0 && KPT <= 16) {
    // the KPT + 3 table words ge(i0 + r - k) the thread needs start at a
    // 16-byte boundary: wv[m] = ge at index start + m, m = KPT - 1 + r - t
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
  } else {
    const int* tw = s.tge + i0 - k0 + D - 1;   // tw[r - (k - k0)] = ge(i0 + r - k)
    int w0 = tw[0], w1 = tw[1], w2 = tw[2], w3 = tw[3];
#pragma unroll
    for (int t = 0; t < KPT; ++t) {
      const int x = X[k0 + t];
      b0 = max(b0, x + w0);
      b1 = max(b1, x + w1);
      b2 = max(b2, x + w2);
      b3 = max(b3, x + w3);
      if (t + 1 < KPT) {
        w3 = w2;
        w2 = w1;
        w1 = w0;
        w0 = tw[-(t + 1)];
      }
    }
  }
  if constexpr (NPART > 1) {
    b0 = group_max<NPART>(b0);
    b1 = group_max<NPART>(b1);
    b2 = group_max<NPART>(b2);
    b3 = group_max<NPART>(b3);
  }
  if (part == 0) {
    int* out = (rows ? s.R : s.S) + i0;
    const int bb[4] = {b0, b1, b2, b3};
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = i0 + r < d ? (bb[r] <= NEG / 2 ? 0 : bb[r] - H) : BIG;
  }
}

template <int D, bool WEIGHTED>
__device__ __forceinline__ float kentry(const PairSmem<D>& s, int i, int k, const int* P, int Ri) {
  const int idx = i - k + D - 1;
  float v = ldx(s.tgm[idx], P[k] + s.tge[idx] - Ri);
  if (WEIGHTED) v *= s.tc1[idx];
  return v;
}

// BF16 kernels of one application into LDS: K1[i][k] from P (as s.P7) and R,
// K2[j][l] from Q (as s.Q7) and S, 16 consecutive entries of one row of both
// per thread and step.  An entry bf16(gm) 2^(P_k + ge - R_i) is assembled
// directly as a BF16 bit pattern by adding the exponent shift to the table
// word; results below the smallest normal BF16 (2^-126, at least 2^-166
// below the row maximum) become 0 or a subnormal pattern.
template <int D>
__device__ __forceinline__ void build_kernels_bf16(PairSmem<D>& s, int d) {
  constexpr int LDB = Cfg<D>::LDB;
  // Rows i >= d feed only output rows/columns that are never read, so they
  // are skipped; chunks of columns k >= d hold exact zeros (P_k = NEG) and
  // are written without table reads.
  const int nch = (d + 15) / 16;          // 16-entry chunks per row that touch k < d
  // item = chunk * d + row: adjacent lanes take adjacent rows of one chunk, so
  // their table reads hit adjacent LDS banks; both kernels of the row share
  // the 16 table words (kt1 with P and R, kt2 with Q and S).
  for (int item = threadIdx.x; item < nch * d; item += PWGS) {
    const int i = item % d, k0 = 16 * (item / d);
    const int* tw = s.tkb + i - k0 + D - 1;    // tw[-t] = word of delta = i - (k0 + t)
    int wd[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) wd[t] = tw[-t];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      // word = table word + ((X_k - R_i + 126) << 7), clamped to [0, 0x7FFF]:
      // below the smallest normal the clamp leaves 0 or a BF16 subnormal
      // pattern (< 2^-126), either negligible against the row maximum.  X_k
      // is clamped to +-2^20 beforehand (X7), so that no sum overflows.
      const int* X7 = (side == 0 ? s.P7 : s.Q7) + k0;
      const int base7 = (126 - (side == 0 ? s.R : s.S)[i]) << 7;
      const int4 xa = *reinterpret_cast<const int4*>(X7), xb = *reinterpret_cast<const int4*>(X7 + 4);
      const int4 xc = *reinterpret_cast<const int4*>(X7 + 8), xd = *reinterpret_cast<const int4*>(X7 + 12);
      const int xs[16] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w,
                          xc.x, xc.y, xc.z, xc.w, xd.x, xd.y, xd.z, xd.w};
      unsigned int pk[8];
#pragma unroll
      for (int t = 0; t < 16; t += 2) {
        const int v0 = min(max(wd[t] + xs[t] + base7, 0), 0x7FFF);
        const int v1 = min(max(wd[t + 1] + xs[t + 1] + base7, 0), 0x7FFF);
        pk[t >> 1] = (unsigned)v0 | ((unsigned)v1 << 16);
      }
      uint4* dst = reinterpret_cast<uint4*>((side == 0 ? opK1b<D>(s) : opK2b<D>(s)) + i * LDB + k0);
      dst[0] = uint4{pk[0], pk[1], pk[2], pk[3]};
      dst[1] = uint4{pk[4], pk[5], pk[6], pk[7]};
    }
  }
  const int nz = D / 16 - nch;            // all-zero chunks per row
  for (int item = threadIdx.x; item < 2 * nz * d; item += PWGS) {
    const int i = item % d, sc = item / d;
    const bool first = sc < nz;
    const int k0 = 16 * (nch + (first ? sc : sc - nz));
    uint4* dst = reinterpret_cast<uint4*>((first ? opK1b<D>(s) : opK2b<D>(s)) + i * LDB + k0);
    dst[0] = uint4{0u, 0u, 0u, 0u};
    dst[1] = uint4{0u, 0u, 0u, 0u};
  }
}

// Tile schedules.  Histogram supports of persistence diagrams lie on or above
// the diagonal (birth <= death), so when every support of the pair does
// ("tri"), u and v vanish below it: contraction 1 skips the l-blocks below a
// row block of X (X[k][l] = 0 for l < k), and contraction 2 computes only the
// output tiles on or above the diagonal, the only cells the update, the error
// and the cost read.  Tiles are spread so that the matrix cores of the four
// SIMDs (waves w and w + 4 share one) get equal work.

// Contraction 1 tile `u` (0 or 1) of wave w: returns false when there is none.
template <int D>
__device__ __forceinline__ bool xk_tile(int w, int u, int& tk, int& tj) {
  constexpr int NT = Cfg<D>::NT;
  if constexpr (NT == 4) {
    // column tj = w mod 4 per SIMD; row blocks {0, 3} and {1, 2} per wave:
    // 5 of the 10 trimmed l-blocks of that column each.
    tj = w & 3;
    tk = (w < 4) ? (u == 0 ? 0 : 3) : (u == 0 ? 1 : 2);
    return true;
  } else {
    const int tile = w + u * PNW;
    tk = tile / NT;
    tj = tile % NT;
    return tile < NT * NT;
  }
}

// Contraction 2 tile `u` of wave w among the upper tiles (tri) or all tiles.
template <int D>
__device__ __forceinline__ bool kt_tile(int w, int u, bool tri, int& ti, int& tj) {
  constexpr int NT = Cfg<D>::NT;
  int tile = w + u * PNW;
  if (!tri) {
    ti = tile / NT;
    tj = tile % NT;
    return tile < NT * NT;
  }
  if (tile >= NT * (NT + 1) / 2) return false;
  ti = 0;
  while (tile >= NT - ti) {
    tile -= NT - ti;
    ++ti;
  }
  tj = ti + tile;
  return true;
}

// The same over a grid of nt x nt tiles (nt known at run time).
__device__ __forceinline__ bool kt_tile_n(int w, int u, bool tri, int nt, int& ti, int& tj) {
  int tile = w + u * PNW;
  if (!tri) {
    ti = tile / nt;
    tj = tile % nt;
    return tile < nt * nt;
  }
  if (tile >= nt * (nt + 1) / 2) return false;
  ti = 0;
  while (tile >= nt - ti) {
    tile -= nt - ti;
    ++ti;
  }
  tj = ti + tile;
  return true;
}

// Contraction 1 of Proposition 2 for the calling wave's tiles (tk, tj):
//   T[k][j] = sum_l X[k][l] * kt2[j][l]   (kt2 times c1 when WEIGHTED: the m of Prop. 3)
// With `trim`, X is zero below the diagonal and l starts at the tile's first row.
template <int D, bool BF16, bool WEIGHTED>
__device__ __forceinline__ void gemm_xk(PairSmem<D>& s, const int* Q, bool trim) {
  constexpr int LDF = Cfg<D>::LDF, LDB = Cfg<D>::LDB;
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index, held in a scalar register
  if constexpr (!BF16 && Cfg<D>::NT == 4) {
    // As below for FP32: one kernel entry kt2[j][l] feeds both tiles.
    int tk0, tk1, tj;
    xk_tile<D>(w, 0, tk0, tj);
    xk_tile<D>(w, 1, tk1, tj);
    const int j = tj * 32 + lr, r0 = tk0 * 32 + lr, r1 = tk1 * 32 + lr;
    const int lb0 = trim ? tk0 * 32 : 0, lb1 = trim ? tk1 * 32 : 0;
    const int Sj = s.S[j];
    const float* X = s.u.f.X;
    floatx16 acc0 = {}, acc1 = {};
#pragma unroll 4
    for (int l0 = lb0; l0 < lb1; l0 += 2) {
      const int l = l0 + lk;
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(X[r0 * LDF + l], kentry<D, WEIGHTED>(s, j, l, Q, Sj), acc0, 0, 0, 0);
    }
#pragma unroll 4
    for (int l0 = lb1; l0 < D; l0 += 2) {
      const int l = l0 + lk;
      const float b = kentry<D, WEIGHTED>(s, j, l, Q, Sj);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(X[r0 * LDF + l], b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(X[r1 * LDF + l], b, acc1, 0, 0, 0);
    }
    mfma_drain();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      s.u.f.T[(tk0 * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc0[r];
      s.u.f.T[(tk1 * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc1[r];
    }
    return;
  }
  if constexpr (BF16 && Cfg<D>::NT == 4) {
    // The wave's two tiles share the column block tj, hence the kt2 operand:
    // one chain alone while only the upper tile's l range is live, then both
    // chains from one read of kt2 (each accumulator sees the same sequence of
    // steps as when the tiles run one after the other).
    int tk0, tk1, tj;
    xk_tile<D>(w, 0, tk0, tj);
    xk_tile<D>(w, 1, tk1, tj);
    const int j = tj * 32 + lr;
    const int lb0 = trim ? tk0 * 32 : 0, lb1 = trim ? tk1 * 32 : 0;
    const __bf16* xa0 = s.u.b.X + (tk0 * 32 + lr) * LDB + 8 * lk;
    const __bf16* xa1 = s.u.b.X + (tk1 * 32 + lr) * LDB + 8 * lk;
    const __bf16* kb = s.u.b.K2 + j * LDB + 8 * lk;
    floatx16 acc0 = {}, acc1 = {};
#pragma unroll 2
    for (int l0 = lb0; l0 < lb1; l0 += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(xa0 + l0);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(kb + l0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc0, 0, 0, 0);
    }
#pragma unroll 2
    for (int l0 = lb1; l0 < D; l0 += 16) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(kb + l0);
      const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(xa0 + l0);
      const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(xa1 + l0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b, acc1, 0, 0, 0);
    }
    mfma_drain();
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bf16x4 v0 = {(__bf16)acc0[4 * q], (__bf16)acc0[4 * q + 1], (__bf16)acc0[4 * q + 2],
                         (__bf16)acc0[4 * q + 3]};
      *reinterpret_cast<bf16x4*>(s.u.b.Tt + j * LDB + tk0 * 32 + 8 * q + 4 * lk) = v0;
      const bf16x4 v1 = {(__bf16)acc1[4 * q], (__bf16)acc1[4 * q + 1], (__bf16)acc1[4 * q + 2],
                         (__bf16)acc1[4 * q + 3]};
      *reinterpret_cast<bf16x4*>(s.u.b.Tt + j * LDB + tk1 * 32 + 8 * q + 4 * lk) = v1;
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int tk, tj;
    if (!xk_tile<D>(w, u, tk, tj)) break;
    const int row = tk * 32 + lr, j = tj * 32 + lr;
    const int lbeg = trim ? tk * 32 : 0;
    floatx16 acc = {};
    if constexpr (BF16) {
      const __bf16* xa = s.u.b.X + row * LDB + 8 * lk;
      const __bf16* kb = s.u.b.K2 + j * LDB + 8 * lk;
#pragma unroll 2
      for (int l0 = lbeg; l0 < D; l0 += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(xa + l0);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(kb + l0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
      mfma_drain();
      // rows r = 4q .. 4q + 3 of the lane's accumulator are 4 consecutive k of
      // Tt's row j: one 8-byte store each
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        const bf16x4 v = {(__bf16)acc[4 * q], (__bf16)acc[4 * q + 1], (__bf16)acc[4 * q + 2], (__bf16)acc[4 * q + 3]};
        *reinterpret_cast<bf16x4*>(s.u.b.Tt + j * LDB + tk * 32 + 8 * q + 4 * lk) = v;
      }
    } else {
      const int Sj = s.S[j];
#pragma unroll 4
      for (int l0 = lbeg; l0 < D; l0 += 2) {
        const int l = l0 + lk;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(s.u.f.X[row * LDF + l], kentry<D, WEIGHTED>(s, j, l, Q, Sj), acc,
                                                   0, 0, 0);
      }
      mfma_drain();
#pragma unroll
      for (int r = 0; r < 16; ++r) s.u.f.T[(tk * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc[r];
    }
  }
}

// Contraction 2 for the calling wave's tiles (ti, tj); after every wave has
// read T, the tiles go to the K x buffer Wb:
//   W[i][j] = sum_k kt1[i][k] * T[k][j]   (kt1 times c1 when WEIGHTED)
// With `tri`, only tiles on or above the diagonal are computed.  Each wave
// runs two independent accumulation chains so that its matrix-core work
// overlaps with the operand reads: its two tiles side by side, or, with one
// tile, the two halves of the k range (added at the end).
template <int D, bool BF16, bool WEIGHTED>
__device__ __forceinline__ void gemm_kt(PairSmem<D>& s, const int* P, float* Wb, bool tri) {
  constexpr int LDF = Cfg<D>::LDF, LDB = Cfg<D>::LDB;
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index, held in a scalar register
  if constexpr (Cfg<D>::NT == 4) {
    if (tri) {
      // The 10 upper tiles: waves 0-3 take two tiles of one row block, which
      // share the kt1 operand, (0,0)+(0,1), (0,2)+(0,3), (1,1)+(1,2),
      // (2,2)+(2,3); waves 4 and 5 take (1,3) and (3,3), each as two
      // accumulation chains over the halves of k; waves 6 and 7 rest.
      floatx16 acc0 = {}, acc1 = {};
      int ti = 0, tj = 0;
      if (w < 4) {
        ti = w < 2 ? 0 : w - 1;
        tj = w == 0 ? 0 : (w == 2 ? 1 : 2);
      } else if (w < 6) {
        ti = w == 4 ? 1 : 3;
        tj = 3;
      }
      const int ia = ti * 32 + lr, ja = tj * 32 + lr;
      if (w < 4) {
        if constexpr (BF16) {
          const __bf16* ka = s.u.b.K1 + ia * LDB + 8 * lk;
          const __bf16* t0 = s.u.b.Tt + ja * LDB + 8 * lk;
          const __bf16* t1 = t0 + 32 * LDB;
#pragma unroll 2
          for (int k0 = 0; k0 < D; k0 += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(ka + k0);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(t0 + k0);
            const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(t1 + k0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
          }
        } else {
          // one kernel entry for both tiles; operands of step k0 + 2 are read
          // while the matrix cores run step k0
          const int Ra = s.R[ia];
          const float* T = s.u.f.T;
          float a = kentry<D, WEIGHTED>(s, ia, lk, P, Ra), b0 = T[lk * LDF + ja], b1 = T[lk * LDF + ja + 32];
          for (int k0 = 0; k0 < D; k0 += 2) {
            const int kn = (k0 + 2 < D ? k0 + 2 : 0) + lk;
            const float na = kentry<D, WEIGHTED>(s, ia, kn, P, Ra), nb0 = T[kn * LDF + ja],
                        nb1 = T[kn * LDF + ja + 32];
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc1, 0, 0, 0);
            a = na;
            b0 = nb0;
            b1 = nb1;
          }
        }
        mfma_drain();
      } else if (w < 6) {
        if constexpr (BF16) {
          const __bf16* ka = s.u.b.K1 + ia * LDB + 8 * lk;
          const __bf16* ta = s.u.b.Tt + ja * LDB + 8 * lk;
#pragma unroll 2
          for (int k0 = 0; k0 < D / 2; k0 += 16) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(ka + k0);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(ta + k0);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(ka + k0 + D / 2);
            const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(ta + k0 + D / 2);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc1, 0, 0, 0);
          }
        } else {
          const int Ra = s.R[ia];
          const float* T = s.u.f.T;
          constexpr int H2 = D / 2;
          float a0 = kentry<D, WEIGHTED>(s, ia, lk, P, Ra), b0 = T[lk * LDF + ja];
          float a1 = kentry<D, WEIGHTED>(s, ia, lk + H2, P, Ra), b1 = T[(lk + H2) * LDF + ja];
          for (int k0 = 0; k0 < H2; k0 += 2) {
            const int kn = (k0 + 2 < H2 ? k0 + 2 : 0) + lk;
            const float na0 = kentry<D, WEIGHTED>(s, ia, kn, P, Ra), nb0 = T[kn * LDF + ja];
            const float na1 = kentry<D, WEIGHTED>(s, ia, kn + H2, P, Ra), nb1 = T[(kn + H2) * LDF + ja];
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc1, 0, 0, 0);
            a0 = na0;
            b0 = nb0;
            a1 = na1;
            b1 = nb1;
          }
        }
        mfma_drain();
#pragma unroll
        for (int r = 0; r < 16; ++r) acc0[r] += acc1[r];
      }
      __syncthreads();
      if (w < 6) {
#pragma unroll
        for (int r = 0; r < 16; ++r) Wb[(ti * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + tj * 32 + lr] = acc0[r];
      }
      if (w < 4) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
          Wb[(ti * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + (tj + 1) * 32 + lr] = acc1[r];
      }
      __syncthreads();
      return;
    }
  }
  int ti0, tj0, ti1, tj1;
  const bool has0 = kt_tile<D>(w, 0, tri, ti0, tj0);
  const bool two = has0 && kt_tile<D>(w, 1, tri, ti1, tj1);
  if (!two) {
    ti1 = ti0;
    tj1 = tj0;
  }
  // chain a: tile 0 over k in [0, len); chain b: tile 1 over [0, len), or
  // tile 0 over [len, D)
  const int len = two ? D : D / 2;
  const int kb = two ? 0 : D / 2;
  floatx16 acc0 = {}, acc1 = {};
  if (has0) {
    const int ia = ti0 * 32 + lr, ja = tj0 * 32 + lr;
    const int ib = ti1 * 32 + lr, jb = tj1 * 32 + lr;
    if constexpr (BF16) {
      const __bf16* ka = s.u.b.K1 + ia * LDB + 8 * lk;
      const __bf16* ta = s.u.b.Tt + ja * LDB + 8 * lk;
      const __bf16* kc = s.u.b.K1 + ib * LDB + 8 * lk + kb;
      const __bf16* tc = s.u.b.Tt + jb * LDB + 8 * lk + kb;
#pragma unroll 2
      for (int k0 = 0; k0 < len; k0 += 16) {
        const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(ka + k0);
        const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(ta + k0);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(kc + k0);
        const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(tc + k0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc1, 0, 0, 0);
      }
    } else {
      // Operands of step k0 + 2 are read while the matrix cores run step k0.
      const int Ra = s.R[ia], Rb = s.R[ib];
      const float* T = s.u.f.T;
      float a0 = kentry<D, WEIGHTED>(s, ia, lk, P, Ra), b0 = T[lk * LDF + ja];
      float a1 = kentry<D, WEIGHTED>(s, ib, lk + kb, P, Rb), b1 = T[(lk + kb) * LDF + jb];
      for (int k0 = 0; k0 < len; k0 += 2) {
        const int kn = (k0 + 2 < len ? k0 + 2 : 0) + lk;
        const float na0 = kentry<D, WEIGHTED>(s, ia, kn, P, Ra), nb0 = T[kn * LDF + ja];
        const float na1 = kentry<D, WEIGHTED>(s, ib, kn + kb, P, Rb), nb1 = T[(kn + kb) * LDF + jb];
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc1, 0, 0, 0);
        a0 = na0;
        b0 = nb0;
        a1 = na1;
        b1 = nb1;
      }
    }
    mfma_drain();
    if (!two) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc0[r] += acc1[r];
    }
  }
  __syncthreads();
  if (has0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Wb[(ti0 * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + tj0 * 32 + lr] = acc0[r];
    if (two) {
#pragma unroll
      for (int r = 0; r < 16; ++r) Wb[(ti1 * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + tj1 * 32 + lr] = acc1[r];
    }
  }
  __syncthreads();
}

// The contractions for grids beyond 128 (operands in the global slice): one
// tile at a time per wave, tiles w, w + 8, ...; the K x buffer has its own
// storage, so each tile is stored as soon as it is done.  Only the tiles that
// hold rows or columns below d are computed, and the depth runs to d rounded
// up to 16: X is zero beyond its d columns and the kernels beyond d rows, and
// nothing reads T or W beyond the tiles of the grid (d = 200: 49 of 64 tiles
// at depth 208 of 256).
// One accumulation chain of nst BF16 MFMA steps over operands in the
// workspace slice (L2-resident): the loads run PFG steps ahead in a rotating
// register buffer, so that several global reads are in flight behind each
// MFMA; the scheduling barriers keep that order.
template <int PFG>
__device__ __forceinline__ void chain_bf16_g(const __bf16* pa, const __bf16* pb, int nst, floatx16& acc) {
  bf16x8 a[PFG], b[PFG];
#pragma unroll
  for (int u = 0; u < PFG; ++u) {
    if (u < nst) {
      a[u] = *reinterpret_cast<const bf16x8*>(pa + 16 * u);
      b[u] = *reinterpret_cast<const bf16x8*>(pb + 16 * u);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  for (int st0 = 0; st0 < nst; st0 += PFG) {
#pragma unroll
    for (int u = 0; u < PFG; ++u) {
      const int st = st0 + u;
      if (st < nst) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[u], b[u], acc, 0, 0, 0);
        if (st + PFG < nst) {
          a[u] = *reinterpret_cast<const bf16x8*>(pa + 16 * (st + PFG));
          b[u] = *reinterpret_cast<const bf16x8*>(pb + 16 * (st + PFG));
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int D, bool BF16, bool WEIGHTED>
__device__ __forceinline__ void gemm_xk_g(PairSmem<D>& s, const int* Q, bool trim, int d) {
  constexpr int LDF = Cfg<D>::LDF, LDB = Cfg<D>::LDB;
  const int NT = (d + 31) >> 5, KD = (d + 15) & ~15;
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int tile = w; tile < NT * NT; tile += PNW) {
    const int tk = tile / NT, tj = tile % NT;
    const int row = tk * 32 + lr, j = tj * 32 + lr;
    const int lbeg = trim ? tk * 32 : 0;
    floatx16 acc = {};
    if constexpr (BF16) {
      const __bf16* xa = opXb<D>(s) + row * LDB + 8 * lk;
      const __bf16* kb = opK2b<D>(s) + j * LDB + 8 * lk;
      chain_bf16_g<4>(xa + lbeg, kb + lbeg, (KD - lbeg) >> 4, acc);
      mfma_drain();
      // four 8-byte stores per lane (columns tk * 32 + 8 q + 4 lk .. + 3 of row j)
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      __bf16* tt = opTtb<D>(s) + j * LDB + tk * 32 + 4 * lk;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<bf16x4*>(tt + 8 * q) =
            bf16x4{(__bf16)acc[4 * q], (__bf16)acc[4 * q + 1], (__bf16)acc[4 * q + 2], (__bf16)acc[4 * q + 3]};
    } else {
      const int Sj = s.S[j];
      const float* X = opXf<D>(s);
#pragma unroll 4
      for (int l0 = lbeg; l0 < KD; l0 += 2) {
        const int l = l0 + lk;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(X[row * LDF + l], kentry<D, WEIGHTED>(s, j, l, Q, Sj), acc, 0, 0,
                                                   0);
      }
      mfma_drain();
      float* T = opTf<D>(s);
#pragma unroll
      for (int r = 0; r < 16; ++r) T[(tk * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc[r];
    }
  }
}

template <int D, bool BF16, bool WEIGHTED>
__device__ __forceinline__ void gemm_kt_g(PairSmem<D>& s, const int* P, float* Wb, bool tri, int d) {
  constexpr int LDF = Cfg<D>::LDF, LDB = Cfg<D>::LDB;
  const int NT = (d + 31) >> 5, KD = (d + 15) & ~15;
  const int lane = threadIdx.x & 63, lr = lane & 31, lk = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int ti, tj;
  for (int u = 0; kt_tile_n(w, u, tri, NT, ti, tj); ++u) {
    const int i = ti * 32 + lr, j = tj * 32 + lr;
    floatx16 acc = {};
    if constexpr (BF16) {
      const __bf16* ka = opK1b<D>(s) + i * LDB + 8 * lk;
      const __bf16* tb = opTtb<D>(s) + j * LDB + 8 * lk;
      chain_bf16_g<4>(ka, tb, KD >> 4, acc);
    } else {
      const int Ri = s.R[i];
      const float* T = opTf<D>(s);
#pragma unroll 4
      for (int k0 = 0; k0 < KD; k0 += 2) {
        const int k = k0 + lk;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(kentry<D, WEIGHTED>(s, i, k, P, Ri), T[k * LDF + j], acc, 0, 0, 0);
      }
    }
    mfma_drain();
#pragma unroll
    for (int r = 0; r < 16; ++r) Wb[(ti * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc[r];
  }
  __syncthreads();
}

// Contractions of one K application (LDS or global operands).
template <int D, bool BF16, bool WEIGHTED1, bool WEIGHTED2>
__device__ __forceinline__ void contract(PairSmem<D>& s, const int* P, const int* Q, float* Wb, bool trim, bool tri,
                                         int d) {
  if constexpr (D <= 128) {
    gemm_xk<D, BF16, WEIGHTED1>(s, Q, trim);
    __syncthreads();
    gemm_kt<D, BF16, WEIGHTED2>(s, P, Wb, tri);
  } else {
    gemm_xk_g<D, BF16, WEIGHTED1>(s, Q, trim, d);
    __syncthreads();
    gemm_kt_g<D, BF16, WEIGHTED2>(s, P, Wb, tri, d);
  }
}

template <int D>
__device__ __forceinline__ void prep_update(PairSmem<D>& s);

// (K x) on the grid for input scales P, Q (residual already in the X buffer of
// the matching format) into the K x buffer, scaled by 2^-(R_i + S_j).  `trim`:
// x vanishes below the diagonal; `tri`: only cells on or above it are read.
template <int D>
__device__ __forceinline__ float* apply_K(PairSmem<D>& s, const int* P, const int* Q, int d, int H, bool lowp,
                                          bool trim, bool tri) {
  prep_update<D>(s);
  compute_RS<D>(s, P, Q, d, H);
  if (lowp) {
    for (int r = threadIdx.x; r < D; r += PWGS) {
      s.P7[r] = min(max(P[r], -(1 << 20)), 1 << 20) << 7;
      s.Q7[r] = min(max(Q[r], -(1 << 20)), 1 << 20) << 7;
    }
  }
  __syncthreads();
  float* Wb = wbuf<D>(s, lowp);
  if (lowp) {
    build_kernels_bf16<D>(s, d);
    __syncthreads();
    contract<D, true, false, false>(s, P, Q, Wb, trim, tri, d);
  } else {
    contract<D, false, false, false>(s, P, Q, Wb, trim, tri, d);
  }
  return Wb;
}

// Zero the whole X buffer in format bf16 (then only support cells get set).
template <int D>
__device__ __forceinline__ void zero_x(PairSmem<D>& s, bool bf16) {
  if (bf16) {
    for (int c = threadIdx.x; c < D * Cfg<D>::LDB / 8; c += PWGS) reinterpret_cast<bf16x8*>(opXb<D>(s))[c] = bf16x8{};
  } else {
    for (int c = threadIdx.x; c < D * Cfg<D>::LDF; c += PWGS) opXf<D>(s)[c] = 0.0f;
  }
}

template <int D>
__device__ __forceinline__ void put_x(PairSmem<D>& s, int cell, float v, bool bf16) {
  const int i = cell / D, j = cell % D;
  if (bf16) opXb<D>(s)[i * Cfg<D>::LDB + j] = (__bf16)v;
  else opXf<D>(s)[i * Cfg<D>::LDF + j] = v;
}

// One side's support list (u on supp(a) or v on supp(b)): per entry the cell
// i * D + j, the target marginal, the scaling residual, the marker q (log2
// estimate, or QSUSP + suspect index) and the refit estimate qe.  Entry e
// belongs to thread e mod PWGS, slot e / PWGS; only its owner touches it.
// SPT > 0: SPT slots per thread in registers.  SPT = 0: the entries live in a
// per-workgroup slice of the workspace (L2-resident), for supports of any size.
template <int SPT>
struct SupList {
  int cell_[SPT];
  float tgt_[SPT];
  float res_[SPT];
  int q_[SPT];
  int qe_[SPT];
  __device__ __forceinline__ static constexpr int nk() { return SPT; }
  // The cell is opaque to the optimiser at every use, so that addresses derived
  // from it are recomputed where needed instead of being kept live in
  // registers across the whole solve.
  __device__ __forceinline__ int cell(int k) const {
    int c = cell_[k];
    asm volatile("" : "+v"(c));
    return c;
  }
  __device__ __forceinline__ float tgt(int k) const { return tgt_[k]; }
  __device__ __forceinline__ float res(int k) const { return res_[k]; }
  __device__ __forceinline__ int q(int k) const { return q_[k]; }
  __device__ __forceinline__ int qe(int k) const { return qe_[k]; }
  __device__ __forceinline__ void set_res(int k, float v) { res_[k] = v; }
  __device__ __forceinline__ void set_q(int k, int v) { q_[k] = v; }
  __device__ __forceinline__ void set_qe(int k, int v) { qe_[k] = v; }
  __device__ __forceinline__ void set_entry(int k, int c, float t) {
    cell_[k] = c;
    tgt_[k] = t;
    res_[k] = 0.0f;
  }
  __device__ __forceinline__ static constexpr int capacity() { return SPT * PWGS; }
};

template <>
struct SupList<0> {
  int* cell_;
  float* tgt_;
  float* res_;
  int* q_;
  int* qe_;
  int n;
  int cap;
  __device__ __forceinline__ int nk() const { return (n + PWGS - 1) / PWGS; }
  __device__ __forceinline__ int ix(int k) const { return (int)threadIdx.x + PWGS * k; }
  __device__ __forceinline__ int cell(int k) const { return ix(k) < n ? cell_[ix(k)] : -1; }
  __device__ __forceinline__ float tgt(int k) const { return ix(k) < n ? tgt_[ix(k)] : 0.0f; }
  __device__ __forceinline__ float res(int k) const { return ix(k) < n ? res_[ix(k)] : 0.0f; }
  __device__ __forceinline__ int q(int k) const { return ix(k) < n ? q_[ix(k)] : QNONE; }
  __device__ __forceinline__ int qe(int k) const { return ix(k) < n ? qe_[ix(k)] : QNONE; }
  __device__ __forceinline__ void set_res(int k, float v) {
    if (ix(k) < n) res_[ix(k)] = v;
  }
  __device__ __forceinline__ void set_q(int k, int v) {
    if (ix(k) < n) q_[ix(k)] = v;
  }
  __device__ __forceinline__ void set_qe(int k, int v) {
    if (ix(k) < n) qe_[ix(k)] = v;
  }
  __device__ __forceinline__ void set_entry(int k, int c, float t) {
    cell_[ix(k)] = c;
    tgt_[ix(k)] = t;
    res_[ix(k)] = 0.0f;
  }
  __device__ __forceinline__ int capacity() const { return cap; }
};

// Build the support list of histogram h (d x d, row-major) in deterministic
// order; returns its total mass, sets too_big when it does not fit and lower
// when some mass lies below the diagonal (cell column < row).
template <int D, int SPT>
__device__ __forceinline__ double build_support(PairSmem<D>& s, const float* __restrict__ h, int d,
                                                SupList<SPT>& sp, bool& too_big, bool& lower) {
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
  too_big = total > sp.capacity();
  if (!too_big) {
    for (int c = c0; c < c1; ++c) {
      const float v = h[c];
      if (v > 0.0f) {
        stCell<D>(s)[off] = (c / d) * D + (c % d);
        stVal<D>(s)[off] = v;
        ++off;
      }
    }
  }
  __syncthreads();
  if constexpr (SPT == 0) sp.n = too_big ? 0 : total;
  const int nk = sp.nk();
#pragma unroll
  for (int k = 0; k < nk; ++k) {
    const int e = threadIdx.x + PWGS * k;
    const bool ok = !too_big && e < total;
    if constexpr (SPT == 0) {
      if (ok) sp.set_entry(k, stCell<D>(s)[e], stVal<D>(s)[e]);
    } else {
      sp.set_entry(k, ok ? stCell<D>(s)[e] : -1, ok ? stVal<D>(s)[e] : 0.0f);
    }
  }
  __syncthreads();
  return mass;
}

// Exact values for the suspects [0, ns) from the input x: sum over the support
// of x of K_(ij),(kl) x_kl (times C_(ij),(kl) when WEIGHTED, Proposition 3)
// with explicit exponents: pass 1 takes the largest term exponent, pass 2 the
// sum of the terms scaled by it.  One wave per suspect (wave w takes suspects
// w, w + PNW, ...), its lanes striding over x's entries: no workgroup barrier
// inside.  x is its support list (register lists are staged to LDS first,
// unless `staged`), or (dense) 1 on every grid cell.  Writes mantissa and
// absolute log2 exponent to out_m / out_e; with FIN, instead the value in the
// natural scale of cell (i, j), 2^-(R_i + S_j), plus the diagonal-bin term
// x_Delta k_Delta,ij of the K application (xD_e, xD_m: x_Delta), flagging
// s.sflag when the total vanishes.
template <int D, int SPT, bool WEIGHTED, bool FIN>
__device__ __forceinline__ void exact_all(PairSmem<D>& s, const SupList<SPT>& xs, bool dense, int d, const int* Px,
                                          const int* Qx, int ns, int* out_e, float* out_m, bool staged = false,
                                          int xD_e = 0, float xD_m = 0.0f) {
  static_assert(SPT <= 1, "register lists of one slot are staged to LDS");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int* xc;
  const float* xr;
  int nx;
  auto finish = [&](int id, int c, int em, float acc) {
    if constexpr (FIN) {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      const ESum g{em - s.R[i] - s.S[j], (double)acc};
      const ESum tot = esum_add(g, ESum{xD_e + s.tgde[dl] - s.R[i] - s.S[j], (double)(xD_m * s.tgdm[dl])});
      if (tot.s > 0.0) {
        out_e[id] = tot.e;
        out_m[id] = (float)tot.s;
      } else {
        atomicOr(&s.sflag, 1);
        out_e[id] = 0;
        out_m[id] = 1.0f;
      }
    } else {
      out_e[id] = em;
      out_m[id] = acc;
    }
  };
  if constexpr (SPT == 1) {
    if (!dense && !staged) {
      const int c = xs.cell(0);
      s.xs_cell[threadIdx.x] = c;
      s.xs_res[threadIdx.x] = c >= 0 ? xs.res(0) : 0.0f;
    }
    if (!staged) __syncthreads();
    xc = s.xs_cell;
    xr = s.xs_res;
    nx = PWGS;
  } else {
    xc = xs.cell_;
    xr = xs.res_;
    nx = xs.n;
    // a global list that fits the staging area is read from LDS instead
    if (!dense && xs.n <= PWGS) {
      const int e = threadIdx.x;
      s.xs_cell[e] = e < xs.n ? xc[e] : -1;
      s.xs_res[e] = e < xs.n ? xr[e] : 0.0f;
      __syncthreads();
    }
  }
  if (dense) nx = d * d;
  {
    // staged x (a register list, or a global list of at most PWGS cells):
    // PWGS / 64 entries per lane, kept in registers for both passes
    bool small = true;
    if constexpr (SPT == 0) small = xs.n <= PWGS;
    if (!dense && small) {
      constexpr int EPL = PWGS / 64;
      int kr[EPL], l[EPL], eb[EPL];
      float xm[EPL];
#pragma unroll
      for (int u = 0; u < EPL; ++u) {
        const int cell = s.xs_cell[lane + 64 * u];
        const float x = s.xs_res[lane + 64 * u];
        const bool ok = cell >= 0 && x > 0.0f;
        kr[u] = ok ? cell / D : 0;
        l[u] = ok ? cell % D : 0;
        xm[u] = ok ? x : 0.0f;
        eb[u] = ok ? Px[kr[u]] + Qx[l[u]] : QNONE;
      }
      // Two suspects per wave at a time, so that two independent wave
      // reductions are in flight; each suspect's terms and their order are
      // those of a wave that takes it alone.
      constexpr int NS = 2;
      for (int id0 = wave * NS; id0 < ns; id0 += PNW * NS) {
        int ti[NS], tj[NS], em[NS];
        float acc[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const int c = suspCell<D, SPT>(s)[id0 + t < ns ? id0 + t : id0];
          ti[t] = c / D;
          tj[t] = c % D;
          em[t] = QNONE;
          acc[t] = 0.0f;
        }
#pragma unroll
        for (int u = 0; u < EPL; ++u)
          if (eb[u] != QNONE)
#pragma unroll
            for (int t = 0; t < NS; ++t)
              em[t] = max(em[t], eb[u] + ilog2f(xm[u]) + s.tge[ti[t] - kr[u] + D - 1] + s.tge[tj[t] - l[u] + D - 1]);
#pragma unroll
        for (int t = 0; t < NS; ++t) em[t] = wave_max(em[t]);
#pragma unroll
        for (int u = 0; u < EPL; ++u) {
          if (eb[u] != QNONE) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
              const int i1 = ti[t] - kr[u] + D - 1, i2 = tj[t] - l[u] + D - 1;
              float mm = xm[u] * s.tgm[i1] * s.tgm[i2];
              if (WEIGHTED) mm *= (s.tc1[i1] + s.tc1[i2]);
              acc[t] += ldx(mm, eb[u] + s.tge[i1] + s.tge[i2] - em[t]);
            }
          }
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) acc[t] = wave_sum(acc[t]);
        if (lane == 0) {
#pragma unroll
          for (int t = 0; t < NS; ++t)
            if (id0 + t < ns) finish(id0 + t, ti[t] * D + tj[t], em[t], acc[t]);
        }
      }
      __syncthreads();
      return;
    }
  }
  // Four suspects per wave, so that each entry of x is read once for four.
  auto generic = [&](const int* xc, const float* xr) {
    constexpr int NT4 = 4;
    for (int id0 = wave * NT4; id0 < ns; id0 += PNW * NT4) {
      const int nt = min(NT4, ns - id0);
      int ti[NT4], tj[NT4], em[NT4];
#pragma unroll
      for (int t = 0; t < NT4; ++t) {
        const int c = t < nt ? suspCell<D, SPT>(s)[id0 + t] : 0;
        ti[t] = c / D;
        tj[t] = c % D;
        em[t] = QNONE;
      }
      for (int e = lane; e < nx; e += 64) {
        int cell;
        float x;
        if (dense) {
          cell = (e / d) * D + (e % d);
          x = 1.0f;
        } else {
          cell = xc[e];
          x = cell >= 0 ? xr[e] : 0.0f;
        }
        if (cell >= 0 && x > 0.0f) {
          const int kr = cell / D, l = cell % D;
          const int eb = Px[kr] + Qx[l] + ilog2f(x);
#pragma unroll
          for (int t = 0; t < NT4; ++t)
            em[t] = max(em[t], eb + s.tge[ti[t] - kr + D - 1] + s.tge[tj[t] - l + D - 1]);
        }
      }
#pragma unroll
      for (int t = 0; t < NT4; ++t) em[t] = wave_max(em[t]);
      float acc[NT4] = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int e = lane; e < nx; e += 64) {
        int cell;
        float x;
        if (dense) {
          cell = (e / d) * D + (e % d);
          x = 1.0f;
        } else {
          cell = xc[e];
          x = cell >= 0 ? xr[e] : 0.0f;
        }
        if (cell >= 0 && x > 0.0f) {
          const int kr = cell / D, l = cell % D;
          const int eb = Px[kr] + Qx[l];
#pragma unroll
          for (int t = 0; t < NT4; ++t) {
            const int i1 = ti[t] - kr + D - 1, i2 = tj[t] - l + D - 1;
            float mm = x * s.tgm[i1] * s.tgm[i2];
            if (WEIGHTED) mm *= (s.tc1[i1] + s.tc1[i2]);
            acc[t] += ldx(mm, eb + s.tge[i1] + s.tge[i2] - em[t]);
          }
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
  };
  generic(xc, xr);
  __syncthreads();
}

// State of one side of the pair (u or v) as seen by the update of the other.
struct Side {
  int ex;      // diagonal entry = mx * 2^ex
  double mx;
  int mres;    // residual span (octaves) of its last update
};

// Reset the per-half-step state of y_update (suspect count, flags, refit
// extrema); called before the K application that feeds it.
template <int D>
__device__ __forceinline__ void prep_update(PairSmem<D>& s) {
  for (int r = threadIdx.x; r < D; r += PWGS) {
#pragma unroll
    for (int sw = 0; sw < 2; ++sw) {
      s.fit[sw][0][r] = INT_MIN;
      s.fit[sw][1][r] = INT_MAX;
      s.fit[sw][2][r] = INT_MIN;
      s.fit[sw][3][r] = INT_MAX;
    }
  }
  if (threadIdx.x == 0) {
    s.nsusp = 0;
    s.sflag = 0;
  }
}

__device__ __forceinline__ int midrange(const int* mx, const int* mn, int r) { return (mx[r] + mn[r]) >> 1; }

// y = target / (K x) on y's support, with K x (scaled by 2^-(R+S)) in Wb
// except at the suspects.  Refits y's scales (Py, Qy), writes the new residual
// to ys.res and, in format out_bf16, to the X buffer (after clearing the cells
// of x's support, or the whole buffer when clear_all), and returns the grid
// part of <y, k_Delta>.  When `check`, first measures the row-marginal error
// of the previous y against K x and may stop there, leaving ys, Py, Qy
// untouched and q holding the suspect markers.  `wb_bf16`: Wb lies in the
// BF16 buffers, which an FP32 X buffer overlaps.
//
// The refit is two sweeps of row/column centring of the per-cell log2
// estimates: each of the four passes folds its extrema into LDS with atomics,
// and the centre of the previous pass is read on the fly, so a half step
// needs five workgroup barriers when no cell is suspect.
template <int D, int SPT>
__device__ __forceinline__ void y_update(PairSmem<D>& s, const float* Wb, bool wb_bf16, SupList<SPT>& ys,
                                         const SupList<SPT>& xsup, bool x_dense, int d, const Side& xs, int H,
                                         const int* Px, const int* Qx, int* Py, int* Qy, bool out_bf16,
                                         bool clear_all, bool check, double& err_out, bool& stop_out, ESum& dot,
                                         int& mres_out, int& bad, int& range, double errD, double m, double tol,
                                         double switch_tol, bool& lowp, int t, int max_iter) {
  constexpr int LDF = Cfg<D>::LDF;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float mxf = (float)xs.mx;
  // Trusted level of a normalised value: everything the contractions drop is
  // below 2^(H + mres + 14 - 126) in these units; keep a 2^-SUSP_MARGIN
  // relative margin (the FP32 unit roundoff: no more than the rounding of
  // the contraction sums themselves).
  const int thr = H + max(xs.mres, 20) + 14 - 126 + SUSP_MARGIN;
  // The X buffer can be cleared now (x was consumed by contraction 1) unless
  // an FP32 X overlaps the BF16 K x buffer still being read.
  const bool late_x = !out_bf16 && wb_bf16;
  const int nk = ys.nk();

  // Pass A: suspects, row extrema of sweep 0, error terms, X clearing.
  int lbad = 0, lover = 0;
  double eg = 0.0;
#pragma unroll
  for (int k = 0; k < nk; ++k) {
    ys.set_q(k, QNONE);
    ys.set_qe(k, QNONE);
    const int c = ys.cell(k);
    if (c >= 0) {
      const int i = c / D, j = c % D;
      const float w = Wb[i * LDF + j];
      const float tg = ys.tgt(k);
      const int dl = j - i + D - 1;
      const int E = xs.ex + s.tgde[dl] - s.R[i] - s.S[j];
      const float Dm = mxf * s.tgdm[dl];
      const int lw = w > 0.0f ? ilog2f(w) : QNONE;
      const int ld = Dm > 0.0f ? E + ilog2f(Dm) : QNONE;
      const int le = max(lw, ld);
      int qk;
      bool sus = false;
      if (le < thr) {
        const int id = atomicAdd(&s.nsusp, 1);
        if (id < suspCap<D, SPT>()) {
          suspCell<D, SPT>(s)[id] = c;
          qk = QSUSP + id;
          sus = true;
        } else {
          lover = 1;
          if (le == QNONE) lbad = 1;
          qk = le == QNONE ? 0 : ilog2f(tg) - le;
        }
      } else {
        qk = ilog2f(tg) - le;
      }
      ys.set_q(k, qk);
      if (!sus) {
        ys.set_qe(k, qk);
        atomicMax(&s.fit[0][0][i], qk);
        atomicMin(&s.fit[0][1][i], qk);
        if (check) {
          const int sh = Py[i] + Qy[j] + s.R[i] + s.S[j];
          const double r = (double)ys.res(k);
          const double row = ldxd(r * (double)w, sh) + ldxd(r * (double)Dm, E + sh);
          eg += fabs(row - (double)tg);
        }
      }
    }
  }
  if constexpr (SPT == 1) {   // x's list, for the exact path should a cell be suspect
    if (!x_dense) {
      const int c = xsup.cell(0);
      s.xs_cell[tid] = c;
      s.xs_res[tid] = c >= 0 ? xsup.res(0) : 0.0f;
    }
  }
  if (!late_x) {
    if (clear_all) {
      zero_x<D>(s, out_bf16);
    } else {
      const int xk = xsup.nk();
#pragma unroll
      for (int k = 0; k < xk; ++k) {
        const int c = xsup.cell(k);
        if (c >= 0) put_x<D>(s, c, 0.0f, out_bf16);
      }
    }
  }
  {
    const double egw = wave_sum(eg);
    const unsigned long long bb = __ballot(lbad), bo = __ballot(lover);
    if (lane == 0) {
      s.red[wave] = egw;
      s.redi[wave] = (bb ? 1 : 0) | (bo ? 2 : 0);
    }
  }
  __syncthreads();
  const int ns = min(s.nsusp, suspCap<D, SPT>());
  double egs = 0.0;
  int flags = 0;
#pragma unroll
  for (int w = 0; w < PNW; ++w) {
    egs += s.red[w];
    flags |= s.redi[w];
  }

  // Suspects: exact values, then their row extrema and error terms.
  if (ns > 0) {
    exact_all<D, SPT, false, true>(s, xsup, x_dense, d, Px, Qx, ns, suspE<D, SPT>(s), suspM<D, SPT>(s), true, xs.ex,
                                   mxf);
    double eg2 = 0.0;
#pragma unroll
    for (int k = 0; k < nk; ++k) {
      const int qk = ys.q(k);
      if (qk >= QSUSP) {
        const int id = qk - QSUSP;
        const int c = ys.cell(k), i = c / D, j = c % D;
        const float tg = ys.tgt(k);
        const int qx = ilog2f(tg) - (suspE<D, SPT>(s)[id] + ilog2f(suspM<D, SPT>(s)[id]));
        ys.set_qe(k, qx);
        atomicMax(&s.fit[0][0][i], qx);
        atomicMin(&s.fit[0][1][i], qx);
        if (check) {
          const int sh = Py[i] + Qy[j] + s.R[i] + s.S[j];
          const double row = ldxd((double)ys.res(k) * (double)suspM<D, SPT>(s)[id], suspE<D, SPT>(s)[id] + sh);
          eg2 += fabs(row - (double)tg);
        }
      }
    }
    eg2 = wave_sum(eg2);
    if (lane == 0) s.reds[wave] = eg2;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < PNW; ++w) egs += s.reds[w];
    flags |= s.sflag;
  }

  if (check) {
    err_out = (egs + errD) / m;
    const bool measured_lowp = lowp;   // never stop on an error measured with BF16 contractions
    // BF16 ends at switch_tol, or at half the iteration budget whatever the
    // error, so that a pair whose BF16 error floor lies above switch_tol still
    // finishes in FP32.
    if (lowp && (err_out <= switch_tol || 2 * t >= max_iter)) lowp = false;
    if ((!measured_lowp && err_out <= tol) || t >= max_iter) {
      stop_out = true;
      if (flags & 1) bad = 1;
      return;
    }
  }
  if (flags & 1) bad = 1;
  if (flags & 2) range |= 2;   // more suspects than the lists hold

  // Column extrema of sweep 0 (against the row centres of sweep 0), then the
  // rows and columns of sweep 1.
#pragma unroll
  for (int k = 0; k < nk; ++k) {
    const int qx = ys.qe(k);
    if (qx != QNONE) {
      const int c = ys.cell(k), i = c / D, j = c % D;
      const int v = qx - midrange(s.fit[0][0], s.fit[0][1], i);
      atomicMax(&s.fit[0][2][j], v);
      atomicMin(&s.fit[0][3][j], v);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < nk; ++k) {
    const int qx = ys.qe(k);
    if (qx != QNONE) {
      const int c = ys.cell(k), i = c / D, j = c % D;
      const int v = qx - midrange(s.fit[0][2], s.fit[0][3], j);
      atomicMax(&s.fit[1][0][i], v);
      atomicMin(&s.fit[1][1][i], v);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < nk; ++k) {
    const int qx = ys.qe(k);
    if (qx != QNONE) {
      const int c = ys.cell(k), i = c / D, j = c % D;
      const int v = qx - midrange(s.fit[1][0], s.fit[1][1], i);
      atomicMax(&s.fit[1][2][j], v);
      atomicMin(&s.fit[1][3][j], v);
    }
  }
  __syncthreads();

  // New scales: natural (-R, -S) plus the centres (rho, sigma) of sweep 1,
  // by the last threads, which hold no support entry unless the support
  // fills the lists (entries sit on threads 0, 1, ...).
  static_assert(D <= PWGS, "one scale per thread");
  {
    const int r = PWGS - 1 - tid;
    if (r < D) {
      Py[r] = s.fit[1][0][r] != INT_MIN ? midrange(s.fit[1][0], s.fit[1][1], r) - s.R[r] : NEG;
      Qy[r] = s.fit[1][2][r] != INT_MIN ? midrange(s.fit[1][2], s.fit[1][3], r) - s.S[r] : NEG;
    }
  }
  ESum acc{NEG, 0.0};
  int maxres = 0;
#pragma unroll
  for (int k = 0; k < nk; ++k) {
    const int c = ys.cell(k);
    if (c >= 0) {
      const int i = c / D, j = c % D;
      const int dl = j - i + D - 1;
      const int rho = midrange(s.fit[1][0], s.fit[1][1], i), sig = midrange(s.fit[1][2], s.fit[1][3], j);
      const int sh = rho + sig;
      const int qk = ys.q(k);
      const float tg = ys.tgt(k);
      float y;
      if (qk >= QSUSP) {
        const int id = qk - QSUSP;
        y = tg / ldx(suspM<D, SPT>(s)[id], suspE<D, SPT>(s)[id] + sh);
      } else {
        const int E = xs.ex + s.tgde[dl] - s.R[i] - s.S[j];
        const float Dm = mxf * s.tgdm[dl];
        y = tg / (ldx(Wb[i * LDF + j], sh) + ldx(Dm, E + sh));
      }
      ys.set_res(k, y);
      if (!late_x) put_x<D>(s, c, y, out_bf16);
      maxres = max(maxres, abs(ys.qe(k) - sh));
      acc = esum_add(acc, ESum{rho - s.R[i] + sig - s.S[j] + s.tgde[dl], (double)y * (double)s.tgdm[dl]});
    }
  }
  {
    const ESum aw = wave_esum(acc);
    const int mw = wave_max(maxres);
    if (lane == 0) {
      s.rede[wave] = aw.e;
      s.reds[wave] = aw.s;
      s.redi[wave] = mw;
    }
  }
  __syncthreads();
  ESum tot{s.rede[0], s.reds[0]};
  int mr = s.redi[0];
#pragma unroll
  for (int w = 1; w < PNW; ++w) {
    tot = esum_add(tot, ESum{s.rede[w], s.reds[w]});
    mr = max(mr, s.redi[w]);
  }
  dot = tot;
  mres_out = mr + 1;
  if (mres_out > 100) range |= 1;
  if (late_x) {   // switch of the X format: every read of the K x buffer is done now
    zero_x<D>(s, out_bf16);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < nk; ++k) {
      const int c = ys.cell(k);
      if (c >= 0) put_x<D>(s, c, ys.res(k), out_bf16);
    }
  }
}

// Warm-start record of one pair's v (and its output after the solve):
// residual on the grid cells (row stride D; only the cells of supp(b) are
// read or written), row and column log2 scales, the diagonal entry
// vmx * 2^vex and the residual span.
template <int D>
struct WarmState {
  float vres[D * D];
  int Pv[D];
  int Qv[D];
  int vex;
  int mres;
  double vmx;
};

// ---------------------------------------------------------------------------
// Error control of section 3, after the last iteration: an upper bound from
// the rounding of the plan onto the transport polytope (Proposition 4, with
// the rounding algorithm of the supplementary material) and a lower bound
// from the c-transforms of alpha = gamma log u.

// Number of entries of a support list (register lists hold at most one per
// thread, in threads 0, 1, ...).
template <int SPT>
__device__ __forceinline__ int list_len(const SupList<SPT>& l) {
  if constexpr (SPT == 0) return l.n;
  else return __syncthreads_count(l.cell(0) >= 0);
}

// (K x)_c, or ((K o C) x)_c when WEIGHTED, grid part only, at every entry c
// of ys, summed exactly over the support of x (exact_all).  The value of
// entry k is m * 2^e, left as ys.q(k) = e and ys.qe(k) = the bits of m.
// Register lists pass through the LDS suspect arrays MAXSUSP entries at a time.
template <int D, int SPT, bool WEIGHTED>
__device__ __forceinline__ void sparse_kx(PairSmem<D>& s, SupList<SPT>& ys, const SupList<SPT>& xs, const int* Px,
                                          const int* Qx, int d, int ny) {
  if constexpr (SPT == 1) {
    for (int c0 = 0; c0 < ny; c0 += MAXSUSP) {
      const int id = (int)threadIdx.x - c0;
      const bool mine = id >= 0 && id < MAXSUSP && ys.cell(0) >= 0;
      if (mine) s.susp_cell[id] = ys.cell(0);
      __syncthreads();
      exact_all<D, 1, WEIGHTED, false>(s, xs, false, d, Px, Qx, min(MAXSUSP, ny - c0), s.susp_e, s.susp_m);
      if (mine) {
        ys.set_q(0, s.susp_e[id]);
        ys.set_qe(0, __float_as_int(s.susp_m[id]));
      }
      __syncthreads();
    }
  } else {
    for (int k = 0; k < ys.nk(); ++k)
      if (ys.ix(k) < ny) suspCell<D, 0>(s)[ys.ix(k)] = ys.cell(k);
    __syncthreads();
    exact_all<D, 0, WEIGHTED, false>(s, xs, false, d, Px, Qx, ny, suspE<D, 0>(s), suspM<D, 0>(s));
    for (int k = 0; k < ys.nk(); ++k) {
      if (ys.ix(k) < ny) {
        ys.set_q(k, suspE<D, 0>(s)[ys.ix(k)]);
        ys.set_qe(k, __float_as_int(suspM<D, 0>(s)[ys.ix(k)]));
      }
    }
    __syncthreads();
  }
}

// y (K x)_c at entry k of ys from sparse_kx's value, plus the diagonal-bin
// term y x_Delta k_Delta(c): a marginal of the plan, in the natural range.
template <int D, int SPT>
__device__ __forceinline__ double marg_at(const PairSmem<D>& s, const SupList<SPT>& ys, int k, float yres,
                                          const int* Py, const int* Qy, int xD_e, double xD_m) {
  const int c = ys.cell(k), i = c / D, j = c % D, dl = j - i + D - 1;
  const int e0 = Py[i] + Qy[j];
  return ldxd((double)yres * (double)__int_as_float(ys.qe(k)), e0 + ys.q(k)) +
         ldxd((double)yres * xD_m * (double)s.tgdm[dl], e0 + xD_e + s.tgde[dl]);
}

// In place over the rows (ROWS) or columns of the d x d part of g (row stride
// D + 1): g[r][o] <- min over x < d of c(o - x) + g[r][x], and the same along
// columns; one wave per line.  A lane's stores depend on the results of all
// of its loads, and the wave issues every load of a line before any store.
template <int D, bool ROWS>
__device__ __forceinline__ void minplus_lines(double* g, const double* c1d, int d) {
  constexpr int LG = D + 1;
  constexpr int NQ = D >= 64 ? D / 64 : 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int line = wave; line < d; line += PNW) {
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = INFINITY;
    for (int x = 0; x < d; ++x) {
      const double gv = ROWS ? g[line * LG + x] : g[x * LG + line];
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] = fmin(acc[q], c1d[min(lane + 64 * q, D - 1) - x + D - 1] + gv);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int o = lane + 64 * q;
      if (o < d) {
        if (ROWS) g[line * LG + o] = acc[q];
        else g[o * LG + line] = acc[q];
      }
    }
  }
}

// Lower bound <alpha^{c cbar}, a> + <alpha^c, b> for alpha = gamma log u
// (u on supp(a) and u_Delta), both transforms over the whole ground space
// (every grid cell and the diagonal bin).  The grid part of each transform is
// separable: one min-plus pass along rows, one along columns.
template <int D, int SPT>
__device__ __forceinline__ double lower_bound(PairSmem<D>& s, const SupList<SPT>& ua, const SupList<SPT>& vb,
                                              const Side& su, int d, double gamma, double aD, double bD,
                                              const double* c1d, const double* cdd) {
  constexpr int LG = D + 1;
  constexpr double LN2 = 0.69314718055994530942;
  static_assert(sizeof(double) * D * LG <= sizeof(float) * 2 * D * Cfg<D>::LDF, "grid in the FP32 operand pair");
  double* g = reinterpret_cast<double*>(opXf<D>(s));
  const int tid = threadIdx.x;
  for (int c = tid; c < D * LG; c += PWGS) g[c] = INFINITY;
  __syncthreads();
  const double alD = su.mx > 0.0 ? gamma * (log(su.mx) + (double)su.ex * LN2) : -INFINITY;
  double mD = -alD;   // alpha^c_Delta: the diagonal bin, then every cell of supp(a)
  for (int k = 0; k < ua.nk(); ++k) {
    const int c = ua.cell(k);
    const float r = ua.res(k);
    if (c >= 0 && r > 0.0f) {
      const int i = c / D, j = c % D;
      const double al = gamma * (log((double)r) + (double)(s.Pu[i] + s.Qu[j]) * LN2);
      g[i * LG + j] = -al;
      mD = fmin(mD, cdd[j - i + D - 1] - al);
    }
  }
  const double acD = block_min<PNW>(mD, s.red);
  minplus_lines<D, true>(g, c1d, d);
  __syncthreads();
  minplus_lines<D, false>(g, c1d, d);
  __syncthreads();
  // alpha^c on the grid (the diagonal bin as one more source), kept negated
  // for the second transform; alpha^{c cbar}_Delta from it.
  double mg = -acD;
  for (int c = tid; c < d * d; c += PWGS) {
    const int i = c / d, j = c % d;
    const double cd = cdd[j - i + D - 1];
    const double v = fmin(g[i * LG + j], cd - alD);
    g[i * LG + j] = -v;
    mg = fmin(mg, cd - v);
  }
  const double accD = block_min<PNW>(mg, s.red);
  double sb = 0.0;
  for (int k = 0; k < vb.nk(); ++k) {
    const int c = vb.cell(k);
    if (c >= 0) sb -= (double)vb.tgt(k) * g[(c / D) * LG + c % D];
  }
  sb = block_sum<PNW>(sb, s.red) + bD * acD;
  minplus_lines<D, true>(g, c1d, d);
  __syncthreads();
  minplus_lines<D, false>(g, c1d, d);
  __syncthreads();
  double sa = 0.0;
  for (int k = 0; k < ua.nk(); ++k) {
    const int c = ua.cell(k);
    if (c >= 0) {
      const int i = c / D, j = c % D;
      sa += (double)ua.tgt(k) * fmin(g[i * LG + j], cdd[j - i + D - 1] - acD);
    }
  }
  sa = block_sum<PNW>(sa, s.red) + aD * accD;
  __syncthreads();
  return sa + sb;
}

// Upper bound <R, C> of Proposition 4: X = min(a / r(P), 1) scales u, then
// Y = min(b / c(diag(X) P), 1) scales v, and the plan P'' of the scaled pair
// plus the rank-one term e_r e_c^T / |e_c|_1 (e_r, e_c: the marginal
// deficits of P'') is priced.  Every K application is an exact sum over the
// supports; the residuals of ua and vb are left scaled.
template <int D, int SPT>
__device__ __forceinline__ double upper_bound(PairSmem<D>& s, SupList<SPT>& ua, SupList<SPT>& vb, const Side& su,
                                              const Side& sv, ESum kv, int d, double aD, double bD,
                                              const double* c1d, const double* cdd) {
  constexpr int LDF = Cfg<D>::LDF;
  static_assert(sizeof(float) * 2 * D * LDF + sizeof(double) * 4 * D <= sizeof(__bf16) * 4 * D * Cfg<D>::LDB,
                "deficit grids and their sums in the operand buffers");
  const int tid = threadIdx.x;
  float* er = opXf<D>(s);                 // e_r on the grid, row stride LDF
  float* ec = er + D * LDF;               // e_c
  double* sums = reinterpret_cast<double*>(er + 2 * D * LDF);   // row, column sums of e_r; of e_c
  for (int c = tid; c < 2 * D * LDF; c += PWGS) er[c] = 0.0f;
  const int na = list_len(ua), nb = list_len(vb);
  // 1. u' = X u with r(P) = u (K v)
  sparse_kx<D, SPT, false>(s, ua, vb, s.Pv, s.Qv, d, na);
  for (int k = 0; k < ua.nk(); ++k) {
    const float r = ua.res(k);
    if (ua.cell(k) >= 0 && r > 0.0f) {
      const double rp = marg_at<D, SPT>(s, ua, k, r, s.Pu, s.Qu, sv.ex, sv.mx);
      const double a = ua.tgt(k);
      if (rp > a) ua.set_res(k, (float)((double)r * (a / rp)));
    }
  }
  const double rD = ldxd(su.mx * kv.s, su.ex + kv.e);
  const double uD = rD > aD ? su.mx * (aD / rD) : su.mx;   // u'_Delta = uD 2^su.ex
  __syncthreads();
  // 2. v' = Y v with c(P') = v (K^T u'); e_c = b - v' (K^T u')
  sparse_kx<D, SPT, false>(s, vb, ua, s.Pu, s.Qu, d, nb);
  ESum kuD{NEG, 0.0};
  for (int k = 0; k < ua.nk(); ++k) {
    const int c = ua.cell(k);
    const float r = ua.res(k);
    if (c >= 0 && r > 0.0f) {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      kuD = esum_add(kuD, ESum{s.Pu[i] + s.Qu[j] + s.tgde[dl], (double)r * (double)s.tgdm[dl]});
    }
  }
  kuD = esum_add(block_esum<PNW>(kuD, s.rede, s.reds), ESum{su.ex, uD});   // (K^T u')_Delta
  double ec1 = 0.0, eccd = 0.0;
  for (int k = 0; k < vb.nk(); ++k) {
    const int c = vb.cell(k);
    if (c >= 0) {
      const float r = vb.res(k);
      const double b = vb.tgt(k);
      double cp = 0.0;
      if (r > 0.0f) {
        cp = marg_at<D, SPT>(s, vb, k, r, s.Pv, s.Qv, su.ex, uD);
        if (cp > b) {
          const float rn = (float)((double)r * (b / cp));
          vb.set_res(k, rn);
          cp = rn > 0.0f ? marg_at<D, SPT>(s, vb, k, rn, s.Pv, s.Qv, su.ex, uD) : 0.0;
        }
      }
      const double e = b - cp;
      const int i = c / D, j = c % D;
      ec[i * LDF + j] = (float)e;
      ec1 += fabs(e);
      eccd += e * cdd[j - i + D - 1];
    }
  }
  const double cPD = ldxd(sv.mx * kuD.s, sv.ex + kuD.e);
  const double vD = cPD > bD ? sv.mx * (bD / cPD) : sv.mx;   // v'_Delta = vD 2^sv.ex
  const double ecD = bD - ldxd(vD * kuD.s, sv.ex + kuD.e);
  __syncthreads();
  // 3. e_r = a - u' (K v')
  sparse_kx<D, SPT, false>(s, ua, vb, s.Pv, s.Qv, d, na);
  ESum kvD{NEG, 0.0};
  for (int k = 0; k < vb.nk(); ++k) {
    const int c = vb.cell(k);
    const float r = vb.res(k);
    if (c >= 0 && r > 0.0f) {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      kvD = esum_add(kvD, ESum{s.Pv[i] + s.Qv[j] + s.tgde[dl], (double)r * (double)s.tgdm[dl]});
    }
  }
  kvD = esum_add(block_esum<PNW>(kvD, s.rede, s.reds), ESum{sv.ex, vD});   // (K v')_Delta
  double ercd = 0.0;
  for (int k = 0; k < ua.nk(); ++k) {
    const int c = ua.cell(k);
    if (c >= 0) {
      const float r = ua.res(k);
      const double e = (double)ua.tgt(k) - (r > 0.0f ? marg_at<D, SPT>(s, ua, k, r, s.Pu, s.Qu, sv.ex, vD) : 0.0);
      const int i = c / D, j = c % D;
      er[i * LDF + j] = (float)e;
      ercd += e * cdd[j - i + D - 1];
    }
  }
  const double erD = aD - ldxd(uD * kvD.s, su.ex + kvD.e);
  // 4. <P'', C>: grid to grid by (K o C) v', and the two diagonal-bin blocks
  sparse_kx<D, SPT, true>(s, ua, vb, s.Pv, s.Qv, d, na);
  double g = 0.0;
  for (int k = 0; k < ua.nk(); ++k) {
    const int c = ua.cell(k);
    const float r = ua.res(k);
    if (c >= 0 && r > 0.0f) {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      const int e0 = s.Pu[i] + s.Qu[j];
      g += ldxd((double)r * (double)__int_as_float(ua.qe(k)), e0 + ua.q(k));
      g += ldxd((double)r * vD * (double)s.tgdm[dl] * cdd[dl], e0 + sv.ex + s.tgde[dl]);
    }
  }
  for (int k = 0; k < vb.nk(); ++k) {
    const int c = vb.cell(k);
    const float r = vb.res(k);
    if (c >= 0 && r > 0.0f) {
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      g += ldxd((double)r * uD * (double)s.tgdm[dl] * cdd[dl], s.Pv[i] + s.Qv[j] + su.ex + s.tgde[dl]);
    }
  }
  // 5. the rank-one term: <e_r e_c^T, C> on the grid is separable into the
  // row sums and the column sums of e_r and e_c
  for (int x = tid; x < 4 * D; x += PWGS) {
    const int which = x / D, o = x % D;
    const float* G = which < 2 ? er : ec;
    double acc = 0.0;
    if (o < d) {
      if (which & 1)
        for (int i = 0; i < d; ++i) acc += (double)G[i * LDF + o];
      else
        for (int j = 0; j < d; ++j) acc += (double)G[o * LDF + j];
    }
    sums[x] = acc;
  }
  __syncthreads();
  double tr = 0.0;
  for (int x = tid; x < 2 * d * d; x += PWGS) {
    const int h = x / (d * d), y = x % (d * d), i = y / d, k = y % d;
    tr += sums[h * D + i] * c1d[i - k + D - 1] * sums[(2 + h) * D + k];
  }
  const double gs = block_sum<PNW>(g, s.red);
  const double en = block_sum<PNW>(ec1, s.red) + fabs(ecD);
  const double tt = block_sum<PNW>(tr, s.red) + ecD * block_sum<PNW>(ercd, s.red) + erD * block_sum<PNW>(eccd, s.red);
  __syncthreads();
  return gs + (en > 0.0 ? tt / en : 0.0);
}

// BOUNDS: also the error-control bounds (a kernel variant of its own, so
// that the plain solve keeps its register allocation).
template <int D, int SPT, bool BOUNDS>
__device__ __forceinline__ void solve_pair(const PairParams& prm, PairSmem<D>& s, long long pair) {
  const int tid = threadIdx.x;
  const int d = prm.d;

  if constexpr (D > 128) {
    if (tid == 0) s.gops = prm.ops + (size_t)blockIdx.x * GlobalOps<D>::BYTES;
  }
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
  SupList<SPT> ua, vb;   // u on supp(a), v on supp(b)
  if constexpr (SPT == 0) {
    int* base = reinterpret_cast<int*>(prm.lists + (size_t)blockIdx.x * prm.list_stride);
    constexpr int CAP = D * D;
    ua = SupList<0>{base, reinterpret_cast<float*>(base + CAP), reinterpret_cast<float*>(base + 2 * CAP),
                    base + 3 * CAP, base + 4 * CAP, 0, CAP};
    base += 5 * CAP;
    vb = SupList<0>{base, reinterpret_cast<float*>(base + CAP), reinterpret_cast<float*>(base + 2 * CAP),
                    base + 3 * CAP, base + 4 * CAP, 0, CAP};
    if (tid == 0) s.gsusp = base + 5 * CAP;   // suspect arrays after the two lists
  }
  bool big_a, big_b, low_a, low_b;
  const double mA = build_support<D, SPT>(s, A, d, ua, big_a, low_a);
  const double mB = build_support<D, SPT>(s, B, d, vb, big_b, low_b);
  const bool tri = !low_a && !low_b;   // u and v vanish below the diagonal
  if (big_a || big_b) {
    if (tid == 0) prm.redo[pair] = (unsigned char)(prm.only_redo + 1);
    return;
  }
  if (tid == 0) prm.redo[pair] = (unsigned char)prm.only_redo;
  const double aD = mB, bD = mA, m = mA + mB;
  if (m <= 0.0) {
    if (tid == 0) {
      prm.cost[pair] = 0.0;
      prm.iters[2 * pair] = 0;
      prm.iters[2 * pair + 1] = 0;
      prm.err[pair] = 0.0f;
      prm.status[pair] = 0;
      if (prm.done) post_done(prm.done, prm.done_tag, pair, 0.0, 0, 0, 0.0f, 0);
      if constexpr (BOUNDS) {
        if (prm.upper) prm.upper[pair] = 0.0;
        if (prm.lower) prm.lower[pair] = 0.0;
      }
    }
    return;
  }
  WarmState<D>* ws = prm.state ? reinterpret_cast<WarmState<D>*>(prm.state) + pair : nullptr;
  const bool warm = ws && prm.state_in;

  bool lowp = prm.precision == 1;
  const int nka = ua.nk(), nkb = vb.nk();
  ESum kv{NEG, 0.0};
  Side su{0, 0.0, 0}, sv{0, 1.0, 0};
  bool v_dense;   // v is the all-ones start (dense, not on supp(b))
  zero_x<D>(s, lowp);
  if (warm) {
    // v from the previous solve of this pair (it lives on supp(b)).
    for (int r = tid; r < D; r += PWGS) {
      s.Pv[r] = ws->Pv[r];
      s.Qv[r] = ws->Qv[r];
      s.Pu[r] = NEG;
      s.Qu[r] = NEG;
    }
    sv = Side{ws->vex, ws->vmx, ws->mres};
    __syncthreads();
#pragma unroll
    for (int k = 0; k < nkb; ++k) {
      const int c = vb.cell(k);
      if (c >= 0) {
        const float r = ws->vres[c];
        vb.set_res(k, r);
        put_x<D>(s, c, r, lowp);
        const int i = c / D, j = c % D, dl = j - i + D - 1;
        kv = esum_add(kv, ESum{s.Pv[i] + s.Qv[j] + s.tgde[dl], (double)r * (double)s.tgdm[dl]});
      }
    }
    v_dense = false;
  } else {
    // v = 1 on every grid cell and on the diagonal bin.
    for (int r = tid; r < D; r += PWGS) {
      s.Pv[r] = r < d ? 0 : NEG;
      s.Qv[r] = r < d ? 0 : NEG;
      s.Pu[r] = NEG;
      s.Qu[r] = NEG;
    }
    __syncthreads();
    for (int c = tid; c < d * d; c += PWGS) {
      const int i = c / d, j = c % d;
      put_x<D>(s, i * D + j, 1.0f, lowp);
      kv = esum_add(kv, ESum{s.tgde[j - i + D - 1], (double)s.tgdm[j - i + D - 1]});
    }
#pragma unroll
    for (int k = 0; k < nkb; ++k) vb.set_res(k, 1.0f);
    v_dense = true;
  }
#pragma unroll
  for (int k = 0; k < nka; ++k) ua.set_q(k, QNONE);
  kv = esum_add(block_esum<PNW>(kv, s.rede, s.reds), ESum{sv.ex, sv.mx});   // (K v)_Delta = <v, k_Delta> + v_Delta
  ESum ku{NEG, 0.0};

  int t = 0, it_lp = 0, it_hp = 0, bad = 0, range = 0;
  if (warm && sv.mres > 100) range |= 1;   // a warm start whose residuals FP32 cannot hold
  bool x_lp = lowp;      // format of the residual currently in the X buffer
  double err = INFINITY;
  __syncthreads();
  for (;;) {
    // u-update: u = a / K v, after checking the marginal error of (u, v).
    const bool lp_now = lowp;
    const int Hv = headroom(sv.mres);
    const float* Wb = apply_K<D>(s, s.Pv, s.Qv, d, Hv, lp_now, tri && !v_dense, tri);
    bool stop = false;
    ESum dotu;
    const double errD = (t >= 1) ? fabs(ldxd(su.mx * kv.s, su.ex + kv.e) - aD) : 0.0;
    y_update<D, SPT>(s, Wb, lp_now, ua, vb, v_dense, d, sv, Hv, s.Pv, s.Qv, s.Pu, s.Qu, lp_now,
                     v_dense || x_lp != lp_now, t >= 1, err, stop, dotu, su.mres, bad, range, errD, m, prm.tol,
                     prm.switch_tol, lowp, t, prm.max_iter);
    if (stop || bad) break;
    if (SPT == 1 && (range & 2)) break;
    x_lp = lp_now;
    su.ex = -kv.e;
    su.mx = aD / kv.s;
    ku = esum_add(dotu, ESum{su.ex, su.mx});
    // v-update: v = b / K^T u (K is symmetric).  No barrier needed here: the
    // update ended with one, and the next shared-memory writes (refit
    // extrema, scales, kernels) touch nothing read after it.
    const int Hu = headroom(su.mres);
    Wb = apply_K<D>(s, s.Pu, s.Qu, d, Hu, lp_now, tri, tri);
    ESum dotv;
    bool nostop = false;
    double dummy = 0.0;
    y_update<D, SPT>(s, Wb, lp_now, vb, ua, false, d, su, Hu, s.Pu, s.Qu, s.Pv, s.Qv, lowp, x_lp != lowp, false,
                     dummy, nostop, dotv, sv.mres, bad, range, 0.0, m, prm.tol, prm.switch_tol, lowp, t,
                     prm.max_iter);
    v_dense = false;
    x_lp = lowp;
    sv.ex = -ku.e;
    sv.mx = bD / ku.s;
    kv = esum_add(dotv, ESum{sv.ex, sv.mx});
    ++t;
    if (lp_now) ++it_lp;
    else ++it_hp;
    if (bad) break;
    if (SPT == 1 && (range & 2)) break;
  }
  if (SPT == 1 && (range & 2)) {
    // The LDS suspect list overflowed: the global-list variant, whose
    // suspect arrays hold every cell, solves the pair again from the start.
    if (tid == 0) prm.redo[pair] = (unsigned char)(prm.only_redo + 1);
    return;
  }

  // Transport cost of Proposition 3 for (u_t, v_t), FP32 contractions and FP64 sums:
  //   sum_ij u_ij (m V k^T + k V m^T)_ij + u_Delta <V, m_Delta> + v_Delta <U, m_Delta>.
  // R, S still hold the scales of the kernels built from (Pv, Qv), and q marks
  // the entries of supp(a) whose K v needed the exact path: their first term
  // is recomputed the same way.
  __syncthreads();
  zero_x<D>(s, false);
  __syncthreads();
  if (v_dense) {
    for (int c = tid; c < d * d; c += PWGS) put_x<D>(s, (c / d) * D + (c % d), 1.0f, false);
  } else {
#pragma unroll
    for (int k = 0; k < nkb; ++k) {
      const int c = vb.cell(k);
      if (c >= 0) put_x<D>(s, c, vb.res(k), false);
    }
  }
  __syncthreads();
  double g = 0.0;
  float* Wf = wbuf<D>(s, false);
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) contract<D, false, false, true>(s, s.Pv, s.Qv, Wf, tri && !v_dense, tri, d);
    else contract<D, false, true, false>(s, s.Pv, s.Qv, Wf, tri && !v_dense, tri, d);
#pragma unroll
    for (int k = 0; k < nka; ++k) {
      const int c = ua.cell(k);
      if (c >= 0 && ua.q(k) < QSUSP) {
        const float r = ua.res(k);
        if (r > 0.0f) {
          const int i = c / D, j = c % D;
          g += ldxd((double)r * (double)Wf[i * Cfg<D>::LDF + j], s.Pu[i] + s.Qu[j] + s.R[i] + s.S[j]);
        }
      }
    }
    __syncthreads();
  }
  const int ns = bad ? 0 : min(s.nsusp, suspCap<D, SPT>());
  if (ns > 0) {
    exact_all<D, SPT, true, false>(s, vb, v_dense, d, s.Pv, s.Qv, ns, suspE<D, SPT>(s), suspM<D, SPT>(s));
#pragma unroll
    for (int k = 0; k < nka; ++k) {
      const int qk = ua.q(k);
      if (qk >= QSUSP) {
        const float r = ua.res(k);
        if (r > 0.0f) {
          const int c = ua.cell(k), i = c / D, j = c % D;
          const int id = qk - QSUSP;
          g += ldxd((double)r * (double)suspM<D, SPT>(s)[id], suspE<D, SPT>(s)[id] + s.Pu[i] + s.Qu[j]);
        }
      }
    }
  }
  const double lnvD = log(sv.mx) + (double)sv.ex * 0.69314718055994530942;   // log v_Delta
#pragma unroll
  for (int k = 0; k < nka; ++k) {
    const int c = ua.cell(k);
    if (c >= 0) {
      const float r = ua.res(k);
      const int i = c / D, j = c % D, dl = j - i + D - 1;
      if (r > 0.0f)
        g += ldxd(sv.mx * (double)r * (double)s.tgdm[dl] * (double)s.tcd[dl], sv.ex + s.Pu[i] + s.Qu[j] + s.tgde[dl]);
      if (prm.gout) {
        // gradient term of Proposition 5 at this cell: log u + log v_Delta
        const double lu = r > 0.0f ? (log((double)r) + (double)(s.Pu[i] + s.Qu[j]) * 0.69314718055994530942) : 0.0;
        prm.gout[(size_t)pair * d * d + i * d + j] = lu + lnvD;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < nkb; ++k) {
    const int c = vb.cell(k);
    if (c >= 0) {
      const float r = vb.res(k);
      if (!v_dense && r > 0.0f) {
        const int i = c / D, j = c % D, dl = j - i + D - 1;
        g += ldxd(su.mx * (double)r * (double)s.tgdm[dl] * (double)s.tcd[dl], su.ex + s.Pv[i] + s.Qv[j] + s.tgde[dl]);
      }
      if (ws && !v_dense) ws->vres[c] = r;
    }
  }
  if (ws && !v_dense) {
    for (int r = tid; r < D; r += PWGS) {
      ws->Pv[r] = s.Pv[r];
      ws->Qv[r] = s.Qv[r];
    }
    if (tid == 0) {
      ws->vex = sv.ex;
      ws->vmx = sv.mx;
      ws->mres = sv.mres;
    }
  }
  const double cost = block_sum<PNW>(g, s.red);
  if constexpr (BOUNDS) {
    // needs a u from at least one iteration
    double up = NAN, lo = NAN;
    if (!bad && t > 0) {
      double* c1d = reinterpret_cast<double*>(&s.fit[0][0][0]);
      double* cdd = c1d + 2 * D;
      for (int x = tid; x < 2 * D; x += PWGS) {
        const double dl = fabs((double)(x - (D - 1)));
        c1d[x] = pow(dl / d, prm.p);
        cdd[x] = 2.0 * pow(dl / (2.0 * d), prm.p);
      }
      __syncthreads();
      if (prm.lower) lo = lower_bound<D, SPT>(s, ua, vb, su, d, prm.gamma, aD, bD, c1d, cdd);
      if (prm.upper) up = upper_bound<D, SPT>(s, ua, vb, su, sv, kv, d, aD, bD, c1d, cdd);
    }
    if (tid == 0) {
      if (prm.upper) prm.upper[pair] = up;
      if (prm.lower) prm.lower[pair] = lo;
    }
  }
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
}

// One workgroup per pair; the grid may be smaller than the batch (global-list
// variant), in which case each workgroup takes pairs blockIdx.x, + gridDim.x, ...
template <int D, int SPT, bool BOUNDS = false>
__global__ __launch_bounds__(PWGS) void sinkhorn_pair_kernel(PairParams prm) {
  __shared__ PairSmem<D> s;
  if (prm.stop && *prm.stop) return;
  if constexpr (SPT > 0 && D <= 128) {   // one pair per workgroup
    const long long pair = prm.perm ? prm.perm[blockIdx.x] : blockIdx.x;
    if (prm.only_redo && prm.redo[pair] != prm.only_redo) return;
    solve_pair<D, SPT, BOUNDS>(prm, s, pair);
  } else {
    for (long long idx = blockIdx.x; idx < prm.n_pairs; idx += gridDim.x) {
      const long long pair = (SPT > 0 && prm.perm) ? prm.perm[idx] : idx;
      if (prm.only_redo && prm.redo[pair] != prm.only_redo) continue;
      solve_pair<D, SPT, BOUNDS>(prm, s, pair);
      __syncthreads();
    }
  }
}

}  // namespace pdsink
