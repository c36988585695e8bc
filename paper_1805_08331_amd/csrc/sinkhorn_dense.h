// Dense fused per-pair Sinkhorn kernel: Algorithm 1 of Lacombe, Cuturi, Oudot
// (NeurIPS 2018) on the d x d grid plus the diagonal bin, with the scaling
// vectors held as dense grids.  It computes the same iteration as the
// compact-support kernel and serves the pairs whose histogram supports are too
// large for that kernel's per-thread lists (any support, up to the full grid).
// One workgroup per pair; every iterate stays in LDS and registers.
//
// Work layout.  The grid is padded to D = 32, 64 or 128 and cut into 32 x 32
// tiles; the workgroup has one wave per tile.  A wave computes its tile of
// both contractions of Proposition 2 on the matrix cores and owns the 16 grid
// cells of its accumulator layout (lane l, register r: row 8(r/4) + 4(l/32) +
// r%4, column l%32 of the tile), so the result of K x is consumed straight
// from the accumulators by the elementwise update.
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

#include "sinkhorn_pair.h"  // PairParams

namespace pdsink {
namespace dense {

constexpr int MAXSUSP = 256;   // suspects handled per half step
constexpr int XCHUNK = 4;      // suspects evaluated together
constexpr int QSUSP = 1 << 28; // per-cell marker: cell is suspect number q - QSUSP
constexpr int CELLS = 16;      // grid cells per lane (one 32x32 accumulator tile per wave)
constexpr int HEAD = 40;       // kernel headroom octaves for an input residual within 2^20

template <int D>
struct Cfg {
  static constexpr int NT = D / 32;        // tiles per grid dimension
  static constexpr int NW = NT * NT;       // waves: one output tile each
  static constexpr int WGS = NW * 64;      // threads per workgroup
  static constexpr int LDF = D + 1;        // FP32 row stride: rows start in different banks
  static constexpr int LDB = D + 8;        // BF16 row stride: 16-byte aligned rows
};

template <int D>
struct PairSmem {
  using C = Cfg<D>;
  union {
    struct {
      float X[D * C::LDF];    // input residual (A operand of contraction 1)
      float T[D * C::LDF];    // X kt2^T, row-major [k][j]
    } f;
    struct {
      __bf16 X[D * C::LDB];
      __bf16 Tt[D * C::LDB];  // X kt2^T, transposed [j][k] (B operand of contraction 2)
      __bf16 K1[D * C::LDB];  // kt1 [i][k]
      __bf16 K2[D * C::LDB];  // kt2 [j][l]
    } b;
  } u;
  int tge[2 * D], tgde[2 * D];
  float tgm[2 * D], tgdm[2 * D], tc1[2 * D], tcd[2 * D];
  int Pu[D], Qu[D], Pv[D], Qv[D], R[D], S[D];
  int rmx[D], rmn[D], cmx[D], cmn[D], rho[D], sig[D];
  double red[C::NW];
  double reds[C::NW];
  int rede[C::NW];
  int redi[C::NW];
  int nsusp;
  int susp_cell[MAXSUSP];
  int susp_e[MAXSUSP];     // value = susp_m * 2^susp_e (natural scale, or absolute for the cost)
  float susp_m[MAXSUSP];
  int susp_q[MAXSUSP];
  int xmax[C::NW][XCHUNK];
  float xsum[C::NW][XCHUNK];
};

// Grid coordinates of register r of the calling lane (accumulator layout).
template <int D>
struct Cell {
  int i0, j;
  __device__ Cell() {
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));   // recompute per use instead of holding every cell's offsets live
    const int lane = tid & 63, w = tid >> 6;
    i0 = (w / Cfg<D>::NT) * 32 + 4 * (lane >> 5);
    j = (w % Cfg<D>::NT) * 32 + (lane & 31);
  }
  __device__ int i(int r) const { return i0 + 8 * (r >> 2) + (r & 3); }
};

// Keeps the scheduler from interleaving the unrolled per-cell iterations (which
// would hold every cell's temporaries live at once and spill).
__device__ __forceinline__ void cell_fence() { __builtin_amdgcn_sched_barrier(0); }

// Kernel headroom for an input whose residual spans +-mres octaves.
__device__ __forceinline__ int headroom(int mres) { return max(0, min(HEAD, HEAD + 20 - mres)); }

// R_i = max_k (P_k + ge(i - k)) - H over valid input rows k; rows i >= d get BIG
// so that their kernel rows are exactly zero.
template <int D>
__device__ __forceinline__ void compute_RS(PairSmem<D>& s, const int* P, const int* Q, int d, int H) {
  for (int r = threadIdx.x; r < 2 * D; r += Cfg<D>::WGS) {
    const bool rows = r < D;
    const int i = rows ? r : r - D;
    const int* X = rows ? P : Q;
    int best = BIG;
    if (i < d) {
      best = NEG;
#pragma unroll 4
      for (int k = 0; k < d; ++k) {
        const int p = X[k];
        if (p > NEG / 2) best = max(best, p + s.tge[i - k + D - 1]);
      }
      best = best <= NEG / 2 ? 0 : best - H;   // empty input: every kernel entry is 0 anyway
    }
    (rows ? s.R : s.S)[i] = best;
  }
}

template <int D, bool WEIGHTED>
__device__ __forceinline__ float kentry(const PairSmem<D>& s, int i, int k, const int* P, int Ri) {
  const int idx = i - k + D - 1;
  float v = ldx(s.tgm[idx], P[k] + s.tge[idx] - Ri);
  if (WEIGHTED) v *= s.tc1[idx];
  return v;
}

// BF16 kernels of one application into LDS: K1[i][k] from P and R, K2[j][l]
// from Q and S; 16 consecutive entries of one row per thread.
template <int D>
__device__ __forceinline__ void build_kernels_bf16(PairSmem<D>& s, const int* P, const int* Q) {
  constexpr int LDB = Cfg<D>::LDB;
  for (int e0 = threadIdx.x * 16; e0 < 2 * D * D; e0 += Cfg<D>::WGS * 16) {
    const bool first = e0 < D * D;
    const int e = first ? e0 : e0 - D * D;
    const int i = e / D, k0 = e % D;
    const int* X = first ? P : Q;
    const int Ri = (first ? s.R : s.S)[i];
    __bf16* dst = (first ? s.u.b.K1 : s.u.b.K2) + i * LDB + k0;
    bf16x8 v0, v1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      v0[t] = (__bf16)kentry<D, false>(s, i, k0 + t, X, Ri);
      v1[t] = (__bf16)kentry<D, false>(s, i, k0 + 8 + t, X, Ri);
    }
    *reinterpret_cast<bf16x8*>(dst) = v0;
    *reinterpret_cast<bf16x8*>(dst + 8) = v1;
  }
}

// Contraction 1 of Proposition 2 for the calling wave's tile (tk, tj):
//   T[k][j] = sum_l X[k][l] * kt2[j][l]   (kt2 times c1 when WEIGHTED: the m of Prop. 3)
template <int D, bool BF16, bool WEIGHTED>
__device__ __forceinline__ void gemm_xk(PairSmem<D>& s, const int* Q) {
  constexpr int NT = Cfg<D>::NT, LDF = Cfg<D>::LDF, LDB = Cfg<D>::LDB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 31, lk = lane >> 5;
  const int tk = w / NT, tj = w % NT;
  const int row = tk * 32 + lr, j = tj * 32 + lr;
  floatx16 acc = {};
  if constexpr (BF16) {
    const __bf16* xa = s.u.b.X + row * LDB + 8 * lk;
    const __bf16* kb = s.u.b.K2 + j * LDB + 8 * lk;
#pragma unroll 2
    for (int l0 = 0; l0 < D; l0 += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(xa + l0);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(kb + l0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    mfma_drain();
#pragma unroll
    for (int r = 0; r < 16; ++r) s.u.b.Tt[j * LDB + tk * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)] = (__bf16)acc[r];
  } else {
    const int Sj = s.S[j];
#pragma unroll 4
    for (int l0 = 0; l0 < D; l0 += 2) {
      const int l = l0 + lk;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(s.u.f.X[row * LDF + l], kentry<D, WEIGHTED>(s, j, l, Q, Sj), acc,
                                                 0, 0, 0);
    }
    mfma_drain();
#pragma unroll
    for (int r = 0; r < 16; ++r) s.u.f.T[(tk * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc[r];
  }
}

// Contraction 2 for the calling wave's tile (ti, tj), result left in registers:
//   W[i][j] = sum_k kt1[i][k] * T[k][j]   (kt1 times c1 when WEIGHTED)
template <int D, bool BF16, bool WEIGHTED>
__device__ __forceinline__ floatx16 gemm_kt(PairSmem<D>& s, const int* P) {
  constexpr int NT = Cfg<D>::NT, LDF = Cfg<D>::LDF, LDB = Cfg<D>::LDB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 31, lk = lane >> 5;
  const int ti = w / NT, tj = w % NT;
  const int i = ti * 32 + lr, j = tj * 32 + lr;
  floatx16 acc = {};
  if constexpr (BF16) {
    const __bf16* ka = s.u.b.K1 + i * LDB + 8 * lk;
    const __bf16* tb = s.u.b.Tt + j * LDB + 8 * lk;
#pragma unroll 2
    for (int k0 = 0; k0 < D; k0 += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(ka + k0);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(tb + k0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
  } else {
    const int Ri = s.R[i];
#pragma unroll 4
    for (int k0 = 0; k0 < D; k0 += 2) {
      const int k = k0 + lk;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(kentry<D, WEIGHTED>(s, i, k, P, Ri), s.u.f.T[k * LDF + j], acc,
                                                 0, 0, 0);
    }
  }
  mfma_drain();
  return acc;
}

// (K x) on the grid for input scales P, Q (residual already in the X buffer of
// the matching format); returns the calling lane's 16 cells, scaled by
// 2^-(R_i + S_j).
template <int D>
__device__ __forceinline__ floatx16 apply_K(PairSmem<D>& s, const int* P, const int* Q, int d, int H, bool lowp) {
  compute_RS<D>(s, P, Q, d, H);
  __syncthreads();
  floatx16 W;
  if (lowp) {
    build_kernels_bf16<D>(s, P, Q);
    __syncthreads();
    gemm_xk<D, true, false>(s, Q);
    __syncthreads();
    W = gemm_kt<D, true, false>(s, P);
  } else {
    gemm_xk<D, false, false>(s, Q);
    __syncthreads();
    W = gemm_kt<D, false, false>(s, P);
  }
  __syncthreads();
  return W;
}

// Store the calling lane's 16 cells of a residual as the next contraction input.
template <int D>
__device__ __forceinline__ void store_x(PairSmem<D>& s, const float (&xt)[CELLS], bool bf16) {
  const Cell<D> c;
#pragma unroll
  for (int r = 0; r < CELLS; ++r) {
    cell_fence();
    if (bf16) s.u.b.X[c.i(r) * Cfg<D>::LDB + c.j] = (__bf16)xt[r];
    else s.u.f.X[c.i(r) * Cfg<D>::LDF + c.j] = xt[r];
  }
}

// Residual of the calling lane's cell r as stored in the X buffer.
template <int D>
__device__ __forceinline__ float load_x(const PairSmem<D>& s, const Cell<D>& c, int r, bool bf16) {
  return bf16 ? (float)s.u.b.X[c.i(r) * Cfg<D>::LDB + c.j] : s.u.f.X[c.i(r) * Cfg<D>::LDF + c.j];
}

// Exact values for the suspects [base, base + cnt) from the input x (residual
// in the X buffer in format x_bf16, scales Px, Qx): sum over the support of x of K_(ij),(kl) x_kl (times
// C_(ij),(kl) when WEIGHTED, Proposition 3) with explicit exponents: pass 1
// takes each target's largest term exponent, pass 2 the sum of the terms
// scaled by it.  Writes mantissa and absolute log2 exponent to out_m / out_e.
template <int D, bool WEIGHTED>
__device__ __forceinline__ void exact_chunk(PairSmem<D>& s, bool x_bf16, const int* Px, const int* Qx, int base, int cnt,
                            int* out_e, float* out_m) {
  constexpr int NW = Cfg<D>::NW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Cell<D> cl;
  int ti[XCHUNK], tj[XCHUNK], em[XCHUNK];
#pragma unroll
  for (int t = 0; t < XCHUNK; ++t) {
    const int c = t < cnt ? s.susp_cell[base + t] : 0;
    ti[t] = c / D;
    tj[t] = c % D;
    em[t] = QNONE;
  }
#pragma unroll
  for (int r = 0; r < CELLS; ++r) {
    cell_fence();
    const float x = load_x<D>(s, cl, r, x_bf16);
    if (x > 0.0f) {
      const int k = cl.i(r), l = cl.j;
      const int eb = Px[k] + Qx[l] + ilog2f(x);
#pragma unroll
      for (int t = 0; t < XCHUNK; ++t) em[t] = max(em[t], eb + s.tge[ti[t] - k + D - 1] + s.tge[tj[t] - l + D - 1]);
    }
  }
#pragma unroll
  for (int t = 0; t < XCHUNK; ++t) em[t] = wave_max(em[t]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < XCHUNK; ++t) s.xmax[wave][t] = em[t];
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < XCHUNK; ++t) {
    int v = s.xmax[0][t];
#pragma unroll 4
    for (int w = 1; w < NW; ++w) v = max(v, s.xmax[w][t]);
    em[t] = v;
  }
  float acc[XCHUNK];
#pragma unroll
  for (int t = 0; t < XCHUNK; ++t) acc[t] = 0.0f;
#pragma unroll
  for (int r = 0; r < CELLS; ++r) {
    cell_fence();
    const float x = load_x<D>(s, cl, r, x_bf16);
    if (x > 0.0f) {
      const int k = cl.i(r), l = cl.j;
      const int eb = Px[k] + Qx[l];
#pragma unroll
      for (int t = 0; t < XCHUNK; ++t) {
        const int i1 = ti[t] - k + D - 1, i2 = tj[t] - l + D - 1;
        float mm = x * s.tgm[i1] * s.tgm[i2];
        if (WEIGHTED) mm *= (s.tc1[i1] + s.tc1[i2]);
        acc[t] += ldx(mm, eb + s.tge[i1] + s.tge[i2] - em[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < XCHUNK; ++t) acc[t] = wave_sum(acc[t]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < XCHUNK; ++t) s.xsum[wave][t] = acc[t];
  }
  __syncthreads();
  if (tid < cnt) {
    float v = 0.0f;
    int e = s.xmax[0][tid];
#pragma unroll 4
    for (int w = 0; w < NW; ++w) {
      v += s.xsum[w][tid];
      e = max(e, s.xmax[w][tid]);
    }
    out_e[tid] = e;
    out_m[tid] = v;
  }
  __syncthreads();
}

// State of one side of the pair (u or v) as seen by the update of the other.
struct Side {
  int ex;      // diagonal entry = mx * 2^ex
  double mx;
  int mres;    // residual span (octaves) of its last update
};

// y = target / (K x), with the lane's cells of K x in W (scaled by 2^-(R+S)),
// except at the suspects.  Refits y's scales (Py, Qy), writes the new residual
// to yt and, in format out_bf16, to the X buffer, and returns the grid part of
// <y, k_Delta>.  When `check`, first measures the row-marginal error of the
// previous y against K x and may stop there, leaving yt, Py, Qy untouched and
// q holding the suspect markers.
template <int D>
__device__ __forceinline__ void y_update(PairSmem<D>& s, const floatx16& W, const float* __restrict__ tgt, int d, const Side& xs,
                         int H, bool x_bf16, const int* Px, const int* Qx, float (&yt)[CELLS],
                         int (&q)[CELLS], int* Py, int* Qy, bool out_bf16, bool check, double& err_out,
                         bool& stop_out, ESum& dot, int& mres_out, int& bad, int& range, double errD, double m,
                         double tol, double switch_tol, bool& lowp, int t, int max_iter) {
  constexpr int NW = Cfg<D>::NW, WGS = Cfg<D>::WGS;
  const int tid = threadIdx.x;
  const Cell<D> cl;
  const float mxf = (float)xs.mx;
  // Trusted level of a normalised value: everything the contractions drop is
  // below 2^(H + mres + 14 - 126) in these units; keep a 2^-40 relative margin.
  const int thr = H + max(xs.mres, 20) + 14 - 126 + 40;
  if (tid == 0) s.nsusp = 0;
  __syncthreads();
  int lbad = 0, lover = 0;
#pragma unroll
  for (int r = 0; r < CELLS; ++r) {
    cell_fence();
    const int i = cl.i(r), j = cl.j;
    const float tv = (i < d && j < d) ? tgt[i * d + j] : 0.0f;
    if (tv > 0.0f) {
      const float w = W[r];
      const int dl = j - i + D - 1;
      const int E = xs.ex + s.tgde[dl] - s.R[i] - s.S[j];
      const float Dm = mxf * s.tgdm[dl];
      const int lw = w > 0.0f ? ilog2f(w) : QNONE;
      const int ld = Dm > 0.0f ? E + ilog2f(Dm) : QNONE;
      const int le = max(lw, ld);
      if (le < thr) {
        const int id = atomicAdd(&s.nsusp, 1);
        if (id < MAXSUSP) {
          s.susp_cell[id] = i * D + j;
          q[r] = QSUSP + id;
        } else {
          lover = 1;
          if (le == QNONE) lbad = 1;
          q[r] = le == QNONE ? 0 : ilog2f(tv) - le;
        }
      } else {
        q[r] = ilog2f(tv) - le;
      }
    } else {
      q[r] = QNONE;
    }
  }
  __syncthreads();
  const int ns = min(s.nsusp, MAXSUSP);
  if (ns > 0) {
    for (int base = 0; base < ns; base += XCHUNK)
      exact_chunk<D, false>(s, x_bf16, Px, Qx, base, min(XCHUNK, ns - base), s.susp_e + base, s.susp_m + base);
    for (int id = tid; id < ns; id += WGS) {
      const int c = s.susp_cell[id], i = c / D, j = c % D;
      const int dl = j - i + D - 1;
      const ESum g{s.susp_e[id] - s.R[i] - s.S[j], (double)s.susp_m[id]};
      const ESum tot = esum_add(g, ESum{xs.ex + s.tgde[dl] - s.R[i] - s.S[j], (double)(mxf * s.tgdm[dl])});
      if (!(tot.s > 0.0)) {
        lbad = 1;
        s.susp_e[id] = 0;
        s.susp_m[id] = 1.0f;
        s.susp_q[id] = 0;
      } else {
        const float mt = (float)tot.s;
        s.susp_e[id] = tot.e;
        s.susp_m[id] = mt;
        s.susp_q[id] = ilog2f(tgt[i * d + j]) - (tot.e + ilog2f(mt));
      }
    }
    __syncthreads();
  }
  if (check) {
    double eg = 0.0;
#pragma unroll
    for (int r = 0; r < CELLS; ++r) {
    cell_fence();
      if (q[r] != QNONE) {
        const int i = cl.i(r), j = cl.j;
        const float tv = tgt[i * d + j];
        const int sh = Py[i] + Qy[j] + s.R[i] + s.S[j];
        double row;
        if (q[r] >= QSUSP) {
          const int id = q[r] - QSUSP;
          row = ldxd((double)yt[r] * (double)s.susp_m[id], s.susp_e[id] + sh);
        } else {
          const int dl = j - i + D - 1;
          const int E = xs.ex + s.tgde[dl] - s.R[i] - s.S[j];
          const float Dm = mxf * s.tgdm[dl];
          row = ldxd((double)yt[r] * (double)W[r], sh) + ldxd((double)yt[r] * (double)Dm, E + sh);
        }
        eg += fabs(row - (double)tv);
      }
    }
    eg = block_sum<NW>(eg, s.red);
    err_out = (eg + errD) / m;
    const bool measured_lowp = lowp;   // never stop on an error measured with BF16 contractions
    if (lowp && err_out <= switch_tol) lowp = false;
    if ((!measured_lowp && err_out <= tol) || t >= max_iter) {
      stop_out = true;
      if (__syncthreads_or(lbad)) bad = 1;
      return;
    }
  }
  if (__syncthreads_or(lbad)) bad = 1;
  if (__syncthreads_or(lover)) range = 1;

  // Two sweeps of row/column centring of the log2 estimates.
  for (int r = tid; r < D; r += WGS) {
    s.rho[r] = 0;
    s.sig[r] = 0;
  }
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int r = tid; r < D; r += WGS) {
      s.rmx[r] = INT_MIN;
      s.rmn[r] = INT_MAX;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CELLS; ++r) {
    cell_fence();
      if (q[r] != QNONE) {
        const int i = cl.i(r), j = cl.j;
        const int qv = q[r] >= QSUSP ? s.susp_q[q[r] - QSUSP] : q[r];
        const int v = qv - s.sig[j];
        atomicMax(&s.rmx[i], v);
        atomicMin(&s.rmn[i], v);
      }
    }
    __syncthreads();
    for (int r = tid; r < D; r += WGS) {
      s.rho[r] = s.rmx[r] != INT_MIN ? ((s.rmx[r] + s.rmn[r]) >> 1) : 0;
      s.cmx[r] = INT_MIN;
      s.cmn[r] = INT_MAX;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CELLS; ++r) {
    cell_fence();
      if (q[r] != QNONE) {
        const int i = cl.i(r), j = cl.j;
        const int qv = q[r] >= QSUSP ? s.susp_q[q[r] - QSUSP] : q[r];
        const int v = qv - s.rho[i];
        atomicMax(&s.cmx[j], v);
        atomicMin(&s.cmn[j], v);
      }
    }
    __syncthreads();
    for (int r = tid; r < D; r += WGS) s.sig[r] = s.cmx[r] != INT_MIN ? ((s.cmx[r] + s.cmn[r]) >> 1) : 0;
    __syncthreads();
  }
  for (int r = tid; r < D; r += WGS) {
    Py[r] = s.rmx[r] != INT_MIN ? s.rho[r] - s.R[r] : NEG;
    Qy[r] = s.cmx[r] != INT_MIN ? s.sig[r] - s.S[r] : NEG;
  }
  __syncthreads();

  ESum acc{NEG, 0.0};
  int maxres = 0;
#pragma unroll
  for (int r = 0; r < CELLS; ++r) {
    cell_fence();
    float y = 0.0f;
    if (q[r] != QNONE) {
      const int i = cl.i(r), j = cl.j;
      const float tv = tgt[i * d + j];
      const int dl = j - i + D - 1;
      const int sh = s.rho[i] + s.sig[j];
      int qv;
      if (q[r] >= QSUSP) {
        const int id = q[r] - QSUSP;
        y = tv / ldx(s.susp_m[id], s.susp_e[id] + sh);
        qv = s.susp_q[id];
      } else {
        const int E = xs.ex + s.tgde[dl] - s.R[i] - s.S[j];
        const float Dm = mxf * s.tgdm[dl];
        y = tv / (ldx(W[r], sh) + ldx(Dm, E + sh));
        qv = q[r];
      }
      maxres = max(maxres, abs(qv - sh));
      acc = esum_add(acc, ESum{Py[i] + Qy[j] + s.tgde[dl], (double)y * (double)s.tgdm[dl]});
    }
    yt[r] = y;
  }
  __syncthreads();   // the exact path may still be reading x from the X buffer
  store_x<D>(s, yt, out_bf16);
  dot = block_esum<NW>(acc, s.rede, s.reds);
  mres_out = block_max<NW>(maxres, s.redi) + 1;
  if (mres_out > 100) range = 1;
}

template <int D>
__global__ __launch_bounds__(Cfg<D>::WGS) void sinkhorn_pair_kernel(PairParams prm) {
  using C = Cfg<D>;
  constexpr int NW = C::NW, WGS = C::WGS;
  __shared__ PairSmem<D> s;
  const int tid = threadIdx.x;
  const long long pair = blockIdx.x;
  if (prm.redo[pair] != prm.only_redo) return;
  const int d = prm.d;
  const Cell<D> cl;

  for (int x = tid; x < 2 * D; x += WGS) {
    const bool in = x < 2 * D - 1;
    s.tge[x] = in ? prm.ge[x] : NEG;
    s.tgm[x] = in ? prm.gm[x] : 0.0f;
    s.tgde[x] = in ? prm.gde[x] : NEG;
    s.tgdm[x] = in ? prm.gdm[x] : 0.0f;
    s.tc1[x] = in ? prm.c1[x] : 0.0f;
    s.tcd[x] = in ? prm.cd[x] : 0.0f;
  }
  const float* __restrict__ A = prm.hist_a + (size_t)prm.ia[pair] * d * d;
  const float* __restrict__ B = prm.hist_b + (size_t)prm.ib[pair] * d * d;
  double sa = 0.0, sb = 0.0;
  for (int c = tid; c < d * d; c += WGS) {
    sa += A[c];
    sb += B[c];
  }
  const double mA = block_sum<NW>(sa, s.red);
  const double mB = block_sum<NW>(sb, s.red);
  const double aD = mB, bD = mA, m = mA + mB;
  if (m <= 0.0) {
    if (tid == 0) {
      prm.cost[pair] = 0.0;
      prm.iters[2 * pair] = 0;
      prm.iters[2 * pair + 1] = 0;
      prm.err[pair] = 0.0f;
      prm.status[pair] = 0;
    }
    return;
  }

  bool lowp = prm.precision == 1;
  // u lives in registers (ut) and, between its update and the next contraction,
  // in the X buffer; v lives in the X buffer only.
  float ut[CELLS];
  int q[CELLS];
  // v = 1 on every grid cell and on the diagonal bin.
  for (int r = tid; r < D; r += WGS) {
    s.Pv[r] = r < d ? 0 : NEG;
    s.Qv[r] = r < d ? 0 : NEG;
    s.Pu[r] = NEG;
    s.Qu[r] = NEG;
  }
  ESum kv{NEG, 0.0};
  {
    float v0[CELLS];
#pragma unroll
    for (int r = 0; r < CELLS; ++r) {
    cell_fence();
      const int i = cl.i(r), j = cl.j;
      const bool in = i < d && j < d;
      v0[r] = in ? 1.0f : 0.0f;
      ut[r] = 0.0f;
      q[r] = QNONE;
      if (in) kv = esum_add(kv, ESum{s.tgde[j - i + D - 1], (double)s.tgdm[j - i + D - 1]});
    }
    __syncthreads();
    store_x<D>(s, v0, lowp);
  }
  Side su{0, 0.0, 0}, sv{0, 1.0, 0};
  kv = esum_add(block_esum<NW>(kv, s.rede, s.reds), ESum{0, 1.0});   // (K v)_Delta = <v, k_Delta> + v_Delta
  ESum ku{NEG, 0.0};

  int t = 0, it_lp = 0, it_hp = 0, bad = 0, range = 0;
  bool x_lp = lowp;    // format of the residual currently in the X buffer
  double err = INFINITY;
  __syncthreads();
  for (;;) {
    // u-update: u = a / K v, after checking the marginal error of (u, v).
    const bool lp_now = lowp;
    const int Hv = headroom(sv.mres);
    floatx16 W = apply_K<D>(s, s.Pv, s.Qv, d, Hv, lp_now);
    bool stop = false;
    ESum dotu;
    const double errD = (t >= 1) ? fabs(ldxd(su.mx * kv.s, su.ex + kv.e) - aD) : 0.0;
    y_update<D>(s, W, A, d, sv, Hv, x_lp, s.Pv, s.Qv, ut, q, s.Pu, s.Qu, lp_now, t >= 1, err, stop, dotu, su.mres,
                bad, range, errD, m, prm.tol, prm.switch_tol, lowp, t, prm.max_iter);
    if (stop || bad) break;
    x_lp = lp_now;
    su.ex = -kv.e;
    su.mx = aD / kv.s;
    ku = esum_add(dotu, ESum{su.ex, su.mx});
    __syncthreads();
    // v-update: v = b / K^T u (K is symmetric).
    const int Hu = headroom(su.mres);
    W = apply_K<D>(s, s.Pu, s.Qu, d, Hu, lp_now);
    ESum dotv;
    bool nostop = false;
    double dummy = 0.0;
    {
      float vnew[CELLS];
      y_update<D>(s, W, B, d, su, Hu, x_lp, s.Pu, s.Qu, vnew, q, s.Pv, s.Qv, lowp, false, dummy, nostop, dotv,
                  sv.mres, bad, range, 0.0, m, prm.tol, prm.switch_tol, lowp, t, prm.max_iter);
    }
    x_lp = lowp;
    sv.ex = -ku.e;
    sv.mx = bD / ku.s;
    kv = esum_add(dotv, ESum{sv.ex, sv.mx});
    ++t;
    if (lp_now) ++it_lp;
    else ++it_hp;
    __syncthreads();
    if (bad) break;
  }

  // Transport cost of Proposition 3 for (u_t, v_t), FP32 contractions and FP64 sums:
  //   sum_ij u_ij (m V k^T + k V m^T)_ij + u_Delta <V, m_Delta> + v_Delta <U, m_Delta>.
  // R, S still hold the scales of the kernels built from (Pv, Qv), and q marks
  // the cells of supp(a) whose K v needed the exact path: their first term is
  // recomputed the same way.  v is in the X buffer; as FP32 from here on.
  __syncthreads();
  if (x_lp) {
    float v32[CELLS];
#pragma unroll
    for (int r = 0; r < CELLS; ++r) v32[r] = load_x<D>(s, cl, r, true);
    __syncthreads();
    store_x<D>(s, v32, false);
  }
  __syncthreads();
  double g = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) gemm_xk<D, false, false>(s, s.Qv);
    else gemm_xk<D, false, true>(s, s.Qv);
    __syncthreads();
    const floatx16 M = pass == 0 ? gemm_kt<D, false, true>(s, s.Pv) : gemm_kt<D, false, false>(s, s.Pv);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CELLS; ++r) {
    cell_fence();
      if (ut[r] > 0.0f && q[r] < QSUSP) {
        const int i = cl.i(r), j = cl.j;
        g += ldxd((double)ut[r] * (double)M[r], s.Pu[i] + s.Qu[j] + s.R[i] + s.S[j]);
      }
    }
  }
  const int ns = bad ? 0 : min(s.nsusp, MAXSUSP);
  if (ns > 0) {
    for (int base = 0; base < ns; base += XCHUNK)
      exact_chunk<D, true>(s, false, s.Pv, s.Qv, base, min(XCHUNK, ns - base), s.susp_e + base, s.susp_m + base);
#pragma unroll
    for (int r = 0; r < CELLS; ++r) {
    cell_fence();
      if (q[r] >= QSUSP && ut[r] > 0.0f) {
        const int i = cl.i(r), j = cl.j;
        const int id = q[r] - QSUSP;
        g += ldxd((double)ut[r] * (double)s.susp_m[id], s.susp_e[id] + s.Pu[i] + s.Qu[j]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < CELLS; ++r) {
    cell_fence();
    const int i = cl.i(r), j = cl.j;
    const int dl = j - i + D - 1;
    const double w = (double)s.tgdm[dl] * (double)s.tcd[dl];
    const float vr = load_x<D>(s, cl, r, false);
    if (vr > 0.0f) g += ldxd(su.mx * (double)vr * w, su.ex + s.Pv[i] + s.Qv[j] + s.tgde[dl]);
    if (ut[r] > 0.0f) g += ldxd(sv.mx * (double)ut[r] * w, sv.ex + s.Pu[i] + s.Qu[j] + s.tgde[dl]);
  }
  const double cost = block_sum<NW>(g, s.red);
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
  }
}

}  // namespace dense
}  // namespace pdsink
