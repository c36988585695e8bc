// Fused per-pair Sinkhorn kernel: Algorithm 1 of Lacombe, Cuturi, Oudot
// (NeurIPS 2018) on the d x d grid plus the diagonal bin, one workgroup per
// pair, every iterate resident in LDS and registers.
//
// Numerical representation (the paper is silent on stabilisation).  A scaling
// vector x on the grid is stored as x_ij = 2^(P_i + Q_j) * xt_ij with integer
// row/column log2 scales P, Q (int32) and an FP32 residual xt; the diagonal
// entry as m * 2^e.  Because 2^(P_i + Q_j) factors over rows and columns, the
// separable K application of Proposition 2 stays a pair of 1-D contractions:
//   K x (grid) = 2^(R_i + S_j) * (kt1 * Xt * kt2^T)_ij + x_Delta k_Delta,ij
// with per-row/column "absorbed" 1-D kernels
//   kt1[i][k] = 2^(P_k + g(i-k) - R_i),  R_i = max_k (P_k + ge(i-k)),
// g(delta) = -(|delta|/d)^p / gamma * log2(e), and kt2 likewise from Q.  Each
// kernel entry is built exactly as ldexp(mantissa(delta), integer exponent),
// from per-context tables, without transcendental instructions.
//
// After each half step the new scaling y = target / (K x) is re-expressed:
// natural scales (-R, -S) plus integer offsets (rho, sigma) obtained by two
// sweeps of row/column centring of the per-cell log2 estimates, which keeps
// the residual within a few tens of octaves (the non-separable part of the
// potentials).  All of this is exact re-representation of the same iterates:
// only FP32 rounding of the contractions and divisions remains.
//
// The two separable normalisations cannot see every four-index product: at a
// few cells, every term of (K x)_ij can fall below the FP32 range even though
// the value matters.  Everything the contractions drop is below ~2^-82 in the
// natural scale, so a cell whose normalised value is >= 2^-40 is exact to
// ~2^-42 relative; cells below that ("suspects") are recomputed exactly, as a
// sum over the input's support with explicit exponents, and those exact values
// are used for the update, the marginal error and the transport cost.
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
};

constexpr int MAXSUSP = 256;   // suspects handled per half step
constexpr int XCHUNK = 8;      // suspects evaluated together
constexpr int QSUSP = 1 << 28; // q marker: cell is suspect number q - QSUSP
constexpr int SUSP_LOG2 = -40; // trusted range of a normalised K x value

template <int D>
struct PairSmem {
  static constexpr int LDF = D + 1;   // +1 float: consecutive rows start in different banks
  float buf[2][D * LDF];
  int tge[2 * D], tgde[2 * D];
  float tgm[2 * D], tgdm[2 * D], tc1[2 * D], tcd[2 * D];
  int Pu[D], Qu[D], Pv[D], Qv[D], R[D], S[D];
  int rmx[D], rmn[D], cmx[D], cmn[D], rho[D], sig[D];
  double red[NWAVE];
  double reds[NWAVE];
  int rede[NWAVE];
  int redi[NWAVE];
  // cells whose separable value fell below the trusted range, recomputed exactly
  int nsusp;
  int susp_cell[MAXSUSP];
  int susp_e[MAXSUSP];     // exact value = susp_m * 2^susp_e, in the natural scale 2^(R_i + S_j)
  float susp_m[MAXSUSP];
  int susp_q[MAXSUSP];
  int xmax[NWAVE][XCHUNK];
  float xsum[NWAVE][XCHUNK];
};

// R_i = max_k (P_k + ge(i - k)) over valid input rows k; rows i >= d get BIG so
// that their kernel rows are exactly zero.
template <int D>
__device__ void compute_RS(PairSmem<D>& s, const int* P, const int* Q, int d) {
  for (int r = threadIdx.x; r < 2 * D; r += WG) {
    const bool rows = r < D;
    const int i = rows ? r : r - D;
    const int* X = rows ? P : Q;
    int best = BIG;
    if (i < d) {
      best = NEG;
      for (int k = 0; k < d; ++k) {
        const int p = X[k];
        if (p > NEG / 2) best = max(best, p + s.tge[i - k + D - 1]);
      }
      if (best <= NEG / 2) best = 0;   // empty input: every kernel entry is 0 anyway
    }
    (rows ? s.R : s.S)[i] = best;
  }
}

// GEMM 1 of Proposition 2:  T[k][j] = sum_l X[k][l] * kt2[j][l],
// kt2[j][l] = 2^(Q_l + g(j-l) - S_j) (times c1(j-l) when WEIGHTED: the m kernel
// of Proposition 3).  32x32 output tiles spread over the 4 waves.
template <int D, bool BF16, bool WEIGHTED>
__device__ void gemm_xk(const PairSmem<D>& s, const float* X, float* T, const int* Q) {
  constexpr int NT = D / 32, LDF = PairSmem<D>::LDF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 31, lk = lane >> 5;
  for (int t = wave; t < NT * NT; t += NWAVE) {
    const int ti = t / NT, tj = t % NT;
    const int row = ti * 32 + lr, j = tj * 32 + lr;
    const int Sj = s.S[j];
    floatx16 acc = {};
    if constexpr (BF16) {
      for (int l0 = 0; l0 < D; l0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int l = l0 + 8 * lk + e;
          const int idx = j - l + D - 1;
          float kv = ldx(s.tgm[idx], Q[l] + s.tge[idx] - Sj);
          if (WEIGHTED) kv *= s.tc1[idx];
          a[e] = (__bf16)X[row * LDF + l];
          b[e] = (__bf16)kv;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
      for (int l0 = 0; l0 < D; l0 += 2) {
        const int l = l0 + lk;
        const int idx = j - l + D - 1;
        float kv = ldx(s.tgm[idx], Q[l] + s.tge[idx] - Sj);
        if (WEIGHTED) kv *= s.tc1[idx];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(X[row * LDF + l], kv, acc, 0, 0, 0);
      }
    }
    mfma_drain();
#pragma unroll
    for (int r = 0; r < 16; ++r) T[(ti * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc[r];
  }
}

// GEMM 2 of Proposition 2:  W[i][j] = sum_k kt1[i][k] * T[k][j],
// kt1[i][k] = 2^(P_k + g(i-k) - R_i) (times c1(i-k) when WEIGHTED).
template <int D, bool BF16, bool WEIGHTED>
__device__ void gemm_kt(const PairSmem<D>& s, const float* T, float* W, const int* P) {
  constexpr int NT = D / 32, LDF = PairSmem<D>::LDF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 31, lk = lane >> 5;
  for (int t = wave; t < NT * NT; t += NWAVE) {
    const int ti = t / NT, tj = t % NT;
    const int i = ti * 32 + lr, j = tj * 32 + lr;
    const int Ri = s.R[i];
    floatx16 acc = {};
    if constexpr (BF16) {
      for (int k0 = 0; k0 < D; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = k0 + 8 * lk + e;
          const int idx = i - k + D - 1;
          float kv = ldx(s.tgm[idx], P[k] + s.tge[idx] - Ri);
          if (WEIGHTED) kv *= s.tc1[idx];
          a[e] = (__bf16)kv;
          b[e] = (__bf16)T[k * LDF + j];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
      for (int k0 = 0; k0 < D; k0 += 2) {
        const int k = k0 + lk;
        const int idx = i - k + D - 1;
        float kv = ldx(s.tgm[idx], P[k] + s.tge[idx] - Ri);
        if (WEIGHTED) kv *= s.tc1[idx];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(kv, T[k * LDF + j], acc, 0, 0, 0);
      }
    }
    mfma_drain();
#pragma unroll
    for (int r = 0; r < 16; ++r) W[(ti * 32 + 8 * (r >> 2) + 4 * lk + (r & 3)) * LDF + j] = acc[r];
  }
}

// K x on the grid into IN (its input X is consumed), using TMP for T.
template <int D>
__device__ void apply_K(PairSmem<D>& s, float* IN, float* TMP, const int* P, const int* Q, int d, bool lowp) {
  compute_RS<D>(s, P, Q, d);
  __syncthreads();
  if (lowp) gemm_xk<D, true, false>(s, IN, TMP, Q);
  else gemm_xk<D, false, false>(s, IN, TMP, Q);
  __syncthreads();
  if (lowp) gemm_kt<D, true, false>(s, TMP, IN, P);
  else gemm_kt<D, false, false>(s, TMP, IN, P);
  __syncthreads();
}


// Exact values for the suspects [base, base + cnt) from the input x (residual
// xt in registers, scales Px, Qx): sum over the support of x of
// K_(ij),(kl) x_kl (times C_(ij),(kl) when WEIGHTED, Proposition 3), with
// explicit exponents: pass 1 takes each target's largest term exponent, pass 2
// the sum of the terms scaled by it.  Writes mantissa and absolute log2
// exponent of each target's value to out_m / out_e.
template <int D, bool WEIGHTED>
__device__ void exact_chunk(PairSmem<D>& s, const float (&xt)[D * D / WG], const int* Px, const int* Qx, int base,
                            int cnt, int* out_e, float* out_m) {
  constexpr int NC = D * D / WG;
  constexpr int LOGD = (D == 32) ? 5 : (D == 64) ? 6 : 7;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int ti[XCHUNK], tj[XCHUNK], em[XCHUNK];
#pragma unroll
  for (int t = 0; t < XCHUNK; ++t) {
    const int c = t < cnt ? s.susp_cell[base + t] : 0;
    ti[t] = c >> LOGD;
    tj[t] = c & (D - 1);
    em[t] = QNONE;
  }
#pragma unroll
  for (int kk = 0; kk < NC; ++kk) {
    const float x = xt[kk];
    if (x > 0.0f) {
      const int c = tid + WG * kk, k = c >> LOGD, l = c & (D - 1);
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
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) v = max(v, s.xmax[w][t]);
    em[t] = v;
  }
  float acc[XCHUNK];
#pragma unroll
  for (int t = 0; t < XCHUNK; ++t) acc[t] = 0.0f;
#pragma unroll
  for (int kk = 0; kk < NC; ++kk) {
    const float x = xt[kk];
    if (x > 0.0f) {
      const int c = tid + WG * kk, k = c >> LOGD, l = c & (D - 1);
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
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) v += s.xsum[w][tid];
    out_e[tid] = s.xmax[0][tid];
    for (int w = 1; w < NWAVE; ++w) out_e[tid] = max(out_e[tid], s.xmax[w][tid]);
    out_m[tid] = v;
  }
  __syncthreads();
}

// y = target / (K x), with K x (scaled by 2^(R_i + S_j)) in Wb except at the
// suspects, and x_Delta = mx 2^ex.  Refits y's scales (Py, Qy), writes the new
// residual to yt (registers) and Ob (operand of the next contraction) and
// returns the grid part of <y, k_Delta>.  When `check`, first measures the
// row-marginal error of the previous y against (K x) and may stop there,
// leaving yt, Py, Qy untouched and q holding the suspect markers.
template <int D>
__device__ void y_update(PairSmem<D>& s, const float* Wb, float* Ob, const float* __restrict__ tgt, int d, int ex,
                         double mx, const float (&xt)[D * D / WG], const int* Px, const int* Qx,
                         float (&yt)[D * D / WG], int (&q)[D * D / WG], int* Py, int* Qy, bool check,
                         double& err_out, bool& stop_out, ESum& dot, int& bad, int& range, double errD, double m,
                         double tol, double switch_tol, bool& lowp, int t, int max_iter) {
  constexpr int NC = D * D / WG, LDF = PairSmem<D>::LDF;
  constexpr int LOGD = (D == 32) ? 5 : (D == 64) ? 6 : 7;
  const int tid = threadIdx.x;
  const float mxf = (float)mx;
  if (tid == 0) s.nsusp = 0;
  __syncthreads();
  int lbad = 0, lover = 0;
#pragma unroll
  for (int kk = 0; kk < NC; ++kk) {
    const int c = tid + WG * kk;
    const int i = c >> LOGD, j = c & (D - 1);
    const float tv = (i < d && j < d) ? tgt[i * d + j] : 0.0f;
    if (tv > 0.0f) {
      const float W = Wb[i * LDF + j];
      const int dl = j - i + D - 1;
      const int E = ex + s.tgde[dl] - s.R[i] - s.S[j];
      const float Dm = mxf * s.tgdm[dl];
      const int lw = W > 0.0f ? ilog2f(W) : QNONE;
      const int ld = Dm > 0.0f ? E + ilog2f(Dm) : QNONE;
      const int le = max(lw, ld);
      if (le < SUSP_LOG2) {
        const int id = atomicAdd(&s.nsusp, 1);
        if (id < MAXSUSP) {
          s.susp_cell[id] = c;
          q[kk] = QSUSP + id;
        } else {
          lover = 1;
          if (le == QNONE) lbad = 1;
          q[kk] = le == QNONE ? 0 : ilog2f(tv) - le;
        }
      } else {
        q[kk] = ilog2f(tv) - le;
      }
    } else {
      q[kk] = QNONE;
    }
  }
  __syncthreads();
  const int ns = min(s.nsusp, MAXSUSP);
  if (ns > 0) {
    for (int base = 0; base < ns; base += XCHUNK)
      exact_chunk<D, false>(s, xt, Px, Qx, base, min(XCHUNK, ns - base), s.susp_e + base, s.susp_m + base);
    for (int id = tid; id < ns; id += WG) {
      const int c = s.susp_cell[id], i = c >> LOGD, j = c & (D - 1);
      const int dl = j - i + D - 1;
      const ESum g{s.susp_e[id] - s.R[i] - s.S[j], (double)s.susp_m[id]};
      const ESum tot = esum_add(g, ESum{ex + s.tgde[dl] - s.R[i] - s.S[j], (double)(mxf * s.tgdm[dl])});
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
    for (int kk = 0; kk < NC; ++kk) {
      if (q[kk] != QNONE) {
        const int c = tid + WG * kk;
        const int i = c >> LOGD, j = c & (D - 1);
        const float tv = tgt[i * d + j];
        const int sh = Py[i] + Qy[j] + s.R[i] + s.S[j];
        double row;
        if (q[kk] >= QSUSP) {
          const int id = q[kk] - QSUSP;
          row = ldxd((double)yt[kk] * (double)s.susp_m[id], s.susp_e[id] + sh);
        } else {
          const float W = Wb[i * LDF + j];
          const int dl = j - i + D - 1;
          const int E = ex + s.tgde[dl] - s.R[i] - s.S[j];
          const float Dm = mxf * s.tgdm[dl];
          row = ldxd((double)yt[kk] * (double)W, sh) + ldxd((double)yt[kk] * (double)Dm, E + sh);
        }
        eg += fabs(row - (double)tv);
      }
    }
    eg = block_sum(eg, s.red);
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
  for (int r = tid; r < D; r += WG) {
    s.rho[r] = 0;
    s.sig[r] = 0;
  }
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int r = tid; r < D; r += WG) {
      s.rmx[r] = INT_MIN;
      s.rmn[r] = INT_MAX;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < NC; ++kk) {
      if (q[kk] != QNONE) {
        const int c = tid + WG * kk;
        const int i = c >> LOGD, j = c & (D - 1);
        const int qv = q[kk] >= QSUSP ? s.susp_q[q[kk] - QSUSP] : q[kk];
        const int v = qv - s.sig[j];
        atomicMax(&s.rmx[i], v);
        atomicMin(&s.rmn[i], v);
      }
    }
    __syncthreads();
    for (int r = tid; r < D; r += WG) {
      s.rho[r] = s.rmx[r] != INT_MIN ? ((s.rmx[r] + s.rmn[r]) >> 1) : 0;
      s.cmx[r] = INT_MIN;
      s.cmn[r] = INT_MAX;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < NC; ++kk) {
      if (q[kk] != QNONE) {
        const int c = tid + WG * kk;
        const int i = c >> LOGD, j = c & (D - 1);
        const int qv = q[kk] >= QSUSP ? s.susp_q[q[kk] - QSUSP] : q[kk];
        const int v = qv - s.rho[i];
        atomicMax(&s.cmx[j], v);
        atomicMin(&s.cmn[j], v);
      }
    }
    __syncthreads();
    for (int r = tid; r < D; r += WG) s.sig[r] = s.cmx[r] != INT_MIN ? ((s.cmx[r] + s.cmn[r]) >> 1) : 0;
    __syncthreads();
  }
  for (int r = tid; r < D; r += WG) {
    Py[r] = s.rmx[r] != INT_MIN ? s.rho[r] - s.R[r] : NEG;
    Qy[r] = s.cmx[r] != INT_MIN ? s.sig[r] - s.S[r] : NEG;
  }
  __syncthreads();

  ESum acc{NEG, 0.0};
  int maxres = 0;
#pragma unroll
  for (int kk = 0; kk < NC; ++kk) {
    const int c = tid + WG * kk;
    const int i = c >> LOGD, j = c & (D - 1);
    float y = 0.0f;
    if (q[kk] != QNONE) {
      const float tv = tgt[i * d + j];
      const int dl = j - i + D - 1;
      const int sh = s.rho[i] + s.sig[j];
      int qv;
      if (q[kk] >= QSUSP) {
        const int id = q[kk] - QSUSP;
        y = tv / ldx(s.susp_m[id], s.susp_e[id] + sh);
        qv = s.susp_q[id];
      } else {
        const float W = Wb[i * LDF + j];
        const int E = ex + s.tgde[dl] - s.R[i] - s.S[j];
        const float Dm = mxf * s.tgdm[dl];
        y = tv / (ldx(W, sh) + ldx(Dm, E + sh));
        qv = q[kk];
      }
      maxres = max(maxres, abs(qv - sh));
      acc = esum_add(acc, ESum{Py[i] + Qy[j] + s.tgde[dl], (double)y * (double)s.tgdm[dl]});
    }
    yt[kk] = y;
    Ob[i * LDF + j] = y;
  }
  dot = block_esum(acc, s.rede, s.reds);
  if (block_max(maxres, s.redi) > 100) range = 1;
}

template <int D>
__global__ __launch_bounds__(WG) void sinkhorn_pair_kernel(PairParams prm) {
  constexpr int NC = D * D / WG, LDF = PairSmem<D>::LDF;
  constexpr int LOGD = (D == 32) ? 5 : (D == 64) ? 6 : 7;
  __shared__ PairSmem<D> s;
  const int tid = threadIdx.x;
  const long long pair = blockIdx.x;
  const int d = prm.d;

  for (int x = tid; x < 2 * D; x += WG) {
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
  for (int c = tid; c < d * d; c += WG) {
    sa += A[c];
    sb += B[c];
  }
  const double mA = block_sum(sa, s.red);
  const double mB = block_sum(sb, s.red);
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

  float* IN = s.buf[0];
  float* TMP = s.buf[1];
  float ut[NC], vt[NC];
  int q[NC];
  // v = 1 on every grid cell and on the diagonal bin.
  for (int r = tid; r < D; r += WG) {
    s.Pv[r] = r < d ? 0 : NEG;
    s.Qv[r] = r < d ? 0 : NEG;
    s.Pu[r] = NEG;
    s.Qu[r] = NEG;
  }
  ESum kv{NEG, 0.0};
#pragma unroll
  for (int kk = 0; kk < NC; ++kk) {
    const int c = tid + WG * kk;
    const int i = c >> LOGD, j = c & (D - 1);
    const bool in = i < d && j < d;
    vt[kk] = in ? 1.0f : 0.0f;
    ut[kk] = 0.0f;
    q[kk] = QNONE;
    IN[i * LDF + j] = vt[kk];
    if (in) kv = esum_add(kv, ESum{s.tgde[j - i + D - 1], (double)s.tgdm[j - i + D - 1]});
  }
  int ev = 0, eu = 0;
  double mv = 1.0, mu = 0.0;
  kv = esum_add(block_esum(kv, s.rede, s.reds), ESum{0, 1.0});   // (K v)_Delta = <v, k_Delta> + v_Delta
  ESum ku{NEG, 0.0};

  int t = 0, it_lp = 0, it_hp = 0, bad = 0, range = 0;
  bool lowp = prm.precision == 1;
  double err = INFINITY;
  __syncthreads();
  for (;;) {
    // u-update: u = a / K v, after checking the marginal error of (u, v).
    const bool lp_now = lowp;
    apply_K<D>(s, IN, TMP, s.Pv, s.Qv, d, lp_now);
    bool stop = false;
    ESum dotu;
    const double errD = (t >= 1) ? fabs(ldxd(mu * kv.s, eu + kv.e) - aD) : 0.0;
    y_update<D>(s, IN, TMP, A, d, ev, mv, vt, s.Pv, s.Qv, ut, q, s.Pu, s.Qu, t >= 1, err, stop, dotu, bad, range,
                errD, m, prm.tol, prm.switch_tol, lowp, t, prm.max_iter);
    if (stop || bad) break;
    eu = -kv.e;
    mu = aD / kv.s;
    ku = esum_add(dotu, ESum{eu, mu});
    float* sw = IN;
    IN = TMP;
    TMP = sw;
    __syncthreads();
    // v-update: v = b / K^T u (K is symmetric).
    apply_K<D>(s, IN, TMP, s.Pu, s.Qu, d, lp_now);
    ESum dotv;
    bool nostop = false;
    double dummy = 0.0;
    y_update<D>(s, IN, TMP, B, d, eu, mu, ut, s.Pu, s.Qu, vt, q, s.Pv, s.Qv, false, dummy, nostop, dotv, bad, range,
                0.0, m, prm.tol, prm.switch_tol, lowp, t, prm.max_iter);
    ev = -ku.e;
    mv = bD / ku.s;
    kv = esum_add(dotv, ESum{ev, mv});
    sw = IN;
    IN = TMP;
    TMP = sw;
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
  // recomputed the same way.
  double g = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < NC; ++kk) {
      const int c = tid + WG * kk;
      IN[(c >> LOGD) * LDF + (c & (D - 1))] = vt[kk];
    }
    __syncthreads();
    if (pass == 0) gemm_xk<D, false, false>(s, IN, TMP, s.Qv);
    else gemm_xk<D, false, true>(s, IN, TMP, s.Qv);
    __syncthreads();
    if (pass == 0) gemm_kt<D, false, true>(s, TMP, IN, s.Pv);
    else gemm_kt<D, false, false>(s, TMP, IN, s.Pv);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < NC; ++kk) {
      const int c = tid + WG * kk;
      const int i = c >> LOGD, j = c & (D - 1);
      if (ut[kk] > 0.0f && q[kk] < QSUSP) {
        const int sh = s.Pu[i] + s.Qu[j] + s.R[i] + s.S[j];
        g += ldxd((double)ut[kk] * (double)IN[i * LDF + j], sh);
      }
    }
  }
  const int ns = bad ? 0 : min(s.nsusp, MAXSUSP);
  if (ns > 0) {
    for (int base = 0; base < ns; base += XCHUNK)
      exact_chunk<D, true>(s, vt, s.Pv, s.Qv, base, min(XCHUNK, ns - base), s.susp_e + base, s.susp_m + base);
#pragma unroll
    for (int kk = 0; kk < NC; ++kk) {
      if (q[kk] >= QSUSP && ut[kk] > 0.0f) {
        const int c = tid + WG * kk;
        const int i = c >> LOGD, j = c & (D - 1);
        const int id = q[kk] - QSUSP;
        g += ldxd((double)ut[kk] * (double)s.susp_m[id], s.susp_e[id] + s.Pu[i] + s.Qu[j]);
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < NC; ++kk) {
    const int c = tid + WG * kk;
    const int i = c >> LOGD, j = c & (D - 1);
    const int dl = j - i + D - 1;
    const double w = (double)s.tgdm[dl] * (double)s.tcd[dl];
    if (vt[kk] > 0.0f) g += ldxd(mu * (double)vt[kk] * w, eu + s.Pv[i] + s.Qv[j] + s.tgde[dl]);
    if (ut[kk] > 0.0f) g += ldxd(mv * (double)ut[kk] * w, ev + s.Pu[i] + s.Qu[j] + s.tgde[dl]);
  }
  const double cost = block_sum(g, s.red);
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

}  // namespace pdsink
