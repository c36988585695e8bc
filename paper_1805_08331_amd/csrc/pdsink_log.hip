// Log-domain Sinkhorn for the pairs that the scaled solve flags.
//
// The scaled solve keeps u and v as 2^(P_i + Q_j) times an FP32 residual.
// When the kernel is so sharp that one grid step costs tens of octaves
// (gamma d^2 well below 1), the scalings stop being close to a row times
// column product and the residual leaves its range (status RANGE, or a
// vanished product, NONFINITE).  This path reruns such a pair from the start
// with the same iteration (alternating updates from v = 1, u first, the
// marginal error of section 3 checked before every u-update, Proposition 3's
// cost) written with log-sum-exp in FP64 over the two supports:
//   log u_c = log a_c - LSE_e(log v_e - C_ce / gamma)   (e over supp(b) and Delta)
// and likewise for v, with C_ce = c(i - k) + c(j - l) on the grid and
// c_Delta on the diagonal bin.  The first u-update sees v = 1 on every grid
// cell, whose sum factors over the two axes.  Work per iteration is
// O(|supp a| |supp b|) exponentials, each to FP32 accuracy from an FP64
// argument; maxima, logarithms and the cost are FP64.
#include <hip/hip_runtime.h>

#include <math.h>

#include "pdsink_device.h"
#include "sinkhorn_log.h"

namespace pdsink {

namespace {

constexpr int LWG = 512;
constexpr int LNW = LWG / 64;

// One support entry as a source of the log-sum-exps: its log scaling and its
// cell (i << 16) | j, read with one 16-byte load.
struct alignas(16) Src {
  double ls;
  int cell;
  int pad;
};

struct LogSmem {
  static constexpr int cap = LOG_CAP;   // support cells per side the arrays hold
  Src src[2][LOG_CAP];      // side 0: a (u), side 1: b (v)
  double lt[2][LOG_CAP];    // log targets
  double lk[2][LOG_CAP];    // log of the latest K application at each cell
  double c1d[512];          // c(delta) = (|delta| / d)^p, index delta + d - 1
  double cdd[512];          // c_Delta by delta = j - i, index delta + d - 1
  double red[LNW];
  int cnt[LWG];
  int n[2];
};

// The same lists in a global slice of the workspace slot (beyond the grid the
// lower bound uses), for supports beyond LOG_CAP cells; the tables and the
// reduction buffers stay in the workgroup's LDS.  The members mirror
// LogSmem's, so the solve below is written once for both.
struct LogGlobal {
  int cap;
  Src* stage;     // LDS staging area of STAGE source entries (the unused LDS lists)
  Src* src[2];
  double* lt[2];
  double* lk[2];
  double* c1d;
  double* cdd;
  double* red;
  int* cnt;
  int* n;
};

__device__ __forceinline__ double block_max_d(double v, double* red) { return -block_min<LNW>(-v, red); }

// exp(y) for y <= 0 to about 1e-7 relative: y log2(e) = n + f split in FP64
// (|f| <= 1/2), 2^f by the hardware base-2 exponential, then the exact 2^n.
// Below e^-700 (and for y = -inf) the result is 0.
__device__ __forceinline__ double exp_neg(double y) {
  if (!(y > -700.0)) return 0.0;
  const double t = y * 1.4426950408889634;
  const double n = rint(t);
  return ldexp((double)__builtin_amdgcn_exp2f((float)(t - n)), (int)n);
}

// log(exp(x) + exp(y)) for x, y that may be -inf.
__device__ __forceinline__ double lse2(double x, double y) {
  const double m = fmax(x, y);
  if (m == -INFINITY) return -INFINITY;
  return m + log(exp(x - m) + exp(y - m));
}

// Support list of one histogram, in cell order: counts per thread chunk, a
// serial scan of the 512 counts, then each thread writes its chunk.  Returns
// false (and leaves the list empty) when the support exceeds LOG_CAP.
template <class SM>
__device__ bool build_list(SM& S, int side, const float* __restrict__ h, int d) {
  const int n = d * d, per = (n + LWG - 1) / LWG;
  const int c0 = min((int)threadIdx.x * per, n), c1 = min(c0 + per, n);
  int k = 0;
  for (int c = c0; c < c1; ++c) k += h[c] > 0.0f;
  S.cnt[threadIdx.x] = k;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < LWG; ++t) {
      const int v = S.cnt[t];
      S.cnt[t] = acc;
      acc += v;
    }
    S.n[side] = acc;
  }
  __syncthreads();
  const int total = S.n[side];
  if (total > S.cap) return false;
  int off = S.cnt[threadIdx.x];
  for (int c = c0; c < c1; ++c) {
    const float v = h[c];
    if (v > 0.0f) {
      S.src[side][off].cell = ((c / d) << 16) | (c % d);
      S.lt[side][off] = log((double)v);
      ++off;
    }
  }
  __syncthreads();
  return true;
}

// LSE over the sources of side `src` (plus the diagonal-bin source xD) of
// ls - C / gamma at grid cell (i, j); four sources per step.  P2: the ground
// exponent is 2, so C = ((i - k)^2 + (j - l)^2) / d^2 without table reads.
template <bool P2, class SM>
__device__ __forceinline__ double lse_at(const SM& S, int src, int i, int j, int d, double xD, double ig) {
  const int ns = S.n[src];
  const Src* sr = S.src[src];
  const double* ci = S.c1d + i + d - 1;   // ci[-k] = c(i - k)
  const double* cj = S.c1d + j + d - 1;
  const double igd = ig / ((double)d * (double)d);
  auto x_of = [&](int e) {
    const Src q = sr[e];
    const int k = q.cell >> 16, l = q.cell & 0xFFFF;
    if constexpr (P2) {
      const int di = i - k, dj = j - l;
      return q.ls - (double)(di * di + dj * dj) * igd;
    } else {
      return q.ls - (ci[-k] + cj[-l]) * ig;
    }
  };
  double m0 = xD, m1 = -INFINITY, m2 = -INFINITY, m3 = -INFINITY;
  int e = 0;
  for (; e + 4 <= ns; e += 4) {
    m0 = fmax(m0, x_of(e));
    m1 = fmax(m1, x_of(e + 1));
    m2 = fmax(m2, x_of(e + 2));
    m3 = fmax(m3, x_of(e + 3));
  }
  for (; e < ns; ++e) m0 = fmax(m0, x_of(e));
  const double m = fmax(fmax(m0, m1), fmax(m2, m3));
  if (m == -INFINITY) return -INFINITY;
  double s0 = exp_neg(xD - m), s1 = 0.0, s2 = 0.0, s3 = 0.0;
  e = 0;
  for (; e + 4 <= ns; e += 4) {
    s0 += exp_neg(x_of(e) - m);
    s1 += exp_neg(x_of(e + 1) - m);
    s2 += exp_neg(x_of(e + 2) - m);
    s3 += exp_neg(x_of(e + 3) - m);
  }
  for (; e < ns; ++e) s0 += exp_neg(x_of(e) - m);
  return m + log((s0 + s1) + (s2 + s3));
}

// The same log-sum-exp with SPLIT lanes per target cell (adjacent lanes of
// a quad), each over every SPLIT-th source; the partial maxima and sums are
// combined across the quad.  Every lane of the group returns the result.
template <bool P2, int SPLIT, class SM>
__device__ __forceinline__ double lse_split(const SM& S, int src, int i, int j, int d, double xD, double ig,
                                            int part) {
  const int ns = S.n[src];
  const Src* sr = S.src[src];
  const double* ci = S.c1d + i + d - 1;
  const double* cj = S.c1d + j + d - 1;
  const double igd = ig / ((double)d * (double)d);
  auto x_of = [&](int e) {
    const Src q = sr[e];
    const int k = q.cell >> 16, l = q.cell & 0xFFFF;
    if constexpr (P2) {
      const int di = i - k, dj = j - l;
      return q.ls - (double)(di * di + dj * dj) * igd;
    } else {
      return q.ls - (ci[-k] + cj[-l]) * ig;
    }
  };
  double m0 = part == 0 ? xD : -INFINITY, m1 = -INFINITY;
  int e = part;
  for (; e + SPLIT < ns; e += 2 * SPLIT) {
    m0 = fmax(m0, x_of(e));
    m1 = fmax(m1, x_of(e + SPLIT));
  }
  if (e < ns) m0 = fmax(m0, x_of(e));
  double m = fmax(m0, m1);
  m = fmax(m, dpp_d<DPP_QXOR1>(m));
  if constexpr (SPLIT == 4) m = fmax(m, dpp_d<DPP_QXOR2>(m));
  if (m == -INFINITY) return -INFINITY;
  double s0 = part == 0 ? exp_neg(xD - m) : 0.0, s1 = 0.0;
  e = part;
  for (; e + SPLIT < ns; e += 2 * SPLIT) {
    s0 += exp_neg(x_of(e) - m);
    s1 += exp_neg(x_of(e + SPLIT) - m);
  }
  if (e < ns) s0 += exp_neg(x_of(e) - m);
  double sum = s0 + s1;
  sum += dpp_d<DPP_QXOR1>(sum);
  if constexpr (SPLIT == 4) sum += dpp_d<DPP_QXOR2>(sum);
  return m + log(sum);
}

// lk[tgt][e] = LSE over side `src` (plus the diagonal bin, log scaling xDb)
// of ls - C / gamma at every cell e of side tgt: four lanes per cell when
// the targets fit a quarter of the workgroup, two when they fit half.
template <bool P2, class SM>
__device__ void apply_lse(SM& S, int tgt, int src, int d, double xDb, double ig) {
  const int nt = S.n[tgt], tid = threadIdx.x;
  if (nt <= LWG / 4) {
    const int t = tid >> 2, part = tid & 3;
    if (t < nt) {
      const int c = S.src[tgt][t].cell, i = c >> 16, j = c & 0xFFFF;
      const double v = lse_split<P2, 4>(S, src, i, j, d, xDb - S.cdd[j - i + d - 1] * ig, ig, part);
      if (part == 0) S.lk[tgt][t] = v;
    }
  } else if (nt <= LWG / 2) {
    const int t = tid >> 1, part = tid & 1;
    if (t < nt) {
      const int c = S.src[tgt][t].cell, i = c >> 16, j = c & 0xFFFF;
      const double v = lse_split<P2, 2>(S, src, i, j, d, xDb - S.cdd[j - i + d - 1] * ig, ig, part);
      if (part == 0) S.lk[tgt][t] = v;
    }
  } else {
    for (int e = tid; e < nt; e += LWG) {
      const int c = S.src[tgt][e].cell, i = c >> 16, j = c & 0xFFFF;
      S.lk[tgt][e] = lse_at<P2>(S, src, i, j, d, xDb - S.cdd[j - i + d - 1] * ig, ig);
    }
  }
}

// apply_lse for lists in the workspace: the sources are staged through LDS
// in chunks of STAGE entries, and each thread keeps TPT targets in registers,
// so that one LDS read of a source serves TPT targets.  Per target a running
// maximum and a sum scaled to it (the log-sum-exp taken in one pass per
// chunk: the chunk's maximum, then its terms); the diagonal-bin source
// starts the sum.  Targets beyond LWG * TPT take further rounds.
constexpr int STAGE = 2 * LOG_CAP;
constexpr int TPT = 8;
template <bool P2>
__device__ void apply_lse(LogGlobal& G, int tgt, int src, int d, double xDb, double ig) {
  const int nt = G.n[tgt], ns = G.n[src], tid = threadIdx.x;
  const double igd = ig / ((double)d * (double)d);
  for (int r0 = 0; r0 < nt; r0 += LWG * TPT) {
    int ti[TPT], tj[TPT];
    double m[TPT], sm[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      const int t = r0 + tid + k * LWG;
      const bool ok = t < nt;
      const int c = ok ? G.src[tgt][t].cell : 0;
      ti[k] = c >> 16;
      tj[k] = c & 0xFFFF;
      m[k] = ok ? xDb - G.cdd[tj[k] - ti[k] + d - 1] * ig : -INFINITY;   // the diagonal-bin source
      sm[k] = ok ? 1.0 : 0.0;
    }
    for (int c0 = 0; c0 < ns; c0 += STAGE) {
      const int nc = min(STAGE, ns - c0);
      __syncthreads();
      for (int e = tid; e < nc; e += LWG) G.stage[e] = G.src[src][c0 + e];
      __syncthreads();
      auto x_of = [&](const Src& q, int k) {
        const int kk = q.cell >> 16, l = q.cell & 0xFFFF;
        if constexpr (P2) {
          const int di = ti[k] - kk, dj = tj[k] - l;
          return q.ls - (double)(di * di + dj * dj) * igd;
        } else {
          return q.ls - (G.c1d[ti[k] - kk + d - 1] + G.c1d[tj[k] - l + d - 1]) * ig;
        }
      };
      double cm[TPT];
#pragma unroll
      for (int k = 0; k < TPT; ++k) cm[k] = -INFINITY;
      for (int e = 0; e < nc; ++e) {
        const Src q = G.stage[e];
#pragma unroll
        for (int k = 0; k < TPT; ++k) cm[k] = fmax(cm[k], x_of(q, k));
      }
      double cs[TPT];
#pragma unroll
      for (int k = 0; k < TPT; ++k) {
        const double mn = fmax(m[k], cm[k]);
        cs[k] = mn == -INFINITY ? 0.0 : sm[k] * exp_neg(m[k] - mn);
        m[k] = mn;
      }
      for (int e = 0; e < nc; ++e) {
        const Src q = G.stage[e];
#pragma unroll
        for (int k = 0; k < TPT; ++k) cs[k] += exp_neg(x_of(q, k) - m[k]);
      }
#pragma unroll
      for (int k = 0; k < TPT; ++k) sm[k] = cs[k];
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      const int t = r0 + tid + k * LWG;
      if (t < nt) G.lk[tgt][t] = m[k] == -INFINITY ? -INFINITY : m[k] + log(sm[k]);
    }
  }
}

// LSE over the sources of side `src` plus xD of ls - c_Delta / gamma: the
// K application at the diagonal bin (C_Delta,Delta = 0).
template <class SM>
__device__ double lse_delta(SM& S, int src, int d, double xD, double ig) {
  const int n = S.n[src];
  double m = -INFINITY;
  for (int e = threadIdx.x; e < n; e += LWG) {
    const int c = S.src[src][e].cell, i = c >> 16, j = c & 0xFFFF;
    m = fmax(m, S.src[src][e].ls - S.cdd[j - i + d - 1] * ig);
  }
  m = fmax(block_max_d(m, S.red), xD);
  if (m == -INFINITY) return -INFINITY;
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += LWG) {
    const int c = S.src[src][e].cell, i = c >> 16, j = c & 0xFFFF;
    s += exp_neg(S.src[src][e].ls - S.cdd[j - i + d - 1] * ig - m);
  }
  s = block_sum<LNW>(s, S.red) + exp_neg(xD - m);
  return m + log(s);
}

// The error-control bounds of section 3 for the final log scalings (the
// same definitions as the scaled path's: lower = <alpha^{c cbar}, a> +
// <alpha^c, b> with alpha = gamma log u over the whole ground space; upper =
// <R, C> of the rounded plan, Proposition 4).

// In place over the rows (ROWS) or columns of the d x d grid g (row stride
// d + 1): g[r][o] <- min over x of c(o - x) + g[r][x]; one wave per line.
template <bool ROWS>
__device__ void log_minplus(double* g, const double* c1d, int d) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int LG = d + 1;
  for (int line = wave; line < d; line += LNW) {
    double acc[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    for (int x = 0; x < d; ++x) {
      const double gv = ROWS ? g[line * LG + x] : g[x * LG + line];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = min(lane + 64 * q, d - 1);
        acc[q] = fmin(acc[q], c1d[o - x + d - 1] + gv);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = lane + 64 * q;
      if (o < d) {
        if (ROWS) g[line * LG + o] = acc[q];
        else g[o * LG + line] = acc[q];
      }
    }
  }
}

template <class SM>
__device__ double log_lower_bound(SM& S, double* g, int d, double gamma, double luD, double aD, double bD) {
  const int tid = threadIdx.x, LG = d + 1;
  for (int c = tid; c < d * LG; c += LWG) g[c] = INFINITY;
  __syncthreads();
  const double alD = gamma * luD;
  double mD = -alD;
  for (int e = tid; e < S.n[0]; e += LWG) {
    const int c = S.src[0][e].cell, i = c >> 16, j = c & 0xFFFF;
    const double al = gamma * S.src[0][e].ls;
    g[i * LG + j] = -al;
    mD = fmin(mD, S.cdd[j - i + d - 1] - al);
  }
  const double acD = block_min<LNW>(mD, S.red);   // alpha^c at the diagonal bin
  log_minplus<true>(g, S.c1d, d);
  __syncthreads();
  log_minplus<false>(g, S.c1d, d);
  __syncthreads();
  double mg = -acD;
  for (int c = tid; c < d * d; c += LWG) {
    const int i = c / d, j = c % d;
    const double cd = S.cdd[j - i + d - 1];
    const double v = fmin(g[i * LG + j], cd - alD);   // alpha^c on the grid
    g[i * LG + j] = -v;
    mg = fmin(mg, cd - v);
  }
  const double accD = block_min<LNW>(mg, S.red);  // alpha^{c cbar} at the diagonal bin
  double sb = 0.0;
  for (int e = tid; e < S.n[1]; e += LWG) {
    const int c = S.src[1][e].cell, i = c >> 16, j = c & 0xFFFF;
    sb -= exp(S.lt[1][e]) * g[i * LG + j];
  }
  sb = block_sum<LNW>(sb, S.red) + bD * acD;
  log_minplus<true>(g, S.c1d, d);
  __syncthreads();
  log_minplus<false>(g, S.c1d, d);
  __syncthreads();
  double sa = 0.0;
  for (int e = tid; e < S.n[0]; e += LWG) {
    const int c = S.src[0][e].cell, i = c >> 16, j = c & 0xFFFF;
    sa += exp(S.lt[0][e]) * fmin(g[i * LG + j], S.cdd[j - i + d - 1] - acD);
  }
  sa = block_sum<LNW>(sa, S.red) + aD * accD;
  return sa + sb;
}

// Upper bound: on entry lk[0] holds log (K v) at the cells of supp(a) and
// lkD0 at the diagonal bin, for the final (u, v).  The log scalings of both
// sides are left scaled by X and Y.
template <class SM>
__device__ double log_upper_bound(SM& S, int d, double ig, double luD, double lvD, double lkD0, double aD,
                                  double bD, bool p2) {
  const int tid = threadIdx.x;
  // X = min(a / r(P), 1) on u
  for (int e = tid; e < S.n[0]; e += LWG)
    S.src[0][e].ls += fmin(S.lt[0][e] - S.src[0][e].ls - S.lk[0][e], 0.0);
  luD += fmin(log(aD) - luD - lkD0, 0.0);
  __syncthreads();
  // Y = min(b / c(P'), 1) on v; e_c = b - c(P'') into lk[1]
  if (p2) apply_lse<true>(S, 1, 0, d, luD, ig);
  else apply_lse<false>(S, 1, 0, d, luD, ig);
  __syncthreads();
  const double l1D = lse_delta(S, 0, d, luD, ig);
  double ec1 = 0.0, eccd = 0.0;
  for (int e = tid; e < S.n[1]; e += LWG) {
    const int c = S.src[1][e].cell, i = c >> 16, j = c & 0xFFFF;
    S.src[1][e].ls += fmin(S.lt[1][e] - S.src[1][e].ls - S.lk[1][e], 0.0);
    const double ec = exp(S.lt[1][e]) - exp(S.src[1][e].ls + S.lk[1][e]);
    S.lk[1][e] = ec;
    ec1 += fabs(ec);
    eccd += ec * S.cdd[j - i + d - 1];
  }
  lvD += fmin(log(bD) - lvD - l1D, 0.0);
  const double ecD = bD - exp(lvD + l1D);
  __syncthreads();
  // e_r = a - r(P'') into lk[0]
  if (p2) apply_lse<true>(S, 0, 1, d, lvD, ig);
  else apply_lse<false>(S, 0, 1, d, lvD, ig);
  __syncthreads();
  const double l0D = lse_delta(S, 1, d, lvD, ig);
  double ercd = 0.0;
  for (int e = tid; e < S.n[0]; e += LWG) {
    const int c = S.src[0][e].cell, i = c >> 16, j = c & 0xFFFF;
    const double er = exp(S.lt[0][e]) - exp(S.src[0][e].ls + S.lk[0][e]);
    S.lk[0][e] = er;
    ercd += er * S.cdd[j - i + d - 1];
  }
  const double erD = aD - exp(luD + l0D);
  __syncthreads();
  // <P'', C> and the rank-one term, both over the two supports and Delta
  double g = 0.0, tr = 0.0;
  for (int e = tid; e < S.n[0]; e += LWG) {
    const int c = S.src[0][e].cell, i = c >> 16, j = c & 0xFFFF;
    const double lu = S.src[0][e].ls, er = S.lk[0][e];
    for (int f = 0; f < S.n[1]; ++f) {
      const int c2 = S.src[1][f].cell, k = c2 >> 16, l = c2 & 0xFFFF;
      const double C = S.c1d[i - k + d - 1] + S.c1d[j - l + d - 1];
      g += exp(lu + S.src[1][f].ls - C * ig) * C;
      tr += er * S.lk[1][f] * C;
    }
    const double cd = S.cdd[j - i + d - 1];
    g += exp(lu + lvD - cd * ig) * cd;
  }
  for (int f = tid; f < S.n[1]; f += LWG) {
    const int c = S.src[1][f].cell, i = c >> 16, j = c & 0xFFFF;
    const double cd = S.cdd[j - i + d - 1];
    g += exp(luD + S.src[1][f].ls - cd * ig) * cd;
  }
  const double gs = block_sum<LNW>(g, S.red);
  const double en = block_sum<LNW>(ec1, S.red) + fabs(ecD);
  const double tt = block_sum<LNW>(tr, S.red) + ecD * block_sum<LNW>(ercd, S.red) + erD * block_sum<LNW>(eccd, S.red);
  return gs + (en > 0.0 ? tt / en : 0.0);
}

// Returns false, writing nothing, when a support does not fit S's lists.
template <class SM>
__device__ bool solve_log_pair(const LogParams& prm, SM& S, long long pair) {
  const int d = prm.d, tid = threadIdx.x;
  const double ig = 1.0 / prm.gamma;
  const bool p2 = prm.p == 2.0;
  const float* A = prm.hist_a + (size_t)prm.ia[pair] * d * d;
  const float* B = prm.hist_b + (size_t)prm.ib[pair] * d * d;
  for (int x = tid; x < 2 * d - 1; x += LWG) {
    const double dl = fabs((double)(x - (d - 1)));
    S.c1d[x] = pow(dl / d, prm.p);
    S.cdd[x] = 2.0 * pow(dl / (2.0 * d), prm.p);
  }
  if (!build_list(S, 0, A, d) || !build_list(S, 1, B, d)) return false;
  double ma = 0.0, mb = 0.0;
  for (int e = tid; e < S.n[0]; e += LWG) ma += exp(S.lt[0][e]);
  for (int e = tid; e < S.n[1]; e += LWG) mb += exp(S.lt[1][e]);
  ma = block_sum<LNW>(ma, S.red);
  mb = block_sum<LNW>(mb, S.red);
  const double aD = mb, bD = ma, m = ma + mb;
  const double ltD0 = log(aD), ltD1 = log(bD);
  // First u-update against v = 1 on the whole grid and on Delta:
  // (K 1)_ij = r_i r_j + k_Delta(i, j), r_i = sum_k exp(-c(i - k) / gamma);
  // (K 1)_Delta = sum over the grid of k_Delta + 1.  log r_i goes to lk[1].
  for (int i = tid; i < d; i += LWG) {
    double mx = -INFINITY;
    for (int k = 0; k < d; ++k) mx = fmax(mx, -S.c1d[i - k + d - 1] * ig);
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += exp(-S.c1d[i - k + d - 1] * ig - mx);
    S.lk[1][i] = mx + log(s);
  }
  __syncthreads();
  for (int e = tid; e < S.n[0]; e += LWG) {
    const int c = S.src[0][e].cell, i = c >> 16, j = c & 0xFFFF;
    S.lk[0][e] = lse2(S.lk[1][i] + S.lk[1][j], -S.cdd[j - i + d - 1] * ig);
  }
  double mxD = 0.0;   // the Delta source (C = 0)
  for (int c = tid; c < d * d; c += LWG) mxD = fmax(mxD, -S.cdd[c % d - c / d + d - 1] * ig);
  mxD = block_max_d(mxD, S.red);
  double sD = 0.0;
  for (int c = tid; c < d * d; c += LWG) sD += exp(-S.cdd[c % d - c / d + d - 1] * ig - mxD);
  sD = block_sum<LNW>(sD, S.red) + exp(-mxD);
  double lkD0 = mxD + log(sD);
  double luD = -INFINITY, lvD = 0.0;
  int t = 0;
  double err = INFINITY;
  for (;;) {
    if (t >= 1) {
      double e1 = 0.0;
      for (int e = tid; e < S.n[0]; e += LWG) e1 += fabs(exp(S.src[0][e].ls + S.lk[0][e]) - exp(S.lt[0][e]));
      e1 = block_sum<LNW>(e1, S.red) + fabs(exp(luD + lkD0) - aD);
      err = e1 / m;
      if (err <= prm.tol || t >= prm.max_iter) break;
    }
    // u-update
    for (int e = tid; e < S.n[0]; e += LWG) S.src[0][e].ls = S.lt[0][e] - S.lk[0][e];
    luD = ltD0 - lkD0;
    __syncthreads();
    // v-update: v = b / K^T u
    if (p2) apply_lse<true>(S, 1, 0, d, luD, ig);
    else apply_lse<false>(S, 1, 0, d, luD, ig);
    __syncthreads();
    const double lkD1 = lse_delta(S, 0, d, luD, ig);
    for (int e = tid; e < S.n[1]; e += LWG) S.src[1][e].ls = S.lt[1][e] - S.lk[1][e];
    lvD = ltD1 - lkD1;
    __syncthreads();
    ++t;
    // K v for the next check and u-update
    if (p2) apply_lse<true>(S, 0, 1, d, lvD, ig);
    else apply_lse<false>(S, 0, 1, d, lvD, ig);
    __syncthreads();
    lkD0 = lse_delta(S, 1, d, lvD, ig);
  }
  // Proposition 3's value <P_t, C> summed over the supports and the Delta blocks.
  double g = 0.0;
  for (int e = tid; e < S.n[0]; e += LWG) {
    const int c = S.src[0][e].cell, i = c >> 16, j = c & 0xFFFF;
    const double lu = S.src[0][e].ls;
    for (int f = 0; f < S.n[1]; ++f) {
      const int c2 = S.src[1][f].cell, k = c2 >> 16, l = c2 & 0xFFFF;
      const double C = S.c1d[i - k + d - 1] + S.c1d[j - l + d - 1];
      g += exp(lu + S.src[1][f].ls - C * ig) * C;
    }
    const double cd = S.cdd[j - i + d - 1];
    g += exp(lu + lvD - cd * ig) * cd;
  }
  for (int f = tid; f < S.n[1]; f += LWG) {
    const int c = S.src[1][f].cell, i = c >> 16, j = c & 0xFFFF;
    const double cd = S.cdd[j - i + d - 1];
    g += exp(luD + S.src[1][f].ls - cd * ig) * cd;
  }
  const double cost = block_sum<LNW>(g, S.red);
  double lo = NAN, up = NAN;
  if (prm.lower && t > 0) {
    double* grid = reinterpret_cast<double*>(prm.scratch + (size_t)blockIdx.x * prm.scratch_stride);
    lo = log_lower_bound(S, grid, d, prm.gamma, luD, aD, bD);
  }
  if (prm.upper && t > 0) up = log_upper_bound(S, d, ig, luD, lvD, lkD0, aD, bD, p2);
  if (tid == 0) {
    int st = ST_LOG;
    if (!(err <= prm.tol)) st |= 1;
    if (!isfinite(cost)) st |= 2;
    prm.cost[pair] = cost;
    prm.iters[2 * pair] = 0;
    prm.iters[2 * pair + 1] = t;
    prm.err[pair] = (float)err;
    prm.status[pair] = st;
    if (prm.upper) prm.upper[pair] = up;
    if (prm.lower) prm.lower[pair] = lo;
  }
  return true;
}

// Pass 1 (GLOBAL = false): every flagged pair whose supports fit the LDS
// lists.  Pass 2 (GLOBAL = true): the flagged pairs pass 1 left (no LOG_PATH
// bit yet), from lists in the workspace slot; a pair beyond those keeps its
// flags.  Two kernels, so that each gets its own register allocation.
template <bool GLOBAL>
__global__ __launch_bounds__(LWG) void sinkhorn_log_kernel(LogParams prm) {
  __shared__ LogSmem S;
  if constexpr (!GLOBAL) {
    for (long long pair = blockIdx.x; pair < prm.n_pairs; pair += gridDim.x) {
      if (!(prm.status[pair] & 6)) continue;   // NONFINITE or RANGE
      solve_log_pair(prm, S, pair);
      __syncthreads();
    }
  } else {
    __shared__ LogGlobal G;   // in LDS, so that the solve's reference to it stays off the stack
    if (threadIdx.x == 0) {
      // the slot's global lists start after the grid of the lower bound
      const size_t grid_bytes = ((size_t)8 * prm.d * (prm.d + 1) + 255) & ~(size_t)255;
      char* slot = prm.scratch + (size_t)blockIdx.x * prm.scratch_stride;
      const long long gcap =
          prm.scratch_stride > grid_bytes ? (long long)((prm.scratch_stride - grid_bytes) / 64) : 0;
      G.cap = (int)min(gcap, (long long)prm.d * prm.d);
      char* base = slot + grid_bytes;
      for (int side = 0; side < 2; ++side) {
        G.src[side] = reinterpret_cast<Src*>(base + (size_t)side * G.cap * 16);
        G.lt[side] = reinterpret_cast<double*>(base + (size_t)2 * G.cap * 16 + (size_t)side * G.cap * 8);
        G.lk[side] = reinterpret_cast<double*>(base + (size_t)2 * G.cap * 24 + (size_t)side * G.cap * 8);
      }
      G.stage = &S.src[0][0];
      G.c1d = S.c1d;
      G.cdd = S.cdd;
      G.red = S.red;
      G.cnt = S.cnt;
      G.n = S.n;
    }
    __syncthreads();
    if (G.cap <= LOG_CAP) return;
    for (long long pair = blockIdx.x; pair < prm.n_pairs; pair += gridDim.x) {
      const int st = prm.status[pair];
      if (!(st & 6) || (st & ST_LOG)) continue;   // unflagged, or solved by pass 1
      solve_log_pair(prm, G, pair);
      __syncthreads();
    }
  }
}

}  // namespace

int launch_log_path(const LogParams& lp, int n_slots, hipStream_t st) {
  hipLaunchKernelGGL(sinkhorn_log_kernel<false>, dim3((unsigned)n_slots), dim3(LWG), 0, st, lp);
  if (hipGetLastError() != hipSuccess) return -1;
  hipLaunchKernelGGL(sinkhorn_log_kernel<true>, dim3((unsigned)n_slots), dim3(LWG), 0, st, lp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pdsink
