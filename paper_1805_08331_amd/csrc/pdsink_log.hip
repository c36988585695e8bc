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
  Src src[2][LOG_CAP];      // side 0: a (u), side 1: b (v)
  double lt[2][LOG_CAP];    // log targets
  double lk[2][LOG_CAP];    // log of the latest K application at each cell
  double c1d[512];          // c(delta) = (|delta| / d)^p, index delta + d - 1
  double cdd[512];          // c_Delta by delta = j - i, index delta + d - 1
  double red[LNW];
  int cnt[LWG];
  int n[2];
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
__device__ bool build_list(LogSmem& S, int side, const float* __restrict__ h, int d) {
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
  if (total > LOG_CAP) return false;
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
template <bool P2>
__device__ __forceinline__ double lse_at(const LogSmem& S, int src, int i, int j, int d, double xD, double ig) {
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

// LSE over the sources of side `src` plus xD of ls - c_Delta / gamma: the
// K application at the diagonal bin (C_Delta,Delta = 0).
__device__ double lse_delta(LogSmem& S, int src, int d, double xD, double ig) {
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

__device__ void solve_log_pair(const LogParams& prm, LogSmem& S, long long pair) {
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
  if (!build_list(S, 0, A, d) || !build_list(S, 1, B, d)) return;   // stays flagged
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
    for (int e = tid; e < S.n[1]; e += LWG) {
      const int c = S.src[1][e].cell, i = c >> 16, j = c & 0xFFFF;
      S.lk[1][e] = p2 ? lse_at<true>(S, 0, i, j, d, luD - S.cdd[j - i + d - 1] * ig, ig)
                      : lse_at<false>(S, 0, i, j, d, luD - S.cdd[j - i + d - 1] * ig, ig);
    }
    const double lkD1 = lse_delta(S, 0, d, luD, ig);
    for (int e = tid; e < S.n[1]; e += LWG) S.src[1][e].ls = S.lt[1][e] - S.lk[1][e];
    lvD = ltD1 - lkD1;
    __syncthreads();
    ++t;
    // K v for the next check and u-update
    for (int e = tid; e < S.n[0]; e += LWG) {
      const int c = S.src[0][e].cell, i = c >> 16, j = c & 0xFFFF;
      S.lk[0][e] = p2 ? lse_at<true>(S, 1, i, j, d, lvD - S.cdd[j - i + d - 1] * ig, ig)
                      : lse_at<false>(S, 1, i, j, d, lvD - S.cdd[j - i + d - 1] * ig, ig);
    }
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
  if (tid == 0) {
    int st = ST_LOG;
    if (!(err <= prm.tol)) st |= 1;
    if (!isfinite(cost)) st |= 2;
    prm.cost[pair] = cost;
    prm.iters[2 * pair] = 0;
    prm.iters[2 * pair + 1] = t;
    prm.err[pair] = (float)err;
    prm.status[pair] = st;
    if (prm.upper) prm.upper[pair] = NAN;
    if (prm.lower) prm.lower[pair] = NAN;
  }
}

__global__ __launch_bounds__(LWG) void sinkhorn_log_kernel(LogParams prm) {
  __shared__ LogSmem S;
  for (long long pair = blockIdx.x; pair < prm.n_pairs; pair += gridDim.x) {
    if (!(prm.status[pair] & 6)) continue;   // NONFINITE or RANGE
    solve_log_pair(prm, S, pair);
    __syncthreads();
  }
}

}  // namespace

int launch_log_path(const LogParams& lp, int n_slots, hipStream_t st) {
  hipLaunchKernelGGL(sinkhorn_log_kernel, dim3((unsigned)n_slots), dim3(LWG), 0, st, lp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pdsink
