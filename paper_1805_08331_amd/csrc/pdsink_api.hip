// C ABI of the pdsink library: contexts, discretisation and the batched
// Sinkhorn entry points (declared in include/pdsink.h).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/pdsink.h"
#include "pdsink_device.h"
#include "sinkhorn_dense.h"
#include "sinkhorn_pair.h"

using namespace pdsink;



struct pdsink_ctx {
  pdsink_params prm;
  int device;
  int D;              // padded grid: 32, 64 or 128
  int* ge;            // device tables, 2*D - 1 entries each
  float* gm;
  int* gde;
  float* gdm;
  float* c1;
  float* cd;
  int* kb;
};

namespace {

int pad_grid(int d) { return d <= 32 ? 32 : (d <= 64 ? 64 : 128); }

struct DeviceGuard {
  int old = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) return;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

// exact split of 2^g into mantissa * 2^e with e = ceil(g), mantissa in (0.5, 1]
void split_pow2(double g, int* e, float* m) {
  double c = std::ceil(g);
  if (c < -(double)(1 << 20)) c = -(double)(1 << 20);
  *e = (int)c;
  *m = (float)std::exp2(g - c);
}

// Table word of a BF16 kernel entry: bf16(m) 2^e (m in (0.5, 1], rounded to
// nearest even) as (e' << 7) | m7 with bf16(m) 2^e = (1 + m7/128) 2^(e' - 1),
// so that adding (s << 7) gives the BF16 bit pattern of the entry times 2^(s - 126)
// whenever that is a normal number.
int bf16_word(int e, float m) {
  uint32_t u;
  std::memcpy(&u, &m, 4);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;   // round to nearest even
  const int field = (int)((u >> 7) & 0xFF);
  const int m7 = (int)(u & 0x7F);
  return ((e + field - 126) << 7) | m7;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int last_error() { return hipGetLastError() == hipSuccess ? PDSINK_OK : PDSINK_EDEVICE; }

__global__ __launch_bounds__(WG) void discretize_kernel(const float* __restrict__ pts, const int64_t* __restrict__ off,
                                                        int d, float* __restrict__ hist, double* __restrict__ mass,
                                                        int* __restrict__ n_bad) {
  extern __shared__ float h[];
  __shared__ double red[NWAVE];
  const int64_t n = blockIdx.x;
  for (int c = threadIdx.x; c < d * d; c += WG) h[c] = 0.0f;
  __syncthreads();
  const int64_t p0 = off[n], p1 = off[n + 1];
  double kept = 0.0;
  int bad = 0;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += WG) {
    const float b = pts[2 * p], t = pts[2 * p + 1];
    const bool ok = isfinite(b) && isfinite(t) && b >= 0.0f && t <= 1.0f && b <= t;
    if (!ok) {
      ++bad;
      continue;
    }
    // floor(x d) of a float32 x times an integer d < 2^24 is exact in double.
    const int i = min((int)floor((double)b * d), d - 1);
    const int j = min((int)floor((double)t * d), d - 1);
    atomicAdd(&h[i * d + j], 1.0f);
    kept += 1.0;
  }
  kept = block_sum(kept, red);
  if (n_bad) {
    bad = wave_sum(bad);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(n_bad, bad);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < d * d; c += WG) hist[n * d * d + c] = h[c];
  if (threadIdx.x == 0) mass[n] = kept;
}

template <int D, int SPT>
int launch_pairs(PairParams pp, int level, hipStream_t st) {
  pp.only_redo = level;
  hipLaunchKernelGGL((sinkhorn_pair_kernel<D, SPT>), dim3((unsigned)pp.n_pairs), dim3(PWGS), 0, st, pp);
  return last_error();
}

template <int D>
int launch_dense(PairParams pp, int level, hipStream_t st) {
  pp.only_redo = level;
  hipLaunchKernelGGL((dense::sinkhorn_pair_kernel<D>), dim3((unsigned)pp.n_pairs), dim3(dense::Cfg<D>::WGS), 0, st,
                     pp);
  return last_error();
}

// Level 0 runs every pair in the compact kernel with one support entry per
// thread (supports up to 512 cells per side); pairs that do not fit flag
// themselves and run again at level 1 with two entries per thread (1024
// cells), then at level 2 in the dense kernel.  All launches go to the same
// stream, with no host synchronisation; a level with no flagged pair exits at
// once.
template <int D>
int launch_levels(PairParams pp, hipStream_t st) {
  int rc = launch_pairs<D, 1>(pp, 0, st);
  if (!rc) rc = launch_pairs<D, 2>(pp, 1, st);
  if (!rc) rc = launch_dense<D>(pp, 2, st);
  return rc;
}

int run_pairs(const pdsink_ctx* ctx, int64_t n_pairs, const float* ha, const float* hb, const int32_t* ia,
              const int32_t* ib, double* cost, int32_t* iters, float* err, int32_t* status, unsigned char* redo,
              hipStream_t st) {
  PairParams pp;
  pp.d = ctx->prm.d;
  pp.tol = ctx->prm.tol;
  pp.max_iter = ctx->prm.max_iter;
  pp.precision = ctx->prm.precision;
  pp.switch_tol = ctx->prm.switch_tol;
  pp.ge = ctx->ge;
  pp.gm = ctx->gm;
  pp.gde = ctx->gde;
  pp.gdm = ctx->gdm;
  pp.c1 = ctx->c1;
  pp.cd = ctx->cd;
  pp.kb = ctx->kb;
  pp.hist_a = ha;
  pp.hist_b = hb;
  pp.ia = ia;
  pp.ib = ib;
  pp.n_pairs = n_pairs;
  pp.cost = cost;
  pp.iters = iters;
  pp.err = err;
  pp.status = status;
  pp.redo = redo;
  switch (ctx->D) {
    case 32: return launch_levels<32>(pp, st);
    case 64: return launch_levels<64>(pp, st);
    default: return launch_levels<128>(pp, st);
  }
}

// pair q = (diagram q / k, centroid q % k)
__global__ void kmeans_pairs_kernel(int64_t n_diag, int k, int32_t* ia, int32_t* ib) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_diag * k) return;
  ia[q] = (int32_t)(q / k);
  ib[q] = (int32_t)(q % k);
}

__global__ void kmeans_argmin_kernel(int64_t n_diag, int k, const double* __restrict__ cost, int32_t* assign,
                                     double* dist, const int32_t* __restrict__ st_in, int32_t* st_out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_diag) return;
  int best = 0;
  double bv = INFINITY;
  for (int c = 0; c < k; ++c) {
    const double v = cost[n * k + c];
    if (dist) dist[n * k + c] = v;
    if (st_out) st_out[n * k + c] = st_in[n * k + c];
    if (v < bv) {     // strict: ties keep the lowest index; NaN never wins
      bv = v;
      best = c;
    }
  }
  assign[n] = best;
}


}  // namespace

extern "C" {

const char* pdsink_strerror(int code) {
  switch (code) {
    case PDSINK_OK: return "ok";
    case PDSINK_EINVAL: return "invalid argument";
    case PDSINK_ENOMEM: return "workspace too small or out of device memory";
    case PDSINK_EDEVICE: return "HIP runtime error";
    case PDSINK_ERANGE: return "result not representable";
    default: return "unknown error";
  }
}

int pdsink_ctx_create(const pdsink_params* params, int device, pdsink_ctx** out) {
  if (!params || !out) return PDSINK_EINVAL;
  *out = nullptr;
  const pdsink_params& p = *params;
  if (p.d < 2 || p.d > 128 || !(p.p >= 1.0) || !(p.gamma > 0.0) || !(p.tol >= 0.0) || p.max_iter < 1 ||
      (p.precision != PDSINK_FP32 && p.precision != PDSINK_BF16_REFINE) || !(p.switch_tol >= 0.0) ||
      !std::isfinite(p.gamma) || !std::isfinite(p.p))
    return PDSINK_EINVAL;
  DeviceGuard g(device);
  if (!g.ok) return PDSINK_EDEVICE;
  const int D = pad_grid(p.d);
  const int n = 2 * D - 1;
  std::vector<int> ge(n), gde(n);
  std::vector<float> gm(n), gdm(n), c1(n), cd(n);
  std::vector<int> kb(n);
  const double l2e = 1.0 / std::log(2.0);
  for (int x = 0; x < n; ++x) {
    const int delta = std::abs(x - (D - 1));
    if (delta < p.d) {
      const double c = std::pow((double)delta / p.d, p.p);            // 1-D step cost (|delta| h)^p
      const double cdl = 2.0 * std::pow((double)delta / (2.0 * p.d), p.p);  // diagonal cost 2 (|delta| h / 2)^p
      split_pow2(-c / p.gamma * l2e, &ge[x], &gm[x]);
      split_pow2(-cdl / p.gamma * l2e, &gde[x], &gdm[x]);
      c1[x] = (float)c;
      cd[x] = (float)cdl;
      kb[x] = bf16_word(ge[x], gm[x]);
    } else {
      ge[x] = gde[x] = NEG;
      gm[x] = gdm[x] = 0.0f;
      c1[x] = cd[x] = 0.0f;
      kb[x] = -(1 << 27);
    }
  }
  pdsink_ctx* ctx = new (std::nothrow) pdsink_ctx;
  if (!ctx) return PDSINK_ENOMEM;
  std::memset(ctx, 0, sizeof(*ctx));
  ctx->prm = p;
  ctx->device = device;
  ctx->D = D;
  char* base = nullptr;
  const size_t bytes = (size_t)n * 4 * 7;
  if (hipMalloc(&base, bytes) != hipSuccess) {
    delete ctx;
    return PDSINK_ENOMEM;
  }
  ctx->ge = (int*)base;
  ctx->gm = (float*)(base + n * 4);
  ctx->gde = (int*)(base + n * 8);
  ctx->gdm = (float*)(base + n * 12);
  ctx->c1 = (float*)(base + n * 16);
  ctx->cd = (float*)(base + n * 20);
  ctx->kb = (int*)(base + n * 24);
  bool ok = hipMemcpy(ctx->ge, ge.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(ctx->gm, gm.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(ctx->gde, gde.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(ctx->gdm, gdm.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(ctx->c1, c1.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(ctx->cd, cd.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(ctx->kb, kb.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    (void)hipFree(base);
    delete ctx;
    return PDSINK_EDEVICE;
  }
  *out = ctx;
  return PDSINK_OK;
}

void pdsink_ctx_destroy(pdsink_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipFree(ctx->ge);
  delete ctx;
}

int pdsink_ctx_params(const pdsink_ctx* ctx, pdsink_params* out) {
  if (!ctx || !out) return PDSINK_EINVAL;
  *out = ctx->prm;
  return PDSINK_OK;
}

int pdsink_workspace_bytes(const pdsink_ctx* ctx, int op, int64_t n_items, size_t* bytes) {
  if (!ctx || !bytes || n_items < 0) return PDSINK_EINVAL;
  switch (op) {
    case PDSINK_OP_DIST: *bytes = align256(n_items); return PDSINK_OK;
    case PDSINK_OP_KMEANS:   // ia, ib, cost, iters, err, status, redo per pair
      *bytes = align256(n_items * 4) * 2 + align256(n_items * 8) + align256(n_items * 8) + align256(n_items * 4) * 2 +
               align256(n_items);
      return PDSINK_OK;
    case PDSINK_OP_BARYCENTER: *bytes = 256; return PDSINK_OK;
    default: return PDSINK_EINVAL;
  }
}

int pd_discretize(pdsink_ctx* ctx, const float* pts, const int64_t* offsets, int64_t n_diag, float* hist,
                  double* mass, int32_t* n_bad, void* stream) {
  if (!ctx || n_diag < 0) return PDSINK_EINVAL;
  if (n_diag == 0) return PDSINK_OK;
  if (!offsets || !hist || !mass || n_diag > INT_MAX) return PDSINK_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  const int d = ctx->prm.d;
  hipLaunchKernelGGL(discretize_kernel, dim3((unsigned)n_diag), dim3(WG), (size_t)d * d * sizeof(float),
                     (hipStream_t)stream, pts, offsets, d, hist, mass, n_bad);
  return last_error();
}

int sinkhorn_dist_batch(pdsink_ctx* ctx, int64_t n_pairs, const float* hist_a, const float* hist_b,
                        const int32_t* ia, const int32_t* ib, double* cost, int32_t* iters, float* err,
                        int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || n_pairs < 0) return PDSINK_EINVAL;
  if (n_pairs == 0) return PDSINK_OK;
  if (n_pairs > INT_MAX || !hist_a || !hist_b || !ia || !ib || !cost || !iters || !err || !status)
    return PDSINK_EINVAL;
  size_t need = 0;
  pdsink_workspace_bytes(ctx, PDSINK_OP_DIST, n_pairs, &need);
  if (!ws || ws_bytes < need) return PDSINK_ENOMEM;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  return run_pairs(ctx, n_pairs, hist_a, hist_b, ia, ib, cost, iters, err, status, (unsigned char*)ws,
                   (hipStream_t)stream);
}

int kmeans_assign(pdsink_ctx* ctx, int64_t n_diag, const float* hist, int32_t k, const float* centroids,
                  int32_t* assign, double* dist, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || n_diag < 0 || k < 1) return PDSINK_EINVAL;
  if (n_diag == 0) return PDSINK_OK;
  if (!hist || !centroids || !assign) return PDSINK_EINVAL;
  const int64_t np = n_diag * (int64_t)k;
  if (np > INT_MAX) return PDSINK_EINVAL;
  size_t need = 0;
  pdsink_workspace_bytes(ctx, PDSINK_OP_KMEANS, np, &need);
  if (!ws || ws_bytes < need) return PDSINK_ENOMEM;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  char* w = (char*)ws;
  int32_t* ia = (int32_t*)w;
  w += align256(np * 4);
  int32_t* ib = (int32_t*)w;
  w += align256(np * 4);
  double* cost = (double*)w;
  w += align256(np * 8);
  int32_t* iters = (int32_t*)w;
  w += align256(np * 8);
  float* err = (float*)w;
  w += align256(np * 4);
  int32_t* st = (int32_t*)w;
  w += align256(np * 4);
  unsigned char* redo = (unsigned char*)w;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(kmeans_pairs_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, n_diag, k, ia, ib);
  int rc = last_error();
  if (rc) return rc;
  rc = run_pairs(ctx, np, hist, centroids, ia, ib, cost, iters, err, st, redo, s);
  if (rc) return rc;
  hipLaunchKernelGGL(kmeans_argmin_kernel, dim3((unsigned)((n_diag + 255) / 256)), dim3(256), 0, s, n_diag, k, cost,
                     assign, dist, st, status);
  return last_error();
}

int pd_barycenter(pdsink_ctx* ctx, int64_t n_diag, const float* hist, double lambda, int32_t max_outer,
                  double energy_rtol, int32_t init_uniform, float* z, double* energy, int32_t* outer, void* ws,
                  size_t ws_bytes, void* stream) {
  (void)ctx; (void)n_diag; (void)hist; (void)lambda; (void)max_outer; (void)energy_rtol; (void)init_uniform;
  (void)z; (void)energy; (void)outer; (void)ws; (void)ws_bytes; (void)stream;
  return PDSINK_EINVAL;   // implemented in the barycenter source
}

}  // extern "C"
