// C ABI of the pdsink library: contexts, discretisation and the batched
// Sinkhorn entry points (declared in include/pdsink.h).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstddef>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/pdsink.h"
#include "pdsink_device.h"
#include "sinkhorn_log.h"
#include "sinkhorn_pair.h"
#include "sinkhorn_fast.h"

using namespace pdsink;

// Scratch of sinkhorn_dist_batch_noalloc: routing flags, launch order and the
// per-slot support lists, in one array that each GPU holds from the loading of
// this code object until the process ends.  In host code this name is not a
// device address: host code uses the per-device address that
// hipGetSymbolAddress returned (scratch_lookup), never the name itself.
static __device__ __align__(256) unsigned char scratch[PDSINK_NOALLOC_SCRATCH_BYTES];

namespace pdsink {
// The bounds variant of the pair kernel (pdsink_bounds.hip).
int launch_pair_bounds(int D, PairParams pp, int n_slots, hipStream_t st);
}  // namespace pdsink



struct pdsink_ctx {
  pdsink_params prm;
  int device;
  int D;              // padded grid: 32, 64, 128 or 256
  int* ge;            // device tables, 2*D - 1 entries each
  float* gm;
  int* gde;
  float* gdm;
  float* c1;
  float* cd;
  int* kb;
  // the same seven tables in the 128-padded layout the resident kernel reads
  // (the tables above when D = 128; their own allocation at grids 33 to 64,
  // whose general kernel keeps the 64-padded layout; NULL where the context
  // never runs the resident kernel)
  int* rge;
  float* rgm;
  int* rgde;
  float* rgdm;
  float* rc1;
  float* rcd;
  int* rkb;
  char* rbase;        // the resident tables' own allocation, or NULL
  int n_cu;           // compute units of the device: workgroups of the global-list variant
  void* scratch;      // device address of `scratch` on this device, NULL if the lookup failed
};

namespace {

constexpr int MAX_DEVICES = 256;
std::mutex scratch_mu;
void* scratch_addr[MAX_DEVICES];

// Device address of `scratch` on `device`, which must be the current device;
// looked up once per device and kept.
int scratch_lookup(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return PDSINK_EINVAL;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();   // leave no sticky error for the next launch check
      return PDSINK_EDEVICE;
    }
    scratch_addr[device] = p;
  }
  *out = scratch_addr[device];
  return PDSINK_OK;
}

int pad_grid(int d) { return d <= 32 ? 32 : (d <= 64 ? 64 : (d <= 128 ? 128 : 256)); }

// Grids the resident-kernel variant takes (K depth 16 ceil(d / 16), 3 to 7
// MFMA steps), and whether a context runs it: on request, or by default where
// it measured faster than the general kernel (1024 pairs of 50-500 points,
// gamma 1e-3, tol 1e-3): with BF16 contractions at every grid it takes (1.6x
// to 2x at d = 40 to 100), with FP32 contractions from d = 65 (at d = 40 to
// 64 the general kernel's 64-padded layout was as fast or faster: 21 against
// 26 ms per batch at d = 50).
constexpr int RESIDENT_DMIN = 33;
bool resident_grid(int d) { return d >= RESIDENT_DMIN && d <= FAST_DMAX; }
bool resident_for(int d, int kernel, int precision) {
  if (!resident_grid(d)) return false;
  if (kernel == PDSINK_KERNEL_RESIDENT) return true;
  return kernel == PDSINK_KERNEL_AUTO && (precision == PDSINK_BF16_REFINE || d >= RESIDENT_AUTO_DMIN);
}

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

// One workgroup per diagram.  The counts go to an LDS histogram (GLOBAL_H:
// straight to the output, zeroed first, for grids whose histogram exceeds
// 64 KB); float atomic adds of whole counts below 2^24 are exact, so the
// result does not depend on their order.
template <bool GLOBAL_H>
__global__ __launch_bounds__(WG) void discretize_kernel(const float* __restrict__ pts, const int64_t* __restrict__ off,
                                                        int d, float* __restrict__ hist, double* __restrict__ mass,
                                                        int* __restrict__ n_bad) {
  extern __shared__ float hs[];
  __shared__ double red[NWAVE];
  const int64_t n = blockIdx.x;
  float* h = GLOBAL_H ? hist + n * d * d : hs;
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
  if (!GLOBAL_H) {
    __syncthreads();
    for (int c = threadIdx.x; c < d * d; c += WG) hist[n * d * d + c] = h[c];
  }
  if (threadIdx.x == 0) mass[n] = kept;
}

// Launch order of the pairs.  The batch runs one workgroup per pair (one per
// compute unit at a time), so its length is set by the solves that start
// last; the iteration count of a pair is largest when one of its diagrams is
// small (much of its mass goes to the diagonal), so pairs are launched by
// increasing min(|supp a|, |supp b|), counted on the device and bucketed
// (ORDER_BINS buckets; the order within a bucket is arbitrary and does not
// affect any result).
constexpr int ORDER_BINS = 1024;
size_t order_bytes(int64_t n) { return align256((size_t)n * 4) * 2 + align256((size_t)ORDER_BINS * 4); }

__global__ void order_zero_kernel(int* bins) {
  for (int b = threadIdx.x; b < ORDER_BINS; b += blockDim.x) bins[b] = 0;
}

__global__ __launch_bounds__(WG) void order_key_kernel(const float* __restrict__ ha, const float* __restrict__ hb,
                                                       const int32_t* ia, const int32_t* ib, int d, int shift,
                                                       int* key, int* bins) {
  __shared__ int ra[NWAVE], rb[NWAVE];
  const long long q = blockIdx.x;
  const float* A = ha + (size_t)ia[q] * d * d;
  const float* B = hb + (size_t)ib[q] * d * d;
  int ca = 0, cb = 0;
  for (int c = threadIdx.x; c < d * d; c += WG) {
    ca += A[c] > 0.0f;
    cb += B[c] > 0.0f;
  }
  ca = wave_sum(ca);
  cb = wave_sum(cb);
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = ca;
    rb[threadIdx.x >> 6] = cb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int ta = 0, tb = 0;
    for (int w = 0; w < NWAVE; ++w) {
      ta += ra[w];
      tb += rb[w];
    }
    const int k = min(min(ta, tb) >> shift, ORDER_BINS - 1);
    key[q] = k;
    atomicAdd(&bins[k], 1);
  }
}

// Exclusive scan of the bucket counts (one workgroup of ORDER_BINS threads).
__global__ __launch_bounds__(ORDER_BINS) void order_scan_kernel(int* bins) {
  __shared__ int t[ORDER_BINS];
  const int b = threadIdx.x;
  const int v = bins[b];
  t[b] = v;
  __syncthreads();
  for (int off = 1; off < ORDER_BINS; off <<= 1) {
    const int add = b >= off ? t[b - off] : 0;
    __syncthreads();
    t[b] += add;
    __syncthreads();
  }
  bins[b] = t[b] - v;
}

__global__ __launch_bounds__(WG) void order_scatter_kernel(const int* key, int* bins, int* perm, long long n) {
  const long long q = (long long)blockIdx.x * WG + threadIdx.x;
  if (q < n) perm[atomicAdd(&bins[key[q]], 1)] = (int)q;
}

// Optional per-pair buffers of a distance launch.
struct PairExtras {
  char* lists = nullptr;      // global support lists, list_bytes(D) per workgroup slot
  char* ops = nullptr;        // operand slices (D = 256), GlobalOps<256>::BYTES per slot
  int n_slots = 0;            // workgroup slots (grid of the global-list variant)
  char* state = nullptr;      // WarmState per pair
  int state_in = 0;
  const int* stop = nullptr;  // device flag: the solve launches do nothing when set
  double* gout = nullptr;     // [n_pairs][d * d] gradient terms
  double* upper = nullptr;    // [n_pairs] error-control bounds
  double* lower = nullptr;
  char* order = nullptr;      // order_bytes(n_pairs): keys, permutation, buckets
  DoneRec* done = nullptr;    // per-pair completion records, posted with done_tag
  unsigned done_tag = 0;
};

static_assert(sizeof(pdsink_done) == sizeof(DoneRec) && offsetof(pdsink_done, tag) == offsetof(DoneRec, tag) &&
                  offsetof(pdsink_done, iters) == offsetof(DoneRec, it),
              "pdsink_done and DoneRec share one layout");

size_t list_bytes(int D) { return align256((size_t)52 * D * D); }   // 2 sides x 5 arrays + 3 suspect arrays, x D^2 x 4 bytes
size_t warm_bytes(int D) {
  switch (D) {
    case 32: return sizeof(WarmState<32>);
    case 64: return sizeof(WarmState<64>);
    case 128: return sizeof(WarmState<128>);
    default: return sizeof(WarmState<256>);
  }
}
size_t ops_bytes(int D) { return D > 128 ? GlobalOps<256>::BYTES : 0; }
// Per workgroup slot of a launch: support lists, plus operand buffers beyond D = 128.
size_t slot_bytes(int D) { return list_bytes(D) + ops_bytes(D); }
int64_t slots_for(const pdsink_ctx* ctx, int64_t n_pairs) { return n_pairs < ctx->n_cu ? n_pairs : ctx->n_cu; }

// Level 0 runs every pair with one support entry per thread and register
// lists (supports up to 512 cells per side); pairs that do not fit flag
// themselves and run at level 1 with their lists in the workspace, one
// workgroup per compute unit striding over the batch.  Both launches go to
// the same stream, with no host synchronisation; when no pair is flagged the
// second launch only reads the flags.
//
// `rp`, when given, is pp with the resident kernel's tables (the 128-padded
// layout): grids up to 100 without warm start or gradient output then run
// level 0 in the resident-kernel variant, and the pairs it does not take
// (supports beyond 512 cells or below the diagonal, suspect-list overflow)
// go to the global-list launch of the general kernel at its own padding D.
template <int D>
int launch_levels(PairParams pp, const PairParams* rp, int n_slots, hipStream_t st) {
  if (pp.upper || pp.lower) return launch_pair_bounds(D, pp, n_slots, st) ? PDSINK_EDEVICE : PDSINK_OK;
  pp.only_redo = 0;
  if constexpr (D <= 128) {
    if (rp && !pp.state && !pp.gout) {
      PairParams r = *rp;
      r.only_redo = 0;
      const unsigned g = (unsigned)r.n_pairs;
      switch ((r.d + 15) / 16) {
        case 3: hipLaunchKernelGGL(sinkhorn_fast_kernel<3>, dim3(g), dim3(PWGS), 0, st, r); break;
        case 4: hipLaunchKernelGGL(sinkhorn_fast_kernel<4>, dim3(g), dim3(PWGS), 0, st, r); break;
        case 5: hipLaunchKernelGGL(sinkhorn_fast_kernel<5>, dim3(g), dim3(PWGS), 0, st, r); break;
        case 6: hipLaunchKernelGGL(sinkhorn_fast_kernel<6>, dim3(g), dim3(PWGS), 0, st, r); break;
        default: hipLaunchKernelGGL(sinkhorn_fast_kernel<7>, dim3(g), dim3(PWGS), 0, st, r); break;
      }
      int rc = last_error();
      if (rc) return rc;
      pp.only_redo = 1;
      hipLaunchKernelGGL((sinkhorn_pair_kernel<D, 0>), dim3((unsigned)n_slots), dim3(PWGS), 0, st, pp);
      return last_error();
    }
  }
  // beyond D = 128 every launch strides over the batch with one operand slice per slot
  const unsigned g0 = D > 128 ? (unsigned)n_slots : (unsigned)pp.n_pairs;
  hipLaunchKernelGGL((sinkhorn_pair_kernel<D, 1>), dim3(g0), dim3(PWGS), 0, st, pp);
  int rc = last_error();
  if (rc) return rc;
  pp.only_redo = 1;
  hipLaunchKernelGGL((sinkhorn_pair_kernel<D, 0>), dim3((unsigned)n_slots), dim3(PWGS), 0, st, pp);
  return last_error();
}

int launch_log(const pdsink_ctx* ctx, int64_t n_pairs, const float* ha, const float* hb, const int32_t* ia,
               const int32_t* ib, double* cost, int32_t* iters, float* err, int32_t* status, const PairExtras& ex,
               hipStream_t st);

// Completion records of the pairs whose status carries NONFINITE, RANGE or
// LOG_PATH: the solve launches post every other pair themselves.
__global__ void done_sweep_kernel(long long n, const double* __restrict__ cost, const int32_t* __restrict__ iters,
                                  const float* __restrict__ err, const int32_t* __restrict__ status, DoneRec* done,
                                  unsigned tag) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int st = status[q];
  if (st & (PDSINK_ST_NONFINITE | PDSINK_ST_RANGE | PDSINK_ST_LOG_PATH))
    post_done(done, tag, q, cost[q], iters[2 * q], iters[2 * q + 1], err[q], st);
}

int run_pairs(const pdsink_ctx* ctx, int64_t n_pairs, const float* ha, const float* hb, const int32_t* ia,
              const int32_t* ib, double* cost, int32_t* iters, float* err, int32_t* status, unsigned char* redo,
              const PairExtras& ex, hipStream_t st) {
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
  pp.lists = ex.lists;
  pp.list_stride = list_bytes(ctx->D);
  pp.ops = ex.ops;
  pp.state = ex.state;
  pp.state_in = ex.state_in;
  pp.gout = ex.gout;
  pp.stop = ex.stop;
  pp.done = ex.done;
  pp.done_tag = ex.done_tag;
  pp.upper = ex.upper;
  pp.lower = ex.lower;
  pp.gamma = ctx->prm.gamma;
  pp.p = ctx->prm.p;
  pp.perm = nullptr;
  if (ex.order && n_pairs > ctx->n_cu) {
    int* key = reinterpret_cast<int*>(ex.order);
    int* perm = reinterpret_cast<int*>(ex.order + align256((size_t)n_pairs * 4));
    int* bins = reinterpret_cast<int*>(ex.order + 2 * align256((size_t)n_pairs * 4));
    const int d = ctx->prm.d;
    int shift = 0;
    while (((d * d) >> shift) >= ORDER_BINS) ++shift;
    hipLaunchKernelGGL(order_zero_kernel, dim3(1), dim3(WG), 0, st, bins);
    hipLaunchKernelGGL(order_key_kernel, dim3((unsigned)n_pairs), dim3(WG), 0, st, ha, hb, ia, ib, d, shift, key, bins);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(ORDER_BINS), 0, st, bins);
    hipLaunchKernelGGL(order_scatter_kernel, dim3((unsigned)((n_pairs + WG - 1) / WG)), dim3(WG), 0, st, key, bins, perm,
                       (long long)n_pairs);
    const int rc = last_error();
    if (rc) return rc;
    pp.perm = perm;
  }
  int rc;
  PairParams rpp = pp;
  const PairParams* rp = nullptr;
  if (ctx->rge && resident_for(ctx->prm.d, ctx->prm.kernel, ctx->prm.precision)) {
    rpp.ge = ctx->rge;
    rpp.gm = ctx->rgm;
    rpp.gde = ctx->rgde;
    rpp.gdm = ctx->rgdm;
    rpp.c1 = ctx->rc1;
    rpp.cd = ctx->rcd;
    rpp.kb = ctx->rkb;
    rp = &rpp;
  }
  switch (ctx->D) {
    case 32: rc = launch_levels<32>(pp, rp, ex.n_slots, st); break;
    case 64: rc = launch_levels<64>(pp, rp, ex.n_slots, st); break;
    case 128: rc = launch_levels<128>(pp, rp, ex.n_slots, st); break;
    default: rc = launch_levels<256>(pp, rp, ex.n_slots, st); break;
  }
  if (rc) return rc;
  if (!ex.state && !ex.gout) {
    rc = launch_log(ctx, n_pairs, ha, hb, ia, ib, cost, iters, err, status, ex, st);
    if (rc) return rc;
  }
  if (!ex.done) return PDSINK_OK;
  // Completion records of the pairs the solve launches did not post (flagged
  // NONFINITE or RANGE there): their results are final once the log-domain
  // launches are done.
  hipLaunchKernelGGL(done_sweep_kernel, dim3((unsigned)((n_pairs + WG - 1) / WG)), dim3(WG), 0, st,
                     (long long)n_pairs, cost, iters, err, status, ex.done, ex.done_tag);
  return last_error();
}

int launch_log(const pdsink_ctx* ctx, int64_t n_pairs, const float* ha, const float* hb, const int32_t* ia,
               const int32_t* ib, double* cost, int32_t* iters, float* err, int32_t* status, const PairExtras& ex,
               hipStream_t st) {
  // Pairs flagged NONFINITE or RANGE are solved again in the log domain (same
  // stream, no host synchronisation; a launch that only reads the flags when
  // none is).  Not for the barycenter solves, which need the scaled form of v.
  LogParams lp;
  lp.d = ctx->prm.d;
  lp.p = ctx->prm.p;
  lp.gamma = ctx->prm.gamma;
  lp.tol = ctx->prm.tol;
  lp.max_iter = ctx->prm.max_iter;
  lp.hist_a = ha;
  lp.hist_b = hb;
  lp.ia = ia;
  lp.ib = ib;
  lp.n_pairs = n_pairs;
  lp.cost = cost;
  lp.iters = iters;
  lp.err = err;
  lp.status = status;
  lp.upper = ex.upper;
  lp.lower = ex.lower;
  lp.scratch = ex.lists;   // the slots' list areas, free once the solve launches are done
  lp.scratch_stride = slot_bytes(ctx->D);
  return launch_log_path(lp, ex.n_slots, st) ? PDSINK_EDEVICE : PDSINK_OK;
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

// Barycenter pairs: q = (z, hist[q]).
__global__ void bary_pairs_kernel(int64_t n, int32_t* ia, int32_t* ib) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) {
    ia[q] = 0;
    ib[q] = (int32_t)q;
  }
}

// Mass of each histogram (FP64, fixed order within the workgroup).
__global__ __launch_bounds__(WG) void hist_mass_kernel(const float* __restrict__ hist, int d, double* mass) {
  __shared__ double red[NWAVE];
  const int64_t n = blockIdx.x;
  double m = 0.0;
  for (int c = threadIdx.x; c < d * d; c += WG) m += hist[n * d * d + c];
  m = block_sum(m, red);
  if (threadIdx.x == 0) mass[n] = m;
}

// Uniform measure on the cells j >= i with the mean of the N masses.
__global__ void bary_uniform_kernel(const double* mass, int64_t n, int d, float* z) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d * d) return;
  double m = 0.0;
  for (int64_t q = 0; q < n; ++q) m += mass[q];
  m /= (double)n;
  const int i = c / d, j = c % d;
  z[c] = j >= i ? (float)(m / (0.5 * d * (d + 1))) : 0.0f;
}

// Device state of the barycenter's outer loop: the host enqueues every outer
// step, and the stopping test of Algorithm 2 runs on the device.
struct BaryCtl {
  int stop;       // set once the loop has ended: later launches do nothing
  int err;        // an inner solve left the scaled range (PDSINK_ERANGE)
  int outer;      // outer steps taken
  int pad;
  double energy;  // E_t of the last step taken
  double prev;    // E_{t-1}
};

__global__ void bary_ctl_init_kernel(BaryCtl* ctl) {
  if (threadIdx.x == 0) {
    ctl->stop = 0;
    ctl->err = 0;
    ctl->outer = 0;
    ctl->pad = 0;
    ctl->energy = 0.0;
    ctl->prev = 0.0;
  }
}

// Energy of outer step t (Algorithm 2: the mean of the pairs' Sinkhorn costs,
// summed in a fixed order) and the stopping test: relative change below
// rtol, or the last step.  A solve that left the scaled range (NONFINITE or
// RANGE) stops the loop with the error flag: z keeps the last good iterate.
__global__ __launch_bounds__(WG) void bary_energy_kernel(const double* __restrict__ cost,
                                                         const int32_t* __restrict__ st, int64_t n, int t,
                                                         int max_outer, double rtol, BaryCtl* ctl) {
  __shared__ double red[NWAVE];
  __shared__ int redi[NWAVE];
  if (ctl->stop) return;
  double sum = 0.0;
  int bad = 0;
  for (int64_t q = threadIdx.x; q < n; q += WG) {
    sum += cost[q];
    bad |= (st[q] & (PDSINK_ST_NONFINITE | PDSINK_ST_RANGE)) != 0;
  }
  sum = block_sum(sum, red);
  bad = block_max(bad, redi);
  if (threadIdx.x != 0) return;
  if (bad) {
    ctl->err = 1;
    ctl->stop = 1;
    return;
  }
  const double E = sum / (double)n;
  ctl->energy = E;
  ctl->outer = t + 1;
  if ((t > 0 && fabs(E / ctl->prev - 1.0) < rtol) || t == max_outer - 1) ctl->stop = 1;
  else ctl->prev = E;
}

// Multiplicative step of Algorithm 2 on the support of z, gradient summed
// over the diagrams in a fixed order (nothing once the loop has stopped).
__global__ void bary_step_kernel(const double* __restrict__ gout, int64_t n, int d, double scale, float* z,
                                 const BaryCtl* __restrict__ ctl) {
  if (ctl->stop) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d * d) return;
  const float zc = z[c];
  if (!(zc > 0.0f)) return;
  double gsum = 0.0;
  for (int64_t q = 0; q < n; ++q) gsum += gout[q * d * d + c];
  z[c] = (float)((double)zc * exp(-scale * gsum));
}

// out[m] = hist[idx[m]] (d * d floats each).
__global__ void gather_hist_kernel(const float* __restrict__ hist, const int32_t* __restrict__ idx, int dd,
                                   float* __restrict__ out) {
  const int64_t m = blockIdx.y;
  const float* src = hist + (int64_t)idx[m] * dd;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < dd; c += gridDim.x * blockDim.x) out[m * dd + c] = src[c];
}

// Algorithm 1's initial v for sinkhorn_dist_batch: the natural log of v on the
// d x d grid cells and on the diagonal bin, [n_pairs][d * d + 1], to the scaled
// form the pair kernel starts from (WarmState).  Only the cells of supp(b)
// (hist_b[ib[q]] > 0) are kept: v_ij = vres * 2^(Pv_i + Qv_j) with the row and
// column log2 scales at the midranges of the integer parts of log2 v, so that
// the residuals span at most +-mres octaves; every other cell gets vres = 0.
// The diagonal bin: v_Delta = vmx 2^vex with vmx in [0.5, 1) (0 for -inf).
template <int D>
__global__ __launch_bounds__(WG) void warm_pack_kernel(const double* __restrict__ state,
                                                       const float* __restrict__ hist_b,
                                                       const int32_t* __restrict__ ib, int d,
                                                       WarmState<D>* __restrict__ wsa) {
  __shared__ int lo[D], hi[D], P[D], Q[D];
  __shared__ int red[NWAVE];
  const int tid = threadIdx.x;
  const int64_t q = blockIdx.x;
  const int dd = d * d;
  const double* lv = state + q * (int64_t)(dd + 1);
  const float* hb = hist_b + (int64_t)ib[q] * dd;
  WarmState<D>& w = wsa[q];
  constexpr double LOG2E = 1.4426950408889634074;
  constexpr double LIM = (double)(1 << 22);   // |log2 v| beyond this: out of range anyway
  auto expo = [&](int c, double& l2) -> bool {   // log2 v at a cell of supp(b), if finite
    const double x = lv[c];
    if (!(hb[c] > 0.0f) || !(x > -INFINITY) || !(x < INFINITY)) return false;
    l2 = fmin(fmax(x * LOG2E, -LIM), LIM);
    return true;
  };
  for (int i = tid; i < D; i += WG) {
    lo[i] = INT_MAX;
    hi[i] = INT_MIN;
  }
  __syncthreads();
  for (int c = tid; c < dd; c += WG) {
    double l2;
    if (expo(c, l2)) {
      const int e = (int)floor(l2);
      atomicMin(&lo[c / d], e);
      atomicMax(&hi[c / d], e);
    }
  }
  __syncthreads();
  for (int i = tid; i < D; i += WG) {
    P[i] = hi[i] >= lo[i] ? (lo[i] + hi[i]) >> 1 : NEG;
    lo[i] = INT_MAX;
    hi[i] = INT_MIN;
  }
  __syncthreads();
  for (int c = tid; c < dd; c += WG) {
    double l2;
    if (expo(c, l2)) {
      const int e = (int)floor(l2) - P[c / d];
      atomicMin(&lo[c % d], e);
      atomicMax(&hi[c % d], e);
    }
  }
  __syncthreads();
  for (int j = tid; j < D; j += WG) Q[j] = hi[j] >= lo[j] ? (lo[j] + hi[j]) >> 1 : NEG;
  __syncthreads();
  int span = 0;
  for (int c = tid; c < dd; c += WG) {
    const int i = c / d, j = c % d;
    double l2;
    float r = 0.0f;
    if (expo(c, l2)) {
      const double t = l2 - (double)P[i] - (double)Q[j];
      span = max(span, (int)fabs(floor(t)));
      r = (float)exp2(t);
    }
    w.vres[i * D + j] = r;
  }
  span = wave_max(span);
  if ((tid & 63) == 0) red[tid >> 6] = span;
  for (int i = tid; i < D; i += WG) {
    w.Pv[i] = P[i];
    w.Qv[i] = Q[i];
  }
  __syncthreads();
  if (tid == 0) {
    int m = 0;
    for (int k = 0; k < NWAVE; ++k) m = max(m, red[k]);
    w.mres = m + 1;
    const double x = lv[dd];
    if (x > -INFINITY && x < INFINITY) {
      const double l2 = fmin(fmax(x * LOG2E, -LIM), LIM);
      const double e = floor(l2) + 1.0;
      w.vex = (int)e;
      w.vmx = exp2(l2 - e);
    } else {
      w.vex = 0;
      w.vmx = 0.0;
    }
  }
}

// The final v of each pair (WarmState, written by the solve) back to the
// natural log of v on the grid cells and the diagonal bin; -inf where v = 0
// (every cell off supp(b)).
template <int D>
__global__ __launch_bounds__(WG) void warm_unpack_kernel(const WarmState<D>* __restrict__ wsa, int d,
                                                         double* __restrict__ state) {
  constexpr double LN2 = 0.69314718055994530942;
  const int64_t q = blockIdx.x;
  const int dd = d * d;
  const WarmState<D>& w = wsa[q];
  double* lv = state + q * (int64_t)(dd + 1);
  for (int c = threadIdx.x; c < dd; c += WG) {
    const int i = c / d, j = c % d;
    const float r = w.vres[i * D + j];
    lv[c] = (r > 0.0f && w.Pv[i] != NEG && w.Qv[j] != NEG)
                ? (log2((double)r) + (double)w.Pv[i] + (double)w.Qv[j]) * LN2
                : -INFINITY;
  }
  if (threadIdx.x == 0) lv[dd] = w.vmx > 0.0 ? (log2(w.vmx) + (double)w.vex) * LN2 : -INFINITY;
}

template <int D>
int launch_warm(bool pack, const double* state_in, double* state_out, const float* hist_b, const int32_t* ib,
                int d, int64_t n, char* ws, hipStream_t st) {
  WarmState<D>* w = reinterpret_cast<WarmState<D>*>(ws);
  if (pack)
    hipLaunchKernelGGL(warm_pack_kernel<D>, dim3((unsigned)n), dim3(WG), 0, st, state_in, hist_b, ib, d, w);
  else
    hipLaunchKernelGGL(warm_unpack_kernel<D>, dim3((unsigned)n), dim3(WG), 0, st, w, d, state_out);
  return last_error();
}

int warm_convert(int D, bool pack, double* state, const float* hist_b, const int32_t* ib, int d, int64_t n,
                 char* ws, hipStream_t st) {
  switch (D) {
    case 32: return launch_warm<32>(pack, state, state, hist_b, ib, d, n, ws, st);
    case 64: return launch_warm<64>(pack, state, state, hist_b, ib, d, n, ws, st);
    case 128: return launch_warm<128>(pack, state, state, hist_b, ib, d, n, ws, st);
    default: return launch_warm<256>(pack, state, state, hist_b, ib, d, n, ws, st);
  }
}

// Entropic sharpening of histograms (pd_sharpen): histogram blockIdx.x of z,
// one workgroup.  With l_c = log(z_c / max z) <= 0 on the positive cells, the
// normalised power p^beta has entropy H(beta) = log Z - beta A / Z, where
// Z = sum exp(beta l_c) and A = sum exp(beta l_c) l_c; H falls with beta from
// the entropy of z at beta = 1 towards log n_max.  All in FP64 with
// fixed-order reductions, so every thread takes the same branches; beta is
// bracketed by doubling and found by bisection down to adjacent doubles.
__global__ __launch_bounds__(WG) void sharpen_kernel(float* __restrict__ z, int dd, double h0,
                                                     double* __restrict__ beta_out) {
  __shared__ double red[NWAVE];
  __shared__ int redi[NWAVE];
  float* zn = z + (int64_t)blockIdx.x * dd;
  const int tid = threadIdx.x;
  double m = 0.0;
  int zbits = 0;
  for (int c = tid; c < dd; c += WG) {
    const float v = zn[c];
    if (v > 0.0f) {
      m += (double)v;
      zbits = max(zbits, __float_as_int(v));   // positive floats order as their bits
    }
  }
  const double M = block_sum(m, red);
  const float zmax = __int_as_float(block_max(zbits, redi));
  if (!(M > 0.0)) {
    if (tid == 0 && beta_out) beta_out[blockIdx.x] = 1.0;
    return;
  }
  double cnt = 0.0;
  for (int c = tid; c < dd; c += WG) cnt += zn[c] == zmax ? 1.0 : 0.0;
  const double n_max = block_sum(cnt, red);
  const double lmax = log((double)zmax);
  auto sums = [&](double beta, double& Z, double& A) {
    double zs = 0.0, as = 0.0;
    for (int c = tid; c < dd; c += WG) {
      const float v = zn[c];
      if (v > 0.0f) {
        const double l = log((double)v) - lmax;
        const double w = exp(beta * l);
        zs += w;
        as += w * l;
      }
    }
    Z = block_sum(zs, red);
    A = block_sum(as, red);
  };
  auto entropy_at = [&](double beta) {
    double Z, A;
    sums(beta, Z, A);
    return log(Z) - beta * A / Z;
  };
  double beta = 1.0;
  if (entropy_at(1.0) <= h0) {
    if (tid == 0 && beta_out) beta_out[blockIdx.x] = 1.0;
    return;
  }
  if (h0 <= log(n_max)) {   // the limit: the mass evenly over the maximal cells
    const float share = (float)(M / n_max);
    for (int c = tid; c < dd; c += WG) zn[c] = zn[c] == zmax ? share : 0.0f;
    if (tid == 0 && beta_out) beta_out[blockIdx.x] = INFINITY;
    return;
  }
  double lo = 1.0, hi = 2.0;
  while (entropy_at(hi) > h0 && hi < 0x1p60) {
    lo = hi;
    hi *= 2.0;
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (entropy_at(mid) > h0) lo = mid;
    else hi = mid;
  }
  beta = 0.5 * (lo + hi);
  double Z, A;
  sums(beta, Z, A);
  for (int c = tid; c < dd; c += WG) {
    const float v = zn[c];
    if (v > 0.0f) zn[c] = (float)(M * exp(beta * (log((double)v) - lmax)) / Z);
  }
  if (tid == 0 && beta_out) beta_out[blockIdx.x] = beta;
}

// Quantisation of histograms to point counts: each cell rounded to the
// nearest integer, halves upwards, in FP64 from the float32 value (exact).
__global__ void quantize_kernel(const float* __restrict__ z, int64_t total, float* __restrict__ q) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < total) q[c] = (float)floor((double)z[c] + 0.5);
}

// sinkhorn_dist_batch and sinkhorn_dist_bounds_batch: the workspace is the
// routing flags, the list slots, the launch order and (with `state`) the
// scaled warm-start records.
// Tables of the 1-D kernels and costs of a context (section 3, the tables
// before Propositions 2 and 3) in the layout padded to D, index delta + D - 1,
// built on the host in FP64 and uploaded in one allocation; the seven
// pointers are set on success (the first one owns the allocation).
int upload_tables(const pdsink_params& p, int D, int** ge_d, float** gm_d, int** gde_d, float** gdm_d, float** c1_d,
                  float** cd_d, int** kb_d) {
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
  char* base = nullptr;
  if (hipMalloc(&base, (size_t)n * 4 * 7) != hipSuccess) return PDSINK_ENOMEM;
  const void* src[7] = {ge.data(), gm.data(), gde.data(), gdm.data(), c1.data(), cd.data(), kb.data()};
  for (int t = 0; t < 7; ++t) {
    if (hipMemcpy(base + (size_t)t * n * 4, src[t], (size_t)n * 4, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(base);
      return PDSINK_EDEVICE;
    }
  }
  *ge_d = (int*)base;
  *gm_d = (float*)(base + n * 4);
  *gde_d = (int*)(base + n * 8);
  *gdm_d = (float*)(base + n * 12);
  *c1_d = (float*)(base + n * 16);
  *cd_d = (float*)(base + n * 20);
  *kb_d = (int*)(base + n * 24);
  return PDSINK_OK;
}

int dist_impl(pdsink_ctx* ctx, int64_t n_pairs, const float* hist_a, const float* hist_b, const int32_t* ia,
              const int32_t* ib, double* state, double* cost, int32_t* iters, float* err, int32_t* status,
              double* upper, double* lower, void* ws, size_t ws_bytes, void* stream, pdsink_done* done = nullptr,
              uint32_t done_tag = 0) {
  if (!ctx || n_pairs < 0) return PDSINK_EINVAL;
  if (n_pairs == 0) return PDSINK_OK;
  if (n_pairs > INT_MAX || !hist_a || !hist_b || !ia || !ib || !cost || !iters || !err || !status)
    return PDSINK_EINVAL;
  size_t need = 0;
  pdsink_workspace_bytes(ctx, state ? PDSINK_OP_DIST_WARM : PDSINK_OP_DIST, n_pairs, &need);
  if (!ws || ws_bytes < need) return PDSINK_ENOMEM;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  const hipStream_t st = (hipStream_t)stream;
  PairExtras ex;
  ex.n_slots = (int)slots_for(ctx, n_pairs);
  ex.lists = (char*)ws + align256(n_pairs);
  ex.ops = ex.lists + ex.n_slots * list_bytes(ctx->D);
  ex.order = ex.lists + ex.n_slots * slot_bytes(ctx->D);
  ex.upper = upper;
  ex.lower = lower;
  ex.done = reinterpret_cast<DoneRec*>(done);
  ex.done_tag = done_tag;
  if (state) {
    ex.state = ex.order + order_bytes(n_pairs);
    ex.state_in = 1;
    const int rc = warm_convert(ctx->D, true, state, hist_b, ib, ctx->prm.d, n_pairs, ex.state, st);
    if (rc) return rc;
  }
  int rc = run_pairs(ctx, n_pairs, hist_a, hist_b, ia, ib, cost, iters, err, status, (unsigned char*)ws, ex, st);
  if (rc || !state) return rc;
  return warm_convert(ctx->D, false, state, hist_b, ib, ctx->prm.d, n_pairs, ex.state, st);
}

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
  if (p.d < 2 || p.d > 256 || !(p.p >= 1.0) || !(p.gamma > 0.0) || !(p.tol >= 0.0) || p.max_iter < 1 ||
      (p.precision != PDSINK_FP32 && p.precision != PDSINK_BF16_REFINE) || !(p.switch_tol >= 0.0) ||
      !std::isfinite(p.gamma) || !std::isfinite(p.p) || p.gamma < 1e-5 || p.kernel < PDSINK_KERNEL_AUTO ||
      p.kernel > PDSINK_KERNEL_GENERAL ||
      (p.kernel == PDSINK_KERNEL_RESIDENT && (p.d < RESIDENT_DMIN || p.d > FAST_DMAX)))
    return PDSINK_EINVAL;
  DeviceGuard g(device);
  if (!g.ok) return PDSINK_EDEVICE;
  const int D = pad_grid(p.d);
  pdsink_ctx* ctx = new (std::nothrow) pdsink_ctx;
  if (!ctx) return PDSINK_ENOMEM;
  std::memset(ctx, 0, sizeof(*ctx));
  ctx->prm = p;
  ctx->device = device;
  ctx->D = D;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1) ncu = 1;
    ctx->n_cu = ncu;
  }
  // With the context's device current: the no-allocation call's scratch.  A
  // failed lookup leaves ctx->scratch NULL, and only that call reports it.
  (void)scratch_lookup(device, &ctx->scratch);
  int rc = upload_tables(p, D, &ctx->ge, &ctx->gm, &ctx->gde, &ctx->gdm, &ctx->c1, &ctx->cd, &ctx->kb);
  if (rc == PDSINK_OK && resident_grid(p.d) && p.kernel != PDSINK_KERNEL_GENERAL) {
    // the resident kernel reads the 128-padded layout
    if (D == 128) {
      ctx->rge = ctx->ge;
      ctx->rgm = ctx->gm;
      ctx->rgde = ctx->gde;
      ctx->rgdm = ctx->gdm;
      ctx->rc1 = ctx->c1;
      ctx->rcd = ctx->cd;
      ctx->rkb = ctx->kb;
    } else {
      rc = upload_tables(p, 128, &ctx->rge, &ctx->rgm, &ctx->rgde, &ctx->rgdm, &ctx->rc1, &ctx->rcd, &ctx->rkb);
      if (rc == PDSINK_OK) ctx->rbase = reinterpret_cast<char*>(ctx->rge);
    }
  }
  if (rc != PDSINK_OK) {
    if (ctx->ge) (void)hipFree(ctx->ge);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return PDSINK_OK;
}

void pdsink_ctx_destroy(pdsink_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipFree(ctx->ge);
  if (ctx->rbase) (void)hipFree(ctx->rbase);
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
    case PDSINK_OP_DIST:   // routing flag per pair, support lists per slot, launch order
      *bytes = align256(n_items) + slots_for(ctx, n_items) * slot_bytes(ctx->D) + order_bytes(n_items);
      return PDSINK_OK;
    case PDSINK_OP_DIST_WARM:   // the same, then one scaled warm-start record per pair
      *bytes = align256(n_items) + slots_for(ctx, n_items) * slot_bytes(ctx->D) + order_bytes(n_items) +
               align256(n_items * warm_bytes(ctx->D));
      return PDSINK_OK;
    case PDSINK_OP_KMEANS:   // ia, ib, cost, iters, err, status, redo per pair, lists per slot, launch order
      *bytes = align256(n_items * 4) * 2 + align256(n_items * 8) + align256(n_items * 8) + align256(n_items * 4) * 2 +
               align256(n_items) + slots_for(ctx, n_items) * slot_bytes(ctx->D) + order_bytes(n_items);
      return PDSINK_OK;
    case PDSINK_OP_BARYCENTER:   // the KMEANS arrays for n pairs, warm states, gradient terms
      *bytes = align256(n_items * 4) * 2 + align256(n_items * 8) + align256(n_items * 8) + align256(n_items * 4) * 2 +
               align256(n_items) + slots_for(ctx, n_items) * slot_bytes(ctx->D) +
               align256(n_items * warm_bytes(ctx->D)) + align256(n_items * 8 * (size_t)ctx->prm.d * ctx->prm.d) +
               256;   // the outer loop's device state
      return PDSINK_OK;
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
  if ((size_t)d * d * sizeof(float) <= 65536)
    hipLaunchKernelGGL(discretize_kernel<false>, dim3((unsigned)n_diag), dim3(WG), (size_t)d * d * sizeof(float),
                       (hipStream_t)stream, pts, offsets, d, hist, mass, n_bad);
  else
    hipLaunchKernelGGL(discretize_kernel<true>, dim3((unsigned)n_diag), dim3(WG), 0, (hipStream_t)stream, pts, offsets,
                       d, hist, mass, n_bad);
  return last_error();
}

int sinkhorn_dist_batch(pdsink_ctx* ctx, int64_t n_pairs, const float* hist_a, const float* hist_b,
                        const int32_t* ia, const int32_t* ib, double* state, double* cost, int32_t* iters,
                        float* err, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  return dist_impl(ctx, n_pairs, hist_a, hist_b, ia, ib, state, cost, iters, err, status, nullptr, nullptr, ws,
                   ws_bytes, stream);
}

int sinkhorn_dist_batch_notify(pdsink_ctx* ctx, int64_t n_pairs, const float* hist_a, const float* hist_b,
                               const int32_t* ia, const int32_t* ib, double* cost, int32_t* iters, float* err,
                               int32_t* status, pdsink_done* done, uint32_t tag, void* ws, size_t ws_bytes,
                               void* stream) {
  if (n_pairs > 0 && (!done || tag == 0)) return PDSINK_EINVAL;
  return dist_impl(ctx, n_pairs, hist_a, hist_b, ia, ib, nullptr, cost, iters, err, status, nullptr, nullptr, ws,
                   ws_bytes, stream, done, tag);
}

int sinkhorn_dist_batch_noalloc(pdsink_ctx* ctx, int64_t n_pairs, const float* hist_a, const float* hist_b,
                                const int32_t* ia, const int32_t* ib, double* cost, int32_t* iters, float* err,
                                int32_t* status, void* stream) {
  if (!ctx || n_pairs < 0) return PDSINK_EINVAL;
  if (n_pairs == 0) return PDSINK_OK;
  if (!hist_a || !hist_b || !ia || !ib || !cost || !iters || !err || !status) return PDSINK_EINVAL;
  if (n_pairs > PDSINK_NOALLOC_MAX_PAIRS) return PDSINK_ENOMEM;
  if (!ctx->scratch) return PDSINK_EDEVICE;
  // The workspace of sinkhorn_dist_batch, carved from the scratch array: flags
  // and launch order first, then as many list slots as the rest holds.
  const size_t head = align256((size_t)n_pairs) + order_bytes(n_pairs);
  const int64_t fit = (int64_t)((PDSINK_NOALLOC_SCRATCH_BYTES - head) / slot_bytes(ctx->D));
  if (fit < 1) return PDSINK_ENOMEM;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  char* base = static_cast<char*>(ctx->scratch);
  PairExtras ex;
  const int64_t want = slots_for(ctx, n_pairs);
  ex.n_slots = (int)(want < fit ? want : fit);
  ex.order = base + align256((size_t)n_pairs);
  ex.lists = ex.order + order_bytes(n_pairs);
  ex.ops = ex.lists + ex.n_slots * list_bytes(ctx->D);
  return run_pairs(ctx, n_pairs, hist_a, hist_b, ia, ib, cost, iters, err, status, (unsigned char*)base, ex,
                   (hipStream_t)stream);
}

int sinkhorn_dist_bounds_batch(pdsink_ctx* ctx, int64_t n_pairs, const float* hist_a, const float* hist_b,
                               const int32_t* ia, const int32_t* ib, double* cost, int32_t* iters, float* err,
                               int32_t* status, double* upper, double* lower, void* ws, size_t ws_bytes,
                               void* stream) {
  return dist_impl(ctx, n_pairs, hist_a, hist_b, ia, ib, nullptr, cost, iters, err, status, upper, lower, ws,
                   ws_bytes, stream);
}

int pd_sharpen(pdsink_ctx* ctx, int64_t n, float* z, double h0, double* beta, void* stream) {
  if (!ctx || n < 0 || !(h0 >= 0.0) || !std::isfinite(h0)) return PDSINK_EINVAL;
  if (n == 0) return PDSINK_OK;
  if (!z || n > INT_MAX) return PDSINK_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  hipLaunchKernelGGL(sharpen_kernel, dim3((unsigned)n), dim3(WG), 0, (hipStream_t)stream, z,
                     ctx->prm.d * ctx->prm.d, h0, beta);
  return last_error();
}

int pd_quantize(pdsink_ctx* ctx, int64_t n, const float* z, float* q, void* stream) {
  if (!ctx || n < 0) return PDSINK_EINVAL;
  if (n == 0) return PDSINK_OK;
  if (!z || !q) return PDSINK_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  const int64_t total = n * (int64_t)ctx->prm.d * ctx->prm.d;
  if (total / 256 + 1 > (int64_t)UINT_MAX) return PDSINK_EINVAL;
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream, z,
                     total, q);
  return last_error();
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
  w += align256(np);
  PairExtras ex;
  ex.lists = w;
  ex.n_slots = (int)slots_for(ctx, np);
  ex.ops = w + ex.n_slots * list_bytes(ctx->D);
  ex.order = w + ex.n_slots * slot_bytes(ctx->D);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(kmeans_pairs_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, n_diag, k, ia, ib);
  int rc = last_error();
  if (rc) return rc;
  rc = run_pairs(ctx, np, hist, centroids, ia, ib, cost, iters, err, st, redo, ex, s);
  if (rc) return rc;
  hipLaunchKernelGGL(kmeans_argmin_kernel, dim3((unsigned)((n_diag + 255) / 256)), dim3(256), 0, s, n_diag, k, cost,
                     assign, dist, st, status);
  return last_error();
}

int pd_barycenter(pdsink_ctx* ctx, int64_t n_diag, const float* hist, double lambda, int32_t max_outer,
                  double energy_rtol, int32_t init_uniform, float* z, double* energy, int32_t* outer, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!ctx || n_diag < 1 || n_diag > INT_MAX || !hist || !z || !energy || !outer || max_outer < 1 ||
      !(lambda >= 0.0) || !std::isfinite(lambda) || !(energy_rtol >= 0.0))
    return PDSINK_EINVAL;
  const int64_t N = n_diag;
  size_t need = 0;
  pdsink_workspace_bytes(ctx, PDSINK_OP_BARYCENTER, N, &need);
  if (!ws || ws_bytes < need) return PDSINK_ENOMEM;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  const int d = ctx->prm.d;
  char* w = (char*)ws;
  int32_t* ia = (int32_t*)w;
  w += align256(N * 4);
  int32_t* ib = (int32_t*)w;
  w += align256(N * 4);
  double* cost = (double*)w;
  w += align256(N * 8);
  int32_t* iters = (int32_t*)w;
  w += align256(N * 8);
  float* err = (float*)w;
  w += align256(N * 4);
  int32_t* st = (int32_t*)w;
  w += align256(N * 4);
  unsigned char* redo = (unsigned char*)w;
  w += align256(N);
  PairExtras ex;
  ex.lists = w;
  ex.n_slots = (int)slots_for(ctx, N);
  ex.ops = w + ex.n_slots * list_bytes(ctx->D);
  w += ex.n_slots * slot_bytes(ctx->D);
  ex.state = w;
  w += align256(N * warm_bytes(ctx->D));
  ex.gout = (double*)w;
  hipStream_t s = (hipStream_t)stream;

  hipLaunchKernelGGL(bary_pairs_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, ia, ib);
  int rc = last_error();
  if (rc) return rc;
  if (init_uniform) {
    // uniform on the cells j >= i, total mass = mean diagram mass (reusing cost[] for the masses)
    hipLaunchKernelGGL(hist_mass_kernel, dim3((unsigned)N), dim3(WG), 0, s, hist, d, cost);
    hipLaunchKernelGGL(bary_uniform_kernel, dim3((unsigned)((d * d + 255) / 256)), dim3(256), 0, s, cost, N, d, z);
    if ((rc = last_error())) return rc;
  }
  // Every outer step is enqueued at once; the energy kernel of step t runs the
  // stopping test on the device, and the launches after it do nothing.  One
  // synchronisation at the end reads the result.
  BaryCtl* ctl = reinterpret_cast<BaryCtl*>(ex.gout + (size_t)N * d * d);
  ex.stop = &ctl->stop;
  hipLaunchKernelGGL(bary_ctl_init_kernel, dim3(1), dim3(64), 0, s, ctl);
  if ((rc = last_error())) return rc;
  for (int t = 0; t < max_outer; ++t) {
    ex.state_in = t > 0;
    rc = run_pairs(ctx, N, z, hist, ia, ib, cost, iters, err, st, redo, ex, s);
    if (rc) return rc;
    hipLaunchKernelGGL(bary_energy_kernel, dim3(1), dim3(WG), 0, s, cost, st, N, t, max_outer, energy_rtol, ctl);
    // z <- z exp(-lambda grad), grad = (gamma / N) sum_i (log u_i + log v_i,Delta)  (Proposition 5)
    hipLaunchKernelGGL(bary_step_kernel, dim3((unsigned)((d * d + 255) / 256)), dim3(256), 0, s, ex.gout, N, d,
                       lambda * ctx->prm.gamma / (double)N, z, ctl);
    if ((rc = last_error())) return rc;
  }
  BaryCtl h;
  if (hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return PDSINK_EDEVICE;
  if (h.err) return PDSINK_ERANGE;
  *energy = h.energy;
  *outer = h.outer;
  return PDSINK_OK;
}

int pdsink_phase_profile(uint64_t* out, int reset) {
#if PDSINK_PROFILE
  if (!out) return PDSINK_EINVAL;
  unsigned long long h[PH_COUNT];
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpyFromSymbol(h, HIP_SYMBOL(g_phase), sizeof(h), 0, hipMemcpyDeviceToHost) != hipSuccess)
    return PDSINK_EDEVICE;
  for (int k = 0; k < PH_COUNT; ++k) out[k] = h[k];
  if (reset) {
    const unsigned long long z[PH_COUNT] = {};
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase), z, sizeof(z), 0, hipMemcpyHostToDevice) != hipSuccess)
      return PDSINK_EDEVICE;
  }
  return PDSINK_OK;
#else
  (void)out;
  (void)reset;
  return PDSINK_EINVAL;
#endif
}

int pdsink_lloyd_workspace_bytes(const pdsink_ctx* ctx, int64_t n_diag, int32_t k, size_t* bytes) {
  if (!ctx || !bytes || n_diag < 0 || k < 1) return PDSINK_EINVAL;
  const int64_t dd = (int64_t)ctx->prm.d * ctx->prm.d;
  size_t kw = 0, bw = 0;
  pdsink_workspace_bytes(ctx, PDSINK_OP_KMEANS, n_diag * k, &kw);
  pdsink_workspace_bytes(ctx, PDSINK_OP_BARYCENTER, n_diag, &bw);
  *bytes = align256(kw) + align256(n_diag * k * 8) + align256(n_diag * 4) + align256(n_diag * dd * 4) + bw;
  return PDSINK_OK;
}

int kmeans_lloyd(pdsink_ctx* ctx, int64_t n_diag, const float* hist, int32_t k, const int32_t* init, int32_t rounds,
                 double lambda, int32_t max_outer, double energy_rtol, float* centroids, int32_t* assign,
                 double* objective, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || n_diag < 1 || k < 1 || k > n_diag || !hist || !init || rounds < 0 || !centroids || !assign ||
      max_outer < 1 || (int64_t)n_diag * k > INT_MAX)
    return PDSINK_EINVAL;
  for (int c = 0; c < k; ++c) {
    if (init[c] < 0 || init[c] >= n_diag) return PDSINK_EINVAL;
    for (int e = 0; e < c; ++e)
      if (init[e] == init[c]) return PDSINK_EINVAL;
  }
  size_t need = 0;
  pdsink_lloyd_workspace_bytes(ctx, n_diag, k, &need);
  if (!ws || ws_bytes < need) return PDSINK_ENOMEM;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PDSINK_EDEVICE;
  const int64_t dd = (int64_t)ctx->prm.d * ctx->prm.d;
  size_t kw = 0, bw = 0;
  pdsink_workspace_bytes(ctx, PDSINK_OP_KMEANS, n_diag * k, &kw);
  pdsink_workspace_bytes(ctx, PDSINK_OP_BARYCENTER, n_diag, &bw);
  char* w = (char*)ws;
  char* kws = w;
  w += align256(kw);
  double* dist = (double*)w;
  w += align256(n_diag * k * 8);
  int32_t* midx = (int32_t*)w;
  w += align256(n_diag * 4);
  float* memb = (float*)w;
  w += align256(n_diag * dd * 4);
  char* bws = w;
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < k; ++c)
    if (hipMemcpyAsync(centroids + c * dd, hist + (int64_t)init[c] * dd, dd * 4, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return PDSINK_EDEVICE;
  std::vector<int32_t> ha(n_diag), members;
  std::vector<double> hd(n_diag * k);
  members.reserve(n_diag);
  for (int r = 0; r < rounds; ++r) {
    int rc = kmeans_assign(ctx, n_diag, hist, k, centroids, assign, dist, nullptr, kws, kw, stream);
    if (rc) return rc;
    if (hipMemcpyAsync(ha.data(), assign, n_diag * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hd.data(), dist, n_diag * k * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PDSINK_EDEVICE;
    double obj = 0.0;
    for (int64_t n = 0; n < n_diag; ++n) obj += hd[n * k + ha[n]];
    if (!std::isfinite(obj)) return PDSINK_ERANGE;
    if (objective) objective[r] = obj;
    for (int c = 0; c < k; ++c) {
      members.clear();
      for (int64_t n = 0; n < n_diag; ++n)
        if (ha[n] == c) members.push_back((int32_t)n);
      if (members.empty()) continue;
      const int64_t m = (int64_t)members.size();
      if (hipMemcpyAsync(midx, members.data(), m * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return PDSINK_EDEVICE;
      hipLaunchKernelGGL(gather_hist_kernel, dim3((unsigned)((dd + 255) / 256), (unsigned)m), dim3(256), 0, s, hist,
                         midx, (int)dd, memb);
      if ((rc = last_error())) return rc;
      double E = 0.0;
      int32_t outer = 0;
      size_t bneed = 0;
      pdsink_workspace_bytes(ctx, PDSINK_OP_BARYCENTER, m, &bneed);
      rc = pd_barycenter(ctx, m, memb, lambda, max_outer, energy_rtol, 1, centroids + c * dd, &E, &outer, bws, bneed,
                         stream);
      if (rc) return rc;
    }
  }
  return PDSINK_OK;
}

}  // extern "C"
