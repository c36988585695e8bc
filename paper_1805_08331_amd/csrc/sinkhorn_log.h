// Log-domain path of Algorithm 1 for the pairs the scaled solve flags
// (PDSINK_ST_NONFINITE or PDSINK_ST_RANGE): interface shared by the C ABI and
// its translation unit (pdsink_log.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace pdsink {

struct LogParams {
  int d;
  double p;
  double gamma;
  double tol;
  int max_iter;
  const float* hist_a;
  const float* hist_b;
  const int* ia;
  const int* ib;
  long long n_pairs;
  double* cost;
  int* iters;
  float* err;
  int* status;
  double* upper;   // optional error-control bounds of the pairs this path solves
  double* lower;
  char* scratch;          // per workgroup: scratch_stride bytes, at least 8 d (d + 1)
  size_t scratch_stride;
};

constexpr int LOG_CAP = 1024;   // support cells per side the log-domain path takes
constexpr int ST_LOG = 8;       // status bit: solved by the log-domain path

// One launch over the batch (n_slots workgroups striding over the pairs);
// returns 0, or -1 when the launch failed.
int launch_log_path(const LogParams& lp, int n_slots, hipStream_t st);

}  // namespace pdsink
