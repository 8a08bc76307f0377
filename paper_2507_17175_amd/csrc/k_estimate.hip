// Phase estimators over a probability vector P (paper section 4.2, the
// precision evaluation): the max-norm estimator (the outcome m of largest
// probability, over N), the weighted average sum_m P(m) m / N / sum P, and the
// circular mean arg(sum_m P(m) exp(2 pi i m / N)) / (2 pi).
//
// Two launches per vector: every block reduces a fixed contiguous range of m
// (threads stride by the block size, then an LDS tree), and one block
// combines the block partials in index order. The partition depends only on
// N, so the FP64 sums are reproducible run to run.
#include "qpe_internal.hpp"

namespace qpe {

namespace {

constexpr int kEstThreads = 256;

struct EstPartial {
  double best;   // largest P met (-1 before any)
  int64_t idx;   // its smallest index (-1 before any)
  double s0;     // sum P
  double s1;     // sum P m / N
  double sc;     // sum P cos(2 pi m / N)
  double ss;     // sum P sin(2 pi m / N)
};

__device__ inline void est_merge(EstPartial& a, const EstPartial& b) {
  if (b.idx >= 0 && (a.idx < 0 || b.best > a.best || (b.best == a.best && b.idx < a.idx))) {
    a.best = b.best;
    a.idx = b.idx;
  }
  a.s0 += b.s0;
  a.s1 += b.s1;
  a.sc += b.sc;
  a.ss += b.ss;
}

// In-block tree over kEstThreads partials held in LDS; the result lands in
// element 0. Every thread of the block must call it.
__device__ inline void est_block_reduce(EstPartial* sh) {
  for (int w = kEstThreads / 2; w > 0; w >>= 1) {
    __syncthreads();
    if (int(threadIdx.x) < w) est_merge(sh[threadIdx.x], sh[threadIdx.x + w]);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kEstThreads) k_est_partial(const double* __restrict__ P, int n, int64_t chunk,
                                                             EstPartial* __restrict__ part) {
  __shared__ EstPartial sh[kEstThreads];
  const int64_t N = int64_t(1) << n;
  const int64_t m0 = int64_t(blockIdx.x) * chunk;
  const int64_t m1 = min(m0 + chunk, N);
  const double inv_n = ldexp(1.0, -n);
  EstPartial acc{-1.0, -1, 0.0, 0.0, 0.0, 0.0};
  for (int64_t m = m0 + threadIdx.x; m < m1; m += kEstThreads) {
    const double p = P[m];
    // NaN fails every comparison, so it never becomes the maximum.
    if (p > acc.best) {
      acc.best = p;
      acc.idx = m;
    }
    const double x = double(m) * inv_n;  // exact
    double sv, cv;
    sincospi(2.0 * x, &sv, &cv);
    acc.s0 += p;
    acc.s1 += p * x;
    acc.sc += p * cv;
    acc.ss += p * sv;
  }
  sh[threadIdx.x] = acc;
  est_block_reduce(sh);
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kEstThreads) k_est_final(const EstPartial* __restrict__ part, int nparts, int n,
                                                           double* __restrict__ out) {
  __shared__ EstPartial sh[kEstThreads];
  EstPartial acc{-1.0, -1, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += kEstThreads) est_merge(acc, part[b]);
  sh[threadIdx.x] = acc;
  est_block_reduce(sh);
  if (threadIdx.x != 0) return;
  const EstPartial r = sh[0];
  const double two_pi = 6.283185307179586476925286766559;
  double circ = atan2(r.ss, r.sc) / two_pi;
  if (circ < 0.0) circ += 1.0;
  if (circ >= 1.0) circ -= 1.0;  // rounding of a tiny negative angle
  out[0] = r.idx >= 0 ? ldexp(double(r.idx), -n) : __longlong_as_double(0x7ff8000000000000ll);
  out[1] = r.s1 / r.s0;
  out[2] = circ;
  out[3] = r.s0;
  reinterpret_cast<int64_t*>(out)[4] = r.idx;
  reinterpret_cast<int64_t*>(out)[5] = 0;
}

}  // namespace

int est_blocks(int n) {
  const int64_t N = int64_t(1) << n;
  const int64_t want = (N + 4095) / 4096;
  return int(want < kEstMaxBlocks ? want : kEstMaxBlocks);
}

size_t est_workspace_bytes() { return align_up(size_t(kEstMaxBlocks) * sizeof(EstPartial)); }

hipError_t launch_estimate(const double* P, int n, void* scratch, double* out, hipStream_t s) {
  const int B = est_blocks(n);
  const int64_t N = int64_t(1) << n;
  const int64_t chunk = (N + B - 1) / B;
  EstPartial* part = static_cast<EstPartial*>(scratch);
  hipLaunchKernelGGL(k_est_partial, dim3(B), dim3(kEstThreads), 0, s, P, n, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_est_final, dim3(1), dim3(kEstThreads), 0, s, part, B, n, out);
  return hipGetLastError();
}

}  // namespace qpe
