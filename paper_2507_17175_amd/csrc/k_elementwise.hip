// Bandwidth-bound kernels of the QPE path: Hadamard layer, twiddle tables,
// operator split into BF16 pieces, Newton-Schulz identity subtraction with
// the unitarity defect, probability readout and the per-run report; their
// grouped (batched) forms; and the device-side builders of the batch
// descriptors and launch tables.
#include "qpe_internal.hpp"

#include <cmath>

namespace qpe {

namespace {

constexpr int kThreads = 256;

inline int grid_for(int64_t work, int per_block = kThreads, int cap = 256 * 64) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

__device__ inline double h_scale(int n) {
  // 2^(-n/2): exact power of two times sqrt(1/2) for odd n
  return ldexp(1.0, -(n / 2)) * ((n & 1) ? 0.70710678118654752440 : 1.0);
}

// ----------------------------------------------------------- device bodies

// H on every qubit of |0...0> gives the uniform superposition, so every row
// of the (N x d) state becomes psi * 2^(-n/2) (Fig. 1, H layer). The complex64
// form writes two amplitudes per float4 (pairs [p0, p1)).
__device__ inline void h_range_c64(const double2* __restrict__ psi, float4* __restrict__ out, int64_t p0, int64_t p1,
                                   int dmask, double scale, int64_t stride) {
  for (int64_t q = p0; q < p1; q += stride) {
    double2 a = psi[(2 * q) & dmask];
    double2 b = psi[(2 * q + 1) & dmask];
    out[q] = make_float4(float(a.x * scale), float(a.y * scale), float(b.x * scale), float(b.y * scale));
  }
}

__device__ inline void h_range_c128(const double2* __restrict__ psi, double2* __restrict__ out, int64_t e0, int64_t e1,
                                    int dmask, double scale, int64_t stride) {
  for (int64_t q = e0; q < e1; q += stride) {
    double2 a = psi[q & dmask];
    out[q] = make_double2(a.x * scale, a.y * scale);
  }
}

// tw_lo[t] = exp(-2 pi i t / N) for t < 2^h; tw_hi[u] = exp(-2 pi i u 2^h / N).
// The angle -2 t / N (in units of pi) is exact in binary.
__device__ inline void twiddle_entry(double2* __restrict__ tw_hi, double2* __restrict__ tw_lo, int n, int h,
                                     int64_t t) {
  int64_t nlo = int64_t(1) << h;
  int64_t e = t < nlo ? t : ((t - nlo) << h);
  double x = -ldexp(double(e), 1 - n);  // -2 e / N
  double sv, cv;
  sincospi(x, &sv, &cv);
  if (t < nlo)
    tw_lo[t] = make_double2(cv, sv);
  else
    tw_hi[t - nlo] = make_double2(cv, sv);
}

// Round a double to the nearest BF16 value (ties to even); returns the BF16
// bit pattern and the rounded value as a double. Magnitudes here lie far
// inside the normal range of both formats.
__device__ inline uint16_t bf16_rne(double x, double* rounded) {
  if (x == 0.0) {
    *rounded = 0.0;
    return 0;
  }
  uint64_t b = __double_as_longlong(x);
  uint64_t lsb = (b >> 45) & 1;
  b += ((uint64_t(1) << 44) - 1) + lsb;
  b &= ~((uint64_t(1) << 45) - 1);
  double y = __longlong_as_double(b);
  *rounded = y;
  float f = float(y);  // exact: y has 8 significant bits
  return uint16_t(__float_as_uint(f) >> 16);
}

// Operator preparation for the mixed controlled GEMM: the complex FP64
// matrix V (d x d) is split, per real component w, into three BF16 pieces
// w = hi + mid + lo (each the RNE rounding of the remaining residual). Plane
// p = 2 * piece + component (component 0 = real, 1 = imaginary). Inside a
// plane the layout is blocked by 16 columns: element (row j, col c) sits at
// ((c / 16) * d + j) * 16 + c % 16, so that a tile of consecutive rows and 16
// consecutive columns is contiguous.
__device__ inline void split_value(double2 v, uint16_t* __restrict__ planes, int t, int64_t e) {
  const int64_t d = int64_t(1) << t;
  const int64_t dd = d * d;
  int64_t j = e >> t, c = e & (d - 1);
  int64_t dst = (((c >> 4) * d + j) << 4) + (c & 15);
  double w[2] = {v.x, v.y};
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
    double r0 = w[comp], q0, q1, q2;
    uint16_t hi = bf16_rne(r0, &q0);
    double r1 = r0 - q0;
    uint16_t mid = bf16_rne(r1, &q1);
    double r2 = r1 - q1;
    uint16_t lo = bf16_rne(r2, &q2);
    planes[(0 * 2 + comp) * dd + dst] = hi;
    planes[(1 * 2 + comp) * dd + dst] = mid;
    planes[(2 * 2 + comp) * dd + dst] = lo;
  }
}

// Operator preparation for the split-FP16 controlled GEMM: each FP64
// component w of V, scaled by 2^kOpScaleLog2F16, is split into two FP16
// pieces (hi = RNE(w'), lo = RNE(w' - hi)); plane p = 2 piece + component,
// blocked by 16 columns as the BF16 planes.
__device__ inline void split_value_f16(double2 v, uint16_t* __restrict__ planes, int t, int64_t e) {
  const int64_t d = int64_t(1) << t;
  uint16_t p[4];
  split_f16_pieces(v, p);
#pragma unroll
  for (int pl = 0; pl < 4; ++pl) planes[pl * d * d + plane_offset(d, e >> t, e & (d - 1))] = p[pl];
}

// The same for the four columns c .. c+3 (c a multiple of 4, d >= 4) of one
// row, starting at element e0: they share a 16-column block, so each plane
// takes their four pieces as one 8-byte store.
__device__ inline void split4_f16(const double2 (&v)[4], uint16_t* __restrict__ planes, int t, int64_t e0) {
  const int64_t d = int64_t(1) << t;
  const int64_t dd = d * d;
  const int64_t dst = plane_offset(d, e0 >> t, e0 & (d - 1));
  uint16_t p[4][4];  // [plane][column]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint16_t q[4];
    split_f16_pieces(v[i], q);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) p[pl][i] = q[pl];
  }
#pragma unroll
  for (int pl = 0; pl < 4; ++pl)
    *reinterpret_cast<uint2*>(planes + pl * dd + dst) =
        make_uint2(uint32_t(p[pl][0]) | (uint32_t(p[pl][1]) << 16), uint32_t(p[pl][2]) | (uint32_t(p[pl][3]) << 16));
}

__device__ inline void split_entry(const double2* __restrict__ V, uint16_t* __restrict__ planes, int t, int64_t e,
                                   bool conj = false, bool f16 = false) {
  double2 v = V[e];
  if (conj) v.y = -v.y;
  if (f16)
    split_value_f16(v, planes, t, e);
  else
    split_value(v, planes, t, e);
}

// The state scale sigma of the split-FP16 products: a power of two with
// sigma r in [2^13, 2^14), r = ||psi|| 2^(-n/2) the norm of every state row
// (the H layer gives every row psi 2^(-n/2), and unitary steps keep it), so
// that no scaled amplitude exceeds 2^14 (FP16 overflows at 65520). One block.
__device__ inline void state_scale_block(const double2* __restrict__ psi, int n, int t, float* __restrict__ sigma) {
  __shared__ double red[kThreads];
  double q = 0.0;
  for (int i = threadIdx.x; i < (1 << t); i += kThreads) q += psi[i].x * psi[i].x + psi[i].y * psi[i].y;
  red[threadIdx.x] = q;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = sqrt(red[0]) * h_scale(n);
    int e = 0;
    if (r > 0.0 && r < 1e300) (void)frexp(r, &e);  // r = m 2^e, m in [0.5, 1)
    const int sh = min(max(kOpScaleLog2F16 - e, -100), 100);
    *sigma = r > 0.0 && r < 1e300 ? ldexpf(1.0f, sh) : 1.0f;
  }
}

__device__ inline double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

// Newton-Schulz support: G <- G - I over elements [e0, e1) (stride), then
// defect = max(defect, max |G_ij|). The max of non-negative doubles is
// order-independent, so the atomic on the IEEE bit pattern (monotone for
// non-negative values) is deterministic.
// Block-wide max of the threads' mx into *defect_bits (every thread calls).
__device__ inline void block_max_to(double mx, unsigned long long* __restrict__ defect_bits) {
  __shared__ double red[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) mx = nan_max(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) mx = nan_max(mx, red[w]);
    if (mx != mx) mx = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf
    atomicMax(defect_bits, (unsigned long long)__double_as_longlong(mx));
  }
}

// The partial slots of a split Gram product (G2: the `extra` slots after
// slot 0, d^2 apart) added to g in slot order.
__device__ inline double2 add_gram_slots(double2 g, const double2* __restrict__ G2, int extra, int64_t dd, int64_t e) {
  for (int sl = 0; sl < extra; ++sl) {
    const double2 h = G2[sl * dd + e];
    g.x += h.x;
    g.y += h.y;
  }
  return g;
}

__device__ inline void subi_range(double2* __restrict__ G, const double2* __restrict__ G2, int d, int64_t e0,
                                  int64_t e1, int64_t stride, unsigned long long* __restrict__ defect_bits) {
  double mx = 0.0;
  const int t = 31 - __builtin_clz(unsigned(d));
  const int extra = G2 ? gram_extra_slots(t) : 0;
  for (int64_t e = e0; e < e1; e += stride) {
    double2 g = G[e];
    const bool diag = (e / d) == (e % d);
    if (G2) g = add_gram_slots(g, G2, extra, int64_t(d) * d, e);
    if (diag) g.x -= 1.0;
    if (G2 || diag) G[e] = g;
    mx = nan_max(mx, sqrt(g.x * g.x + g.y * g.y));
  }
  block_max_to(mx, defect_bits);
}

// Readout rows: P(m(p)) = 2^-n sum_r |X[p][r]|^2 in FP64 (components widened
// before squaring). The DFT passes leave out the inverse QFT's 2^(-n/2), so
// the exact power of two 2^-n restores it here. One row per group of
// G = min(d, 64) lanes of a wave; a fixed shuffle tree makes the sum order
// deterministic. `base` is the wave's first row.
template <typename T>
__device__ inline void prob_rows(const T* __restrict__ X, double* __restrict__ prob, int n, int t,
                                 const DftPlan& plan, double scale, int64_t base) {
  const int64_t N = int64_t(1) << n;
  const int d = 1 << t;
  const int G = d < 64 ? d : 64;
  const int lane = threadIdx.x & 63;
  int64_t p = base + lane / G;
  int c0 = lane % G;
  double acc = 0.0;
  if (p < N) {
    const T* row = X + p * d;
    // unrolled so that several loads are in flight; the sum keeps its order
#pragma unroll 4
    for (int c = c0; c < d; c += G) {
      T v = row[c];
      double re = double(v.x), im = double(v.y);
      acc += re * re + im * im;
    }
  }
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (c0 == 0 && p < N) prob[prob_index(p, n, plan)] = acc * scale;
}

// Readout after a fused last DFT pass: row p's partial sums, one per column
// group, added in group order.
__device__ inline void finish_row(const double* __restrict__ part, double* __restrict__ prob, int n, int groups,
                                  const DftPlan& plan, double scale, int64_t p) {
  const int64_t N = int64_t(1) << n;
  double acc = 0.0;
  for (int g = 0; g < groups; ++g) acc += part[g * N + p];
  prob[prob_index(p, n, plan)] = acc * scale;
}

// Report: prob_sum, ||psi||^2, the input's peak weight, the defect and the
// flags, by one block. With `part` (nparts pairs: partial sum, non-finite
// flag, from k_report_partial) it adds the partial sums instead of reading
// the 2^n probabilities itself. rot_peak: the rotated input's peak weight, or
// null for max_i |psi_i|^2 / ||psi||^2 of psi itself; check: flag a peak
// weight above kPeakFlag.
__device__ inline void report_block(const double* __restrict__ prob, int n, const double2* __restrict__ psi, int t,
                                    const unsigned long long* __restrict__ defect_bits,
                                    const double* __restrict__ rot_peak, bool check, double* __restrict__ report,
                                    const double* __restrict__ part = nullptr, int nparts = 0) {
  __shared__ double red[3][kThreads];
  __shared__ int any_bad;
  const int64_t N = int64_t(1) << n;
  const int d = 1 << t;
  double s = 0.0, q = 0.0, mx = 0.0;
  bool bad = false;
  if (part) {
    for (int i = threadIdx.x; i < nparts; i += kThreads) {
      s += part[2 * i];
      bad |= part[2 * i + 1] != 0.0;
    }
  } else {
    for (int64_t i = threadIdx.x; i < N; i += kThreads) {
      double v = prob[i];
      bad |= !(v == v) || v > 1e300 || v < -1e300;
      s += v;
    }
  }
  for (int i = threadIdx.x; i < d; i += kThreads) {
    const double w = psi[i].x * psi[i].x + psi[i].y * psi[i].y;
    q += w;
    mx = fmax(mx, w);
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = q;
  red[2][threadIdx.x] = mx;
  if (threadIdx.x == 0) any_bad = 0;
  __syncthreads();
  if (bad) atomicOr(&any_bad, 1);
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double defect = defect_bits ? __longlong_as_double((long long)defect_bits[0]) : 0.0;
    double ps = red[0][0], pn = red[1][0];
    const double peak = rot_peak ? rot_peak[0] : (pn > 0.0 ? red[2][0] / pn : 0.0);
    unsigned flags = 0;
    if (defect > 1e-6 || defect != defect) flags |= 1u;
    if (any_bad || !(fabs(ps - pn) <= 1e-4 * pn)) flags |= 2u;
    if (check && peak > kPeakFlag) flags |= 4u;
    report[0] = defect;
    report[1] = ps;
    report[2] = pn;
    report[3] = peak;
    reinterpret_cast<uint32_t*>(report + 4)[0] = flags;
    reinterpret_cast<uint32_t*>(report + 4)[1] = 0u;
  }
}

// ------------------------------------------------------ single-instance kernels

__global__ void __launch_bounds__(kThreads) k_h_broadcast_c64(const double2* __restrict__ psi,
                                                              float4* __restrict__ out, int64_t pairs,
                                                              int dmask, double scale) {
  h_range_c64(psi, out, blockIdx.x * int64_t(kThreads) + threadIdx.x, pairs, dmask, scale,
              int64_t(gridDim.x) * kThreads);
}

__global__ void k_h_single_c64(const double2* __restrict__ psi, float2* __restrict__ out, double scale) {
  if (threadIdx.x == 0) out[0] = make_float2(float(psi[0].x * scale), float(psi[0].y * scale));
}

__global__ void __launch_bounds__(kThreads) k_h_broadcast_c128(const double2* __restrict__ psi,
                                                               double2* __restrict__ out, int64_t total,
                                                               int dmask, double scale) {
  h_range_c128(psi, out, blockIdx.x * int64_t(kThreads) + threadIdx.x, total, dmask, scale,
               int64_t(gridDim.x) * kThreads);
}

__global__ void __launch_bounds__(kThreads) k_twiddles(double2* __restrict__ tw_hi, double2* __restrict__ tw_lo,
                                                       int n, int h) {
  int64_t total = (int64_t(1) << h) + (int64_t(1) << (n - h));
  for (int64_t t = blockIdx.x * int64_t(kThreads) + threadIdx.x; t < total; t += int64_t(gridDim.x) * kThreads)
    twiddle_entry(tw_hi, tw_lo, n, h, t);
}

// Newton-Schulz correction X E in split BF16 (E = X^H X - I is ~1e-15, so
// X rounded to FP32 times E in BF16 pieces, three piece pairs, gives X E to
// ~1e-20): X32 = complex64(X), and planes = split(conj(E)) = split(E^T) (E
// is Hermitian), so that the controlled-product kernel's row x V^T with
// V = conj(E) computes row x E. These per-element bodies serve the batched
// path; the single-instance path runs the fused kernels below.
__device__ inline void ns_prep_entry(const double2* __restrict__ X, const double2* __restrict__ E,
                                     float2* __restrict__ X32, uint16_t* __restrict__ planes, int t, int64_t e) {
  double2 x = X[e];
  X32[e] = make_float2(float(x.x), float(x.y));
  split_entry(E, planes, t, e, true);
}

// out = X - (X E) / 2 in FP64 (one Newton-Schulz step).
__device__ inline void ns_update_entry(const double2* __restrict__ X, const float2* __restrict__ XE,
                                       double2* __restrict__ out, int64_t e) {
  double2 x = X[e];
  float2 c = XE[e];
  out[e] = make_double2(x.x - 0.5 * double(c.x), x.y - 0.5 * double(c.y));
}


// Mixed-form Newton-Schulz preparation in one pass: E = G (+ the slots in G2) - I with the
// defect max |E_ij|, X32 = complex64(X), planes = split(conj(E)). E itself
// is not stored (only its planes are used).
__global__ void __launch_bounds__(kThreads) k_ns_prep_fused(const double2* __restrict__ X,
                                                            const double2* __restrict__ G,
                                                            const double2* __restrict__ G2, float2* __restrict__ X32,
                                                            uint16_t* __restrict__ planes, int t,
                                                            unsigned long long* __restrict__ defect_bits) {
  const int64_t d = int64_t(1) << t, dd = d * d;
  const int extra = G2 ? gram_extra_slots(t) : 0;
  double mx = 0.0;
  for (int64_t e = blockIdx.x * int64_t(kThreads) + threadIdx.x; e < dd; e += int64_t(gridDim.x) * kThreads) {
    double2 g = G[e];
    if (G2) g = add_gram_slots(g, G2, extra, dd, e);
    if ((e >> t) == (e & (d - 1))) g.x -= 1.0;
    mx = nan_max(mx, sqrt(g.x * g.x + g.y * g.y));
    const double2 x = X[e];
    X32[e] = make_float2(float(x.x), float(x.y));
    split_value(make_double2(g.x, -g.y), planes, t, e);
  }
  block_max_to(mx, defect_bits);
}

// The Newton-Schulz update and the operator split of the new power in one
// pass: out = X - XE / 2, planes = split(out).
template <bool F16>
__global__ void __launch_bounds__(kThreads) k_ns_update_split(const double2* __restrict__ X,
                                                              const float2* __restrict__ XE,
                                                              double2* __restrict__ out,
                                                              uint16_t* __restrict__ planes, int t) {
  const int64_t dd = int64_t(1) << (2 * t);
  if constexpr (F16) {
    // four consecutive elements per thread (d >= 32)
    for (int64_t e0 = 4 * (blockIdx.x * int64_t(kThreads) + threadIdx.x); e0 < dd;
         e0 += 4 * int64_t(gridDim.x) * kThreads) {
      double2 o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double2 x = X[e0 + i];
        const float2 c = XE[e0 + i];
        o[i] = make_double2(x.x - 0.5 * double(c.x), x.y - 0.5 * double(c.y));
        out[e0 + i] = o[i];
      }
      split4_f16(o, planes, t, e0);
    }
  } else {
    for (int64_t e = blockIdx.x * int64_t(kThreads) + threadIdx.x; e < dd; e += int64_t(gridDim.x) * kThreads) {
      const double2 x = X[e];
      const float2 c = XE[e];
      const double2 o = make_double2(x.x - 0.5 * double(c.x), x.y - 0.5 * double(c.y));
      out[e] = o;
      split_value(o, planes, t, e);
    }
  }
}

template <bool F16>
__global__ void __launch_bounds__(kThreads) k_split_pieces(const double2* __restrict__ V, uint16_t* __restrict__ planes,
                                                           int t) {
  const int64_t dd = int64_t(1) << (2 * t);
  if constexpr (F16) {
    // four consecutive elements per thread (d >= 32)
    for (int64_t e0 = 4 * (blockIdx.x * int64_t(kThreads) + threadIdx.x); e0 < dd;
         e0 += 4 * int64_t(gridDim.x) * kThreads) {
      double2 v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = V[e0 + i];
      split4_f16(v, planes, t, e0);
    }
  } else {
    for (int64_t e = blockIdx.x * int64_t(kThreads) + threadIdx.x; e < dd; e += int64_t(gridDim.x) * kThreads)
      split_entry(V, planes, t, e, false, false);
  }
}

__global__ void __launch_bounds__(kThreads) k_state_scale(const double2* __restrict__ psi, int n, int t,
                                                          float* __restrict__ sigma) {
  state_scale_block(psi, n, t, sigma);
}

__global__ void __launch_bounds__(kThreads) k_sub_identity_defect(double2* __restrict__ G,
                                                                  const double2* __restrict__ G2, int d,
                                                                  unsigned long long* __restrict__ defect_bits) {
  subi_range(G, G2, d, blockIdx.x * int64_t(kThreads) + threadIdx.x, int64_t(d) * d, int64_t(gridDim.x) * kThreads,
             defect_bits);
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_prob(const T* __restrict__ X, double* __restrict__ prob, int n, int t,
                                                   DftPlan plan, double scale) {
  const int64_t N = int64_t(1) << n;
  const int d = 1 << t;
  const int G = d < 64 ? d : 64;
  const int rows_per_wave = 64 / G;
  const int64_t wave = (blockIdx.x * int64_t(kThreads) + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(gridDim.x) * kThreads) >> 6;
  for (int64_t base = wave * rows_per_wave; base < N; base += nwaves * rows_per_wave)
    prob_rows<T>(X, prob, n, t, plan, scale, base);
}

__global__ void __launch_bounds__(kThreads) k_prob_finish(const double* __restrict__ part, double* __restrict__ prob,
                                                          int n, int groups, DftPlan plan, double scale) {
  const int64_t N = int64_t(1) << n;
  for (int64_t p = blockIdx.x * int64_t(kThreads) + threadIdx.x; p < N; p += int64_t(gridDim.x) * kThreads)
    finish_row(part, prob, n, groups, plan, scale, p);
}

// Row position of outcome m after the DFT passes (the inverse of prob_index):
// bits [B_q, B_{q+1}) of m move to bits [n - B_{q+1}, n - B_q) of p.
__device__ inline int64_t state_position(int64_t m, int n, const DftPlan& plan) {
  int64_t p = 0;
  int hi = n, lo = 0;
  for (int q = 0; q < plan.npass; ++q) {
    hi -= plan.bits[q];
    const int64_t digit = (m >> lo) & ((int64_t(1) << plan.bits[q]) - 1);
    p |= digit << hi;
    lo += plan.bits[q];
  }
  return p;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_gather_state(const T* __restrict__ X, T* __restrict__ out, int n, int t,
                                                           DftPlan plan, double scale) {
  const int64_t total = int64_t(1) << (n + t);
  const int64_t dmask = (int64_t(1) << t) - 1;
  for (int64_t e = blockIdx.x * int64_t(kThreads) + threadIdx.x; e < total; e += int64_t(gridDim.x) * kThreads) {
    const int64_t m = e >> t, r = e & dmask;
    const T v = X[(state_position(m, n, plan) << t) + r];
    T o;
    o.x = decltype(v.x)(double(v.x) * scale);
    o.y = decltype(v.y)(double(v.y) * scale);
    out[e] = o;
  }
}

__global__ void __launch_bounds__(kThreads) k_report(const double* __restrict__ prob, int n,
                                                     const double2* __restrict__ psi, int t,
                                                     const unsigned long long* __restrict__ defect_bits,
                                                     const double* __restrict__ rot_peak, int check,
                                                     double* __restrict__ report, const double* __restrict__ part,
                                                     int nparts) {
  report_block(prob, n, psi, t, defect_bits, rot_peak, check != 0, report, part, nparts);
}

// First stage of the report for large registers: block b sums the
// probabilities [b C, (b + 1) C), C = kReportChunk, in a fixed order (a
// strided pass per thread, then a fixed tree) and flags non-finite values.
constexpr int kReportChunk = 4096;

__global__ void __launch_bounds__(kThreads) k_report_partial(const double* __restrict__ prob,
                                                             double* __restrict__ part) {
  __shared__ double red[kThreads];
  __shared__ int any_bad;
  const double* p = prob + int64_t(blockIdx.x) * kReportChunk;
  double s = 0.0;
  bool bad = false;
#pragma unroll 4
  for (int i = threadIdx.x; i < kReportChunk; i += kThreads) {
    const double v = p[i];
    bad |= !(v == v) || v > 1e300 || v < -1e300;
    s += v;
  }
  red[threadIdx.x] = s;
  if (threadIdx.x == 0) any_bad = 0;
  __syncthreads();
  if (bad) atomicOr(&any_bad, 1);
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0];
    part[2 * blockIdx.x + 1] = any_bad ? 1.0 : 0.0;
  }
}

// After a stand-alone controlled step (whole state in buf0, updated rows
// written to `other`), copy the rows with bit k set back into buf0.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_copy_rows_back(T* __restrict__ state, const T* __restrict__ other, int n,
                                                             int t, int k) {
  const int64_t half = (int64_t(1) << (n - 1)) << t;
  for (int64_t e = blockIdx.x * int64_t(kThreads) + threadIdx.x; e < half; e += int64_t(gridDim.x) * kThreads) {
    int64_t i = e >> t;
    int64_t c = e & ((int64_t(1) << t) - 1);
    int64_t j = ctrl_row(i, k);
    state[(j << t) + c] = other[(j << t) + c];
  }
}

// ----------------------------------------------------------- batch setup

struct DescArgs {
  int first, count;
  BatchProblem p[kBatchChunk];
};

__global__ void k_batch_descs(InstDesc* __restrict__ desc, char* ws, DescArgs a) {
  int i = threadIdx.x;
  if (i >= a.count) return;
  const BatchProblem& p = a.p[i];
  InstDesc D;
  D.n = p.n;
  D.t = p.t;
  D.U = static_cast<const double2*>(p.U);
  D.psi = static_cast<const double2*>(p.psi);
  D.U_src = static_cast<const double2*>(p.U_src);
  D.psi_src = static_cast<const double2*>(p.psi_src);
  D.prob = p.prob;
  D.report = static_cast<double*>(p.report);
  D.ws = ws + p.ws_offset;
  desc[a.first + i] = D;
}

struct TableArgs {
  int nlaunch;
  BatchLaunch l[kBatchLaunchChunk];
};

// One block per launch: its members in instance order and the prefix sums
// of their workgroup counts. The instances are taken 256 at a time; within
// a chunk an LDS scan gives each member its slot and its prefix.
constexpr int kTableThreads = 256;

__global__ void __launch_bounds__(kTableThreads) k_batch_tables(const InstDesc* __restrict__ desc, int ninst,
                                                                int32_t* __restrict__ tables, TableArgs a,
                                                                int mixed, int bflags) {
  if (blockIdx.x >= unsigned(a.nlaunch)) return;  // uniform over the block
  const BatchLaunch L = a.l[blockIdx.x];
  int32_t* tab = tables + L.table_off;
  const int tid = threadIdx.x;
  auto tiles_of = [&](int i) -> int64_t {
    return i < ninst ? batch_tiles(L.kind, L.step, desc[i].n, desc[i].t, mixed != 0, bflags & kBatchPolar,
                                   bflags & kBatchDoubling, bflags)
                     : 0;
  };
  __shared__ int sc[kTableThreads];
  __shared__ long long sr[kTableThreads];
  // number of members (the prefix array follows the member list)
  int mine = 0;
  for (int i = tid; i < ninst; i += kTableThreads) mine += tiles_of(i) > 0 ? 1 : 0;
  sc[tid] = mine;
  __syncthreads();
  for (int w = kTableThreads / 2; w > 0; w >>= 1) {
    if (tid < w) sc[tid] += sc[tid + w];
    __syncthreads();
  }
  const int count = sc[0];
  __syncthreads();
  int carry_c = 0;
  long long carry_r = 0;
  for (int base = 0; base < ninst; base += kTableThreads) {
    const int i = base + tid;
    const int64_t ti = tiles_of(i);
    const int f = ti > 0 ? 1 : 0;
    sc[tid] = f;
    sr[tid] = ti > 0 ? ti : 0;
    __syncthreads();
    // inclusive scans (Hillis-Steele)
    for (int w = 1; w < kTableThreads; w <<= 1) {
      const int c = tid >= w ? sc[tid - w] : 0;
      const long long r = tid >= w ? sr[tid - w] : 0;
      __syncthreads();
      sc[tid] += c;
      sr[tid] += r;
      __syncthreads();
    }
    if (f) {
      const int slot = carry_c + sc[tid] - 1;
      tab[1 + slot] = i;
      tab[1 + count + slot] = int32_t(carry_r + sr[tid] - ti);
    }
    carry_c += sc[kTableThreads - 1];
    carry_r += sr[kTableThreads - 1];
    __syncthreads();
  }
  if (tid == 0) {
    tab[0] = count;
    tab[1 + count + count] = int32_t(carry_r);
  }
}

// --------------------------------------------------------- batched kernels

__device__ inline const double2* power_ptr(const InstDesc& D, const RunLayout& L, int slot) {
  if (slot == 0) return D.U;
  return reinterpret_cast<const double2*>(D.ws + (slot == 1 ? L.vbuf : L.tbuf));
}

template <typename T>
__global__ void __launch_bounds__(kThreads) kb_elementwise(int kind, int step, const InstDesc* __restrict__ desc,
                                                           const int32_t* __restrict__ table, int bflags,
                                                           int64_t tile0) {
  const bool polar = (bflags & kBatchPolar) != 0, dbl = (bflags & kBatchDoubling) != 0;
  constexpr bool mixed = sizeof(T) == 8;
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const RunLayout L = run_layout(D.n, D.t, mixed, polar);
  const int n = D.n, t = D.t, d = 1 << t;
  const int64_t N = int64_t(1) << n;
  unsigned long long* defect = reinterpret_cast<unsigned long long*>(D.ws + L.scratch);
  switch (kind) {
    case BK_ZERO:
      if (threadIdx.x == 0) defect[0] = 0ull;
      break;
    case BK_HLAYER: {
      // the prefix-doubling form only needs row 0
      int64_t e0 = local * kHTile, e1 = min(e0 + int64_t(kHTile), dbl ? int64_t(d) : N * d);
      if (mixed) {
        h_range_c64(D.psi, reinterpret_cast<float4*>(D.ws + L.state0), e0 / 2 + threadIdx.x, e1 / 2, d - 1,
                    h_scale(n), kThreads);
        // an odd element count (row 0 alone with d = 1, prefix doubling) ends
        // with one amplitude the pair writes do not cover
        if ((e1 & 1) && threadIdx.x == 0) {
          const double2 a = D.psi[(e1 - 1) & (d - 1)];
          const double sc = h_scale(n);
          reinterpret_cast<float2*>(D.ws + L.state0)[e1 - 1] = make_float2(float(a.x * sc), float(a.y * sc));
        }
      } else
        h_range_c128(D.psi, reinterpret_cast<double2*>(D.ws + L.state0), e0 + threadIdx.x, e1, d - 1, h_scale(n),
                     kThreads);
      break;
    }
    case BK_TWIDDLE: {
      const int h = tw_split(n);
      int64_t e = local * kThreads + threadIdx.x;
      if (e < (int64_t(1) << h) + (int64_t(1) << (n - h)))
        twiddle_entry(reinterpret_cast<double2*>(D.ws + L.tw_hi), reinterpret_cast<double2*>(D.ws + L.tw_lo), n, h,
                      e);
      break;
    }
    case BK_SUBI: {
      int64_t e0 = local * kSubiTile, e1 = min(e0 + int64_t(kSubiTile), int64_t(d) * d);
      subi_range(reinterpret_cast<double2*>(D.ws + L.gbuf),
                 gram_split(t) ? reinterpret_cast<const double2*>(D.ws + L.gbuf2) : nullptr, d, e0 + threadIdx.x,
                 e1, kThreads, defect);
      break;
    }
    case BK_NSPREP:
    case BK_NSUPD: {
      // X = vbuf, E (then XE) = gbuf, X32 (then V_k) = tbuf
      const double2* X = reinterpret_cast<const double2*>(D.ws + L.vbuf);
      int64_t e0 = local * kSplitTile, e1 = min(e0 + int64_t(kSplitTile), int64_t(d) * d);
      if (kind == BK_NSPREP) {
        const double2* E = reinterpret_cast<const double2*>(D.ws + L.gbuf);
        float2* x32 = reinterpret_cast<float2*>(D.ws + L.tbuf);
        uint16_t* planes = reinterpret_cast<uint16_t*>(D.ws + L.planes);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) ns_prep_entry(X, E, x32, planes, t, e);
      } else {
        const float2* xe = reinterpret_cast<const float2*>(D.ws + L.gbuf);
        double2* out = reinterpret_cast<double2*>(D.ws + L.tbuf);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) ns_update_entry(X, xe, out, e);
      }
      break;
    }
    case BK_PCOPY: {
      const double2* X = reinterpret_cast<const double2*>(D.ws + L.vbuf);
      double2* out = reinterpret_cast<double2*>(D.ws + L.tbuf);
      int64_t e0 = local * kSplitTile, e1 = min(e0 + int64_t(kSplitTile), int64_t(d) * d);
      for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) out[e] = X[e];
      break;
    }
    case BK_SPLIT: {
      const double2* V = power_ptr(D, L, power_slot(step, polar));
      uint16_t* planes = reinterpret_cast<uint16_t*>(D.ws + L.planes);
      const bool f16 = (bflags & kBatchF16) != 0;
      int64_t e0 = local * kSplitTile, e1 = min(e0 + int64_t(kSplitTile), int64_t(d) * d);
      if (f16) {
        // four consecutive elements per thread (d >= 32)
        for (int64_t e = e0 + 4 * threadIdx.x; e < e1; e += 4 * kThreads) {
          double2 v[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = V[e + i];
          split4_f16(v, planes, t, e);
        }
      } else {
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) split_entry(V, planes, t, e, false, false);
      }
      break;
    }
    case BK_SCALE:
      state_scale_block(D.psi, n, t, reinterpret_cast<float*>(defect + kScratchSigma));
      break;
    case BK_PROB: {
      const DftPlan plan = make_dft_plan(n);
      if (fused_readout(n)) {
        // the partials of the fused last pass, in the second state buffer
        const double* part = reinterpret_cast<const double*>(D.ws + L.state1);
        const int groups = readout_groups(mixed, n, t);
        for (int r = 0; r < kProbRounds; ++r) {
          const int64_t p = (local * kProbRounds + r) * kThreads + threadIdx.x;
          if (p < (int64_t(1) << n)) finish_row(part, D.prob, n, groups, plan, ldexp(1.0, -n), p);
        }
        break;
      }
      const int G = d < 64 ? d : 64;
      const int rows_per_wave = 64 / G;
      for (int r = 0; r < kProbRounds; ++r) {
        const int64_t base = ((local * kProbRounds + r) * 4 + (threadIdx.x >> 6)) * rows_per_wave;
        prob_rows<T>(reinterpret_cast<const T*>(D.ws + L.state0), D.prob, n, t, plan, ldexp(1.0, -n), base);
      }
      break;
    }
    case BK_REPORT:
      if (D.report) {
        const bool rot = rotate_on(mixed, t, batch_rot_mode(bflags), polar);
        report_block(D.prob, n, D.psi_src, t, polar ? defect : nullptr,
                     rot ? reinterpret_cast<const double*>(defect + kScratchPeak) : nullptr, mixed && t >= 5,
                     D.report);
      }
      break;
  }
}

}  // namespace

hipError_t launch_h_broadcast(bool mixed, const void* psi, void* state, int n, int t, hipStream_t s,
                              bool first_row_only) {
  // first_row_only: write row 0 only (the prefix-doubling form), still
  // scaled by 2^(-n/2).
  const int64_t total = int64_t(1) << (first_row_only ? t : n + t);
  if (mixed && total == 1) {
    // a single complex64 amplitude cannot use the float4 pair writes
    hipLaunchKernelGGL(k_h_single_c64, dim3(1), dim3(64), 0, s, static_cast<const double2*>(psi),
                       static_cast<float2*>(state), std::ldexp(1.0, -(n / 2)) * ((n & 1) ? std::sqrt(0.5) : 1.0));
    return hipGetLastError();
  }
  const double scale = std::ldexp(1.0, -(n / 2)) * ((n & 1) ? std::sqrt(0.5) : 1.0);
  if (mixed) {
    // total >= 2 because n >= 1
    int64_t pairs = total / 2;
    hipLaunchKernelGGL(k_h_broadcast_c64, dim3(grid_for(pairs)), dim3(kThreads), 0, s,
                       static_cast<const double2*>(psi), static_cast<float4*>(state), pairs, (1 << t) - 1, scale);
  } else {
    hipLaunchKernelGGL(k_h_broadcast_c128, dim3(grid_for(total)), dim3(kThreads), 0, s,
                       static_cast<const double2*>(psi), static_cast<double2*>(state), total, (1 << t) - 1, scale);
  }
  return hipGetLastError();
}

hipError_t launch_gather_state(bool mixed, const void* X, void* out, int n, int t, const DftPlan& plan, double scale,
                               hipStream_t s) {
  const int64_t total = int64_t(1) << (n + t);
  if (mixed)
    hipLaunchKernelGGL(k_gather_state<float2>, dim3(grid_for(total)), dim3(kThreads), 0, s,
                       static_cast<const float2*>(X), static_cast<float2*>(out), n, t, plan, scale);
  else
    hipLaunchKernelGGL(k_gather_state<double2>, dim3(grid_for(total)), dim3(kThreads), 0, s,
                       static_cast<const double2*>(X), static_cast<double2*>(out), n, t, plan, scale);
  return hipGetLastError();
}

hipError_t launch_twiddles(double2* tw_hi, double2* tw_lo, int n, int h, hipStream_t s) {
  int64_t work = (int64_t(1) << h) + (int64_t(1) << (n - h));
  hipLaunchKernelGGL(k_twiddles, dim3(grid_for(work)), dim3(kThreads), 0, s, tw_hi, tw_lo, n, h);
  return hipGetLastError();
}

hipError_t launch_ns_prep_fused(const double2* X, const double2* G, const double2* G2, float2* X32, uint16_t* planes,
                                int t, unsigned long long* defect_bits, hipStream_t s) {
  int64_t dd = int64_t(1) << (2 * t);
  hipLaunchKernelGGL(k_ns_prep_fused, dim3(grid_for(dd, kThreads, 512)), dim3(kThreads), 0, s, X, G, G2, X32, planes,
                     t, defect_bits);
  return hipGetLastError();
}

hipError_t launch_ns_update_split(const double2* X, const float2* XE, double2* out, uint16_t* planes, int t,
                                  hipStream_t s, bool f16) {
  int64_t dd = int64_t(1) << (2 * t);
  if (f16)
    hipLaunchKernelGGL(k_ns_update_split<true>, dim3(grid_for(dd / 4)), dim3(kThreads), 0, s, X, XE, out, planes, t);
  else
    hipLaunchKernelGGL(k_ns_update_split<false>, dim3(grid_for(dd)), dim3(kThreads), 0, s, X, XE, out, planes, t);
  return hipGetLastError();
}

hipError_t launch_split_pieces(const double2* V, uint16_t* planes, int t, hipStream_t s, bool f16) {
  int64_t dd = int64_t(1) << (2 * t);
  if (f16)
    hipLaunchKernelGGL(k_split_pieces<true>, dim3(grid_for(dd / 4)), dim3(kThreads), 0, s, V, planes, t);
  else
    hipLaunchKernelGGL(k_split_pieces<false>, dim3(grid_for(dd)), dim3(kThreads), 0, s, V, planes, t);
  return hipGetLastError();
}

hipError_t launch_state_scale(const double2* psi, int n, int t, float* sigma, hipStream_t s) {
  hipLaunchKernelGGL(k_state_scale, dim3(1), dim3(kThreads), 0, s, psi, n, t, sigma);
  return hipGetLastError();
}

hipError_t launch_sub_identity_defect(double2* G, const double2* G2, int d, unsigned long long* defect_bits,
                                      hipStream_t s) {
  int64_t dd = int64_t(d) * d;
  hipLaunchKernelGGL(k_sub_identity_defect, dim3(grid_for(dd, kThreads, 1024)), dim3(kThreads), 0, s, G, G2, d,
                     defect_bits);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_prob(bool mixed, const void* state, double* prob, int n, int t, const DftPlan& plan,
                       hipStream_t s) {
  const int64_t N = int64_t(1) << n;
  const int d = 1 << t;
  const int G = d < 64 ? d : 64;
  int64_t waves = (N * G + 63) / 64;
  int grid = grid_for(waves * 64);
  const double scale = std::ldexp(1.0, -n);
  if (mixed)
    hipLaunchKernelGGL(k_prob<float2>, dim3(grid), dim3(kThreads), 0, s, static_cast<const float2*>(state), prob, n,
                       t, plan, scale);
  else
    hipLaunchKernelGGL(k_prob<double2>, dim3(grid), dim3(kThreads), 0, s, static_cast<const double2*>(state), prob,
                       n, t, plan, scale);
  return hipGetLastError();
}

hipError_t launch_prob_finish(const double* part, double* prob, int n, int groups, const DftPlan& plan,
                              hipStream_t s) {
  const int grid = grid_for(int64_t(1) << n);
  hipLaunchKernelGGL(k_prob_finish, dim3(grid), dim3(kThreads), 0, s, part, prob, n, groups, plan,
                     std::ldexp(1.0, -n));
  return hipGetLastError();
}

hipError_t launch_report(const double* prob, int n, const double2* psi, int t, const unsigned long long* defect_bits,
                         const double* rot_peak, bool check, void* report, double* part, hipStream_t s) {
  const int64_t N = int64_t(1) << n;
  int nparts = 0;
  if (part && N >= 4 * kReportChunk) {
    nparts = int(N / kReportChunk);
    hipLaunchKernelGGL(k_report_partial, dim3(nparts), dim3(kThreads), 0, s, prob, part);
  }
  hipLaunchKernelGGL(k_report, dim3(1), dim3(kThreads), 0, s, prob, n, psi, t, defect_bits, rot_peak,
                     check ? 1 : 0, static_cast<double*>(report), nparts ? part : nullptr, nparts);
  return hipGetLastError();
}

hipError_t launch_copy_rows_back(bool mixed, void* state, const void* other, int n, int t, int k, hipStream_t s) {
  int64_t half = (int64_t(1) << (n - 1)) << t;
  if (mixed)
    hipLaunchKernelGGL(k_copy_rows_back<float2>, dim3(grid_for(half)), dim3(kThreads), 0, s,
                       static_cast<float2*>(state), static_cast<const float2*>(other), n, t, k);
  else
    hipLaunchKernelGGL(k_copy_rows_back<double2>, dim3(grid_for(half)), dim3(kThreads), 0, s,
                       static_cast<double2*>(state), static_cast<const double2*>(other), n, t, k);
  return hipGetLastError();
}

hipError_t launch_batch_descs(InstDesc* desc, char* ws, const BatchProblem* probs, int first, int count,
                              hipStream_t s) {
  DescArgs a{};
  a.first = first;
  a.count = count;
  for (int i = 0; i < count; ++i) a.p[i] = probs[i];
  hipLaunchKernelGGL(k_batch_descs, dim3(1), dim3(64), 0, s, desc, ws, a);
  return hipGetLastError();
}

hipError_t launch_batch_tables(const InstDesc* desc, int ninst, int32_t* tables, const BatchLaunch* launches,
                               int nlaunch, bool mixed, int bflags, hipStream_t s) {
  TableArgs a{};
  a.nlaunch = nlaunch;
  for (int i = 0; i < nlaunch; ++i) a.l[i] = launches[i];
  hipLaunchKernelGGL(k_batch_tables, dim3(nlaunch), dim3(kTableThreads), 0, s, desc, ninst, tables, a, mixed ? 1 : 0,
                     bflags);
  return hipGetLastError();
}

hipError_t launch_batch_elementwise(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                                    bool mixed, int bflags, hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    if (mixed)
      hipLaunchKernelGGL(kb_elementwise<float2>, dim3(g), dim3(kThreads), 0, s, kind, step, desc, table, bflags, b);
    else
      hipLaunchKernelGGL(kb_elementwise<double2>, dim3(g), dim3(kThreads), 0, s, kind, step, desc, table, bflags, b);
  });
}

}  // namespace qpe
