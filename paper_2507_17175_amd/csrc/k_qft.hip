// Inverse QFT on the measurement register (Fig. 1, QFT^-1): for every target
// column r, the unitary inverse DFT of length N = 2^n along the row index,
//   A[m] = 2^(-n/2) sum_j exp(-2 pi i j m / N) S[j]
// The passes compute the sum without the 2^(-n/2); the readout applies the
// exact power of two 2^-n to |A|^2 instead.
//
// Decomposition: a sequence of radix-R passes (R = 2^b, b <= 8). Pass q acts
// on blocks of B = N >> (bits before q) consecutive rows; inside a block, row
// j = j1 * M + j2 (M = B / R) and for each (j2, column) the R-point DFT over
// j1 is taken, multiplied by the twiddle exp(-2 pi i j2 m1 / B) and written
// back in place to row m1 * M + j2. After all passes, row p holds outcome
// m = digit_reverse(p) (the readout kernel undoes it). The R-point DFT itself
// is split R = R1 x R2: an R1-point DFT in registers, a twiddle, an exchange
// through LDS, and an R2-point DFT in registers. Threads own consecutive
// (j2, column) elements, so every global access is a contiguous run.
//
// Twiddles exp(-2 pi i x / N) come from two small FP64 tables indexed by
// the exact integer x (x = hi * 2^h + lo), multiplied in FP64.
//
// Fused readout (fused_readout(n): two passes or more, the last of 6-8
// bits): the last pass does not store the transformed state (unless asked
// to keep it) but forms |A|^2 of its outputs in FP64 and sums them over the
// columns a workgroup holds, C = min(d, E) per row, with a fixed tree of
// lane exchanges; it writes one partial per (column group, row) to
// part[cg * N + p], and the readout sums the d / C partials of each row in
// column-group order. This saves the readout's read of the state and the
// last pass's write of it.
#include "qpe_internal.hpp"

namespace qpe {

namespace {

constexpr int kThreads = 256;

template <typename T> struct Real;
template <> struct Real<float2> { typedef float type; };
template <> struct Real<double2> { typedef double type; };

// cos and sin of pi k / 8, k = 0..7: omega_16^k = c16(k) - i s16(k).
__host__ __device__ constexpr double c16(int k) {
  return k == 0 ? 1.0 : k == 1 ? 0.92387953251128675613 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.38268343236508977173 : k == 4 ? 0.0 : k == 5 ? -0.38268343236508977173
       : k == 6 ? -0.70710678118654752440 : -0.92387953251128675613;
}
__host__ __device__ constexpr double s16(int k) {
  return k == 0 ? 0.0 : k == 1 ? 0.38268343236508977173 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.92387953251128675613 : k == 4 ? 1.0 : k == 5 ? 0.92387953251128675613
       : k == 6 ? 0.70710678118654752440 : 0.38268343236508977173;
}

__host__ __device__ constexpr int brev(int m, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((m >> i) & 1) << (bits - 1 - i);
  return r;
}

template <int P> struct Log2 { static constexpr int v = 1 + Log2<P / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

// In-register radix-2 decimation-in-frequency DFT of P <= 16 points
// (forward sign). On return re/im[brev(m)] holds output m.
template <typename R, int P>
__device__ __forceinline__ void dft_regs(R* re, R* im) {
#pragma unroll
  for (int s = P / 2; s >= 1; s >>= 1) {
#pragma unroll
    for (int st = 0; st < P; st += 2 * s) {
#pragma unroll
      for (int i = 0; i < s; ++i) {
        R ar = re[st + i], ai = im[st + i], br = re[st + i + s], bi = im[st + i + s];
        re[st + i] = ar + br;
        im[st + i] = ai + bi;
        R dr = ar - br, di = ai - bi;
        const int kw = i * (8 / s);  // omega_{2s}^i = omega_16^{8 i / s}
        if (kw == 0) {
          re[st + i + s] = dr;
          im[st + i + s] = di;
        } else if (kw == 4) {
          re[st + i + s] = di;
          im[st + i + s] = -dr;
        } else {
          // rotated in FP64 with FP64 constants and rounded once: FP32
          // constants miss c^2 + s^2 = 1 by 1e-8 to 6e-8, the same way for
          // every element through this butterfly
          const double c = c16(kw), sn = s16(kw), xr = double(dr), xi = double(di);
          re[st + i + s] = R(xr * c + xi * sn);
          im[st + i + s] = R(xi * c - xr * sn);
        }
      }
    }
  }
}

// exp(-2 pi i x / N), x in [0, N), as (cos, sin) in FP64.
__device__ __forceinline__ double2 twiddle(int64_t x, const double2* __restrict__ tw_hi,
                                           const double2* __restrict__ tw_lo, int h) {
  double2 a = tw_hi[x >> h], b = tw_lo[x & ((int64_t(1) << h) - 1)];
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// y * w for an element held in the state's precision, in FP64.
template <typename T, typename R>
__device__ __forceinline__ T twiddled(R yr, R yi, double2 w) {
  T o;
  o.x = R(double(yr) * w.x - double(yi) * w.y);
  o.y = R(double(yr) * w.y + double(yi) * w.x);
  return o;
}

// Sums of v[0..R) over each aligned group of C consecutive lanes (C a power
// of two, 1 <= C <= 64, the same in the whole wave) by recursive halving:
// at lane offset o = C/2, C/4, ..., while a lane holds more than one value,
// the lane with bit o set keeps the upper half of its values and sends the
// lower half to its partner, which keeps the lower half, and each adds what
// it received; once a single value is left, the remaining offsets are plain
// exchange-and-add steps. On return the lane holds the group's sums for
// j = first .. first + cnt - 1 in v[0..cnt); `owner` marks one lane per
// distinct set of sums. The tree is fixed, so the sums are reproducible.
template <int R>
__device__ __forceinline__ void group_sums(double (&v)[R], int C, int lane, int& first, int& cnt, bool& owner) {
  first = 0;
  cnt = R;
  int o = C >> 1;
#pragma unroll
  for (int h = R; h > 1; h >>= 1) {
    if (o >= 1) {  // (uniform; no early exit, so the loop unrolls)
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < h / 2; ++i) {
        const double keep = up ? v[h / 2 + i] : v[i];
        const double send = up ? v[i] : v[h / 2 + i];
        v[i] = keep + __shfl_xor(send, o);
      }
      if (up) first += h / 2;
      cnt = h / 2;
      o >>= 1;
    }
  }
  const int rest = o;  // offsets left for the single value
  for (; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o);
  owner = rest == 0 || (lane & (2 * rest - 1)) == 0;
}

// Largest LDS exchange buffer of a pass with one DFT row per thread
// (R1 = R2 = 16): 16 x 16 x 16 points.
constexpr int kQftLds = 4096;

// DFT rows per thread of a radix-256 pass (qft_two_rows): two for complex64
// passes of 32 elements or more, so that a workgroup covers 32 elements
// (256-byte row runs; 14 % faster at 2^26 amplitudes); one for complex128,
// where it did not pay.

// Workgroup `block` of one pass; L: LDS scratch of R1 R2 E points. EM > 1
// (R2 > 1 only): each thread takes EM of the R2 DFT rows of phase A, so a
// workgroup covers E = EM kThreads / R2 consecutive elements and each row
// access is EM times longer.
// FUSE: the last pass with the fused readout (part: the partials; keep: also
// store the transformed state).
template <typename T, int R1, int R2, int EM = 1, bool FUSE = false>
__device__ __forceinline__ void qft_tile(T* __restrict__ buf0, const T* __restrict__ buf1, int gather, int n, int t,
                                         int pass_bits, int bits_before, const double2* __restrict__ tw_hi,
                                         const double2* __restrict__ tw_lo, int h, int64_t block,
                                         T* __restrict__ L, double* __restrict__ part = nullptr,
                                         bool keep = true) {
  typedef typename Real<T>::type R;
  static_assert(EM == 1 || R2 > 1, "the in-register pass takes one element per thread");
  constexpr int E = EM * kThreads / R2;  // elements per workgroup
  static_assert(!FUSE || (R2 > 1 && E <= 64 && (E * R1) % kThreads == 0),
                "fused readout: column groups within a wave, every lane in every round");
  // the grouped kernel's buffer holds EM kQftLds points
  static_assert(R1 * R2 * E <= EM * kQftLds, "LDS exchange buffer");
  constexpr int L1 = Log2<R1>::v, L2 = Log2<R2>::v;

  const int bq_log = n - bits_before;        // rows per block (log2)
  const int m_log = bq_log - pass_bits;      // rows between DFT points (log2)
  const int64_t md = int64_t(1) << (m_log + t);
  const int64_t total_e = int64_t(1) << (n + t - pass_bits);
  const int64_t f0 = block * E;
  const int tid = threadIdx.x;

  auto element = [&](int e, int64_t& base, int64_t& j2) {
    int64_t f = f0 + e;
    int64_t blk = f >> (m_log + t), rem = f & (md - 1);
    j2 = rem >> t;
    base = (blk << (bq_log + t)) + rem;
  };

  // Phase A: R1-point DFTs over j1a (j1 = j1a * R2 + j1b).
  {
    const int e = tid % E;
    const bool ok = f0 + e < total_e;
    int64_t base = 0, j2 = 0;
    if (ok) element(e, base, j2);
    R re[EM][R1], im[EM][R1];
#pragma unroll
    for (int r = 0; r < EM; ++r) {
      const int j1b = tid / E + r * (R2 / EM);
#pragma unroll
      for (int a = 0; a < R1; ++a) {
        int64_t idx = base + int64_t(a * R2 + j1b) * md;
        T v;
        v.x = R(0);
        v.y = R(0);
        if (ok) {
          const T* src = (gather && (__builtin_popcountll(uint64_t(idx >> t)) & 1)) ? buf1 : buf0;
          v = src[idx];
        }
        re[r][a] = v.x;
        im[r][a] = v.y;
      }
    }
#pragma unroll
    for (int r = 0; r < EM; ++r) {
      const int j1b = tid / E + r * (R2 / EM);
      dft_regs<R, R1>(re[r], im[r]);
      // The twiddles of consecutive m1 are successive powers of one table
      // value (exp(-2 pi i (j2 2^bits_before) m1 / N) = w1^m1), formed by FP64
      // products: one table lookup per thread instead of one per output.
      if (R2 == 1) {
        if (ok) {
          const double2 w1 = twiddle(j2 << bits_before, tw_hi, tw_lo, h);
          double2 w = make_double2(1.0, 0.0);
#pragma unroll
          for (int m1 = 0; m1 < R1; ++m1) {
            R yr = re[r][brev(m1, L1)], yi = im[r][brev(m1, L1)];
            T o;
            if (m1 == 0) {
              o.x = yr;
              o.y = yi;
            } else {
              w = m1 == 1 ? w1 : cmul(w, w1);
              o = twiddled<T, R>(yr, yi, w);
            }
            buf0[base + int64_t(m1) * md] = o;
          }
        }
      } else {
        const double2 w1 = twiddle(int64_t(j1b) << (n - pass_bits), tw_hi, tw_lo, h);
        double2 w = make_double2(1.0, 0.0);
#pragma unroll
        for (int m1a = 0; m1a < R1; ++m1a) {
          R yr = re[r][brev(m1a, L1)], yi = im[r][brev(m1a, L1)];
          T o;
          if (m1a == 0 || j1b == 0) {
            o.x = yr;
            o.y = yi;
          } else {
            w = m1a == 1 ? w1 : cmul(w, w1);
            o = twiddled<T, R>(yr, yi, w);
          }
          L[(m1a * R2 + j1b) * E + e] = o;
        }
      }
    }
  }
  if (R2 == 1) return;
  __syncthreads();

  // Phase B: R2-point DFTs over j1b, outer twiddle, store (or, fused, the
  // column sums of |A|^2).
  const int d = 1 << t;
  const int C = d < E ? d : E;  // lanes (columns) that share a row
  for (int u = tid; u < E * R1; u += kThreads) {
    const int e = u % E, m1a = u / E;
    const bool ok = f0 + e < total_e;
    if (!FUSE && !ok) continue;  // (fused: every lane takes part in the sums)
    int64_t base = 0, j2 = 0;
    if (ok) element(e, base, j2);
    R re[R2], im[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) {
      T v = L[(m1a * R2 + b) * E + e];
      re[b] = v.x;
      im[b] = v.y;
    }
    dft_regs<R, R2>(re, im);
    // twiddle of m1 = m1a + R1 m1b: exp(-2 pi i j2 m1 2^bits_before / N)
    // = w0 * ws^m1b with w0 for m1a and ws for the step R1
    const double2 w0 = twiddle((j2 * m1a) << bits_before, tw_hi, tw_lo, h);
    const double2 ws = twiddle((j2 * R1) << bits_before, tw_hi, tw_lo, h);
    double2 w = w0;
    double sq[R2];
#pragma unroll
    for (int m1b = 0; m1b < R2; ++m1b) {
      const int m1 = m1a + R1 * m1b;
      R yr = re[brev(m1b, L2)], yi = im[brev(m1b, L2)];
      if (m1b > 0) w = cmul(w, ws);
      T o;
      if (j2 == 0 || m1 == 0) {
        o.x = yr;
        o.y = yi;
      } else {
        o = twiddled<T, R>(yr, yi, w);
      }
      if (!FUSE || keep) {
        if (ok) buf0[base + int64_t(m1) * md] = o;
      }
      if (FUSE) {
        const double xr = double(o.x), xi = double(o.y);
        sq[m1b] = ok ? xr * xr + xi * xi : 0.0;
      }
    }
    if constexpr (FUSE) {
      int first, cnt;
      bool owner;
      group_sums<R2>(sq, C, tid & 63, first, cnt, owner);
      // row of output m1: (base >> t) + m1 2^m_log; column group col / C
      const int64_t N = int64_t(1) << n;
      const int64_t cg = (base & (d - 1)) / C;
#pragma unroll
      for (int j = 0; j < R2; ++j)
        if (owner && ok && j < cnt) {
          const int m1 = m1a + R1 * (first + j);
          part[cg * N + (base >> t) + (int64_t(m1) << m_log)] = sq[j];
        }
    }
  }
}

template <typename T, int R1, int R2, int EM>
__global__ void __launch_bounds__(kThreads) k_qft_pass(T* __restrict__ buf0, const T* __restrict__ buf1, int gather,
                                                       int n, int t, int pass_bits, int bits_before,
                                                       const double2* __restrict__ tw_hi,
                                                       const double2* __restrict__ tw_lo, int h) {
  __shared__ T L[R2 > 1 ? R1 * R2 * (EM * kThreads / R2) : 1];
  qft_tile<T, R1, R2, EM>(buf0, buf1, gather, n, t, pass_bits, bits_before, tw_hi, tw_lo, h, blockIdx.x, L);
}

// The last pass with the fused readout (no gather: a last pass of two or
// more reads only buf0).
template <typename T, int R1, int R2, int EM>
__global__ void __launch_bounds__(kThreads) k_qft_last_fused(T* __restrict__ buf0, int n, int t, int pass_bits,
                                                             int bits_before, const double2* __restrict__ tw_hi,
                                                             const double2* __restrict__ tw_lo, int h,
                                                             double* __restrict__ part, int keep) {
  __shared__ T L[R1 * R2 * (EM * kThreads / R2)];
  qft_tile<T, R1, R2, EM, true>(buf0, nullptr, 0, n, t, pass_bits, bits_before, tw_hi, tw_lo, h, blockIdx.x, L, part,
                                keep != 0);
}

// Grouped pass `pass` over the instances of a launch table: each instance
// runs its own schedule (make_dft_plan of its n), so the radix is chosen
// per workgroup.
// WIDE: some instance of the launch takes two rows per thread in this pass
// (the LDS buffer then holds twice the points).
template <typename T, bool WIDE>
__global__ void __launch_bounds__(kThreads) kb_qft(int pass, const InstDesc* __restrict__ desc,
                                                   const int32_t* __restrict__ table, int bflags, int64_t tile0) {
  constexpr bool mixed = sizeof(T) == 8;
  __shared__ T L[WIDE ? 2 * kQftLds : kQftLds];
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const RunLayout lay = run_layout(D.n, D.t, mixed, (bflags & kBatchPolar) != 0);
  const DftPlan plan = make_dft_plan(D.n);
  int before = 0;
  for (int q = 0; q < pass; ++q) before += plan.bits[q];
  T* b0 = reinterpret_cast<T*>(D.ws + lay.state0);
  const T* b1 = reinterpret_cast<const T*>(D.ws + lay.state1);
  const double2* hi = reinterpret_cast<const double2*>(D.ws + lay.tw_hi);
  const double2* lo = reinterpret_cast<const double2*>(D.ws + lay.tw_lo);
  // the gate route's state sits in two buffers after the controlled steps
  const int g = (pass == 0 && !(bflags & kBatchDoubling)) ? 1 : 0;
  const int h = tw_split(D.n), n = D.n, t = D.t;
  switch (plan.bits[pass]) {
    case 1: qft_tile<T, 2, 1>(b0, b1, g, n, t, 1, before, hi, lo, h, local, L); break;
    case 2: qft_tile<T, 4, 1>(b0, b1, g, n, t, 2, before, hi, lo, h, local, L); break;
    case 3: qft_tile<T, 8, 1>(b0, b1, g, n, t, 3, before, hi, lo, h, local, L); break;
    case 4: qft_tile<T, 16, 1>(b0, b1, g, n, t, 4, before, hi, lo, h, local, L); break;
    case 5: qft_tile<T, 16, 2>(b0, b1, g, n, t, 5, before, hi, lo, h, local, L); break;
    case 6: qft_tile<T, 16, 4>(b0, b1, g, n, t, 6, before, hi, lo, h, local, L); break;
    case 7: qft_tile<T, 16, 8>(b0, b1, g, n, t, 7, before, hi, lo, h, local, L); break;
    case 8:
      if (WIDE && qft_two_rows(mixed, 8, n, t))
        qft_tile<T, 16, 16, 2>(b0, b1, g, n, t, 8, before, hi, lo, h, local, L);
      else
        qft_tile<T, 16, 16, 1>(b0, b1, g, n, t, 8, before, hi, lo, h, local, L);
      break;
  }
}

// The fused last pass of the instances whose pass `pass` is their last
// (launch kind BK_QFT_LAST): partials in the instance's second state buffer,
// which no pass after the first reads.
template <typename T, bool WIDE>
__global__ void __launch_bounds__(kThreads) kb_qft_last(int pass, const InstDesc* __restrict__ desc,
                                                        const int32_t* __restrict__ table, int bflags,
                                                        int64_t tile0) {
  constexpr bool mixed = sizeof(T) == 8;
  __shared__ T L[WIDE ? 2 * kQftLds : kQftLds];
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const RunLayout lay = run_layout(D.n, D.t, mixed, (bflags & kBatchPolar) != 0);
  const DftPlan plan = make_dft_plan(D.n);
  int before = 0;
  for (int q = 0; q < pass; ++q) before += plan.bits[q];
  T* b0 = reinterpret_cast<T*>(D.ws + lay.state0);
  double* part = reinterpret_cast<double*>(D.ws + lay.state1);
  const double2* hi = reinterpret_cast<const double2*>(D.ws + lay.tw_hi);
  const double2* lo = reinterpret_cast<const double2*>(D.ws + lay.tw_lo);
  const int h = tw_split(D.n), n = D.n, t = D.t;
  switch (plan.bits[pass]) {
    case 6: qft_tile<T, 16, 4, 1, true>(b0, nullptr, 0, n, t, 6, before, hi, lo, h, local, L, part, false); break;
    case 7: qft_tile<T, 16, 8, 1, true>(b0, nullptr, 0, n, t, 7, before, hi, lo, h, local, L, part, false); break;
    case 8:
      if (WIDE && qft_two_rows(mixed, 8, n, t))
        qft_tile<T, 16, 16, 2, true>(b0, nullptr, 0, n, t, 8, before, hi, lo, h, local, L, part, false);
      else
        qft_tile<T, 16, 16, 1, true>(b0, nullptr, 0, n, t, 8, before, hi, lo, h, local, L, part, false);
      break;
  }
}

template <typename T, int R1, int R2, int EM = 1>
hipError_t go(void* b0, const void* b1, bool gather, int n, int t, int pb, int bb, const double2* hi,
              const double2* lo, int h, hipStream_t s) {
  constexpr int E = EM * kThreads / R2;
  int64_t total_e = int64_t(1) << (n + t - pb);
  int64_t grid = (total_e + E - 1) / E;
  hipLaunchKernelGGL((k_qft_pass<T, R1, R2, EM>), dim3(unsigned(grid)), dim3(kThreads), 0, s, static_cast<T*>(b0),
                     static_cast<const T*>(b1), gather ? 1 : 0, n, t, pb, bb, hi, lo, h);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch(void* b0, const void* b1, bool gather, int n, int t, int pb, int bb, const double2* hi,
                    const double2* lo, int h, hipStream_t s) {
  switch (pb) {
    case 1: return go<T, 2, 1>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
    case 2: return go<T, 4, 1>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
    case 3: return go<T, 8, 1>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
    case 4: return go<T, 16, 1>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
    case 5: return go<T, 16, 2>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
    case 6: return go<T, 16, 4>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
    case 7: return go<T, 16, 8>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
    case 8:
      if (qft_two_rows(sizeof(T) == 8, 8, n, t)) return go<T, 16, 16, 2>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
      return go<T, 16, 16, 1>(b0, b1, gather, n, t, pb, bb, hi, lo, h, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int R1, int R2, int EM = 1>
hipError_t go_fused(void* b0, int n, int t, int pb, int bb, const double2* hi, const double2* lo, int h, double* part,
                    bool keep, hipStream_t s) {
  constexpr int E = EM * kThreads / R2;
  int64_t total_e = int64_t(1) << (n + t - pb);
  int64_t grid = (total_e + E - 1) / E;
  hipLaunchKernelGGL((k_qft_last_fused<T, R1, R2, EM>), dim3(unsigned(grid)), dim3(kThreads), 0, s,
                     static_cast<T*>(b0), n, t, pb, bb, hi, lo, h, part, keep ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_fused(void* b0, int n, int t, int pb, int bb, const double2* hi, const double2* lo, int h,
                          double* part, bool keep, hipStream_t s) {
  switch (pb) {
    case 6: return go_fused<T, 16, 4>(b0, n, t, pb, bb, hi, lo, h, part, keep, s);
    case 7: return go_fused<T, 16, 8>(b0, n, t, pb, bb, hi, lo, h, part, keep, s);
    case 8:
      if (qft_two_rows(sizeof(T) == 8, 8, n, t)) return go_fused<T, 16, 16, 2>(b0, n, t, pb, bb, hi, lo, h, part, keep, s);
      return go_fused<T, 16, 16, 1>(b0, n, t, pb, bb, hi, lo, h, part, keep, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_qft_last_fused(bool mixed, void* buf0, int n, int t, int pass_bits, int bits_before,
                                 const double2* tw_hi, const double2* tw_lo, int h, double* part, bool keep,
                                 hipStream_t s) {
  return mixed ? dispatch_fused<float2>(buf0, n, t, pass_bits, bits_before, tw_hi, tw_lo, h, part, keep, s)
               : dispatch_fused<double2>(buf0, n, t, pass_bits, bits_before, tw_hi, tw_lo, h, part, keep, s);
}

hipError_t launch_batch_qft(int pass, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                            bool wide, int bflags, hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    if (mixed && wide)
      hipLaunchKernelGGL((kb_qft<float2, true>), dim3(g), dim3(kThreads), 0, s, pass, desc, table, bflags, b);
    else if (mixed)
      hipLaunchKernelGGL((kb_qft<float2, false>), dim3(g), dim3(kThreads), 0, s, pass, desc, table, bflags, b);
    else
      hipLaunchKernelGGL((kb_qft<double2, false>), dim3(g), dim3(kThreads), 0, s, pass, desc, table, bflags, b);
  });
}

hipError_t launch_batch_qft_last(int pass, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                                 bool wide, int bflags, hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    if (mixed && wide)
      hipLaunchKernelGGL((kb_qft_last<float2, true>), dim3(g), dim3(kThreads), 0, s, pass, desc, table, bflags, b);
    else if (mixed)
      hipLaunchKernelGGL((kb_qft_last<float2, false>), dim3(g), dim3(kThreads), 0, s, pass, desc, table, bflags, b);
    else
      hipLaunchKernelGGL((kb_qft_last<double2, false>), dim3(g), dim3(kThreads), 0, s, pass, desc, table, bflags, b);
  });
}

hipError_t launch_qft_pass(bool mixed, void* buf0, const void* buf1, bool gather, int n, int t, int pass_bits,
                           int bits_before, const double2* tw_hi, const double2* tw_lo, int h, hipStream_t s) {
  return mixed ? dispatch<float2>(buf0, buf1, gather, n, t, pass_bits, bits_before, tw_hi, tw_lo, h, s)
               : dispatch<double2>(buf0, buf1, gather, n, t, pass_bits, bits_before, tw_hi, tw_lo, h, s);
}

}  // namespace qpe
