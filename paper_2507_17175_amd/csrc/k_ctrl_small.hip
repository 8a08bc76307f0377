// Controlled step (Fig. 1, controlled U^(2^k)) for target registers of at
// most 4 qubits (d <= 16). A d x d operator is too small to fill a matrix
// core tile, and the step is bound by HBM traffic, so each thread owns one
// gathered state row: it forms s <- V s with the operator broadcast from
// LDS. A workgroup moves its 256 rows between HBM and LDS with consecutive
// lanes on consecutive amplitudes (a thread reading its own row straight
// from HBM would touch a different cache line per lane), and the result goes
// to the other ping-pong buffer the same way. FP64 form: complex128 state,
// FP64 arithmetic. Mixed form: complex64 state, the operator rounded once to
// FP32, FP32 FMAs.
#include "qpe_internal.hpp"

namespace qpe {

namespace {

constexpr int kThreads = 256;

template <typename T> struct Real;
template <> struct Real<float2> { typedef float type; };
template <> struct Real<double2> { typedef double type; };

// The D amplitudes a thread moves of the gathered rows [i0, i0 + kThreads)
// of step k: element e = tid + q kThreads (row e / D, amplitude e % D), so
// that consecutive lanes read consecutive amplitudes.
template <typename T, int D>
__device__ __forceinline__ void load_tile_regs(const T* __restrict__ buf0, const T* __restrict__ buf1, int k,
                                               uint64_t pmask, int64_t i0, int64_t M, T (&r)[D]) {
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const int e = threadIdx.x + q * kThreads, row = e / D, c = e % D;
    const int64_t i = i0 + row;
    if (i < M) {
      const int64_t j = step_row(i, k, pmask);
      r[q] = ((src_buffer(j, pmask) ? buf1 : buf0) + j * D)[c];
    }
  }
}

// Gathered rows of step k in tiles of kThreads: tiles b = tile0, tile0 +
// stride, ... below tile_end. Each tile goes HBM -> registers -> LDS (X,
// rows padded to D + 1 amplitudes); thread r then computes row r from LDS;
// the result goes back through LDS to the other ping-pong buffer. For
// complex64 the next tile's loads are issued before the current tile is
// computed (complex128 rows would not fit in registers beside the row being
// computed).
template <typename T, int D>
__device__ __forceinline__ void ctrl_small_tiles(T* __restrict__ buf0, T* __restrict__ buf1, const T* __restrict__ Vs,
                                                 int k, uint64_t pmask, int64_t tile0, int64_t tile_end,
                                                 int64_t stride, int64_t M, T* __restrict__ X) {
  typedef typename Real<T>::type R;
  constexpr int P = D + 1;
  constexpr bool kAhead = sizeof(T) == 8;
  T rv[kAhead ? D : 1];
  int64_t b = tile0;
  if constexpr (kAhead)
    if (b < tile_end && b * kThreads < M) load_tile_regs<T, D>(buf0, buf1, k, pmask, b * kThreads, M, rv);
  for (; b < tile_end && b * kThreads < M; b += stride) {
    const int64_t i0 = b * kThreads;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const int e = threadIdx.x + q * kThreads;
      const int64_t i = i0 + e / D;
      if (i < M) {
        if constexpr (kAhead) {
          X[(e / D) * P + e % D] = rv[q];
        } else {
          const int64_t j = step_row(i, k, pmask);
          X[(e / D) * P + e % D] = ((src_buffer(j, pmask) ? buf1 : buf0) + j * D)[e % D];
        }
      }
    }
    __syncthreads();
    if constexpr (kAhead) {
      const int64_t nb = b + stride;
      if (nb < tile_end && nb * kThreads < M) load_tile_regs<T, D>(buf0, buf1, k, pmask, nb * kThreads, M, rv);
    }
    if (i0 + threadIdx.x < M) {
      T* x = X + threadIdx.x * P;
      R xr[D], xi[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T v = x[c];
        xr[c] = v.x;
        xi[c] = v.y;
      }
      // Rolled: unrolling lets the compiler hoist all d*d operator entries
      // out of the row loop into registers, which spills.
#pragma unroll 1
      for (int r = 0; r < D; ++r) {
        R yr = R(0), yi = R(0);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const T v = Vs[r * D + c];
          const R vr = v.x, vi = v.y;
          yr = fma(vr, xr[c], yr);
          yr = fma(-vi, xi[c], yr);
          yi = fma(vr, xi[c], yi);
          yi = fma(vi, xr[c], yi);
        }
        T o;
        o.x = yr;
        o.y = yi;
        x[r] = o;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const int e = threadIdx.x + q * kThreads, row = e / D, c = e % D;
      const int64_t i = i0 + row;
      if (i < M) {
        const int64_t j = step_row(i, k, pmask);
        ((src_buffer(j, pmask) ? buf0 : buf1) + j * D)[c] = X[row * P + c];
      }
    }
    __syncthreads();  // X is staged again for the next tile
  }
}

// The operator rounded to the state's type, into LDS.
template <typename T, int D>
__device__ __forceinline__ void load_operator(const double2* __restrict__ V, T* __restrict__ Vs) {
  typedef typename Real<T>::type R;
  for (int e = threadIdx.x; e < D * D; e += kThreads) {
    T v;
    v.x = R(V[e].x);
    v.y = R(V[e].y);
    Vs[e] = v;
  }
  __syncthreads();
}

// Rows [0, M) in tiles of kThreads: tiles b = tile0, tile0 + stride, ...
// below tile_end; Vs is LDS of D * D elements. With STAGE and D >= 8 the
// rows go through X (LDS of kThreads * (D + 1) elements); otherwise each
// thread reads and writes its own row directly, which costs less for rows of
// at most four amplitudes (32 or 64 bytes), where the LDS round trip saves
// nothing.
template <typename T, int D, bool STAGE>
__device__ __forceinline__ void ctrl_small_rows(T* __restrict__ buf0, T* __restrict__ buf1,
                                                const double2* __restrict__ V, int k, uint64_t pmask, int64_t tile0,
                                                int64_t tile_end, int64_t M, int64_t stride, T* __restrict__ Vs,
                                                T* __restrict__ X) {
  load_operator<T, D>(V, Vs);
  if constexpr (STAGE && D >= 8) {
    ctrl_small_tiles<T, D>(buf0, buf1, Vs, k, pmask, tile0, tile_end, stride, M, X);
  } else {
    typedef typename Real<T>::type R;
    for (int64_t b = tile0; b < tile_end && b * kThreads < M; b += stride) {
      const int64_t i = b * kThreads + threadIdx.x;
      if (i >= M) break;
      const int64_t j = step_row(i, k, pmask);
      const int p = src_buffer(j, pmask);
      const T* src = (p ? buf1 : buf0) + j * D;
      T* dst = (p ? buf0 : buf1) + j * D;
      R xr[D], xi[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T v = src[c];
        xr[c] = v.x;
        xi[c] = v.y;
      }
      // rolled for larger d, as in the staged tile
      constexpr int kRowUnroll = D >= 8 ? 1 : D;
#pragma unroll kRowUnroll
      for (int r = 0; r < D; ++r) {
        R yr = R(0), yi = R(0);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const T v = Vs[r * D + c];
          const R vr = v.x, vi = v.y;
          yr = fma(vr, xr[c], yr);
          yr = fma(-vi, xi[c], yr);
          yi = fma(vr, xi[c], yi);
          yi = fma(vi, xr[c], yi);
        }
        T o;
        o.x = yr;
        o.y = yi;
        dst[r] = o;
      }
    }
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(kThreads) k_ctrl_small(T* __restrict__ buf0, T* __restrict__ buf1,
                                                         const double2* __restrict__ V, int n, int k, uint64_t pmask) {
  __shared__ T Vs[D * D];
  __shared__ T X[D >= 8 ? kThreads * (D + 1) : 1];
  const int64_t M = int64_t(1) << (n - 1);
  ctrl_small_rows<T, D, true>(buf0, buf1, V, k, pmask, blockIdx.x, INT64_MAX, M, gridDim.x, Vs, X);
}

// Grouped controlled step k over the d <= 16 instances of a launch table:
// kSmallTiles tiles of 256 gathered rows per workgroup. STAGE (LDS staging for d = 8, 16) is
// launched only when such instances take part: its LDS tile would otherwise
// only lower the occupancy of the d <= 4 rows.
template <typename T, bool STAGE>
__global__ void __launch_bounds__(kThreads) kb_ctrl_small(int step, const InstDesc* __restrict__ desc,
                                                          const int32_t* __restrict__ table, int bflags,
                                                          int64_t tile0) {
  constexpr bool mixed = sizeof(T) == 8;
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const bool pol = (bflags & kBatchPolar) != 0, dbl = (bflags & kBatchDoubling) != 0;
  const RunLayout L = run_layout(D.n, D.t, mixed, pol);
  const int slot = power_slot(step, pol);
  const double2* V = slot == 0 ? D.U : reinterpret_cast<const double2*>(D.ws + (slot == 1 ? L.vbuf : L.tbuf));
  T* b0 = reinterpret_cast<T*>(D.ws + L.state0);
  // prefix doubling: rows [0, 2^k) -> rows [2^k, 2^(k+1)) of state0
  T* b1 = dbl ? b0 + (int64_t(1) << step) * (int64_t(1) << D.t) : reinterpret_cast<T*>(D.ws + L.state1);
  const uint64_t pmask = dbl ? kDoubling : (uint64_t(1) << step) - 1;
  const int64_t M = int64_t(1) << (dbl ? step : D.n - 1);
  const int64_t t0 = local * kSmallTiles, t1 = t0 + kSmallTiles;
  __shared__ T Vs[16 * 16];
  __shared__ T X[STAGE ? kThreads * 17 : 1];
  switch (D.t) {
    case 0: ctrl_small_rows<T, 1, STAGE>(b0, b1, V, step, pmask, t0, t1, M, 1, Vs, X); break;
    case 1: ctrl_small_rows<T, 2, STAGE>(b0, b1, V, step, pmask, t0, t1, M, 1, Vs, X); break;
    case 2: ctrl_small_rows<T, 4, STAGE>(b0, b1, V, step, pmask, t0, t1, M, 1, Vs, X); break;
    case 3: ctrl_small_rows<T, 8, STAGE>(b0, b1, V, step, pmask, t0, t1, M, 1, Vs, X); break;
    case 4: ctrl_small_rows<T, 16, STAGE>(b0, b1, V, step, pmask, t0, t1, M, 1, Vs, X); break;
  }
}

template <typename T, int D>
hipError_t go(void* b0, void* b1, const double2* V, int n, int k, uint64_t pmask, hipStream_t s) {
  int64_t M = int64_t(1) << (n - 1);
  int64_t g = (M + kThreads * kSmallTiles - 1) / (kThreads * kSmallTiles);
  if (g > 256 * 32) g = 256 * 32;
  hipLaunchKernelGGL((k_ctrl_small<T, D>), dim3(int(g)), dim3(kThreads), 0, s, static_cast<T*>(b0),
                     static_cast<T*>(b1), V, n, k, pmask);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch(void* b0, void* b1, const double2* V, int n, int t, int k, uint64_t pmask, hipStream_t s) {
  switch (t) {
    case 0: return go<T, 1>(b0, b1, V, n, k, pmask, s);
    case 1: return go<T, 2>(b0, b1, V, n, k, pmask, s);
    case 2: return go<T, 4>(b0, b1, V, n, k, pmask, s);
    case 3: return go<T, 8>(b0, b1, V, n, k, pmask, s);
    case 4: return go<T, 16>(b0, b1, V, n, k, pmask, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_ctrl_small(bool mixed, void* buf0, void* buf1, const double2* V, int n, int t, int k,
                             uint64_t pmask, hipStream_t s) {
  return mixed ? dispatch<float2>(buf0, buf1, V, n, t, k, pmask, s)
               : dispatch<double2>(buf0, buf1, V, n, t, k, pmask, s);
}

hipError_t launch_batch_ctrl_small(int step, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                                   bool stage, int bflags, hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    if (mixed && stage)
      hipLaunchKernelGGL((kb_ctrl_small<float2, true>), dim3(g), dim3(kThreads), 0, s, step, desc, table, bflags, b);
    else if (mixed)
      hipLaunchKernelGGL((kb_ctrl_small<float2, false>), dim3(g), dim3(kThreads), 0, s, step, desc, table, bflags, b);
    else if (stage)
      hipLaunchKernelGGL((kb_ctrl_small<double2, true>), dim3(g), dim3(kThreads), 0, s, step, desc, table, bflags, b);
    else
      hipLaunchKernelGGL((kb_ctrl_small<double2, false>), dim3(g), dim3(kThreads), 0, s, step, desc, table, bflags, b);
  });
}

}  // namespace qpe
