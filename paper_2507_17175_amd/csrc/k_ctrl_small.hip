// Controlled step (Fig. 1, controlled U^(2^k)) for target registers of at
// most 4 qubits (d <= 16). A d x d operator is too small to fill a matrix
// core tile, and the step is bound by HBM traffic, so each thread owns one
// gathered state row: it loads the d amplitudes, forms s <- V s with the
// operator broadcast from LDS, and writes the row to the other ping-pong
// buffer. FP64 form: complex128 state, FP64 arithmetic. Mixed form:
// complex64 state, the operator rounded once to FP32, FP32 FMAs.
#include "qpe_internal.hpp"

namespace qpe {

namespace {

constexpr int kThreads = 256;

template <typename T> struct Real;
template <> struct Real<float2> { typedef float type; };
template <> struct Real<double2> { typedef double type; };

// Rows i in [i0, i1) (stride) of the gathered set of step k.
template <typename T, int D>
__device__ __forceinline__ void ctrl_small_rows(T* __restrict__ buf0, T* __restrict__ buf1,
                                                const double2* __restrict__ V, int k, uint64_t pmask, int64_t i0,
                                                int64_t i1, int64_t stride) {
  typedef typename Real<T>::type R;
  __shared__ R Vre[D * D], Vim[D * D];
  for (int e = threadIdx.x; e < D * D; e += kThreads) {
    Vre[e] = R(V[e].x);
    Vim[e] = R(V[e].y);
  }
  __syncthreads();
  for (int64_t i = i0; i < i1; i += stride) {
    int64_t j = step_row(i, k, pmask);
    int p = src_buffer(j, pmask);
    const T* src = (p ? buf1 : buf0) + j * D;
    T* dst = (p ? buf0 : buf1) + j * D;
    R xr[D], xi[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T v = src[c];
      xr[c] = v.x;
      xi[c] = v.y;
    }
    // Rolled for larger d: unrolling lets the compiler hoist all d*d
    // operator entries out of the row loop into registers, which spills.
    constexpr int kRowUnroll = D >= 8 ? 1 : D;
#pragma unroll kRowUnroll
    for (int r = 0; r < D; ++r) {
      R yr = R(0), yi = R(0);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        R vr = Vre[r * D + c], vi = Vim[r * D + c];
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

template <typename T, int D>
__global__ void __launch_bounds__(kThreads) k_ctrl_small(T* __restrict__ buf0, T* __restrict__ buf1,
                                                         const double2* __restrict__ V, int n, int k, uint64_t pmask) {
  const int64_t M = int64_t(1) << (n - 1);
  ctrl_small_rows<T, D>(buf0, buf1, V, k, pmask, blockIdx.x * int64_t(kThreads) + threadIdx.x, M,
                        int64_t(gridDim.x) * kThreads);
}

// Grouped controlled step k over the d <= 16 instances of a launch table:
// 256 gathered rows per workgroup.
template <typename T>
__global__ void __launch_bounds__(kThreads) kb_ctrl_small(int step, const InstDesc* __restrict__ desc,
                                                          const int32_t* __restrict__ table, int bflags,
                                                          int64_t tile0) {
  constexpr bool mixed = sizeof(T) == 8;
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = desc[i];
  const bool pol = (bflags & kBatchPolar) != 0, dbl = (bflags & kBatchDoubling) != 0;
  const RunLayout L = run_layout(D.n, D.t, mixed, pol);
  const int slot = power_slot(step, pol);
  const double2* V = slot == 0 ? D.U : reinterpret_cast<const double2*>(D.ws + (slot == 1 ? L.vbuf : L.tbuf));
  T* b0 = reinterpret_cast<T*>(D.ws + L.state0);
  // prefix doubling: rows [0, 2^k) -> rows [2^k, 2^(k+1)) of state0
  T* b1 = dbl ? b0 + (int64_t(1) << step) * (int64_t(1) << D.t) : reinterpret_cast<T*>(D.ws + L.state1);
  const uint64_t pmask = dbl ? kDoubling : (uint64_t(1) << step) - 1;
  const int64_t M = int64_t(1) << (dbl ? step : D.n - 1);
  const int64_t i0 = local * kThreads + threadIdx.x;
  switch (D.t) {
    case 0: ctrl_small_rows<T, 1>(b0, b1, V, step, pmask, i0, M, int64_t(1) << 62); break;
    case 1: ctrl_small_rows<T, 2>(b0, b1, V, step, pmask, i0, M, int64_t(1) << 62); break;
    case 2: ctrl_small_rows<T, 4>(b0, b1, V, step, pmask, i0, M, int64_t(1) << 62); break;
    case 3: ctrl_small_rows<T, 8>(b0, b1, V, step, pmask, i0, M, int64_t(1) << 62); break;
    case 4: ctrl_small_rows<T, 16>(b0, b1, V, step, pmask, i0, M, int64_t(1) << 62); break;
  }
}

template <typename T, int D>
hipError_t go(void* b0, void* b1, const double2* V, int n, int k, uint64_t pmask, hipStream_t s) {
  int64_t M = int64_t(1) << (n - 1);
  int64_t g = (M + kThreads - 1) / kThreads;
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
                                   int bflags, hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    if (mixed)
      hipLaunchKernelGGL(kb_ctrl_small<float2>, dim3(g), dim3(kThreads), 0, s, step, desc, table, bflags, b);
    else
      hipLaunchKernelGGL(kb_ctrl_small<double2>, dim3(g), dim3(kThreads), 0, s, step, desc, table, bflags, b);
  });
}

}  // namespace qpe
