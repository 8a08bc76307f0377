// Rotation of the target register (paper section 2: the readout P(m) is the
// squared norm of the final state marginalised over the target register, so
// any unitary change of that register's basis leaves P unchanged):
//
//   U' = M U M^H,   psi' = M psi,   M = D2 H D1 / sqrt(d),
//
// H the d x d Walsh-Hadamard matrix (entries (-1)^popcount(i & j)), D1 a
// diagonal of signs, D2 a diagonal of unit phases. The run then emulates the
// circuit for (U', psi'), whose state rows are M times the original ones.
// Why: the matrix cores sum each group of 16 BF16 products with an error of
// up to a few units in the last place; for state rows spread over many
// components with unrelated phases these errors average out, but a row
// concentrated on a few basis vectors presents the same large product in
// every row and the errors add up coherently over the n steps. H D1 spreads
// such rows over all d components, and D2 gives the components unrelated
// phases (H D1 alone maps e_0 to a vector of equal entries +-1/sqrt(d),
// exact in BF16, whose errors again line up).
//
// The diagonals come from a key, a hash of the bits of U and psi, so no fixed
// input is concentrated again by the rotation; of four sign patterns D1
// derived from the key the one whose psi' has the smallest peak weight
// max_i |psi'_i|^2 / ||psi||^2 is kept, and that weight is reported.
//
// Arithmetic is FP64 throughout. With the Kronecker identity
// vec(H X H) = (H (x) H) vec(X) (row-major, H symmetric), M U M^H is one
// Walsh-Hadamard transform of length d^2 over the flattened D1 U D1, scaled
// by 1/d (an exact power of two), then each element (r, c) times
// D2_r conj(D2_c): passes of at most 8 bits through LDS, additions only, no
// d x d products.
#include "qpe_internal.hpp"

#include <cmath>

namespace qpe {

namespace {

constexpr int kThreads = 256;
constexpr int kPsiLds = 4096;  // psi' is transformed in LDS up to this d

// SplitMix64's output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", 2014), used here as a 64-bit mixer.
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Order-dependent, non-linear combination of a running hash with a word.
__device__ inline uint64_t combine(uint64_t h, uint64_t w) {
  return mix64(h * 0x9e3779b97f4a7c15ull + w + 0x632be59bd9b4e019ull);
}

__device__ inline uint64_t hash_elem(uint64_t h, double2 v) {
  h = combine(h, uint64_t(__double_as_longlong(v.x)));
  return combine(h, uint64_t(__double_as_longlong(v.y)));
}

// The sign diagonal D1 of a key: entry i is -1 when the top bit of a mix of
// (key, i) is set.
__device__ inline double sign_of(uint64_t key, int64_t i) {
  return (mix64(key + uint64_t(i) * 0xd1b54a32d192ed03ull) >> 63) ? -1.0 : 1.0;
}

// The phase diagonal D2 of a key: entry i is exp(2 pi i u) with u in [0, 1)
// from the top 53 bits of another mix of (key, i).
__device__ inline double2 phase_of(uint64_t key, int64_t i) {
  const uint64_t h = mix64((key ^ 0x8cb92ba72f3d8dd7ull) + uint64_t(i) * 0xaef17502108ef2d9ull);
  const double u = double(h >> 11) * 0x1.0p-53;
  double sv, cv;
  sincospi(2.0 * u, &sv, &cv);
  return make_double2(cv, sv);
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmul_conj(double2 a, double2 b) {  // a conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// Fixed-shape tree over the block's 256 values (deterministic).
__device__ inline uint64_t block_combine(uint64_t h, uint64_t* red) {
  red[threadIdx.x] = h;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = combine(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const uint64_t r = red[0];
  __syncthreads();
  return r;
}

__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Partial hash w of U: block w of G folds the chunks w, w + G, ... of
// kRotHashChunk elements, each thread its own strided elements in order,
// then the block's fixed tree; written to hash[w].
__device__ inline void rot_hash_block(const double2* __restrict__ U, int t, int64_t w,
                                      unsigned long long* __restrict__ hash) {
  __shared__ uint64_t red[kThreads];
  const int64_t dd = int64_t(1) << (2 * t);
  const int64_t G = rot_hash_blocks(t), nchunks = cdiv(dd, kRotHashChunk);
  uint64_t h = mix64(uint64_t(threadIdx.x) + 1);
  for (int64_t c = w; c < nchunks; c += G) {
    const int64_t e1 = min((c + 1) * kRotHashChunk, dd);
    for (int64_t e = c * kRotHashChunk + threadIdx.x; e < e1; e += kThreads) h = hash_elem(h, U[e]);
  }
  h = block_combine(h, red);
  if (threadIdx.x == 0) hash[w] = h;
}

// In-place unnormalised Walsh-Hadamard transform of v[0 .. 2^t) by one
// block, stage by stage (v in LDS, or in global memory for large d: each
// stage touches every element once, from one thread).
__device__ inline void wht_block(double2* v, int t) {
  const int64_t half = int64_t(1) << (t - 1);
  for (int h = 0; h < t; ++h) {
    for (int64_t p = threadIdx.x; p < half; p += kThreads) {
      const int64_t i0 = ((p >> h) << (h + 1)) | (p & ((int64_t(1) << h) - 1));
      const int64_t i1 = i0 | (int64_t(1) << h);
      const double2 a = v[i0], b = v[i1];
      v[i0] = make_double2(a.x + b.x, a.y + b.y);
      v[i1] = make_double2(a.x - b.x, a.y - b.y);
    }
    __syncthreads();
  }
}

// The key from the partial hashes of U and a hash of psi; then psi' = M psi
// for the best of four sign patterns; key and peak weight into scratch.
__device__ inline void rot_psi_block(const double2* __restrict__ psi, int t, unsigned long long* __restrict__ scratch,
                                     double2* __restrict__ psi_out, double2* lds) {
  __shared__ uint64_t redh[kThreads];
  __shared__ double redd[kThreads];
  const int64_t d = int64_t(1) << t;
  const int64_t G = rot_hash_blocks(t);
  uint64_t h = mix64(uint64_t(threadIdx.x) + 0x51ull);
  double nrm = 0.0;
  if (threadIdx.x < G) h = combine(h, uint64_t(scratch[kScratchHash + threadIdx.x]));
  for (int64_t i = threadIdx.x; i < d; i += kThreads) {
    const double2 v = psi[i];
    h = hash_elem(h, v);
    nrm += v.x * v.x + v.y * v.y;
  }
  const uint64_t key0 = block_combine(h, redh);
  const double norm2 = block_sum(nrm, redd);
  double2* v = d <= kPsiLds ? lds : psi_out;
  double best = 0.0;
  int bestc = 0;
  for (int c = 0; c < 5; ++c) {
    // candidates 0..3, then the chosen one again for the output
    const uint64_t key = combine(key0, uint64_t(c < 4 ? c : bestc));
    for (int64_t i = threadIdx.x; i < d; i += kThreads) {
      const double2 a = psi[i];
      const double sg = sign_of(key, i);
      v[i] = make_double2(sg * a.x, sg * a.y);
    }
    __syncthreads();
    wht_block(v, t);
    if (c == 4) break;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += kThreads) mx = fmax(mx, v[i].x * v[i].x + v[i].y * v[i].y);
    mx = block_max(mx, redd);
    const double peak = norm2 > 0.0 ? mx / (double(d) * norm2) : 0.0;
    if (c == 0 || peak < best) {
      best = peak;
      bestc = c;
    }
  }
  // 1 / sqrt(d): an exact power of two for even t
  const double scale = ldexp(1.0, -(t / 2)) * ((t & 1) ? 0.70710678118654752440 : 1.0);
  const uint64_t key = combine(key0, uint64_t(bestc));
  for (int64_t i = threadIdx.x; i < d; i += kThreads) {
    const double2 a = cmul(v[i], phase_of(key, i));
    psi_out[i] = make_double2(a.x * scale, a.y * scale);
  }
  if (threadIdx.x == 0) {
    scratch[kScratchKey] = key;
    scratch[kScratchPeak] = (unsigned long long)__double_as_longlong(best);
  }
}

// Factors a Walsh-Hadamard pass applies to element i of its vector, with
// d = 2^ts, r = i >> ts, c = i & (d - 1):
constexpr int kInSign2 = 1;      // on loading, D1_r D1_c (both sides of D1 U D1)
constexpr int kInConjPhase = 2;  // on loading, conj(D2_c)
constexpr int kOutPhase2 = 4;    // on storing, D2_r conj(D2_c)
constexpr int kOutSign = 8;      // on storing, D1_c

// One tile of a Walsh-Hadamard pass over bits [s, s + b) of a vector of
// 2^Ltot elements. Lines are the index values outside the bit group; a tile
// holds NL consecutive lines x 2^b, loaded so that consecutive threads touch
// consecutive addresses. `mode` selects the factors above; `scale` is
// applied on storing.
template <typename T>
__device__ inline void wht_pass_tile(const T* __restrict__ in, T* __restrict__ out, int Ltot, int s, int b,
                                     int64_t tile, uint64_t key, int mode, int ts, double scale) {
  __shared__ double2 lds[kWhtTile + kWhtTile / 2];
  const int lb = min(11 - b, Ltot - b);  // log2 of the lines per tile
  const int NL = 1 << lb, R = 1 << b, pitch = R + 1;
  const int E = NL << b;
  const int64_t l0 = tile * NL;
  const int64_t smask = (int64_t(1) << s) - 1, tmask = (int64_t(1) << ts) - 1;
  auto index = [&](int q, int& ll, int& g) -> int64_t {
    if (s == 0) {
      g = q & (R - 1);
      ll = q >> b;
    } else {
      ll = q & (NL - 1);
      g = q >> lb;
    }
    const int64_t l = l0 + ll;
    return ((l >> s) << (s + b)) | (int64_t(g) << s) | (l & smask);
  };
  for (int q = threadIdx.x; q < E; q += kThreads) {
    int ll, g;
    const int64_t i = index(q, ll, g);
    const T a = in[i];
    double2 v = make_double2(double(a.x), double(a.y));
    if (mode & kInSign2) {
      const double sg = sign_of(key, i >> ts) * sign_of(key, i & tmask);
      v.x *= sg;
      v.y *= sg;
    }
    if (mode & kInConjPhase) v = cmul_conj(v, phase_of(key, i & tmask));
    lds[ll * pitch + g] = v;
  }
  __syncthreads();
  for (int h = 0; h < b; ++h) {
    for (int p = threadIdx.x; p < E / 2; p += kThreads) {
      const int ll = p >> (b - 1), jj = p & ((R >> 1) - 1);
      const int g0 = ((jj >> h) << (h + 1)) | (jj & ((1 << h) - 1));
      double2* x = lds + ll * pitch + g0;
      const double2 u = x[0], w = x[1 << h];
      x[0] = make_double2(u.x + w.x, u.y + w.y);
      x[1 << h] = make_double2(u.x - w.x, u.y - w.y);
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < E; q += kThreads) {
    int ll, g;
    const int64_t i = index(q, ll, g);
    double2 v = lds[ll * pitch + g];
    double f = scale;
    if (mode & kOutSign) f *= sign_of(key, i & tmask);
    if (mode & kOutPhase2) v = cmul_conj(cmul(v, phase_of(key, i >> ts)), phase_of(key, i & tmask));
    T o;
    o.x = decltype(o.x)(v.x * f);
    o.y = decltype(o.y)(v.y * f);
    out[i] = o;
  }
}

// ------------------------------------------------------ single-instance kernels

__global__ void __launch_bounds__(kThreads) k_rot_hash(const double2* __restrict__ U, int t,
                                                       unsigned long long* __restrict__ scratch) {
  rot_hash_block(U, t, blockIdx.x, scratch + kScratchHash);
}

__global__ void __launch_bounds__(kThreads) k_rot_psi(const double2* __restrict__ psi, int t,
                                                      unsigned long long* __restrict__ scratch,
                                                      double2* __restrict__ psi_out) {
  __shared__ double2 v[kPsiLds];
  rot_psi_block(psi, t, scratch, psi_out, v);
}

// Pass q of M U M^H: bits [s, s + b) of the 2t-bit flattened index.
__global__ void __launch_bounds__(kThreads) k_rot_u_pass(const double2* __restrict__ in, double2* __restrict__ out,
                                                         int t, int s, int b, int first, int last,
                                                         const unsigned long long* __restrict__ scratch) {
  const uint64_t key = scratch[kScratchKey];
  wht_pass_tile<double2>(in, out, 2 * t, s, b, blockIdx.x, key, (first ? kInSign2 : 0) | (last ? kOutPhase2 : 0), t,
                         last ? ldexp(1.0, -t) : 1.0);
}

// Pass over bits [s, s + b) of the low t bits of an (n + t)-bit state.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_unrotate_pass(T* __restrict__ state, int n, int t, int s, int b,
                                                            int last, const unsigned long long* __restrict__ scratch,
                                                            int64_t tile0) {
  const uint64_t key = scratch[kScratchKey];
  const double scale = last ? ldexp(1.0, -(t / 2)) * ((t & 1) ? 0.70710678118654752440 : 1.0) : 1.0;
  wht_pass_tile<T>(state, state, n + t, s, b, tile0 + blockIdx.x, key,
                   (s == 0 ? kInConjPhase : 0) | (last ? kOutSign : 0), t, scale);
}

// ------------------------------------------------------------ batched kernel

template <int KIND>
__global__ void __launch_bounds__(kThreads) kb_rotate(int step, const InstDesc* __restrict__ desc,
                                                      const int32_t* __restrict__ table, int mixed, int bflags,
                                                      int64_t tile0) {
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const RunLayout L = run_layout(D.n, D.t, mixed != 0, (bflags & kBatchPolar) != 0);
  unsigned long long* scratch = reinterpret_cast<unsigned long long*>(D.ws + L.scratch);
  const int t = D.t;
  // the host pointed U and psi of the descriptor at the rotated buffers
  double2* Ur = const_cast<double2*>(D.U);
  double2* pr = const_cast<double2*>(D.psi);
  if constexpr (KIND == BK_ROTHASH) {
    rot_hash_block(D.U_src, t, local, scratch + kScratchHash);
  } else if constexpr (KIND == BK_ROTPSI) {
    __shared__ double2 v[kPsiLds];
    rot_psi_block(D.psi_src, t, scratch, pr, v);
  } else {
    const DftPlan pl = rot_plan(t);
    int s = 0;
    for (int q = 0; q < step; ++q) s += pl.bits[q];
    const bool last = step == pl.npass - 1;
    wht_pass_tile<double2>(step == 0 ? D.U_src : Ur, Ur, 2 * t, s, pl.bits[step], local, scratch[kScratchKey],
                           (step == 0 ? kInSign2 : 0) | (last ? kOutPhase2 : 0), t, last ? ldexp(1.0, -t) : 1.0);
  }
}

}  // namespace

hipError_t launch_rot_hash(const double2* U, int t, unsigned long long* scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_rot_hash, dim3(unsigned(rot_hash_blocks(t))), dim3(kThreads), 0, s, U, t, scratch);
  return hipGetLastError();
}

hipError_t launch_rot_psi(const double2* psi, int t, unsigned long long* scratch, double2* psi_out, hipStream_t s) {
  hipLaunchKernelGGL(k_rot_psi, dim3(1), dim3(kThreads), 0, s, psi, t, scratch, psi_out);
  return hipGetLastError();
}

hipError_t launch_rot_u(const double2* U, double2* Ur, int t, const unsigned long long* scratch, hipStream_t s) {
  const DftPlan pl = rot_plan(t);
  const unsigned tiles = unsigned(cdiv(int64_t(1) << (2 * t), kWhtTile));
  int sh = 0;
  for (int q = 0; q < pl.npass; ++q) {
    hipLaunchKernelGGL(k_rot_u_pass, dim3(tiles), dim3(kThreads), 0, s, q == 0 ? U : Ur, Ur, t, sh, pl.bits[q],
                       q == 0 ? 1 : 0, q == pl.npass - 1 ? 1 : 0, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sh += pl.bits[q];
  }
  return hipSuccess;
}

hipError_t launch_unrotate_state(bool mixed, void* state, int n, int t, const unsigned long long* scratch,
                                 hipStream_t s) {
  const DftPlan pl = make_dft_plan(t);
  const int64_t tiles = cdiv(int64_t(1) << (n + t), kWhtTile);
  int sh = 0;
  for (int q = 0; q < pl.npass; ++q) {
    const int last = q == pl.npass - 1 ? 1 : 0;
    hipError_t e = for_grid_chunks(tiles, [&](unsigned g, int64_t base) {
      if (mixed)
        hipLaunchKernelGGL(k_unrotate_pass<float2>, dim3(g), dim3(kThreads), 0, s, static_cast<float2*>(state), n, t,
                           sh, pl.bits[q], last, scratch, base);
      else
        hipLaunchKernelGGL(k_unrotate_pass<double2>, dim3(g), dim3(kThreads), 0, s, static_cast<double2*>(state), n,
                           t, sh, pl.bits[q], last, scratch, base);
    });
    if (e != hipSuccess) return e;
    sh += pl.bits[q];
  }
  return hipSuccess;
}

hipError_t launch_batch_rotate(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                               bool mixed, int bflags, hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    if (kind == BK_ROTHASH)
      hipLaunchKernelGGL(kb_rotate<BK_ROTHASH>, dim3(g), dim3(kThreads), 0, s, step, desc, table, mixed ? 1 : 0,
                         bflags, b);
    else if (kind == BK_ROTPSI)
      hipLaunchKernelGGL(kb_rotate<BK_ROTPSI>, dim3(g), dim3(kThreads), 0, s, step, desc, table, mixed ? 1 : 0,
                         bflags, b);
    else
      hipLaunchKernelGGL(kb_rotate<BK_ROTU>, dim3(g), dim3(kThreads), 0, s, step, desc, table, mixed ? 1 : 0,
                         bflags, b);
  });
}

}  // namespace qpe
