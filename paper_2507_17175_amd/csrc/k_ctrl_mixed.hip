// Mixed-form controlled step (Fig. 1, controlled U^(2^k)) on the gfx950
// matrix cores: for every row j of the complex64 state whose bit k is set,
//   S[j, :] <- S[j, :] V^T      (the target vector s becomes V s),
// as a complex GEMM of the gathered rows (M = N/2) with V^T (d x d).
//
// Precision: each FP32 state component a is split on the fly into three
// BF16 pieces a = a_h + a_m + a_l (RNE of the running residual, exact in
// FP32), and each FP64 operator component w was split the same way by the
// operator-preparation kernel. Of the nine piece products the six with index
// sum <= 2 are kept (hh, hm, mh, hl, mm, lh): the dropped ones sit below
// 2^-24 relative. Products are exact BF16 x BF16 terms accumulated in FP32 by
// v_mfma_f32_32x32x16_bf16. The complex product uses four real products:
//   re += a.re w.re + a.im (-w.im),   im += a.re w.im + a.im w.re.
//
// The state ping-pongs between two buffers (read buf[parity], write the
// other), so there is no copy-back and no read-after-write hazard between
// workgroups that share rows. The operator arrives pre-split as six BF16
// planes (hi/mid/lo x re/im), blocked by 16 columns so that the K slab of a
// column tile is one contiguous run.
//
// Kernels:
//  * k_ctrl_bf16x6_db (variant 2; the default below eight tiles per CU): 8
//    wave64s (two per SIMD, so one wave's LDS waits are covered by the
//    other's matrix-core work), K slab of 16 complex, double-buffered LDS:
//    the split-and-store of slab s+1 and the global loads of slab s+2 are
//    interleaved with the MFMAs of slab s, one barrier per slab. LDS rows are
//    padded to 48 bytes: the 16-byte fragment reads of 16 consecutive rows
//    then cover all 64 banks once.
//  * k_ctrl_bf16x6_pp (variant 6): the same tile and buffers, with the two
//    waves of each SIMD one phase apart: one runs a slab's MFMAs while the
//    other does its LDS and memory work.
//  * k_ctrl_bf16x6_pp2 (variant 7; the default from eight tiles per CU): as
//    variant 6, but each wave group splits and stores its own state rows
//    during its matrix phase, one MFMA at a time between the vector work.
//  * k_ctrl_bf16x6 (variant 1, and the small-launch default): 4 wave64s, K
//    slab of 32 complex, single LDS buffer with register prefetch.
//  * variants 3-5: the double-buffered kernel with the compiler's own issue
//    order, a triple-buffered swizzled-LDS kernel, and one that takes the
//    operator fragments from L2 straight into registers.
#include <type_traits>

#include "qpe_internal.hpp"

namespace qpe {

namespace {

constexpr int kPlaneBlock = 16;  // column blocking of the operator planes

typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
typedef __attribute__((__vector_size__(2 * sizeof(uint32_t)))) uint32_t u32x2;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

__device__ inline void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  float r1 = x - (float)h;
  m = (__bf16)r1;
  float r2 = r1 - (float)m;
  l = (__bf16)r2;
}

template <typename V>
__device__ inline V negate(V v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= (u32x4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(V, u);
}

typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(_Float16)))) _Float16 f16x4;

// Arithmetic schemes of the split products. Each operand component is a sum
// of P pieces in a 16-bit format; of the P x P piece products the pairs
// (PA[c], PB[c]), c < NPAIR, are kept, in that order (smallest first), and
// accumulated in FP32 by the matrix cores.
//
// Bf16x6: three BF16 pieces per operand (RNE of the running residual), the
// six pairs with index sum <= 2.
struct Bf16x6 {
  typedef bf16x8 v8;
  typedef bf16x4 v4;
  typedef __bf16 elem;
  static constexpr int P = 3, NPAIR = 6;
  static constexpr int PA[6] = {2, 1, 0, 1, 0, 0};
  static constexpr int PB[6] = {0, 1, 2, 0, 1, 0};
  // issue plan of the ping-pong matrix phase (one MFMA, then this many
  // vector ALU ops, for kValuGroups MFMAs; then LDS writes and loads)
  static constexpr int kValuGroups = 26, kValuPer = 3, kDsGroups = 3;
  __device__ static void split(float x, float, elem (&o)[3]) { split3(x, o[0], o[1], o[2]); }
  __device__ static f32x16 mfma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static float out_scale(float) { return 1.0f; }
};

// F16x3: the state scaled by sigma and the operator by 2^14 (powers of two,
// chosen so that no piece overflows FP16 and the low pieces stay normal for
// all but negligible elements), two FP16 pieces each (x = h + l, l the RNE of
// x - h), the three pairs lh, hl, hh; the FP32 sum is scaled back by
// 1 / (sigma 2^14). The dropped l l term is below 2^-22 relative, the
// representation errors 2^-22 each.
struct F16x3 {
  typedef f16x8 v8;
  typedef f16x4 v4;
  typedef _Float16 elem;
  static constexpr int P = 2, NPAIR = 3;
  static constexpr int PA[3] = {1, 0, 0};
  static constexpr int PB[3] = {0, 1, 0};
  static constexpr int kValuGroups = 8, kValuPer = 2, kDsGroups = 2;
  __device__ static void split(float x, float sigma, elem (&o)[2]) {
    const float y = x * sigma;  // exact: sigma is a power of two
    o[0] = (_Float16)y;
    o[1] = (_Float16)(y - (float)o[0]);  // y - h is exact in FP32
  }
  __device__ static f32x16 mfma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  __device__ static float out_scale(float sigma) { return 1.0f / (sigma * float(kOpScaleF16)); }
};

__device__ inline int2 xcd_tile(int tiles_m, int tiles_n) {
  const int total = tiles_m * tiles_n;
  int w = blockIdx.x;
  if ((total & 7) == 0) w = (w & 7) * (total >> 3) + (w >> 3);
  return make_int2(w / tiles_n, w % tiles_n);
}

// Six MFMA products of one (row block, column block) pair for one K chunk of
// 16: piece pairs with index sum <= 2, four real products per complex one.
// C0 = 3 keeps only the pairs hm, mh, hh (index sum <= 1, relative error
// ~2^-16): enough for the Newton-Schulz product X E, whose size is that of
// the unitarity defect (~1e-15), so its error stays ~1e-20 absolute.
template <int FM, int FN, int C0 = 0>
__device__ __forceinline__ void mma_bf16x6(f32x16 (&acc_re)[FM][FN], f32x16 (&acc_im)[FM][FN],
                                           const bf16x8 (&av)[FM][6], const bf16x8 (&bv)[FN][6],
                                           const bf16x8 (&bneg)[FN][3]) {
  constexpr int PA[6] = {2, 1, 0, 1, 0, 0};
  constexpr int PB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
  for (int c = C0; c < 6; ++c) {
    const int pa = PA[c], pb = PB[c];
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int y = 0; y < FN; ++y) {
        acc_re[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa], bv[y][2 * pb], acc_re[x][y], 0, 0, 0);
        acc_im[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa], bv[y][2 * pb + 1], acc_im[x][y], 0, 0, 0);
      }
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int y = 0; y < FN; ++y) {
        acc_re[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa + 1], bneg[y][pb], acc_re[x][y], 0, 0, 0);
        acc_im[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa + 1], bv[y][2 * pb], acc_im[x][y], 0, 0, 0);
      }
  }
}

// The four MFMA products of piece pair c alone (c = 0..5 in the order of
// mma_bf16x6), so that other work can be placed between the pairs.
template <int FM, int FN>
__device__ __forceinline__ void mma_pair(int c, f32x16 (&acc_re)[FM][FN], f32x16 (&acc_im)[FM][FN],
                                         const bf16x8 (&av)[FM][6], const bf16x8 (&bv)[FN][6],
                                         const bf16x8 (&bneg)[FN][3]) {
  constexpr int PA[6] = {2, 1, 0, 1, 0, 0};
  constexpr int PB[6] = {0, 1, 2, 0, 1, 0};
  const int pa = PA[c], pb = PB[c];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) {
      acc_re[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa], bv[y][2 * pb], acc_re[x][y], 0, 0, 0);
      acc_im[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa], bv[y][2 * pb + 1], acc_im[x][y], 0, 0, 0);
    }
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) {
      acc_re[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa + 1], bneg[y][pb], acc_re[x][y], 0, 0, 0);
      acc_im[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[x][2 * pa + 1], bv[y][2 * pb], acc_im[x][y], 0, 0, 0);
    }
}

// The products of one K chunk of 16 for a scheme: for each kept piece pair,
// four real products per complex one (re += a.re w.re + a.im (-w.im),
// im += a.re w.im + a.im w.re), in the order of mma_bf16x6.
// NEG: negate the imaginary operator fragment next to its use instead of
// taking it from bneg (shorter register lifetimes for wide tiles).
template <class S, int FM, int FN, bool NEG = false>
__device__ __forceinline__ void mma_pair_s(int c, f32x16 (&acc_re)[FM][FN], f32x16 (&acc_im)[FM][FN],
                                           const typename S::v8 (&av)[FM][2 * S::P],
                                           const typename S::v8 (&bv)[FN][2 * S::P],
                                           const typename S::v8 (&bneg)[FN][S::P]) {
  const int pa = S::PA[c], pb = S::PB[c];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) {
      acc_re[x][y] = S::mfma(av[x][2 * pa], bv[y][2 * pb], acc_re[x][y]);
      acc_im[x][y] = S::mfma(av[x][2 * pa], bv[y][2 * pb + 1], acc_im[x][y]);
    }
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) {
      acc_re[x][y] = S::mfma(av[x][2 * pa + 1], NEG ? negate(bv[y][2 * pb + 1]) : bneg[y][pb], acc_re[x][y]);
      acc_im[x][y] = S::mfma(av[x][2 * pa + 1], bv[y][2 * pb], acc_im[x][y]);
    }
}

template <class S, int FM, int FN, int C0 = 0, bool NEG = false>
__device__ __forceinline__ void mma_pieces(f32x16 (&acc_re)[FM][FN], f32x16 (&acc_im)[FM][FN],
                                           const typename S::v8 (&av)[FM][2 * S::P],
                                           const typename S::v8 (&bv)[FN][2 * S::P],
                                           const typename S::v8 (&bneg)[FN][S::P]) {
#pragma unroll
  for (int c = C0; c < S::NPAIR; ++c) mma_pair_s<S, FM, FN, NEG>(c, acc_re, acc_im, av, bv, bneg);
}

// Output layout of the 32x32 MFMA: lane l, element v holds row
// 8 * (v / 4) + 4 * (l / 32) + v % 4, column l % 32 of the block.
template <int FM, int FN>
__device__ __forceinline__ void store_tile(const f32x16 (&acc_re)[FM][FN], const f32x16 (&acc_im)[FM][FN],
                                           float2* buf0, float2* buf1, int M, int d, int k, uint64_t pmask, int row0,
                                           int col0, int lane, float oscale = 1.0f) {
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      int gi = row0 + 32 * x + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (gi >= M) continue;
      int64_t j = step_row(gi, k, pmask);
      float2* dst = (src_buffer(j, pmask) ? buf0 : buf1) + j * d + col0 + (lane & 31);
#pragma unroll
      for (int y = 0; y < FN; ++y) dst[32 * y] = make_float2(acc_re[x][y][v] * oscale, acc_im[x][y][v] * oscale);
    }
}

// ----------------------------------------------------------------- variant 2
template <class S, int BM, int BN, int WM, int WN, bool IL = true, int C0 = 0>
__device__ __forceinline__ void ctrl_db_tile(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                             const uint16_t* __restrict__ planes, int n, int t, int k,
                                             uint64_t pmask, int tile_m, int tile_n, float sigma = 1.0f) {
  constexpr int NP = 2 * S::P;  // planes per operand (pieces x re/im)
  constexpr int NT = 512;
  static_assert(WM * WN == 8, "8 waves");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KS = 16;       // complex K per slab
  constexpr int ROW = 24;      // padded LDS row in 16-bit elements (48 bytes)
  constexpr int A_PLANE = BM * ROW, B_PLANE = BN * ROW;
  constexpr int BUF = NP * (A_PLANE + B_PLANE);
  constexpr int CA = BM * KS / 4 / NT;  // 4-complex A chunks per thread
  constexpr int NB = 2 * NP * BN;          // 16-byte B chunks per slab
  constexpr int CB = (NB + NT - 1) / NT;   // per thread (the last one guarded)
  static_assert(CA >= 1 && CA * NT * 4 == BM * KS, "tile/thread mismatch");

  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int M = 1 << (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = tile_m * BM, j0 = tile_n * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;

  // Rows past M (only when M < BM) read row M-1 instead: the loads stay
  // unconditional (a guarded load becomes a branch that makes the compiler
  // wait for all outstanding loads), and the epilogue drops those rows.
  const float2* src_row[CA];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int c = tid + q * NT;
    int gi = min(i0 + c / 4, M - 1);
    int64_t j = step_row(gi, k, pmask);
    src_row[q] = (src_buffer(j, pmask) ? buf1 : buf0) + j * d + 4 * (c & 3);
  }

  float4 ra[CA][2];
  u32x4 rb[CB];

  auto load_global = [&](int s) {
    const int k0 = s * KS;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0);
      ra[q][0] = p[0];
      ra[q][1] = p[1];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      if (NB % NT != 0 && idx >= NB) break;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      rb[q] = *reinterpret_cast<const u32x4*>(planes + pl * dd + (int64_t(s) * d + j0 + (w >> 1)) * kPlaneBlock +
                                              8 * (w & 1));
    }
  };

  // The split of the prefetched A slab, one complex column u (0..3) of each
  // thread's 4-complex chunk at a time, into pieces pc (plane 2 piece + re/im).
  typename S::v4 pc[CA][NP];
  auto split_part = [&](int u) {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4 w = ra[q][u >> 1];
      typename S::elem o[S::P];
      S::split((u & 1) ? w.z : w.x, sigma, o);  // real part
#pragma unroll
      for (int pc2 = 0; pc2 < S::P; ++pc2) pc[q][2 * pc2][u] = o[pc2];
      S::split((u & 1) ? w.w : w.y, sigma, o);  // imaginary part
#pragma unroll
      for (int pc2 = 0; pc2 < S::P; ++pc2) pc[q][2 * pc2 + 1][u] = o[pc2];
    }
  };
  auto write_a = [&](int b) {
    uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tid + q * NT;
      int r = c / 4, kq = c & 3;
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        *reinterpret_cast<typename S::v4*>(base + pl * A_PLANE + r * ROW + 4 * kq) = pc[q][pl];
    }
  };
  auto write_b = [&](int b) {
    uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      if (NB % NT != 0 && idx >= NB) break;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      *reinterpret_cast<u32x4*>(base + NP * A_PLANE + pl * B_PLANE + (w >> 1) * ROW + 8 * (w & 1)) = rb[q];
    }
  };
  auto store_lds = [&](int b) {
#pragma unroll
    for (int u = 0; u < 4; ++u) split_part(u);
    write_a(b);
    write_b(b);
  };

  f32x16 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc_re[x][y][v] = 0.f;
        acc_im[x][y][v] = 0.f;
      }

  const int nk = d / KS;
  const int lr = lane & 31, ko = (lane >> 5) * 8;
  load_global(0);
  store_lds(0);
  if (nk > 1) load_global(1);
  __syncthreads();

  for (int s = 0; s < nk; ++s) {
    const uint16_t* base = lds + (s & 1) * BUF;
    typedef typename S::v8 V8;
    V8 av[FM][NP], bv[FN][NP], bneg[FN][S::P];
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        av[x][pl] = *reinterpret_cast<const V8*>(base + pl * A_PLANE + (wi0 + 32 * x + lr) * ROW + ko);
#pragma unroll
    for (int y = 0; y < FN; ++y) {
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        bv[y][pl] = *reinterpret_cast<const V8*>(base + NP * A_PLANE + pl * B_PLANE + (wj0 + 32 * y + lr) * ROW + ko);
#pragma unroll
      for (int pc = 0; pc < S::P; ++pc) bneg[y][pc] = negate(bv[y][2 * pc + 1]);
    }
    // The store of slab s+1 and the loads of slab s+2 are unconditional: the
    // last iteration writes the idle buffer (read in slab nk-2, which every
    // wave has left) and the last two reload slab nk-1.
    const int nb = (s + 1) & 1, ns = min(s + 2, nk - 1);
    if (IL) {
      // Explicit issue order: after each piece pair's MFMAs, a share of the
      // next slab's split, LDS stores and global loads. In-order issue then
      // runs that vector work while the matrix cores are still busy,
      // instead of after the last MFMA of the slab.
#pragma unroll
      for (int c = 0; c < S::NPAIR; ++c) {
        if (c >= C0) mma_pair_s<S, FM, FN>(c, acc_re, acc_im, av, bv, bneg);
        __builtin_amdgcn_sched_barrier(0);
        if (c == 0) write_b(nb);
        if (c < 2) {
          split_part(2 * c);
          split_part(2 * c + 1);
        }
        if (c == 1) write_a(nb);
        if (c == 2) load_global(ns);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      mma_pieces<S, FM, FN, C0>(acc_re, acc_im, av, bv, bneg);
      store_lds(nb);
      load_global(ns);
    }
    __syncthreads();
  }

  store_tile<FM, FN>(acc_re, acc_im, buf0, buf1, M, d, k, pmask, i0 + wi0, j0 + wj0, lane, S::out_scale(sigma));
}

template <int BM, int BN, int WM, int WN, bool IL = true, int C0 = 0>
__global__ void __launch_bounds__(512) k_ctrl_bf16x6_db(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                         const uint16_t* __restrict__ planes, int n, int t, int k,
                                                         uint64_t pmask) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_db_tile<Bf16x6, BM, BN, WM, WN, IL, C0>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(512) k_ctrl_f16x3_db(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                        const uint16_t* __restrict__ planes, int n, int t, int k,
                                                        uint64_t pmask, const float* __restrict__ sigma) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_db_tile<F16x3, BM, BN, WM, WN>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y, *sigma);
}

// ----------------------------------------------------------------- variant 6
// Ping-pong issue: the eight waves form two groups of four (waves 0-3 and
// 4-7; each SIMD holds one wave of each) that run the same slab loop one
// phase apart. A slab has a memory phase (fragment reads of slab s, split
// and LDS stores of slab s+1, global loads of slab s+2) and a matrix phase
// (the 48 MFMAs of slab s), and every phase ends at a workgroup barrier, so
// on each SIMD one wave feeds the matrix core while the other does its
// memory work. Buffer hazards: slab s+1 is stored into buffer (s+1)&1 by
// group 0 in phase 2s and by group 1 in phase 2s+1; that buffer was last
// read (slab s-1) in phases 2s-2 and 2s-1, and is read again (slab s+1) in
// phases 2s+2 and 2s+3, each on the other side of a barrier.
template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void ctrl_pp_tile(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                             const uint16_t* __restrict__ planes, int n, int t, int k,
                                             uint64_t pmask, int tile_m, int tile_n) {
  constexpr int NT = 512;
  static_assert(WM * WN == 8, "8 waves");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KS = 16;
  constexpr int ROW = 24;
  constexpr int A_PLANE = BM * ROW, B_PLANE = BN * ROW;
  constexpr int BUF = 6 * (A_PLANE + B_PLANE);
  constexpr int CA = BM * KS / 4 / NT;
  constexpr int NB = 12 * BN;
  constexpr int CB = (NB + NT - 1) / NT;
  static_assert(CA >= 1 && CA * NT * 4 == BM * KS, "tile/thread mismatch");

  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int M = 1 << (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = wave >> 2;
  const int i0 = tile_m * BM, j0 = tile_n * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;

  const float2* src_row[CA];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int c = tid + q * NT;
    int gi = min(i0 + c / 4, M - 1);
    int64_t j = step_row(gi, k, pmask);
    src_row[q] = (src_buffer(j, pmask) ? buf1 : buf0) + j * d + 4 * (c & 3);
  }

  float4 ra[CA][2];
  u32x4 rb[CB];
  auto load_global = [&](int s) {
    const int k0 = s * KS;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0);
      ra[q][0] = p[0];
      ra[q][1] = p[1];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      if (NB % NT != 0 && idx >= NB) break;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      rb[q] = *reinterpret_cast<const u32x4*>(planes + pl * dd + (int64_t(s) * d + j0 + (w >> 1)) * kPlaneBlock +
                                              8 * (w & 1));
    }
  };
  auto store_lds = [&](int b) {
    uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      bf16x4 pc[6];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 w = ra[q][u >> 1];
        __bf16 h, m, l;
        split3((u & 1) ? w.z : w.x, h, m, l);
        pc[0][u] = h;
        pc[2][u] = m;
        pc[4][u] = l;
        split3((u & 1) ? w.w : w.y, h, m, l);
        pc[1][u] = h;
        pc[3][u] = m;
        pc[5][u] = l;
      }
      int c = tid + q * NT;
      int r = c / 4, kq = c & 3;
#pragma unroll
      for (int pl = 0; pl < 6; ++pl) *reinterpret_cast<bf16x4*>(base + pl * A_PLANE + r * ROW + 4 * kq) = pc[pl];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      if (NB % NT != 0 && idx >= NB) break;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      *reinterpret_cast<u32x4*>(base + 6 * A_PLANE + pl * B_PLANE + (w >> 1) * ROW + 8 * (w & 1)) = rb[q];
    }
  };

  f32x16 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc_re[x][y][v] = 0.f;
        acc_im[x][y][v] = 0.f;
      }

  const int nk = d / KS;
  const int lr = lane & 31, ko = (lane >> 5) * 8;
  load_global(0);
  store_lds(0);
  if (nk > 1) load_global(1);
  __syncthreads();
  if (grp == 1) __syncthreads();

  for (int s = 0; s < nk; ++s) {
    // memory phase
    const uint16_t* base = lds + (s & 1) * BUF;
    bf16x8 av[FM][6], bv[FN][6], bneg[FN][3];
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        av[x][pl] = *reinterpret_cast<const bf16x8*>(base + pl * A_PLANE + (wi0 + 32 * x + lr) * ROW + ko);
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        bv[y][pl] =
            *reinterpret_cast<const bf16x8*>(base + 6 * A_PLANE + pl * B_PLANE + (wj0 + 32 * y + lr) * ROW + ko);
    // As in the double-buffered kernel, the store of slab s+1 and the loads
    // of slab s+2 are unconditional (the last slabs rewrite the idle buffer
    // and reload slab nk-1).
    store_lds((s + 1) & 1);
    load_global(min(s + 2, nk - 1));
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int pc = 0; pc < 3; ++pc) bneg[y][pc] = negate(bv[y][2 * pc + 1]);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    // matrix phase
    mma_bf16x6<FM, FN>(acc_re, acc_im, av, bv, bneg);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
  }
  if (grp == 0) __syncthreads();

  store_tile<FM, FN>(acc_re, acc_im, buf0, buf1, M, d, k, pmask, i0 + wi0, j0 + wj0, lane);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(512) k_ctrl_bf16x6_pp(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                         const uint16_t* __restrict__ planes, int n, int t, int k,
                                                         uint64_t pmask) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_pp_tile<BM, BN, WM, WN>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y);
}

// ----------------------------------------------------------------- variant 7
// Ping-pong with the state half of the tile private to each wave group:
// waves 0-3 use state rows 0-63 and waves 4-7 rows 64-127, so each group
// splits and stores its own rows of slab s+1 during its matrix phase of slab
// s (interleaved with its MFMAs), and the memory phase keeps only the
// fragment reads and the shared operator half. Hazards (group g's memory
// phase of slab s is phase 2s+g, its matrix phase 2s+1+g): its rows of
// buffer (s+1)&1 are written in phase 2s+1+g, read in 2s+2+g and were last
// read in 2s-2+g; the operator half is handled as in variant 6.
template <class S, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void ctrl_pp2_tile(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                              const uint16_t* __restrict__ planes, int n, int t, int k,
                                              uint64_t pmask, int tile_m, int tile_n, float sigma = 1.0f) {
  constexpr int NG = 256;  // threads per group (half of the 512-thread workgroup)
  constexpr int NP = 2 * S::P;
  static_assert(WM == 2 && WN == 4, "a group is one row half of the tile");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KS = 16;
  constexpr int ROW = 24;
  constexpr int A_PLANE = BM * ROW, B_PLANE = BN * ROW;
  constexpr int BUF = NP * (A_PLANE + B_PLANE);
  constexpr int CA = TM * KS / 4 / NG;  // 4-complex chunks of the group's rows per thread
  constexpr int NB = 2 * NP * BN / 2;   // 16-byte operator chunks per group
  constexpr int CB = (NB + NG - 1) / NG;
  static_assert(CA >= 1 && CA * NG * 4 == TM * KS, "tile/thread mismatch");
  static_assert(NB % NG == 0, "operator chunks per group");

  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int M = 1 << (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = wave >> 2, tg = tid & (NG - 1);
  const int i0 = tile_m * BM, j0 = tile_n * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;  // wi0 = grp * TM

  const float2* src_row[CA];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int c = tg + q * NG;
    int gi = min(i0 + wi0 + c / 4, M - 1);
    int64_t j = step_row(gi, k, pmask);
    src_row[q] = (src_buffer(j, pmask) ? buf1 : buf0) + j * d + 4 * (c & 3);
  }

  float4 ra[CA][2];
  u32x4 rb[CB];
  auto load_a = [&](int s) {
    const int k0 = s * KS;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0);
      ra[q][0] = p[0];
      ra[q][1] = p[1];
    }
  };
  auto load_b = [&](int s) {
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = grp * NB + tg + q * NG;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      rb[q] = *reinterpret_cast<const u32x4*>(planes + pl * dd + (int64_t(s) * d + j0 + (w >> 1)) * kPlaneBlock +
                                              8 * (w & 1));
    }
  };
  typename S::v4 pc[CA][NP];
  auto split_part = [&](int u) {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4 w = ra[q][u >> 1];
      typename S::elem o[S::P];
      S::split((u & 1) ? w.z : w.x, sigma, o);
#pragma unroll
      for (int pc2 = 0; pc2 < S::P; ++pc2) pc[q][2 * pc2][u] = o[pc2];
      S::split((u & 1) ? w.w : w.y, sigma, o);
#pragma unroll
      for (int pc2 = 0; pc2 < S::P; ++pc2) pc[q][2 * pc2 + 1][u] = o[pc2];
    }
  };
  auto write_a = [&](int b) {
    uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tg + q * NG;
      int r = wi0 + c / 4, kq = c & 3;
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        *reinterpret_cast<typename S::v4*>(base + pl * A_PLANE + r * ROW + 4 * kq) = pc[q][pl];
    }
  };
  auto write_b = [&](int b) {
    uint16_t* base = lds + b * BUF + NP * A_PLANE;
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = grp * NB + tg + q * NG;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      *reinterpret_cast<u32x4*>(base + pl * B_PLANE + (w >> 1) * ROW + 8 * (w & 1)) = rb[q];
    }
  };

  f32x16 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc_re[x][y][v] = 0.f;
        acc_im[x][y][v] = 0.f;
      }

  const int nk = d / KS;
  const int lr = lane & 31, ko = (lane >> 5) * 8;
  load_a(0);
  load_b(0);
#pragma unroll
  for (int u = 0; u < 4; ++u) split_part(u);
  write_a(0);
  write_b(0);
  // Slab 1 is loaded in the loop's order (operator chunks, then state rows):
  // the compiler's wait counts at the loop head cover both ways in, so with
  // the prologue's order reversed the memory phase would also wait for the
  // state rows loaded at the end of the previous matrix phase.
  if (nk > 1) {
    load_b(1);
    load_a(1);
  }
  __syncthreads();
  if (grp == 1) __syncthreads();

  for (int s = 0; s < nk; ++s) {
    const int nb = (s + 1) & 1, ns = min(s + 2, nk - 1);
    // memory phase: fragments of slab s, the group's operator chunks of
    // slab s+1 (unconditional, as in the other kernels), loads of slab s+2
    const uint16_t* base = lds + (s & 1) * BUF;
    typedef typename S::v8 V8;
    V8 av[FM][NP], bv[FN][NP], bneg[FN][S::P];
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        av[x][pl] = *reinterpret_cast<const V8*>(base + pl * A_PLANE + (wi0 + 32 * x + lr) * ROW + ko);
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        bv[y][pl] = *reinterpret_cast<const V8*>(base + NP * A_PLANE + pl * B_PLANE + (wj0 + 32 * y + lr) * ROW + ko);
    write_b(nb);
    load_b(ns);
    // wide tiles (two column blocks per wave) negate next to each use
    constexpr bool kNeg = FN > 1;
    if constexpr (!kNeg) {
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int pc2 = 0; pc2 < S::P; ++pc2) bneg[y][pc2] = negate(bv[y][2 * pc2 + 1]);
    }
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    // matrix phase, with the split and store of the group's rows of slab s+1
    // spread thinly between the MFMAs (one MFMA, then up to three VALU ops)
    mma_pieces<S, FM, FN, 0, kNeg>(acc_re, acc_im, av, bv, bneg);
#pragma unroll
    for (int u = 0; u < 4; ++u) split_part(u);
    write_a(nb);
    load_a(ns);
    constexpr int kMfma = FM * FN * 4 * S::NPAIR;
    constexpr int kRest = kMfma - S::kValuGroups - S::kDsGroups - 2;
    static_assert(kRest >= 0, "issue plan longer than the slab's MFMAs");
#pragma unroll
    for (int i = 0; i < S::kValuGroups; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, S::kValuPer, 0);
    }
#pragma unroll
    for (int i = 0; i < S::kDsGroups; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, kRest, 0);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
  }
  if (grp == 0) __syncthreads();

  store_tile<FM, FN>(acc_re, acc_im, buf0, buf1, M, d, k, pmask, i0 + wi0, j0 + wj0, lane, S::out_scale(sigma));
}

// One tile of a persistent launch: the buffers and operator of its instance,
// the register size and step, and its row block and column tile.
struct PTile {
  float2* buf0;
  float2* buf1;
  const uint16_t* planes;
  int n, k;
  uint64_t pmask;
  int tm, tn;
  float sigma;
};

// Persistent form of the ping-pong schedule: gridDim.x workgroups (one per
// CU), workgroup w takes tiles w, w + G, w + 2G, ... of the launch's `total`
// (G = gridDim.x, a multiple of 8, so a workgroup stays on one XCD and the
// XCD remap of the tile order is that of the one-tile-per-workgroup launch)
// as one stream of K slabs: slab g of the stream is slab g mod nk of tile
// g / nk. prov(L) describes tile L of the launch; all tiles have d = 2^t
// (the tiles of a batched launch may belong to different instances). The
// loads of a tile's first two slabs are issued during the previous tile's
// last two, and a group stores a finished tile at the start of its next
// memory phase, while the other group runs its matrix phase; a launch of T
// tiles thus pays the prologue and the first phase's wait once per
// workgroup instead of once per tile. Every wave runs the same number of
// slabs and barriers (the tile count is uniform over the workgroup).
template <class S, int BM, int BN, int WM, int WN, class Prov>
__device__ __forceinline__ void ctrl_pp2p_tiles(int t, int total, Prov prov) {
  constexpr int NG = 256;
  constexpr int NP = 2 * S::P;
  static_assert(WM == 2 && WN == 4, "a group is one row half of the tile");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KS = 16;
  constexpr int ROW = 24;
  constexpr int A_PLANE = BM * ROW, B_PLANE = BN * ROW;
  constexpr int BUF = NP * (A_PLANE + B_PLANE);
  constexpr int CA = TM * KS / 4 / NG;
  constexpr int NB = 2 * NP * BN / 2;
  constexpr int CB = (NB + NG - 1) / NG;
  static_assert(CA >= 1 && CA * NG * 4 == TM * KS, "tile/thread mismatch");
  static_assert(NB % NG == 0, "operator chunks per group");

  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int G = int(gridDim.x), w = int(blockIdx.x);
  const int count = (total - w + G - 1) / G;  // tiles of this workgroup
  if (count <= 0) return;                     // (the launcher keeps G <= total)
  const int nk = d / KS;                      // a power of two
  const int lg_nk = 31 - __builtin_clz(unsigned(nk));
  const int gmax = count * nk - 1;
  // this workgroup's i-th tile
  auto tile_of = [&](int i) {
    int L = w + i * G;
    if ((total & 7) == 0) L = (L & 7) * (total >> 3) + (L >> 3);
    return prov(L);
  };

  // wave-uniform values live in scalar registers
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave >> 2, tg = tid & (NG - 1);
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;

  // loads follow the tile of the slab they fetch
  int load_tile = -1, lj0 = 0;
  const uint16_t* lplanes = nullptr;
  float lsigma = 1.0f;
  const float2* src_row[CA];
  auto set_load_tile = [&](int i) {
    const PTile pt = tile_of(i);
    const int M = 1 << (pt.n - 1);
    load_tile = i;
    lj0 = pt.tn * BN;
    lplanes = pt.planes;
    lsigma = pt.sigma;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tg + q * NG;
      int gi = min(pt.tm * BM + wi0 + c / 4, M - 1);
      int64_t j = step_row(gi, pt.k, pt.pmask);
      src_row[q] = (src_buffer(j, pt.pmask) ? pt.buf1 : pt.buf0) + j * d + 4 * (c & 3);
    }
  };

  float4 ra[CA][2];
  float ra_sigma = 1.0f;  // the state scale of the tile whose rows ra holds
  u32x4 rb[CB];
  auto load_a = [&](int g) {
    const int k0 = (g & (nk - 1)) * KS;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0);
      ra[q][0] = p[0];
      ra[q][1] = p[1];
    }
  };
  // operator chunk q of a thread: plane (grp NB + q NG) / 2BN (wave-uniform,
  // as NG divides 2BN), column and half from the thread's index; the address
  // is a wave-uniform base plus a 32-bit per-lane offset
  static_assert((BN * 2) % NG == 0 && NB % (BN * 2) == 0, "operator chunk layout");
  auto load_b = [&](int g) {
    const int sl = g & (nk - 1);
    // (the empty asm keeps the compiler from hoisting one 64-bit address per
    // chunk out of the loop, which costs eight registers)
    uint32_t lo = uint32_t((tg >> 1) * kPlaneBlock + 8 * (tg & 1));
    asm volatile("" : "+v"(lo));
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const int pl = (grp * NB + q * NG) / (BN * 2);
      const uint32_t off = lo + uint32_t((q * NG) % (BN * 2) / 2 * kPlaneBlock);
      const uint16_t* base = lplanes + (int64_t(pl) * dd + (int64_t(sl) * d + lj0) * kPlaneBlock);
      rb[q] = *reinterpret_cast<const u32x4*>(base + off);
    }
  };
  typename S::v4 pc[CA][NP];
  auto split_part = [&](int u) {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4 x = ra[q][u >> 1];
      typename S::elem o[S::P];
      S::split((u & 1) ? x.z : x.x, ra_sigma, o);
#pragma unroll
      for (int pc2 = 0; pc2 < S::P; ++pc2) pc[q][2 * pc2][u] = o[pc2];
      S::split((u & 1) ? x.w : x.y, ra_sigma, o);
#pragma unroll
      for (int pc2 = 0; pc2 < S::P; ++pc2) pc[q][2 * pc2 + 1][u] = o[pc2];
    }
  };
  auto write_a = [&](int b) {
    uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tg + q * NG;
      int r = wi0 + c / 4, kq = c & 3;
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        *reinterpret_cast<typename S::v4*>(base + pl * A_PLANE + r * ROW + 4 * kq) = pc[q][pl];
    }
  };
  auto write_b = [&](int b) {
    uint16_t* base = lds + b * BUF + NP * A_PLANE;
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const int pl = (grp * NB + q * NG) / (BN * 2);
      const int wv = (q * NG + tg) % (BN * 2);
      *reinterpret_cast<u32x4*>(base + pl * B_PLANE + (wv >> 1) * ROW + 8 * (wv & 1)) = rb[q];
    }
  };

  f32x16 acc_re[FM][FN], acc_im[FM][FN];
  auto zero_acc = [&]() {
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          acc_re[x][y][v] = 0.f;
          acc_im[x][y][v] = 0.f;
        }
  };
  auto store_acc = [&](int i) {
    const PTile pt = tile_of(i);
    store_tile<FM, FN>(acc_re, acc_im, pt.buf0, pt.buf1, 1 << (pt.n - 1), d, pt.k, pt.pmask, pt.tm * BM + wi0,
                       pt.tn * BN + wj0, lane, S::out_scale(pt.sigma));
  };
  zero_acc();

  const int lr = lane & 31, ko = (lane >> 5) * 8;
  set_load_tile(0);
  load_a(0);
  load_b(0);
  ra_sigma = lsigma;
#pragma unroll
  for (int u = 0; u < 4; ++u) split_part(u);
  write_a(0);
  write_b(0);
  load_b(1);  // nk >= 2: slab 1 is in tile 0; loaded in the loop's order
  load_a(1);
  __syncthreads();
  if (grp == 1) __syncthreads();

  for (int g = 0; g <= gmax; ++g) {
    const int nb = (g + 1) & 1, g2 = min(g + 2, gmax);
    // memory phase: the operator chunks of slab g+1, the finished tile (a
    // group's first memory phase of a new tile), the fragments of slab g and
    // the loads of slab g+2, in the tile of g+2
    write_b(nb);
    if ((g & (nk - 1)) == 0 && g > 0) {
      __builtin_amdgcn_sched_barrier(0);
      store_acc((g >> lg_nk) - 1);
      zero_acc();
      __builtin_amdgcn_sched_barrier(0);
    }
    const uint16_t* base = lds + (g & 1) * BUF;
    typedef typename S::v8 V8;
    V8 av[FM][NP], bv[FN][NP], bneg[FN][S::P];
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        av[x][pl] = *reinterpret_cast<const V8*>(base + pl * A_PLANE + (wi0 + 32 * x + lr) * ROW + ko);
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        bv[y][pl] = *reinterpret_cast<const V8*>(base + NP * A_PLANE + pl * B_PLANE + (wj0 + 32 * y + lr) * ROW + ko);
    if ((g2 >> lg_nk) != load_tile) set_load_tile(g2 >> lg_nk);
    load_b(g2);
    constexpr bool kNeg = FN > 1;
    if constexpr (!kNeg) {
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int pc2 = 0; pc2 < S::P; ++pc2) bneg[y][pc2] = negate(bv[y][2 * pc2 + 1]);
    }
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    // matrix phase, with the split and store of the group's rows of slab g+1
    mma_pieces<S, FM, FN, 0, kNeg>(acc_re, acc_im, av, bv, bneg);
#pragma unroll
    for (int u = 0; u < 4; ++u) split_part(u);
    write_a(nb);
    load_a(g2);
    ra_sigma = lsigma;
    constexpr int kMfma = FM * FN * 4 * S::NPAIR;
    constexpr int kRest = kMfma - S::kValuGroups - S::kDsGroups - 2;
    static_assert(kRest >= 0, "issue plan longer than the slab's MFMAs");
#pragma unroll
    for (int i = 0; i < S::kValuGroups; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, S::kValuPer, 0);
    }
#pragma unroll
    for (int i = 0; i < S::kDsGroups; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, kRest, 0);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
  }
  if (grp == 0) __syncthreads();

  store_acc(count - 1);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(512) k_ctrl_bf16x6_pp2(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                          const uint16_t* __restrict__ planes, int n, int t, int k,
                                                          uint64_t pmask) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_pp2_tile<Bf16x6, BM, BN, WM, WN>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(512) k_ctrl_f16x3_pp2(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                         const uint16_t* __restrict__ planes, int n, int t, int k,
                                                         uint64_t pmask, const float* __restrict__ sigma) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_pp2_tile<F16x3, BM, BN, WM, WN>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y, *sigma);
}

// The persistent wide-tile kernel (gridDim.x workgroups, a multiple of 8).
template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(512) k_ctrl_f16x3_pp2p(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                          const uint16_t* __restrict__ planes, int n, int t, int k,
                                                          uint64_t pmask, const float* __restrict__ sigma) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const float sg = *sigma;
  ctrl_pp2p_tiles<F16x3, BM, BN, WM, WN>(t, tiles_m * tiles_n, [=](int L) {
    return PTile{buf0, buf1, planes, n, k, pmask, L / tiles_n, L % tiles_n, sg};
  });
}

// ----------------------------------------------------------------- variant 4
// Triple-buffered LDS with unpadded 32-byte rows. A row r holds the two
// 16-byte K chunks of one slab; chunk h sits at position h ^ ((r >> 3) & 1),
// so the 16 rows that one quarter of a wave touches in a fragment read, an A
// store (8 bytes per lane) or a B store (16 bytes per lane) cover each bank
// once. With three buffers the slab s + 1 buffer is complete one barrier
// earlier than it is needed, so the fragment reads of slab s + 1 are issued
// before the barrier that ends slab s and their latency overlaps it. The
// global loads run four slabs ahead; the split of slab s + 2 is stored
// between the MFMA groups of slab s.
template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void ctrl_tb_tile(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                             const uint16_t* __restrict__ planes, int n, int t, int k,
                                             uint64_t pmask, int tile_m, int tile_n) {
  constexpr int NT = 512;
  static_assert(WM * WN == 8, "8 waves");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KS = 16;   // complex K per slab
  constexpr int ROW = 16;  // bf16 per LDS row (32 bytes)
  constexpr int A_PLANE = BM * ROW, B_PLANE = BN * ROW;
  constexpr int BUF = 6 * (A_PLANE + B_PLANE);
  constexpr int CA = BM * KS / 4 / NT;   // 4-complex A chunks per thread
  constexpr int NB = 12 * BN;            // 16-byte B chunks per slab
  constexpr int CB = (NB + NT - 1) / NT;  // per thread (the last one guarded)
  static_assert(CA >= 1 && CA * NT * 4 == BM * KS, "tile/thread mismatch");
  static_assert(3 * BUF * 2 <= 160 * 1024, "LDS budget");

  __shared__ __attribute__((aligned(16))) uint16_t lds[3 * BUF];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int M = 1 << (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = tile_m * BM, j0 = tile_n * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;
  // bf16 offset of 16-byte chunk h of LDS row r
  auto sw = [](int r, int h) { return r * ROW + 8 * (h ^ ((r >> 3) & 1)); };

  // Rows past M (only when M < BM) read row M-1 (unconditional loads).
  const float2* src_row[CA];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int c = tid + q * NT;
    int gi = min(i0 + c / 4, M - 1);
    int64_t j = step_row(gi, k, pmask);
    src_row[q] = (src_buffer(j, pmask) ? buf1 : buf0) + j * d + 4 * (c & 3);
  }

  // two register sets: slab s + 2 is split from set s & 1, which was loaded
  // two slabs earlier, so a global load has two slabs of time to arrive
  float4 ra[2][CA][2];
  u32x4 rb[2][CB];
  auto load_global = [&](auto setc, int s) {
    constexpr int S = decltype(setc)::value;
    const int k0 = s * KS;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0);
      ra[S][q][0] = p[0];
      ra[S][q][1] = p[1];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      if (NB % NT != 0 && idx >= NB) break;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      rb[S][q] = *reinterpret_cast<const u32x4*>(planes + pl * dd +
                                                 (int64_t(s) * d + j0 + (w >> 1)) * kPlaneBlock + 8 * (w & 1));
    }
  };
  bf16x4 pc[CA][6];
  auto split_part = [&](auto setc, int u) {
    constexpr int S = decltype(setc)::value;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4 w = ra[S][q][u >> 1];
      __bf16 h, m, l;
      split3((u & 1) ? w.z : w.x, h, m, l);
      pc[q][0][u] = h;
      pc[q][2][u] = m;
      pc[q][4][u] = l;
      split3((u & 1) ? w.w : w.y, h, m, l);
      pc[q][1][u] = h;
      pc[q][3][u] = m;
      pc[q][5][u] = l;
    }
  };
  auto write_a = [&](int b) {
    uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tid + q * NT;
      int r = c / 4, kq = c & 3;
      const int off = sw(r, kq >> 1) + 4 * (kq & 1);
#pragma unroll
      for (int pl = 0; pl < 6; ++pl) *reinterpret_cast<bf16x4*>(base + pl * A_PLANE + off) = pc[q][pl];
    }
  };
  auto write_b = [&](auto setc, int b) {
    constexpr int S = decltype(setc)::value;
    uint16_t* base = lds + b * BUF + 6 * A_PLANE;
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      if (NB % NT != 0 && idx >= NB) break;
      int pl = idx / (BN * 2), w = idx % (BN * 2);
      *reinterpret_cast<u32x4*>(base + pl * B_PLANE + sw(w >> 1, w & 1)) = rb[S][q];
    }
  };

  f32x16 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc_re[x][y][v] = 0.f;
        acc_im[x][y][v] = 0.f;
      }

  const int lr = lane & 31, kh = lane >> 5;
  bf16x8 av[FM][6], bv[FN][6], bneg[FN][3];
  auto read_frags = [&](int b) {
    const uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        av[x][pl] = *reinterpret_cast<const bf16x8*>(base + pl * A_PLANE + sw(wi0 + 32 * x + lr, kh));
#pragma unroll
    for (int y = 0; y < FN; ++y) {
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        bv[y][pl] = *reinterpret_cast<const bf16x8*>(base + 6 * A_PLANE + pl * B_PLANE + sw(wj0 + 32 * y + lr, kh));
#pragma unroll
      for (int pc2 = 0; pc2 < 3; ++pc2) bneg[y][pc2] = negate(bv[y][2 * pc2 + 1]);
    }
  };

  const int nk = d / KS;  // a power of two >= 4 here (d >= 64)
  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, 1>;
  load_global(Set0{}, 0);
#pragma unroll
  for (int u = 0; u < 4; ++u) split_part(Set0{}, u);
  write_a(0);
  write_b(Set0{}, 0);
  load_global(Set1{}, 1);
#pragma unroll
  for (int u = 0; u < 4; ++u) split_part(Set1{}, u);
  write_a(1);
  write_b(Set1{}, 1);
  load_global(Set0{}, 2);
  load_global(Set1{}, 3);
  __syncthreads();
  read_frags(0);

  // slab s: MFMAs from buffer s % 3; the split of slab s + 2 (register set
  // s & 1) goes to buffer (s + 2) % 3 between the MFMA groups; then set s & 1
  // is reloaded with slab s + 4, and the fragments of slab s + 1 are read.
  auto slab = [&](auto setc, int s, int bcur) {
    const int b1 = bcur == 2 ? 0 : bcur + 1;
    const int b2 = b1 == 2 ? 0 : b1 + 1;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      mma_pair<FM, FN>(c, acc_re, acc_im, av, bv, bneg);
      __builtin_amdgcn_sched_barrier(0);
      if (c < 4) split_part(setc, c);
      if (c == 3) write_a(b2);
      if (c == 4) write_b(setc, b2);
      if (c == 5) load_global(setc, min(s + 4, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    // Slab s + 1 was stored before the previous barrier: read it now. (In
    // the last iteration this reads a buffer whose contents go unused.)
    read_frags(b1);
    __syncthreads();
    return b1;
  };
  int bcur = 0;
  for (int s = 0; s < nk; s += 2) {
    bcur = slab(Set0{}, s, bcur);
    bcur = slab(Set1{}, s + 1, bcur);
  }

  store_tile<FM, FN>(acc_re, acc_im, buf0, buf1, M, d, k, pmask, i0 + wi0, j0 + wj0, lane);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(512) k_ctrl_bf16x6_tb(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                         const uint16_t* __restrict__ planes, int n, int t, int k,
                                                         uint64_t pmask) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_tb_tile<BM, BN, WM, WN>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y);
}

// ----------------------------------------------------------------- variant 5
// Like variant 2 for the state operand, but the operator fragments bypass
// LDS: each wave loads its own B fragments (for one 32-column block and one
// plane, lane l needs the 8 K values 8 (l / 32) .. of column l % 32, which in
// the blocked plane layout are 16 contiguous bytes, so a wave's load covers
// 1 KB contiguously) straight into registers one slab ahead. This halves the
// LDS stores per slab at the price of reading each operator fragment from L2
// once per wave row (WM times) instead of once per workgroup.
template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void ctrl_bg_tile(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                             const uint16_t* __restrict__ planes, int n, int t, int k,
                                             uint64_t pmask, int tile_m, int tile_n) {
  constexpr int NT = 512;
  static_assert(WM * WN == 8, "8 waves");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KS = 16;   // complex K per slab
  constexpr int ROW = 24;  // padded LDS row in bf16 (48 bytes)
  constexpr int A_PLANE = BM * ROW;
  constexpr int BUF = 6 * A_PLANE;
  constexpr int CA = BM * KS / 4 / NT;
  static_assert(CA >= 1 && CA * NT * 4 == BM * KS, "tile/thread mismatch");

  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int M = 1 << (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = tile_m * BM, j0 = tile_n * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;
  const int lr = lane & 31, ko = (lane >> 5) * 8;

  const float2* src_row[CA];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int c = tid + q * NT;
    int gi = min(i0 + c / 4, M - 1);
    int64_t j = step_row(gi, k, pmask);
    src_row[q] = (src_buffer(j, pmask) ? buf1 : buf0) + j * d + 4 * (c & 3);
  }
  // operator fragment base of this lane: column j0 + wj0 + 32 y + lr
  const uint16_t* bsrc = planes + int64_t(j0 + wj0 + lr) * kPlaneBlock + ko;

  float4 ra[CA][2];
  auto load_a = [&](int s) {
    const int k0 = s * KS;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0);
      ra[q][0] = p[0];
      ra[q][1] = p[1];
    }
  };
  bf16x8 bset[2][FN][6];
  auto load_b = [&](auto setc, int s) {
    constexpr int S = decltype(setc)::value;
    const uint16_t* p0 = bsrc + int64_t(s) * d * kPlaneBlock;
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        bset[S][y][pl] = *reinterpret_cast<const bf16x8*>(p0 + pl * dd + 32 * y * kPlaneBlock);
  };
  bf16x4 pc[CA][6];
  auto split_part = [&](int u) {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const float4 w = ra[q][u >> 1];
      __bf16 h, m, l;
      split3((u & 1) ? w.z : w.x, h, m, l);
      pc[q][0][u] = h;
      pc[q][2][u] = m;
      pc[q][4][u] = l;
      split3((u & 1) ? w.w : w.y, h, m, l);
      pc[q][1][u] = h;
      pc[q][3][u] = m;
      pc[q][5][u] = l;
    }
  };
  auto write_a = [&](int b) {
    uint16_t* base = lds + b * BUF;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tid + q * NT;
      int r = c / 4, kq = c & 3;
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        *reinterpret_cast<bf16x4*>(base + pl * A_PLANE + r * ROW + 4 * kq) = pc[q][pl];
    }
  };

  f32x16 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc_re[x][y][v] = 0.f;
        acc_im[x][y][v] = 0.f;
      }

  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, 1>;
  const int nk = d / KS;  // a power of two >= 2
  load_a(0);
#pragma unroll
  for (int u = 0; u < 4; ++u) split_part(u);
  write_a(0);
  load_a(min(1, nk - 1));
  load_b(Set0{}, 0);
  __syncthreads();

  // slab s: operator fragments from register set s & 1 (loaded during slab
  // s - 1), state fragments from LDS buffer s & 1; the next slab's operator
  // fragments go to the other set, its state slab to the other buffer.
  auto slab = [&](auto setc, int s) {
    constexpr int S = decltype(setc)::value;
    constexpr int SN = 1 - S;
    const uint16_t* base = lds + S * BUF;
    bf16x8 av[FM][6], bneg[FN][3];
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        av[x][pl] = *reinterpret_cast<const bf16x8*>(base + pl * A_PLANE + (wi0 + 32 * x + lr) * ROW + ko);
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int pc2 = 0; pc2 < 3; ++pc2) bneg[y][pc2] = negate(bset[S][y][2 * pc2 + 1]);
    load_b(std::integral_constant<int, SN>{}, min(s + 1, nk - 1));
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      mma_pair<FM, FN>(c, acc_re, acc_im, av, bset[S], bneg);
      __builtin_amdgcn_sched_barrier(0);
      if (c < 4) split_part(c);
      if (c == 3) write_a(SN);
      if (c == 5) load_a(min(s + 2, nk - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  };
  for (int s = 0; s < nk; s += 2) {
    slab(Set0{}, s);
    slab(Set1{}, s + 1);
  }

  store_tile<FM, FN>(acc_re, acc_im, buf0, buf1, M, d, k, pmask, i0 + wi0, j0 + wj0, lane);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(512) k_ctrl_bf16x6_bg(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                         const uint16_t* __restrict__ planes, int n, int t, int k,
                                                         uint64_t pmask) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_bg_tile<BM, BN, WM, WN>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y);
}

// ----------------------------------------------------------------- variant 1
template <class S, int BM, int BN, int WM, int WN, int C0 = 0>
__device__ __forceinline__ void ctrl_v1_tile(float2* __restrict__ buf0, float2* __restrict__ buf1,
                                             const uint16_t* __restrict__ planes, int n, int t, int k,
                                             uint64_t pmask, int tile_m, int tile_n, float sigma = 1.0f) {
  constexpr int NT = 256;
  constexpr int NP = 2 * S::P;
  constexpr int KS = 32;   // complex K per slab (two operator-plane blocks)
  constexpr int ROW = 40;  // padded LDS row in 16-bit elements (80 bytes)
  static_assert(WM * WN == 4, "4 waves");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int CA = BM * 4 / NT;      // 8-complex A chunks per thread
  constexpr int CB = NP * BN * 4 / NT;  // 16-byte B chunks per thread
  static_assert(CA >= 1 && CB >= 1, "tile too small");

  __shared__ __attribute__((aligned(16))) uint16_t As[NP * BM * ROW];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[NP * BN * ROW];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int M = 1 << (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = tile_m * BM, j0 = tile_n * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;

  // Rows past M read row M-1 (unconditional loads; see variant 2).
  const float2* src_row[CA];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int c = tid + q * NT;
    int gi = min(i0 + c / 4, M - 1);
    int64_t j = step_row(gi, k, pmask);
    src_row[q] = (src_buffer(j, pmask) ? buf1 : buf0) + j * d;
  }

  float4 ra[CA][4];
  u32x4 rb[CB];

  auto load_global = [&](int kt) {
    const int k0 = kt * KS;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tid + q * NT;
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0 + 8 * (c & 3));
#pragma unroll
      for (int u = 0; u < 4; ++u) ra[q][u] = p[u];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      int pl = idx / (BN * 4), w = idx % (BN * 4);
      int col = w / 4, kc = w & 3;
      int64_t blk = 2 * int64_t(kt) + (kc >> 1);
      rb[q] = *reinterpret_cast<const u32x4*>(planes + pl * dd + (blk * d + j0 + col) * kPlaneBlock + 8 * (kc & 1));
    }
  };

  auto store_lds = [&]() {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tid + q * NT;
      int r = c / 4, kc = c & 3;
      typename S::v8 pc[NP];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float v[4] = {ra[q][u].x, ra[q][u].y, ra[q][u].z, ra[q][u].w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          typename S::elem o[S::P];
          S::split(v[2 * h], sigma, o);
#pragma unroll
          for (int pc2 = 0; pc2 < S::P; ++pc2) pc[2 * pc2][2 * u + h] = o[pc2];
          S::split(v[2 * h + 1], sigma, o);
#pragma unroll
          for (int pc2 = 0; pc2 < S::P; ++pc2) pc[2 * pc2 + 1][2 * u + h] = o[pc2];
        }
      }
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        *reinterpret_cast<typename S::v8*>(&As[(pl * BM + r) * ROW + 8 * kc]) = pc[pl];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * NT;
      int pl = idx / (BN * 4), w = idx % (BN * 4);
      int col = w / 4, kc = w & 3;
      *reinterpret_cast<u32x4*>(&Bs[(pl * BN + col) * ROW + 8 * kc]) = rb[q];
    }
  };

  f32x16 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc_re[x][y][v] = 0.f;
        acc_im[x][y][v] = 0.f;
      }

  const int nk = d / KS;
  load_global(0);
  store_lds();
  __syncthreads();

  const int lr = lane & 31, lk = (lane >> 5) * 8;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load_global(kt + 1);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int ko = kk * 16 + lk;
      typedef typename S::v8 V8;
      V8 av[FM][NP], bv[FN][NP], bneg[FN][S::P];
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int pl = 0; pl < NP; ++pl)
          av[x][pl] = *reinterpret_cast<const V8*>(&As[(pl * BM + wi0 + 32 * x + lr) * ROW + ko]);
#pragma unroll
      for (int y = 0; y < FN; ++y) {
#pragma unroll
        for (int pl = 0; pl < NP; ++pl)
          bv[y][pl] = *reinterpret_cast<const V8*>(&Bs[(pl * BN + wj0 + 32 * y + lr) * ROW + ko]);
#pragma unroll
        for (int pc = 0; pc < S::P; ++pc) bneg[y][pc] = negate(bv[y][2 * pc + 1]);
      }
      mma_pieces<S, FM, FN, C0>(acc_re, acc_im, av, bv, bneg);
    }
    __syncthreads();
    if (kt + 1 < nk) {
      store_lds();
      __syncthreads();
    }
  }

  store_tile<FM, FN>(acc_re, acc_im, buf0, buf1, M, d, k, pmask, i0 + wi0, j0 + wj0, lane, S::out_scale(sigma));
}

template <int BM, int BN, int WM, int WN, int C0 = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_ctrl_bf16x6(float2* __restrict__ buf0, float2* __restrict__ buf1, const uint16_t* __restrict__ planes, int n, int t,
              int k, uint64_t pmask) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_v1_tile<Bf16x6, BM, BN, WM, WN, C0>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_ctrl_f16x3(float2* __restrict__ buf0, float2* __restrict__ buf1, const uint16_t* __restrict__ planes, int n, int t,
             int k, uint64_t pmask, const float* __restrict__ sigma) {
  const int tiles_m = ((1 << (n - 1)) + BM - 1) / BM, tiles_n = (1 << t) / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  ctrl_v1_tile<F16x3, BM, BN, WM, WN>(buf0, buf1, planes, n, t, k, pmask, tile.x, tile.y, *sigma);
}

// Grouped controlled step k over the instances of a launch table; the tile
// shape follows the operator size class of the launch (d = 32, 64, >= 128;
// the last with the ping-pong schedule, or the in-step one when INSTEP:
// both give the same bits).
// The BK_NS_* kinds run the Newton-Schulz correction X E of power step
// `step` instead: X (complex64, in tbuf) rows [0, d) times the split planes of
// E, written to gbuf, through the prefix-doubling mapping of a t+1 qubit
// register.
template <int KIND, bool INSTEP = false, bool F16 = false>
__global__ void __launch_bounds__(KIND == BK_CTRL_M32 || KIND == BK_NS_M32 ? 256 : 512)
kb_ctrl_mixed(int step, const InstDesc* __restrict__ desc, const int32_t* __restrict__ table, int bflags,
              int64_t tile0) {
  constexpr bool NS = KIND == BK_NS_M32 || KIND == BK_NS_M64 || KIND == BK_NS_M128;
  constexpr int BN = (KIND == BK_CTRL_M32 || KIND == BK_NS_M32)   ? 32
                     : (KIND == BK_CTRL_M64 || KIND == BK_NS_M64) ? 64
                     : KIND == BK_CTRL_M256                       ? 256
                                                                  : 128;
  static_assert(KIND != BK_CTRL_M256 || F16, "128 x 256 tiles exist for split FP16 only");
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const bool dbl = NS || (bflags & kBatchDoubling) != 0;
  const RunLayout L = run_layout(D.n, D.t, true, (bflags & kBatchPolar) != 0);
  const uint16_t* planes = reinterpret_cast<const uint16_t*>(D.ws + L.planes);
  float2* s0;
  float2* s1;
  int n, k;
  if (NS) {
    s0 = reinterpret_cast<float2*>(D.ws + L.tbuf);
    s1 = reinterpret_cast<float2*>(D.ws + L.gbuf);
    n = D.t + 1;
    k = D.t;
  } else {
    s0 = reinterpret_cast<float2*>(D.ws + L.state0);
    // prefix doubling: rows [0, 2^k) -> rows [2^k, 2^(k+1)) of state0, as a
    // k+1 qubit register whose second buffer starts at row 2^k
    s1 = dbl ? s0 + (int64_t(1) << step) * (int64_t(1) << D.t) : reinterpret_cast<float2*>(D.ws + L.state1);
    n = dbl ? step + 1 : D.n;
    k = step;
  }
  const uint64_t pmask = dbl ? kDoubling : (uint64_t(1) << step) - 1;
  const int tiles_n = (1 << D.t) / BN;
  const int tm = int(local / tiles_n), tn = int(local % tiles_n);
  constexpr int C0 = NS ? 3 : 0;  // the Newton-Schulz product needs three piece pairs
  static_assert(!(NS && F16), "the Newton-Schulz product runs in split BF16");
  typedef typename std::conditional<F16, F16x3, Bf16x6>::type S;
  float sigma = 1.0f;
  if constexpr (F16) sigma = *reinterpret_cast<const float*>(D.ws + L.scratch + 8 * kScratchSigma);
  if constexpr (BN == 32)
    ctrl_v1_tile<S, 128, 32, 4, 1, C0>(s0, s1, planes, n, D.t, k, pmask, tm, tn, sigma);
  else if constexpr (BN == 64)
    ctrl_db_tile<S, 128, 64, 4, 2, true, C0>(s0, s1, planes, n, D.t, k, pmask, tm, tn, sigma);
  else if constexpr (BN == 256)
    ctrl_pp2_tile<S, 128, 256, 2, 4>(s0, s1, planes, n, D.t, k, pmask, tm, tn, sigma);
  else if constexpr (NS || INSTEP)
    ctrl_db_tile<S, 128, 128, 2, 4, true, C0>(s0, s1, planes, n, D.t, k, pmask, tm, tn, sigma);
  else
    ctrl_pp2_tile<S, 128, 128, 2, 4>(s0, s1, planes, n, D.t, k, pmask, tm, tn, sigma);
}

// The split-FP16 controlled step of the batch's instances with d = 2^t >=
// 256 (all of one t) on one persistent workgroup per CU: the workgroups take
// the launch's tiles in turn across the instances, each tile's buffers,
// operator and state scale from its instance's descriptor.
__global__ void __launch_bounds__(512) kb_ctrl_wide_persistent(int step, const InstDesc* __restrict__ desc,
                                                                const int32_t* __restrict__ table, int bflags,
                                                                int total, int t) {
  const bool dbl = (bflags & kBatchDoubling) != 0, pol = (bflags & kBatchPolar) != 0;
  ctrl_pp2p_tiles<F16x3, 128, 256, 2, 4>(t, total, [=](int L) {
    int64_t local;
    const int i = find_member(table, L, &local);
    const InstDesc D = load_desc(desc, i);
    const RunLayout R = run_layout(D.n, D.t, true, pol);
    float2* s0 = reinterpret_cast<float2*>(D.ws + R.state0);
    // prefix doubling: rows [0, 2^k) -> rows [2^k, 2^(k+1)) of state0
    float2* s1 = dbl ? s0 + (int64_t(1) << step) * (int64_t(1) << D.t) : reinterpret_cast<float2*>(D.ws + R.state1);
    const int tiles_n = (1 << D.t) / 256;
    return PTile{s0,
                 s1,
                 reinterpret_cast<const uint16_t*>(D.ws + R.planes),
                 dbl ? step + 1 : D.n,
                 step,
                 dbl ? kDoubling : (uint64_t(1) << step) - 1,
                 int(local / tiles_n),
                 int(local % tiles_n),
                 *reinterpret_cast<const float*>(D.ws + R.scratch + 8 * kScratchSigma)};
  });
}

template <int NT, typename K, typename... X>
hipError_t launch(K kernel, int BM, int BN, float2* buf0, float2* buf1, const uint16_t* planes, int n, int t, int k,
                  uint64_t pmask, hipStream_t s, X... extra) {
  int M = 1 << (n - 1);
  int tiles = ((M + BM - 1) / BM) * ((1 << t) / BN);
  hipLaunchKernelGGL(kernel, dim3(tiles), dim3(NT), 0, s, buf0, buf1, planes, n, t, k, pmask, extra...);
  return hipGetLastError();
}

// Split-FP16 controlled step: the tile choices of the default split-BF16
// path (variant 1: the 4-wave kernel throughout, 2: the in-step schedule
// for every size, 7: ping-pong for d >= 128; the BF16-only designs 3-6 fall
// back to the default), variant 8: the ping-pong schedule on 128 x 256 tiles
// (64 x 64 outputs per wave), whose matrix phase holds 48 MFMAs per wave
// like the split-BF16 kernel's (the 128 x 128 tile gives each phase only 24,
// and the fixed cost of a phase then weighs twice as much), and which reads
// the operator planes half as often per row; variant 9, the default from
// d = 256 on (launches of 512 tiles or more): variant 8 in its persistent
// form (2 % faster at c3, 0.3 % at c2).
// Compute units of the current device (the persistent kernel's grid).
int cu_count() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] <= 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cached[dev] = c;
  }
  return cached[dev];
}

hipError_t launch_ctrl_f16(float2* buf0, float2* buf1, const uint16_t* planes, int n, int t, int k, uint64_t pmask,
                           hipStream_t s, int variant, const float* sigma) {
  // Variants 7 and 8 choose the schedule of launches with enough tiles to
  // fill the chip (>= 256); smaller ones (early prefix-doubling steps) keep
  // the default choices.
  const int64_t wide_tiles = ((int64_t(1) << (n - 1)) + 127) / 128 * (t >= 8 ? (1 << t) / 256 : 0);
  const bool dflt = variant == 0 || (variant >= 3 && variant <= 6);
  if (t >= 8 && ((variant == 9 && wide_tiles >= 256) || (dflt && wide_tiles >= 512))) {
    // persistent: one workgroup per CU (a multiple of 8, for the XCD order)
    int g = cu_count() & ~7;
    if (g < 8) g = 8;
    if (int64_t(g) > wide_tiles) g = int(wide_tiles);
    hipLaunchKernelGGL((k_ctrl_f16x3_pp2p<128, 256, 2, 4>), dim3(g), dim3(512), 0, s, buf0, buf1, planes, n, t, k,
                       pmask, sigma);
    return hipGetLastError();
  }
  if (t >= 8 && variant == 8 && wide_tiles >= 256)
    return launch<512>(k_ctrl_f16x3_pp2<128, 256, 2, 4>, 128, 256, buf0, buf1, planes, n, t, k, pmask, s, sigma);
  if (variant >= 8) variant = 0;
  if (variant == 1) {
    if (t >= 7) return launch<256>(k_ctrl_f16x3<128, 128, 2, 2>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s, sigma);
    if (t == 6) return launch<256>(k_ctrl_f16x3<128, 64, 2, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s, sigma);
    if (t == 5) return launch<256>(k_ctrl_f16x3<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s, sigma);
    return hipErrorInvalidValue;
  }
  const int64_t big_tiles = ((int64_t(1) << (n - 1)) + 127) / 128 * (t >= 7 ? (1 << t) / 128 : 1);
  if (variant != 2 && t >= 6 && big_tiles < 256)
    return launch<256>(k_ctrl_f16x3<64, 64, 2, 2>, 64, 64, buf0, buf1, planes, n, t, k, pmask, s, sigma);
  if (t >= 7 && (variant == 7 || (variant != 2 && big_tiles >= 2048)))
    return launch<512>(k_ctrl_f16x3_pp2<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s, sigma);
  if (t >= 7)
    return launch<512>(k_ctrl_f16x3_db<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s, sigma);
  if (t == 6) return launch<512>(k_ctrl_f16x3_db<128, 64, 4, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s, sigma);
  if (t == 5) return launch<256>(k_ctrl_f16x3<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s, sigma);
  return hipErrorInvalidValue;
}

}  // namespace

int ctrl_mixed_variants() { return 9; }

hipError_t launch_ctrl_mixed(float2* buf0, float2* buf1, const uint16_t* planes, int n, int t, int k, uint64_t pmask,
                             hipStream_t s, int variant, const float* sigma_f16) {
  if (sigma_f16) return launch_ctrl_f16(buf0, buf1, planes, n, t, k, pmask, s, variant, sigma_f16);
  if (variant >= 8) variant = 0;  // the wide tiles are split-FP16 kernels
  if (variant == 1) {
    if (t >= 7) return launch<256>(k_ctrl_bf16x6<128, 128, 2, 2>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 6) return launch<256>(k_ctrl_bf16x6<128, 64, 2, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s);
    return hipErrorInvalidValue;
  }
  if (variant == 7) {
    // ping-pong with group-private state rows
    if (t >= 7) return launch<512>(k_ctrl_bf16x6_pp2<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 6) return launch<512>(k_ctrl_bf16x6_pp<128, 64, 4, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s);
    return hipErrorInvalidValue;
  }
  if (variant == 6) {
    // ping-pong wave groups
    if (t >= 7) return launch<512>(k_ctrl_bf16x6_pp<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 6) return launch<512>(k_ctrl_bf16x6_pp<128, 64, 4, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s);
    return hipErrorInvalidValue;
  }
  if (variant == 5) {
    // operator fragments straight from L2 into registers
    if (t >= 7) return launch<512>(k_ctrl_bf16x6_bg<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 6) return launch<512>(k_ctrl_bf16x6_bg<128, 64, 4, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s);
    return hipErrorInvalidValue;
  }
  if (variant == 4) {
    // triple-buffered, swizzled LDS
    if (t >= 7) return launch<512>(k_ctrl_bf16x6_tb<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 6) return launch<512>(k_ctrl_bf16x6_tb<128, 64, 4, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s);
    return hipErrorInvalidValue;
  }
  if (variant == 3) {
    // the double-buffered kernel with the compiler's own issue order
    if (t >= 7)
      return launch<512>(k_ctrl_bf16x6_db<128, 128, 2, 4, false>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 6)
      return launch<512>(k_ctrl_bf16x6_db<128, 64, 4, 2, false>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s);
    if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s);
    return hipErrorInvalidValue;
  }
  // Few rows (the Newton-Schulz correction X E, early prefix-doubling
  // steps): 64 x 64 tiles keep four times as many CUs busy.
  const int64_t big_tiles = ((int64_t(1) << (n - 1)) + 127) / 128 * (t >= 7 ? (1 << t) / 128 : 1);
  if (t >= 6 && big_tiles < 256)
    return launch<256>(k_ctrl_bf16x6<64, 64, 2, 2>, 64, 64, buf0, buf1, planes, n, t, k, pmask, s);
  // At eight or more tiles per CU the ping-pong kernel with group-private
  // state rows is a few per cent faster; below that (the middle
  // prefix-doubling steps) the interleaved one.
  if (variant == 0 && t >= 7 && big_tiles >= 2048)
    return launch<512>(k_ctrl_bf16x6_pp2<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
  if (t >= 7) return launch<512>(k_ctrl_bf16x6_db<128, 128, 2, 4>, 128, 128, buf0, buf1, planes, n, t, k, pmask, s);
  if (t == 6) return launch<512>(k_ctrl_bf16x6_db<128, 64, 4, 2>, 128, 64, buf0, buf1, planes, n, t, k, pmask, s);
  if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1>, 128, 32, buf0, buf1, planes, n, t, k, pmask, s);
  return hipErrorInvalidValue;
}

hipError_t launch_ns_product(float2* x32, float2* xe, const uint16_t* planes, int t, hipStream_t s) {
  // rows [0, d) of x32 times the planes, into rows [0, d) of xe: the
  // prefix-doubling mapping of a (t + 1)-qubit register
  const int n = t + 1;
  const uint64_t pmask = kDoubling;
  const int64_t big_tiles = (int64_t(1) << t) / 128 * (t >= 7 ? (1 << t) / 128 : 1);
  if (t >= 6 && big_tiles < 256)
    return launch<256>(k_ctrl_bf16x6<64, 64, 2, 2, 3>, 64, 64, x32, xe, planes, n, t, t, pmask, s);
  if (t >= 7)
    return launch<512>(k_ctrl_bf16x6_db<128, 128, 2, 4, true, 3>, 128, 128, x32, xe, planes, n, t, t, pmask, s);
  if (t == 6)
    return launch<512>(k_ctrl_bf16x6_db<128, 64, 4, 2, true, 3>, 128, 64, x32, xe, planes, n, t, t, pmask, s);
  if (t == 5) return launch<256>(k_ctrl_bf16x6<128, 32, 4, 1, 3>, 128, 32, x32, xe, planes, n, t, t, pmask, s);
  return hipErrorInvalidValue;
}

hipError_t launch_batch_ctrl_mixed(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                                   int bflags, hipStream_t s, int wide_t) {
  const int p = bflags;
  if ((bflags & kBatchF16) && kind == BK_CTRL_M256 && (bflags & kBatchPersistent) && wide_t >= 8 &&
      tiles >= 512 && tiles < (int64_t(1) << 31)) {
    int g = cu_count() & ~7;
    if (g < 8) g = 8;
    hipLaunchKernelGGL(kb_ctrl_wide_persistent, dim3(g), dim3(512), 0, s, step, desc, table, p, int(tiles), wide_t);
    return hipGetLastError();
  }
  if (bflags & kBatchF16) {
    switch (kind) {
      case BK_CTRL_M32:
        return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
          hipLaunchKernelGGL((kb_ctrl_mixed<BK_CTRL_M32, false, true>), dim3(g), dim3(256), 0, s, step, desc, table, p,
                             b);
        });
      case BK_CTRL_M64:
        return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
          hipLaunchKernelGGL((kb_ctrl_mixed<BK_CTRL_M64, false, true>), dim3(g), dim3(512), 0, s, step, desc, table, p,
                             b);
        });
      case BK_CTRL_M128:
        if (bflags & kBatchCtrlInStep)
          return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
            hipLaunchKernelGGL((kb_ctrl_mixed<BK_CTRL_M128, true, true>), dim3(g), dim3(512), 0, s, step, desc, table,
                               p, b);
          });
        return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
          hipLaunchKernelGGL((kb_ctrl_mixed<BK_CTRL_M128, false, true>), dim3(g), dim3(512), 0, s, step, desc, table, p,
                             b);
        });
      case BK_CTRL_M256:
        return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
          hipLaunchKernelGGL((kb_ctrl_mixed<BK_CTRL_M256, false, true>), dim3(g), dim3(512), 0, s, step, desc, table,
                             p, b);
        });
      default:
        break;  // the Newton-Schulz kinds run in split BF16
    }
  }
  switch (kind) {
    case BK_CTRL_M32:
      return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
        hipLaunchKernelGGL(kb_ctrl_mixed<BK_CTRL_M32>, dim3(g), dim3(256), 0, s, step, desc, table, p, b);
      });
    case BK_CTRL_M64:
      return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
        hipLaunchKernelGGL(kb_ctrl_mixed<BK_CTRL_M64>, dim3(g), dim3(512), 0, s, step, desc, table, p, b);
      });
    case BK_CTRL_M128:
      if (bflags & kBatchCtrlInStep)
        return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
          hipLaunchKernelGGL((kb_ctrl_mixed<BK_CTRL_M128, true>), dim3(g), dim3(512), 0, s, step, desc, table, p, b);
        });
      return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
        hipLaunchKernelGGL(kb_ctrl_mixed<BK_CTRL_M128>, dim3(g), dim3(512), 0, s, step, desc, table, p, b);
      });
    case BK_NS_M32:
      return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
        hipLaunchKernelGGL(kb_ctrl_mixed<BK_NS_M32>, dim3(g), dim3(256), 0, s, step, desc, table, p, b);
      });
    case BK_NS_M64:
      return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
        hipLaunchKernelGGL(kb_ctrl_mixed<BK_NS_M64>, dim3(g), dim3(512), 0, s, step, desc, table, p, b);
      });
    case BK_NS_M128:
      return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
        hipLaunchKernelGGL(kb_ctrl_mixed<BK_NS_M128>, dim3(g), dim3(512), 0, s, step, desc, table, p, b);
      });
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qpe
