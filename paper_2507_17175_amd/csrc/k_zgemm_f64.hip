// Complex FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// Serves the power chain V_{k+1} = V_k V_k, the Newton-Schulz products
// V^H V and V - V E / 2, and the FP64-form controlled step (rows of the state
// whose control bit is set, times V^T). A complex product is carried as three
// real MFMA products (Gauss) on three accumulators:
//   t1 += a.re b.re,  t2 += a.im b.im,  t3 += (a.re + a.im)(b.re + b.im),
// then re = t1 - t2 and im = t3 - t1 - t2 in the epilogue.
//
// Tiling: 256 or 512 threads = 4 or 8 wave64s in a WM x WN grid; the
// workgroup tile is BM x BN complex outputs, the K loop steps by BK = 16
// complex. Operands are staged in LDS as [k][i] / [k][j] (i or j
// contiguous, one double2 of padding per row), and the next K slab is
// prefetched into registers while the current one feeds the MFMAs. (A
// second LDS buffer, one barrier per slab instead of two, measured 2-4 %
// slower on every shape here: twice the LDS per workgroup leaves fewer
// workgroups per CU to cover the barriers.) The 1-D grid is remapped so that each of
// the 8 XCDs (which own separate L2 caches) walks a contiguous range of
// tiles, keeping the tiles of one row block on one XCD.
#include "qpe_internal.hpp"

namespace qpe {

namespace {


enum { OP_N = 0, OP_T = 1, OP_C = 2 };

struct GatherArgs {
  double2* buf0;
  double2* buf1;
  int k;
  uint64_t pmask;
};

// buf0 or buf1 by arithmetic on the addresses: a plain select between two
// fields of the by-value argument struct compiles into a per-lane load of
// the pointer from the argument segment, then a wait, then the data load.
__device__ inline double2* pick(const GatherArgs& g, int which) {
  uintptr_t b0 = reinterpret_cast<uintptr_t>(g.buf0);
  uintptr_t delta = reinterpret_cast<uintptr_t>(g.buf1) - b0;
  return reinterpret_cast<double2*>(b0 + (which ? delta : uintptr_t(0)));
}

__device__ inline int2 xcd_tile_of(int w, int tiles_m, int tiles_n) {
  const int total = tiles_m * tiles_n;
  if ((total & 7) == 0) w = (w & 7) * (total >> 3) + (w >> 3);
  return make_int2(w / tiles_n, w % tiles_n);
}

// Epilogue of a wave's FM x FN blocks of 16 x 16 outputs whose first row and
// column are row0 and col0: re = t1 - t2, im = t3 - t1 - t2, then alpha, beta,
// the Hermitian mirror, the gather mapping or the operator planes.
template <bool GATHER, int FM, int FN>
__device__ __forceinline__ void zgemm_epilogue(const ZgemmArgs& a, const GatherArgs& g,
                                               const f64x4 (&acc_t1)[FM][FN], const f64x4 (&acc_t2)[FM][FN],
                                               const f64x4 (&acc_t3)[FM][FN], int row0, int col0, int lr, int lk) {
  // Output layout of the 16x16 f64 MFMA: lane l, element v holds
  // row 4 * v + l / 16, column l % 16 of the block.
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int gi = row0 + x * 16 + 4 * v + lk;
        int gj = col0 + y * 16 + lr;
        if (gi >= a.M || gj >= a.N) continue;
        const double t1 = acc_t1[x][y][v], t2 = acc_t2[x][y][v];
        double re = t1 - t2, im = acc_t3[x][y][v] - t1 - t2;
        if (GATHER) {
          int64_t j = step_row(gi, g.k, g.pmask);
          double2* dst = pick(g, 1 - src_buffer(j, g.pmask));
          dst[j * a.ldc + gj] = make_double2(re, im);
        } else {
          double2 o;
          o.x = a.alpha.x * re - a.alpha.y * im;
          o.y = a.alpha.x * im + a.alpha.y * re;
          if (a.beta.x != 0.0 || a.beta.y != 0.0) {
            double2 c = a.Cin[int64_t(gi) * a.ldcin + gj];
            o.x += a.beta.x * c.x - a.beta.y * c.y;
            o.y += a.beta.x * c.y + a.beta.y * c.x;
          }
          // Hermitian product: only tiles on or above the diagonal run; an
          // element below the diagonal is always the conjugate of the one
          // above it (never computed directly, also inside a diagonal tile),
          // so the result does not depend on the tile size (the Gauss form
          // rounds C[i][j] and conj(C[j][i]) differently).
          if (a.herm && gi > gj) continue;
          a.C[int64_t(gi) * a.ldc + gj] = o;
          if (a.herm && gi < gj) a.C[int64_t(gj) * a.ldc + gi] = make_double2(o.x, -o.y);
          if (a.planes) {
            // the operator split of the next controlled step, from the
            // values just stored (lanes of one row write 16 contiguous
            // entries of a plane)
            uint16_t q[4];
            split_f16_pieces(o, q);
            const int64_t dd = int64_t(a.N) * a.N, off = plane_offset(a.N, gi, gj);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) a.planes[pl * dd + off] = q[pl];
          }
        }
      }
}

template <int OPA, int OPB, bool GATHER, int BM, int BN, int WM, int WN, int kBK = 16>
__device__ __forceinline__ void zgemm_tile(const ZgemmArgs& a, const GatherArgs& g, int tile_m, int tile_n) {
  constexpr int kThreads = 64 * WM * WN;
  static_assert(WM * WN == 4 || WM * WN == 8, "4 or 8 waves");
  constexpr int TM = BM / WM, TN = BN / WN;  // wave tile
  constexpr int FM = TM / 16, FN = TN / 16;  // 16x16 MFMA blocks per wave
  constexpr int LA = BM * kBK / kThreads;    // A elements per thread per slab
  constexpr int LB = BN * kBK / kThreads;
  static_assert(LA * kThreads == BM * kBK && LB * kThreads == BN * kBK, "tile/thread mismatch");
  constexpr int PA = BM + 1, PB = BN + 1;    // padded LDS row length

  __shared__ double2 As[kBK * PA];
  __shared__ double2 Bs[kBK * PB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = tile_m * BM, j0 = tile_n * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;

  // Per-thread A row pointers (gather mode: rows of the state).
  double2 ra[LA], rb[LB];

  auto load_a = [&](int k0) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      int idx = tid + q * kThreads;
      int r, kk;
      if (OPA == OP_N) {
        r = idx / kBK;
        kk = idx % kBK;
      } else {
        kk = idx / BM;
        r = idx % BM;
      }
      int gi = i0 + r, gk = k0 + kk;
      // Out-of-range elements load a clamped in-range address and are
      // zeroed by a select: the load itself stays unconditional (a guarded
      // load becomes a branch after which the compiler waits for every
      // outstanding load).
      const bool ok = gi < a.M && gk < a.K;
      const int ci = min(gi, a.M - 1), ck = min(gk, a.K - 1);
      double2 v;
      if (GATHER) {
        int64_t j = step_row(ci, g.k, g.pmask);
        v = pick(g, src_buffer(j, g.pmask))[j * a.lda + ck];
      } else if (OPA == OP_N) {
        v = a.A[int64_t(ci) * a.lda + ck];
      } else {
        v = a.A[int64_t(ck) * a.lda + ci];
        if (OPA == OP_C) v.y = -v.y;
      }
      ra[q] = ok ? v : make_double2(0.0, 0.0);
    }
  };
  auto store_a = [&]() {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      int idx = tid + q * kThreads;
      int r, kk;
      if (OPA == OP_N) {
        r = idx / kBK;
        kk = idx % kBK;
      } else {
        kk = idx / BM;
        r = idx % BM;
      }
      As[kk * PA + r] = ra[q];
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      int idx = tid + q * kThreads;
      int c, kk;
      if (OPB == OP_N) {
        kk = idx / BN;
        c = idx % BN;
      } else {
        c = idx / kBK;
        kk = idx % kBK;
      }
      int gj = j0 + c, gk = k0 + kk;
      const bool ok = gj < a.N && gk < a.K;
      const int cj = min(gj, a.N - 1), ck = min(gk, a.K - 1);
      double2 v;
      if (OPB == OP_N) {
        v = a.B[int64_t(ck) * a.ldb + cj];
      } else {
        v = a.B[int64_t(cj) * a.ldb + ck];
        if (OPB == OP_C) v.y = -v.y;
      }
      rb[q] = ok ? v : make_double2(0.0, 0.0);
    }
  };
  auto store_b = [&]() {
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      int idx = tid + q * kThreads;
      int c, kk;
      if (OPB == OP_N) {
        kk = idx / BN;
        c = idx % BN;
      } else {
        c = idx / kBK;
        kk = idx % kBK;
      }
      Bs[kk * PB + c] = rb[q];
    }
  };

  // Three real products per complex product (Gauss): with a = ar + i ai and
  // b = br + i bi, t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar + ai)(br + bi),
  // then re = t1 - t2 and im = t3 - t1 - t2 (normwise as accurate as the
  // four-product form, within a small constant factor).
  f64x4 acc_t1[FM][FN], acc_t2[FM][FN], acc_t3[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) {
      acc_t1[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
      acc_t2[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
      acc_t3[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
    }

  const int nk = (a.K + kBK - 1) / kBK;
  load_a(0);
  load_b(0);
  store_a();
  store_b();
  __syncthreads();

  const int lr = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) {
      load_a((kt + 1) * kBK);
      load_b((kt + 1) * kBK);
    }
#pragma unroll
    for (int k4 = 0; k4 < kBK / 4; ++k4) {
      const int kr = k4 * 4 + lk;
      double2 av[FM], bv[FN];
      double as[FM], bs[FN];
#pragma unroll
      for (int x = 0; x < FM; ++x) {
        av[x] = As[kr * PA + wi0 + x * 16 + lr];
        as[x] = av[x].x + av[x].y;
      }
#pragma unroll
      for (int y = 0; y < FN; ++y) {
        bv[y] = Bs[kr * PB + wj0 + y * 16 + lr];
        bs[y] = bv[y].x + bv[y].y;
      }
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) {
          acc_t1[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].x, bv[y].x, acc_t1[x][y], 0, 0, 0);
          acc_t2[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].y, bv[y].y, acc_t2[x][y], 0, 0, 0);
          acc_t3[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[x], bs[y], acc_t3[x][y], 0, 0, 0);
        }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      store_a();
      store_b();
      __syncthreads();
    }
  }

  zgemm_epilogue<GATHER, FM, FN>(a, g, acc_t1, acc_t2, acc_t3, i0 + wi0, j0 + wj0, lr, lk);
}

// Tile (row, column) of workgroup w among the T (T + 1) / 2 tiles on or above
// the diagonal of a T x T tile grid, row by row.
__device__ inline int2 upper_tile(int w, int T) {
  int tm = 0;
  while (w >= T - tm) {
    w -= T - tm;
    ++tm;
  }
  return make_int2(tm, tm + w);
}

template <int OPA, int OPB, bool GATHER, int BM, int BN, int WM, int WN, int BK>
__global__ void __launch_bounds__(64 * WM * WN) k_zgemm(ZgemmArgs a, GatherArgs g) {
  const int tiles_m = (a.M + BM - 1) / BM, tiles_n = (a.N + BN - 1) / BN;
  const int2 tile = a.herm ? upper_tile(blockIdx.x, tiles_m) : xcd_tile_of(blockIdx.x, tiles_m, tiles_n);
  zgemm_tile<OPA, OPB, GATHER, BM, BN, WM, WN, BK>(a, g, tile.x, tile.y);
}

// Zeros over the 64 x 64 tile (tm, tn) of a d x d matrix and its mirror.
template <int NT>
__device__ inline void zero_tile64(double2* C, int d, int tm, int tn) {
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e >> 6, j = e & 63;
    C[int64_t(tm * 64 + i) * d + tn * 64 + j] = make_double2(0.0, 0.0);
    C[int64_t(tn * 64 + i) * d + tm * 64 + j] = make_double2(0.0, 0.0);
  }
}

// Run `part` of the stream-K plan of G = X^H X (gram_split(t)): its slab
// units, tile by tile, each tile's share added into the run's slot of that
// tile (slot 0: G, slot s >= 1: G2 + (s - 1) d^2); the run that holds a
// tile's last slab also clears the tile's slots beyond its own.
template <int WM, int WN>
__device__ void gram_run(const double2* X, double2* G, double2* G2, int t, int64_t part) {
  const GramPlan P = gram_plan(t);
  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  ZgemmArgs a{};
  a.M = a.N = d;
  a.lda = a.ldb = a.ldc = a.ldcin = d;
  a.alpha = make_double2(1.0, 0.0);
  a.beta = make_double2(0.0, 0.0);
  a.herm = 1;
  GatherArgs g{};
  int64_t x = part * P.W;
  const int64_t x1 = min(x + P.W, P.total);
  while (x < x1) {
    const int64_t u = x / P.nk;
    const int k0 = int(x - u * P.nk);
    const int k1 = int(min(int64_t(P.nk), k0 + (x1 - x)));
    const int slot = int(part - u * P.nk / P.W);
    const int2 tile = upper_tile(int(u), P.T);
    // op(A) = X^H: element (k, i) is conj(X[k][i]); op(B) = X: (k, j) is X[k][j]
    a.A = X + int64_t(k0) * 16 * d;
    a.B = X + int64_t(k0) * 16 * d;
    a.K = (k1 - k0) * 16;
    a.C = slot == 0 ? G : G2 + (slot - 1) * dd;
    zgemm_tile<OP_C, OP_N, false, 64, 64, WM, WN>(a, g, tile.x, tile.y);
    if (k1 == P.nk)
      for (int sl = slot + 1; sl < P.slots; ++sl) zero_tile64<64 * WM * WN>(G2 + (sl - 1) * dd, d, tile.x, tile.y);
    x += k1 - k0;
  }
}

__global__ void __launch_bounds__(512) k_gram_split(const double2* __restrict__ X, double2* __restrict__ G,
                                                    double2* __restrict__ G2, int t) {
  gram_run<4, 2>(X, G, G2, t, blockIdx.x);
}

// ---- grouped (batched) forms: one launch over the instances of a table ----

// Power-chain products of step k for every instance that takes part, with
// 32 x 32 tiles: BK_SQ  X_k = V_{k-1} V_{k-1};  BK_GRAM  G = X^H X;
// BK_CORR  V_k = X - X (G - I) / 2.
// G64: instances with d >= 64 take 64 x 64 tiles (4 waves, 32 x 32 each),
// the others 32 x 32; the tile shape does not change the order of any sum.
template <int KIND, bool G64>
__global__ void __launch_bounds__(256) kb_zgemm(int step, const InstDesc* __restrict__ desc,
                                                const int32_t* __restrict__ table, int mixed, int bflags,
                                                int64_t tile0) {
  constexpr int OPA = KIND == BK_GRAM ? OP_C : OP_N;
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const bool pol = (bflags & kBatchPolar) != 0;
  const RunLayout L = run_layout(D.n, D.t, mixed != 0, pol);
  const int d = 1 << D.t;
  const bool big = G64 && D.t >= 6;
  const int T = big ? 64 : kBatchGemmTile;
  const int tiles_n = int((d + T - 1) / T);
  double2* vbuf = reinterpret_cast<double2*>(D.ws + L.vbuf);
  double2* tbuf = reinterpret_cast<double2*>(D.ws + L.tbuf);
  double2* gbuf = reinterpret_cast<double2*>(D.ws + L.gbuf);
  ZgemmArgs a{};
  a.M = a.N = a.K = d;
  a.lda = a.ldb = a.ldc = a.ldcin = d;
  a.alpha = make_double2(1.0, 0.0);
  a.beta = make_double2(0.0, 0.0);
  if (KIND == BK_SQ) {
    const int src = power_slot(step - 1, pol);
    const double2* cur = src == 0 ? D.U : (src == 1 ? vbuf : tbuf);
    a.A = a.B = cur;
    a.C = pol ? vbuf : (power_slot(step, pol) == 1 ? vbuf : tbuf);
  } else if (KIND == BK_GRAM) {
    a.A = a.B = vbuf;
    a.C = gbuf;
  } else {  // BK_CORR
    a.A = vbuf;
    a.B = gbuf;
    a.alpha = make_double2(-0.5, 0.0);
    a.beta = make_double2(1.0, 0.0);
    a.Cin = vbuf;
    a.C = tbuf;
  }
  GatherArgs g{};
  if (KIND == BK_GRAM) {
    a.herm = 1;
    const int2 tile = upper_tile(int(local), tiles_n);
    if constexpr (G64) {
      if (big) {
        zgemm_tile<OPA, OP_N, false, 64, 64, 2, 2>(a, g, tile.x, tile.y);
        return;
      }
    }
    zgemm_tile<OPA, OP_N, false, kBatchGemmTile, kBatchGemmTile, 2, 2>(a, g, tile.x, tile.y);
  } else {
    if constexpr (G64) {
      if (big) {
        zgemm_tile<OPA, OP_N, false, 64, 64, 2, 2>(a, g, int(local / tiles_n), int(local % tiles_n));
        return;
      }
    }
    zgemm_tile<OPA, OP_N, false, kBatchGemmTile, kBatchGemmTile, 2, 2>(a, g, int(local / tiles_n),
                                                                       int(local % tiles_n));
  }
}

// Gram products of step k by the stream-K plan (gram_split instances): run
// `local` of the instance, with the single-instance path's workgroup shape.
__global__ void __launch_bounds__(512) kb_gram_split(int step, const InstDesc* __restrict__ desc,
                                                     const int32_t* __restrict__ table, int mixed, int bflags,
                                                     int64_t tile0) {
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const RunLayout L = run_layout(D.n, D.t, mixed != 0, (bflags & kBatchPolar) != 0);
  gram_run<4, 2>(reinterpret_cast<const double2*>(D.ws + L.vbuf), reinterpret_cast<double2*>(D.ws + L.gbuf),
                 reinterpret_cast<double2*>(D.ws + L.gbuf2), D.t, local);
}

// FP64-form controlled step k with 64 x 64 tiles.
__global__ void __launch_bounds__(256) kb_ctrl_f64(int step, const InstDesc* __restrict__ desc,
                                                   const int32_t* __restrict__ table, int bflags, int64_t tile0) {
  int64_t local;
  const int i = find_member(table, tile0 + blockIdx.x, &local);
  const InstDesc D = load_desc(desc, i);
  const bool pol = (bflags & kBatchPolar) != 0, dbl = (bflags & kBatchDoubling) != 0;
  const RunLayout L = run_layout(D.n, D.t, false, pol);
  const int d = 1 << D.t;
  const int slot = power_slot(step, pol);
  ZgemmArgs a{};
  a.M = dbl ? (1 << step) : (1 << (D.n - 1));
  a.N = a.K = d;
  a.lda = a.ldb = a.ldc = d;
  a.B = slot == 0 ? D.U : reinterpret_cast<const double2*>(D.ws + (slot == 1 ? L.vbuf : L.tbuf));
  double2* s0 = reinterpret_cast<double2*>(D.ws + L.state0);
  // prefix doubling: rows [0, 2^k) -> rows [2^k, 2^(k+1)) of state0
  GatherArgs g{s0, dbl ? s0 + (int64_t(1) << step) * d : reinterpret_cast<double2*>(D.ws + L.state1), step,
               dbl ? kDoubling : (uint64_t(1) << step) - 1};
  const int tiles_n = (d + 63) / 64;
  zgemm_tile<OP_N, OP_T, true, 64, 64, 2, 2>(a, g, int(local / tiles_n), int(local % tiles_n));
}

template <int OPA, int OPB, bool GATHER, int BM, int BN, int WM, int WN, int BK = 16>
hipError_t go(const ZgemmArgs& a_in, const GatherArgs& g, hipStream_t s) {
  ZgemmArgs a = a_in;
  // the Hermitian shortcut needs square tiles on a square product
  if (a.herm && (BM != BN || a.M != a.N)) a.herm = 0;
  const int T = (a.M + BM - 1) / BM;
  const int tiles = a.herm ? T * (T + 1) / 2 : T * ((a.N + BN - 1) / BN);
  hipLaunchKernelGGL((k_zgemm<OPA, OPB, GATHER, BM, BN, WM, WN, BK>), dim3(tiles), dim3(64 * WM * WN), 0, s, a, g);
  return hipGetLastError();
}

// Tile variants of the power-chain GEMM: (BM, BN, waves, K slab).
//   1: 32x32, 4 waves, 16   2: 64x64, 4 waves, 16   3: 64x64, 8 waves, 16
//   4: 128x64, 8 waves, 16  5: 64x32, 4 waves, 16   6: 64x64, 8 waves, 32
//   7: 32x32, 4 waves, 32
// The K slab only groups the MFMA steps between barriers; every variant
// accumulates each output over K in the same order.
template <int OPA, int OPB>
hipError_t dispatch_size(const ZgemmArgs& a, hipStream_t s, int variant) {
  GatherArgs g{};
  if (variant == 0) {
    // Default (measured on MI355X): 64x64 tiles with 8 waves once there
    // are >= 128 of them (X = V V at d = 1024: 122-126 us against 144-152 us
    // on 32x32 tiles; d = 2048: 829 vs 1019 us), 32x32 tiles below (d = 256:
    // 15.0 us with 32-deep K slabs, 16.6 us with 16-deep, 31.6 us on 64x64).
    // A Hermitian product runs only the tiles on or above the diagonal, so
    // it needs a larger grid before 64x64 tiles fill the chip (the Gram
    // products at d = 1024 and 2048 take the stream-K plan instead).
    // The 32-deep slab halves the barriers of the small tiles; with K < 32
    // it would only add zero steps.
    const int64_t t64 = (a.M + 63) / 64;
    const int small = a.K >= 32 ? 7 : 1;
    if (a.herm && a.M == a.N)
      variant = t64 * (t64 + 1) / 2 >= 256 ? 3 : small;
    else
      variant = t64 * ((a.N + 63) / 64) >= 128 ? 3 : small;
  }
  // A Hermitian product mirrors inside square tiles only; the rectangular
  // variants run it on the square tile of their class, so that every
  // variant gives the same bits (the Gauss form rounds C[i][j] and
  // conj(C[j][i]) differently, so computing both directly would not).
  if (a.herm && variant == 4) variant = 3;
  if (a.herm && variant == 5) variant = 1;
  switch (variant) {
    case 1: return go<OPA, OPB, false, 32, 32, 2, 2>(a, g, s);
    case 2: return go<OPA, OPB, false, 64, 64, 2, 2>(a, g, s);
    case 3: return go<OPA, OPB, false, 64, 64, 4, 2>(a, g, s);
    case 4: return go<OPA, OPB, false, 128, 64, 4, 2>(a, g, s);
    case 5: return go<OPA, OPB, false, 64, 32, 2, 2>(a, g, s);
    case 6: return go<OPA, OPB, false, 64, 64, 4, 2, 32>(a, g, s);
    case 7: return go<OPA, OPB, false, 32, 32, 2, 2, 32>(a, g, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int zgemm_variants() { return 7; }
int ctrl_f64_variants() { return 2; }

hipError_t launch_zgemm(int opA, int opB, const ZgemmArgs& a, hipStream_t s, int variant) {
  switch (opA * 3 + opB) {
    case 0: return dispatch_size<OP_N, OP_N>(a, s, variant);
    case 1: return dispatch_size<OP_N, OP_T>(a, s, variant);
    case 2: return dispatch_size<OP_N, OP_C>(a, s, variant);
    case 3: return dispatch_size<OP_T, OP_N>(a, s, variant);
    case 4: return dispatch_size<OP_T, OP_T>(a, s, variant);
    case 5: return dispatch_size<OP_T, OP_C>(a, s, variant);
    case 6: return dispatch_size<OP_C, OP_N>(a, s, variant);
    case 7: return dispatch_size<OP_C, OP_T>(a, s, variant);
    case 8: return dispatch_size<OP_C, OP_C>(a, s, variant);
  }
  return hipErrorInvalidValue;
}

// Controlled step variants: 1: 64x64, 4 waves; 2: 128x64, 8 waves (the
// default: with three accumulator sets per tile the 4-wave variant needs 280
// VGPRs and runs one wave per SIMD: 3.4 ms vs 4.8 ms per step at n = 16,
// t = 10). Small sizes fall back to 32x32 tiles.
hipError_t launch_ctrl_f64(double2* buf0, double2* buf1, const double2* V, int n, int t, int k, uint64_t pmask,
                           hipStream_t s, int variant) {
  const int d = 1 << t;
  ZgemmArgs a{};
  a.M = 1 << (n - 1);
  a.N = d;
  a.K = d;
  a.lda = d;
  a.B = V;
  a.ldb = d;
  a.ldc = d;
  GatherArgs g{buf0, buf1, k, pmask};
  if (a.M < 128 || d < 64) return go<OP_N, OP_T, true, 32, 32, 2, 2>(a, g, s);
  if (variant == 0) variant = 2;
  switch (variant) {
    case 1: return go<OP_N, OP_T, true, 64, 64, 2, 2>(a, g, s);
    case 2: return go<OP_N, OP_T, true, 128, 64, 4, 2>(a, g, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gram_split(const double2* X, double2* G, double2* G2, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_split, dim3(gram_parts(t)), dim3(512), 0, s, X, G, G2, t);
  return hipGetLastError();
}

hipError_t launch_batch_gram_split(int step, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                                   int bflags, hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    hipLaunchKernelGGL(kb_gram_split, dim3(g), dim3(512), 0, s, step, desc, table, mixed ? 1 : 0, bflags, b);
  });
}

hipError_t launch_batch_zgemm(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                              bool mixed, int bflags, hipStream_t s) {
  const int m = mixed ? 1 : 0, p = bflags;
  const bool g64 = (bflags & kBatchGemm64) != 0;
  auto go_kind = [&](auto kernel) {
    return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
      hipLaunchKernelGGL(kernel, dim3(g), dim3(256), 0, s, step, desc, table, m, p, b);
    });
  };
  switch (kind) {
    case BK_SQ:
      return g64 ? go_kind(kb_zgemm<BK_SQ, true>) : go_kind(kb_zgemm<BK_SQ, false>);
    case BK_GRAM:
      return g64 ? go_kind(kb_zgemm<BK_GRAM, true>) : go_kind(kb_zgemm<BK_GRAM, false>);
    case BK_CORR:
      return g64 ? go_kind(kb_zgemm<BK_CORR, true>) : go_kind(kb_zgemm<BK_CORR, false>);
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_ctrl_f64(int step, const InstDesc* desc, const int32_t* table, int64_t tiles, int bflags,
                                 hipStream_t s) {
  return for_grid_chunks(tiles, [&](unsigned g, int64_t b) {
    hipLaunchKernelGGL(kb_ctrl_f64, dim3(g), dim3(256), 0, s, step, desc, table, bflags, b);
  });
}

}  // namespace qpe
