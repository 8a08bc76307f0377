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
// Tiling: 4 wave64s, workgroup tile BM rows x BN complex columns, K slab of
// 32 complex. The FP32 A slab is split into 6 BF16 planes (3 pieces x re/im)
// as it is written to LDS; the B slab arrives pre-split and pre-blocked from
// HBM. LDS rows are padded to 80 bytes so that the 16-byte fragment reads of
// 32 consecutive rows hit distinct banks. The state ping-pongs between two
// buffers (read buf[parity], write the other), so there is no copy-back and
// no read-after-write hazard between workgroups that share rows.
#include "qpe_internal.hpp"

namespace qpe {

namespace {

constexpr int kThreads = 256;
constexpr int kBK = 32;   // complex K per slab (= blocking of the operator planes)
constexpr int kRow = 40;  // padded LDS row, in bf16 elements (80 bytes)

typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

__device__ inline void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  float r1 = x - (float)h;
  m = (__bf16)r1;
  float r2 = r1 - (float)m;
  l = (__bf16)r2;
}

__device__ inline bf16x8 negate(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= (u32x4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(bf16x8, u);
}

__device__ inline int2 xcd_tile(int tiles_m, int tiles_n) {
  const int total = tiles_m * tiles_n;
  int w = blockIdx.x;
  if ((total & 7) == 0) w = (w & 7) * (total >> 3) + (w >> 3);
  return make_int2(w / tiles_n, w % tiles_n);
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_ctrl_bf16x6(float2* __restrict__ buf0, float2* __restrict__ buf1, const uint16_t* __restrict__ planes, int n, int t,
              int k, uint64_t pmask) {
  static_assert(WM * WN == 4, "4 waves");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int CA = BM * 4 / kThreads;        // 8-complex A chunks per thread
  constexpr int CB = 6 * BN * 4 / kThreads;    // 16-byte B chunks per thread
  static_assert(CA >= 1 && CB >= 1, "tile too small");

  __shared__ __attribute__((aligned(16))) uint16_t As[6 * BM * kRow];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[6 * BN * kRow];

  const int d = 1 << t;
  const int64_t dd = int64_t(d) * d;
  const int M = 1 << (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_m = (M + BM - 1) / BM, tiles_n = d / BN;
  const int2 tile = xcd_tile(tiles_m, tiles_n);
  const int i0 = tile.x * BM, j0 = tile.y * BN;
  const int wi0 = (wave / WN) * TM, wj0 = (wave % WN) * TN;

  // Source row pointers of this thread's A chunks.
  const float2* src_row[CA];
  bool row_ok[CA];
#pragma unroll
  for (int q = 0; q < CA; ++q) {
    int c = tid + q * kThreads;
    int gi = i0 + c / 4;
    row_ok[q] = gi < M;
    int64_t j = ctrl_row(row_ok[q] ? gi : 0, k);
    src_row[q] = (row_parity(j, pmask) ? buf1 : buf0) + j * d;
  }

  float4 ra[CA][4];
  u32x4 rb[CB];

  auto load_global = [&](int kt) {
    const int k0 = kt * kBK;
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tid + q * kThreads;
      const float4* p = reinterpret_cast<const float4*>(src_row[q] + k0 + 8 * (c & 3));
#pragma unroll
      for (int u = 0; u < 4; ++u) ra[q][u] = row_ok[q] ? p[u] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * kThreads;
      int pl = idx / (BN * 4), w = idx % (BN * 4);
      const u32x4* p = reinterpret_cast<const u32x4*>(planes + pl * dd + (int64_t(kt) * d + j0) * kBK) + w;
      rb[q] = *p;
    }
  };

  auto store_lds = [&]() {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      int c = tid + q * kThreads;
      int r = c / 4, kc = c & 3;
      bf16x8 pc[6];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float v[4] = {ra[q][u].x, ra[q][u].y, ra[q][u].z, ra[q][u].w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          __bf16 a, b, cc;
          split3(v[2 * h], a, b, cc);       // real part
          pc[0][2 * u + h] = a;
          pc[2][2 * u + h] = b;
          pc[4][2 * u + h] = cc;
          split3(v[2 * h + 1], a, b, cc);   // imaginary part
          pc[1][2 * u + h] = a;
          pc[3][2 * u + h] = b;
          pc[5][2 * u + h] = cc;
        }
      }
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        *reinterpret_cast<bf16x8*>(&As[(pl * BM + r) * kRow + 8 * kc]) = pc[pl];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      int idx = tid + q * kThreads;
      int pl = idx / (BN * 4), w = idx % (BN * 4);
      int col = w / 4, kc = w & 3;
      *reinterpret_cast<u32x4*>(&Bs[(pl * BN + col) * kRow + 8 * kc]) = rb[q];
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

  const int nk = d / kBK;
  load_global(0);
  store_lds();
  __syncthreads();

  const int lr = lane & 31, lk = (lane >> 5) * 8;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load_global(kt + 1);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int ko = kk * 16 + lk;
      bf16x8 av[FM][6];
      bf16x8 bv[FN][6], bneg[FN][3];
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int pl = 0; pl < 6; ++pl)
          av[x][pl] = *reinterpret_cast<const bf16x8*>(&As[(pl * BM + wi0 + 32 * x + lr) * kRow + ko]);
#pragma unroll
      for (int y = 0; y < FN; ++y) {
#pragma unroll
        for (int pl = 0; pl < 6; ++pl)
          bv[y][pl] = *reinterpret_cast<const bf16x8*>(&Bs[(pl * BN + wj0 + 32 * y + lr) * kRow + ko]);
#pragma unroll
        for (int pc = 0; pc < 3; ++pc) bneg[y][pc] = negate(bv[y][2 * pc + 1]);
      }
      // piece pairs (A piece, B piece) with index sum <= 2
      constexpr int PA[6] = {2, 1, 0, 1, 0, 0};
      constexpr int PB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
      for (int c = 0; c < 6; ++c) {
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
    __syncthreads();
    if (kt + 1 < nk) {
      store_lds();
      __syncthreads();
    }
  }

  // Epilogue. Output layout of the 32x32 MFMA: lane l, element v holds row
  // 8 * (v / 4) + 4 * (l / 32) + v % 4, column l % 32 of the block.
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      int gi = i0 + wi0 + 32 * x + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (gi >= M) continue;
      int64_t j = ctrl_row(gi, k);
      float2* dst = (row_parity(j, pmask) ? buf0 : buf1) + j * d + j0 + wj0 + lr;
#pragma unroll
      for (int y = 0; y < FN; ++y) dst[32 * y] = make_float2(acc_re[x][y][v], acc_im[x][y][v]);
    }
}

template <int BM, int BN, int WM, int WN>
hipError_t go(float2* buf0, float2* buf1, const uint16_t* planes, int n, int t, int k, uint64_t pmask,
              hipStream_t s) {
  int M = 1 << (n - 1);
  int tiles = ((M + BM - 1) / BM) * ((1 << t) / BN);
  hipLaunchKernelGGL((k_ctrl_bf16x6<BM, BN, WM, WN>), dim3(tiles), dim3(kThreads), 0, s, buf0, buf1, planes, n, t, k,
                     pmask);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ctrl_mixed(float2* buf0, float2* buf1, const uint16_t* planes, int n, int t, int k, uint64_t pmask,
                             hipStream_t s) {
  if (t >= 7) return go<128, 128, 2, 2>(buf0, buf1, planes, n, t, k, pmask, s);
  if (t == 6) return go<128, 64, 2, 2>(buf0, buf1, planes, n, t, k, pmask, s);
  if (t == 5) return go<128, 32, 4, 1>(buf0, buf1, planes, n, t, k, pmask, s);
  return hipErrorInvalidValue;
}

}  // namespace qpe
