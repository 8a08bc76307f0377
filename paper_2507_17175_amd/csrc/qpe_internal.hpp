// Internal declarations shared by the HIP translation units of libqpe.
// Host-side launchers return the hipError_t of the launch; device helpers are
// header-inline so each kernel file stays self-contained.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qpe {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

// Pass schedule of the inverse DFT along the measurement axis: pass q is a
// radix-2^bits[q] pass; sum of bits = n. After all passes, row position p
// holds outcome m = digit_reverse(p) (see prob_index).
struct DftPlan {
  int npass;
  int bits[8];
};

// Row position after the DFT passes -> outcome index m.
// Digit q of p sits in bits [n - B_{q+1}, n - B_q) of p (B_q = bits[0] + ...
// + bits[q-1]) and moves to bits [B_q, B_{q+1}) of m.
__host__ __device__ inline int64_t prob_index(int64_t p, int n, const DftPlan& plan) {
  int64_t m = 0;
  int hi = n, lo = 0;
  for (int q = 0; q < plan.npass; ++q) {
    hi -= plan.bits[q];
    int64_t digit = (p >> hi) & ((int64_t(1) << plan.bits[q]) - 1);
    m |= digit << lo;
    lo += plan.bits[q];
  }
  return m;
}

// Row j of the measurement register that is the i-th row with bit k set.
__host__ __device__ inline int64_t ctrl_row(int64_t i, int k) {
  int64_t lowmask = (int64_t(1) << k) - 1;
  return ((i >> k) << (k + 1)) | (int64_t(1) << k) | (i & lowmask);
}

// Buffer that holds row j before a controlled step: the state ping-pongs
// between two buffers and row j has moved once for every set bit of j that
// belongs to an earlier step, so with pmask = 2^k - 1 (steps 0..k-1 done)
// the row sits in buf[popcount(j & pmask) & 1]. pmask = 0 reads buf0.
__host__ __device__ inline int row_parity(int64_t j, uint64_t pmask) {
  return __builtin_popcountll(uint64_t(j) & pmask) & 1;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_h_broadcast(bool mixed, const void* psi, void* state, int n, int t, hipStream_t s);
hipError_t launch_twiddles(double2* tw_hi, double2* tw_lo, int n, int h, hipStream_t s);
hipError_t launch_split_pieces(const double2* V, uint16_t* planes, int t, hipStream_t s);
hipError_t launch_sub_identity_defect(double2* G, int d, unsigned long long* defect_bits, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int count, hipStream_t s);
hipError_t launch_prob(bool mixed, const void* state, double* prob, int n, int t, const DftPlan& plan,
                       hipStream_t s);
hipError_t launch_report(const double* prob, int n, const double2* psi, int t,
                         const unsigned long long* defect_bits, void* report, hipStream_t s);
hipError_t launch_copy_rows_back(bool mixed, void* state, const void* other, int n, int t, int k,
                                 hipStream_t s);

// C = alpha op(A) op(B) + beta Cin, complex FP64. op: 0 = N, 1 = T, 2 = C.
struct ZgemmArgs {
  int M, N, K;
  const double2* A;
  long lda;
  const double2* B;
  long ldb;
  double2 alpha, beta;
  const double2* Cin;
  long ldcin;
  double2* C;
  long ldc;
};
hipError_t launch_zgemm(int opA, int opB, const ZgemmArgs& a, hipStream_t s, int variant);
int zgemm_variants();

// Controlled step k, FP64 form: rows j with bit k set, read from
// buf[row_parity(j,k)], written to the other buffer: s <- V s.
hipError_t launch_ctrl_f64(double2* buf0, double2* buf1, const double2* V, int n, int t, int k,
                           uint64_t pmask, hipStream_t s, int variant);
int ctrl_f64_variants();
// Controlled step k, mixed form (d >= 32): split-BF16 operator planes
// (blocked by 16 columns). variant 0 = default, 1..ctrl_mixed_variants().
hipError_t launch_ctrl_mixed(float2* buf0, float2* buf1, const uint16_t* planes, int n, int t, int k,
                             uint64_t pmask, hipStream_t s, int variant);
int ctrl_mixed_variants();
// Controlled step k for d <= 16 on the vector ALUs (both forms).
hipError_t launch_ctrl_small(bool mixed, void* buf0, void* buf1, const double2* V, int n, int t, int k,
                             uint64_t pmask, hipStream_t s);

// One inverse-DFT pass. gather: read row p from buf[popcount(p) & 1] (the
// state after the controlled steps), write to buf0; otherwise in place on buf0.
hipError_t launch_qft_pass(bool mixed, void* buf0, const void* buf1, bool gather, int n, int t,
                           int pass_bits, int bits_before, const double2* tw_hi, const double2* tw_lo,
                           int h, hipStream_t s);

DftPlan make_dft_plan(int n);

}  // namespace qpe
