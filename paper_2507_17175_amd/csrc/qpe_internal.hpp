// Internal declarations shared by the HIP translation units of libqpe.
// Host-side launchers return the hipError_t of the launch; device helpers and
// the plan functions are header-inline and __host__ __device__, so the host
// (which sizes grids and workspaces) and the device (which builds the batch
// tables) evaluate exactly the same formulas.
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

// Radix-256 passes over the complex64 state take two DFT rows per thread (a
// workgroup covers 32 consecutive elements instead of 16) when the pass has
// at least 32 elements (2^(n + t - 8)); below that the second row only halves
// the number of threads with work.
__host__ __device__ inline bool qft_two_rows(bool mixed, int pass_bits, int n, int t) {
  return mixed && pass_bits == 8 && n + t >= 13;
}

// Passes of at most 8 bits (radix 256 = 16 x 16 through LDS), balanced.
__host__ __device__ inline DftPlan make_dft_plan(int n) {
  DftPlan p{};
  p.npass = (n + 7) / 8;
  int base = n / p.npass, extra = n % p.npass;
  for (int q = 0; q < p.npass; ++q) p.bits[q] = base + (q < extra ? 1 : 0);
  return p;
}

// Elements (consecutive (row offset, column) pairs) per workgroup of a pass
// of `bits` bits: 256 / R2 for the R1 x R2 split, twice that with two DFT
// rows per thread.
__host__ __device__ inline int qft_elems(bool mixed, int bits, int n, int t) {
  const int r2 = bits > 4 ? (1 << (bits - 4)) : 1;
  return (256 / r2) * (qft_two_rows(mixed, bits, n, t) ? 2 : 1);
}

// The readout is fused into the last DFT pass when there are two passes or
// more (the last one then reads only the first state buffer, so the second
// holds the partial sums) and the last pass has 6 to 8 bits (its workgroup
// holds 16 to 64 elements, so the lanes of one row sit in one wave).
__host__ __device__ inline bool fused_readout(int n) {
  const DftPlan p = make_dft_plan(n);
  return p.npass >= 2 && p.bits[p.npass - 1] >= 6;
}

// Partial sums per row of the fused readout: d / min(d, E) column groups for
// the last pass's E; the partials take readout_groups * 2^n doubles.
__host__ __device__ inline int readout_groups(bool mixed, int n, int t) {
  const DftPlan p = make_dft_plan(n);
  const int e = qft_elems(mixed, p.bits[p.npass - 1], n, t), d = 1 << t;
  return d > e ? d / e : 1;
}

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

// Prefix doubling: since the measurement register starts in |0...0>, the
// rows [2^k, 2^(k+1)) of the state equal rows [0, 2^k) times V_k^T, so step k
// can read rows i < 2^k of buf0 and write them to buf1 = buf0 + 2^k rows.
// The controlled-step kernels take this mapping when the top bit of their
// pmask argument is set (the gate route's masks 2^k - 1 never reach it).
constexpr uint64_t kDoubling = uint64_t(1) << 63;

// Row of the i-th output of a controlled step.
__host__ __device__ inline int64_t step_row(int64_t i, int k, uint64_t pmask) {
  return (pmask & kDoubling) ? i : ctrl_row(i, k);
}
// Buffer (0/1) that row j is read from; it is written to the other one.
__host__ __device__ inline int src_buffer(int64_t j, uint64_t pmask) {
  return (pmask & kDoubling) ? 0 : row_parity(j, pmask);
}

// ------------------------------------------------------ workspace layout

constexpr size_t kAlign = 256;
__host__ __device__ inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
__host__ __device__ inline int tw_split(int n) { return (n + 1) / 2; }

// The Gram product X^H X of the Newton-Schulz step computes only its upper
// tiles. At d = 1024 and 2048 their count (136 or 528 tiles of 64 x 64)
// leaves the 256 CUs unevenly loaded, so the product runs stream-K: the
// (upper tile, 16-deep K slab) units, tile by tile, are cut into
// gram_parts(t) equal runs of consecutive units, one workgroup each. A run adds
// its slabs of one tile into a partial "slot" (the number of runs that
// started in that tile before it); slot 0 is gbuf, slots 1.. follow each
// other in gbuf2, and the identity subtraction adds them in slot order. The
// tile's last run clears the slots no run of it reached. The plan depends
// on d only, so the batched path, which follows it too, adds the same
// partial sums.
__host__ __device__ inline bool gram_split(int t) { return t == 10 || t == 11; }
// Runs (workgroups) of the plan: two per CU, so that one covers the other's
// barriers (measured on MI355X, with the slot sums of the identity
// subtraction: d = 1024: 82 + 25 us against 91 + 21 us with 256 runs and
// 107-111 + 18 us for 32 x 32 tiles in two K halves; d = 2048: 491 + 36 us
// against 595 + 36 us with 256 runs and 571 us in two K halves).
__host__ __device__ inline int gram_parts(int) { return 512; }
struct GramPlan {
  int T, nk;       // upper tiles per side (d / 64), slabs per tile (d / 16)
  int64_t total, W;  // units, units per run
  int slots;       // partial slots (the most runs any tile meets)
};
__host__ __device__ inline GramPlan gram_plan(int t) {
  GramPlan g;
  const int d = 1 << t;
  g.T = d / 64;
  g.nk = d / 16;
  g.total = int64_t(g.T) * (g.T + 1) / 2 * g.nk;
  g.W = (g.total + gram_parts(t) - 1) / gram_parts(t);
  // a tile's units [u nk, u nk + nk) meet runs floor(u nk / W) ..
  // floor((u nk + nk - 1) / W): at most ceil((nk - 1) / W) + 1 of them
  g.slots = int((g.nk - 1 + g.W - 1) / g.W) + 1;
  return g;
}
// Matrices of partial sums in gbuf2 (0 when the Gram product is not split).
__host__ __device__ inline int gram_extra_slots(int t) { return gram_split(t) ? gram_plan(t).slots - 1 : 0; }

// The instance's small scratch region holds, as 8-byte words: the unitarity
// defect (the bits of a non-negative double, atomically maxed), the key of the
// target rotation, the rotated input's peak weight, the state scale sigma of
// the split-FP16 products (a float in the word's first 4 bytes), and from
// word kScratchHash on the partial hashes of the rotation key
// (kRotHashBlocks).
constexpr int kScratchDefect = 0, kScratchKey = 1, kScratchPeak = 2, kScratchSigma = 3, kScratchHash = 8;
// Split-FP16 products: the operator is scaled by this power of two before
// its split (entries of a unitary operator are at most 1 in magnitude).
constexpr int kOpScaleLog2F16 = 14;
constexpr double kOpScaleF16 = double(1 << kOpScaleLog2F16);

// x rounded to the nearest FP16 value, ties to even (|x| below the FP16
// overflow threshold): the FP16 grid spacing is 2^(e - 10) for |x| in
// [2^e, 2^(e+1)), e >= -14, and 2^-24 below 2^-14 (subnormals).
__device__ inline double f16_round(double x) {
  const double a = fabs(x);
  if (a < 0x1p-14) return rint(x * 0x1p24) * 0x1p-24;
  const int e = ilogb(a);
  // x / q with q = 2^(e - 10), as an exact product by 2^(10 - e)
  return rint(x * ldexp(1.0, 10 - e)) * ldexp(1.0, e - 10);
}

__device__ inline uint16_t f16_bits(double exact_f16) {
  return __builtin_bit_cast(uint16_t, (_Float16)(float)exact_f16);  // exact conversions
}

// The split-FP16 pieces of one operator entry v: each FP64 component w,
// scaled by kOpScaleF16, becomes hi = RNE(w) and lo = RNE(w - hi) in FP16;
// p[2 piece + component].
__device__ inline void split_f16_pieces(double2 v, uint16_t (&p)[4]) {
  const double w[2] = {v.x * kOpScaleF16, v.y * kOpScaleF16};
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
    const double hi = f16_round(w[comp]);
    const double lo = f16_round(w[comp] - hi);
    p[comp] = f16_bits(hi);
    p[2 + comp] = f16_bits(lo);
  }
}

// Offset of entry (j, c) of a d x d operator in one of its split planes,
// which are blocked by 16 columns: block c / 16 holds rows 0 .. d-1 of those
// columns, each row's 16 entries contiguous.
__host__ __device__ inline int64_t plane_offset(int64_t d, int64_t j, int64_t c) {
  return (((c >> 4) * d + j) << 4) + (c & 15);
}
constexpr int kRotHashBlocks = 256;
constexpr int kRotHashChunk = 4096;  // operator elements per hash chunk
constexpr size_t kScratchBytes = (kScratchHash + kRotHashBlocks) * 8;

// Regions of one instance's workspace (byte offsets from its base).
struct RunLayout {
  size_t state0, state1, vbuf, tbuf, gbuf, gbuf2, planes, tw_hi, tw_lo, scratch, planes2, total;
};

// planes2: a second set of operator planes after every other region (so the
// offsets of the others do not depend on it), for single prefix-doubling runs
// with split-FP16 products, which alternate the two sets by step parity.
__host__ __device__ inline RunLayout run_layout(int n, int t, bool mixed, bool polar, bool planes2 = false) {
  RunLayout L{};
  const size_t d = size_t(1) << t, N = size_t(1) << n;
  const size_t amp = mixed ? 8 : 16;
  const size_t mat = d * d * 16;
  size_t off = 0;
  L.state0 = off;
  off = align_up(off + N * d * amp);
  L.state1 = off;
  off = align_up(off + N * d * amp);
  L.vbuf = off;
  off = align_up(off + mat);
  L.tbuf = off;
  off = align_up(off + mat);
  L.gbuf = off;
  if (polar) off = align_up(off + mat);
  L.gbuf2 = off;
  if (polar) off = align_up(off + gram_extra_slots(t) * mat);
  L.planes = off;
  if (mixed && t >= 5) off = align_up(off + 6 * d * d * 2);
  const int h = tw_split(n);
  L.tw_hi = off;
  off = align_up(off + (N >> h) * 16);
  L.tw_lo = off;
  off = align_up(off + (size_t(1) << h) * 16);
  L.scratch = off;
  off = align_up(off + kScratchBytes);
  L.planes2 = off;
  if (planes2 && mixed && t >= 5) off = align_up(off + 6 * d * d * 2);
  L.total = off;
  return L;
}

// Target rotation (paper section 2: P(m) is a marginal over the target
// register, so a unitary change of that register's basis leaves it
// unchanged): U <- M U M^H, psi <- M psi with M = D2 H D1 / sqrt(d), H the
// Walsh-Hadamard matrix, D1 a diagonal of signs and D2 one of phases, both
// drawn from a hash of U and psi. On by default in the mixed form for
// d >= 32 (the matrix-core path) when the polar step treats U as unitary;
// forced on by QPE_MIX_TARGET and off with QPE_NO_MIX_TARGET.
enum RotMode { kRotDefault = 0, kRotForce = 1, kRotOff = 2 };
__host__ __device__ inline bool rotate_on(bool mixed, int t, int mode, bool polar) {
  if (t == 0 || mode == kRotOff) return false;
  return mode == kRotForce || (mixed && polar && t >= 5);
}

// The powers that get a Newton-Schulz step (unless QPE_NO_POLAR), in a run
// whose powers are V_0 .. V_{n-1}: every fourth one (k = 3, 7, 11, ...) and
// the last. A squaring doubles the unitarity defect of its operand and adds
// a rounding of order eps sqrt(d); one Newton-Schulz step brings a defect
// delta down to about 1.5 delta^2, i.e. to the rounding level. Between two
// corrections the defect therefore grows at most about eightfold from that
// level (about 1e-15 at d = 512..1024), far inside what the probabilities
// notice, at a quarter of the cost of correcting every power. Correcting the
// last power means that every run with n >= 2 measures the defect of the
// operators it applies last.
__host__ __device__ inline bool ns_step(int k, int n) { return k >= 1 && ((k & 3) == 3 || k == n - 1); }

// Where V_k lives during a run: 0 = U itself, 1 = vbuf, 2 = tbuf. With the
// polar step every square goes to vbuf and V_k to tbuf (the corrected
// square, or at steps without a correction a copy of it; the single-instance
// path reads the square where it is); without it the squares alternate
// between vbuf (odd k) and tbuf.
__host__ __device__ inline int power_slot(int k, bool polar) {
  if (k == 0) return 0;
  if (polar) return 2;
  return (k & 1) ? 1 : 2;
}

// ------------------------------------------------------------- batching
//
// A batched run enqueues one grouped launch per (kind, step): every instance
// that takes part contributes batch_tiles(...) workgroups, and a per-launch
// table (count, members[count], prefix[count+1]) maps a workgroup to its
// instance and local tile. The tables are built on the device from the
// instance descriptors, so nothing is copied from the host.

enum BatchKind {
  BK_ZERO = 0,
  BK_ROTHASH,  // target rotation: partial hashes of U,
  BK_ROTPSI,   //   the key, M psi and its peak weight,
  BK_ROTU,     //   the Walsh-Hadamard passes of U (step = pass)
  BK_SCALE,    // state scale of the split-FP16 products
  BK_HLAYER,
  BK_TWIDDLE,
  BK_SQ,
  BK_GRAM,
  BK_SUBI,
  BK_CORR,
  BK_NSPREP,   // split-BF16 Newton-Schulz correction (mixed form, d >= 32):
  BK_NS_M32,   //   prep, X E on the controlled-product kernel (by size
  BK_NS_M64,   //   class), update
  BK_NS_M128,
  BK_NSUPD,
  BK_PCOPY,    // steps without a correction: V_k = the square (vbuf -> tbuf)
  BK_SPLIT,
  BK_CTRL_SMALL,
  BK_CTRL_M32,
  BK_CTRL_M64,
  BK_CTRL_M128,
  BK_CTRL_M256,  // split FP16, d >= 256: 128 x 256 tiles
  BK_CTRL_F64,
  BK_QFT,
  BK_PROB,
  BK_REPORT,
  BK_QFT_LAST,  // the last DFT pass of an instance with the fused readout
  BK_GRAM_SK,   // the Gram product of d = 1024 and 2048 (stream-K runs)
  BK_COUNT
};

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kHTile = 4096;     // complex amplitudes per H-layer tile
constexpr int kSplitTile = 4096; // operator elements per split tile
constexpr int kSubiTile = 16384; // operator elements per identity-subtraction tile
constexpr int kBatchGemmTile = 32;
constexpr int kProbRounds = 8;   // row groups per readout workgroup
// 256-row tiles per workgroup of the d <= 16 controlled step (the next
// tile's loads overlap the current one; measured on the 177 d <= 16
// instances of the 512-instance batch: 1.52 ms of these launches per batch
// with 2 tiles, 1.58 with 4, 1.87 with 8, 1.84 with one tile and no overlap)
constexpr int kSmallTiles = 2;

struct InstDesc {
  int32_t n, t;
  const double2* U;    // the operator the run uses (rotated, when rotated)
  const double2* psi;  // the input the run uses (rotated, when rotated)
  const double2* U_src;    // the caller's U and psi
  const double2* psi_src;
  double* prob;
  double* report;  // 5 doubles, or null
  char* ws;        // this instance's region of the workspace
};

// The same record as the grouped kernels read it: every pointer in it
// addresses device global memory. Read through plain pointers, whose address
// space the compiler cannot see, the instance's buffers would be accessed
// with flat instructions, and a flat load counts in the LDS wait counter too:
// each wait for LDS data (before every workgroup barrier of the tiled
// kernels) would then also wait for all global loads still in flight.
#define QPE_GLOBAL __attribute__((address_space(1)))
struct InstDescGlobal {
  int32_t n, t;
  const QPE_GLOBAL double2* U;
  const QPE_GLOBAL double2* psi;
  const QPE_GLOBAL double2* U_src;
  const QPE_GLOBAL double2* psi_src;
  QPE_GLOBAL double* prob;
  QPE_GLOBAL double* report;
  QPE_GLOBAL char* ws;
};
static_assert(sizeof(InstDescGlobal) == sizeof(InstDesc) && offsetof(InstDescGlobal, ws) == offsetof(InstDesc, ws),
              "one layout");

// Descriptor i, with pointers the compiler knows to be global.
__device__ __forceinline__ InstDesc load_desc(const InstDesc* desc, int i) {
  const InstDescGlobal g = reinterpret_cast<const InstDescGlobal*>(desc)[i];
  InstDesc D;
  D.n = g.n;
  D.t = g.t;
  D.U = (const double2*)g.U;
  D.psi = (const double2*)g.psi;
  D.U_src = (const double2*)g.U_src;
  D.psi_src = (const double2*)g.psi_src;
  D.prob = (double*)g.prob;
  D.report = (double*)g.report;
  D.ws = (char*)g.ws;
  return D;
}

// Passes of the Walsh-Hadamard transform over the 2t bits of a flattened
// d x d operator (balanced passes of at most 8 bits, as the DFT plan).
__host__ __device__ inline DftPlan rot_plan(int t) { return make_dft_plan(2 * t); }
constexpr int kWhtTile = 2048;  // elements per Walsh-Hadamard tile
__host__ __device__ inline int64_t rot_hash_blocks(int t) {
  const int64_t c = cdiv(int64_t(1) << (2 * t), kRotHashChunk);
  return c < kRotHashBlocks ? c : kRotHashBlocks;
}

// Workgroups instance (n, t) contributes to launch (kind, step); 0 if it
// takes no part. step = controlled step k, or the DFT pass index.
// Flag bits of the grouped kernels' `bflags` argument.
// kBatchGemm64: the power-chain products of operators with d >= 64 use
// 64 x 64 tiles (32 x 32 otherwise); kBatchCtrlInStep: the d >= 128
// controlled step uses the in-step schedule instead of the ping-pong one.
// Neither changes the order of any sum, so results are the same bit for bit.
constexpr int kBatchPolar = 1, kBatchDoubling = 2, kBatchGemm64 = 4, kBatchCtrlInStep = 8;
// kBatchF16: the controlled steps of d >= 32 run as split-FP16 products
constexpr int kBatchF16 = 64;
// kBatchPersistent (batched controlled-step variant 3): the split-FP16
// controlled step of the d >= 256 instances runs on one persistent workgroup
// per CU (the launcher applies it when those instances share one d)
constexpr int kBatchPersistent = 128;
// target rotation mode (RotMode) in bits 4-5
constexpr int kBatchRotShift = 4;
__host__ __device__ inline int batch_rot_mode(int bflags) { return (bflags >> kBatchRotShift) & 3; }

// Tile edge of the grouped power-chain products of an instance with 2^t x 2^t
// operators.
__host__ __device__ inline int batch_gemm_tile(int t, int bflags) {
  return ((bflags & kBatchGemm64) && t >= 6) ? 64 : kBatchGemmTile;
}

__host__ __device__ inline int64_t batch_tiles(int kind, int step, int n, int t, bool mixed, bool polar,
                                               bool dbl = false, int bflags = 0) {
  const int64_t N = int64_t(1) << n, d = int64_t(1) << t;
  // rows a controlled step writes: the gate route's N/2 rows with bit k set,
  // or the 2^k new rows of the prefix-doubling form
  const int64_t half = dbl ? (step < n ? (int64_t(1) << step) : 0) : N / 2;
  // power step `step` gets a Newton-Schulz correction
  const bool ns = polar && step >= 1 && ns_step(step, n);
  switch (kind) {
    case BK_ZERO:
      return 1;
    case BK_ROTHASH:
      return rotate_on(mixed, t, batch_rot_mode(bflags), polar) ? rot_hash_blocks(t) : 0;
    case BK_ROTPSI:
      return rotate_on(mixed, t, batch_rot_mode(bflags), polar) ? 1 : 0;
    case BK_ROTU: {
      if (!rotate_on(mixed, t, batch_rot_mode(bflags), polar)) return 0;
      const DftPlan pl = rot_plan(t);
      return step < pl.npass ? cdiv(d * d, kWhtTile) : 0;
    }
    case BK_SCALE:
      return ((bflags & kBatchF16) && mixed && t >= 5) ? 1 : 0;
    case BK_HLAYER:
      return cdiv(dbl ? d : N * d, kHTile);
    case BK_TWIDDLE: {
      int h = tw_split(n);
      return cdiv((int64_t(1) << h) + (int64_t(1) << (n - h)), 256);
    }
    case BK_SQ: {
      const int64_t T = cdiv(d, batch_gemm_tile(t, bflags));
      return (step >= 1 && step < n) ? T * T : 0;
    }
    case BK_GRAM: {
      // Hermitian: the tiles on or above the diagonal
      const int64_t T = cdiv(d, batch_gemm_tile(t, bflags));
      return (ns && step < n && !gram_split(t)) ? T * (T + 1) / 2 : 0;
    }
    case BK_GRAM_SK:  // the runs of the stream-K plan
      return (ns && step < n && gram_split(t)) ? int64_t(gram_parts(t)) : 0;
    case BK_CORR: {
      const int64_t T = cdiv(d, batch_gemm_tile(t, bflags));
      return (ns && !(mixed && t >= 5) && step < n) ? T * T : 0;
    }
    case BK_NSPREP:
    case BK_NSUPD:
      return (ns && mixed && t >= 5 && step < n) ? cdiv(d * d, kSplitTile) : 0;
    case BK_NS_M32:
      return (ns && mixed && t == 5 && step < n) ? cdiv(d, 128) * (d / 32) : 0;
    case BK_NS_M64:
      return (ns && mixed && t == 6 && step < n) ? cdiv(d, 128) * (d / 64) : 0;
    case BK_NS_M128:
      return (ns && mixed && t >= 7 && step < n) ? cdiv(d, 128) * (d / 128) : 0;
    case BK_SUBI:
      return (ns && step < n) ? cdiv(d * d, kSubiTile) : 0;
    case BK_PCOPY:
      return (polar && step >= 1 && !ns_step(step, n) && step < n) ? cdiv(d * d, kSplitTile) : 0;
    case BK_SPLIT:
      return (mixed && t >= 5 && step < n) ? cdiv(d * d, kSplitTile) : 0;
    case BK_CTRL_SMALL:
      return (t <= 4 && step < n) ? cdiv(half, 256 * kSmallTiles) : 0;
    case BK_CTRL_M32:
      return (mixed && t == 5 && step < n) ? cdiv(half, 128) * (d / 32) : 0;
    case BK_CTRL_M64:
      return (mixed && t == 6 && step < n) ? cdiv(half, 128) * (d / 64) : 0;
    case BK_CTRL_M128:
      return (mixed && (t == 7 || (t >= 8 && !(bflags & kBatchF16))) && step < n) ? cdiv(half, 128) * (d / 128) : 0;
    case BK_CTRL_M256:
      return (mixed && t >= 8 && (bflags & kBatchF16) && step < n) ? cdiv(half, 128) * (d / 256) : 0;
    case BK_CTRL_F64:
      return (!mixed && t >= 5 && step < n) ? cdiv(half, 64) * cdiv(d, 64) : 0;
    case BK_QFT:
    case BK_QFT_LAST: {
      DftPlan pl = make_dft_plan(n);
      if (step >= pl.npass) return 0;
      // the fused last pass runs in its own launch kind
      if ((kind == BK_QFT_LAST) != (fused_readout(n) && step == pl.npass - 1)) return 0;
      const int b = pl.bits[step];
      return cdiv((N * d) >> b, qft_elems(mixed, b, n, t));
    }
    case BK_PROB: {
      // fused readout: one row per thread; else rows of G lanes
      if (fused_readout(n)) return cdiv(N, 256 * kProbRounds);
      int64_t G = d < 64 ? d : 64;
      return cdiv(N, 4 * (64 / G) * kProbRounds);
    }
    case BK_REPORT:
      return 1;
  }
  return 0;
}

// Instance and local tile of workgroup `tile` in a launch table.
// The first tile of each member, pre[], rises strictly from pre[0] = 0, so
// the member is the last entry <= tile. Each round the 64 lanes of the wave
// sample the remaining range at 64 evenly spaced entries (one load each) and
// a ballot picks the segment: two dependent rounds up to 4096 members,
// instead of a binary search's log2(count). Every lane of a full wave must
// call it (all grouped kernels do, first thing, with blocks of whole waves).
__device__ inline int find_member(const int32_t* __restrict__ tab, int64_t tile, int64_t* local) {
  const int count = tab[0];
  const int32_t* mem = tab + 1;
  const int32_t* pre = tab + 1 + count;
  const int lane = threadIdx.x & 63;
  int lo = 0, len = count;  // invariant: pre[lo] <= tile, the answer is in [lo, lo + len)
  while (len > 1) {
    const int step = (len + 63) >> 6;
    const bool le = lane * step < len && pre[lo + lane * step] <= tile;
    const unsigned long long m = __ballot(le);  // bit 0 is set: pre[lo] <= tile
    const int last = 63 - __clzll(m);
    lo += last * step;
    len = min(step, len - last * step);
  }
  *local = tile - pre[lo];
  return mem[lo];
}

// A grouped launch of more workgroups than this is split into several
// launches over consecutive tile ranges (argument tile0 of the grouped
// kernels), which keeps every grid far below the 2^32 work-item limit.
constexpr int64_t kMaxGridBlocks = int64_t(1) << 22;

template <typename F>
hipError_t for_grid_chunks(int64_t tiles, F&& launch_one) {
  for (int64_t base = 0; base < tiles; base += kMaxGridBlocks) {
    const int64_t g = tiles - base < kMaxGridBlocks ? tiles - base : kMaxGridBlocks;
    launch_one(unsigned(g), base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct BatchLaunch {
  int32_t kind, step, table_off;  // table_off in int32 units
};

// ---------------------------------------------------------------- launchers
hipError_t launch_h_broadcast(bool mixed, const void* psi, void* state, int n, int t, hipStream_t s,
                              bool first_row_only = false);
hipError_t launch_twiddles(double2* tw_hi, double2* tw_lo, int n, int h, hipStream_t s);
// f16: the two FP16 pieces of the split-FP16 products (four planes) instead
// of the three BF16 pieces (six planes).
hipError_t launch_split_pieces(const double2* V, uint16_t* planes, int t, hipStream_t s, bool f16 = false);
// sigma (device float) <- the state scale of the split-FP16 products for
// input psi and n measurement qubits.
hipError_t launch_state_scale(const double2* psi, int n, int t, float* sigma, hipStream_t s);
// Newton-Schulz correction in split BF16 (mixed form): E = G - I and its
// defect, X32 = complex64(X) and planes = split(conj(E)) in one pass (E itself
// not stored); after XE = X32 E on the split-BF16 kernel, out = X - XE / 2
// and the split of out into the planes in one pass.
hipError_t launch_ns_prep_fused(const double2* X, const double2* G, const double2* G2, float2* X32, uint16_t* planes,
                                int t, unsigned long long* defect_bits, hipStream_t s);
hipError_t launch_ns_update_split(const double2* X, const float2* XE, double2* out, uint16_t* planes, int t,
                                  hipStream_t s, bool f16 = false);
// G <- G (+ G2 when not null) - I, and the defect max |G_ij| (atomic max).
hipError_t launch_sub_identity_defect(double2* G, const double2* G2, int d, unsigned long long* defect_bits,
                                      hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int count, hipStream_t s);
// Target rotation (k_rotate.hip). scratch: the instance's scratch words
// (kScratch*). launch_rot_hash writes the partial hashes of U;
// launch_rot_psi combines them with a hash of psi into the key, tries four
// sign diagonals derived from it and keeps the one whose M psi has the
// smallest peak weight max_i |(M psi)_i|^2 / ||psi||^2 (key and peak into
// scratch, M psi into psi_out); launch_rot_u writes Ur = M U M^H.
hipError_t launch_rot_hash(const double2* U, int t, unsigned long long* scratch, hipStream_t s);
hipError_t launch_rot_psi(const double2* psi, int t, unsigned long long* scratch, double2* psi_out, hipStream_t s);
hipError_t launch_rot_u(const double2* U, double2* Ur, int t, const unsigned long long* scratch, hipStream_t s);
// Undo the rotation on a final statevector (N x d, outcome rows): every row
// a <- M^H a (complex64 when mixed, else complex128), in place.
hipError_t launch_unrotate_state(bool mixed, void* state, int n, int t, const unsigned long long* scratch,
                                 hipStream_t s);
hipError_t launch_prob(bool mixed, const void* state, double* prob, int n, int t, const DftPlan& plan,
                       hipStream_t s);
// The readout after a fused last pass: prob[m] = 2^-n sum_cg part[cg 2^n + p]
// for the row p of outcome m, over the `groups` column groups in order.
hipError_t launch_prob_finish(const double* part, double* prob, int n, int groups, const DftPlan& plan,
                              hipStream_t s);
// part (optional): device scratch of 2^n / 256 bytes (16-byte aligned) for
// the partial sums of a two-stage sum when 2^n >= 16384.
// rot_peak: the rotated input's peak weight (scratch word kScratchPeak) when
// the run rotated, else null (the peak of psi itself is reported); check:
// flag QPE_REPORT_CONCENTRATED when that peak exceeds kPeakFlag (mixed form,
// matrix-core path).
constexpr double kPeakFlag = 0.5;
hipError_t launch_report(const double* prob, int n, const double2* psi, int t,
                         const unsigned long long* defect_bits, const double* rot_peak, bool check, void* report,
                         double* part, hipStream_t s);
// Final statevector in outcome order: out[m][r] = scale * X[p][r] where row
// position p of the DFT output holds outcome m (prob_index(p) = m).
hipError_t launch_gather_state(bool mixed, const void* X, void* out, int n, int t, const DftPlan& plan, double scale,
                               hipStream_t s);
hipError_t launch_copy_rows_back(bool mixed, void* state, const void* other, int n, int t, int k,
                                 hipStream_t s);

// Phase estimators of one probability vector (k_estimate.hip): writes the
// six 8-byte fields of qpe_estimates to out. scratch: est_workspace_bytes().
constexpr int kEstMaxBlocks = 1024;
int est_blocks(int n);
size_t est_workspace_bytes();
hipError_t launch_estimate(const double* P, int n, void* scratch, double* out, hipStream_t s);

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
  // Hermitian result (op(A) = B^H, alpha real, beta 0): only tiles on or
  // above the diagonal are computed; each mirrors itself below it.
  int herm;
  // When set (a square product, M = N = ldc, herm 0): the epilogue also
  // writes the split-FP16 pieces of every entry of C (split_f16_pieces) to
  // the four planes, d^2 entries each, at plane_offset(N, row, column).
  uint16_t* planes;
};
hipError_t launch_zgemm(int opA, int opB, const ZgemmArgs& a, hipStream_t s, int variant);
int zgemm_variants();
// The split Gram product (gram_split(t)) by the stream-K plan: slot 0 of
// G = X^H X in G, slots 1.. in G2 (d x d each, consecutive).
hipError_t launch_gram_split(const double2* X, double2* G, double2* G2, int t, hipStream_t s);
// The same for the instances of a launch table (kind BK_GRAM_SK, step k).
hipError_t launch_batch_gram_split(int step, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                                   int bflags, hipStream_t s);

// Controlled step k, FP64 form: rows j with bit k set, read from
// buf[row_parity(j,k)], written to the other buffer: s <- V s.
hipError_t launch_ctrl_f64(double2* buf0, double2* buf1, const double2* V, int n, int t, int k,
                           uint64_t pmask, hipStream_t s, int variant);
int ctrl_f64_variants();
// Controlled step k, mixed form (d >= 32): split-BF16 operator planes
// (blocked by 16 columns). variant 0 = default, 1..ctrl_mixed_variants().
// sigma_f16: null for the split-BF16 products (six pairs of three BF16
// pieces, operator planes from launch_split_pieces); else the device address
// of the state scale sigma of the split-FP16 products (three pairs of two
// FP16 pieces, planes from launch_split_pieces with f16).
hipError_t launch_ctrl_mixed(float2* buf0, float2* buf1, const uint16_t* planes, int n, int t, int k,
                             uint64_t pmask, hipStream_t s, int variant, const float* sigma_f16 = nullptr);
int ctrl_mixed_variants();
// The Newton-Schulz product XE = X32 E (d x d) on the split-BF16 kernel with
// three piece pairs (E is of the size of the unitarity defect), X32 and the
// planes of conj(E) as written by launch_ns_prep.
hipError_t launch_ns_product(float2* x32, float2* xe, const uint16_t* planes, int t, hipStream_t s);
// Controlled step k for d <= 16 on the vector ALUs (both forms).
hipError_t launch_ctrl_small(bool mixed, void* buf0, void* buf1, const double2* V, int n, int t, int k,
                             uint64_t pmask, hipStream_t s);

// One inverse-DFT pass. gather: read row p from buf[popcount(p) & 1] (the
// state after the controlled steps), write to buf0; otherwise in place on buf0.
hipError_t launch_qft_pass(bool mixed, void* buf0, const void* buf1, bool gather, int n, int t,
                           int pass_bits, int bits_before, const double2* tw_hi, const double2* tw_lo,
                           int h, hipStream_t s);
// The last pass with the fused readout (fused_readout(n)): reads buf0, writes
// readout_groups(mixed, n, t) x 2^n partial sums to part (8-byte aligned,
// distinct from buf0) and, with keep, the transformed state to buf0.
hipError_t launch_qft_last_fused(bool mixed, void* buf0, int n, int t, int pass_bits, int bits_before,
                                 const double2* tw_hi, const double2* tw_lo, int h, double* part, bool keep,
                                 hipStream_t s);

// ---- batched launchers: one grouped launch over the instances of a table ----
struct BatchProblem {
  int32_t n, t;
  const void* U;
  const void* psi;
  const void* U_src;
  const void* psi_src;
  double* prob;
  void* report;
  uint64_t ws_offset;
};
constexpr int kBatchChunk = 48;  // problems per descriptor-setup launch
constexpr int kBatchLaunchChunk = 160;
hipError_t launch_batch_descs(InstDesc* desc, char* ws, const BatchProblem* probs, int first, int count,
                              hipStream_t s);
hipError_t launch_batch_tables(const InstDesc* desc, int ninst, int32_t* tables, const BatchLaunch* launches,
                               int nlaunch, bool mixed, int bflags, hipStream_t s);
// Elementwise kinds (zero, H layer, twiddles, identity subtraction, split,
// readout, report).
hipError_t launch_batch_elementwise(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                                    bool mixed, int bflags, hipStream_t s);
// Target-rotation kinds (BK_ROTHASH, BK_ROTPSI, BK_ROTU).
hipError_t launch_batch_rotate(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                               bool mixed, int bflags, hipStream_t s);
hipError_t launch_batch_zgemm(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                              bool mixed, int bflags, hipStream_t s);
hipError_t launch_batch_ctrl_f64(int step, const InstDesc* desc, const int32_t* table, int64_t tiles, int bflags,
                                 hipStream_t s);
hipError_t launch_batch_ctrl_mixed(int kind, int step, const InstDesc* desc, const int32_t* table, int64_t tiles,
                                   int bflags, hipStream_t s, int wide_t = 0);
// stage: some instance of the launch has d = 8 or 16 (rows staged in LDS).
hipError_t launch_batch_ctrl_small(int step, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                                   bool stage, int bflags, hipStream_t s);
// wide: some instance of the launch takes two rows per thread in this pass.
hipError_t launch_batch_qft(int pass, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                            bool wide, int bflags, hipStream_t s);
// The same for the instances whose pass `pass` is their fused last pass.
hipError_t launch_batch_qft_last(int pass, const InstDesc* desc, const int32_t* table, int64_t tiles, bool mixed,
                                 bool wide, int bflags, hipStream_t s);

}  // namespace qpe
