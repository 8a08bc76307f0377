// C ABI of the QPE emulator: argument checks, workspace layout and the order
// in which the stage kernels are enqueued (paper section 2, Fig. 1).
//
// Path for one instance (n measurement qubits, d = 2^t):
//   H layer        every state row <- psi * 2^(-n/2)
//   for k < n:     V_k = (V_{k-1})^2 in FP64, Newton-Schulz re-unitarised;
//                  rows with bit k set <- row V_k^T (FP64 MFMA, split-BF16
//                  MFMA, or VALU for d <= 16); state ping-pongs between two
//                  buffers so the controlled GEMM never needs a copy-back
//   inverse QFT    radix-2^b passes along the row axis
//   readout        P(m) = sum_r |A[m, r]|^2 in FP64, digit order undone
// Nothing here allocates device memory: all scratch lives in the caller's
// workspace, so a run can be captured into a HIP graph.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qpe.h"
#include "qpe_internal.hpp"

#define QPE_API extern "C" __attribute__((visibility("default")))

struct qpe_timer_pair {
  hipEvent_t start, stop;
  int which;
};

struct qpe_ctx {
  int device;
  hipStream_t stream;
  std::string last_error;
  // optional per-kernel timing
  std::vector<qpe_timer_pair> timers;
  size_t timers_used = 0;
  bool timing = false;
  unsigned timer_mask = (1u << QPE_TIMER_COUNT) - 1;  // timer classes that record events
  // kernel variant per class (0 = default)
  int variant[QPE_KERNEL_COUNT][QPE_MAX_N_MAT + 1] = {};
  // fault injection for tests of the error path: the checked HIP call with
  // this ordinal (counting from 1 on this context) is reported as failed
  // without being made; 0 = off (environment variable QPE_FAULT_INJECT at
  // creation)
  long fault_at = 0;
  long hip_calls = 0;
  // second stream and events of the two-stream batch schedule (created on
  // first use, default priority)
  hipStream_t aux = nullptr;
  std::vector<hipEvent_t> sched_ev;
};

namespace {

using namespace qpe;

bool misaligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) != 0; }

// The controlled products of the mixed form run as split-FP16 products
// (three FP16 products per real one) unless QPE_SPLIT_BF16 asks for the
// six-product BF16 scheme; the FP16 scaling needs the row norms a unitary U
// keeps, so without the polar step the BF16 scheme runs.
bool use_f16(int form, unsigned flags) {
  return form == QPE_FORM_MIXED && !(flags & QPE_NO_POLAR) && !(flags & QPE_SPLIT_BF16);
}

// (A batch lays out its instances with the same sizes; its grouped kernels
// never use the second plane set.)
RunLayout run_layout(int n, int t, int form, unsigned flags) {
  return qpe::run_layout(n, t, form == QPE_FORM_MIXED, !(flags & QPE_NO_POLAR),
                         (flags & QPE_PREFIX_DOUBLING) && use_f16(form, flags));
}

int rot_mode(unsigned flags) {
  if (flags & QPE_MIX_TARGET) return kRotForce;
  if (flags & QPE_NO_MIX_TARGET) return kRotOff;
  return kRotDefault;
}

// ---- batched runs -------------------------------------------------------
//
// Workspace of a batched run: [launch tables][instance descriptors]
// [instance 0 region][instance 1 region]... Every region is 256-aligned.
struct BatchPlan {
  std::vector<BatchLaunch> launches;
  std::vector<int64_t> tiles;  // workgroups of each launch
  size_t table_bytes = 0, desc_off = 0, inst_off = 0, total = 0;
  std::vector<size_t> inst_base;  // byte offset of each instance region
  bool ok = true;                 // false if a launch exceeds the grid limit
};

// tile_flags: the kBatchGemm64 bit of the launch (it changes tile counts,
// not the launch list or the table sizes)
BatchPlan plan_batch(const qpe_problem* p, int count, int form, unsigned flags, bool with_report,
                     int tile_flags = 0) {
  BatchPlan P;
  const bool mixed = form == QPE_FORM_MIXED, polar = !(flags & QPE_NO_POLAR);
  const bool dbl = (flags & QPE_PREFIX_DOUBLING) != 0;
  tile_flags |= (rot_mode(flags) << kBatchRotShift) | (use_f16(form, flags) ? kBatchF16 : 0);
  int32_t table_ints = 0;
  auto add = [&](int kind, int step) {
    int members = 0;
    int64_t tiles = 0;
    for (int i = 0; i < count; ++i) {
      int64_t w = batch_tiles(kind, step, p[i].n_meas, p[i].n_mat, mixed, polar, dbl, tile_flags);
      if (w > 0) {
        ++members;
        tiles += w;
      }
    }
    if (tiles == 0) return;
    if (tiles >= (int64_t(1) << 31)) P.ok = false;
    P.launches.push_back(BatchLaunch{kind, step, table_ints});
    P.tiles.push_back(tiles);
    table_ints += 2 + 2 * members;
  };
  int maxn = 0, maxpass = 0, maxrot = 0;
  for (int i = 0; i < count; ++i) {
    maxn = p[i].n_meas > maxn ? p[i].n_meas : maxn;
    int np = make_dft_plan(p[i].n_meas).npass;
    maxpass = np > maxpass ? np : maxpass;
    if (rotate_on(mixed, p[i].n_mat, rot_mode(flags), polar)) {
      np = rot_plan(p[i].n_mat).npass;
      maxrot = np > maxrot ? np : maxrot;
    }
  }
  add(BK_ZERO, 0);
  add(BK_ROTHASH, 0);
  add(BK_ROTPSI, 0);
  for (int q = 0; q < maxrot; ++q) add(BK_ROTU, q);
  add(BK_SCALE, 0);
  add(BK_HLAYER, 0);
  add(BK_TWIDDLE, 0);
  for (int k = 0; k < maxn; ++k) {
    if (k >= 1) {
      add(BK_SQ, k);
      if (polar) {
        add(BK_GRAM, k);
        add(BK_GRAM_SK, k);
        add(BK_SUBI, k);
        add(BK_CORR, k);
        add(BK_NSPREP, k);
        add(BK_NS_M32, k);
        add(BK_NS_M64, k);
        add(BK_NS_M128, k);
        add(BK_NSUPD, k);
        add(BK_PCOPY, k);
      }
    }
    if (mixed) {
      add(BK_SPLIT, k);
      add(BK_CTRL_SMALL, k);
      add(BK_CTRL_M32, k);
      add(BK_CTRL_M64, k);
      add(BK_CTRL_M128, k);
      add(BK_CTRL_M256, k);
    } else {
      add(BK_CTRL_SMALL, k);
      add(BK_CTRL_F64, k);
    }
  }
  for (int q = 0; q < maxpass; ++q) {
    add(BK_QFT, q);
    add(BK_QFT_LAST, q);
  }
  add(BK_PROB, 0);
  if (with_report) add(BK_REPORT, 0);
  P.table_bytes = align_up(size_t(table_ints) * 4);
  P.desc_off = P.table_bytes;
  P.inst_off = P.desc_off + align_up(size_t(count) * sizeof(InstDesc));
  size_t off = P.inst_off;
  P.inst_base.resize(count);
  for (int i = 0; i < count; ++i) {
    P.inst_base[i] = off;
    off += run_layout(p[i].n_meas, p[i].n_mat, form, flags).total;
  }
  P.total = off;
  return P;
}

size_t workspace_need(const qpe_problem* p, int count, int form, unsigned flags) {
  if (count == 1) return run_layout(p[0].n_meas, p[0].n_mat, form, flags).total;
  return plan_batch(p, count, form, flags, true).total;
}

qpe_status check_sizes(int n, int t) {
  if (n < 1 || n > QPE_MAX_N_MEAS || t < 0 || t > QPE_MAX_N_MAT || n + t > QPE_MAX_TOTAL_QUBITS)
    return QPE_ERR_SIZE;
  return QPE_OK;
}

qpe_status check_problem(const qpe_problem& p, bool need_ptrs) {
  qpe_status s = check_sizes(p.n_meas, p.n_mat);
  if (s != QPE_OK) return s;
  if (!need_ptrs) return QPE_OK;
  if (!p.U || !p.psi || !p.prob) return QPE_ERR_ARG;
  if (misaligned(p.U, 16) || misaligned(p.psi, 16) || misaligned(p.prob, 8)) return QPE_ERR_ALIGN;
  return QPE_OK;
}

qpe_status check_form_flags(int form, unsigned flags) {
  if (form != QPE_FORM_FP64 && form != QPE_FORM_MIXED) return QPE_ERR_ARG;
  if (flags & ~unsigned(QPE_NO_POLAR | QPE_PREFIX_DOUBLING | QPE_MIX_TARGET | QPE_NO_MIX_TARGET | QPE_SPLIT_BF16))
    return QPE_ERR_ARG;
  if ((flags & QPE_MIX_TARGET) && (flags & QPE_NO_MIX_TARGET)) return QPE_ERR_ARG;
  return QPE_OK;
}

qpe_status check_workspace(const void* ws, size_t have, size_t need) {
  if (need == 0) return QPE_OK;
  if (!ws) return QPE_ERR_WORKSPACE;
  if (misaligned(ws, kAlign)) return QPE_ERR_WORKSPACE;
  if (have < need) return QPE_ERR_WORKSPACE;
  return QPE_OK;
}

// Makes ctx->device current for the duration of a call and restores the
// caller's device afterwards.
struct DeviceGuard {
  int old = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) return;
    if (old != dev && hipSetDevice(dev) != hipSuccess) return;
    ok = true;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
  }
};

qpe_status hip_fail(qpe_ctx* ctx, hipError_t e, const char* what) {
  ctx->last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return QPE_ERR_HIP;
}

// True when this checked HIP call is the one QPE_FAULT_INJECT names.
bool injected_fault(qpe_ctx* ctx) { return ctx->fault_at > 0 && ++ctx->hip_calls == ctx->fault_at; }

// Brackets the launches made inside its scope with a pair of events on the
// context stream when timing is enabled and the pool has room.
struct TimerScope {
  qpe_ctx* ctx;
  long idx = -1;
  TimerScope(qpe_ctx* c, int which) : ctx(c) {
    if (which >= 0 && c->timing && ((c->timer_mask >> which) & 1u) && c->timers_used < c->timers.size()) {
      idx = long(c->timers_used++);
      c->timers[idx].which = which;
      (void)hipEventRecord(c->timers[idx].start, c->stream);
    }
  }
  ~TimerScope() {
    if (idx >= 0) (void)hipEventRecord(ctx->timers[idx].stop, ctx->stream);
  }
};

#define QPE_HIP(ctx, expr)                                                              \
  do {                                                                                  \
    const bool inj_ = injected_fault(ctx);                                              \
    hipError_t e_ = inj_ ? hipErrorLaunchFailure : (expr);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, inj_ ? "injected fault (QPE_FAULT_INJECT): " #expr : #expr); \
  } while (0)

// V_next = cur^2, then (unless no_polar) one Newton-Schulz step
//   X <- X (3I - X^H X) / 2 = X - X (X^H X - I) / 2,
// whose E = X^H X - I also yields the unitarity defect max|E_ij|.
// sq and out are distinct from cur; out may equal the dead predecessor.
// With planes (the mixed form, d >= 32) the correction X E runs on the
// split-BF16 kernel: X rounded to complex64 (staged in out) times E split
// into BF16 pieces, three piece pairs (E is O(defect), so the product's
// error is O(1e-5 defect), far below the FP64 rounding of X), accumulated
// in FP32 into g, which E no longer needs by then.
// With planes, the Newton-Schulz update also splits its result into them,
// and with split-FP16 products so does the square's epilogue when there is
// no correction; *planes_hold_out is then set.
// s: the stream (null: the context's); before_update (optional): an event
// the stream waits for after the square and the Gram product, before the
// Newton-Schulz stages write `out` and the planes.
qpe_status square_and_polar(qpe_ctx* ctx, int d, const double2* cur, double2* sq, double2* g, double2* out,
                            bool polar, unsigned long long* defect, uint16_t* planes = nullptr,
                            double2* g2 = nullptr, bool* planes_hold_out = nullptr, bool f16 = false,
                            hipStream_t stream = nullptr, hipEvent_t before_update = nullptr) {
  hipStream_t s = stream ? stream : ctx->stream;
  const int tz = 31 - __builtin_clz(unsigned(d));  // log2 d
  ZgemmArgs a{};
  a.M = a.N = a.K = d;
  a.A = cur;
  a.lda = d;
  a.B = cur;
  a.ldb = d;
  a.alpha = make_double2(1.0, 0.0);
  a.beta = make_double2(0.0, 0.0);
  a.C = sq;
  a.ldc = d;
  // Without a correction the square is the next operator: with split-FP16
  // products its epilogue also writes the planes.
  const bool fuse_split = !polar && planes && f16 && tz >= 5;
  if (fuse_split) a.planes = planes;
  QPE_HIP(ctx, launch_zgemm(0, 0, a, s, ctx->variant[QPE_KERNEL_ZGEMM][tz]));
  if (fuse_split && planes_hold_out) *planes_hold_out = true;
  if (!polar) return QPE_OK;
  a.planes = nullptr;
  ZgemmArgs h = a;
  h.A = sq;
  h.B = sq;
  h.C = g;
  h.herm = 1;
  // G = X^H X; at d = 1024 and 2048 by the stream-K plan, its partial
  // slots in g and g2
  if (gram_split(tz))
    QPE_HIP(ctx, launch_gram_split(sq, g, g2, tz, s));
  else
    QPE_HIP(ctx, launch_zgemm(2, 0, h, s, ctx->variant[QPE_KERNEL_ZGEMM][tz]));
  if (before_update) QPE_HIP(ctx, hipStreamWaitEvent(s, before_update, 0));
  double2* gs = gram_split(tz) ? g2 : nullptr;
  if (planes && tz >= 5) {
    // E = G - I with the defect, X -> complex64 and the split of conj(E) in
    // one pass; after the product, the update also splits the new power
    // into the planes, which then hold the operator of the next step.
    float2* x32 = reinterpret_cast<float2*>(out);
    float2* xe = reinterpret_cast<float2*>(g);
    QPE_HIP(ctx, launch_ns_prep_fused(sq, g, gs, x32, planes, tz, defect, s));
    QPE_HIP(ctx, launch_ns_product(x32, xe, planes, tz, s));
    QPE_HIP(ctx, launch_ns_update_split(sq, xe, out, planes, tz, s, f16));
    if (planes_hold_out) *planes_hold_out = true;
    return QPE_OK;
  }
  QPE_HIP(ctx, launch_sub_identity_defect(g, gs, d, defect, s));
  ZgemmArgs c = a;
  c.A = sq;
  c.B = g;
  c.alpha = make_double2(-0.5, 0.0);
  c.beta = make_double2(1.0, 0.0);
  c.Cin = sq;
  c.ldcin = d;
  c.C = out;
  QPE_HIP(ctx, launch_zgemm(0, 0, c, s, ctx->variant[QPE_KERNEL_ZGEMM][tz]));  // X - X E / 2
  return QPE_OK;
}

// sigma_f16: device address of the state scale for split-FP16 products, or
// null for the split-BF16 ones.
qpe_status controlled(qpe_ctx* ctx, bool mixed, int n, int t, int k, const double2* V, void* s0, void* s1,
                      uint16_t* planes, uint64_t pmask, bool need_split = true, const float* sigma_f16 = nullptr) {
  hipStream_t s = ctx->stream;
  if (t <= 4) {
    TimerScope ts(ctx, QPE_TIMER_CTRL_GEMM);
    QPE_HIP(ctx, launch_ctrl_small(mixed, s0, s1, V, n, t, k, pmask, s));
  } else if (mixed) {
    if (need_split) {
      TimerScope ts(ctx, QPE_TIMER_SPLIT);
      QPE_HIP(ctx, launch_split_pieces(V, planes, t, s, sigma_f16 != nullptr));
    }
    TimerScope ts(ctx, QPE_TIMER_CTRL_GEMM);
    QPE_HIP(ctx, launch_ctrl_mixed(static_cast<float2*>(s0), static_cast<float2*>(s1), planes, n, t, k, pmask, s,
                                    ctx->variant[QPE_KERNEL_CTRL_MIXED][t], sigma_f16));
  } else {
    TimerScope ts(ctx, QPE_TIMER_CTRL_GEMM);
    QPE_HIP(ctx, launch_ctrl_f64(static_cast<double2*>(s0), static_cast<double2*>(s1), V, n, t, k, pmask, s,
                                 ctx->variant[QPE_KERNEL_CTRL_F64][t]));
  }
  return QPE_OK;
}

// The inverse QFT passes and the readout. s1: the second state buffer (read
// by the first pass when gather) or, with no gather, any buffer of at least
// readout_groups(mixed, n, t) 2^n doubles distinct from s0; when the readout
// is fused into the last pass (fused_readout(n)), its partial sums go to s1,
// which the first pass has read by then. keep: leave the transformed state
// in s0 (the fused last pass otherwise does not store it).
qpe_status iqft_and_probs(qpe_ctx* ctx, bool mixed, int n, int t, void* s0, void* s1, bool gather, double* prob,
                          double2* tw_hi, double2* tw_lo, bool keep = false) {
  hipStream_t s = ctx->stream;
  const int h = tw_split(n);
  QPE_HIP(ctx, launch_twiddles(tw_hi, tw_lo, n, h, s));
  DftPlan plan = make_dft_plan(n);
  const bool fuse = fused_readout(n);
  double* part = static_cast<double*>(s1);
  int before = 0;
  for (int q = 0; q < plan.npass; ++q) {
    TimerScope ts(ctx, QPE_TIMER_QFT);
    if (fuse && q == plan.npass - 1)
      QPE_HIP(ctx, launch_qft_last_fused(mixed, s0, n, t, plan.bits[q], before, tw_hi, tw_lo, h, part, keep, s));
    else
      QPE_HIP(ctx, launch_qft_pass(mixed, s0, s1, gather && q == 0, n, t, plan.bits[q], before, tw_hi, tw_lo, h, s));
    before += plan.bits[q];
  }
  TimerScope ts(ctx, QPE_TIMER_PROB);
  if (fuse)
    QPE_HIP(ctx, launch_prob_finish(part, prob, n, readout_groups(mixed, n, t), plan, s));
  else
    QPE_HIP(ctx, launch_prob(mixed, s0, prob, n, t, plan, s));
  return QPE_OK;
}

// Target rotation: Ur = M U M^H and pr = M psi with M = D2 H D1 / sqrt(d),
// the key of the diagonals and the peak weight of pr in the instance's
// scratch words.
qpe_status rotate_target(qpe_ctx* ctx, int t, const double2* U, const double2* psi, double2* Ur, double2* pr,
                         unsigned long long* scratch) {
  hipStream_t s = ctx->stream;
  TimerScope ts(ctx, QPE_TIMER_POWERS);
  QPE_HIP(ctx, launch_rot_hash(U, t, scratch, s));
  QPE_HIP(ctx, launch_rot_psi(psi, t, scratch, pr, s));
  QPE_HIP(ctx, launch_rot_u(U, Ur, t, scratch, s));
  return QPE_OK;
}

// Events of one run of the two-stream schedule: at most two hops per step
// plus the fork and the join, so no event is recorded twice in one run.
constexpr int kSchedEvents = 2 * QPE_MAX_N_MEAS + 4;

// The second stream and `nev` events of the two-stream schedule.
qpe_status ensure_sched(qpe_ctx* ctx, int nev) {
  if (!ctx->aux) QPE_HIP(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
  while (int(ctx->sched_ev.size()) < nev) {
    hipEvent_t e = nullptr;
    QPE_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->sched_ev.push_back(e);
  }
  return QPE_OK;
}

// keep_state: leave the final state (after the inverse QFT) in state0.
// allow_aux: the prefix-doubling form may use the two-stream schedule.
qpe_status run_one(qpe_ctx* ctx, const qpe_problem& p, int form, unsigned flags, char* ws, qpe_report* report,
                   bool keep_state = false, bool allow_aux = true) {
  const int n = p.n_meas, t = p.n_mat, d = 1 << t;
  const bool mixed = form == QPE_FORM_MIXED;
  const bool polar = !(flags & QPE_NO_POLAR);
  const RunLayout L = run_layout(n, t, form, flags);
  hipStream_t s = ctx->stream;
  void* s0 = ws + L.state0;
  void* s1 = ws + L.state1;
  double2* A = reinterpret_cast<double2*>(ws + L.vbuf);
  double2* B = reinterpret_cast<double2*>(ws + L.tbuf);
  double2* G = polar ? reinterpret_cast<double2*>(ws + L.gbuf) : nullptr;
  double2* G2 = (polar && gram_split(t)) ? reinterpret_cast<double2*>(ws + L.gbuf2) : nullptr;
  uint16_t* planes0 = (mixed && t >= 5) ? reinterpret_cast<uint16_t*>(ws + L.planes) : nullptr;
  unsigned long long* defect = reinterpret_cast<unsigned long long*>(ws + L.scratch);
  const double2* psi = static_cast<const double2*>(p.psi);

  const bool dbl = (flags & QPE_PREFIX_DOUBLING) != 0;
  const size_t amp = mixed ? 8 : 16;
  QPE_HIP(ctx, launch_zero_u64(defect, 1, s));
  const double2* U0 = static_cast<const double2*>(p.U);
  const double2* psi0 = psi;
  const bool rot = rotate_on(mixed, t, rot_mode(flags), polar);
  if (rot) {
    // U' goes to A: it is read as V_0 by step 0 and by the first square,
    // which writes B; A is next written by the power step of k = 1 (when
    // it gets a Newton-Schulz step) or k = 2. M psi goes to the second state buffer, read by the H layer
    // before step 0 writes there (the prefix-doubling form never does).
    double2* Ur = A;
    double2* pr = static_cast<double2*>(s1);
    qpe_status st = rotate_target(ctx, t, U0, psi, Ur, pr, defect);
    if (st != QPE_OK) return st;
    U0 = Ur;
    psi0 = pr;
  }
  const bool f16 = use_f16(form, flags) && t >= 5;
  // The operator planes of step k. The prefix-doubling form with split-FP16
  // products alternates two sets by the parity of k: every power from V_1 on
  // is split on the power chain's stream (by the square's epilogue or the
  // Newton-Schulz update), so power step k, which writes set k & 1, only has
  // to wait for controlled step k-2, the last reader of that set.
  const bool par = dbl && f16;
  auto planes_of = [&](int k) { return par && (k & 1) ? reinterpret_cast<uint16_t*>(ws + L.planes2) : planes0; };
  float* sigma = reinterpret_cast<float*>(defect + kScratchSigma);
  if (f16) QPE_HIP(ctx, launch_state_scale(psi0, n, t, sigma, s));
  {
    // Prefix doubling writes every row j >= 1 in the step of its top bit,
    // so the H layer only has to fill row 0.
    TimerScope ts(ctx, QPE_TIMER_HLAYER);
    QPE_HIP(ctx, launch_h_broadcast(mixed, psi0, s0, n, t, s, dbl));
  }
  // Prefix-doubling form: the power chain runs on the context's second
  // stream, one step ahead of the controlled products, most of which are
  // small (step k has 2^k rows), so the squarings overlap them. Power step k
  // writes the buffer that held V_{k-2} and the planes of step k (so it waits
  // for controlled step k-2) and, with a Newton-Schulz correction, also
  // V_{k-1}'s buffer. Those stages also wait for controlled step k-1 where
  // V_{k-1} is read on the context stream: by the controlled step itself
  // (d <= 16, the FP64 form) or by its operator split (the split-BF16
  // scheme, with one plane set; V_0 at k = 1). Controlled step k waits for
  // power step k. One stream while the power
  // chain's timer class records (its events go to the context stream),
  // without allow_aux (qpe_run_static), or with the one-stream schedule
  // variant.
  const bool timers = ctx->timing && ((ctx->timer_mask >> QPE_TIMER_POWERS) & 1u);
  const bool pipe = dbl && allow_aux && n >= 2 && !timers && ctx->variant[QPE_KERNEL_BATCH_SCHED][0] != 1;
  hipEvent_t ctrl_done[QPE_MAX_N_MEAS] = {};
  int next_ev = 0;
  bool aux_open = false;  // the second stream has work the context stream has not waited for
  auto mark = [&](hipStream_t on, hipEvent_t* out) -> qpe_status {
    hipEvent_t e = ctx->sched_ev[size_t(next_ev++) % ctx->sched_ev.size()];
    QPE_HIP(ctx, hipEventRecord(e, on));
    *out = e;
    return QPE_OK;
  };
  if (pipe) {
    qpe_status st = ensure_sched(ctx, kSchedEvents);
    if (st != QPE_OK) return st;
    hipEvent_t fork;
    if ((st = mark(s, &fork)) != QPE_OK) return st;  // after the rotation and the H layer
    QPE_HIP(ctx, hipStreamWaitEvent(ctx->aux, fork, 0));
  }
  const double2* cur = U0;
  qpe_status loop_st = [&]() -> qpe_status {
  for (int k = 0; k < n; ++k) {
    bool planes_ready = false;  // the Newton-Schulz update already split V_k
    if (k > 0) {
      double2* sq = (cur == A) ? B : A;
      double2* other = (sq == A) ? B : A;
      const bool pk = polar && ns_step(k, n);  // this power gets the correction
      hipStream_t sp = pipe ? ctx->aux : s;
      hipEvent_t before_update = nullptr;
      if (pipe) {
        if (k >= 2) QPE_HIP(ctx, hipStreamWaitEvent(ctx->aux, ctrl_done[k - 2], 0));
        if (pk && !(par && k >= 2)) before_update = ctrl_done[k - 1];
        aux_open = true;
      }
      TimerScope ts(ctx, QPE_TIMER_POWERS);
      qpe_status st = square_and_polar(ctx, d, cur, sq, G, other, pk, defect, planes_of(k), G2, &planes_ready, f16,
                                       sp, before_update);
      if (st != QPE_OK) return st;
      cur = pk ? other : sq;
      if (pipe) {
        hipEvent_t done;
        if ((st = mark(ctx->aux, &done)) != QPE_OK) return st;
        QPE_HIP(ctx, hipStreamWaitEvent(s, done, 0));
        aux_open = false;
      }
    }
    qpe_status st;
    if (dbl) {
      // rows [0, 2^k) of s0 -> rows [2^k, 2^(k+1)) of s0: 2^k outputs, as a
      // "register" of k+1 qubits whose second buffer starts at row 2^k.
      char* upper = static_cast<char*>(s0) + (size_t(1) << k) * size_t(d) * amp;
      st = controlled(ctx, mixed, k + 1, t, k, cur, s0, upper, planes_of(k), kDoubling, !planes_ready,
                      f16 ? sigma : nullptr);
    } else {
      st = controlled(ctx, mixed, n, t, k, cur, s0, s1, planes0, (uint64_t(1) << k) - 1, !planes_ready,
                      f16 ? sigma : nullptr);
    }
    if (st != QPE_OK) return st;
    if (pipe && (st = mark(s, &ctrl_done[k])) != QPE_OK) return st;
  }
  return QPE_OK;
  }();
  if (loop_st != QPE_OK) {
    if (aux_open) {
      // a failed run still leaves the context stream ordered after the work
      // already enqueued on the second one (best effort, unchecked)
      hipEvent_t e = ctx->sched_ev[size_t(next_ev) % ctx->sched_ev.size()];
      if (hipEventRecord(e, ctx->aux) == hipSuccess) (void)hipStreamWaitEvent(s, e, 0);
    }
    return loop_st;
  }
  qpe_status st = iqft_and_probs(ctx, mixed, n, t, s0, s1, !dbl, p.prob, reinterpret_cast<double2*>(ws + L.tw_hi),
                                 reinterpret_cast<double2*>(ws + L.tw_lo), keep_state);
  if (st != QPE_OK) return st;
  // the second state buffer is free once the inverse QFT has read it
  if (report)
    QPE_HIP(ctx, launch_report(p.prob, n, psi, t, polar ? defect : nullptr,
                               rot ? reinterpret_cast<const double*>(defect + kScratchPeak) : nullptr,
                               mixed && t >= 5, report, static_cast<double*>(s1), s));
  return QPE_OK;
}

// Batched run: one grouped launch per (stage, step) covers every instance
// that takes part in it. The descriptors and launch tables are written on
// the device by setup kernels whose inputs travel as kernel arguments, so
// the whole sequence can be captured into a HIP graph and replayed.
int timer_of(int kind) {
  switch (kind) {
    case BK_HLAYER: return QPE_TIMER_HLAYER;
    case BK_ROTHASH: case BK_ROTPSI: case BK_ROTU: return QPE_TIMER_POWERS;
    case BK_SQ: case BK_GRAM: case BK_GRAM_SK: case BK_SUBI: case BK_CORR:
    case BK_NSPREP: case BK_NS_M32: case BK_NS_M64: case BK_NS_M128: case BK_NSUPD: case BK_PCOPY:
      return QPE_TIMER_POWERS;
    case BK_SPLIT: return QPE_TIMER_SPLIT;
    case BK_CTRL_SMALL: case BK_CTRL_M32: case BK_CTRL_M64: case BK_CTRL_M128: case BK_CTRL_M256:
    case BK_CTRL_F64:
      return QPE_TIMER_CTRL_GEMM;
    case BK_QFT: case BK_QFT_LAST: return QPE_TIMER_QFT;
    case BK_PROB: case BK_REPORT: return QPE_TIMER_PROB;
  }
  return -1;
}

// Variant bits of the grouped kernels from the context's batched classes.
int batch_variant_flags(const qpe_ctx* ctx) {
  int f = 0;
  if (ctx->variant[QPE_KERNEL_BATCH_GEMM][0] == 2) f |= kBatchGemm64;
  const int vc = ctx->variant[QPE_KERNEL_BATCH_CTRL][0];
  if (vc == 1) f |= kBatchCtrlInStep;
  if (vc == 3) f |= kBatchPersistent;
  return f;
}

// Launch kinds of power step k that only read V_{k-1} and write the
// instance's square and Gram buffers, which no state-side launch touches:
// they may run while the controlled products of step k-1 still read V_{k-1}
// and the operator planes.
bool chain_ahead(int kind) { return kind == BK_SQ || kind == BK_GRAM || kind == BK_GRAM_SK || kind == BK_SUBI; }
// The rest of power step k: they write V_k's slot, the planes (the mixed
// Newton-Schulz product stages conj(E) there) or the staging in it, so they
// wait for the controlled products of step k-1.
bool chain_after(int kind) {
  return kind == BK_CORR || kind == BK_NSPREP || kind == BK_NS_M32 || kind == BK_NS_M64 || kind == BK_NS_M128 ||
         kind == BK_NSUPD || kind == BK_PCOPY;
}
// State-side launches of controlled step k.
bool state_step(int kind) {
  return kind == BK_SPLIT || kind == BK_CTRL_SMALL || kind == BK_CTRL_M32 || kind == BK_CTRL_M64 ||
         kind == BK_CTRL_M128 || kind == BK_CTRL_M256 || kind == BK_CTRL_F64;
}
// allow_aux: the two-stream schedule may be used (it creates the second
// stream and its events on first use).
qpe_status run_batch(qpe_ctx* ctx, const qpe_problem* p, int count, int form, unsigned flags, char* ws,
                     qpe_report* report, bool allow_aux = true) {
  const bool mixed = form == QPE_FORM_MIXED, polar = !(flags & QPE_NO_POLAR);
  const int bf = (polar ? kBatchPolar : 0) | ((flags & QPE_PREFIX_DOUBLING) ? kBatchDoubling : 0) |
                 batch_variant_flags(ctx) | (rot_mode(flags) << kBatchRotShift) |
                 (use_f16(form, flags) ? kBatchF16 : 0);
  hipStream_t s = ctx->stream;
  const BatchPlan P = plan_batch(p, count, form, flags, true, bf & kBatchGemm64);
  int32_t* tables = reinterpret_cast<int32_t*>(ws);
  InstDesc* desc = reinterpret_cast<InstDesc*>(ws + P.desc_off);
  for (int first = 0; first < count; first += kBatchChunk) {
    BatchProblem chunk[kBatchChunk];
    int c = count - first < kBatchChunk ? count - first : kBatchChunk;
    for (int i = 0; i < c; ++i) {
      const qpe_problem& q = p[first + i];
      const void* Uq = q.U;
      const void* pq = q.psi;
      if (rotate_on(mixed, q.n_mat, rot_mode(flags), polar)) {
        // The instance's own idle buffers: the grouped power chain writes its
        // first square to vbuf and its corrected power (or, without the
        // polar step, the square of k = 2) to tbuf, so U' sits in tbuf (read
        // as V_0 by step 0 and by the first square); M psi in the second
        // state buffer. The grouped rotation kernels write both.
        char* b = ws + P.inst_base[first + i];
        const RunLayout L = run_layout(q.n_meas, q.n_mat, form, flags);
        Uq = b + L.tbuf;
        pq = b + L.state1;
      }
      chunk[i] = BatchProblem{q.n_meas, q.n_mat, Uq, pq, q.U, q.psi, q.prob,
                              report ? static_cast<void*>(report + first + i) : nullptr,
                              uint64_t(P.inst_base[first + i])};
    }
    QPE_HIP(ctx, launch_batch_descs(desc, ws, chunk, first, c, s));
  }
  bool stage_small = false;  // an instance with d = 8 or 16 takes the small controlled step
  for (int i = 0; i < count; ++i) stage_small |= p[i].n_mat == 3 || p[i].n_mat == 4;
  // the t shared by every instance with d >= 256, or 0 (the persistent wide
  // controlled step needs one d per launch)
  int wide_t = -1;
  for (int i = 0; i < count; ++i)
    if (p[i].n_mat >= 8) wide_t = (wide_t < 0 || wide_t == p[i].n_mat) ? p[i].n_mat : 0;
  if (wide_t < 0) wide_t = 0;
  const int nl = int(P.launches.size());
  for (int first = 0; first < nl; first += kBatchLaunchChunk) {
    int c = nl - first < kBatchLaunchChunk ? nl - first : kBatchLaunchChunk;
    QPE_HIP(ctx, launch_batch_tables(desc, count, tables, P.launches.data() + first, c, mixed, bf, s));
  }
  // Two-stream schedule: the power chain goes to ctx->aux. Step k's first
  // state-side launch waits for the chain through step k; the second part
  // of power step k waits for the state side through step k-1 (the plan
  // lists, for each k, the chain's launches before the state's). Per-kernel
  // timers bracket launches on the context stream, so while the power
  // chain's timer class records, the run keeps one stream.
  const bool timers = ctx->timing && ((ctx->timer_mask >> QPE_TIMER_POWERS) & 1u);
  const bool pipe = allow_aux && polar && ctx->variant[QPE_KERNEL_BATCH_SCHED][0] != 1 && !timers;
  int next_ev = 0;
  bool forked = false, aux_pending = false;
  int ctrl_waited = -1;  // the last step whose state-side launches the chain waited for
  hipStream_t s_state = s;
  auto hop = [&](hipStream_t from, hipStream_t to) -> qpe_status {
    // `to` waits for everything enqueued on `from` so far
    hipEvent_t e = ctx->sched_ev[size_t(next_ev++) % ctx->sched_ev.size()];
    QPE_HIP(ctx, hipEventRecord(e, from));
    QPE_HIP(ctx, hipStreamWaitEvent(to, e, 0));
    return QPE_OK;
  };
  if (pipe) {
    qpe_status st = ensure_sched(ctx, kSchedEvents);
    if (st != QPE_OK) return st;
  }
  qpe_status result = [&]() -> qpe_status {
  for (int l = 0; l < nl; ++l) {
    const BatchLaunch& L = P.launches[l];
    const int32_t* tab = tables + L.table_off;
    const int64_t tiles = P.tiles[l];
    s = s_state;
    if (pipe) {
      const bool ahead = chain_ahead(L.kind), after = chain_after(L.kind);
      qpe_status st = QPE_OK;
      if (!forked && (ahead || after || state_step(L.kind))) {
        // the chain starts once the set-up launches (rotation, tables) are done
        forked = true;
        if ((st = hop(s_state, ctx->aux)) != QPE_OK) return st;
      }
      if (ahead || after) {
        if (after && ctrl_waited < L.step - 1) {
          ctrl_waited = L.step - 1;
          if ((st = hop(s_state, ctx->aux)) != QPE_OK) return st;
        }
        s = ctx->aux;
        aux_pending = true;
      } else if (aux_pending) {
        // every later state-side launch needs the chain's work so far (and
        // the run ends joined)
        aux_pending = false;
        if ((st = hop(ctx->aux, s_state)) != QPE_OK) return st;
      }
    }
    TimerScope ts(ctx, timer_of(L.kind));
    switch (L.kind) {
      case BK_SQ:
      case BK_GRAM:
      case BK_CORR:
        QPE_HIP(ctx, launch_batch_zgemm(L.kind, L.step, desc, tab, tiles, mixed, bf, s));
        break;
      case BK_GRAM_SK:
        QPE_HIP(ctx, launch_batch_gram_split(L.step, desc, tab, tiles, mixed, bf, s));
        break;
      case BK_CTRL_SMALL:
        QPE_HIP(ctx, launch_batch_ctrl_small(L.step, desc, tab, tiles, mixed, stage_small, bf, s));
        break;
      case BK_CTRL_M32:
      case BK_CTRL_M64:
      case BK_CTRL_M128:
      case BK_CTRL_M256:
      case BK_NS_M32:
      case BK_NS_M64:
      case BK_NS_M128:
        QPE_HIP(ctx, launch_batch_ctrl_mixed(L.kind, L.step, desc, tab, tiles, bf, s, wide_t));
        break;
      case BK_CTRL_F64:
        QPE_HIP(ctx, launch_batch_ctrl_f64(L.step, desc, tab, tiles, bf, s));
        break;
      case BK_ROTHASH:
      case BK_ROTPSI:
      case BK_ROTU:
        QPE_HIP(ctx, launch_batch_rotate(L.kind, L.step, desc, tab, tiles, mixed, bf, s));
        break;
      case BK_QFT:
      case BK_QFT_LAST: {
        bool wide = false;  // an instance takes two rows per thread in this pass
        for (int i = 0; i < count && !wide; ++i) {
          const DftPlan pl = make_dft_plan(p[i].n_meas);
          wide = L.step < pl.npass && qft_two_rows(mixed, pl.bits[L.step], p[i].n_meas, p[i].n_mat);
        }
        if (L.kind == BK_QFT)
          QPE_HIP(ctx, launch_batch_qft(L.step, desc, tab, tiles, mixed, wide, bf, s));
        else
          QPE_HIP(ctx, launch_batch_qft_last(L.step, desc, tab, tiles, mixed, wide, bf, s));
        break;
      }
      default:
        QPE_HIP(ctx, launch_batch_elementwise(L.kind, L.step, desc, tab, tiles, mixed, bf, s));
    }
  }
  if (pipe && aux_pending) {
    aux_pending = false;
    return hop(ctx->aux, s_state);
  }
  return QPE_OK;
  }();
  if (result != QPE_OK && aux_pending) {
    // a failed run still leaves the context stream ordered after the work
    // already enqueued on the second one (best effort, unchecked)
    hipEvent_t e = ctx->sched_ev[size_t(next_ev) % ctx->sched_ev.size()];
    if (hipEventRecord(e, ctx->aux) == hipSuccess) (void)hipStreamWaitEvent(s_state, e, 0);
  }
  return result;
}

const char* const kStatusText[] = {
    "QPE_OK",
    "QPE_ERR_ARG: null pointer, unknown form or flag, or bad count",
    "QPE_ERR_SIZE: n_meas or n_mat out of range",
    "QPE_ERR_ALIGN: a device pointer is misaligned",
    "QPE_ERR_WORKSPACE: workspace missing, misaligned or too small",
    "QPE_ERR_OOM: host allocation failed",
    "QPE_ERR_NO_DEVICE: no usable HIP device",
    "QPE_ERR_HIP: a HIP call or kernel launch failed",
    "QPE_ERR_UNSUPPORTED: not implemented by this library",
};

}  // namespace

QPE_API const char* qpe_status_string(int status) {
  if (status < 0 || status > QPE_ERR_UNSUPPORTED) return "unknown qpe_status";
  return kStatusText[status];
}

QPE_API const char* qpe_version(void) { return "0.1.0"; }

QPE_API const char* qpe_last_error(const qpe_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

// ---------------------------------------------- static workspace (no allocation)
//
// qpe_run_static runs in this array instead of a caller workspace. Each
// device the library runs on holds its own copy (loaded with the code object,
// kept until the process ends). In host code the name `scratch` is only a
// host-side stand-in: its device address on each device comes from
// hipGetSymbolAddress, taken once per device when the first context on that
// device is created, and only that address is used afterwards.
static __device__ __align__(256) unsigned char scratch[QPE_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
hipError_t g_static_err[kMaxDevices] = {};
bool g_static_tried[kMaxDevices] = {};

// With `device` current: look up the array's address on it (once).
void fetch_static_workspace(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (g_static_tried[device]) return;
  g_static_tried[device] = true;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) {
    g_static_ptr[device] = p;
  } else {
    g_static_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
    (void)hipGetLastError();  // do not leave the error for the caller's next call
  }
}

void* static_workspace(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  *err = g_static_err[device];
  return g_static_ptr[device];
}
}  // namespace

QPE_API qpe_status qpe_ctx_create(qpe_ctx** out, int device, void* stream) {
  if (!out) return QPE_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return QPE_ERR_NO_DEVICE;
  if (device < 0 || device >= count) return QPE_ERR_NO_DEVICE;
  qpe_ctx* c = new (std::nothrow) qpe_ctx;
  if (!c) return QPE_ERR_OOM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (const char* f = std::getenv("QPE_FAULT_INJECT")) c->fault_at = std::strtol(f, nullptr, 10);
  {
    // set-up of the static workspace on this device (its failure only
    // affects qpe_run_static, which then reports it), and the second stream
    // and events of the two-stream batch schedule, created here so that a
    // first batched run under graph capture creates nothing (best effort:
    // the first batched run retries what failed, and reports a failure)
    DeviceGuard guard(device);
    if (guard.ok) {
      fetch_static_workspace(device);
      if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) c->aux = nullptr;
      for (int i = 0; i < kSchedEvents; ++i) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) break;
        c->sched_ev.push_back(e);
      }
    }
  }
  *out = c;
  return QPE_OK;
}

static int variant_count(int kernel_class) {
  switch (kernel_class) {
    case QPE_KERNEL_CTRL_MIXED: return ctrl_mixed_variants();
    case QPE_KERNEL_ZGEMM: return zgemm_variants();
    case QPE_KERNEL_CTRL_F64: return ctrl_f64_variants();
    case QPE_KERNEL_BATCH_CTRL: return 3;
    case QPE_KERNEL_BATCH_GEMM: return 2;
    case QPE_KERNEL_BATCH_SCHED: return 2;
  }
  return -1;
}

QPE_API qpe_status qpe_kernel_variants(int kernel_class, int* count) {
  if (!count) return QPE_ERR_ARG;
  int c = variant_count(kernel_class);
  if (c < 0) return QPE_ERR_ARG;
  *count = c;
  return QPE_OK;
}

QPE_API qpe_status qpe_ctx_set_variant(qpe_ctx* ctx, int kernel_class, int n_mat, int variant) {
  if (!ctx) return QPE_ERR_ARG;
  int c = variant_count(kernel_class);
  if (c < 0 || variant < 0 || variant > c) return QPE_ERR_ARG;
  if (n_mat < -1 || n_mat > QPE_MAX_N_MAT) return QPE_ERR_SIZE;
  const bool batched = kernel_class == QPE_KERNEL_BATCH_CTRL || kernel_class == QPE_KERNEL_BATCH_GEMM ||
                       kernel_class == QPE_KERNEL_BATCH_SCHED;
  for (int t = 0; t <= QPE_MAX_N_MAT; ++t)
    if (batched || n_mat < 0 || t == n_mat) ctx->variant[kernel_class][t] = variant;
  return QPE_OK;
}

QPE_API qpe_status qpe_ctx_get_variant(const qpe_ctx* ctx, int kernel_class, int n_mat, int* variant) {
  if (!ctx || !variant || variant_count(kernel_class) < 0) return QPE_ERR_ARG;
  if (n_mat < 0 || n_mat > QPE_MAX_N_MAT) return QPE_ERR_SIZE;
  *variant = ctx->variant[kernel_class][n_mat];
  return QPE_OK;
}

// Autotuner: for each kernel class the problem uses, time whole circuits
// with every variant of that class (the other stages do not change) and keep
// the fastest for this n_mat. Classes are tuned one after another, each with
// the choices made so far in place.
QPE_API qpe_status qpe_autotune(qpe_ctx* ctx, const qpe_problem* problem, int form, unsigned flags, void* workspace,
                                size_t workspace_bytes, int reps, int* chosen, double* class_ms) {
  if (!ctx || !chosen) return QPE_ERR_ARG;
  if (reps < 1 || reps > 1000) return QPE_ERR_ARG;
  qpe_status s = qpe_check_run(problem, 1, form, flags, workspace, workspace_bytes, nullptr);
  if (s != QPE_OK) return s;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  const int t = problem->n_mat;
  const bool mixed = form == QPE_FORM_MIXED;
  bool uses[QPE_KERNEL_COUNT] = {};
  uses[QPE_KERNEL_ZGEMM] = problem->n_meas >= 2;
  uses[QPE_KERNEL_CTRL_MIXED] = mixed && t >= 5;
  uses[QPE_KERNEL_CTRL_F64] = !mixed && t >= 5;
  if (class_ms)
    for (int i = 0; i < QPE_KERNEL_COUNT * QPE_TUNE_MAX_VARIANTS; ++i) class_ms[i] = -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(ctx, hipErrorOutOfMemory, "hipEventCreate");
  }
  // timing a run with the per-launch timers on would time them too
  const bool was_timing = ctx->timing;
  ctx->timing = false;
  qpe_status st = QPE_OK;
  char* ws = static_cast<char*>(workspace);
  for (int c = 0; c < QPE_KERNEL_COUNT && st == QPE_OK; ++c) {
    chosen[c] = ctx->variant[c][t];
    if (!uses[c]) continue;
    const int nv = variant_count(c);
    double best = 1e300;
    int best_v = 0;
    for (int v = 0; v <= nv && v < QPE_TUNE_MAX_VARIANTS && st == QPE_OK; ++v) {
      ctx->variant[c][t] = v;
      st = run_one(ctx, *problem, form, flags, ws, nullptr);  // warm-up
      if (st != QPE_OK) break;
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = hip_fail(ctx, hipErrorUnknown, "hipEventRecord"); break; }
      for (int r = 0; r < reps && st == QPE_OK; ++r) st = run_one(ctx, *problem, form, flags, ws, nullptr);
      if (st != QPE_OK) break;
      hipError_t he = hipEventRecord(e1, ctx->stream);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) { st = hip_fail(ctx, he, "autotune timing"); break; }
      const double per = double(ms) / reps;
      if (class_ms) class_ms[c * QPE_TUNE_MAX_VARIANTS + v] = per;
      if (per < best) {
        best = per;
        best_v = v;
      }
    }
    ctx->variant[c][t] = best_v;
    chosen[c] = best_v;
  }
  ctx->timing = was_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

QPE_API qpe_status qpe_autotune_batch(qpe_ctx* ctx, const qpe_problem* problems, int count, int form,
                                      unsigned flags, void* workspace, size_t workspace_bytes, int reps,
                                      int* chosen, double* class_ms) {
  if (!ctx || !chosen || count < 2) return QPE_ERR_ARG;
  if (reps < 1 || reps > 1000) return QPE_ERR_ARG;
  qpe_status s = qpe_check_run(problems, count, form, flags, workspace, workspace_bytes, nullptr);
  if (s != QPE_OK) return s;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  const bool mixed = form == QPE_FORM_MIXED;
  bool uses[QPE_KERNEL_COUNT] = {};
  for (int i = 0; i < count; ++i) {
    uses[QPE_KERNEL_BATCH_GEMM] |= problems[i].n_meas >= 2;
    uses[QPE_KERNEL_BATCH_SCHED] |= problems[i].n_meas >= 2 && !(flags & QPE_NO_POLAR);
    uses[QPE_KERNEL_BATCH_CTRL] |= mixed && problems[i].n_mat >= 7;
  }
  if (class_ms)
    for (int i = 0; i < QPE_KERNEL_COUNT * QPE_TUNE_MAX_VARIANTS; ++i) class_ms[i] = -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(ctx, hipErrorOutOfMemory, "hipEventCreate");
  }
  const bool was_timing = ctx->timing;
  ctx->timing = false;
  qpe_status st = QPE_OK;
  char* ws = static_cast<char*>(workspace);
  for (int c = 0; c < QPE_KERNEL_COUNT && st == QPE_OK; ++c) {
    chosen[c] = ctx->variant[c][0];
    if (!uses[c]) continue;
    const int nv = variant_count(c);
    double best = 1e300;
    int best_v = 0;
    auto set_all = [&](int v) {
      for (int t = 0; t <= QPE_MAX_N_MAT; ++t) ctx->variant[c][t] = v;
    };
    for (int v = 0; v <= nv && v < QPE_TUNE_MAX_VARIANTS && st == QPE_OK; ++v) {
      set_all(v);
      st = run_batch(ctx, problems, count, form, flags, ws, nullptr);  // warm-up
      if (st != QPE_OK) break;
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = hip_fail(ctx, hipErrorUnknown, "hipEventRecord"); break; }
      for (int r = 0; r < reps && st == QPE_OK; ++r) st = run_batch(ctx, problems, count, form, flags, ws, nullptr);
      if (st != QPE_OK) break;
      hipError_t he = hipEventRecord(e1, ctx->stream);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) { st = hip_fail(ctx, he, "autotune timing"); break; }
      const double per = double(ms) / reps;
      if (class_ms) class_ms[c * QPE_TUNE_MAX_VARIANTS + v] = per;
      if (per < best) {
        best = per;
        best_v = v;
      }
    }
    set_all(best_v);
    chosen[c] = best_v;
  }
  ctx->timing = was_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

QPE_API qpe_status qpe_ctx_set_stream(qpe_ctx* ctx, void* stream) {
  if (!ctx) return QPE_ERR_ARG;
  ctx->stream = static_cast<hipStream_t>(stream);
  return QPE_OK;
}

static void free_timers(qpe_ctx* ctx) {
  for (auto& p : ctx->timers) {
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  ctx->timers.clear();
  ctx->timers_used = 0;
  ctx->timing = false;
}

QPE_API qpe_status qpe_ctx_destroy(qpe_ctx* ctx) {
  if (ctx) {
    free_timers(ctx);
    DeviceGuard guard(ctx->device);
    for (hipEvent_t e : ctx->sched_ev) (void)hipEventDestroy(e);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  }
  delete ctx;
  return QPE_OK;
}

QPE_API qpe_status qpe_ctx_enable_timing(qpe_ctx* ctx, int max_pairs) {
  if (!ctx || max_pairs < 1 || max_pairs > (1 << 20)) return QPE_ERR_ARG;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  free_timers(ctx);
  ctx->timers.reserve(size_t(max_pairs));
  for (int i = 0; i < max_pairs; ++i) {
    qpe_timer_pair p{};
    hipError_t e = hipEventCreate(&p.start);
    if (e == hipSuccess) e = hipEventCreate(&p.stop);
    if (e != hipSuccess) {
      free_timers(ctx);
      return hip_fail(ctx, e, "hipEventCreate");
    }
    p.which = -1;
    ctx->timers.push_back(p);
  }
  ctx->timing = true;
  return QPE_OK;
}

QPE_API qpe_status qpe_ctx_set_timing_mask(qpe_ctx* ctx, unsigned mask) {
  if (!ctx || (mask >> QPE_TIMER_COUNT) != 0u) return QPE_ERR_ARG;
  ctx->timer_mask = mask;
  return QPE_OK;
}

QPE_API qpe_status qpe_ctx_reset_timing(qpe_ctx* ctx) {
  if (!ctx) return QPE_ERR_ARG;
  ctx->timers_used = 0;
  return QPE_OK;
}

QPE_API qpe_status qpe_ctx_read_timing(qpe_ctx* ctx, int timer, int* launches, double* total_ms) {
  if (!ctx || !launches || !total_ms || timer < 0 || timer >= QPE_TIMER_COUNT) return QPE_ERR_ARG;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  int cnt = 0;
  double sum = 0.0;
  for (size_t i = 0; i < ctx->timers_used; ++i) {
    const qpe_timer_pair& p = ctx->timers[i];
    if (p.which != timer) continue;
    QPE_HIP(ctx, hipEventSynchronize(p.stop));
    float ms = 0.f;
    QPE_HIP(ctx, hipEventElapsedTime(&ms, p.start, p.stop));
    ++cnt;
    sum += ms;
  }
  *launches = cnt;
  *total_ms = sum;
  return QPE_OK;
}

QPE_API qpe_status qpe_workspace_size(const qpe_problem* problems, int count, int form, unsigned flags,
                                      size_t* bytes) {
  if (!problems || !bytes || count < 1) return QPE_ERR_ARG;
  qpe_status s = check_form_flags(form, flags);
  if (s != QPE_OK) return s;
  for (int i = 0; i < count; ++i) {
    s = check_problem(problems[i], false);
    if (s != QPE_OK) return s;
  }
  if (count > 1 && !plan_batch(problems, count, form, flags, true).ok) return QPE_ERR_SIZE;
  *bytes = workspace_need(problems, count, form, flags);
  return QPE_OK;
}

QPE_API qpe_status qpe_check_run(const qpe_problem* problems, int count, int form, unsigned flags,
                                 const void* workspace, size_t workspace_bytes, const void* report) {
  if (!problems || count < 1) return QPE_ERR_ARG;
  qpe_status s = check_form_flags(form, flags);
  if (s != QPE_OK) return s;
  for (int i = 0; i < count; ++i) {
    s = check_problem(problems[i], true);
    if (s != QPE_OK) return s;
  }
  if (report && misaligned(report, 8)) return QPE_ERR_ALIGN;
  if (count > 1 && !plan_batch(problems, count, form, flags, true).ok) return QPE_ERR_SIZE;
  return check_workspace(workspace, workspace_bytes, workspace_need(problems, count, form, flags));
}

namespace {
// qpe_run; allow_aux = false keeps a batch on the context stream alone (the
// two-stream schedule creates its stream and events on first use).
qpe_status run_checked(qpe_ctx* ctx, const qpe_problem* problems, int count, int form, unsigned flags,
                       void* workspace, size_t workspace_bytes, qpe_report* report, bool allow_aux) {
  if (!ctx) return QPE_ERR_ARG;
  qpe_status s = qpe_check_run(problems, count, form, flags, workspace, workspace_bytes, report);
  if (s != QPE_OK) return s;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  if (count == 1)
    return run_one(ctx, problems[0], form, flags, static_cast<char*>(workspace), report, false, allow_aux);
  return run_batch(ctx, problems, count, form, flags, static_cast<char*>(workspace), report, allow_aux);
}
}  // namespace

QPE_API qpe_status qpe_run(qpe_ctx* ctx, const qpe_problem* problems, int count, int form, unsigned flags,
                           void* workspace, size_t workspace_bytes, qpe_report* report) {
  return run_checked(ctx, problems, count, form, flags, workspace, workspace_bytes, report, true);
}

QPE_API qpe_status qpe_run_static(qpe_ctx* ctx, const qpe_problem* problems, int count, int form, unsigned flags,
                                  qpe_report* report) {
  if (!ctx) return QPE_ERR_ARG;
  size_t need = 0;
  qpe_status s = qpe_workspace_size(problems, count, form, flags, &need);
  if (s != QPE_OK) return s;
  if (need > size_t(QPE_STATIC_WORKSPACE_BYTES)) {
    ctx->last_error = "qpe_run_static: these problems need a workspace of " + std::to_string(need) +
                      " bytes; the static workspace holds " + std::to_string(size_t(QPE_STATIC_WORKSPACE_BYTES));
    return QPE_ERR_WORKSPACE;
  }
  hipError_t e = hipSuccess;
  void* ws = static_workspace(ctx->device, &e);
  if (!ws) return hip_fail(ctx, e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
  // a run ignores the workspace's contents on entry; with one stream it
  // creates and allocates nothing
  return run_checked(ctx, problems, count, form, flags, ws, size_t(QPE_STATIC_WORKSPACE_BYTES), report, false);
}

QPE_API qpe_status qpe_run_state(qpe_ctx* ctx, const qpe_problem* problem, int form, unsigned flags,
                                 void* workspace, size_t workspace_bytes, void* state_out, qpe_report* report) {
  if (!ctx || !state_out) return QPE_ERR_ARG;
  qpe_status s = qpe_check_run(problem, 1, form, flags, workspace, workspace_bytes, report);
  if (s != QPE_OK) return s;
  if (misaligned(state_out, form == QPE_FORM_MIXED ? 8 : 16)) return QPE_ERR_ALIGN;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  s = run_one(ctx, *problem, form, flags, static_cast<char*>(workspace), report, true);
  if (s != QPE_OK) return s;
  const int n = problem->n_meas, t = problem->n_mat;
  const RunLayout L = run_layout(n, t, form, flags);
  // the DFT passes leave the transform unnormalised: A = 2^(-n/2) X
  const double scale = std::ldexp(1.0, -(n / 2)) * ((n & 1) ? std::sqrt(0.5) : 1.0);
  QPE_HIP(ctx, launch_gather_state(form == QPE_FORM_MIXED, static_cast<char*>(workspace) + L.state0, state_out, n,
                                   t, make_dft_plan(n), scale, ctx->stream));
  // a rotated run's final state is M times the circuit's: rotate it back
  if (rotate_on(form == QPE_FORM_MIXED, t, rot_mode(flags), !(flags & QPE_NO_POLAR)))
    QPE_HIP(ctx, launch_unrotate_state(form == QPE_FORM_MIXED, state_out, n, t,
                                       reinterpret_cast<const unsigned long long*>(static_cast<char*>(workspace) +
                                                                                   L.scratch),
                                       ctx->stream));
  return QPE_OK;
}

// ------------------------------------------------------------ stage entries

QPE_API qpe_status qpe_powers_workspace_size(int n_mat, size_t* bytes) {
  if (!bytes) return QPE_ERR_ARG;
  if (n_mat < 0 || n_mat > QPE_MAX_N_MAT) return QPE_ERR_SIZE;
  size_t mat = (size_t(1) << (2 * n_mat)) * 16;
  *bytes = (2 + gram_extra_slots(n_mat)) * align_up(mat) + align_up(64);
  return QPE_OK;
}

QPE_API qpe_status qpe_powers(qpe_ctx* ctx, int n_mat, const void* U, int count_k, unsigned flags, void* V_out,
                              void* workspace, size_t workspace_bytes, qpe_report* report) {
  if (!ctx || !U || !V_out) return QPE_ERR_ARG;
  if (n_mat < 0 || n_mat > QPE_MAX_N_MAT || count_k < 1 || count_k > QPE_MAX_N_MEAS) return QPE_ERR_SIZE;
  if (flags & ~unsigned(QPE_NO_POLAR | QPE_PREFIX_DOUBLING)) return QPE_ERR_ARG;
  if (misaligned(U, 16) || misaligned(V_out, 16) || (report && misaligned(report, 8))) return QPE_ERR_ALIGN;
  size_t need = 0;
  qpe_powers_workspace_size(n_mat, &need);
  qpe_status s = check_workspace(workspace, workspace_bytes, need);
  if (s != QPE_OK) return s;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  const int d = 1 << n_mat;
  const size_t mat = size_t(d) * d;
  char* ws = static_cast<char*>(workspace);
  double2* sq = reinterpret_cast<double2*>(ws);
  double2* g = reinterpret_cast<double2*>(ws + align_up(mat * 16));
  double2* g2 = gram_split(n_mat) ? reinterpret_cast<double2*>(ws + 2 * align_up(mat * 16)) : nullptr;
  unsigned long long* defect =
      reinterpret_cast<unsigned long long*>(ws + (2 + gram_extra_slots(n_mat)) * align_up(mat * 16));
  double2* V = static_cast<double2*>(V_out);
  const bool polar = !(flags & QPE_NO_POLAR);
  QPE_HIP(ctx, launch_zero_u64(defect, 1, ctx->stream));
  QPE_HIP(ctx, hipMemcpyAsync(V, U, mat * 16, hipMemcpyDeviceToDevice, ctx->stream));
  for (int k = 1; k < count_k; ++k) {
    const double2* cur = V + (k - 1) * mat;
    double2* out = V + k * mat;
    const bool pk = polar && ns_step(k, count_k);
    s = square_and_polar(ctx, d, cur, pk ? sq : out, g, out, pk, defect, nullptr, g2);
    if (s != QPE_OK) return s;
  }
  if (report) {
    // Only the defect is meaningful here; copy it into the first field.
    QPE_HIP(ctx, hipMemcpyAsync(report, defect, sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  }
  return QPE_OK;
}

QPE_API qpe_status qpe_controlled_step_workspace_size(int n_meas, int n_mat, int form, size_t* bytes) {
  if (!bytes) return QPE_ERR_ARG;
  qpe_status s = check_sizes(n_meas, n_mat);
  if (s != QPE_OK) return s;
  if (form != QPE_FORM_FP64 && form != QPE_FORM_MIXED) return QPE_ERR_ARG;
  const size_t d = size_t(1) << n_mat, N = size_t(1) << n_meas;
  size_t amp = form == QPE_FORM_MIXED ? 8 : 16;
  *bytes = align_up(N * d * amp) + ((form == QPE_FORM_MIXED && n_mat >= 5) ? align_up(6 * d * d * 2) : 0);
  return QPE_OK;
}

QPE_API qpe_status qpe_controlled_step(qpe_ctx* ctx, int n_meas, int n_mat, int form, int k, const void* V,
                                       void* state, void* workspace, size_t workspace_bytes) {
  if (!ctx || !V || !state) return QPE_ERR_ARG;
  size_t need = 0;
  qpe_status s = qpe_controlled_step_workspace_size(n_meas, n_mat, form, &need);
  if (s != QPE_OK) return s;
  if (k < 0 || k >= n_meas) return QPE_ERR_SIZE;
  if (misaligned(V, 16) || misaligned(state, 16)) return QPE_ERR_ALIGN;
  s = check_workspace(workspace, workspace_bytes, need);
  if (s != QPE_OK) return s;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  const bool mixed = form == QPE_FORM_MIXED;
  const size_t d = size_t(1) << n_mat, N = size_t(1) << n_meas;
  char* ws = static_cast<char*>(workspace);
  void* other = ws;
  uint16_t* planes = reinterpret_cast<uint16_t*>(ws + align_up(N * d * (mixed ? 8 : 16)));
  // pmask 0: every row is read from `state`; updated rows land in `other`.
  s = controlled(ctx, mixed, n_meas, n_mat, k, static_cast<const double2*>(V), state, other, planes, 0);
  if (s != QPE_OK) return s;
  QPE_HIP(ctx, launch_copy_rows_back(mixed, state, other, n_meas, n_mat, k, ctx->stream));
  return QPE_OK;
}

// Twiddle tables, then (fused readout) the partial sums of the last pass.
QPE_API qpe_status qpe_iqft_workspace_size(int n_meas, int n_mat, int form, size_t* bytes) {
  if (!bytes) return QPE_ERR_ARG;
  qpe_status s = check_sizes(n_meas, n_mat);
  if (s != QPE_OK) return s;
  if (form != QPE_FORM_FP64 && form != QPE_FORM_MIXED) return QPE_ERR_ARG;
  const int h = tw_split(n_meas);
  *bytes = align_up((size_t(1) << (n_meas - h)) * 16) + align_up((size_t(1) << h) * 16);
  if (fused_readout(n_meas))
    *bytes += align_up((size_t(readout_groups(form == QPE_FORM_MIXED, n_meas, n_mat)) << n_meas) * 8);
  return QPE_OK;
}

QPE_API qpe_status qpe_iqft_probs(qpe_ctx* ctx, int n_meas, int n_mat, int form, void* state, double* prob,
                                  void* workspace, size_t workspace_bytes) {
  if (!ctx || !state || !prob) return QPE_ERR_ARG;
  size_t need = 0;
  qpe_status s = qpe_iqft_workspace_size(n_meas, n_mat, form, &need);
  if (s != QPE_OK) return s;
  if (misaligned(state, 16) || misaligned(prob, 8)) return QPE_ERR_ALIGN;
  s = check_workspace(workspace, workspace_bytes, need);
  if (s != QPE_OK) return s;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  const int h = tw_split(n_meas);
  char* ws = static_cast<char*>(workspace);
  const size_t hi_bytes = align_up((size_t(1) << (n_meas - h)) * 16), lo_bytes = align_up((size_t(1) << h) * 16);
  double2* tw_hi = reinterpret_cast<double2*>(ws);
  double2* tw_lo = reinterpret_cast<double2*>(ws + hi_bytes);
  void* part = ws + hi_bytes + lo_bytes;  // used only with the fused readout
  return iqft_and_probs(ctx, form == QPE_FORM_MIXED, n_meas, n_mat, state, part, false, prob, tw_hi, tw_lo);
}

// ------------------------------------------------------------- estimators

QPE_API qpe_status qpe_estimate_workspace_size(int count, size_t* bytes) {
  if (!bytes || count < 1) return QPE_ERR_ARG;
  *bytes = size_t(count) * est_workspace_bytes();
  return QPE_OK;
}

QPE_API qpe_status qpe_estimate(qpe_ctx* ctx, const qpe_problem* problems, int count, qpe_estimates* out,
                                void* workspace, size_t workspace_bytes) {
  if (!ctx || !problems || !out || count < 1) return QPE_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    if (!problems[i].prob) return QPE_ERR_ARG;
    if (problems[i].n_meas < 1 || problems[i].n_meas > QPE_MAX_N_MEAS) return QPE_ERR_SIZE;
    if (misaligned(problems[i].prob, 8)) return QPE_ERR_ALIGN;
  }
  if (misaligned(out, 8)) return QPE_ERR_ALIGN;
  size_t need = 0;
  qpe_estimate_workspace_size(count, &need);
  qpe_status s = check_workspace(workspace, workspace_bytes, need);
  if (s != QPE_OK) return s;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  char* ws = static_cast<char*>(workspace);
  for (int i = 0; i < count; ++i)
    QPE_HIP(ctx, launch_estimate(problems[i].prob, problems[i].n_meas, ws + size_t(i) * est_workspace_bytes(),
                                 reinterpret_cast<double*>(out + i), ctx->stream));
  return QPE_OK;
}

QPE_API qpe_status qpe_zgemm(qpe_ctx* ctx, char opA, char opB, int M, int N, int K, const double* alpha,
                             const void* A, int lda, const void* B, int ldb, const double* beta, const void* Cin,
                             int ldcin, void* C, int ldc) {
  if (!ctx || !alpha || !beta || !A || !B || !C) return QPE_ERR_ARG;
  auto op_code = [](char o) { return o == 'N' ? 0 : o == 'T' ? 1 : o == 'C' ? 2 : -1; };
  int oa = op_code(opA), ob = op_code(opB);
  if (oa < 0 || ob < 0) return QPE_ERR_ARG;
  if (M < 1 || N < 1 || K < 1 || M > 65536 || N > 65536 || K > 65536) return QPE_ERR_SIZE;
  const bool use_cin = beta[0] != 0.0 || beta[1] != 0.0;
  if (use_cin && !Cin) return QPE_ERR_ARG;
  // leading dimensions must cover a row of the stored (not op'ed) matrix
  if (lda < (oa == 0 ? K : M) || ldb < (ob == 0 ? N : K) || ldc < N || (use_cin && ldcin < N)) return QPE_ERR_SIZE;
  if (misaligned(A, 16) || misaligned(B, 16) || misaligned(C, 16) || (use_cin && misaligned(Cin, 16)))
    return QPE_ERR_ALIGN;
  ctx->last_error.clear();
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
  ZgemmArgs a{};
  a.M = M;
  a.N = N;
  a.K = K;
  a.A = static_cast<const double2*>(A);
  a.lda = lda;
  a.B = static_cast<const double2*>(B);
  a.ldb = ldb;
  a.alpha = make_double2(alpha[0], alpha[1]);
  a.beta = make_double2(beta[0], beta[1]);
  a.Cin = static_cast<const double2*>(Cin);
  a.ldcin = ldcin;
  a.C = static_cast<double2*>(C);
  a.ldc = ldc;
  int tz = 31 - __builtin_clz(unsigned(N));  // size key: floor(log2 N), clamped
  if (tz > QPE_MAX_N_MAT) tz = QPE_MAX_N_MAT;
  QPE_HIP(ctx, launch_zgemm(oa, ob, a, ctx->stream, ctx->variant[QPE_KERNEL_ZGEMM][tz]));
  return QPE_OK;
}
