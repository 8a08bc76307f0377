/* Host-side checks of the C ABI (include/qpe.h) that need no device: every
 * entry point's argument, size, alignment and workspace validation, the
 * workspace planning of single and batched runs (up to thousands of uneven
 * instances), status strings and variant queries. Built against a copy of
 * the library whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer, so that any out-of-bounds access, overflow or
 * undefined operation in that code aborts the run. Prints "HOST CHECKS OK"
 * and exits 0 when every expectation holds. Fake device pointers are never
 * dereferenced by these paths. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "qpe.h"

static int failures = 0, checks = 0;

#define EXPECT(cond, ...)                                      \
  do {                                                         \
    ++checks;                                                  \
    if (!(cond)) {                                             \
      ++failures;                                              \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);     \
      fprintf(stderr, __VA_ARGS__);                            \
      fprintf(stderr, "\n");                                   \
    }                                                          \
  } while (0)

static qpe_problem prob(int n, int t, uintptr_t base) {
  qpe_problem p;
  p.n_meas = n;
  p.n_mat = t;
  p.U = (const void *)(base + 0x10000);
  p.psi = (const void *)(base + 0x20000);
  p.prob = (double *)(base + 0x30000);
  return p;
}

static uint64_t lcg(uint64_t *s) {
  *s = *s * 6364136223846793005ull + 1442695040888963407ull;
  return *s >> 33;
}

static void status_and_misc(void) {
  for (int s = -3; s <= 12; ++s) {
    const char *txt = qpe_status_string(s);
    EXPECT(txt && strlen(txt) > 0, "status string %d", s);
  }
  EXPECT(strcmp(qpe_status_string(QPE_OK), "QPE_OK") == 0, "QPE_OK text");
  EXPECT(qpe_version() && strlen(qpe_version()) >= 5, "version");
  EXPECT(strcmp(qpe_last_error(NULL), "") == 0, "last_error(NULL)");
  for (int c = -2; c <= QPE_KERNEL_COUNT + 1; ++c) {
    int v = -1;
    qpe_status st = qpe_kernel_variants(c, &v);
    if (c >= 0 && c < QPE_KERNEL_COUNT)
      EXPECT(st == QPE_OK && v >= 1 && v < QPE_TUNE_MAX_VARIANTS, "variants of class %d: %d %d", c, st, v);
    else
      EXPECT(st == QPE_ERR_ARG, "variants of bad class %d", c);
  }
  EXPECT(qpe_kernel_variants(0, NULL) == QPE_ERR_ARG, "variants NULL out");
}

static void single_sizes(void) {
  const unsigned flag_sets[] = {0u,
                                QPE_NO_POLAR,
                                QPE_PREFIX_DOUBLING,
                                QPE_MIX_TARGET,
                                QPE_NO_MIX_TARGET,
                                QPE_SPLIT_BF16,
                                QPE_NO_POLAR | QPE_MIX_TARGET,
                                QPE_PREFIX_DOUBLING | QPE_NO_MIX_TARGET | QPE_SPLIT_BF16};
  for (int form = -1; form <= 2; ++form)
    for (size_t fi = 0; fi < sizeof(flag_sets) / sizeof(flag_sets[0]); ++fi)
      for (int n = -1; n <= QPE_MAX_N_MEAS + 1; ++n)
        for (int t = -1; t <= QPE_MAX_N_MAT + 1; ++t) {
          qpe_problem p = prob(n, t, 0);
          size_t bytes = 0;
          qpe_status st = qpe_workspace_size(&p, 1, form, flag_sets[fi], &bytes);
          const int size_ok = n >= 1 && n <= QPE_MAX_N_MEAS && t >= 0 && t <= QPE_MAX_N_MAT &&
                              n + t <= QPE_MAX_TOTAL_QUBITS;
          if (form != QPE_FORM_FP64 && form != QPE_FORM_MIXED) {
            EXPECT(st == QPE_ERR_ARG, "bad form %d", form);
          } else if (!size_ok) {
            EXPECT(st == QPE_ERR_SIZE, "size n=%d t=%d -> %d", n, t, st);
          } else {
            EXPECT(st == QPE_OK, "size n=%d t=%d form %d flags %u -> %d", n, t, form, flag_sets[fi], st);
            /* at least the two state buffers */
            const size_t amp = form == QPE_FORM_MIXED ? 8 : 16;
            EXPECT(bytes >= 2 * (((size_t)1 << n) << t) * amp, "workspace too small n=%d t=%d", n, t);
            /* the pre-flight agrees with the size, one byte short fails */
            qpe_status c0 = qpe_check_run(&p, 1, form, flag_sets[fi], (void *)0x100000, bytes, NULL);
            qpe_status c1 = qpe_check_run(&p, 1, form, flag_sets[fi], (void *)0x100000, bytes - 1, NULL);
            EXPECT(c0 == QPE_OK && c1 == QPE_ERR_WORKSPACE, "check_run n=%d t=%d: %d %d", n, t, c0, c1);
          }
        }
  /* unknown flag bits, both rotation flags */
  qpe_problem p = prob(8, 4, 0);
  size_t b = 0;
  EXPECT(qpe_workspace_size(&p, 1, QPE_FORM_MIXED, 1u << 9, &b) == QPE_ERR_ARG, "unknown flag");
  EXPECT(qpe_workspace_size(&p, 1, QPE_FORM_MIXED, QPE_MIX_TARGET | QPE_NO_MIX_TARGET, &b) == QPE_ERR_ARG,
         "rotation on and off");
  EXPECT(qpe_workspace_size(NULL, 1, QPE_FORM_MIXED, 0, &b) == QPE_ERR_ARG, "NULL problems");
  EXPECT(qpe_workspace_size(&p, 0, QPE_FORM_MIXED, 0, &b) == QPE_ERR_ARG, "count 0");
  EXPECT(qpe_workspace_size(&p, 1, QPE_FORM_MIXED, 0, NULL) == QPE_ERR_ARG, "NULL bytes");
}

static void alignment_and_pointers(void) {
  qpe_problem p = prob(9, 5, 0);
  size_t need = 0;
  EXPECT(qpe_workspace_size(&p, 1, QPE_FORM_MIXED, 0, &need) == QPE_OK, "size");
  void *ws = (void *)0x100000;
  EXPECT(qpe_check_run(&p, 1, QPE_FORM_MIXED, 0, ws, need, NULL) == QPE_OK, "valid");
  EXPECT(qpe_check_run(&p, 1, QPE_FORM_MIXED, 0, (char *)ws + 16, need, NULL) == QPE_ERR_WORKSPACE, "ws align");
  EXPECT(qpe_check_run(&p, 1, QPE_FORM_MIXED, 0, NULL, need, NULL) == QPE_ERR_WORKSPACE, "ws NULL");
  EXPECT(qpe_check_run(&p, 1, QPE_FORM_MIXED, 0, ws, need, (void *)0x10004) == QPE_ERR_ALIGN, "report align");
  qpe_problem q = p;
  q.U = (const void *)0x10008;
  EXPECT(qpe_check_run(&q, 1, QPE_FORM_MIXED, 0, ws, need, NULL) == QPE_ERR_ALIGN, "U align");
  q = p;
  q.psi = NULL;
  EXPECT(qpe_check_run(&q, 1, QPE_FORM_MIXED, 0, ws, need, NULL) == QPE_ERR_ARG, "psi NULL");
  q = p;
  q.prob = (double *)0x30004;
  EXPECT(qpe_check_run(&q, 1, QPE_FORM_MIXED, 0, ws, need, NULL) == QPE_ERR_ALIGN, "prob align");
}

static void batches(void) {
  uint64_t seed = 12345;
  const int counts[] = {2, 3, 17, 160, 161, 512, 4500};
  for (size_t ci = 0; ci < sizeof(counts) / sizeof(counts[0]); ++ci) {
    const int count = counts[ci];
    qpe_problem *ps = (qpe_problem *)malloc(sizeof(qpe_problem) * (size_t)count);
    for (int i = 0; i < count; ++i) {
      const int t = (int)(lcg(&seed) % 11);
      const int n = 1 + (int)(lcg(&seed) % (count > 600 ? 6 : 14));
      ps[i] = prob(n, t, (uintptr_t)i << 20);
    }
    for (int form = 0; form <= 1; ++form)
      for (unsigned flags = 0; flags < 32; ++flags) {
        if ((flags & QPE_MIX_TARGET) && (flags & QPE_NO_MIX_TARGET)) continue;
        size_t need = 0, one = 0, sum = 0;
        qpe_status st = qpe_workspace_size(ps, count, form, flags, &need);
        EXPECT(st == QPE_OK, "batch of %d form %d flags %u -> %d", count, form, flags, st);
        for (int i = 0; i < count; ++i) {
          EXPECT(qpe_workspace_size(ps + i, 1, form, flags, &one) == QPE_OK, "member %d", i);
          sum += one;
        }
        /* a batch lays every instance's region plus tables in front */
        EXPECT(need >= sum, "batch %d needs %zu < %zu", count, need, sum);
        EXPECT(qpe_check_run(ps, count, form, flags, (void *)0x100000, need, NULL) == QPE_OK, "batch check");
        EXPECT(qpe_check_run(ps, count, form, flags, (void *)0x100000, need - 1, NULL) == QPE_ERR_WORKSPACE,
               "batch short");
      }
    /* one bad member spoils the batch */
    ps[count / 2].n_mat = QPE_MAX_N_MAT + 1;
    size_t b = 0;
    EXPECT(qpe_workspace_size(ps, count, QPE_FORM_MIXED, 0, &b) == QPE_ERR_SIZE, "bad member");
    free(ps);
  }
}

static void stage_entries(void) {
  size_t b = 0;
  for (int t = -1; t <= QPE_MAX_N_MAT + 1; ++t) {
    qpe_status st = qpe_powers_workspace_size(t, &b);
    EXPECT((t >= 0 && t <= QPE_MAX_N_MAT) ? st == QPE_OK : st == QPE_ERR_SIZE, "powers ws t=%d", t);
  }
  EXPECT(qpe_powers_workspace_size(4, NULL) == QPE_ERR_ARG, "powers NULL");
  for (int n = 0; n <= 31; n += 5)
    for (int t = 0; t <= 16; t += 4)
      for (int form = 0; form <= 2; ++form) {
        qpe_status a = qpe_controlled_step_workspace_size(n, t, form, &b);
        qpe_status c = qpe_iqft_workspace_size(n, t, form, &b);
        const int ok = n >= 1 && n <= QPE_MAX_N_MEAS && t <= QPE_MAX_N_MAT && n + t <= QPE_MAX_TOTAL_QUBITS;
        if (!ok) {
          EXPECT(a == QPE_ERR_SIZE && c == QPE_ERR_SIZE, "stage sizes n=%d t=%d", n, t);
        } else if (form > 1) {
          EXPECT(a == QPE_ERR_ARG && c == QPE_ERR_ARG, "stage form %d", form);
        } else {
          EXPECT(a == QPE_OK && c == QPE_OK, "stage ok n=%d t=%d", n, t);
        }
      }
  EXPECT(qpe_estimate_workspace_size(0, &b) == QPE_ERR_ARG, "estimate 0");
  EXPECT(qpe_estimate_workspace_size(7, &b) == QPE_OK && b % 256 == 0 && b > 0, "estimate 7");
}

static void null_context(void) {
  qpe_problem p = prob(8, 3, 0);
  double al[2] = {1.0, 0.0};
  int chosen[QPE_KERNEL_COUNT];
  int v = 0, launches = 0;
  double ms = 0.0;
  EXPECT(qpe_run(NULL, &p, 1, 1, 0, (void *)0x100000, 1 << 20, NULL) == QPE_ERR_ARG, "run");
  EXPECT(qpe_run_static(NULL, &p, 1, 1, 0, NULL) == QPE_ERR_ARG, "run_static");
  EXPECT(qpe_run_state(NULL, &p, 1, 0, (void *)0x100000, 1 << 20, (void *)0x200000, NULL) == QPE_ERR_ARG, "state");
  EXPECT(qpe_powers(NULL, 3, (void *)0x1000, 2, 0, (void *)0x2000, (void *)0x100000, 1 << 20, NULL) == QPE_ERR_ARG,
         "powers");
  EXPECT(qpe_zgemm(NULL, 'N', 'N', 4, 4, 4, al, (void *)0x1000, 4, (void *)0x1000, 4, al, (void *)0x1000, 4,
                   (void *)0x1000, 4) == QPE_ERR_ARG, "zgemm");
  EXPECT(qpe_controlled_step(NULL, 8, 3, 1, 0, (void *)0x1000, (void *)0x2000, (void *)0x100000, 1 << 20) ==
             QPE_ERR_ARG, "ctrl step");
  EXPECT(qpe_iqft_probs(NULL, 8, 3, 1, (void *)0x1000, (double *)0x2000, (void *)0x100000, 1 << 20) == QPE_ERR_ARG,
         "iqft");
  EXPECT(qpe_estimate(NULL, &p, 1, (qpe_estimates *)0x1000, (void *)0x100000, 1 << 20) == QPE_ERR_ARG, "estimate");
  EXPECT(qpe_autotune(NULL, &p, 1, 0, (void *)0x100000, 1 << 20, 2, chosen, NULL) == QPE_ERR_ARG, "autotune");
  EXPECT(qpe_autotune_batch(NULL, &p, 2, 1, 0, (void *)0x100000, 1 << 20, 2, chosen, NULL) == QPE_ERR_ARG, "tune b");
  EXPECT(qpe_ctx_set_stream(NULL, NULL) == QPE_ERR_ARG, "set_stream");
  EXPECT(qpe_ctx_set_variant(NULL, 0, -1, 0) == QPE_ERR_ARG, "set_variant");
  EXPECT(qpe_ctx_get_variant(NULL, 0, 5, &v) == QPE_ERR_ARG, "get_variant");
  EXPECT(qpe_ctx_enable_timing(NULL, 4) == QPE_ERR_ARG, "enable_timing");
  EXPECT(qpe_ctx_set_timing_mask(NULL, 1) == QPE_ERR_ARG, "timing_mask");
  EXPECT(qpe_ctx_reset_timing(NULL) == QPE_ERR_ARG, "reset_timing");
  EXPECT(qpe_ctx_read_timing(NULL, 0, &launches, &ms) == QPE_ERR_ARG, "read_timing");
  EXPECT(qpe_ctx_destroy(NULL) == QPE_OK, "destroy NULL");
  EXPECT(qpe_ctx_create(NULL, 0, NULL) == QPE_ERR_ARG, "create NULL");
}

/* With a device, the host-side context state; without one, the error. */
static void context_host_state(void) {
  qpe_ctx *ctx = NULL;
  qpe_status st = qpe_ctx_create(&ctx, 0, NULL);
  if (st != QPE_OK) {
    EXPECT(st == QPE_ERR_NO_DEVICE && ctx == NULL, "create without a device -> %d", st);
    EXPECT(qpe_ctx_create(&ctx, -1, NULL) == QPE_ERR_NO_DEVICE, "bad device");
    return;
  }
  int v = -1;
  for (int c = 0; c < QPE_KERNEL_COUNT; ++c) {
    int nv = 0;
    qpe_kernel_variants(c, &nv);
    EXPECT(qpe_ctx_set_variant(ctx, c, -1, nv) == QPE_OK, "set last variant");
    EXPECT(qpe_ctx_set_variant(ctx, c, -1, nv + 1) == QPE_ERR_ARG, "set beyond");
    EXPECT(qpe_ctx_get_variant(ctx, c, 3, &v) == QPE_OK && v == nv, "get");
    EXPECT(qpe_ctx_set_variant(ctx, c, 99, 0) == QPE_ERR_SIZE, "bad n_mat");
    qpe_ctx_set_variant(ctx, c, -1, 0);
  }
  EXPECT(qpe_ctx_set_timing_mask(ctx, 1u << QPE_TIMER_COUNT) == QPE_ERR_ARG, "mask beyond");
  EXPECT(qpe_ctx_enable_timing(ctx, 0) == QPE_ERR_ARG, "pairs 0");
  qpe_problem big = prob(16, 10, 0);
  EXPECT(qpe_run_static(ctx, &big, 1, QPE_FORM_MIXED, 0, NULL) == QPE_ERR_WORKSPACE, "static too big");
  EXPECT(strstr(qpe_last_error(ctx), "static workspace holds") != NULL, "static message");
  EXPECT(qpe_ctx_destroy(ctx) == QPE_OK, "destroy");
}

int main(void) {
  status_and_misc();
  single_sizes();
  alignment_and_pointers();
  batches();
  stage_entries();
  null_context();
  context_host_state();
  if (failures) {
    fprintf(stderr, "%d of %d host checks failed\n", failures, checks);
    return 1;
  }
  printf("HOST CHECKS OK %d\n", checks);
  return 0;
}
