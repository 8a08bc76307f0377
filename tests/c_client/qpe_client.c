/*
 * A plain C caller of the QPE C ABI (include/qpe.h), with no Python and no
 * torch: it allocates the device memory and the workspace itself, runs on a
 * stream of its own, and checks the result against the closed form of an
 * exactly representable eigenphase (paper section 2: an eigenvector input
 * whose phase is k / 2^n puts all probability on outcome m = k), in both
 * arithmetic forms, then the host-side error codes. Prints "ok" and exits 0
 * on success; prints the failed check and exits 1 otherwise.
 *
 * U = Q diag(exp(2 pi i phi_j)) Q with Q = I - 2 v v^T / (v^T v) (a real
 * Householder reflection: symmetric and orthogonal), phi_0 = k / 2^n and the
 * other phases irrational-looking; the input is Q e_0, U's eigenvector for
 * phi_0.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "qpe.h"

#define N_MEAS 10
#define N_MAT 6
#define K_PHASE 357

static int fail(const char *what, const char *detail) {
  printf("FAILED: %s %s\n", what, detail ? detail : "");
  return 1;
}

#define HIP_OK(x)                                              \
  do {                                                         \
    hipError_t e_ = (x);                                       \
    if (e_ != hipSuccess) return fail(#x, hipGetErrorString(e_)); \
  } while (0)

#define QPE_IS(x, want)                                                  \
  do {                                                                   \
    qpe_status s_ = (x);                                                 \
    if (s_ != (want)) return fail(#x, qpe_status_string((int)s_));      \
  } while (0)

int main(void) {
  const int n = N_MEAS, t = N_MAT, d = 1 << N_MAT, N = 1 << N_MEAS;
  const double two_pi = 6.283185307179586476925286766559;

  /* host operands (complex128 as interleaved re, im) */
  double *Q = malloc(sizeof(double) * d * d);
  double *U = malloc(sizeof(double) * 2 * d * d);
  double *psi = malloc(sizeof(double) * 2 * d);
  double *P = malloc(sizeof(double) * N);
  double *v = malloc(sizeof(double) * d);
  if (!Q || !U || !psi || !P || !v) return fail("malloc", NULL);
  double vv = 0.0;
  for (int i = 0; i < d; ++i) {
    v[i] = 1.0 + 0.37 * i - 0.011 * i * i;
    vv += v[i] * v[i];
  }
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) Q[r * d + c] = (r == c ? 1.0 : 0.0) - 2.0 * v[r] * v[c] / vv;
  /* U = Q D Q, D_jj = exp(2 pi i phi_j) */
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      double re = 0.0, im = 0.0;
      for (int j = 0; j < d; ++j) {
        const double phi = j == 0 ? (double)K_PHASE / N : fmod(0.1234567 + 0.7071067811865476 * j, 1.0);
        re += Q[r * d + j] * cos(two_pi * phi) * Q[j * d + c];
        im += Q[r * d + j] * sin(two_pi * phi) * Q[j * d + c];
      }
      U[2 * (r * d + c)] = re;
      U[2 * (r * d + c) + 1] = im;
    }
  for (int i = 0; i < d; ++i) {
    psi[2 * i] = Q[i * d + 0];
    psi[2 * i + 1] = 0.0;
  }

  hipStream_t stream;
  HIP_OK(hipStreamCreate(&stream));
  void *dU, *dpsi;
  double *dP;
  HIP_OK(hipMalloc(&dU, sizeof(double) * 2 * d * d));
  HIP_OK(hipMalloc(&dpsi, sizeof(double) * 2 * d));
  HIP_OK(hipMalloc((void **)&dP, sizeof(double) * N));
  HIP_OK(hipMemcpy(dU, U, sizeof(double) * 2 * d * d, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dpsi, psi, sizeof(double) * 2 * d, hipMemcpyHostToDevice));

  qpe_ctx *ctx = NULL;
  QPE_IS(qpe_ctx_create(&ctx, 0, stream), QPE_OK);
  qpe_problem prob = {n, t, dU, dpsi, dP};

  const int forms[2] = {QPE_FORM_MIXED, QPE_FORM_FP64};
  const double tol[2] = {1e-6, 1e-10};
  for (int f = 0; f < 2; ++f) {
    size_t bytes = 0;
    QPE_IS(qpe_workspace_size(&prob, 1, forms[f], 0, &bytes), QPE_OK);
    void *ws;
    HIP_OK(hipMalloc(&ws, bytes));
    QPE_IS(qpe_run(ctx, &prob, 1, forms[f], 0, ws, bytes, NULL), QPE_OK);
    HIP_OK(hipStreamSynchronize(stream));
    HIP_OK(hipMemcpy(P, dP, sizeof(double) * N, hipMemcpyDeviceToHost));
    double worst = 0.0;
    for (int m = 0; m < N; ++m) {
      const double e = fabs(P[m] - (m == K_PHASE ? 1.0 : 0.0));
      if (e > worst) worst = e;
    }
    printf("form %d: max |P - delta_k| = %.3e\n", forms[f], worst);
    if (!(worst <= tol[f])) return fail("closed form", forms[f] == QPE_FORM_MIXED ? "mixed" : "fp64");
    /* a workspace one byte short is refused before anything is enqueued */
    QPE_IS(qpe_run(ctx, &prob, 1, forms[f], 0, ws, bytes - 1, NULL), QPE_ERR_WORKSPACE);
    HIP_OK(hipFree(ws));
  }

  /* host-side checks */
  QPE_IS(qpe_run(NULL, &prob, 1, QPE_FORM_MIXED, 0, NULL, 0, NULL), QPE_ERR_ARG);
  qpe_problem big = {QPE_MAX_N_MEAS + 1, 0, dU, dpsi, dP};
  size_t b2 = 0;
  QPE_IS(qpe_workspace_size(&big, 1, QPE_FORM_MIXED, 0, &b2), QPE_ERR_SIZE);
  if (!qpe_status_string(QPE_ERR_HIP)) return fail("qpe_status_string", NULL);

  QPE_IS(qpe_ctx_destroy(ctx), QPE_OK);
  HIP_OK(hipFree(dU));
  HIP_OK(hipFree(dpsi));
  HIP_OK(hipFree(dP));
  HIP_OK(hipStreamDestroy(stream));
  free(Q);
  free(U);
  free(psi);
  free(P);
  free(v);
  printf("ok\n");
  return 0;
}
