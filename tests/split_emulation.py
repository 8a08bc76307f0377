"""CPU emulation of the mixed form's split products (test infrastructure).

A plain numpy model of the arithmetic the controlled products of the mixed
form use, to evaluate a splitting scheme before (and beside) the GPU kernels:

  * split-BF16 x6: each FP32 state component and each FP64 operator
    component as three BF16 pieces (round to nearest even of the running
    residual), the six piece products with index sum <= 2;
  * split-FP16 x3: the state scaled by sigma = 2^(14 - e) with
    ||psi|| 2^(-n/2) = m 2^e, m in [0.5, 1), and the operator by 2^14 (powers
    of two), two FP16 pieces each, the three products lh, hl, hh, the sum
    scaled back.

Piece products are exact in FP32 (at most 16 or 22 significant bits) and are
summed by FP32 matrix products (numpy's BLAS, a different order from the
matrix cores). The state between steps is complex64, the inverse QFT an FP32
FFT, the readout an FP64 sum, as in the mixed form. The powers are the exact
spectral ones (the GPU forms them in FP64 to ~1e-13). Nothing here is shared
with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft


def bf16_from_f32(x):
    """Round float32 values to BF16 (ties to even); returns float32."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def bf16_from_f64(x):
    """Round float64 values to BF16 (ties to even), once; returns float64."""
    b = np.asarray(x, np.float64).view(np.uint64)
    lsb = (b >> np.uint64(45)) & np.uint64(1)
    b = (b + np.uint64((1 << 44) - 1) + lsb) & ~np.uint64((1 << 45) - 1)
    return b.view(np.float64)


def state_pieces(a, scheme, sigma):
    a = np.asarray(a, np.float32)
    if scheme == "fp16x3":
        s = a * np.float32(sigma)
        h = s.astype(np.float16).astype(np.float32)
        return [h, (s - h).astype(np.float16).astype(np.float32)]
    h = bf16_from_f32(a)
    r = a - h
    m = bf16_from_f32(r)
    return [h, m, bf16_from_f32(r - m)]


def operator_pieces(w, scheme):
    w = np.asarray(w, np.float64)
    if scheme == "fp16x3":
        s = w * 2.0 ** 14
        h = s.astype(np.float16).astype(np.float64)  # numpy rounds float64 -> float16 once
        return [h.astype(np.float32), (s - h).astype(np.float16).astype(np.float32)]
    h = bf16_from_f64(w)
    r = w - h
    m = bf16_from_f64(r)
    return [p.astype(np.float32) for p in (h, m, bf16_from_f64(r - m))]


PAIRS = {"fp16x3": [(1, 0), (0, 1), (0, 0)], "bf16x6": [(2, 0), (1, 1), (0, 2), (1, 0), (0, 1), (0, 0)]}


def state_scale(psi, n):
    r = float(np.linalg.norm(psi)) * 2.0 ** (-n / 2.0)
    _, e = math.frexp(r)
    return 2.0 ** (14 - e)


def controlled_step(S, V, k, scheme, sigma):
    """Rows of S (complex64, N x d) with bit k set <- row V^T, emulated."""
    j = np.arange(S.shape[0])
    rows = j[((j >> k) & 1) == 1]
    A = S[rows]
    ar = state_pieces(A.real, scheme, sigma)
    ai = state_pieces(A.imag, scheme, sigma)
    W = V.T
    wr, wi = operator_pieces(W.real, scheme), operator_pieces(W.imag, scheme)
    re = np.zeros(A.shape, np.float32)
    im = np.zeros(A.shape, np.float32)
    for p, q in PAIRS[scheme]:
        re += ar[p] @ wr[q] - ai[p] @ wi[q]
        im += ar[p] @ wi[q] + ai[p] @ wr[q]
    f = np.float32(1.0 / (sigma * 2.0 ** 14)) if scheme == "fp16x3" else np.float32(1.0)
    S[rows] = (re * f + 1j * (im * f)).astype(np.complex64)


def rotation(d, rng):
    """M = D2 H D1 / sqrt(d): random signs D1, random unit phases D2."""
    t = d.bit_length() - 1
    H = np.array([[1.0]])
    for _ in range(t):
        H = np.kron(H, np.array([[1.0, 1.0], [1.0, -1.0]]))
    D1 = rng.choice([-1.0, 1.0], d)
    D2 = np.exp(2j * np.pi * rng.random(d))
    return (D2[:, None] * H * D1[None, :]) / math.sqrt(d)


def mixed_probs(Q, phis, psi, n, scheme, rot=None):
    """P(m) of the QPE circuit for U = Q diag(exp(2 pi i phi)) Q^H (Q unitary)
    and input psi, with the controlled products emulated in `scheme` and,
    if rot (a unitary d x d M) is given, the target register rotated first."""
    psi = np.asarray(psi, np.complex128)
    Q = np.asarray(Q, np.complex128)
    if rot is not None:
        Q, psi = rot @ Q, rot @ psi
    N = 1 << n
    S = np.empty((N, Q.shape[0]), np.complex64)
    S[:] = (psi / math.sqrt(N)).astype(np.complex64)[None, :]
    sigma = state_scale(psi, n)
    for k in range(n):
        lam = np.exp(2j * np.pi * np.mod(phis * float(1 << k), 1.0))
        controlled_step(S, (Q * lam[None, :]) @ Q.conj().T, k, scheme, sigma)
    A = scipy.fft.fft(S, axis=0, norm="ortho")
    return (A.real.astype(np.float64) ** 2 + A.imag.astype(np.float64) ** 2).sum(axis=1)
