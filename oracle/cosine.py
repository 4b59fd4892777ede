"""Cosine track: phase-correlation alignment and thresholded cosine (FP64).

Follows paper Sec. 3.2.1(1), Eqs. 3-5 (Fourier shift theorem, normalised
cross-power spectrum, inverse transform whose peak gives the translation) and
Sec. 2.2.1, Eq. 2 (cosine similarity against T_cos with a strict ">").

Readings fixed here (the paper is silent or garbled on these):

* Shifts are circular on the N x N grid (Eqs. 3-5 are exact only for cyclic
  shifts of a DFT grid).  The window of a clip with marker half-width w is
  [-w, w]^2 taken modulo N; when 2w+1 > N every residue appears once, named by
  its representative in [-N/2, N/2-1].
* Eq. 4 divides by |G F*|, undefined where a bin vanishes.  Each clip's
  spectrum is whitened on its own, W(k) = F(k)/|F(k)| if |F(k)| > EPS else 0
  (EPS = 1e-2, absolute, pixel units); wherever both bins are non-zero this
  equals Eq. 4's pairwise normalisation.
* Eq. 5 gives only "a delta"; the surface is divided by K, the number of
  bins where the cross-power spectrum is non-zero, so a self match and an
  exact cyclic shift peak at exactly 1.  This does not move the argmax.
* The shift s is the member's displacement relative to the fixed
  representative (Eq. 3 with g = member, f = representative; Sec. 3.1 step 3
  keeps the representative fixed); the member's center becomes its marker
  center plus s, and s ranges over the member's window.
* Near-ties in the peak: every shift within TAU = 1e-9 of the window maximum
  is a candidate; among them the larger pixel overlap c(s) wins, then the
  smaller |dy|+|dx|, then the lexicographically smaller (dy, dx).
* The DCT of Eq. 2 is read as the full orthonormal 2-D DCT-II.  By Parseval
  its cosine equals the cosine of the pixel vectors, so the score is computed
  from pixels: score = c / sqrt(n_mem * n_rep) with c the overlap count at s.
* Thresholds are exact rationals p/q (0.95 = 19/20); the bit is the integer
  test c^2 q^2 > p^2 n_mem n_rep.  An empty clip covers only itself.
"""
from __future__ import annotations

import math

import numpy as np

EPS = 1e-2
TAU = 1e-9


def window_axis(w: int, N: int) -> np.ndarray:
    """Shift values along one axis for half-window w on an N-grid (C0 rule)."""
    if 2 * w + 1 <= N:
        return np.arange(-w, w + 1, dtype=np.int64)
    return np.arange(-(N // 2), N // 2, dtype=np.int64)


def window(w: int, N: int):
    """All (dy, dx) of the member's window, as an int64 array [|W|, 2]."""
    ax = window_axis(w, N)
    dy, dx = np.meshgrid(ax, ax, indexing="ij")
    return np.stack([dy.ravel(), dx.ravel()], axis=1)


def spectrum(a: np.ndarray) -> np.ndarray:
    """F = unnormalised forward 2-D DFT, kernel exp(-2 pi i (u y + v x)/N)."""
    return np.fft.fft2(a.astype(np.float64))


def whiten(F: np.ndarray, eps: float = EPS) -> np.ndarray:
    """Per-bin unit phasor F/|F| where |F| > eps, zero elsewhere (Eq. 4)."""
    mag = np.abs(F)
    out = np.zeros_like(F)
    nz = mag > eps
    out[nz] = F[nz] / mag[nz]
    return out


def cross_power(W_mem: np.ndarray, W_rep: np.ndarray):
    """R = W_mem * conj(W_rep) (Eq. 4 with g = member, f = rep) and K = #nonzero."""
    R = W_mem * np.conj(W_rep)
    K = int(np.count_nonzero((W_mem != 0) & (W_rep != 0)))
    return R, K


def surface(W_mem: np.ndarray, W_rep: np.ndarray):
    """Phase-correlation surface r[dy mod N, dx mod N] (Eq. 5) and K.

    r(s) = (1/K) sum_k R(k) exp(+2 pi i k.s / N); real because R is
    Hermitian.  Uses the library inverse FFT: ifft2 includes 1/N^2.
    """
    R, K = cross_power(W_mem, W_rep)
    N = R.shape[0]
    if K == 0:
        return np.zeros((N, N)), 0
    r = np.fft.ifft2(R).real * (N * N / K)
    return r, K


def surface_at(W_mem, W_rep, shifts):
    """The same surface evaluated term by term at the given (dy, dx) shifts."""
    R, K = cross_power(W_mem, W_rep)
    N = R.shape[0]
    u = np.arange(N)[:, None]
    v = np.arange(N)[None, :]
    out = []
    for dy, dx in np.asarray(shifts).reshape(-1, 2):
        ph = np.exp(2j * np.pi * (u * int(dy) + v * int(dx)) / N)
        out.append((R * ph).sum().real / K if K else 0.0)
    return np.array(out)


def whitened_image(W: np.ndarray) -> np.ndarray:
    """img = N * w with w the inverse DFT of the whitened spectrum (Eq. 4).

    W is Hermitian (the raster is real and the whitening keeps |F| symmetric),
    so w is real; ifft2 includes 1/N^2.  sum img^2 = number of non-zero bins
    (Parseval), so the values are of order one.
    """
    N = W.shape[0]
    return np.fft.ifft2(W).real * N


def correlate_images(img_mem: np.ndarray, img_rep: np.ndarray, shifts) -> np.ndarray:
    """sum_x img_rep(x) img_mem((x + s) mod N) at each shift s = (dy, dx).

    By Parseval this equals K r(s) of Eq. 5 (the surface before division by
    K): the spatial form of the same correlation.
    """
    out = []
    for dy, dx in np.asarray(shifts).reshape(-1, 2):
        moved = np.roll(img_mem, (-int(dy), -int(dx)), axis=(0, 1))  # moved[x] = img_mem[x + s]
        out.append(float((img_rep * moved).sum()))
    return np.array(out)


def overlap(a_rep: np.ndarray, a_mem: np.ndarray, dy: int, dx: int) -> int:
    """c(s) = sum_x a_rep(x) a_mem((x + s) mod N), an integer."""
    shifted = np.roll(a_mem, shift=(-int(dy), -int(dx)), axis=(0, 1))
    return int(np.count_nonzero(a_rep & shifted))


def tie_key(c: int, dy: int, dx: int):
    """Order of preference among near-tied shifts (smaller key wins)."""
    return (-c, abs(dy) + abs(dx), dy, dx)


def bit(c: int, n_mem: int, n_rep: int, p: int, q: int) -> bool:
    """Eq. 2 with T = p/q: c / sqrt(n_mem n_rep) > p/q, as an exact integer test."""
    if n_mem == 0 or n_rep == 0:
        return False
    return c * c * q * q > p * p * n_mem * n_rep


def score(c: int, n_mem: int, n_rep: int) -> float:
    """Cosine of the two pixel vectors at the chosen shift, in FP64."""
    if n_mem == 0 or n_rep == 0:
        return 0.0
    return c / math.sqrt(float(n_mem) * float(n_rep))


def align(a_mem, a_rep, W_mem, W_rep, w_mem: int, p: int, q: int, with_surface=False):
    """Align member to the fixed representative and score it (Eqs. 2-5).

    Returns dict(s=(dy, dx), c, score, bit, r1, K, ties).  For an empty clip
    the surface is undefined: s = (0, 0), c = 0, bit = False.
    """
    N = a_mem.shape[0]
    n_mem = int(np.count_nonzero(a_mem))
    n_rep = int(np.count_nonzero(a_rep))
    if n_mem == 0 or n_rep == 0:
        return dict(s=(0, 0), c=0, score=0.0, bit=False, r1=0.0, K=0, ties=0)
    r, K = surface(W_mem, W_rep)
    shifts = window(w_mem, N)
    vals = r[shifts[:, 0] % N, shifts[:, 1] % N]
    r1 = float(vals.max())
    cand = shifts[vals >= r1 - TAU]
    best = None
    for dy, dx in cand:
        c = overlap(a_rep, a_mem, dy, dx)
        key = tie_key(c, int(dy), int(dx))
        if best is None or key < best[0]:
            best = (key, int(dy), int(dx), c)
    _, dy, dx, c = best
    out = dict(s=(dy, dx), c=c, score=score(c, n_mem, n_rep),
               bit=bit(c, n_mem, n_rep, p, q), r1=r1, K=K, ties=int(cand.shape[0]))
    if with_surface:
        out["surface"] = r
        out["window_values"] = vals
    return out
