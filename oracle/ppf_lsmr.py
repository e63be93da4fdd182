"""Oracle (test infrastructure only; never on the product path): inversion of
the polyphase filterbank by LSMR, in plain numpy FP64.

Winchen et al., Sec. 3 ("Computing requirements"): to recover the signal at
5 ns resolution, the polyphase filter is inverted by solving the sparse
linear system H x = y for the filtered subband data y with the iterative
LSMR method (Fong & Saunders 2011, SIAM J. Sci. Comput. 33, 2950); about 25
iterations are reported to converge.

The operator.  H is the analysis filterbank of the station (prototype h of
L = P M taps), restricted to the recorded channels k[]:
    y_k[m] = sum_{l<L} h[l] exp(+2 pi i k l / M) x[m M + M - 1 - l]
for frames m = 0 .. F + P - 2 of a real series x of F frames (F M samples,
zero outside).  Indexing x so that frame m of y sees the frames m - P + 1
.. m of x makes the block frame-aligned: n_frames = F + P - 1 output frames
for F unknown frames.  With r = l mod M and t = l div M this is a
polyphase FIR per column r, followed by an M-point transform:
    v_m[r]  = sum_{t<P} h[t M + r] x[(m - t) M + M - 1 - r]
    y_k[m]  = sum_{r<M} v_m[r] exp(+2 pi i k r / M).
The real adjoint (x real, y complex with the real inner product Re <a, b>)
is H^T y = Re(H^H y):
    W_m[r]  = Re sum_k y_k[m] exp(-2 pi i k r / M)
    (H^T y)[j M + M - 1 - r] = sum_{t<P} h[t M + r] W_{j + t}[r].

LSMR from x_0 = 0 with no damping, in the notation of Fong & Saunders
(Algorithm 1: Golub-Kahan bidiagonalisation, rotations P_k and Pbar_k, the
vectors h_k and hbar_k).  With fewer recorded channels than M / 2 the system
is underdetermined, and LSMR from zero tends to the minimum-norm
least-squares solution.
"""
from __future__ import annotations

import numpy as np


def analysis(h: np.ndarray, M: int, k, x: np.ndarray) -> np.ndarray:
    """H x.  x: real [F M]; returns y: complex [len(k)][F + P - 1]."""
    h = np.asarray(h, dtype=np.float64)
    P = h.size // M
    x = np.asarray(x, dtype=np.float64)
    F = x.size // M
    assert x.size == F * M and F >= 1
    xr = x.reshape(F, M)[:, ::-1]            # xr[j][r] = x[j M + M - 1 - r]
    hp = h.reshape(P, M)
    v = np.zeros((F + P - 1, M))
    for t in range(P):                       # v_m[r] += h[t M + r] xr[m - t][r]
        v[t:t + F] += hp[t] * xr
    Y = np.fft.ifft(v, axis=1) * M           # sum_r v_m[r] exp(+2 pi i k r / M)
    return np.ascontiguousarray(Y[:, np.asarray(k)].T)


def adjoint(h: np.ndarray, M: int, k, y: np.ndarray) -> np.ndarray:
    """H^T y.  y: complex [len(k)][n_frames]; returns real [(n_frames - P + 1) M]."""
    h = np.asarray(h, dtype=np.float64)
    P = h.size // M
    y = np.asarray(y, dtype=np.complex128)
    n_frames = y.shape[1]
    F = n_frames - P + 1
    assert F >= 1
    S = np.zeros((n_frames, M), dtype=np.complex128)
    S[:, np.asarray(k)] = y.T
    W = np.fft.fft(S, axis=1).real           # Re sum_k y_k exp(-2 pi i k r / M)
    hp = h.reshape(P, M)
    xr = np.zeros((F, M))
    for t in range(P):                       # xr[j][r] += h[t M + r] W[j + t][r]
        xr += hp[t] * W[t:t + F]
    return np.ascontiguousarray(xr[:, ::-1]).reshape(-1)


def _norm(a) -> float:
    return float(np.sqrt(np.sum(np.abs(a) ** 2)))


def lsmr(A, At, b, n_iter: int):
    """LSMR (no damping) from x_0 = 0 for n_iter iterations, or until the
    bidiagonalisation ends (alpha or beta zero: x is then exact).

    A maps real vectors to arrays shaped like b; At is its real adjoint.
    Returns (x, anorm) with anorm[k] = |zetabar_{k+1}| = ||A^T r_k|| for
    k = 0 .. iterations done."""
    beta = _norm(b)
    x = None
    if beta == 0.0:
        v0 = At(np.zeros_like(b))
        return np.zeros_like(v0), [0.0]
    u = b / beta
    v = At(u)
    alpha = _norm(v)
    x = np.zeros_like(v)
    if alpha == 0.0:
        return x, [0.0]
    v = v / alpha
    # Initial state (Fong & Saunders, Algorithm 1, step 1).
    alphabar = alpha
    zetabar = alpha * beta
    rho = 1.0
    rhobar = 1.0
    cbar = 1.0
    sbar = 0.0
    hvec = v.copy()
    hbar = np.zeros_like(v)
    anorm = [abs(zetabar)]
    for _ in range(n_iter):
        # Bidiagonalisation: beta_{k+1} u_{k+1} = A v_k - alpha_k u_k,
        # alpha_{k+1} v_{k+1} = A^T u_{k+1} - beta_{k+1} v_k.
        u = A(v) - alpha * u
        beta = _norm(u)
        if beta > 0.0:
            u = u / beta
        v = At(u) - beta * v
        alpha_new = _norm(v)
        if alpha_new > 0.0:
            v = v / alpha_new
        # Rotation P_k (no damping, so alphahat_k = alphabar_k).
        rho_old = rho
        rho = float(np.hypot(alphabar, beta))
        c = alphabar / rho
        s = beta / rho
        theta_new = s * alpha_new
        alphabar = c * alpha_new
        # Rotation Pbar_k.
        rhobar_old = rhobar
        thetabar = sbar * rho
        t = cbar * rho
        rhobar = float(np.hypot(t, theta_new))
        cbar = t / rhobar
        sbar = theta_new / rhobar
        zeta = cbar * zetabar
        zetabar = -sbar * zetabar
        # Update hbar, x, h.
        hbar = hvec - (thetabar * rho / (rho_old * rhobar_old)) * hbar
        x = x + (zeta / (rho * rhobar)) * hbar
        hvec = v - (theta_new / rho) * hvec
        alpha = alpha_new
        anorm.append(abs(zetabar))
        if beta == 0.0 or alpha == 0.0:
            break
    return x, anorm


def invert(h: np.ndarray, M: int, k, y: np.ndarray, n_iter: int = 25):
    """PPF inversion of one series: LSMR on H x = y.  y: complex
    [len(k)][n_frames]; returns (x real [(n_frames - P + 1) M], anorm)."""
    return lsmr(lambda v: analysis(h, M, k, v),
                lambda u: adjoint(h, M, k, u), y, n_iter)
