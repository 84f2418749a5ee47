"""Spectral solve of the periodic MAC Stokes problem (oracle test pin).

With no elastic term the periodic staggered-grid operator of Sec. 2.2 is
diagonalised by the discrete Fourier transform: per wavenumber (kx, ky) the
unknowns (u^, v^, p^) satisfy a 3x3 system built from the stencil symbols
  Laplacian  lam = (2 cos tx - 2 + 2 cos ty - 2) / h^2,
  gradient   gx = (1 - e^{-i tx}) / h,  gy = (1 - e^{-i ty}) / h,
  divergence dx = (e^{i tx} - 1) / h,  dy = (e^{i ty} - 1) / h,
with t = 2 pi k / N.  This is an independent direct solver for
  c u - mu Lap u + G p = f,  -D u = q,
used to pin the multigrid-FGMRES path at K = 0 and to apply the steady
Stokes solution operator L_h^{-1} of Sec. 4.1.  Gauge: zero-mean pressure;
with c = 0 also zero-mean velocity (the mean of f must then vanish).
"""
from __future__ import annotations

import numpy as np


def solve(fu, fv, c, mu, q=None):
    N = fu.shape[0]
    h = 1.0 / N
    k = np.fft.fftfreq(N) * N
    tx = 2.0 * np.pi * k[None, :] / N
    ty = 2.0 * np.pi * k[:, None] / N
    lam = (2.0 * np.cos(tx) - 2.0 + 2.0 * np.cos(ty) - 2.0) / h**2
    gx = (1.0 - np.exp(-1j * tx)) / h * np.ones_like(ty)
    gy = (1.0 - np.exp(-1j * ty)) / h * np.ones_like(tx)
    dx = (np.exp(1j * tx) - 1.0) / h * np.ones_like(ty)
    dy = (np.exp(1j * ty) - 1.0) / h * np.ones_like(tx)
    a = c - mu * lam
    Fu = np.fft.fft2(fu)
    Fv = np.fft.fft2(fv)
    Q = np.zeros((N, N), complex) if q is None else np.fft.fft2(q)
    Am = np.zeros((N, N, 3, 3), complex)
    Am[..., 0, 0] = a
    Am[..., 1, 1] = a
    Am[..., 0, 2] = gx
    Am[..., 1, 2] = gy
    Am[..., 2, 0] = -dx
    Am[..., 2, 1] = -dy
    # the zero mode is singular (pressure gauge); replace it by a harmless
    # identity system and set it by hand below
    Am[0, 0] = np.eye(3)
    rhs = np.stack([Fu, Fv, Q], axis=-1)[..., None]
    S = np.linalg.solve(Am, rhs)[..., 0]
    U, V, P = S[..., 0].copy(), S[..., 1].copy(), S[..., 2].copy()
    U[0, 0] = Fu[0, 0] / a[0, 0] if a[0, 0] != 0 else 0.0
    V[0, 0] = Fv[0, 0] / a[0, 0] if a[0, 0] != 0 else 0.0
    P[0, 0] = 0.0
    return (np.real(np.fft.ifft2(U)), np.real(np.fft.ifft2(V)), np.real(np.fft.ifft2(P)))
