"""Periodic real-space grid, reciprocal vectors and spectral derivatives.

TEST INFRASTRUCTURE (oracle).  Plain numpy full complex FFTs.

Conventions (the paper evaluates the divergence term of Eq. vftGGA in
reciprocal space and inverse-transforms it, Sec. III B; Hartree and the
local pseudopotential are reciprocal-space forms, Eqs. E2 and E4A):
  * lattice rows a1, a2, a3; grid point r_j = sum_a (j_a/N_a) a_a;
    volume V = |det|, volume element dv = V/N.
  * reciprocal rows b_a with a_a . b_b = 2 pi delta_ab;
    G(m) = m1 b1 + m2 b2 + m3 b3 with signed integer frequencies m_a.
  * forward transform  c(G) = (1/N) sum_r a(r) exp(-i G.r)   (numpy fftn / N);
    inverse           a(r) = sum_G c(G) exp(i G.r)           (numpy ifftn * N).
  * Nyquist rule (a reading: the paper does not say): every G with some
    |m_a| = N_a/2 is dropped from all reciprocal-space operators (gradient,
    divergence, Hartree, pseudopotential, forces).  The kept set is closed
    under G -> -G, so every operator is real and symmetric (derivatives
    antisymmetric) and the potential is the exact gradient of the discrete
    energy.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, lattice, shape):
        self.lattice = np.asarray(lattice, dtype=np.float64).reshape(3, 3)
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.volume = float(abs(np.linalg.det(self.lattice)))
        self.dv = self.volume / self.N
        self.recip = 2.0 * np.pi * np.linalg.inv(self.lattice).T      # rows b_a
        m = [np.fft.fftfreq(n) * n for n in self.shape]
        M1, M2, M3 = np.meshgrid(*m, indexing="ij")
        self.m = (M1, M2, M3)
        self.G = np.stack([M1 * self.recip[0, c] + M2 * self.recip[1, c] + M3 * self.recip[2, c]
                           for c in range(3)])
        self.G2 = np.sum(self.G * self.G, axis=0)
        nyq = np.zeros(self.shape, dtype=bool)
        for Ma, n in zip((M1, M2, M3), self.shape):
            nyq |= np.abs(Ma) == n // 2 if n % 2 == 0 else False
        self.keep = ~nyq
        self.keep_nonzero = self.keep & (self.G2 > 0)

    def points(self):
        """Cartesian grid points, shape (3, N1, N2, N3)."""
        f = [np.arange(n) / n for n in self.shape]
        F1, F2, F3 = np.meshgrid(*f, indexing="ij")
        return np.stack([F1 * self.lattice[0, c] + F2 * self.lattice[1, c] + F3 * self.lattice[2, c]
                         for c in range(3)])

    def fft(self, a):
        return np.fft.fftn(a) / self.N

    def ifft(self, c):
        return np.fft.ifftn(c) * self.N

    def integrate(self, a) -> float:
        return float(np.sum(a) * self.dv)

    def gradient(self, a):
        """Spectral gradient of a real field: shape (3, ...)."""
        c = self.fft(a) * self.keep
        return np.stack([np.real(self.ifft(1j * self.G[k] * c)) for k in range(3)])

    def gradient_from_hat(self, c):
        c = c * self.keep
        return np.stack([np.real(self.ifft(1j * self.G[k] * c)) for k in range(3)])

    def divergence(self, w):
        """Spectral divergence of a real vector field w (3, ...)."""
        acc = np.zeros(self.shape, dtype=np.complex128)
        for k in range(3):
            acc += 1j * self.G[k] * self.fft(w[k])
        return np.real(self.ifft(acc * self.keep))
