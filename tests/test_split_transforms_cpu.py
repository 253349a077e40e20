"""The index algebra of the split plane passes, checked on the CPU against numpy's FFT.

The mixed-precision plane kernels on planes of 32, 64 and 128 points split each plane's work
over several blocks so that no block repeats another's transform: the inverse x2 transform by
decimation in time over i2 mod 4 (the fused gradient pass and the final pass), and the forward
x3 transform of packed real rows by decimation in frequency over the parity of k3 (the density
pass).  These tests restate those decompositions with numpy arrays and compare them with the
plain transforms, so that a sign, twiddle or index slip in the algebra the kernels follow
fails here, without a GPU.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("L", [32, 64, 128])
def test_inverse_four_way_decimation_in_time(L):
    """y[4m + q] = sum_{k<Q} Y_q[k] e^{+2 pi i k m/Q}, Y_q[k] = conj(w)^{kq} sum_s i^{sq} X[k + sQ]."""
    rng = np.random.default_rng(L)
    X = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    y_ref = np.fft.ifft(X) * L                     # unnormalised inverse, e^{+2 pi i k n/L}
    Q = L // 4
    w = np.exp(-2j * np.pi * np.arange(L) / L)     # the kernels' twiddle table
    y = np.empty(L, dtype=complex)
    k = np.arange(Q)
    for q in range(4):
        Y = sum(X[k + s * Q] * (1j) ** (s * q) for s in range(4)) * np.conj(w[(k * q) % L])
        y[q::4] = np.fft.ifft(Y) * Q               # Q-point unnormalised inverse
    assert np.allclose(y, y_ref, rtol=0, atol=1e-12 * np.abs(y_ref).max())


@pytest.mark.parametrize("L", [32, 64, 128])
def test_forward_parity_split_of_packed_real_rows(L):
    """Two real rows packed as z = a + i b: block r forms (z[m] + (-1)^r z[m + H]) w^{rm}, runs an
    H-point forward transform, and separates the two rows' half spectra at k3 = 2j + r from
    Z[k3] and conj Z[L - k3], whose index L - k3 = 2 j' + r, j' = (H - j - r) mod H, has the
    same parity."""
    rng = np.random.default_rng(100 + L)
    a, b = rng.standard_normal(L), rng.standard_normal(L)
    A_ref, B_ref = np.fft.fft(a), np.fft.fft(b)
    z = a + 1j * b
    H = L // 2
    m = np.arange(H)
    w = np.exp(-2j * np.pi * np.arange(L) / L)
    A = np.zeros(H, dtype=complex)
    B = np.zeros(H, dtype=complex)
    for r in range(2):
        Zr = np.fft.fft((z[m] + (-1) ** r * z[m + H]) * w[(r * m) % L])   # Z[2j + r], j < H
        for j in range(L // 4):
            jc = (H - j - r) % H
            Zk, Zc = Zr[j], np.conj(Zr[jc])
            k3 = 2 * j + r
            A[k3] = 0.5 * (Zk + Zc)
            B[k3] = (Zk - Zc) / 2j
    scale = max(np.abs(A_ref).max(), np.abs(B_ref).max())
    assert np.allclose(A, A_ref[:H], rtol=0, atol=1e-12 * scale)
    assert np.allclose(B, B_ref[:H], rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("L", [32, 64, 128])
def test_plane_blocks_of_one_plane_share_an_xcd(L):
    """Block b of the split passes takes plane i1 and part q; with n1 a multiple of 8 the parts
    of one plane are 8 block indices apart (the same XCD under round-robin dispatch over 8), and
    every (i1, q) is taken exactly once."""
    for n1, parts in [(L, 4), (L, 2), (12, 4), (12, 2)]:
        seen = set()
        for blk in range(parts * n1):
            if n1 % 8 == 0:
                i1 = (blk // (8 * parts)) * 8 + (blk % 8)
                q = (blk // 8) % parts
            else:
                i1, q = blk // parts, blk % parts
            seen.add((i1, q))
            if n1 % 8 == 0:
                first = (i1 // 8) * 8 * parts + (i1 % 8)
                assert (blk - first) % 8 == 0 and blk % 8 == first % 8
        assert seen == {(i, q) for i in range(n1) for q in range(parts)}
