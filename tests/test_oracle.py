"""Pins for the CPU oracle (no GPU).

The oracle is checked against what the paper and mathematics fix, never
against itself:
* the factors of eq. (6) / eq. (9) built densely from their Kronecker
  definitions multiply out to E_2N of eq. (5);
* the printed N = 8 worked example of Section III (golden fixture);
* closed forms (delta, constant, single tones), invariants (Parseval,
  linearity, shift, conjugate symmetry, adjoint dot-product, round trip);
* a textbook library routine (numpy.fft, FP64) and pure-Python brute force
  of eq. (1) at N <= 16;
* mutation checks: plausible mistakes planted in a copy of the algorithm in
  this file are each caught by one of the pins above.
"""
import cmath
import math
import os

import numpy as np
import pytest

import oracle
from oracle import factors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "n8_worked_example.txt")
R = math.sqrt(0.5)  # correctly rounded 1/sqrt(2)


def rng_planes(n, batch, seed, dtype=np.float64):
    g = np.random.default_rng(seed)
    return (g.standard_normal((batch, n)).astype(dtype),
            g.standard_normal((batch, n)).astype(dtype))


def npfft(xr, xi):
    y = np.fft.fft(np.asarray(xr, np.float64) + 1j * np.asarray(xi, np.float64), axis=-1)
    return y.real, y.imag


# ---------------------------------------------------------------- golden N=8
def _parse_golden():
    items = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = [s.strip() for s in line.split("=", 1)]
            items[k] = v.split()
    return items


def _golden_matrix(items, key, omega33):
    """Build the printed matrix ``key``; ``omega33`` names the omega^(3,3) used."""
    kind, args = items[key][0], items[key][1:]

    def atom(t):
        if t.startswith("I"):
            return np.eye(int(t[1:]))
        if t == "H2":
            return np.array([[1.0, 1.0], [1.0, -1.0]])
        if t == "omega_3_3":
            return _golden_matrix(items, omega33, omega33)
        return _golden_matrix(items, t, omega33)

    def direct_sum(blocks):
        n = sum(b.shape[0] for b in blocks)
        d = np.zeros((n, n))
        o = 0
        for b in blocks:
            d[o:o + b.shape[0], o:o + b.shape[0]] = b
            o += b.shape[0]
        return d

    if kind == "perm":
        p = np.zeros((len(args), len(args)))
        for r, c in enumerate(args):
            p[r, int(c)] = 1.0
        return p
    if kind == "block":
        vals = [{"r": R, "-r": -R}[a] if a in ("r", "-r") else float(a) for a in args]
        return np.array(vals).reshape(2, 2)
    if kind == "diag":
        return direct_sum([atom(t) for t in args])
    if kind == "kron":
        acc = np.eye(1)
        for j, t in enumerate(args):
            if t == "diag":
                return np.kron(acc, direct_sum([atom(u) for u in args[j + 1:]]))
            acc = np.kron(acc, atom(t))
        return acc
    raise ValueError(kind)


def test_golden_n8_permutation_matches_bit_reversal():
    items = _parse_golden()
    S8 = _golden_matrix(items, "S8", "omega_3_3_formula")
    assert np.array_equal(S8, factors.bitrev_matrix(3))


@pytest.mark.parametrize("key,i,q", [("omega_1_0", 1, 0), ("omega_2_0", 2, 0), ("omega_2_1", 2, 1),
                                     ("omega_3_0", 3, 0), ("omega_3_1", 3, 1), ("omega_3_2", 3, 2),
                                     ("omega_3_3_formula", 3, 3)])
def test_golden_n8_twiddle_blocks(key, i, q):
    items = _parse_golden()
    printed = _golden_matrix(items, key, "omega_3_3_formula")
    assert np.allclose(factors.omega_block(i, q), printed, atol=1e-15, rtol=0)


def test_golden_n8_printed_omega33_is_a_misprint():
    # The printed omega^(3,3) equals omega^(3,1); with it the N = 8 product is
    # not the DFT, with the formula's value it is.
    items = _parse_golden()
    printed = _golden_matrix(items, "omega_3_3_printed", "omega_3_3_printed")
    formula = _golden_matrix(items, "omega_3_3_formula", "omega_3_3_formula")
    assert not np.allclose(printed, formula)
    E = factors.E2N_interleaved(8)
    for key33, ok in (("omega_3_3_formula", True), ("omega_3_3_printed", False)):
        S = np.kron(_golden_matrix(items, "S8", key33), np.eye(2))
        P = S
        for i in (1, 2, 3):
            D = _golden_matrix(items, "D%d_16" % i, key33)
            W = _golden_matrix(items, "W%d_16" % i, key33)
            P = W @ (D @ P)
        assert np.allclose(P, E, atol=1e-13) == ok


@pytest.mark.parametrize("i", [1, 2, 3])
def test_golden_n8_factors_match_kronecker_definitions(i):
    items = _parse_golden()
    assert np.allclose(_golden_matrix(items, "W%d_16" % i, "omega_3_3_formula"), factors.W_factor(3, i))
    assert np.allclose(_golden_matrix(items, "D%d_16" % i, "omega_3_3_formula"), factors.D_factor(3, i),
                       atol=1e-15)


# ------------------------------------------------- dense factor products
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_dense_dit_product_equals_E2N(m):
    n = 1 << m
    assert np.allclose(factors.dit_product(m), factors.E2N_interleaved(n), atol=1e-12, rtol=0)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_dense_dif_product_equals_E2N(m):
    n = 1 << m
    assert np.allclose(factors.dif_product(m), factors.E2N_interleaved(n), atol=1e-12, rtol=0)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_leading_identity_order_reading(m):
    # With the printed leading identity I_(2^(m-1)) the factor for i >= 2 is
    # not 2N x 2N; with I_(2^(m-i)) it is.
    n2 = 2 << m
    for i in range(1, m + 1):
        printed = np.kron(np.kron(np.eye(1 << (m - 1)), factors.H2()), np.eye(1 << i))
        assert (printed.shape[0] == n2) == (i == 1)
        assert factors.W_factor(m, i).shape == (n2, n2)


@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_planar_form_of_factorisation(m):
    # Q^T (eq. 6 product) Q is eq. (5) on [xr; xi].
    n = 1 << m
    Q = factors.perfect_shuffle(n)
    assert np.allclose(Q.T @ factors.dit_product(m) @ Q, factors.E2N_planar(n), atol=1e-12)


@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_fast_oracle_applies_the_dense_factors(m):
    # O2 applied to each unit vector reproduces the dense product column by column.
    n = 1 << m
    eye = np.eye(2 * n)
    xr, xi = eye[:, :n], eye[:, n:]
    yr, yi = oracle.split_fft(xr, xi)
    Q = factors.perfect_shuffle(n)
    dense = Q.T @ factors.dit_product(m) @ Q
    assert np.allclose(np.hstack([yr, yi]).T, dense, atol=1e-12)


# ------------------------------------------------- twiddle blocks
@pytest.mark.parametrize("m", [1, 4, 10, 16])
def test_twiddle_table_against_libm(m):
    c, s = oracle.twiddle_table_f64(m)
    for i in range(1, m + 1):
        half = 1 << (i - 1)
        q = np.arange(half)
        t = 2 * np.pi * q / (1 << i)
        assert np.allclose(c[half:2 * half], np.cos(t), atol=4e-16, rtol=0)
        assert np.allclose(s[half:2 * half], np.sin(t), atol=4e-16, rtol=0)


def test_twiddle_exact_values():
    for i in range(0, 17):
        d = 1 << i
        for q in sorted({0, d // 4, d // 2, 3 * d // 4, d // 8, 3 * d // 8}):
            if q >= d or (4 * q) % d and (8 * q) % d:
                continue
            c, s = oracle.omega(q, i)
            t = 2 * math.pi * q / d
            if (4 * q) % d == 0:  # multiple of pi/2: exactly 0 or +-1
                assert (c, s) == (round(math.cos(t)) + 0.0, round(math.sin(t)) + 0.0)
            else:  # odd multiple of pi/4: |c| == |s|
                assert abs(c) == abs(s) == R
            assert math.copysign(1.0, c) > 0 or c != 0
            assert math.copysign(1.0, s) > 0 or s != 0


@pytest.mark.parametrize("m", [4, 10, 16])
def test_twiddle_f32_is_rounded_f64(m):
    c32, s32 = oracle.twiddle_table_f32(m)
    c64, s64 = oracle.twiddle_table_f64(m)
    assert np.array_equal(c32, c64.astype(np.float32))
    assert np.array_equal(s32, s64.astype(np.float32))
    assert not np.any(np.signbit(c32) & (c32 == 0))
    assert not np.any(np.signbit(s32) & (s32 == 0))


# ------------------------------------------------- O1: eq. (5) direct
@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64, 256, 1024])
def test_direct_matches_numpy_fft(n):
    xr, xi = rng_planes(n, 3, n)
    yr, yi = oracle.dft_direct(xr, xi)
    rr, ri = npfft(xr, xi)
    scale = np.sqrt(n) * 10
    assert np.max(np.abs(yr - rr)) < 1e-13 * scale * n
    assert np.max(np.abs(yi - ri)) < 1e-13 * scale * n


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_direct_brute_force_eq1(n):
    # Pure-Python complex arithmetic of eq. (1).
    xr, xi = rng_planes(n, 2, 100 + n)
    yr, yi = oracle.dft_direct(xr, xi)
    for b in range(2):
        x = [complex(xr[b, j], xi[b, j]) for j in range(n)]
        for k in range(n):
            yk = sum(x[j] * cmath.exp(-2j * math.pi * j * k / n) for j in range(n))
            assert abs(yk - complex(yr[b, k], yi[b, k])) < 1e-13 * n


def test_direct_bins_match_full_rows():
    n = 512
    xr, xi = rng_planes(n, 1, 7)
    yr, yi = oracle.dft_direct(xr, xi)
    ks = np.array([0, 1, 5, 255, 256, 511])
    br, bi = oracle.dft_direct_bins(xr[0], xi[0], ks)
    assert np.allclose(br, yr[0, ks], rtol=0, atol=1e-12)
    assert np.allclose(bi, yi[0, ks], rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 8, 64, 512])
def test_adjoint_direct_is_n_times_inverse(n):
    gr, gi = rng_planes(n, 2, 300 + n)
    ar, ai = oracle.adjoint_direct(gr, gi)
    y = n * np.fft.ifft(gr + 1j * gi, axis=-1)
    assert np.allclose(ar, y.real, atol=1e-10) and np.allclose(ai, y.imag, atol=1e-10)


# ------------------------------------------------- O2: eq. (6) in FP64
ALL_M = list(range(0, 17))


@pytest.mark.parametrize("m", ALL_M)
def test_split_fft_matches_numpy(m):
    n = 1 << m
    batch = max(1, min(8, (1 << 16) // n))
    xr, xi = rng_planes(n, batch, m)
    yr, yi = oracle.split_fft(xr, xi)
    rr, ri = npfft(xr, xi)
    err = oracle.rel_l2_per_row(yr, yi, rr, ri)
    assert err.max() < 1e-14 * max(m, 1)


@pytest.mark.parametrize("m", range(0, 11))
def test_split_fft_matches_direct(m):
    n = 1 << m
    xr, xi = rng_planes(n, 4, 50 + m)
    yr, yi = oracle.split_fft(xr, xi)
    rr, ri = oracle.dft_direct(xr, xi)
    assert oracle.rel_l2_per_row(yr, yi, rr, ri).max() < 1e-13


@pytest.mark.parametrize("m", range(0, 11))
def test_dif_matches_direct(m):
    n = 1 << m
    xr, xi = rng_planes(n, 4, 70 + m)
    yr, yi = oracle.split_fft_dif(xr, xi)
    rr, ri = oracle.dft_direct(xr, xi)
    assert oracle.rel_l2_per_row(yr, yi, rr, ri).max() < 1e-13


@pytest.mark.parametrize("m", [0, 1, 2, 4, 10, 16])
def test_closed_forms(m):
    n = 1 << m
    delta = np.zeros((1, n))
    delta[0, 0] = 1.0
    ones = np.ones((1, n))
    zeros = np.zeros((1, n))
    for fn in (oracle.split_fft, oracle.split_fft_dif):
        yr, yi = fn(delta, zeros)
        assert np.array_equal(yr, ones) and np.all(yi == 0)
        yr, yi = fn(ones, zeros)
        assert np.array_equal(yr, n * delta) and np.all(yi == 0)


@pytest.mark.parametrize("m", [2, 3, 6, 10, 13])
def test_single_tone_pins_sign(m):
    # x_n = exp(+j 2 pi k0 n / N) must give N at bin k0 (a sign error puts it at N - k0).
    n = 1 << m
    k0 = max(1, n // 3)
    t = 2 * np.pi * ((k0 * np.arange(n)) % n) / n
    yr, yi = oracle.split_fft(np.cos(t)[None], np.sin(t)[None])
    expect = np.zeros(n)
    expect[k0] = n
    assert np.allclose(yr[0], expect, atol=1e-9 * n) and np.allclose(yi[0], 0, atol=1e-9 * n)


@pytest.mark.parametrize("m", [3, 8])
def test_shifted_delta_and_real_cosine(m):
    n = 1 << m
    n0 = 3
    x = np.zeros((1, n))
    x[0, n0] = 1.0
    yr, yi = oracle.split_fft(x, np.zeros_like(x))
    k = np.arange(n)
    assert np.allclose(yr[0], np.cos(2 * np.pi * k * n0 / n), atol=1e-13)
    assert np.allclose(yi[0], -np.sin(2 * np.pi * k * n0 / n), atol=1e-13)
    k0 = 2
    c = np.cos(2 * np.pi * k0 * k / n)[None]
    yr, yi = oracle.split_fft(c, np.zeros_like(c))
    assert abs(yr[0, k0] - n / 2) < 1e-10 and abs(yr[0, n - k0] - n / 2) < 1e-10


@pytest.mark.parametrize("m", [4, 9])
def test_invariants(m):
    n = 1 << m
    xr, xi = rng_planes(n, 3, 11 + m)
    ur, ui = rng_planes(n, 3, 12 + m)
    yr, yi = oracle.split_fft(xr, xi)
    # Parseval
    assert np.allclose((yr ** 2 + yi ** 2).sum(-1), n * (xr ** 2 + xi ** 2).sum(-1), rtol=1e-12)
    # linearity
    a, b = 0.75, -1.5
    lr, li = oracle.split_fft(a * xr + b * ur, a * xi + b * ui)
    vr, vi = oracle.split_fft(ur, ui)
    assert np.allclose(lr, a * yr + b * vr, atol=1e-11) and np.allclose(li, a * yi + b * vi, atol=1e-11)
    # circular shift: x_(n - s) <-> y_k e^{-j 2 pi k s / N}
    s = 5
    sr, si = oracle.split_fft(np.roll(xr, s, axis=-1), np.roll(xi, s, axis=-1))
    ph = np.exp(-2j * np.pi * np.arange(n) * s / n)
    z = (yr + 1j * yi) * ph
    assert np.allclose(sr, z.real, atol=1e-10) and np.allclose(si, z.imag, atol=1e-10)
    # conjugate symmetry of a real input
    cr, ci = oracle.split_fft(xr, np.zeros_like(xr))
    idx = (-np.arange(n)) % n
    assert np.allclose(cr, cr[:, idx], atol=1e-11) and np.allclose(ci, -ci[:, idx], atol=1e-11)
    # adjoint: dot-product test and round trip
    gr, gi = oracle.adjoint_direct(ur, ui)
    lhs = (ur * yr + ui * yi).sum(-1)
    rhs = (gr * xr + gi * xi).sum(-1)
    assert np.allclose(lhs, rhs, rtol=1e-11)
    rr, ri = oracle.adjoint_direct(yr, yi)
    assert np.allclose(rr, n * xr, atol=1e-10) and np.allclose(ri, n * xi, atol=1e-10)


# ------------------------------------------------- O2f: FP32 mirror
@pytest.mark.parametrize("m", [4, 10, 16])
def test_mirror_closed_forms_bit_exact(m):
    n = 1 << m
    delta = np.zeros((1, n), np.float32)
    delta[0, 0] = 1
    zeros = np.zeros((1, n), np.float32)
    ones = np.ones((1, n), np.float32)
    yr, yi = oracle.split_fft_f32(delta, zeros)
    assert np.array_equal(yr, ones) and np.all(yi == 0)
    yr, yi = oracle.split_fft_f32(ones, zeros)
    assert np.array_equal(yr, n * delta) and np.all(yi == 0)


@pytest.mark.parametrize("m", ALL_M)
def test_mirror_within_fp32_tolerance(m):
    n = 1 << m
    batch = max(1, min(16, (1 << 17) // n))
    xr, xi = rng_planes(n, batch, 200 + m, np.float32)
    yr, yi = oracle.split_fft_f32(xr, xi)
    rr, ri = oracle.split_fft(xr.astype(np.float64), xi.astype(np.float64))
    tol = 2e-7 * m + 1e-7
    assert oracle.rel_l2_per_row(yr, yi, rr, ri).max() <= tol


@pytest.mark.parametrize("m", [0, 1, 3, 6, 12])
def test_mirror_dif_within_fp32_tolerance(m):
    n = 1 << m
    xr, xi = rng_planes(n, 4, 400 + m, np.float32)
    yr, yi = oracle.split_fft_dif_f32(xr, xi)
    rr, ri = oracle.split_fft(xr.astype(np.float64), xi.astype(np.float64))
    assert oracle.rel_l2_per_row(yr, yi, rr, ri).max() <= 2e-7 * m + 1e-7


@pytest.mark.parametrize("m", [1, 6, 12])
def test_mirror_adjoint_matches_direct_adjoint(m):
    n = 1 << m
    gr, gi = rng_planes(n, 4, 500 + m, np.float32)
    ar, ai = oracle.split_adjoint_f32(gr, gi)
    rr, ri = oracle.adjoint_direct(gr.astype(np.float64), gi.astype(np.float64))
    assert oracle.rel_l2_per_row(ar, ai, rr, ri).max() <= 2e-7 * m + 1e-7


def test_mirror_is_deterministic_across_threads():
    xr, xi = rng_planes(256, 64, 9, np.float32)
    a = oracle.split_fft_f32(xr, xi, nthreads=1)
    b = oracle.split_fft_f32(xr, xi, nthreads=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------- mutation checks
def _dit_numpy(xr, xi, mutation=None):
    """A plain numpy copy of the eq. (6) stages, with optional planted mistakes,
    used only to show that the pins above catch such mistakes."""
    n = xr.shape[-1]
    m = n.bit_length() - 1
    idx = np.array([oracle.bit_reverse(k, m) for k in range(n)])
    if mutation == "no_bitrev":
        idx = np.arange(n)
    yr, yi = xr[..., idx].copy(), xi[..., idx].copy()
    for i in range(1, m + 1):
        Rh = 1 << (i - 1)
        for base in range(0, n, 2 * Rh):
            for q in range(Rh):
                lo, up = base + q, base + Rh + q
                qq = q
                if mutation == "wrong_q" and i == m:
                    qq = (q + 1) % Rh
                t = 2 * np.pi * qq / (1 << i)
                c, s = np.cos(t), np.sin(t)
                if mutation == "sin_sign":
                    s = -s
                if mutation == "transposed_omega":
                    vr = c * yr[..., up] - s * yi[..., up]
                    vi = s * yr[..., up] + c * yi[..., up]
                elif mutation == "dropped_twiddle" and i == m:
                    vr, vi = yr[..., up].copy(), yi[..., up].copy()
                else:
                    vr = c * yr[..., up] + s * yi[..., up]
                    vi = -s * yr[..., up] + c * yi[..., up]
                ur, ui = yr[..., lo].copy(), yi[..., lo].copy()
                if mutation == "dropped_imag_term":
                    vi = c * yi[..., up]
                yr[..., lo], yi[..., lo] = ur + vr, ui + vi
                yr[..., up], yi[..., up] = ur - vr, ui - vi
    return yr, yi


@pytest.mark.parametrize("mutation", ["no_bitrev", "wrong_q", "sin_sign", "transposed_omega",
                                      "dropped_twiddle", "dropped_imag_term"])
def test_pins_catch_planted_mistakes(mutation):
    n = 16
    xr, xi = rng_planes(n, 2, 1)
    good = _dit_numpy(xr, xi)
    rr, ri = npfft(xr, xi)
    assert oracle.rel_l2_per_row(*good, rr, ri).max() < 1e-14
    bad = _dit_numpy(xr, xi, mutation)
    caught = oracle.rel_l2_per_row(*bad, rr, ri).max() > 1e-6
    # single tone pins the sign convention even where random data might not
    k0 = 3
    t = 2 * np.pi * k0 * np.arange(n) / n
    tr, ti = _dit_numpy(np.cos(t)[None], np.sin(t)[None], mutation)
    caught = caught or abs(tr[0, k0] - n) > 1e-9
    assert caught
