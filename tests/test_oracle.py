"""Pins of the CPU FP64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a library routine
(numpy.convolve, numpy.fft, scipy.signal), exact integer arithmetic, a closed
form of eq. (5) (section 2.3), the orthogonality relation of section 2.1, or
the structure of explicit dealiasing (section 3.1).
"""
import numpy as np
import pytest
import scipy.signal

import oracle
import synth


def _gauss_int(L, C=None, seed=0, bound=8):
    shape = (L,) if C is None else (L, C)
    return (synth.gaussian_integers(shape, bound, 90, seed, 0),
            synth.gaussian_integers(shape, bound, 90, seed, 1))


def _exact_int_conv(f, g, M):
    """Brute-force eq. (5) in Python integers (exact)."""
    fr = [(int(z.real), int(z.imag)) for z in f]
    gr = [(int(z.real), int(z.imag)) for z in g]
    L = len(fr)
    out = []
    for k in range(M):
        re = im = 0
        for j in range(max(0, k - L + 1), min(k, L - 1) + 1):
            a, b = fr[j]
            c, d = gr[k - j]
            re += a * c - b * d
            im += a * d + b * c
        out.append(complex(re, im))
    return np.array(out, np.complex128)


@pytest.mark.parametrize("L", [1, 2, 3, 5, 6, 17, 64, 100, 257, 1024])
def test_direct_matches_numpy_convolve(L):
    f, g = synth.pair(L, 91, L)
    M = 2 * L - 1
    ref = np.convolve(f, g)  # library routine, full mode: length 2L-1
    assert oracle.rel_l2(oracle.direct_1d(f, g, M), ref) < 1e-14


@pytest.mark.parametrize("L", [1, 2, 3, 6, 31, 100, 243, 1000, 2187])
def test_padded_matches_numpy_convolve(L):
    f, g = synth.pair(L, 92, L)
    ref = np.convolve(f, g)
    assert oracle.rel_l2(oracle.padded_1d(f, g, 2 * L - 1), ref) < 1e-14


@pytest.mark.parametrize("L,M", [(6, 11), (6, 12), (6, 20), (100, 250), (1, 5)])
def test_output_tail_beyond_2L_minus_1_is_exactly_zero(L, M):
    f, g = synth.pair(L, 93, L)
    for h in (oracle.direct_1d(f, g, M), oracle.padded_1d(f, g, M)):
        assert np.all(h[2 * L - 1:] == 0)
        assert oracle.rel_l2(h[:2 * L - 1], np.convolve(f, g)) < 1e-14


@pytest.mark.parametrize("L", [6, 37, 300])
def test_gaussian_integers_exact(L):
    """Integer inputs: eq. (5) by Python integer arithmetic is exact."""
    f, g = _gauss_int(L, seed=L)
    M = 2 * L - 1
    exact = _exact_int_conv(f, g, M)
    assert np.array_equal(oracle.direct_1d(f, g, M), exact)  # FP64 sums of small integers are exact
    assert np.array_equal(np.round(oracle.padded_1d(f, g, M)), exact)


def test_gaussian_integers_exact_large():
    L = 4096
    f, g = _gauss_int(L, seed=1)
    d = oracle.direct_1d(f, g, 2 * L - 1)
    assert np.array_equal(d, np.round(d))  # integer-valued, no rounding in the direct sum
    assert np.array_equal(np.round(oracle.padded_1d(f, g, 2 * L - 1)), d)


def test_delta_pairs_hit_every_index():
    """delta_a * delta_b = delta_{a+b} for all a, b < L."""
    L = 12
    M = 2 * L - 1
    for a in range(L):
        for b in range(L):
            f = np.zeros(L, complex)
            g = np.zeros(L, complex)
            f[a] = 1.0
            g[b] = 1.0
            want = np.zeros(M, complex)
            want[a + b] = 1.0
            assert np.array_equal(oracle.direct_1d(f, g, M), want)
            assert np.max(np.abs(oracle.padded_1d(f, g, M) - want)) < 1e-15


def test_ones_give_triangle():
    L = 50
    f = np.ones(L, complex)
    k = np.arange(2 * L - 1)
    tri = np.minimum(k + 1, 2 * L - 1 - k).astype(complex)
    assert np.array_equal(oracle.direct_1d(f, f, 2 * L - 1), tri)
    assert np.max(np.abs(oracle.padded_1d(f, f, 2 * L - 1) - tri)) < 1e-12


def test_geometric_closed_form():
    """f_j = z^j, g_j = w^j: h_k = w^k sum_{j=lo}^{hi} (z/w)^j, a finite geometric series."""
    L = 40
    z, w = 0.97 * np.exp(0.3j), 1.01 * np.exp(-0.7j)
    j = np.arange(L)
    f, g = z ** j, w ** j
    M = 2 * L - 1
    k = np.arange(M)
    lo = np.maximum(0, k - L + 1)
    hi = np.minimum(k, L - 1)
    ratio = z / w
    want = w ** k * (ratio ** lo - ratio ** (hi + 1)) / (1 - ratio)
    assert oracle.rel_l2(oracle.direct_1d(f, g, M), want) < 1e-13
    assert oracle.rel_l2(oracle.padded_1d(f, g, M), want) < 1e-13


def test_copies_are_independent_columns():
    L, C = 33, 5
    f, g = synth.pair((L, C), 94, 0)
    h = oracle.direct_1d(f, g, 2 * L - 1)
    hp = oracle.padded_1d(f, g, 2 * L - 1)
    for c in range(C):
        ref = np.convolve(f[:, c], g[:, c])
        assert oracle.rel_l2(h[:, c], ref) < 1e-14
        assert oracle.rel_l2(hp[:, c], ref) < 1e-14


def test_sampled_equals_full():
    L = 500
    f, g = synth.pair(L, 95, 0)
    ks = np.array([0, 1, 7, 250, 499, 500, 998, 999, 1200])
    full = oracle.direct_1d(f, g, 1300)
    assert np.array_equal(oracle.direct_1d_sampled(f, g, ks), full[ks])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 12, 30, 49, 64, 97, 210, 1000, 2048])
def test_dft_matches_numpy_fft(n):
    x = synth.uniform_complex(n, 96, n, 0)
    assert oracle.rel_l2(oracle.dft(x, -1), np.fft.fft(x)) < 1e-14
    assert oracle.rel_l2(oracle.dft(x, +1), n * np.fft.ifft(x)) < 1e-14


def test_dft_orthogonality():
    """sum_j zeta_n^{l j} = n if n | l else 0 (section 2.1): the DFT of ones is n*delta."""
    for n in (6, 16, 35):
        X = oracle.dft(np.ones(n, complex), +1)
        want = np.zeros(n, complex)
        want[0] = n
        assert np.max(np.abs(X - want)) < 1e-12
        for a in range(n):  # DFT of delta_a is zeta^{k a}
            d = np.zeros(n, complex)
            d[a] = 1.0
            want = np.exp(2j * np.pi * ((np.arange(n) * a) % n) / n)
            assert np.max(np.abs(oracle.dft(d, +1) - want)) < 1e-14


@pytest.mark.parametrize("L,N", [(6, 12), (100, 360), (37, 80), (1024, 2048)])
def test_padded_dft_is_N_ifft_of_zero_padding(L, N):
    x = synth.uniform_complex(L, 97, L, 0)
    pad = np.concatenate([x, np.zeros(N - L, complex)])
    assert oracle.rel_l2(oracle.padded_dft(x, N), N * np.fft.ifft(pad)) < 1e-14


def test_friendly_sizes():
    want = {1: 1, 2: 2, 11: 12, 13: 14, 97: 98, 121: 125, 2047: 2048, 4095: 4096, 2 * 3 ** 13 - 1: 2 * 3 ** 13}
    for n, v in want.items():
        assert oracle.friendly_size(n) == v
    for n in range(1, 400):
        s = oracle.friendly_size(n)
        r = s
        for p in (2, 3, 5, 7):
            while r % p == 0:
                r //= p
        assert s >= n and r == 1
        assert all(_not_friendly(c) for c in range(n, s))


def _not_friendly(c):
    for p in (2, 3, 5, 7):
        while c % p == 0:
            c //= p
    return c != 1


@pytest.mark.parametrize("shape", [(1, 7), (5, 1), (6, 9), (16, 16), (13, 40)])
def test_nd2_matches_scipy(shape):
    f, g = synth.pair(shape, 98, shape[0])
    M = tuple(2 * s - 1 for s in shape)
    ref = scipy.signal.convolve(f, g, method="direct")
    assert oracle.rel_l2(oracle.direct_nd(f, g, M), ref) < 1e-14
    assert oracle.rel_l2(oracle.padded_nd(f, g, M), ref) < 1e-14


@pytest.mark.parametrize("shape", [(3, 4, 5), (8, 8, 8), (1, 6, 2)])
def test_nd3_matches_scipy(shape):
    f, g = synth.pair(shape, 99, shape[0])
    M = tuple(2 * s - 1 for s in shape)
    ref = scipy.signal.convolve(f, g, method="direct")
    assert oracle.rel_l2(oracle.direct_nd(f, g, M), ref) < 1e-14
    assert oracle.rel_l2(oracle.padded_nd(f, g, M), ref) < 1e-14


def test_nd_separable_closed_form():
    """f = a (x) b, g = c (x) d  =>  h = (a*c) (x) (b*d)."""
    a = synth.uniform_complex(9, 100, 0, 0)
    b = synth.uniform_complex(14, 100, 1, 0)
    c = synth.uniform_complex(9, 100, 2, 0)
    d = synth.uniform_complex(14, 100, 3, 0)
    f, g = np.outer(a, b), np.outer(c, d)
    M = (17, 27)
    want = np.outer(np.convolve(a, c), np.convolve(b, d))
    assert oracle.rel_l2(oracle.padded_nd(f, g, M), want) < 1e-13
    assert oracle.rel_l2(oracle.direct_nd(f, g, M), want) < 1e-13


def test_nd_with_unit_axis_reduces_to_1d():
    f, g = synth.pair((1, 50), 101, 0)
    h = oracle.padded_nd(f, g, (1, 99))
    assert oracle.rel_l2(h[0], np.convolve(f[0], g[0])) < 1e-14


def test_nd_tail_is_zero():
    f, g = synth.pair((4, 5), 102, 0)
    h = oracle.padded_nd(f, g, (9, 12))
    assert np.all(h[7:, :] == 0) and np.all(h[:, 9:] == 0)


def test_fft_route_error_bound():
    """Round-off of the padded-FFT route stays within O(eps log2 N) of the exact result."""
    L = 1 << 14
    f, g = _gauss_int(L, seed=5, bound=8)
    exact = oracle.direct_1d(f, g, 2 * L - 1)  # exact integers (see test above)
    h = oracle.padded_1d(f, g, 2 * L - 1)
    eps = np.finfo(np.float64).eps
    assert oracle.rel_l2(h, exact) < 4 * eps * np.log2(2 * L)


@pytest.mark.parametrize("name", ["fig2_L6_M11.txt", "int_L37_M80.txt"])
def test_golden_fixtures_exact(name):
    """Stored exact-integer outputs (written by tests/golden/make_golden.py)."""
    from golden_io import load
    L, M, f, g, h = load(name)
    assert f.size == L and h.size == M
    assert np.array_equal(h, _exact_int_conv(f, g, M))
    assert np.array_equal(oracle.direct_1d(f, g, M), h)
    assert np.array_equal(np.round(oracle.padded_1d(f, g, M)), h)



@pytest.mark.parametrize("Lf,Lg", [(1, 9), (2, 100), (12, 100), (12, 1000), (37, 38), (100, 2187)])
def test_unequal_lengths_match_numpy_convolve(Lf, Lg):
    """The unequal case (section 3.5): operands of different lengths."""
    f = synth.uniform_complex(Lf, 103, Lf, 0)
    g = synth.uniform_complex(Lg, 103, Lg, 1)
    ref = np.convolve(f, g)
    for M in (Lf + Lg - 1, Lf + Lg + 5):
        for h in (oracle.direct_1d(f, g, M), oracle.padded_1d(f, g, M)):
            assert oracle.rel_l2(h[:Lf + Lg - 1], ref) < 1e-14
            assert np.all(h[Lf + Lg - 1:] == 0)


def test_unequal_lengths_integer_exact():
    f = synth.gaussian_integers(12, 8, 104, 0, 0)
    g = synth.gaussian_integers(777, 8, 104, 0, 1)
    exact = np.array([sum(complex(int(f[j].real), int(f[j].imag)) * complex(int(g[k - j].real), int(g[k - j].imag))
                          for j in range(max(0, k - 776), min(k, 11) + 1)) for k in range(788)])
    assert np.array_equal(oracle.direct_1d(f, g, 788), exact)
    assert np.array_equal(np.round(oracle.padded_1d(f, g, 788)), exact)


def test_unequal_sampled_matches_full():
    f = synth.uniform_complex(7, 105, 7, 0)
    g = synth.uniform_complex(300, 105, 300, 1)
    full = oracle.direct_1d(f, g, 320)
    ks = np.array([0, 1, 6, 7, 150, 299, 305, 306, 319])
    assert np.array_equal(oracle.direct_1d_sampled(f, g, ks), full[ks])
    assert np.array_equal(oracle.direct_1d_sampled(g, f, ks), oracle.direct_1d(g, f, 320)[ks])



@pytest.mark.parametrize("sf,sg", [((3, 5), (20, 17)), ((20, 2), (4, 30)), ((1, 7), (9, 1)), ((2, 3, 4), (5, 3, 6)),
                                   ((6, 1, 2), (2, 7, 5))])
def test_nd_unequal_matches_scipy(sf, sg):
    """N-D with different extents per operand (section 3.6 with section 3.5's lengths),
    including axes where f is the longer operand."""
    from scipy import signal
    f = synth.uniform_complex(sf, 106, len(sf), 0)
    g = synth.uniform_complex(sg, 106, len(sf), 1)
    ref = signal.convolve(f, g, method="direct")
    K = ref.shape
    M = tuple(k + 2 for k in K)
    h = oracle.padded_nd(f, g, M)
    assert oracle.rel_l2(h[tuple(slice(0, k) for k in K)], ref) < 1e-14
    assert np.all(h[tuple(slice(k, None) if i == 0 else slice(None) for i, k in enumerate(K))] == 0)
    ks = np.arange(int(np.prod(M)))
    d = oracle.direct_nd_sampled(f, g, M, ks).reshape(M)
    assert oracle.rel_l2(d[tuple(slice(0, k) for k in K)], ref) < 1e-14



@pytest.mark.parametrize("L", [1, 2, 7, 100, 1000])
def test_real_matches_numpy_and_complex_oracle(L):
    """The real-arithmetic direct sum against numpy.convolve and against the complex
    oracle on the same data with zero imaginary parts (whose imaginary output is 0)."""
    r = synth.rng(107, L, 0)
    f, g = r.uniform(-1, 1, L), r.uniform(-1, 1, L)
    h = oracle.direct_1d_real(f, g, 2 * L + 3)
    assert np.max(np.abs(h[:2 * L - 1] - np.convolve(f, g))) < 1e-12 and np.all(h[2 * L - 1:] == 0)
    hc = oracle.direct_1d(f.astype(complex), g.astype(complex), 2 * L + 3)
    assert np.all(hc.imag == 0) and np.max(np.abs(hc.real - h)) < 1e-12
    fc, gc = r.uniform(-1, 1, (L, 3)), r.uniform(-1, 1, (L, 3))
    hc3 = oracle.direct_1d_real(fc, gc, 2 * L - 1)
    for c in range(3):
        assert np.max(np.abs(hc3[:, c] - np.convolve(fc[:, c], gc[:, c]))) < 1e-12


def test_real_integer_exact():
    r = synth.rng(108, 0, 0)
    f, g = r.integers(-50, 51, 300).astype(float), r.integers(-50, 51, 300).astype(float)
    exact = [sum(int(f[j]) * int(g[k - j]) for j in range(max(0, k - 299), min(k, 299) + 1)) for k in range(599)]
    assert np.array_equal(oracle.direct_1d_real(f, g, 599), np.array(exact, dtype=float))


# --- multi-convolution of A sequences (section 6.1) -------------------------------------

def _brute_multi(xs, M):
    """The A-fold defining sum by enumerating every index tuple (tiny inputs only)."""
    import itertools
    h = [0j] * M
    for js in itertools.product(*[range(len(x)) for x in xs]):
        k = sum(js)
        if k < M:
            p = 1 + 0j
            for x, j in zip(xs, js):
                p *= x[j]
            h[k] += p
    return np.array(h)


@pytest.mark.parametrize("A,L", [(3, 1), (3, 5), (4, 4), (5, 3), (2, 6)])
def test_multi_matches_tuple_enumeration(A, L):
    r = synth.rng(120, A, L)
    xs = [r.uniform(-1, 1, L) + 1j * r.uniform(-1, 1, L) for _ in range(A)]
    M = A * (L - 1) + 3
    want = _brute_multi(xs, M)
    assert np.max(np.abs(oracle.direct_multi(xs, M) - want)) < 1e-13
    assert np.max(np.abs(oracle.padded_multi(xs, M) - want)) < 1e-13


@pytest.mark.parametrize("A", [2, 3, 4, 6])
def test_multi_matches_numpy_chain_and_copies(A):
    r = synth.rng(121, A, 0)
    L, C = 57, 3
    xs = [r.uniform(-1, 1, (L, C)) + 1j * r.uniform(-1, 1, (L, C)) for _ in range(A)]
    K = A * (L - 1) + 1
    h = oracle.direct_multi(xs, K + 4)
    hp = oracle.padded_multi(xs, K + 4)
    for c in range(C):
        ref = xs[0][:, c]
        for x in xs[1:]:
            ref = np.convolve(ref, x[:, c])
        assert np.max(np.abs(h[:K, c] - ref)) < 1e-12 * np.max(np.abs(ref))
        assert np.all(h[K:, c] == 0)
        assert np.max(np.abs(hp[:K, c] - ref)) < 1e-12 * np.max(np.abs(ref))
    ks = np.array([0, 1, K // 2, K - 1], np.int64)
    assert np.max(np.abs(oracle.multi_sampled(xs, ks) - h[ks])) < 1e-12 * np.max(np.abs(h))


def test_multi_deltas_and_exact_integers():
    """delta_a * delta_b * delta_c = delta_(a+b+c); Gaussian-integer inputs give the exact
    integer result (Python integers) and the A = 2 case is the two-operand oracle."""
    L = 9
    for a, b, c in ((0, 0, 0), (8, 8, 8), (1, 5, 7), (3, 0, 2)):
        xs = [np.eye(L)[i].astype(complex) for i in (a, b, c)]
        h = oracle.direct_multi(xs, 3 * L - 2)
        want = np.zeros(3 * L - 2, complex)
        want[a + b + c] = 1
        assert np.array_equal(h, want)
    xs = [synth.gaussian_integers(40, 6, 122, 0, w) for w in range(4)]
    ex = [complex(int(v.real), int(v.imag)) for v in xs[0]]
    for x in xs[1:]:
        xi = [complex(int(v.real), int(v.imag)) for v in x]
        ex = [sum(ex[j] * xi[k - j] for j in range(max(0, k - len(xi) + 1), min(k, len(ex) - 1) + 1))
              for k in range(len(ex) + len(xi) - 1)]
    assert np.array_equal(oracle.direct_multi(xs, len(ex)), np.array(ex))
    assert np.array_equal(np.round(oracle.padded_multi(xs, len(ex))), np.array(ex))
    assert np.array_equal(oracle.direct_multi(xs[:2], 79), oracle.direct_1d(xs[0], xs[1], 79))
