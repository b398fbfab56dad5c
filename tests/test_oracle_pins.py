"""Pins of the FP64 oracle against things other than itself (CPU only).

* the dense Kronecker matrix of eq. (1) (brute force, m <= 6);
* the paper's factor matrices of eq. (4), built densely from their Section 3
  definitions, multiplied out and compared with eq. (1);
* the explicit N = 8 factors printed in Section 4 (golden fixture);
* numpy.fft per window (an independent library FFT);
* closed forms, Parseval, Hermitian symmetry, adjoint identities;
* the operation counts of eqs. (6)-(7) and the additions total of Section 5.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import recurrence

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example_n8.json")


# ---------------------------------------------------------------------------
# Dense builders written from the definitions of Sections 2-3.
# ---------------------------------------------------------------------------
def bdiag(*mats):
    rows = sum(a.shape[0] for a in mats)
    cols = sum(a.shape[1] for a in mats)
    out = np.zeros((rows, cols), dtype=np.complex128)
    r = c = 0
    for a in mats:
        out[r:r + a.shape[0], c:c + a.shape[1]] = a
        r += a.shape[0]
        c += a.shape[1]
    return out


def eye(n):
    return np.eye(n, dtype=np.complex128)


def w(n, k):
    return np.exp(-2j * np.pi * np.asarray(k, dtype=np.float64) / n)


def E(L):
    idx = np.arange(L)
    return w(L, np.outer(idx, idx))


H2 = np.array([[1, 1], [1, -1]], dtype=np.complex128)


def dense_eq1(m):
    n = 1 << m
    blocks = [np.kron(eye(1 << (m - i)), E(1 << i)) for i in range(1, m + 1)]
    P = np.kron(np.ones((m, 1)), eye(n))
    return bdiag(*blocks) @ P


def Dt(i):
    h = 1 << (i - 1)
    return bdiag(eye(h), np.diag(w(1 << i, np.arange(h))))


def S(i, j):
    return np.kron(eye(1 << (j - 1)), np.kron(H2, eye(1 << (i - j - 1))))


def W(i, j):
    blk = 1 << (i - j)
    return np.kron(eye(1 << (j - 1)), bdiag(eye(blk // 2), np.diag(w(blk, np.arange(blk // 2)))))


def R(i):
    size = 1 << (i - 1)
    out = eye(size)
    for j in range(1, i):                  # R = (W^{i-1} S^{i-1}) ... (W^1 S^1)
        out = W(i, j) @ S(i, j) @ out
    return out


def U(m, i):
    h = 1 << (i - 1)
    top = np.kron(np.ones((1, 2)), eye(h))
    return np.kron(eye(1 << (m - i)), np.vstack([top, np.zeros((h, 2 * h))]))


def V(m, i):
    h = 1 << (i - 1)
    bot = np.hstack([eye(h), -eye(h)])
    return np.kron(eye(1 << (m - i)), np.vstack([np.zeros((h, 2 * h)), bot]))


def T(i):
    L = 1 << i
    t = np.zeros((L, L), dtype=np.complex128)
    for k in range(L):
        t[k, recurrence.bitrev(k, i)] = 1
    return t


def factors(m):
    """(P, A, D, F) for i = 1..m, and Gamma, as dense matrices (Section 3)."""
    n = 1 << m
    out = []
    P1 = np.kron(np.ones((m, 1)), eye(n))
    A1 = bdiag(np.kron(eye(n // 2), H2), eye((m - 1) * n))
    D1 = bdiag(np.kron(eye(n // 2), Dt(1)), eye((m - 1) * n))
    F1 = eye(m * n)
    out.append((P1, A1, D1, F1))
    for i in range(2, m + 1):
        Pi = bdiag(eye((i - 2) * n), np.kron(np.ones((2, 1)), eye(n)), eye((m - i + 1) * n))
        Ai = bdiag(eye((i - 1) * n), np.hstack([U(m, i), V(m, i)]), eye((m - i) * n))
        Di = bdiag(eye((i - 1) * n), np.kron(eye(1 << (m - i)), Dt(i)), eye((m - i) * n))
        Rt = bdiag(eye(1 << (i - 1)), R(i))
        Fi = bdiag(eye((i - 1) * n), np.kron(eye(1 << (m - i)), Rt), eye((m - i) * n))
        out.append((Pi, Ai, Di, Fi))
    G = bdiag(*[np.kron(eye(1 << (m - i)), T(i)) for i in range(1, m + 1)])
    return out, G


def dense_eq4(m):
    fs, G = factors(m)
    acc = None
    for (P, A, D, F) in fs:
        step = F @ D @ A @ P
        acc = step if acc is None else step @ acc
    return G @ acc


def rand_c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


# ---------------------------------------------------------------------------
# Definition pins
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_oracle_matches_dense_kronecker(m):
    rng = np.random.default_rng(100 + m)
    x = rand_c(rng, 1 << m)
    ref = (dense_eq1(m) @ x).reshape(m, -1)
    for method in (oracle.DIRECT, oracle.FFT):
        y = oracle.forward(x, method)
        assert np.max(np.abs(y - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_eq1_block_reading():
    # As printed, I_{2^{m-1}} (x) E_{2^i} is 2^{m-1+i} square, which cannot act on
    # an N-long level; I_{2^{m-i}} (x) E_{2^i} is N x N for every level.
    m = 4
    n = 1 << m
    for i in range(2, m + 1):
        assert np.kron(eye(1 << (m - 1)), E(1 << i)).shape[0] != n
        assert np.kron(eye(1 << (m - i)), E(1 << i)).shape == (n, n)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_eq4_factorisation_equals_eq1(m):
    diff = np.max(np.abs(dense_eq4(m) - dense_eq1(m)))
    assert diff < 1e-12


def _golden_matrix(entry, explicit=True):
    def val(s):
        s = s.strip()
        if s in ("0", "1", "-1"):
            return complex(int(s))
        base, k = s.split("^")
        return complex(w(int(base[1:]), int(k)))
    if explicit:
        return np.array([[val(s) for s in row] for row in entry["rows"]], dtype=np.complex128)
    b = entry["size"]
    blocks = {"0": np.zeros((b, b)), "I": np.eye(b), "-I": -np.eye(b)}
    return np.block([[blocks[s] for s in row] for row in entry["rows"]]).astype(np.complex128)


def test_worked_example_n8_factors():
    g = json.load(open(GOLDEN))
    ex = {k: _golden_matrix(v) for k, v in g["explicit"].items()}
    bl = {k: _golden_matrix(v, explicit=False) for k, v in g["block"].items()}
    assert np.allclose(ex["T2"], T(1)) and np.allclose(ex["T4"], T(2)) and np.allclose(ex["T8"], T(3))
    assert np.allclose(ex["Dtilde2_1"], Dt(1))
    assert np.allclose(ex["Dtilde4_2"], Dt(2))
    assert np.allclose(ex["Dtilde8_3"], Dt(3))
    assert np.allclose(ex["W2_1_of_level2"], W(2, 1))
    assert np.allclose(ex["S2_1_of_level2"], S(2, 1))
    assert np.allclose(ex["S4_1_of_level3"], S(3, 1))
    assert np.allclose(ex["W4_1_of_level3"], W(3, 1))
    assert np.allclose(ex["S4_2_of_level3"], S(3, 2))
    assert np.allclose(ex["W4_2_of_level3"], W(3, 2))
    fs, _ = factors(3)
    assert np.allclose(bl["P2_32x24"], fs[1][0])
    assert np.allclose(bl["P3_32x24"], fs[2][0])
    assert np.allclose(bl["U8_3"], U(3, 3)) and np.allclose(bl["V8_3"], V(3, 3))
    assert np.allclose(bl["U8_2"], U(3, 2)) and np.allclose(bl["V8_2"], V(3, 2))


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 10])
def test_recurrence_model_matches_direct(m):
    rng = np.random.default_rng(200 + m)
    x = rand_c(rng, 1 << m)
    y = recurrence.mrdft_eq4(x)
    ref = oracle.forward(x, oracle.DIRECT)
    assert np.max(np.abs(y - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("m", [1, 4, 7, 10, 12])
def test_fft_route_matches_direct(m):
    rng = np.random.default_rng(300 + m)
    x = rand_c(rng, 1 << m)
    yd = oracle.forward(x, oracle.DIRECT)
    yf = oracle.forward(x, oracle.FFT)
    rel = np.linalg.norm(yd - yf, axis=1) / np.linalg.norm(yd, axis=1)
    assert rel.max() < 1e-13


@pytest.mark.parametrize("m", [3, 9, 14])
def test_numpy_fft_per_window(m):
    rng = np.random.default_rng(400 + m)
    x = rand_c(rng, 1 << m)
    y = oracle.forward(x)
    for i in range(1, m + 1):
        ref = np.fft.fft(x.reshape(-1, 1 << i), axis=1).reshape(-1)
        assert np.linalg.norm(y[i - 1] - ref) / np.linalg.norm(ref) < 1e-13


def test_forward_bin_and_level_agree():
    rng = np.random.default_rng(7)
    m = 11
    x = rand_c(rng, 1 << m)
    y = oracle.forward(x)
    for i in (1, 5, 11):
        assert np.allclose(oracle.forward_level(x, i, oracle.FFT), y[i - 1], atol=1e-10)
        L = 1 << i
        for (wi, k) in [(0, 0), (0, L - 1), ((1 << (m - i)) - 1, L // 3)]:
            assert abs(oracle.forward_bin(x, i, wi, k) - y[i - 1][wi * L + k]) < 1e-10


# ---------------------------------------------------------------------------
# Closed forms and invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n0", [0, 1, 37, 255])
def test_impulse(n0):
    m = 8
    n = 1 << m
    x = np.zeros(n, dtype=np.complex128)
    x[n0] = 1.0
    y = oracle.forward(x)
    for i in range(1, m + 1):
        L = 1 << i
        expect = np.zeros(n, dtype=np.complex128)
        wi = n0 >> i
        expect[wi * L:(wi + 1) * L] = w(L, (n0 % L) * np.arange(L))
        assert np.max(np.abs(y[i - 1] - expect)) < 1e-12


def test_constant():
    m = 9
    c = 0.75 - 2.0j
    y = oracle.forward(np.full(1 << m, c))
    for i in range(1, m + 1):
        L = 1 << i
        expect = np.zeros((1 << (m - i), L), dtype=np.complex128)
        expect[:, 0] = c * L
        assert np.max(np.abs(y[i - 1].reshape(-1, L) - expect)) < 1e-11


@pytest.mark.parametrize("k0", [0, 1, 96, 200])
def test_complex_exponential(k0):
    m = 8
    n = 1 << m
    t = np.arange(n)
    x = np.exp(2j * np.pi * k0 * t / n)
    y = oracle.forward(x)
    for i in range(1, m + 1):
        L = 1 << i
        for wi in range(n // L):
            ph = np.exp(2j * np.pi * k0 * wi * L / n)
            for k in range(L):
                r = np.exp(2j * np.pi * (k0 / n - k / L))
                if abs(r - 1) < 1e-12:
                    expect = ph * L
                else:
                    expect = ph * (1 - r ** L) / (1 - r)
                assert abs(y[i - 1][wi * L + k] - expect) < 1e-9
        if k0 % (1 << (m - i)) == 0:          # single-bin case
            kk = k0 >> (m - i)
            blk = y[i - 1].reshape(-1, L)
            assert np.allclose(np.abs(blk[:, kk]), L)
            mask = np.ones(L, bool)
            mask[kk] = False
            assert np.max(np.abs(blk[:, mask])) < 1e-9


def test_parseval_per_level():
    rng = np.random.default_rng(11)
    m = 13
    x = rand_c(rng, 1 << m)
    y = oracle.forward(x)
    e = np.sum(np.abs(x) ** 2)
    for i in range(1, m + 1):
        assert abs(np.sum(np.abs(y[i - 1]) ** 2) / ((1 << i) * e) - 1) < 1e-12


def test_hermitian_for_real_input():
    rng = np.random.default_rng(12)
    m = 10
    x = rng.standard_normal(1 << m)
    y = oracle.forward(x)
    for i in range(1, m + 1):
        L = 1 << i
        blk = y[i - 1].reshape(-1, L)
        mirror = blk[:, (-np.arange(L)) % L]
        assert np.max(np.abs(blk - np.conj(mirror))) < 1e-10


@pytest.mark.parametrize("method", [oracle.DIRECT, oracle.FFT])
def test_adjoint_identity(method):
    rng = np.random.default_rng(13)
    m = 9
    n = 1 << m
    x = rand_c(rng, n)
    gy = rand_c(rng, m * n).reshape(m, n)
    lhs = np.vdot(gy.reshape(-1), oracle.forward(x, method).reshape(-1))      # <Ax, y>
    rhs = np.vdot(oracle.adjoint(gy, method), x)                               # <A^H y, x>
    assert abs(lhs - rhs) < 1e-9 * abs(lhs)


def test_adjoint_dense_and_gram():
    rng = np.random.default_rng(14)
    for m in (1, 3, 6):
        n = 1 << m
        gy = rand_c(rng, m * n).reshape(m, n)
        ref = dense_eq1(m).conj().T @ gy.reshape(-1)
        assert np.max(np.abs(oracle.adjoint(gy, oracle.DIRECT) - ref)) < 1e-11
        assert np.max(np.abs(oracle.adjoint(gy, oracle.FFT) - ref)) < 1e-11
        x = rand_c(rng, n)
        # A^H A = sum_i 2^i I = (2^{m+1} - 2) I
        g = oracle.adjoint(oracle.forward(x))
        assert np.max(np.abs(g - (2 ** (m + 1) - 2) * x)) < 1e-10 * 2 ** m


def test_adjoint_point():
    rng = np.random.default_rng(15)
    m = 10
    n = 1 << m
    gy = rand_c(rng, m * n).reshape(m, n)
    gx = oracle.adjoint(gy)
    for p in (0, 1, 511, 1023):
        assert abs(oracle.adjoint_point(gy, p) - gx[p]) < 1e-9


# ---------------------------------------------------------------------------
# Spectral loss: exact closed form and FP64 central differences
# ---------------------------------------------------------------------------
def test_spectral_loss_closed_form():
    rng = np.random.default_rng(16)
    m = 10
    x = rng.standard_normal(1 << m)
    z = rng.standard_normal(1 << m)
    nd, L = oracle.spectral_loss(x, z)
    ratio = np.sum((x - z) ** 2) / np.sum(z ** 2)
    assert np.allclose(nd[:, 0] / nd[:, 1], ratio, rtol=1e-12)
    assert np.allclose(nd[:, 1], (2.0 ** np.arange(1, m + 1)) * np.sum(z ** 2), rtol=1e-12)
    assert abs(L - ratio) < 1e-12 * ratio
    g = oracle.spectral_loss_grad(x, z, nd, gL=1.0)
    assert np.allclose(g, 2 * (x - z) / np.sum(z ** 2), rtol=1e-10, atol=1e-14)


def test_spectral_loss_finite_differences():
    rng = np.random.default_rng(17)
    m = 5
    n = 1 << m
    x = rng.standard_normal(n)
    z = rng.standard_normal(n)
    nd, _ = oracle.spectral_loss(x, z)
    g = oracle.spectral_loss_grad(x, z, nd, gL=0.5)
    h = 1e-4
    fd = np.empty(n)
    for p in range(n):
        e = np.zeros(n)
        e[p] = h
        fd[p] = 0.5 * (oracle.spectral_loss(x + e, z)[1] - oracle.spectral_loss(x - e, z)[1]) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-8 * max(1.0, np.max(np.abs(g)))


# ---------------------------------------------------------------------------
# Section 5 operation counts
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8])
def test_operation_counts(m):
    c = recurrence.counts_eq4(m)
    for i in range(1, m + 1):
        assert c.mul[i] == (i + 1) * 2 ** (m - 2)                     # eq. (6)
        assert c.mul_nontrivial[i] == (0 if i == 1 else (i - 2) * 2 ** (m - 2))   # eq. (7)
        assert c.add[i] == 2 * c.mul[i]                                # additions = 2 beta
    assert sum(c.mul) == m * (m + 3) * 2 ** (m - 3)
    assert sum(c.mul_nontrivial) == (m - 1) * (m - 2) * 2 ** (m - 3)


def test_invalid_arguments():
    lib = oracle._load()
    x = np.zeros(4, dtype=np.complex128)
    y = np.zeros(8, dtype=np.complex128)
    assert lib.mro_forward(0, oracle._dp(x), oracle._dp(y), 0) != 0
    assert lib.mro_forward(31, oracle._dp(x), oracle._dp(y), 0) != 0
    assert lib.mro_forward_level(2, 3, oracle._dp(x), oracle._dp(y), 0) != 0
    with pytest.raises(ValueError):
        oracle.forward(np.zeros(6))


def test_spectral_loss_terms_follow_parseval():
    """Each level is a block-diagonal DFT of non-overlapping windows, and one
    window's DFT satisfies E^H E = 2^i I (Section 2, eq. (1)); so the level
    energies of the loss are num_i = 2^i ||x - z||^2 and den_i = 2^i ||z||^2,
    and L = ||x - z||^2 / ||z||^2 whatever m is.  A dropped window, a wrong
    level length or a missing conjugate in the oracle's loss breaks this."""
    rng = np.random.default_rng(77)
    for m in (1, 5, 9):
        x = rng.standard_normal(1 << m)
        z = rng.standard_normal(1 << m)
        nd, L = oracle.spectral_loss(x, z)
        for i in range(1, m + 1):
            assert nd[i - 1, 0] == pytest.approx((2 ** i) * np.sum((x - z) ** 2), rel=1e-12)
            assert nd[i - 1, 1] == pytest.approx((2 ** i) * np.sum(z ** 2), rel=1e-12)
        assert L == pytest.approx(np.sum((x - z) ** 2) / np.sum(z ** 2), rel=1e-12)


# ---------------------------------------------------------------------------
# Packed half-spectrum layout of real signals (optional output).

@pytest.mark.parametrize("m", [2, 3, 7, 10])
def test_half_spectrum_matches_numpy_rfft(m):
    """For a real window numpy.fft.rfft gives bins 0..L/2 (an independent
    library routine): value 0 must be (Re bin 0, Re bin L/2), values
    1..L/2-1 the bins themselves, and bins 0 and L/2 must be real."""
    rng = np.random.default_rng(100 + m)
    x = rng.standard_normal(1 << m)
    h = oracle.forward_half(x)
    assert h.shape == (m, (1 << m) // 2)
    for i in range(1, m + 1):
        L = 1 << i
        r = np.fft.rfft(x.reshape(-1, L), axis=1)
        blk = h[i - 1].reshape(-1, L // 2)
        assert np.max(np.abs(blk[:, 0].real - r[:, 0].real)) < 1e-11
        assert np.max(np.abs(blk[:, 0].imag - r[:, L // 2].real)) < 1e-11
        assert np.max(np.abs(r[:, 0].imag)) < 1e-11 and np.max(np.abs(r[:, L // 2].imag)) < 1e-11
        if L > 2:
            assert np.max(np.abs(blk[:, 1:] - r[:, 1:L // 2])) < 1e-10


def test_half_spectrum_closed_forms():
    """Level 1 packs (x0 + x1, x0 - x1); a constant c packs (c L, 0) into
    value 0 of every window and zeros elsewhere; an alternating signal packs
    (0, L) (all of it at the Nyquist bin)."""
    x = np.array([3.0, -1.0, 2.0, 5.0])
    h = oracle.forward_half(x)
    assert np.allclose(h[0], [2.0 + 4.0j, 7.0 - 3.0j])
    m = 6
    c = np.full(1 << m, 1.5)
    alt = np.array([(-1.0) ** n for n in range(1 << m)])
    hc, ha = oracle.forward_half(c), oracle.forward_half(alt)
    for i in range(1, m + 1):
        L = 1 << i
        bc, ba = hc[i - 1].reshape(-1, L // 2), ha[i - 1].reshape(-1, L // 2)
        assert np.allclose(bc[:, 0], 1.5 * L) and np.allclose(bc[:, 1:], 0.0, atol=1e-12)
        assert np.allclose(ba[:, 0], 1j * L) and np.allclose(ba[:, 1:], 0.0, atol=1e-12)


@pytest.mark.parametrize("m", [2, 5, 9])
def test_half_adjoint_identity(m):
    """The half-spectrum output is real-linear in real x, so its adjoint G
    must satisfy Re<h(x), g> = <x, G g> for every real x and complex g (the
    gradient of the real loss Re<h(x), g>).  A missing factor, a value sent to
    the wrong bin or a dropped Nyquist term breaks it."""
    rng = np.random.default_rng(200 + m)
    n = 1 << m
    x = rng.standard_normal(n)
    g = rng.standard_normal((m, n // 2)) + 1j * rng.standard_normal((m, n // 2))
    lhs = np.real(np.vdot(g.reshape(-1), oracle.forward_half(x).reshape(-1)))
    rhs = float(np.dot(x, oracle.adjoint_half(g)))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))
    # and by brute force on the basis vectors for the smallest case
    if m == 2:
        for p in range(n):
            e = np.zeros(n)
            e[p] = 1.0
            assert oracle.adjoint_half(g)[p] == pytest.approx(
                np.real(np.vdot(g.reshape(-1), oracle.forward_half(e).reshape(-1))), abs=1e-12)


# ---------------------------------------------------------------------------
# Two-dimensional separable MrDFT.

def _direct2d(x):
    """The double sum of every block's 2-D DFT, exponents reduced exactly in
    integers (brute force, tiny images only)."""
    n1, n2 = x.shape
    m1, m2 = n1.bit_length() - 1, n2.bit_length() - 1
    out = np.zeros((m1, m2, n1, n2), dtype=np.complex128)
    for i1 in range(1, m1 + 1):
        L1 = 1 << i1
        for i2 in range(1, m2 + 1):
            L2 = 1 << i2
            for p1 in range(n1):
                b1, k1 = divmod(p1, L1)
                for p2 in range(n2):
                    b2, k2 = divmod(p2, L2)
                    acc = 0j
                    for a in range(L1):
                        for c in range(L2):
                            e1 = (a * k1) % L1
                            e2 = (c * k2) % L2
                            ang = -2.0 * np.pi * (e1 / L1 + e2 / L2)
                            acc += x[b1 * L1 + a, b2 * L2 + c] * complex(np.cos(ang), np.sin(ang))
                    out[i1 - 1, i2 - 1, p1, p2] = acc
    return out


@pytest.mark.parametrize("shape", [(2, 2), (4, 8), (8, 4)])
def test_forward2d_matches_double_sum(shape):
    rng = np.random.default_rng(300 + shape[0] * 10 + shape[1])
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert np.max(np.abs(oracle.forward2d(x) - _direct2d(x))) < 1e-11


def test_forward2d_matches_numpy_fft2_per_block():
    rng = np.random.default_rng(310)
    x = rng.standard_normal((16, 32))
    y = oracle.forward2d(x)
    for i1 in range(1, 5):
        for i2 in range(1, 6):
            L1, L2 = 1 << i1, 1 << i2
            blocks = x.reshape(16 // L1, L1, 32 // L2, L2).transpose(0, 2, 1, 3)
            ref = np.fft.fft2(blocks).transpose(0, 2, 1, 3).reshape(16, 32)
            assert np.max(np.abs(y[i1 - 1, i2 - 1] - ref)) < 1e-10


def test_forward2d_parseval_and_impulse():
    rng = np.random.default_rng(311)
    x = rng.standard_normal((8, 16)) + 1j * rng.standard_normal((8, 16))
    y = oracle.forward2d(x)
    e = np.sum(np.abs(x) ** 2)
    for i1 in range(1, 4):
        for i2 in range(1, 5):
            assert np.sum(np.abs(y[i1 - 1, i2 - 1]) ** 2) == pytest.approx(2 ** (i1 + i2) * e, rel=1e-12)
    # impulse at (p, q): one block per level pair holds w_L1^{(p mod L1) k1} w_L2^{(q mod L2) k2}
    d = np.zeros((8, 16))
    d[5, 11] = 1.0
    yd = oracle.forward2d(d)
    for i1 in range(1, 4):
        for i2 in range(1, 5):
            L1, L2 = 1 << i1, 1 << i2
            blk = np.zeros((8, 16), dtype=np.complex128)
            b1, b2 = 5 // L1, 11 // L2
            k1, k2 = np.arange(L1), np.arange(L2)
            blk[b1 * L1:(b1 + 1) * L1, b2 * L2:(b2 + 1) * L2] = np.outer(
                np.exp(-2j * np.pi * ((5 % L1) * k1 % L1) / L1), np.exp(-2j * np.pi * ((11 % L2) * k2 % L2) / L2))
            assert np.max(np.abs(yd[i1 - 1, i2 - 1] - blk)) < 1e-12


def test_adjoint2d_identity():
    rng = np.random.default_rng(312)
    x = rng.standard_normal((8, 4)) + 1j * rng.standard_normal((8, 4))
    g = rng.standard_normal((3, 2, 8, 4)) + 1j * rng.standard_normal((3, 2, 8, 4))
    lhs = np.vdot(g.reshape(-1), oracle.forward2d(x).reshape(-1))
    rhs = np.vdot(oracle.adjoint2d(g), x)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
