"""Index algebra of the register plane pass's lane-group transforms, on the
CPU.

A line of N points is shared by L lanes of M = N / L values each; the
kernels transform each lane's values in registers and join the lanes with
radix-2 levels (fft.hip: group_fft_dit / group_fft_dif for L = 2, 4 and 8,
group_fft_dit_h / group_fft_dif_h for the exchange of halves).  This module
restates those level schedules with numpy arrays indexed [lane][value] and
checks that they compute the DFT with the layouts the kernels rely on:
  - decimation in time from x[L j + q] in lane q to X[rev(q) M + k],
    rev reversing the log2(L) bits of q;
  - decimation in frequency from that layout to X[L k + q];
  - exchange of halves: between the transforms lane q holds X[c_q + k] and
    X[c_q + 2M + k] (k < M / 2), c_q = (q >> 1) M / 2 + (q & 1) M.
Unnormalised transforms, inverse e^{+2 pi i jk / N}, against numpy's FFT.
Test infrastructure; it shares nothing with the oracle or the library.
"""
import numpy as np
import pytest


def _tw(n, inv):
    w = np.exp(-2j * np.pi * np.arange(n) / n)
    return np.conj(w) if inv else w


def _dft(v, inv):
    return np.fft.ifft(v) * len(v) if inv else np.fft.fft(v)


def _rev(q, bits):
    r = 0
    for b in range(bits):
        r |= ((q >> b) & 1) << (bits - 1 - b)
    return r


def _twiddle(e, n, b, nb, lo_of, inv):
    """Lanes with bit b set multiply value k by w_NB^(lo M + k)."""
    L, M = e.shape
    w = _tw(n, inv)
    st = n // nb
    out = e.copy()
    for q in range(L):
        if (q >> b) & 1:
            lo = lo_of(q)
            out[q] *= w[(lo * M + np.arange(M)) * st]
    return out


def _join(e, b):
    """Lanes q and q ^ 2^b: the bit-clear lane takes own + partner's, the
    other partner's - own."""
    out = e.copy()
    for q in range(e.shape[0]):
        p = q ^ (1 << b)
        out[q] = e[p] + (-1 if (q >> b) & 1 else 1) * e[q]
    return out


def _levels(L):
    """(bit, sub-transform length in units of M, lo of the lane) per level,
    in decimation-in-time order."""
    if L == 2:
        return [(0, 2, lambda q: 0)]
    if L == 4:
        return [(1, 2, lambda q: 0), (0, 4, lambda q: (q >> 1) & 1)]
    return [(2, 2, lambda q: 0), (1, 4, lambda q: (q >> 2) & 1),
            (0, 8, lambda q: 2 * ((q >> 1) & 1) + ((q >> 2) & 1))]


def group_dit(x, L, inv):
    n = len(x)
    M = n // L
    e = np.array([_dft(x[q::L], inv) for q in range(L)])
    for b, mult, lo in _levels(L):
        e = _join(_twiddle(e, n, b, mult * M, lo, inv), b)
    return e


def group_dif(e, L, inv):
    L_, M = e.shape
    n = L * M
    for b, mult, lo in reversed(_levels(L)):
        e = _twiddle(_join(e, b), n, b, mult * M, lo, inv)
    return np.array([_dft(e[q], inv) for q in range(L)])


CASES = [(2, 50), (2, 90), (4, 24), (4, 36), (4, 40), (4, 72), (8, 72), (8, 48)]


@pytest.mark.parametrize("L,n", CASES)
@pytest.mark.parametrize("inv", [True, False])
def test_group_transforms_layouts(L, n, inv):
    rng = np.random.default_rng(n * 10 + L)
    M = n // L
    bits = L.bit_length() - 1
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = _dft(x, inv)
    e = group_dit(x, L, inv)
    got = np.empty(n, complex)
    for q in range(L):
        got[_rev(q, bits) * M + np.arange(M)] = e[q]
    assert np.abs(got - X).max() <= 1e-12 * np.abs(X).max()
    # decimation in frequency from the layout decimation in time leaves
    e_in = np.array([x[_rev(q, bits) * M + np.arange(M)] for q in range(L)])
    e_out = group_dif(e_in, L, inv)
    got = np.empty(n, complex)
    for q in range(L):
        got[L * np.arange(M) + q] = e_out[q]
    assert np.abs(got - X).max() <= 1e-12 * np.abs(X).max()


def _halves_base(q, M):
    return (q >> 1) * (M // 2) + (q & 1) * M


def _swap(x, y, b):
    """A lane-pair move over bit b: the bit-clear lane ends with (x, the
    partner's x), the partner with (the first lane's y, y)."""
    xo, yo = x.copy(), y.copy()
    for q in range(x.shape[0]):
        p = q ^ (1 << b)
        if (q >> b) & 1:
            xo[q] = y[p]
        else:
            yo[q] = x[p]
    return xo, yo


def _halves_level(e, n, b, st, base_of, inv, dit):
    L, M = e.shape
    H = M // 2
    w = _tw(n, inv)
    t = np.array([w[base_of(q) + st * np.arange(H)] for q in range(L)])
    x, y = e[:, :H].copy(), e[:, H:].copy()
    if dit:
        x, y = _swap(x, y, b)
        u = y * t
        return np.concatenate([x + u, x - u], axis=1)
    x, y = x + y, (x - y) * t
    x, y = _swap(x, y, b)
    return np.concatenate([x, y], axis=1)


@pytest.mark.parametrize("n", [24, 40, 48, 64, 72])
@pytest.mark.parametrize("inv", [True, False])
def test_exchange_of_halves_layout(n, inv):
    L, M = 4, n // 4
    H = M // 2
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = _dft(x, inv)
    e = np.array([_dft(x[q::L], inv) for q in range(L)])
    e = _halves_level(e, n, 1, 2, lambda q: (q >> 1) * M, inv, True)
    e = _halves_level(e, n, 0, 1, lambda q: _halves_base(q, M), inv, True)
    got = np.empty(n, complex)
    for q in range(L):
        c = _halves_base(q, M)
        got[c + np.arange(H)] = e[q, :H]
        got[c + 2 * M + np.arange(H)] = e[q, H:]
    assert np.abs(got - X).max() <= 1e-12 * np.abs(X).max()
    # the forward (decimation in frequency) half from that layout
    e_in = np.array([np.concatenate([x[_halves_base(q, M) + np.arange(H)],
                                     x[_halves_base(q, M) + 2 * M + np.arange(H)]]) for q in range(L)])
    e = _halves_level(e_in, n, 0, 1, lambda q: _halves_base(q, M), inv, False)
    e = _halves_level(e, n, 1, 2, lambda q: (q >> 1) * M, inv, False)
    e = np.array([_dft(e[q], inv) for q in range(L)])
    got = np.empty(n, complex)
    for q in range(L):
        got[L * np.arange(M) + q] = e[q]
    assert np.abs(got - X).max() <= 1e-12 * np.abs(X).max()
