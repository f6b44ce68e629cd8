"""CPU pins of the arithmetic behind the reduced-precision product forms.

The dense product (S^-1 - I) W of the deviation form runs as three 16-bit
matrix-core products of hi/lo splits (x = hi + lo, hi = r(x), lo = r(x - hi)):
A_hi B_hi + A_hi B_lo + A_lo B_hi.  These tests emulate the splits with
numpy (float16; bfloat16 by round-to-nearest-even on float32 bits) and check
the error bounds the design relies on: a power-of-two scale putting the
largest |x| in [2^13, 2^14) keeps the fp16 pair inside fp16's range and
accurate to about 2^-22 of |x|, against about 2^-16 for the bf16 pair, and
the three-product sum inherits that difference; the five dithered bf16 copies
of the lo part of S^-1 - I average to it within a tenth of its grid step.  No
GPU code is involved.
"""
import numpy as np


def _bf16(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def _pow2_scale(m):
    """2^e with m 2^e in [2^13, 2^14) (1 for m = 0)."""
    if m == 0.0:
        return np.float32(1.0)
    return np.float32(2.0 ** (13 - int(np.floor(np.log2(m)))))


def _split_f16(x, s):
    xs = np.asarray(x, dtype=np.float32) * s
    hi = xs.astype(np.float16)
    lo = (xs - hi.astype(np.float32)).astype(np.float16)
    return xs, hi.astype(np.float64), lo.astype(np.float64)


def _split_bf16(x):
    x = np.asarray(x, dtype=np.float32)
    hi = _bf16(x)
    lo = _bf16(x - hi)
    return hi.astype(np.float64), lo.astype(np.float64)


def _values(rng, n, decades=8):
    return (rng.standard_normal(n) * np.exp(rng.uniform(-decades, 0.0, n))).astype(np.float32)


def test_scale_puts_the_maximum_in_range():
    rng = np.random.default_rng(3)
    for _ in range(200):
        x = _values(rng, 64) * np.float32(10.0 ** rng.uniform(-12, 3))
        m = float(np.abs(x).max())
        s = _pow2_scale(m)
        assert 2.0 ** 13 <= m * s < 2.0 ** 14
        xs, hi, lo = _split_f16(x, s)
        assert np.isfinite(hi).all() and np.isfinite(lo).all()
    assert _pow2_scale(0.0) == 1.0


def test_fp16_pair_carries_22_bits_bf16_pair_16():
    rng = np.random.default_rng(4)
    x = _values(rng, 200_000)
    m = float(np.abs(x).max())
    xs, hi, lo = _split_f16(x, _pow2_scale(m))
    err16 = np.abs(xs.astype(np.float64) - hi - lo)
    big = np.abs(x) >= m / 1024
    assert (err16[big] / np.abs(xs[big])).max() <= 2.0 ** -22
    # below that, the error is at most fp16's smallest spacing (in scaled units)
    assert err16.max() <= 2.0 ** -22 * np.abs(xs).max()
    hb, lb = _split_bf16(x)
    errb = np.abs(x.astype(np.float64) - hb - lb)
    nz = x != 0
    assert (errb[nz] / np.abs(x[nz])).max() <= 2.0 ** -16


def test_three_product_sum_error():
    """Complex product of an S^-1 - I-like matrix (small, dense) with a W-like one:
    the fp16 form's error is below 2^-20 of sum |A||B| per element, and at least
    sixteen times below the bf16 form's (measured: 6.4e-8 against 4.6e-6)."""
    rng = np.random.default_rng(5)
    n = 96
    a = (0.06 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n))
    b = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * np.exp(
        rng.uniform(-6, 0, (n, n)))
    a = a.astype(np.complex64)
    b = b.astype(np.complex64)
    exact = a.astype(np.complex128) @ b.astype(np.complex128)
    scale = np.abs(a.astype(np.complex128)) @ np.abs(b.astype(np.complex128))

    def three(split_a, split_b):
        (arh, arl), (aih, ail) = split_a
        (brh, brl), (bih, bil) = split_b
        def p(xh, xl, yh, yl):
            return xh @ yh + xh @ yl + xl @ yh
        re = p(arh, arl, brh, brl) - p(aih, ail, bih, bil)
        im = p(arh, arl, bih, bil) + p(aih, ail, brh, brl)
        return re + 1j * im

    sa = _pow2_scale(float(max(np.abs(a.real).max(), np.abs(a.imag).max())))
    sb = _pow2_scale(float(max(np.abs(b.real).max(), np.abs(b.imag).max())))
    fa = [_split_f16(a.real, sa)[1:], _split_f16(a.imag, sa)[1:]]
    fb = [_split_f16(b.real, sb)[1:], _split_f16(b.imag, sb)[1:]]
    g16 = three(fa, fb) / (float(sa) * float(sb))
    gbf = three([_split_bf16(a.real), _split_bf16(a.imag)], [_split_bf16(b.real), _split_bf16(b.imag)])
    e16 = (np.abs(g16 - exact) / scale).max()
    ebf = (np.abs(gbf - exact) / scale).max()
    assert e16 < 2.0 ** -20
    assert ebf > 16 * e16


def _dithered_bf16(r, level, copies=5):
    """The lo part of the bf16 split of S^-1 - I in copy `level` (0..copies-1):
    |r| + d u rounded to bf16, d = (level + 1/2)/copies - 1/2, u the bf16 grid
    step at |r|, the sign of r applied afterwards; r = 0 stays 0."""
    r = np.asarray(r, dtype=np.float32)
    ar = np.abs(r).astype(np.float64)
    d = (level + 0.5) / copies - 0.5
    _, e = np.frexp(ar)
    u = np.ldexp(1.0, e - 8)
    t = (ar + d * u).astype(np.float32) if d != 0.0 else ar.astype(np.float32)
    m = _bf16(t).astype(np.float64)
    out = np.where(r < 0, -m, m)
    return np.where(r == 0, 0.0, out)


def test_dithered_bf16_copies_average_to_the_remainder():
    # The constant S^-1 - I enters every step; its bf16 lo part is stored in five
    # copies with rounding offsets -2/5 .. 2/5 of the grid step, one per step.
    # Their mean is within u/10 of the remainder (plain rounding: up to u/2),
    # the middle copy is the plain rounding, and the sign is applied after the
    # magnitude, so mirror elements (conjugates) stay exact mirrors.
    rng = np.random.default_rng(8)
    x = _values(rng, 100_000)
    hi = _bf16(x)
    r = (x - hi).astype(np.float32)
    ar = np.abs(r).astype(np.float64)
    _, e = np.frexp(ar)
    u = np.ldexp(1.0, e - 8)
    copies = [_dithered_bf16(r, j) for j in range(5)]
    plain = _split_bf16(x)[1]
    assert np.array_equal(copies[2], plain)
    for j, c in enumerate(copies):
        assert np.array_equal(_dithered_bf16(-r, j), -c)
        assert np.all(c[r == 0] == 0.0)
    mean = np.mean(copies, axis=0)
    # away from a binade edge (where the grid step of the rounded value doubles)
    inner = (ar > 0) & (np.frexp(ar + 0.5 * u)[1] == e) & (np.frexp(np.maximum(ar - 0.5 * u, 0))[1] == e)
    err_mean = np.abs(mean - r.astype(np.float64))[inner] / u[inner]
    err_plain = np.abs(plain - r.astype(np.float64))[inner] / u[inner]
    assert err_mean.max() <= 0.1 + 1e-6
    assert err_plain.max() > 0.45
    assert np.sqrt(np.mean(err_mean ** 2)) < 0.25 * np.sqrt(np.mean(err_plain ** 2))
