"""Pins of the oracle's elementary functions against the error bounds of the
published methods they implement (Cody-Waite exp reduction with a degree-13
Taylor polynomial; log1p via 2*atanh(y/(2+y)) with a 17-term series).

References are exact values computed with 40-digit decimal arithmetic at the
binary64 inputs, plus the platform libm for large samples.  Bounds: pexp 1 ulp of
exact (the reduction is exact to ~2^-85 and the polynomial's truncation is below
4e-18, so only the final roundings remain); plog1p 3 ulp (s = y/(2+y) carries two
roundings, then the series and the final product one each); softplus 3 ulp;
sigma 2 ulp; pcosh 1 ulp."""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

getcontext().prec = 40


def ulp_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.spacing(np.abs(ref))


def exact(f, xs):
    return np.array([float(f(Decimal(float(x)))) for x in xs])


def test_pexp_vs_libm_and_exact(orc):
    rng = np.random.default_rng(11)
    x = rng.uniform(-40.0, 40.0, 400_000)
    assert ulp_err(orc.elem_array("pexp", x), np.exp(x)).max() <= 2.0
    xs = x[:20_000]
    assert ulp_err(orc.elem_array("pexp", xs), exact(lambda d: d.exp(), xs)).max() <= 1.0
    assert orc.pexp(0.0) == 1.0
    for k in range(-50, 51):   # e^(k ln2) is 2^k up to the argument's own rounding
        a = k * math.log(2.0)
        assert ulp_err(orc.pexp(a), float(Decimal(a).exp())) <= 1.0


def test_pexp_reduction_constants_are_the_exact_roundings():
    # The reduction's defining identities, with the constants written in elem.c.
    ln2 = Fraction(Decimal(2).ln(getcontext().__class__(prec=100)))
    hi = float.fromhex("0x1.62e42feep-1")
    lo = float.fromhex("0x1.a39ef35793c76p-33")
    inv = float.fromhex("0x1.71547652b82fep+0")
    assert float(Fraction(1) / ln2) == inv
    m, e = math.frexp(hi)
    assert m * 2 ** 32 == int(m * 2 ** 32)            # 32 significant bits
    assert hi <= ln2 < hi + Fraction(2) ** (e - 32)   # truncated, not rounded
    assert float(ln2 - Fraction(hi)) == lo


def test_plog1p(orc):
    rng = np.random.default_rng(12)
    y = rng.uniform(0.0, 1.0, 20_000)
    ref = exact(lambda d: (1 + d).ln(), y)
    assert ulp_err(orc.elem_array("plog1p", y), ref).max() <= 3.0
    tiny = 10.0 ** rng.uniform(-300, 0, 300)
    wide = getcontext().__class__(prec=400)    # 1 + y exact down to y = 1e-300
    ref = exact(lambda d: wide.add(Decimal(1), d).ln(wide), tiny)
    assert ulp_err(orc.elem_array("plog1p", tiny), ref).max() <= 3.0
    big = rng.uniform(0.0, 1.0, 400_000)
    assert ulp_err(orc.elem_array("plog1p", big), np.log1p(big)).max() <= 4.0
    assert orc.plog1p(0.0) == 0.0


def test_softplus_sigma_pcosh(orc):
    rng = np.random.default_rng(13)
    t = rng.uniform(-35.0, 35.0, 20_000)
    ref = exact(lambda d: max(d, Decimal(0)) + (1 + (-abs(d)).exp()).ln(), t)
    assert ulp_err(orc.elem_array("softplus", t), ref).max() <= 3.0
    ref = exact(lambda d: 1 / (1 + (-d).exp()), t)
    assert ulp_err(orc.elem_array("sigma", t), ref).max() <= 2.0
    u = rng.uniform(0.05, 5.0, 20_000)
    ref = exact(lambda d: (d.exp() + (-d).exp()) / 2, u)
    assert ulp_err(orc.elem_array("pcosh", u), ref).max() <= 1.0
    # sigma is the derivative of softplus
    tt = np.linspace(-30.0, 30.0, 2001)
    h = 1e-6
    fd = (orc.elem_array("softplus", tt + h) - orc.elem_array("softplus", tt - h)) / (2 * h)
    assert np.allclose(fd, orc.elem_array("sigma", tt), rtol=1e-7, atol=1e-9)
    assert orc.softplus(0.0) == orc.plog1p(1.0)
    assert orc.sigma(0.0) == 0.5
