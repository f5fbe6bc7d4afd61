"""Pins of the oracle's alloc/do-all microbenchmark.

x = fma(0.01f, v, x) is pinned by exact rational arithmetic with a separately
written round-to-nearest-even into binary32; the churn counts are pinned by
their closed forms."""
from fractions import Fraction

import numpy as np
import pytest

from synth import workloads as W


def rn32(q: Fraction) -> np.float32:
    """Round an exact rational to the nearest binary32, ties to even."""
    if q == 0:
        return np.float32(0.0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    ulp = Fraction(2) ** (max(e, -126) - 23)
    m = a / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return np.float32(sign * float(fl * ulp))


def test_rn32_helper_against_known_values():
    assert rn32(Fraction(1, 3)) == np.float32(1 / 3)
    assert rn32(Fraction(1) + Fraction(1, 2 ** 24)) == np.float32(1.0)        # tie -> even
    assert rn32(Fraction(1) + Fraction(3, 2 ** 24)) == np.float32(1 + 2 ** -22)  # tie -> even (up)
    assert rn32(Fraction(-5, 7)) == np.float32(-5 / 7)


def test_counts_closed_form(orc):
    inp = W.micro_inputs(65536, 10)
    assert inp.n_renew == 21846
    r = orc.micro_run(inp)
    assert r.allocs == 65536 + 10 * 21846 == 283996
    assert r.frees == 10 * 21846 == 218460
    assert int(r.present.sum()) == 65536


def test_fma_single_rounding_exact(orc):
    inp = W.micro_inputs(3000, 10, seed=11)
    r = orc.micro_run(inp)
    k = Fraction(np.float32(0.01).item())
    for i in range(1, 3000, 7):
        if i % 3 == 0:
            continue
        x = Fraction(inp.x0[i].item())
        v = Fraction(inp.v0[i].item())
        for _ in range(10):
            x = Fraction(rn32(k * v + x).item())
        assert np.float32(float(x)).view(np.uint32) == r.x[i].view(np.uint32), i
        assert r.v[i] == inp.v0[i]


def test_renewed_ids_hold_last_inputs(orc):
    inp = W.micro_inputs(999, 4, seed=3)
    r = orc.micro_run(inp)
    # An id 3k is deleted and re-created every step after the update, so it
    # ends with the values of the last step's re-creation.
    for kk in range(inp.n_renew):
        assert r.x[3 * kk] == inp.xs[-1, kk] and r.v[3 * kk] == inp.vs[-1, kk]


def test_zero_velocity_keeps_x(orc):
    inp = W.micro_inputs(300, 5, seed=5)
    inp.v0[:] = 0
    r = orc.micro_run(inp)
    keep = np.arange(300) % 3 != 0
    assert np.array_equal(r.x[keep].view(np.uint32), inp.x0[keep].view(np.uint32))


def test_no_steps_is_identity(orc):
    inp = W.micro_inputs(500, 0, seed=9)
    r = orc.micro_run(inp)
    assert r.allocs == 500 and r.frees == 0
    assert np.array_equal(r.x, inp.x0) and np.array_equal(r.v, inp.v0)
