"""CPU checks of arithmetic claims the kernels rely on (no GPU needed).

Intensity-adaptive P2: the aggregation forms floor(P2 / g) for the intensity
step g in 1..255 as the truncated FP32 product P2 * rcp(g), corrected by at
most one integer step either way.  The hardware reciprocal (v_rcp_f32) is
documented as accurate to 1 ULP, so every FP32 value within one unit of 1/g
is a possible result; the quotient must come out exact for each of them, for
every P2 the entry points accept (P2 <= 8000)."""
import numpy as np


def _candidates(g):
    """FP32 values within one unit in the last place of 1/g (a superset: the
    nearest FP32 value and both of its neighbours)."""
    r0 = np.float32(1.0) / np.float32(g)
    return [np.nextafter(r0, np.float32(0)), r0, np.nextafter(r0, np.float32(1))]


def test_adaptive_p2_quotient_exact_for_all_steps():
    P2 = np.arange(0, 8001, dtype=np.int64)
    fP2 = P2.astype(np.float32)
    for g in range(1, 256):
        want = P2 // g
        for r in _candidates(g):
            prod = (fP2 * np.float32(r)).astype(np.float32)  # one FP32 product, rounded to nearest
            q = np.trunc(prod).astype(np.int64)              # conversion truncates toward zero
            rem = P2 - q * g
            q = q + (rem >= g) - (rem < 0)
            bad = np.flatnonzero(q != want)
            assert bad.size == 0, (g, float(r), int(P2[bad[0]]))


def test_adaptive_p2_needs_the_correction():
    """Without the correction step the truncated product is wrong somewhere
    (so the test above exercises it)."""
    P2 = np.arange(0, 8001, dtype=np.int64)
    fP2 = P2.astype(np.float32)
    wrong = 0
    for g in range(1, 256):
        for r in _candidates(g):
            q = np.trunc((fP2 * np.float32(r)).astype(np.float32)).astype(np.int64)
            wrong += int((q != P2 // g).sum())
    assert wrong > 0
