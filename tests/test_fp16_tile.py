"""The reading behind the fp16 observation tile of the CLUSTERED 48-byte form:
for a threshold t that is exact in fp16, x <= t in fp32 holds exactly when
x rounded toward +infinity to fp16 is <= t.  Checked here with numpy's own
fp16 conversion (round to nearest even) and a step up where that fell below
x, over every finite fp16 threshold and adversarial fp32 values around each;
the kernel's GPU tests check the same votes through the C ABI."""
import numpy as np
import pytest

# nextafter beyond the largest fp16 overflows to infinity, as intended
pytestmark = pytest.mark.filterwarnings("ignore:overflow encountered")


def half_up(x: np.ndarray) -> np.ndarray:
    """fp32 -> fp16, rounding toward +infinity (NaN stays NaN)."""
    x = np.asarray(x, np.float32)
    with np.errstate(over="ignore"):
        h = x.astype(np.float16)
    low = h.astype(np.float32) < x
    b = h.view(np.uint16).astype(np.int32)
    neg = (b & 0x8000) != 0
    b = np.where(low & ~neg, b + 1, b)
    b = np.where(low & neg & (b == 0x8000), 1, b)
    b = np.where(low & neg & (b != 0x8000) & (b != 1), b - 1, b)
    return b.astype(np.uint16).view(np.float16)


def fp16_values(finite_only=True):
    v = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16).view(np.float16)
    return v[np.isfinite(v)] if finite_only else v[~np.isnan(v)]


def probes_around(t: np.ndarray) -> np.ndarray:
    """fp32 values on, just beside, and halfway between fp16 neighbours of t."""
    t32 = t.astype(np.float32)
    up = np.nextafter(t, np.float16(np.inf)).astype(np.float32)
    dn = np.nextafter(t, np.float16(-np.inf)).astype(np.float32)
    mid_up = ((t32.astype(np.float64) + up.astype(np.float64)) / 2).astype(np.float32)
    mid_dn = ((t32.astype(np.float64) + dn.astype(np.float64)) / 2).astype(np.float32)
    out = [t32, up, dn, mid_up, mid_dn]
    for v in (t32, mid_up, mid_dn):
        out += [np.nextafter(v, np.float32(np.inf)), np.nextafter(v, np.float32(-np.inf))]
    return np.concatenate(out)


def test_half_up_is_the_smallest_fp16_at_or_above():
    rng = np.random.default_rng(0)
    x = np.concatenate([probes_around(fp16_values()),
                        rng.standard_normal(20000).astype(np.float32) * np.float32(3e4),
                        np.array([65504.5, 65519.99, 65520, 7e4, 3e38, -65504.5, -65519.99, -65520, -7e4, -3e38,
                                  1e-40, -1e-40, 2.0 ** -25, -2.0 ** -25, 3 * 2.0 ** -26, 0.0, -0.0,
                                  np.inf, -np.inf], np.float32)])
    x = x[np.isfinite(x) | np.isinf(x)]
    h = half_up(x).astype(np.float32)
    assert (h >= x).all()
    # no fp16 value lies in [x, h): the step below h is below x
    below = np.nextafter(half_up(x), np.float16(-np.inf)).astype(np.float32)
    fin = np.isfinite(h) | (h == np.inf)
    assert (below[fin & (h > x)] < x[fin & (h > x)]).all()
    assert np.isnan(half_up(np.array([np.nan], np.float32))).all()


def test_compare_is_exact_for_every_fp16_threshold():
    ts = fp16_values()
    rng = np.random.default_rng(1)
    x = np.concatenate([probes_around(ts), np.array([np.nan, np.inf, -np.inf, 1e-40, -1e-40, 0.0, -0.0, 7e4, -7e4],
                                                     np.float32)])
    hx = half_up(x)
    # every threshold against the probes of a random sample of its neighbours'
    # probes, and every probe against a random sample of thresholds
    for t in np.concatenate([ts[rng.integers(0, ts.size, 400)],
                             np.array([0.0, -0.0, 65504, -65504, 2.0 ** -24, -(2.0 ** -24), 2.0 ** -14, 1.0, 2048,
                                       2049, 0.5, 1000.5], np.float16)]):
        assert np.array_equal(x <= np.float32(t), hx <= t), t
    for t in ts[::97]:
        near = probes_around(np.array([t], np.float16))
        assert np.array_equal(near <= np.float32(t), half_up(near) <= t), t
    assert np.array_equal(np.float32(np.nan) <= np.float32(1.0), half_up(np.float32(np.nan)) <= np.float16(1.0))
