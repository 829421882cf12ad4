"""The rounding reference of the codec tests on hand-made ties and near-ties
(values worked out by hand from the formats' spacings)."""
import numpy as np

from codec_ref import rne


def test_bf16_ties_to_even():
    u = 2.0 ** -7                            # BF16 spacing in [1, 2)
    x = [1 + u / 2, 1 + 3 * u / 2, 1 + u / 2 + 2.0 ** -40, -(1 + u / 2), 3 * 2.0 ** -130 * (1 + u / 2)]
    want = [1.0, 1 + 2 * u, 1 + u, -1.0, 3 * 2.0 ** -130]
    np.testing.assert_array_equal(rne(x, "bf16"), want)


def test_f16_ties_and_subnormals():
    u = 2.0 ** -10                           # FP16 spacing in [1, 2)
    s = 2.0 ** -24                           # FP16 subnormal spacing
    x = [1 + u / 2, 1 + 3 * u / 2, 1 + u / 2 + 2.0 ** -30, 0.5 * s, 1.5 * s, 0.75 * s, 0.375 * s]
    want = [1.0, 1 + 2 * u, 1 + u, 0.0, 2 * s, s, 0.0]
    np.testing.assert_array_equal(rne(x, "f16"), want)


def test_f32_tie():
    u = 2.0 ** -23
    np.testing.assert_array_equal(rne([1 + u / 2, 1 + 3 * u / 2], "f32"), [1.0, 1 + 2 * u])
