"""Host checks of arithmetic identities the kernels rely on (no GPU): the small-operand division
through the FP32 hardware reciprocal (floor((a + 1/2) * rcp(b)) == a // b for a < 2^16, b <= 128,
with the reciprocal anywhere within 1 ulp of 1/b, as the hardware instruction guarantees)."""
import numpy as np


def test_small_division_through_fp32_reciprocal():
    a = np.arange(0, 1 << 16, dtype=np.int64)
    af = a.astype(np.float32) + np.float32(0.5)
    for b in range(1, 129):
        r = np.float32(1.0) / np.float32(b)
        for rb in (np.nextafter(r, np.float32(0)), r, np.nextafter(r, np.float32(np.inf))):
            q = (af * rb).astype(np.int64)  # FP32 product, then truncation toward zero
            np.testing.assert_array_equal(q, a // b)
