"""Host-side identities the policy kernels rely on."""
import numpy as np


def test_depth_scaling_without_division():
    """The first convolution scales a 24-bit depth d to d / (2^24 - 1) in
    FP32 as the bits of d 2^-24 plus one unit in the last place (d >= 1):
    equal to the correctly rounded IEEE quotient for every d."""
    d = np.arange(0, 1 << 24, dtype=np.uint32)
    ieee = (d.astype(np.float32) / np.float32(16777215.0)).view(np.uint32)
    short = (d.astype(np.float32) * np.float32(2.0 ** -24)).view(np.uint32) + (d != 0).astype(np.uint32)
    assert np.array_equal(ieee, short)
