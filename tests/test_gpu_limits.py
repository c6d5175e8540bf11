"""GPU parity at the limit of 4-byte offsets: about 2.0 GB of payload, just
under 2^31 bytes, with int32 row and payload offsets (the last payload
offsets come within 7% of 2^31), unaligned cell widths 0..62, 65 M cells,
plain and partitioned (R = 16). Every output array is compared in full."""
import pytest

from workloads import gen

from .common import assert_matches_oracle, gpu_transpose

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("partitioned", [False, True])
def test_int32_offsets_near_their_limit(partitioned):
    a = gen.random_small(21, n_rows=1 << 20, n_cols=1 << 20, deg_mean=62.0, w_lo=0, w_hi=62,
                         offset_width=4, parts=16)
    assert a.offset_width == 4 and 1.8 * 2 ** 30 < a.payload_bytes < 2 ** 31
    h, st = gpu_transpose(a, partitioned=partitioned, perm=True)
    assert st == 0
    assert_matches_oracle(a, h, partitioned=partitioned)
