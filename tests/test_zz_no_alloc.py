"""lbm_fields_noalloc (static staging, no device allocation) gives the same
fields as lbm_fields, through the C ABI, on two calls in a row: a lattice
staged in three row chunks (the last one ragged), then a smaller one."""
import sys

import numpy as np
import pytest

from paper_1803_09380_amd import lbmib
from paper_1803_09380_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _sim(nx, ny, precision, seed):
    s = lbmib.Sim(nx, ny, 0.8, precision=precision, bc=(lbmib.WALL, lbmib.WALL, lbmib.PERIODIC, lbmib.PERIODIC))
    s.set_fields(*wl.random_fields(seed, nx, ny))
    s.step(3)
    return s


@pytest.mark.parametrize("precision", [lbmib.F64, lbmib.F32_SHIFTED])
def test_fields_noalloc_equal_fields(precision):
    for nx, ny, seed in ((1000, 700, 1), (96, 40, 2)):
        print("fields_noalloc %dx%d precision %d" % (nx, ny, precision), flush=True)
        sys.stdout.flush()
        s = _sim(nx, ny, precision, seed)
        ref = s.fields()
        got = s.fields_noalloc()
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        s.close()


def test_fields_noalloc_rejects_rows_beyond_the_staging_buffer():
    s = lbmib.Sim(349526, 4, 0.8, precision=lbmib.F32_SHIFTED)
    with pytest.raises(lbmib.LbmError) as e:
        s.fields_noalloc()
    assert e.value.code == lbmib.ERR_INVALID
    s.close()
