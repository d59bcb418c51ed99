"""pmor_stream_probe (the streaming-rate ceiling the bench reports beside the
Gram-Schmidt sweeps): argument checks, and a plausible rate (0.3 to 20 TB/s,
a loose bracket: the 8 TB/s HBM peak plus what the last-level cache may add)
for a read-only mix and mixes with one and two written blocks, over blocks of 64
MiB; out-of-range read and write counts are refused."""
import ctypes as C

import pytest

from tests._helpers import ctx as make_ctx

pytestmark = pytest.mark.gpu


def test_stream_probe(gpu_lib):
    from paper_1809_06574_amd import lib as L
    ctx = make_ctx()
    us = C.c_double()
    for nr, w in ((8, 0), (8, 1), (3, 2)):
        nbytes = 64 << 20
        assert L.pmor_stream_probe(ctx.handle, nr, w, nbytes, 3, C.byref(us)) == 0, L.pmor_last_error()
        gbs = (nr + w) * nbytes / (us.value * 1e-6) / 1e9
        assert 300.0 < gbs < 20000.0, (nr, w, gbs)
    for nr, w in ((0, 0), (-4, 0), (9, 0), (36, 0), (8, 3), (8, -1)):
        assert L.pmor_stream_probe(ctx.handle, nr, w, 1 << 20, 1, C.byref(us)) == L.PMOR_EINVAL, (nr, w)
    assert L.pmor_stream_probe(ctx.handle, 8, 0, 12, 1, C.byref(us)) == L.PMOR_EINVAL
    assert L.pmor_stream_probe(ctx.handle, 8, 0, 1 << 20, 0, C.byref(us)) == L.PMOR_EINVAL
