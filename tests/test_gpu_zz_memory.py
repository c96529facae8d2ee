"""Device out-of-memory inside the library (collected last: it fills the card).

With the library's cache released and nearly all free device memory held by
the caller, tc_preprocess of an RMAT scale-20 graph must fail with
TC_ENOMEM (status 2) and leave the library usable: once the memory is given
back, the same call succeeds and counts exactly.
"""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1907_09575_amd as tc
    torch.cuda.set_device(0)
    return tc


def test_out_of_memory_is_an_error_and_recoverable(tc):
    s, d = graphgen.rmat(20, seed=3)
    n = 1 << 20
    src = torch.from_numpy(s).cuda()
    dst = torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    tc.tc_release_cached_memory()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    # leave 256 MiB: far less than the ~1.5 GB the scale-20 preprocessing needs
    hold = torch.empty(max(free - (256 << 20), 0), dtype=torch.uint8, device="cuda")
    print("holding %.1f GiB of %.1f GiB free" % (hold.numel() / 2 ** 30, free / 2 ** 30), flush=True)
    try:
        with pytest.raises(tc.TCError) as e:
            tc.tc_preprocess(src, dst, n)
        assert e.value.status == 2, str(e.value)
    finally:
        del hold
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    g = tc.tc_preprocess(src, dst, n)
    got = int(tc.tc_count(g).item())
    g.free()
    assert got == oracle.count(oracle.preprocess(s, d, n))
