"""Device out-of-memory inside the library (collected last: it fills the card).

With the library's kernels loaded, its cache released and the card filled
by the caller down to 256 MiB, tc_preprocess of an RMAT scale-20 graph must
fail with TC_ENOMEM (status 2) and leave the library usable: once the memory
is given back, the same call succeeds and counts exactly.
"""
import gc

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


def _fill_device(keep_bytes):
    """Allocate device memory until the allocator refuses (down to 16 MiB
    pieces), then give back keep_bytes: what is left free is keep_bytes plus
    less than 16 MiB, whatever the runtime reports as free."""
    spare = torch.empty(keep_bytes, dtype=torch.uint8, device="cuda")
    held = []
    size = 1 << 30
    while size >= (16 << 20):
        try:
            held.append(torch.empty(size, dtype=torch.uint8, device="cuda"))
        except torch.OutOfMemoryError:
            size //= 2
    del spare
    torch.cuda.empty_cache()
    return held


def test_out_of_memory_is_an_error_and_recoverable(tc):
    s, d = graphgen.rmat(20, seed=3)
    n = 1 << 20
    src = torch.from_numpy(s).cuda()
    dst = torch.from_numpy(d).cuda()
    # the library's kernels are loaded (a first launch loads a code object
    # into device memory) before the card is filled
    ws, wd = graphgen.rmat(8, seed=1)
    w = tc.tc_preprocess(torch.from_numpy(ws).cuda(), torch.from_numpy(wd).cuda(), 1 << 8)
    tc.tc_count(w)
    w.free()
    torch.cuda.synchronize()
    # graphs, plans or servers of earlier tests that are only garbage now are
    # freed first (into the library's cache, released next), so that no block
    # of theirs can come back and serve this call from the cache
    gc.collect()
    tc.tc_release_cached_memory()
    torch.cuda.empty_cache()
    stats = tc.tc_memory_stats()
    assert stats["cached"] == 0, stats
    # leave 256 MiB: far less than the scale-20 preprocessing needs (its two
    # key buffers alone take 256 MiB)
    held = _fill_device(256 << 20)
    print("holding %.1f GiB; library: %s" % (sum(h.numel() for h in held) / 2 ** 30, stats), flush=True)
    try:
        with pytest.raises(tc.TCError) as e:
            tc.tc_preprocess(src, dst, n)
        assert e.value.status == 2, str(e.value)
    finally:
        del held
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    g = tc.tc_preprocess(src, dst, n)
    got = int(tc.tc_count(g).item())
    g.free()
    assert got == oracle.count(oracle.preprocess(s, d, n))
