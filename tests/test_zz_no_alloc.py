"""GPU test of tc_count_batched_noalloc (the batched count that allocates no
device memory): through the C ABI its per-graph counts equal those of
tc_count_batched on the same handles, on two calls in a row - the second on
a smaller batch, which must not see anything the first left in the shared
scratch array - and the library's device allocator does not move."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle
import smallgraphs as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1907_09575_amd as tc
    torch.cuda.set_device(0)
    return tc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")


def _lists(count, seed0, max_log2n):
    specs = graphgen.batch_specs(count, seed=seed0)
    out = []
    for sp in specs:
        if sp.n > (1 << max_log2n):
            continue
        s, d = graphgen.generate_many([sp], 1)[0]
        out.append((s, d, sp.n))
    return out


def _c_abi_noalloc(tc, graphs, counts):
    arr = (ctypes.c_void_p * max(len(graphs), 1))()
    for i, g in enumerate(graphs):
        arr[i] = g.handle.value
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = tc._lib.tc_count_batched_noalloc(arr, len(graphs), ctypes.c_void_p(counts.data_ptr()), stream)
    assert st == 0, tc._lib.tc_last_error().decode()


def test_noalloc_equals_count_batched_twice(tc):
    big = _lists(96, 11, 15) + [sg.complete(40), sg.wheel(300), sg.star(30)]
    small = _lists(24, 77, 11)[:9] + [sg.cycle(3)]
    for lists in (big, small):
        print("noalloc case: %d graphs, %d raw pairs" % (len(lists), sum(len(s) for s, _, _ in lists)),
              flush=True)
        graphs = [tc.tc_preprocess(dev(s), dev(d), n) for s, d, n in lists]
        want = tc.tc_count_batched(graphs)
        torch.cuda.synchronize()
        want = want.cpu().numpy()
        # spot values against the oracle
        for i in (0, len(lists) - 1):
            s, d, n = lists[i]
            assert want[i] == oracle.count(oracle.preprocess(s, d, n))
        got = torch.full((len(graphs),), -7, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        stats0 = tc.tc_memory_stats()
        torch_mem0 = torch.cuda.memory_allocated()
        _c_abi_noalloc(tc, graphs, got)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want)
        stats1 = tc.tc_memory_stats()
        assert stats1["in_use"] == stats0["in_use"] and stats1["cached"] == stats0["cached"]
        assert stats1["peak"] == stats0["peak"]
        assert torch.cuda.memory_allocated() == torch_mem0
        for g in graphs:
            g.free()


def test_noalloc_empty_and_errors(tc):
    got = torch.zeros(1, dtype=torch.int64, device="cuda")
    arr = (ctypes.c_void_p * 1)()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert tc._lib.tc_count_batched_noalloc(arr, 0, None, stream) == 0
    assert tc._lib.tc_count_batched_noalloc(arr, -1, ctypes.c_void_p(got.data_ptr()), stream) == 1
    assert tc._lib.tc_count_batched_noalloc(None, 3, ctypes.c_void_p(got.data_ptr()), stream) == 1
