"""GPU parity at RMAT scale 26 (edge factor 16, seed 1: 2^30 raw pairs, the
shape of the paper's g500-s26 input, Table "datasets") against values the
CPU oracle wrote once (tests/golden/rmat26_seed1.json, made by
tests/golden/make_rmat_fixture.py; about 20 minutes of oracle time, too long
to run inside a test). Compared: sizes and work counts, T, SHA-256 digests
of the exported CSR and rank map, and rank (0, 0) and the busiest rank of
the 13 x 13 grid (count and per-shift counts); all 169 ranks sum to T."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat26_seed1.json")


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1907_09575_amd as tc
    torch.cuda.set_device(0)
    return tc


def _sha(t, dtype):
    return hashlib.sha256(np.ascontiguousarray(t.cpu().numpy(), dtype=dtype).tobytes()).hexdigest()


def test_rmat_scale26_against_stored_oracle_values(tc):
    with open(FIXTURE) as f:
        want = json.load(f)
    scale = want["scale"]
    n = 1 << scale
    print("generating RMAT scale %d ..." % scale, flush=True)
    s, d = graphgen.rmat(scale, edge_factor=want["edge_factor"], seed=want["seed"], threads=16)
    assert len(s) == want["m_raw"]
    src = torch.from_numpy(s).to("cuda")
    dst = torch.from_numpy(d).to("cuda")
    del s, d
    print("preprocessing ...", flush=True)
    g = tc.tc_preprocess(src, dst, n)
    del src, dst
    info = g.info()
    for k in ("m", "wedges_plus", "probes", "tasks", "max_out_degree"):
        assert info[k] == want[k], k
    T = int(tc.tc_count(g).item())
    assert T == want["triangles"]
    print("T equal; exporting CSR ...", flush=True)
    rp, col, perm = tc.tc_graph_export(g)
    torch.cuda.synchronize()
    assert _sha(perm, "<i4") == want["sha256_rank_i32le"]
    assert _sha(rp, "<i8") == want["sha256_row_ptr_i64le"]
    del rp, perm
    assert _sha(col, "<i4") == want["sha256_col_i32le"]
    del col
    torch.cuda.empty_cache()
    q = want["grid_q"]
    ps = torch.empty(q, dtype=torch.int64, device="cuda")
    for blk in want["blocks"]:
        print("block (%d, %d) of %d x %d" % (blk["x"], blk["y"], q, q), flush=True)
        cnt, _ = tc.tc_block_count(g, q, blk["x"], blk["y"], per_shift=ps)
        torch.cuda.synchronize()
        assert int(cnt.item()) == blk["count"]
        assert ps.cpu().tolist() == blk["per_shift"]
    print("all %d ranks ..." % (q * q), flush=True)
    total = 0
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    for x in range(q):
        for y in range(q):
            tc.tc_block_count(g, q, x, y, cnt, ps)
            torch.cuda.synchronize()
            b = int(cnt.item())
            assert int(ps.sum().item()) == b
            total += b
    assert total == T
    g.free()
