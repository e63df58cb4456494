"""Parity with many shards, where the grouping and query kernels change
strategy: more than 8 192 shards scatter keys with one atomic per key, more
than 16 384 count them with global atomics and the plain query reads local
seeds from global memory instead of LDS; the streamed build (keys in host
memory) takes the same branches.  Every shard's local seed, the failure
record and every cell are compared with the oracle, and so are all answers
to a mixed query batch."""
import os

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
DEV = "cuda:0"
_NP = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _compare(st, ob, b):
    info = st.info
    g = ob.geom
    assert (info["M"], info["l"], info["sigma"], info["V"], info["c_num"], info["c_den"]) == \
        (g["M"], g["l"], g["sigma"], g["V"], g["c_num"], g["c_den"])
    assert np.array_equal(st.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
    assert st.failures == ob.failures
    cells = st.cells().cpu().numpy().view(_NP[info["cell_bytes"]])
    assert np.array_equal(cells, ob.w.astype(cells.dtype))


@pytest.mark.parametrize("n,h", [(1 << 21, 14), (1 << 21, 15), (1 << 22, 16)])
def test_filter_with_many_shards_equals_the_oracle(n, h):
    b, seed = 8, 6
    print(f"[many] filter n={n} h={h}", flush=True)
    keys = S.member_keys(n, 400 + h, device=DEV)
    st = vf.Structure.build(keys, None, b=b, h=h, seed=seed)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK
    ob = O.build_threaded(keys.cpu().numpy().view(np.uint64), b=b, is_filter=True, h=h,
                          seed=seed, threads=_threads())
    _compare(st, ob, b)
    q, _ = S.queries(keys, 1 << 20, 17)
    want = O.query(ob, q.cpu().numpy().view(np.uint64))
    assert np.array_equal(st.query(q).cpu().numpy().astype(np.uint64), want)
    assert np.array_equal(st.query_grouped(q).cpu().numpy().astype(np.uint64), want)
    if h == 16:
        print("[many] streamed from host memory", flush=True)
        hk = keys.cpu().pin_memory()
        opts = vf.vf_default_opts(h=h)
        sz = vf.vf_plan(n, b, 0.0, True, opts)
        ws = torch.empty(sz.workspace_bytes + ((8 * n + 255) & ~255), dtype=torch.uint8,
                         device=DEV)
        stb = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=DEV)
        rc, hd = vf.vfilter_build_host(hk, b, 0.0, seed, opts, ws, stb, chunk=1 << 20)
        assert rc == vf.VF_OK
        torch.cuda.synchronize()
        sh = vf.Structure(hd, rc, True, b, stb, ws)
        _compare(sh, ob, b)
        assert np.array_equal(sh.query(q).cpu().numpy().astype(np.uint64), want)
        sh.free()
    st.free()


def test_function_with_many_shards_equals_the_oracle():
    n, h, b, seed = 1 << 21, 14, 16, 3
    print(f"[many] function n={n} h={h}", flush=True)
    keys = S.member_keys(n, 420, device=DEV)
    vals = S.values(n, b, 420, device=DEV)
    st = vf.Structure.build(keys, vals, b=b, h=h, seed=seed)
    torch.cuda.synchronize()
    assert st.rc == vf.VF_OK
    ob = O.build_threaded(keys.cpu().numpy().view(np.uint64), vals.cpu().numpy().view(np.uint64),
                          b=b, is_filter=False, h=h, seed=seed, threads=_threads())
    _compare(st, ob, b)
    got = st.query(keys).long() & 0xFFFF
    assert torch.equal(got, vals)
    q, _ = S.queries(keys, 1 << 20, 19)
    want = O.query(ob, q.cpu().numpy().view(np.uint64))
    assert np.array_equal(st.query(q).cpu().numpy().view(np.uint16).astype(np.uint64), want)
    st.free()
