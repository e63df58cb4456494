"""The serving loop on the GPU: a Poisson stream of builds and query
batches served with several slots gives, for every request, exactly the
bytes the same request gives alone (structures are canonical), and a sample
of the served builds and of the query batches against them equals the
oracle."""
import time

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2503_18397_amd as vf
    from paper_2503_18397_amd.serve import Request, Server, poisson_trace
DEV = "cuda:0"


def _inputs(ev):
    data = {}
    for e in ev:
        if e["kind"] != "query":
            keys = S.member_keys(e["n"], 300 + e["id"], device=DEV)
            vals = S.values(e["n"], e["b"], 300 + e["id"], device=DEV)
            data[e["id"]] = (keys, vals)
    for j, e in enumerate(ev):
        if e["kind"] == "query":
            keys = data[e["target"]][0]
            q, _ = S.queries(keys, e["n"], 700 + j, member_share_per_256=230)
            e["keys"] = q
    return data


def test_each_result_is_the_same_alone_and_in_the_mix():
    ev = poisson_trace(5, builds=10, queries=30, build_rate=300.0, query_rate=1500.0,
                       n_lo=1000, n_hi=300000, q_lo=1, q_hi=50000)
    data = _inputs(ev)
    # alone: one request at a time, no server
    alone = {}
    for e in ev:
        if e["kind"] == "query":
            continue
        k, v = data[e["id"]]
        st = vf.Structure.build(k, None if e["kind"] == "vfilter" else v, b=e["b"], eps=0.0175)
        torch.cuda.synchronize()
        assert st.rc == vf.VF_OK
        alone[e["id"]] = st
    want_q = [alone[e["target"]].query(e["keys"]).cpu() for e in ev if e["kind"] == "query"]
    # in the mix: arrivals in real time, four slots
    srv = Server(slots=4)
    reqs, t0 = [], time.perf_counter()
    for j, e in enumerate(ev):
        while time.perf_counter() - t0 < e["t"]:
            time.sleep(0.0002)
        if e["kind"] == "query":
            r = Request(10000 + j, "query", e["keys"], target=e["target"])
        else:
            k, v = data[e["id"]]
            r = Request(e["id"], e["kind"], k, v, b=e["b"], eps=0.0175)
        srv.submit(r)
        reqs.append(r)
    st = srv.drain(timeout=120)
    srv.close()
    summ = st.summary()
    print("[serve]", summ, flush=True)
    assert summ["errors"] == 0
    got_q = [r.result.cpu() for r in reqs if r.kind == "query"]
    for a, b_ in zip(want_q, got_q):
        assert torch.equal(a, b_)
    for r in reqs:
        if r.kind != "query":
            a, b_ = alone[r.rid], r.result
            assert torch.equal(a.cells(), b_.cells())
            assert torch.equal(a.local_seeds(), b_.local_seeds())
            assert a.failures == b_.failures
    # the oracle on the three smallest served builds and every query batch
    # against them
    builds = sorted((r for r in reqs if r.kind != "query"), key=lambda r: r.keys.numel())[:3]
    np_of = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}
    for r in builds:
        res = r.result
        info = res.info
        k_np = r.keys.cpu().numpy().view(np.uint64)
        is_f = r.kind == "vfilter"
        v_np = None if is_f else r.values.cpu().numpy().view(np.uint64)
        print(f"[serve] oracle on build {r.rid}: n={k_np.size} b={info['b']} h={info['h']}",
              flush=True)
        ob = O.build(k_np, v_np, b=info["b"], is_filter=is_f, h=info["h"], seed=0)
        assert np.array_equal(res.local_seeds().cpu().numpy(), ob.t.astype(np.uint8))
        assert res.failures == ob.failures
        cells = res.cells().cpu().numpy().view(np_of[info["cell_bytes"]])
        assert np.array_equal(cells, ob.w.astype(cells.dtype))
        for q in reqs:
            if q.kind == "query" and q.target == r.rid:
                want = O.query(ob, q.keys.cpu().numpy().view(np.uint64))
                got = q.result.cpu().numpy()
                got = got.view(np_of[got.itemsize]) if not is_f else got
                assert np.array_equal(got.astype(np.uint64), want)
