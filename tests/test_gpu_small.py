"""The one-wavefront kernel for small batch instances (at most 128 keys and
256 cells, the whole instance on chip) against the oracle, instance by
instance, and against the peel + band kernel; and the tuning that chooses
between them per size class."""
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


def _batch(count, seed):
    rng = np.random.default_rng(seed)
    n = np.floor(np.exp(rng.uniform(0, np.log(200), count))).astype(np.uint64)
    n[:12] = [0, 1, 2, 3, 15, 16, 17, 63, 64, 127, 128, 129]
    b = rng.choice(np.array([1, 4, 8, 16, 32, 64], np.int32), count).astype(np.int32)
    total = int(n.sum())
    keys = S.member_keys(total, 800 + seed, device=DEV)
    vals = S.batch_values(n, b, 800 + seed, device=DEV)
    return n, b, keys, vals


def _check_all(bt, n, b, keys, vals, seed, tmax=255):
    k_np = keys.cpu().numpy().view(np.uint64)
    v_np = vals.cpu().numpy().view(np.uint64)
    off = np.concatenate([[0], np.cumsum(n.astype(np.int64))])
    fails = bt.failures
    byinst = {}
    for f in fails:
        byinst.setdefault(f[0], []).append(f[1:])
    for i in range(n.size):
        lo, hi = int(off[i]), int(off[i + 1])
        ob = O.build(k_np[lo:hi], v_np[lo:hi], b=int(b[i]), is_filter=False, h=0, seed=seed,
                     tmax=tmax)
        it = bt.item(i)
        t = int(ob.t[0]) if ob.status == 0 else 255
        assert it["local_seed"] == t, i
        assert byinst.get(i, []) == [f[1:] for f in ob.failures], i
        cells = bt.cells(i).cpu().numpy().view(_NP[it["cell_bytes"]])
        want = ob.w[0] if ob.status == 0 else np.zeros(it["V"], np.uint64)
        assert np.array_equal(cells, want.astype(cells.dtype)), i


def test_small_kernel_equals_the_oracle_on_every_instance():
    n, b, keys, vals = _batch(3000, 1)
    print(f"[small] {n.size} instances, {int(n.sum())} keys", flush=True)
    bt = vf.Batch.build(keys, vals, n, b, seed=3, small=1)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_OK
    _check_all(bt, n, b, keys, vals, 3)
    inst = torch.repeat_interleave(torch.arange(n.size, dtype=torch.int32, device=DEV),
                                   torch.as_tensor(n.astype(np.int64), device=DEV))
    assert torch.equal(bt.query(inst, keys), vals)
    # the peel + band kernel builds the same cells
    bb = vf.Batch.build(keys, vals, n, b, seed=3, small=2)
    torch.cuda.synchronize()
    assert bb.rc == vf.VF_OK
    for i in range(n.size):
        assert torch.equal(bt.cells(i), bb.cells(i)), i
        assert bt.item(i)["local_seed"] == bb.item(i)["local_seed"], i
    assert bt.failures == bb.failures
    bt.free()
    bb.free()


def test_small_kernel_failing_instance_and_retries():
    """A key given twice with different values fails every local seed: the
    instance's cells stay zero, its seed is 255 and each attempt is
    recorded; the other instances are unaffected."""
    base = S.member_keys(90, 880, device=DEV)
    keys = torch.cat([base[:40], base[:1], base[40:90]])
    vals = S.values(91, 8, 880, device=DEV)
    vals[40] = (vals[0] + 1) & 0xFF
    n = np.array([41, 50], np.uint64)
    b = np.array([8, 8], np.int32)
    opts_tmax = 4
    bt = vf.Batch.build(keys, vals, n, b, seed=1, small=1, tmax=opts_tmax)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_EFAIL
    assert bt.item(0)["local_seed"] == 255
    assert [f[:3] for f in bt.failures if f[0] == 0] == [(0, t, 1) for t in range(opts_tmax)]
    assert int(bt.cells(0).abs().sum()) == 0
    _check_all(bt, n, b, keys, vals, 1, tmax=opts_tmax)
    bt.free()


def test_tuning_chooses_a_kernel_per_size_class():
    n, b, keys, vals = _batch(6000, 2)
    bt = vf.Batch.build(keys, vals, n, b, seed=5)
    torch.cuda.synchronize()
    assert bt.rc == vf.VF_OK
    t = vf.vf_batch_tuning()
    print("[small] tuning", t, flush=True)
    assert t["tuned"] == 1 and t["max_keys"] == [16, 32, 64, 128]
    assert t["small_groups_per_cu"] in (2, 4, 8, 16)
    for c in range(4):
        if t["sampled"][c] >= 256:
            assert t["ms_small"][c] > 0 and t["ms_band"][c] > 0
            assert t["use_small"][c] == int(t["ms_small"][c] <= t["ms_band"][c])
    # whatever was chosen, the cells equal the oracle's
    _check_all(bt, n[:400], b[:400], keys, vals, 5)
    bt.free()
