"""Host-side checks of the batch API (no GPU): buffer planning follows the
size rule for every instance, bad arguments are rejected, and the batch
shape generator draws what it says."""
import math

import numpy as np
import pytest

import oracle as O
import synthetic as S

vf = pytest.importorskip("paper_2503_18397_amd")


def test_batch_plan_covers_every_instance():
    n = np.array([0, 1, 10, 777, 5000, 49999], dtype=np.uint64)
    b = np.array([1, 4, 8, 16, 32, 64], dtype=np.int32)
    sz = vf.vf_batch_plan(n, b)
    cells = 0
    for ni, bi in zip(n.tolist(), b.tolist()):
        g = O.geometry(ni, 0)
        cb = 1 if bi <= 8 else 2 if bi <= 16 else 4 if bi <= 32 else 8
        cells += (g["V"] * cb + 7) // 8 * 8
    # descriptors (64 B each) + local seeds + cells, each 256-aligned
    want = sum((x + 255) // 256 * 256 for x in (64 * n.size, n.size, cells))
    assert sz.structure_bytes == want
    assert sz.shard_cap == 49999 and sz.h == 0
    assert sz.workspace_bytes > 0


@pytest.mark.parametrize("n,b", [([], []), ([5], [0]), ([5], [65]), ([5, 6], [8])])
def test_batch_plan_rejects_bad_arguments(n, b):
    with pytest.raises((vf.VFError, ValueError)):
        vf.vf_batch_plan(n, b)


def test_batch_shape_is_log_uniform():
    n, b = S.batch_shape(20000, 3)
    assert n.min() >= 10 and n.max() <= 50000
    assert set(b.tolist()) == {1, 4, 8, 16, 32}
    # log-uniform: ln n uniform on [ln 10, ln 50000]; its mean and the share
    # below the geometric midpoint are checked within 5 sigma
    ln = np.log(n.astype(np.float64) + 0.5)
    a, c = math.log(10), math.log(50000)
    sd = (c - a) / math.sqrt(12) / math.sqrt(n.size)
    assert abs(ln.mean() - (a + c) / 2) < 5 * sd + 0.01
    below = (n < math.sqrt(10 * 50000)).mean()
    assert abs(below - 0.5) < 5 * math.sqrt(0.25 / n.size)
    # the mean size matches the log-uniform mean (hi - lo) / ln(hi / lo)
    assert abs(n.mean() / ((50000 - 10) / math.log(5000)) - 1) < 0.05


def test_synthetic_query_chunks_match_the_whole_stream():
    import torch
    keys = S.member_keys(1000, 9)
    q, m = S.queries(keys, 5000, 9)
    q2, m2 = S.queries_chunk(1000, 1200, 2000, 9)
    assert torch.equal(q[1200:3200], q2) and torch.equal(m[1200:3200], m2)


def test_member_index_scaling_is_exact_up_to_2_32_keys():
    import torch
    rng = np.random.default_rng(5)
    u = rng.integers(0, 2 ** 32, 4000, dtype=np.int64)
    for n in (1, 1000, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32):
        got = S._scale(torch.as_tensor(u), n).numpy()
        want = np.array([(int(x) * n) >> 32 for x in u], dtype=np.int64)
        assert np.array_equal(got, want), n
