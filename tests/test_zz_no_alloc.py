"""The allocation-free ranking entry point against afd_threshold.

afd_threshold_noalloc keeps its work space in a static device array instead
of allocating one per call; it must give afd_threshold's results bit for bit
(integer and index outputs), on consecutive calls that reuse the array, the
second with a smaller input.
"""
import numpy as np
import pytest

from oracle import post
from paper_2203_15115_amd import afdcg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    prev = torch.cuda.current_stream()
    s = torch.cuda.Stream()
    torch.cuda.set_stream(s)
    c = afdcg.afd_context_create(0, s.cuda_stream)
    yield c
    afdcg.afd_context_destroy(c)
    torch.cuda.set_stream(prev)


def _field(n, seed):
    rng = np.random.default_rng(seed)
    s = rng.standard_normal(n) * 10 ** rng.uniform(-3, 3, n)
    s[rng.random(n) < 0.2] = 0.5   # ties
    s[rng.random(n) < 0.02] = -0.0
    s[rng.random(n) < 0.02] = 0.0
    return s, rng.integers(0, 40, n).astype(np.int32)


def _run(fn, ctx, s, tie, vf):
    n = s.size
    sd = torch.as_tensor(s).cuda()
    td = None if tie is None else torch.as_tensor(tie).cuda()
    solid = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    order = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    tau = fn(ctx, sd, n, vf, solid, order, tie=td)
    torch.cuda.synchronize()
    return solid.cpu().numpy(), order.cpu().numpy(), tau


@pytest.mark.parametrize("with_tie", [False, True])
def test_noalloc_threshold_equals_threshold(ctx, with_tie):
    # two calls in a row on the shared static work space: the full capacity,
    # then a smaller input (the second must not see the first's leftovers)
    for n, vf, seed in ((afdcg.AFD_THRESHOLD_NOALLOC_MAX, 0.4, 1), (100_003, 0.55, 2), (1, 1.0, 3)):
        s, tie = _field(n, seed)
        tie = tie if with_tie else None
        a = _run(afdcg.afd_threshold_noalloc, ctx, s, tie, vf)
        b = _run(afdcg.afd_threshold, ctx, s, tie, vf)
        assert np.array_equal(a[0], b[0]), n
        assert np.array_equal(a[1], b[1]), n
        assert a[2] == b[2], n
        if n <= 100_003:  # and the oracle
            want, tau = post.threshold(s, vf, tie)
            assert np.array_equal(a[0], want) and a[2] == tau


def test_noalloc_threshold_rejects_oversize(ctx):
    n = afdcg.AFD_THRESHOLD_NOALLOC_MAX + 1
    s = torch.zeros(n, dtype=torch.float64, device="cuda")
    solid = torch.empty(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(afdcg.AfdError) as ei:
        afdcg.afd_threshold_noalloc(ctx, s, n, 0.5, solid)
    assert ei.value.code == afdcg.AFD_E_INVALID_ARG
