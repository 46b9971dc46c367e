"""The backward pass that allocates nothing (library-owned scratch) against the
workspace form, through the C ABI: two calls in a row, the second smaller."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _case(n, seed):
    from paper_2111_05205_amd import _native as N
    from paper_2111_05205_amd import mlp
    g = torch.Generator().manual_seed(seed)
    params = (torch.randn(mlp.NPARAM, generator=g) * 0.05).cuda()
    feat = torch.randn(n, mlp.IN_PAD, generator=g).cuda()
    feat[:, N.MLP_IN:] = 0.0
    dy = torch.randn(n, generator=g).cuda()
    _, act = mlp.forward(params, feat, act=True)
    return params, feat, act, dy


def test_noalloc_backward_equals_workspace_backward():
    from paper_2111_05205_amd import mlp
    for n, seed in ((4096, 1), (777, 2)):
        print(f"no-alloc backward: n={n} seed={seed}", flush=True)
        params, feat, act, dy = _case(n, seed)
        want = mlp.backward(params, feat, act, dy)
        got = mlp.backward_noalloc(params, feat, act, dy)
        torch.cuda.synchronize()
        assert torch.isfinite(want).all()
        assert torch.equal(got, want), (got - want).abs().max().item()


def test_noalloc_backward_rejects_oversized_input():
    from paper_2111_05205_amd import _native as N
    from paper_2111_05205_amd import mlp
    n = N.MLP_NOALLOC_MAX_ROWS + 1
    params, feat, act, dy = _case(n, 3)
    with pytest.raises(Exception, match="exceeds the maximum"):
        mlp.backward_noalloc(params, feat, act, dy)
