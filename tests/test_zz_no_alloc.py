"""The allocation-free network forward (sem_mlp_forward_noalloc) against sem_mlp_forward.

Both run the same kernels on the same rows, so the outputs must be equal bit for bit.  Two calls
in a row, the second with fewer rows and a smaller network (the array keeps the first call's
contents, which must not leak into the second), then the size limits.
"""
import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_14977_amd import binding as B  # noqa: E402


def net(nin, nout, seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(nin, nout, seed)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    return B.blob_pack(nin, nout, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])


def rows(n, nin, seed):
    X = np.random.default_rng(seed).standard_normal((n, nin))
    return torch.tensor(X, dtype=torch.float32, device="cuda")


def test_noalloc_forward_equals_forward_twice():
    print("[gpu] no-alloc forward: 405 -> 81 on 1000 rows, then 325 -> 65 on 37 rows", flush=True)
    for nin, nout, n, seed in ((405, 81, 1000, 1), (325, 65, 37, 2)):
        bl = net(nin, nout, seed)
        X = rows(n, nin, seed + 10)
        ref = B.sem_mlp_forward(bl, X, nout)
        got = B.sem_mlp_forward_noalloc(bl, X, nout)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), (nin, nout, n, float((got - ref).abs().max()))


def test_noalloc_forward_rejects_sizes_beyond_its_array():
    X = rows(16, 420, 3)
    with pytest.raises(B.SemError) as ei:
        B.sem_mlp_forward_noalloc(net(420, 81, 4), X, 81)
    assert ei.value.status == 1
    X = rows(16, 64, 5)
    with pytest.raises(B.SemError) as ei:
        B.sem_mlp_forward_noalloc(net(64, 100, 6), X, 100)
    assert ei.value.status == 1
    # a valid call still works after the rejected ones
    bl = net(64, 16, 7)
    assert torch.equal(B.sem_mlp_forward_noalloc(bl, X, 16), B.sem_mlp_forward(bl, X, 16))
