"""lbmnet_conv3d_noalloc (workspace in the library's fixed device array)
against lbmnet_conv3d (workspace from the caller) through the C ABI: the
same kernels, so every output must be the same bits.  Two calls in a row, the
second on a smaller layer, so the second runs on what the first left in the
shared array."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _layer(torch, nn, dims, cin, cout, relu, seed, noalloc):
    n, d, h, w = dims
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.float32))).to(dev)
    xd = T(rng.normal(size=(n, d, h, w, cin)))
    wd = T(rng.normal(size=(cout, 27, cin)) / np.sqrt(27 * cin))
    bd = T(rng.normal(0, 0.1, cout))
    dyd = T(rng.normal(size=(n, d, h, w, cout)))
    out = (torch.full((n, d, h, w, cout), float("nan"), dtype=torch.float32, device=dev),
           torch.full_like(xd, float("nan")), torch.full_like(wd, float("nan")), torch.full_like(bd, float("nan")))
    st = torch.cuda.current_stream().cuda_stream
    if noalloc:
        nn.lbmnet_conv3d_noalloc(n, d, h, w, cin, cout, relu, xd, wd, bd, dyd, *out, st)
    else:
        ws = nn.lbmnet_conv3d_workspace(n, d, h, w, cin, cout)
        work = torch.empty(ws + 256, dtype=torch.uint8, device=dev)
        off = (-work.data_ptr()) % 256
        nn.lbmnet_conv3d(n, d, h, w, cin, cout, relu, xd, wd, bd, dyd, *out, work[off: off + ws], st)
    torch.cuda.synchronize()
    return [o.cpu() for o in out]


@pytest.mark.parametrize("first,second", [
    (((1, 16, 32, 64), 16, 16, 1), ((1, 4, 4, 32), 16, 16, 1)),       # brick kernels, then a smaller grid
    (((2, 8, 8, 32), 32, 32, 0), ((1, 3, 4, 16), 4, 16, 1)),          # then the general (non-brick) kernels
])
def test_noalloc_layer_equals_workspace_layer(first, second):
    import torch
    from paper_2101_11107_amd import net as nn
    for k, (dims, cin, cout, relu) in enumerate((first, second)):
        print(f"case noalloc call {k}: dims {dims} cin {cin} cout {cout} relu {relu}", flush=True)
        got = _layer(torch, nn, dims, cin, cout, relu, seed=17 + k, noalloc=True)
        ref = _layer(torch, nn, dims, cin, cout, relu, seed=17 + k, noalloc=False)
        for name, a, b in zip(("y", "dx", "dw", "db"), got, ref):
            assert torch.isfinite(b).all(), name
            assert torch.equal(a, b), name


def test_noalloc_forward_only_then_backward():
    """A forward-only call (dy NULL) and then a full call on the same array."""
    import torch
    from paper_2101_11107_amd import net as nn
    dev = torch.device("cuda:0")
    n, d, h, w, cin, cout = 1, 4, 8, 32, 16, 32
    rng = np.random.default_rng(5)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.float32))).to(dev)
    xd = T(rng.normal(size=(n, d, h, w, cin)))
    wd = T(rng.normal(size=(cout, 27, cin)) / np.sqrt(27 * cin))
    bd = T(rng.normal(0, 0.1, cout))
    y1 = torch.empty((n, d, h, w, cout), dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    print("case noalloc forward only", flush=True)
    nn.lbmnet_conv3d_noalloc(n, d, h, w, cin, cout, 1, xd, wd, bd, None, y1, None, None, None, st)
    torch.cuda.synchronize()
    ref = _layer(torch, nn, (n, d, h, w), cin, cout, 1, seed=5, noalloc=False)
    assert torch.equal(y1.cpu(), ref[0])
