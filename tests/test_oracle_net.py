"""Pins of the corrector oracle (tier O3) against library routines, adjoint
identities, closed forms and finite differences."""

import numpy as np
import pytest
import scipy.ndimage

from oracle import o3_net as o3


def _rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def test_conv3d_matches_scipy_correlate():
    """The convolution is a zero-padded 3x3x3 cross-correlation summed over input
    channels: scipy.ndimage.correlate per channel pair."""
    x = _rand((5, 6, 7, 3), 0)
    w = _rand((4, 27, 3), 1)
    b = _rand((4,), 2)
    y = o3.conv3d(x, w, b)
    for co in range(4):
        ref = np.full(x.shape[:3], b[co])
        for ci in range(3):
            ref += scipy.ndimage.correlate(x[..., ci], w[co, :, ci].reshape(3, 3, 3), mode="constant", cval=0.0)
        assert np.max(np.abs(y[..., co] - ref)) < 1e-12


def _fd(f, arr, idx, h=1e-6):
    old = arr[idx]
    arr[idx] = old + h
    fp = f()
    arr[idx] = old - h
    fm = f()
    arr[idx] = old
    return (fp - fm) / (2 * h)


def test_conv3d_backward_finite_differences():
    x = _rand((4, 5, 3, 3), 3)
    w = _rand((2, 27, 3), 4)
    b = _rand((2,), 5)
    g = _rand((4, 5, 3, 2), 6)
    loss = lambda: float((o3.conv3d(x, w, b) * g).sum())
    dx, dw, db = o3.conv3d_backward(x, w, g)
    rng = np.random.default_rng(7)
    for _ in range(6):
        i = tuple(rng.integers(0, s) for s in x.shape)
        assert abs(_fd(loss, x, i) - dx[i]) < 1e-6
        j = tuple(rng.integers(0, s) for s in w.shape)
        assert abs(_fd(loss, w, j) - dw[j]) < 1e-6
    assert abs(_fd(loss, b, (1,)) - db[1]) < 1e-6


def test_pool_and_upsample_adjoints():
    x = _rand((4, 6, 2, 3), 8)
    y = _rand((2, 3, 1, 3), 9)
    assert abs((o3.avgpool2(x) * y).sum() - (x * o3.avgpool2_backward(y)).sum()) < 1e-12
    assert abs((o3.upsample2(y) * x).sum() - (y * o3.upsample2_backward(x)).sum()) < 1e-12
    assert np.allclose(o3.avgpool2(o3.upsample2(y)), y)


def test_trilinear_reproduces_linear_fields():
    """Fine node 2i sits on coarse node i: a linear coarse field is reproduced
    exactly at every fine node whose interpolation stays inside the box."""
    d = np.arange(5.0)
    z, yy, xx = np.meshgrid(d, d, d, indexing="ij")
    coarse = np.stack([1 + 2 * z - yy + 0.5 * xx, 3 * xx, z * 0 + 7], axis=-1)
    fine = o3.trilinear2(coarse)
    fz, fy, fx = np.meshgrid(np.arange(10) / 2, np.arange(10) / 2, np.arange(10) / 2, indexing="ij")
    ref = np.stack([1 + 2 * fz - fy + 0.5 * fx, 3 * fx, fz * 0 + 7], axis=-1)
    inner = (slice(0, 9), slice(0, 9), slice(0, 9))
    assert np.max(np.abs(fine[inner] - ref[inner])) < 1e-12
    assert np.array_equal(fine[::2, ::2, ::2], coarse)


def test_masked_mse_gradient():
    p = _rand((3, 4, 2, 3), 10)
    t = _rand((3, 4, 2, 3), 11)
    m = np.random.default_rng(12).random((3, 4, 2)) > 0.4
    loss, g = o3.masked_mse(p, t, m)
    assert abs(_fd(lambda: o3.masked_mse(p, t, m)[0], p, (1, 2, 1, 0)) - g[1, 2, 1, 0]) < 1e-7
    assert np.all(g[~m] == 0)


def test_adam_first_step_moves_by_lr_times_sign():
    """After bias correction the first Adam step is lr * g / |g| per element."""
    w = _rand((10,), 13)
    g = _rand((10,), 14)
    w1, m, v = o3.adam(w, g, np.zeros(10), np.zeros(10), 1, lr=1e-3, eps=0.0)
    assert np.allclose(w - w1, 1e-3 * np.sign(g), rtol=0, atol=1e-15)


def test_network_gradient_finite_differences():
    """Whole-network backward (U-net, skip, pooling, upsampling, residual)
    against central differences of the masked loss."""
    params = o3.init_params(1)
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(0, 0.05, (4, 4, 4, 3)), (rng.random((4, 4, 4, 1)) > 0.3)], axis=-1)
    target = rng.normal(0, 0.05, (8, 8, 8, 3))
    mask = rng.random((8, 8, 8)) > 0.2

    def loss():
        return o3.masked_mse(o3.forward(params, x)[0], target, mask)[0]

    out, cache = o3.forward(params, x)
    _, dout = o3.masked_mse(out, target, mask)
    grads = o3.backward(params, cache, dout)
    for name in ("e1a", "e2b", "u1", "d1a", "f2", "head"):
        w = params[name][0]
        for _ in range(2):
            i = tuple(rng.integers(0, s) for s in w.shape)
            num = _fd(loss, w, i, h=1e-5)
            assert abs(num - grads[name][0][i]) < 1e-6 * max(1.0, abs(num)) + 1e-9, name
        b = params[name][1]
        num = _fd(loss, b, (0,), h=1e-5)
        assert abs(num - grads[name][1][0]) < 1e-6 * max(1.0, abs(num)) + 1e-9, name


def test_parameter_count():
    p = o3.init_params(0)
    n = sum(w.size + b.size for w, b in p.values())
    assert 120_000 < n < 160_000


def test_bf16_round_matches_torch_and_ties_to_even():
    """The oracle's BF16 rounding agrees with torch's CPU conversion (round to
    nearest, ties to even), including exact ties."""
    import torch
    rng = np.random.default_rng(20)
    x = np.concatenate([rng.normal(size=2000), rng.normal(size=2000) * 1e-30, rng.normal(size=2000) * 1e30])
    bits = rng.integers(0, 2 ** 31, 500, dtype=np.uint64)
    ties = ((bits & 0x7F7F0000) | 0x8000).astype(np.uint32).view(np.float32).astype(np.float64)
    x = np.concatenate([x, ties, -ties, [0.0, 1.0, -2.5]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(o3.bf16_round(x), ref)
    # ties go to the even neighbour: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert o3.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert o3.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_quantized_network_reduces_to_exact_with_identity():
    """With q the identity the storage-rounded forward and backward are the
    exact network; with BF16 rounding the output moves by about the BF16 step."""
    params = o3.init_params(3)
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(0, 0.3, (4, 4, 4, 3)), (rng.random((4, 4, 4, 1)) > 0.3)], axis=-1)
    out, cache = o3.forward(params, x)
    out_i, cache_i = o3.forward(params, x, q=lambda a: a)
    assert np.array_equal(out, out_i)
    g = o3.backward(params, cache, np.ones_like(out))
    gi = o3.backward(params, cache_i, np.ones_like(out))
    assert all(np.array_equal(g[k][0], gi[k][0]) and np.array_equal(g[k][1], gi[k][1]) for k in g)
    out_q, _ = o3.forward(params, x, q=o3.bf16_round)
    rel = np.linalg.norm(out_q - out) / np.linalg.norm(out)
    assert 1e-5 < rel < 3e-2
