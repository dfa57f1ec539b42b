"""Pins of the reference of the learned wall-band correction (CPU only).

The reference is pinned to independent implementations and closed forms: BF16 rounding against
torch's float32 -> bfloat16 conversion; the full-grid forward against torch conv2d (circular
padding along x, zero padding along y); the explicit tile backward against torch autograd; the
tile forward against the full-grid forward; the wall field against closed forms (half-plane,
circle) and a brute-force nearest point (sinusoid); Adam's first step against its closed form."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import learned as L

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(L.NPARAM) * scale
    W1 = p[L.OFF_W1:L.OFF_B1].reshape(9, L.CH, L.CIN)
    W1[:, :, L.NFEAT:] = 0.0
    return p.astype(np.float32)


def _torch_weights(p):
    P = L.unpack(p, round_weights=False)
    def k(W):                                    # (9, o, i) -> (o, i, 3, 3)
        return torch.tensor(W.reshape(3, 3, W.shape[1], W.shape[2]).transpose(2, 3, 0, 1).copy())
    return (k(P["W1"]), torch.tensor(P["b1"]), k(P["W2"]), torch.tensor(P["b2"]),
            k(P["W3"][:, None, :]), torch.tensor([P["b3"]]))


def _tconv(x, w, b):
    x = F.pad(x, (1, 1, 0, 0), mode="circular")
    x = F.pad(x, (0, 0, 1, 1))
    return F.conv2d(x, w, b)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100000) * 10.0 ** rng.integers(-6, 6, 100000),
                        # exact ties between two BF16 values round to even
                        (np.arange(1, 2000, dtype=np.float32).view(np.uint32) << 16 | 0x8000).view(np.float32)])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(L.bf16(x), ref.astype(np.float64))


def test_full_forward_matches_torch_conv2d():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((L.NFEAT, 32, 48))
    p = _params(2)
    out, _, _ = L.forward(p, X, 0.05, rounding=False)
    w1, b1, w2, b2, w3, b3 = _torch_weights(p)
    x = torch.tensor(X)[None]
    h = torch.tanh(_tconv(x, w1, b1))
    h = torch.tanh(_tconv(h, w2, b2))
    ref = 0.05 * _tconv(h, w3, b3)[0, 0].numpy()
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("ty0", [0, 16, 48])
def test_tile_backward_matches_torch_autograd(ty0):
    """Tile rows ty0 - 3 .. ty0 + 18 of a 64-row box (rows outside the box are zero)."""
    rng = np.random.default_rng(3 + ty0)
    ny = 64
    Xt = np.zeros((L.CIN, L.HX, L.HX))
    rows = ty0 - 3 + np.arange(L.HX)
    inside = (rows >= 0) & (rows < ny)
    Xt[:L.NFEAT, inside, :] = rng.standard_normal((L.NFEAT, inside.sum(), L.HX))
    Y = rng.standard_normal((16, 16)) * 0.01
    M = (rng.random((16, 16)) < 0.6).astype(float)
    p = _params(4)
    s_out, ic = 0.05, 1.0 / 77.0
    loss, grad, out = L.tile_gradient(p, Xt, Y, M, ty0, ny, s_out, ic, rounding=False)

    P = L.unpack(p, round_weights=False)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in P.items() if k != "b3"}
    tb3 = torch.tensor(float(P["b3"]), dtype=torch.float64, requires_grad=True)
    in1 = torch.tensor((((ty0 - 2 + np.arange(20)) >= 0) & ((ty0 - 2 + np.arange(20)) < ny)).astype(float))
    in2 = torch.tensor((((ty0 - 1 + np.arange(18)) >= 0) & ((ty0 - 1 + np.arange(18)) < ny)).astype(float))

    def conv_valid(W, x):          # W (9, o, i), x (i, m+2, m+2)
        w = W.reshape(3, 3, W.shape[1], W.shape[2]).permute(2, 3, 0, 1)
        return F.conv2d(x[None], w)[0]
    x = torch.tensor(Xt[:L.NFEAT])
    h1 = torch.tanh(conv_valid(tp["W1"], x) + tp["b1"][:, None, None]) * in1[None, :, None]
    h2 = torch.tanh(conv_valid(tp["W2"], h1) + tp["b2"][:, None, None]) * in2[None, :, None]
    o = s_out * (conv_valid(tp["W3"][:, None, :], h2)[0] + tb3)
    lt = (torch.tensor(M) * (o - torch.tensor(Y)) ** 2).sum() * ic
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-12 * abs(lt.item())
    refs = [(L.OFF_W1, L.OFF_B1, np.pad(tp["W1"].grad.numpy(), ((0, 0), (0, 0), (0, L.CIN - L.NFEAT)))),
            (L.OFF_B1, L.OFF_W2, tp["b1"].grad.numpy()), (L.OFF_W2, L.OFF_B2, tp["W2"].grad.numpy()),
            (L.OFF_B2, L.OFF_W3, tp["b2"].grad.numpy()), (L.OFF_W3, L.OFF_B3, tp["W3"].grad.numpy()),
            (L.OFF_B3, L.NPARAM, np.array([tb3.grad.item()]))]
    for a, b, r in refs:
        r = r.reshape(-1)
        assert np.max(np.abs(grad[a:b] - r)) <= 1e-10 * max(1e-30, np.max(np.abs(r))), (a, b)


def test_tile_forward_equals_the_full_grid_forward():
    rng = np.random.default_rng(5)
    ny, nx = 48, 64
    X = np.zeros((L.CIN, ny, nx))
    X[:L.NFEAT] = L.bf16(rng.standard_normal((L.NFEAT, ny, nx)))
    p = _params(6)
    for rounding, tol in ((False, 1e-12), (True, 2e-3)):
        full, _, _ = L.forward(p, X[:L.NFEAT], 0.05, rounding=rounding)
        for tx0, ty0 in ((0, 0), (48, 16), (16, 32)):
            Xt = L.patch(X, tx0, ty0)
            _, _, out = L.tile_gradient(p, Xt, np.zeros((16, 16)), np.zeros((16, 16)), ty0, ny, 0.05, 1.0,
                                        rounding=rounding)
            ref = full[ty0:ty0 + 16, tx0:tx0 + 16]
            assert np.max(np.abs(out - ref)) <= tol * np.max(np.abs(full)), (rounding, tx0, ty0)


def test_wall_field_closed_forms():
    n, lo, hi = (64, 32), (0.0, 0.0), (2.0, 1.0)
    h = 2.0 / 64
    y = (np.arange(32) + 0.5) * h
    x = (np.arange(64) + 0.5) * h
    d, nn = L.wall_field(n, lo, hi, [W.Shape(W.HALFPLANE, (0.0, 0.3, 0.0, 0.0, 1.0, 0.0))])
    assert np.max(np.abs(d - (y[:, None] - 0.3))) <= 1e-15
    assert np.all(nn[0] == 0) and np.all(nn[1] == 1)
    d, nn = L.wall_field(n, lo, hi, [W.Shape(W.SPHERE, (1.0, 0.4, 0.0, 0.25))])
    r = np.hypot(x[None, :] - 1.0, y[:, None] - 0.4)
    assert np.max(np.abs(d - (r - 0.25))) <= 1e-15
    assert np.max(np.abs(nn[0] * r - (x[None, :] - 1.0))) <= 1e-14


def test_wall_field_sinusoid_is_the_nearest_curve_point():
    n, lo, hi = (128, 64), (0.0, 0.0), (4.0, 2.0)
    p = (0.3, 0.1, 0.5, 0.0)
    d, nn = L.wall_field(n, lo, hi, [W.Shape(W.SINUSOID, p)])
    h = 4.0 / 128
    rng = np.random.default_rng(7)
    s = np.linspace(-1.0, 5.0, 600001)
    ws = np.stack([s, p[0] + p[1] * np.sin(2 * np.pi * s / p[2])])
    for _ in range(200):
        j, i = rng.integers(0, 64), rng.integers(0, 128)
        q = np.array([(i + 0.5) * h, (j + 0.5) * h])
        brute = np.min(np.hypot(ws[0] - q[0], ws[1] - q[1]))
        assert abs(abs(d[j, i]) - brute) <= 1e-6
        above = q[1] >= p[0] + p[1] * np.sin(2 * np.pi * q[0] / p[2])
        assert (d[j, i] >= 0) == above
        assert abs(np.hypot(nn[0, j, i], nn[1, j, i]) - 1) <= 1e-12 and nn[1, j, i] > 0


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = L.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    # bias-corrected moments of the first step are g and g^2: the step is lr g / (|g| + eps)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
