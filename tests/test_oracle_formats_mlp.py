"""Pins of the oracle's number formats and of the learned proposer's maths.

Formats: BF16 and OCP FP8 E4M3 rounding against torch's CPU conversions (a
library routine), every FP8 code round-tripped, the half-way points between
neighbouring codes (ties to even), saturation at 448, and the per-row
power-of-two scale bound.  MLP: exact gradients against central finite
differences and against torch FP64 autograd; Adam's first step in closed form.
"""
import numpy as np
import pytest
import torch

import oracle


def test_bf16_matches_torch_dense_sweep():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
        np.array([0.0, -0.0, 1.0, 3.0e38, -3.4e38, 1e-40, -1e-45], np.float32),
    ]).astype(np.float32)
    # exact half-way cases: bf16 value + half an ulp
    base = rng.standard_normal(4000).astype(np.float32)
    bits = base.view(np.uint32) & np.uint32(0xFFFF0000)
    half = (bits | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, half])
    ours = oracle.to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)


def test_fp8_matches_torch_in_range():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(50000) * 10.0 ** rng.uniform(-4, 2.6, 50000)).astype(np.float32)
    x = x[np.abs(x) < 464.0]
    ours = oracle.to_fp8(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_fp8_codes_roundtrip_and_ties_to_even():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    vals = oracle.from_fp8(codes)
    back = oracle.to_fp8(vals.astype(np.float32))
    # +0 and -0 both decode to zero; everything else round-trips exactly
    np.testing.assert_array_equal(back, codes)
    pos = np.sort(oracle.from_fp8(np.arange(0, 0x7F, dtype=np.uint8)))
    mids = ((pos[:-1] + pos[1:]) / 2).astype(np.float32)
    got = oracle.to_fp8(mids)
    lo = oracle.to_fp8(pos[:-1].astype(np.float32))
    hi = oracle.to_fp8(pos[1:].astype(np.float32))
    even = np.where(lo % 2 == 0, lo, hi)                # the code with even mantissa wins
    np.testing.assert_array_equal(got, even)


def test_fp8_saturates():
    x = np.array([448.0, 464.0, 500.0, 1e9, -1e9, np.inf], np.float32)
    assert oracle.to_fp8(x).tolist() == [0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0x7E]
    assert oracle.from_fp8(np.array([0x7E], np.uint8))[0] == 448.0


def test_fp8_row_scales_are_tight_powers_of_two():
    rng = np.random.default_rng(2)
    X = (rng.standard_normal((200, 33)) * 10.0 ** rng.uniform(-6, 6, (200, 1))).astype(np.float32)
    X[5] = 0
    q, s = oracle.quant_rows_fp8(X)
    amax = np.abs(X).max(1)
    for i in range(200):
        if amax[i] == 0:
            assert s[i] == 1.0
            continue
        m, e = np.frexp(s[i])
        assert m == 0.5                                # power of two
        assert amax[i] / s[i] <= 448.0 and amax[i] / s[i] > 224.0
    deq = oracle.from_fp8(q) * s[:, None]
    rel = np.abs(deq - X) / np.maximum(amax[:, None], 1e-30)
    assert rel.max() <= 2.0 ** -4                      # half an ulp of 3 mantissa bits near amax


def _tiny_net(D=8, H=5, E=3, seed=0):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((H, D)) * 0.5, rng.standard_normal(H) * 0.1,
            rng.standard_normal((E, H)) * 0.5, rng.standard_normal(E) * 0.1,
            rng.standard_normal(D) * 0.2, 1.3)


def test_mlp_gradients_finite_differences():
    W1, b1, W2, b2, mu, sigma = _tiny_net()
    rng = np.random.default_rng(5)
    Xa = rng.standard_normal((6, 8))
    Xp = Xa + 0.3 * rng.standard_normal((6, 8))
    T = 0.5
    loss, gW1, gb1, gW2, gb2 = oracle.mlp_loss_grad(Xa, Xp, W1, b1, W2, b2, mu, sigma, T)
    h = 1e-6
    params = [W1, b1, W2, b2]
    grads = [gW1, gb1, gW2, gb2]
    for P, G in zip(params, grads):
        flat = P.reshape(-1)
        num = np.empty_like(flat)
        for k in range(flat.size):
            old = flat[k]
            flat[k] = old + h
            lp = oracle.mlp_loss_grad(Xa, Xp, W1, b1, W2, b2, mu, sigma, T)[0]
            flat[k] = old - h
            lm = oracle.mlp_loss_grad(Xa, Xp, W1, b1, W2, b2, mu, sigma, T)[0]
            flat[k] = old
            num[k] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(G.reshape(-1), num, rtol=1e-5, atol=1e-8)


def test_mlp_matches_torch_autograd():
    D, H, E, B = 16, 12, 6, 9
    W1, b1, W2, b2, mu, sigma = _tiny_net(D, H, E, seed=3)
    rng = np.random.default_rng(7)
    Xa = rng.standard_normal((B, D))
    Xp = Xa + 0.2 * rng.standard_normal((B, D))
    T = 0.05
    loss, gW1, gb1, gW2, gb2 = oracle.mlp_loss_grad(Xa, Xp, W1, b1, W2, b2, mu, sigma, T)
    tp = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (W1, b1, W2, b2)]

    def f(X):
        z = (torch.tensor(X) - torch.tensor(mu)) / sigma
        h1 = z @ tp[0].T + tp[1]
        a1 = torch.nn.functional.gelu(h1)
        h2 = a1 @ tp[2].T + tp[3]
        return h2 / h2.norm(dim=1, keepdim=True)

    logits = f(Xa) @ f(Xp).T / T
    tl = torch.nn.functional.cross_entropy(logits, torch.arange(B))
    tl.backward()
    assert abs(tl.item() - loss) < 1e-12 * max(1.0, abs(loss))
    for G, t in zip((gW1, gb1, gW2, gb2), tp):
        np.testing.assert_allclose(G, t.grad.numpy(), rtol=1e-10, atol=1e-13)
    F = oracle.mlp_forward(Xa, W1, b1, W2, b2, mu, sigma)
    np.testing.assert_allclose(F, f(Xa).detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    w1, m1, v1 = oracle.adam(w, g, np.zeros(4), np.zeros(4), lr=0.1, beta1=0.9, beta2=0.999,
                             eps=1e-8, step=1)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> w - lr * g / (|g| + eps)
    np.testing.assert_allclose(w1, w - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)


def test_adam_moment_recursion_against_torch():
    """Several Adam steps starting from non-zero moments at a late step count,
    against torch.optim.Adam in FP64 on the CPU: a dropped beta1*m or beta2*v
    term, or a wrong bias correction, changes every step after the first."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(17)
    n = 257
    w = rng.standard_normal(n)
    m = 0.05 * rng.standard_normal(n)
    v = 0.01 * rng.random(n) + 1e-6
    step0 = 40
    lr, b1, b2, eps = 3e-3, 0.8, 0.95, 1e-6
    p = torch.nn.Parameter(torch.tensor(w, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps)
    opt.state[p] = {"step": torch.tensor(float(step0), dtype=torch.float64),
                    "exp_avg": torch.tensor(m, dtype=torch.float64),
                    "exp_avg_sq": torch.tensor(v, dtype=torch.float64)}
    ow, om, ov = w.copy(), m.copy(), v.copy()
    for t in range(1, 6):
        g = rng.standard_normal(n) * (0.1 + t)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        ow, om, ov = oracle.adam(ow, g, om, ov, lr, b1, b2, eps, step0 + t)
        st = opt.state[p]
        np.testing.assert_allclose(om, st["exp_avg"].numpy(), rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(ov, st["exp_avg_sq"].numpy(), rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(ow, p.detach().numpy(), rtol=1e-12, atol=1e-15)
