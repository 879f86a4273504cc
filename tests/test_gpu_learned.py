"""GPU parity of the learned proposer's kernels and of sg_rerank.

Gradients: the GPU rounds layer operands to BF16 and accumulates in FP32; the
oracle evaluates the same network in FP64 with the same BF16-rounded weights.
Per tensor the relative Frobenius error must be <= 2e-2.  Training: the
captured-graph loop and the plain loop must give identical weights, and the
loss must fall.  Re-rank: exact on integer data.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _net(D, H, E, seed):
    rng = np.random.default_rng(seed)
    W1 = (rng.standard_normal((H, D)) * np.sqrt(2.0 / D)).astype(np.float32)
    W2 = (rng.standard_normal((E, H)) * np.sqrt(1.0 / H)).astype(np.float32)
    b1 = (rng.standard_normal(H) * 0.01).astype(np.float32)
    b2 = (rng.standard_normal(E) * 0.01).astype(np.float32)
    # weights exactly representable in BF16 so both sides use the same values
    W1 = oracle.from_bf16(oracle.to_bf16(W1)).astype(np.float32)
    W2 = oracle.from_bf16(oracle.to_bf16(W2)).astype(np.float32)
    return W1, b1, W2, b2


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("D,H,E,B", [(960, 256, 64, 128), (96, 64, 16, 64)])
def test_mlp_gradients_match_oracle(D, H, E, B):
    X = synthdata.l1_nonneg(3000, d=D, seed=D, n_comp=40)
    rng = np.random.default_rng(3)
    anchors = rng.choice(3000, size=B, replace=False)
    positives = rng.choice(3000, size=B, replace=False)
    W1, b1, W2, b2 = _net(D, H, E, seed=1)
    Xg = torch.from_numpy(X).to(DEV)
    mu, sigma = sg.sg_mlp_stats(Xg, anchors)
    mu_h, sigma_h = mu.cpu().numpy(), float(sigma.cpu().numpy()[0])
    # statistics against FP64 numpy on the same rows
    np.testing.assert_allclose(mu_h, X[anchors].astype(np.float64).mean(0), rtol=1e-5, atol=1e-9)
    assert abs(sigma_h - (X[anchors].astype(np.float64) - mu_h).std()) <= 1e-5 * sigma_h
    net = sg.MLP(*(torch.from_numpy(a).to(DEV) for a in (W1, b1, W2, b2)), mu, sigma)
    loss, gW1, gb1, gW2, gb2 = sg.sg_mlp_loss_grad(Xg, net, anchors, positives, T=0.05)
    # the oracle sees the rounded input rows the GPU's first product sees: z in FP64
    oloss, oW1, ob1, oW2, ob2 = oracle.mlp_loss_grad(X[anchors], X[positives], W1, b1, W2, b2, mu_h,
                                                     sigma_h, 0.05)
    assert abs(loss.item() - oloss) <= 2e-2 * abs(oloss)
    for g, o in ((gW1, oW1), (gb1, ob1), (gW2, oW2), (gb2, ob2)):
        assert _rel(g.cpu().numpy(), o) <= 2e-2


def test_mlp_project_matches_oracle():
    D, H, E = 960, 256, 64
    X = synthdata.l1_nonneg(5000, d=D, seed=2, n_comp=30)
    W1, b1, W2, b2 = _net(D, H, E, seed=2)
    Xg = torch.from_numpy(X).to(DEV)
    mu, sigma = sg.sg_mlp_stats(Xg, np.arange(0, 5000, 3))
    net = sg.MLP(*(torch.from_numpy(a).to(DEV) for a in (W1, b1, W2, b2)), mu, sigma)
    F = sg.sg_mlp_project(Xg, net).cpu().numpy()
    oF = oracle.mlp_forward(X[:400], W1, b1, W2, b2, mu.cpu().numpy(), float(sigma.item()))
    assert np.abs(F[:400] - oF).max() < 2e-2
    np.testing.assert_allclose(np.linalg.norm(F, axis=1), 1.0, rtol=1e-5)


def test_mlp_training_graph_equals_plain_and_tracks_oracle():
    """150 Adam steps on the GPU (captured graph and plain loop, bit-identical)
    follow the trajectory of the same loop driven by the FP64 oracle's
    gradients and Adam step."""
    D, H, E, B, steps = 96, 64, 16, 128, 150
    X = synthdata.l1_nonneg(4000, d=D, seed=4, n_comp=25)
    Xg = torch.from_numpy(X).to(DEV)
    knn, _ = oracle.knn(oracle.widen(X), 8)
    rng = np.random.default_rng(0)
    anchors = rng.integers(0, 4000, size=B * steps)
    positives = knn[anchors, rng.integers(0, 8, size=B * steps)]
    W1, b1, W2, b2 = _net(D, H, E, seed=5)
    mu, sigma = sg.sg_mlp_stats(Xg, np.arange(4000))
    nets = [sg.MLP(*(torch.from_numpy(a).to(DEV) for a in (W1, b1, W2, b2)), mu, sigma) for _ in range(2)]
    la = sg.sg_mlp_train(Xg, nets[0], anchors, positives, B, steps, lr=3e-3, use_graph=True)
    lb = sg.sg_mlp_train(Xg, nets[1], anchors, positives, B, steps, lr=3e-3, use_graph=False)
    torch.cuda.synchronize()
    assert torch.equal(la, lb)
    for t0, t1 in ((nets[0].W1, nets[1].W1), (nets[0].W2, nets[1].W2), (nets[0].b1, nets[1].b1)):
        assert torch.equal(t0, t1)
    # the same loop on the oracle (FP64 gradients, FP64 Adam)
    params = [a.astype(np.float64) for a in (W1, b1, W2, b2)]
    ms = [np.zeros_like(p) for p in params]
    vs = [np.zeros_like(p) for p in params]
    mu_h, sigma_h = mu.cpu().numpy(), float(sigma.item())
    ol = []
    for t in range(steps):
        a, p = anchors[t * B:(t + 1) * B], positives[t * B:(t + 1) * B]
        loss, *g = oracle.mlp_loss_grad(X[a], X[p], *params, mu_h, sigma_h, 0.05)
        ol.append(loss)
        for i in range(4):
            params[i], ms[i], vs[i] = oracle.adam(params[i], g[i], ms[i], vs[i], 3e-3, 0.9, 0.999, 1e-8, t + 1)
    gl = la.cpu().numpy().astype(np.float64)
    ol = np.array(ol)
    assert np.max(np.abs(gl - ol) / ol) < 2e-2
    assert abs(gl[-20:].mean() - ol[-20:].mean()) < 5e-3 * ol[-20:].mean()
    assert ol[-20:].mean() < ol[:10].mean()            # it learns
    assert _rel(nets[0].W1.cpu().numpy(), params[0]) < 5e-2
    assert _rel(nets[0].W2.cpu().numpy(), params[2]) < 5e-2


def test_rerank_exact_on_integer_rows():
    X = np.random.default_rng(9).integers(0, 16, size=(1500, 40)).astype(np.float32)
    rng = np.random.default_rng(1)
    cand = np.stack([rng.choice(1500, size=100, replace=False) for _ in range(1500)]).astype(np.int32)
    cand[::7, 5:9] = -1
    cand[::11, 10] = cand[::11, 11]           # a repeated candidate
    nbr, dist = sg.sg_rerank(torch.from_numpy(X).to(DEV), torch.from_numpy(cand).to(DEV), 32)
    onbr, odist = oracle.rerank(oracle.widen(X), cand, 32)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("d,dtype", [(300, np.float32), (301, np.float32), (960, np.float32), (200, np.float16)])
def test_rerank_wide_rows_exact_on_integer_rows(d, dtype):
    """Rows wider than 128 use the wave-per-row re-rank (coalesced loads,
    butterfly sum); on integer-valued rows every order is exact."""
    rng = np.random.default_rng(d)
    n, c = 700, 130
    X = rng.integers(0, 8, size=(n, d)).astype(dtype)
    cand = np.stack([rng.choice(n, size=c, replace=False) for _ in range(n)]).astype(np.int32)
    cand[::5, 3:7] = -1
    cand[::9, 20] = cand[::9, 21]
    nbr, dist = sg.sg_rerank(torch.from_numpy(X).to(DEV), torch.from_numpy(cand).to(DEV), 40)
    onbr, odist = oracle.rerank(oracle.widen(X), cand, 40)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


@pytest.mark.parametrize("d", [64, 200])
def test_learned_graph_with_all_candidates_is_exact(d):
    """c >= n - 1 proposes every row, so the re-ranked lists are the exact kNN."""
    X = synthdata.sift_like_u8(n=250, d=d, seed=d, n_comp=8).astype(np.float32)
    Xg = torch.from_numpy(X).to(DEV)
    P = torch.nn.functional.normalize(torch.from_numpy(X[:, :48].copy()).to(DEV) + 1.0, dim=1)
    nbr, dist = sg.sg_knn_graph_learned(Xg, P.contiguous(), 256, 32)
    onbr, odist = oracle.knn(oracle.widen(X), 32)
    np.testing.assert_array_equal(nbr.cpu().numpy(), onbr)
    np.testing.assert_array_equal(dist.cpu().numpy(), odist.astype(np.float32))


def test_learned_graph_trained_projection_gain():
    """A short training run on clustered data: the learned lists are valid
    (no self, distinct, ascending FP32 distances equal to FP64 ones within
    1e-5), and at the same candidate budget the trained net recovers more exact
    neighbours than the same net untrained and than a random projection."""
    D, H, E, K, c = 96, 64, 16, 16, 64
    X = synthdata.l1_nonneg(3000, d=D, seed=12, n_comp=30)
    Xg = torch.from_numpy(X).to(DEV)
    knn, _ = oracle.knn(oracle.widen(X), K)
    rng = np.random.default_rng(1)
    steps, B = 300, 256
    anchors = rng.integers(0, 3000, size=B * steps)
    positives = knn[anchors, rng.integers(0, K, size=B * steps)]
    W1, b1, W2, b2 = _net(D, H, E, seed=3)
    mu, sigma = sg.sg_mlp_stats(Xg, np.arange(3000))
    mk = lambda: sg.MLP(*(torch.from_numpy(a).to(DEV) for a in (W1, b1, W2, b2)), mu, sigma)
    net, net0 = mk(), mk()
    sg.sg_mlp_train(Xg, net, anchors, positives, B, steps, lr=3e-3)
    F = sg.sg_mlp_project(Xg, net)
    nbr, dist = sg.sg_knn_graph_learned(Xg, F, c, K)
    g, gd = nbr.cpu().numpy(), dist.cpu().numpy()
    assert (g != np.arange(3000)[:, None]).all()
    assert all(len(set(r[r >= 0])) == len(r[r >= 0]) for r in g)
    assert (np.diff(gd, axis=1) >= 0).all()
    d64 = oracle.pair_dist(oracle.widen(X), np.repeat(np.arange(3000)[:, None], K, 1), g, oracle.L2)
    np.testing.assert_allclose(gd, d64, rtol=1e-5, atol=1e-9)
    rec = lambda lists: float(np.mean([len(set(a) & set(b)) / K for a, b in zip(lists, knn)]))
    r_trained = rec(g)
    r_untrained = rec(sg.sg_knn_graph_learned(Xg, sg.sg_mlp_project(Xg, net0), c, K)[0].cpu().numpy())
    G = torch.randn((D, E), generator=torch.Generator().manual_seed(4)).to(DEV)
    Prand = torch.nn.functional.normalize(Xg @ G, dim=1).contiguous()
    r_random = rec(sg.sg_knn_graph_learned(Xg, Prand, c, K)[0].cpu().numpy())
    assert r_trained > 0.85, (r_trained, r_untrained, r_random)
    assert r_trained > r_untrained + 0.05, (r_trained, r_untrained)
    assert r_trained > r_random + 0.05, (r_trained, r_random)
