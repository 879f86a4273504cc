"""GPU parity of the batched shard build (sg_knn_graph_batched) through the C ABI.

Every shard's result must equal the single-shard path (sg_knn_graph, then
sg_prune) bit for bit, and on integer rows the kNN lists must equal the FP64
oracle.  The captured plan must replay to the same result, follow new data
written into the same buffers, and refuse other arguments.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _per_shard(Xg, offs, k, R, metric, prec):
    g, kn = [], []
    for s in range(len(offs) - 1):
        a, b = offs[s], offs[s + 1]
        if b == a:
            continue
        nb, _ = sg.sg_knn_graph(Xg[a:b], k, metric, prec, dist=False)
        kn.append(nb)
        g.append(sg.sg_prune(nb, R))
    return torch.cat(g), torch.cat(kn)


@pytest.mark.parametrize("prec", ["f16", "fp32"])
def test_batched_equals_per_shard_and_oracle_u8(prec):
    sizes = [3000, 0, 700, 4500, 40, 1]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    X = synthdata.sift_like_u8(n=int(offs[-1]), d=128, seed=31, n_comp=60)
    Xg = torch.from_numpy(X).to(DEV)
    k, R = 32, 16
    graphs, knn = sg.sg_knn_graph_batched(Xg, offs, k, R, "l2", prec)
    torch.cuda.synchronize()
    g_ref, k_ref = _per_shard(Xg, offs, k, R, "l2", prec)
    assert torch.equal(knn, k_ref)
    assert torch.equal(graphs, g_ref)
    knn_h = knn.cpu().numpy()
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        if b - a < 2:
            continue
        onbr, _ = oracle.knn(oracle.widen(X[a:b]), k)
        np.testing.assert_array_equal(knn_h[a:b], onbr, err_msg="shard %d" % s)


@pytest.mark.parametrize("prec,rerank", [("bf16", 64), ("fp8", 128)])
def test_batched_rerank_equals_per_shard(prec, rerank):
    # reduced-precision keys, the best `rerank` re-ranked in FP32: the same
    # candidate sets and the same exact re-rank as the single-shard path
    sizes = [2500, 5200, 0, 900]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    X = synthdata.deep_like_unit(n=int(offs[-1]), d=96, seed=23)
    Xg = torch.from_numpy(X).to(DEV)
    k, R = 32, 16
    graphs, knn = sg.sg_knn_graph_batched(Xg, offs, k, R, "ip", prec, rerank=rerank)
    torch.cuda.synchronize()
    g, kn = [], []
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        if b == a:
            continue
        nb, _ = sg.sg_knn_graph(Xg[a:b], k, "ip", prec, rerank=rerank, dist=False)
        kn.append(nb)
        g.append(sg.sg_prune(nb, R))
    assert torch.equal(knn, torch.cat(kn))
    assert torch.equal(graphs, torch.cat(g))


def test_batched_f16_ip_d768_equals_per_shard():
    sizes = [1500, 3200, 800, 4300]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    X = synthdata.laion_like_f16(int(offs[-1]), d=768, seed=5, n_comp=40)
    Xg = torch.from_numpy(X).to(DEV)
    graphs, knn = sg.sg_knn_graph_batched(Xg, offs, 64, 32, "ip", "f16")
    torch.cuda.synchronize()
    g_ref, k_ref = _per_shard(Xg, offs, 64, 32, "ip", "f16")
    assert torch.equal(knn, k_ref)
    assert torch.equal(graphs, g_ref)


def test_batched_plan_replays_and_follows_data():
    sizes = [2500, 900, 4200]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    n = int(offs[-1])
    X1 = synthdata.sift_like_u8(n=n, d=64, seed=1, n_comp=30)
    X2 = synthdata.sift_like_u8(n=n, d=64, seed=2, n_comp=30)
    Xg = torch.from_numpy(X1).to(DEV)
    graphs = torch.empty((n, 16), dtype=torch.int32, device=DEV)
    knn = torch.empty((n, 32), dtype=torch.int32, device=DEV)
    stream = torch.cuda.Stream()
    plan = sg.BatchPlan()
    with torch.cuda.stream(stream):
        sg.sg_knn_graph_batched(Xg, offs, 32, 16, "l2", "f16", out=(graphs, knn), stream=stream, plan=plan)
    stream.synchronize()
    assert plan.ptr.value
    first = (graphs.clone(), knn.clone())
    g_ref, k_ref = _per_shard(Xg, offs, 32, 16, "l2", "f16")
    assert torch.equal(first[0], g_ref) and torch.equal(first[1], k_ref)
    for rep in range(3):   # replays, with eager work in between
        graphs.fill_(-7)
        with torch.cuda.stream(stream):
            sg.sg_knn_graph_batched(Xg, offs, 32, 16, "l2", "f16", out=(graphs, knn), stream=stream, plan=plan)
        stream.synchronize()
        assert torch.equal(graphs, first[0]), rep
        assert torch.equal(knn, first[1]), rep
    Xg.copy_(torch.from_numpy(X2).to(DEV))   # new data, same buffer: the replay reads it
    with torch.cuda.stream(stream):
        sg.sg_knn_graph_batched(Xg, offs, 32, 16, "l2", "f16", out=(graphs, knn), stream=stream, plan=plan)
    stream.synchronize()
    g2, k2 = _per_shard(Xg, offs, 32, 16, "l2", "f16")
    assert torch.equal(graphs, g2) and torch.equal(knn, k2)
    with pytest.raises(sg.SgError):   # other arguments
        with torch.cuda.stream(stream):
            sg.sg_knn_graph_batched(Xg, offs, 32, 8, "l2", "f16", out=(graphs[:, :8].contiguous(), knn),
                                    stream=stream, plan=plan)
    plan.close()


def test_batched_argument_errors():
    Xg = torch.zeros((100, 16), dtype=torch.float32, device=DEV)
    with pytest.raises(sg.SgError):
        sg.sg_knn_graph_batched(Xg, [5, 50, 100], 8, 4)           # offsets[0] != 0
    with pytest.raises(sg.SgError):
        sg.sg_knn_graph_batched(Xg, [0, 50, 100], 300, 4)         # k > 256
    with pytest.raises(sg.SgError):
        sg.sg_knn_graph_batched(Xg, [0, 50, 100], 32, 4, rerank=300)   # re-rank wider than 256
    with pytest.raises(sg.SgError):
        sg.sg_knn_graph_batched(Xg, [0, 50, 100], 256, 129)       # R > 128
    with pytest.raises(sg.SgError):
        sg.sg_knn_graph_batched(Xg, list(range(0, 66)), 8, 4)     # S > 64


@pytest.mark.parametrize("k,R", [(128, 64), (256, 128)])
def test_batched_high_degree_equals_per_shard_and_oracle(k, R):
    # the paper's default (degree 64 from 128 candidates) and stress (128 from
    # 256) settings: lists and pruned graphs as the single-shard path, kNN
    # lists as the oracle on integer rows
    sizes = [1800, 600, 2600]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    X = synthdata.sift_like_u8(n=int(offs[-1]), d=128, seed=41, n_comp=12)
    Xg = torch.from_numpy(X).to(DEV)
    graphs, knn = sg.sg_knn_graph_batched(Xg, offs, k, R, "l2", "f16")
    torch.cuda.synchronize()
    g_ref, k_ref = _per_shard(Xg, offs, k, R, "l2", "f16")
    assert torch.equal(knn, k_ref)
    assert torch.equal(graphs, g_ref)
    knn_h, g_h = knn.cpu().numpy(), graphs.cpu().numpy()
    for s in range(len(sizes)):
        a, b = offs[s], offs[s + 1]
        onbr, _ = oracle.knn(oracle.widen(X[a:b]), k)
        np.testing.assert_array_equal(knn_h[a:b], onbr, err_msg="shard %d" % s)
        np.testing.assert_array_equal(g_h[a:b], oracle.prune(onbr, R), err_msg="shard %d" % s)


def test_batched_autotune_records_a_valid_choice_and_keeps_results():
    sizes = [3000, 700, 4500, 1200]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    X = synthdata.sift_like_u8(n=int(offs[-1]), d=128, seed=37, n_comp=50)
    Xg = torch.from_numpy(X).to(DEV)
    ref_g, ref_k = sg.sg_knn_graph_batched(Xg, offs, 32, 16, "l2", "i8")
    chosen, times = sg.sg_knn_graph_batched_autotune(Xg, offs, 32, 16, "l2", "i8")
    assert 0 <= chosen < len(times) == sg.sg_knn_variant_count(128, 32, "i8")
    assert all(t > 0 for t in times) and times[chosen] == min(times)
    g, k = sg.sg_knn_graph_batched(Xg, offs, 32, 16, "l2", "i8")
    torch.cuda.synchronize()
    assert torch.equal(g, ref_g) and torch.equal(k, ref_k)
