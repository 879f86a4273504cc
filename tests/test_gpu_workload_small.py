"""The small workload end to end on the GPU: 8192 x 96 FP32 rows from a
32-component mixture (std 0.3), k-means into 2 shards with every row also in
its second-nearest shard, exact kNN K = 32 per shard, prune to R = 16, merge.

With 2 shards and omega = 2 every row is in both shards, so both shard graphs
are the unsharded graph and the merge must reproduce it (an identity check of
the merge).  kNN rows are checked under the FP32 rounding-bound rule with no
row allowance; prune and merge are checked bit for bit, both on the oracle's
kNN graph and on the GPU's own kNN graph (the oracle pruning and merging that
same graph).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_10135_amd as sg
import synthdata
from parity import check_rows

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_small_workload_end_to_end():
    X = synthdata.small_f32()
    N, S, omega, K, R = X.shape[0], 2, 2, 32, 16
    init = synthdata.init_rows(N, S, seed=1000)
    Xg = torch.from_numpy(X).to(DEV)
    C, prim, off, mem = sg.sg_partition(Xg, S, omega, 20, init)
    X64 = oracle.widen(X)
    oC, oprim, ooff, omem = oracle.partition(X64, S, omega, 20, init)
    np.testing.assert_array_equal(off.numpy(), ooff)
    np.testing.assert_array_equal(mem.cpu().numpy(), omem)       # both shards = all rows
    assert (prim.cpu().numpy() == oprim).mean() > 0.999

    onbr, odist = oracle.knn(X64, K)
    oP = oracle.prune(onbr, R)
    graphs_gpu = []
    for s in range(S):
        ids = omem[ooff[s]:ooff[s + 1]]
        Xs = Xg[torch.from_numpy(ids.astype(np.int64)).to(DEV)]
        nbr, dist = sg.sg_knn_graph(Xs, K, "l2", "fp32")
        g = nbr.cpu().numpy()
        bad = check_rows(X64, np.arange(N), g, dist.cpu().numpy(), onbr, odist)
        assert not bad, bad[:5]
        # prune on the oracle's kNN graph: bit for bit
        Pg = sg.sg_prune(torch.from_numpy(onbr).to(DEV), R).cpu().numpy()
        np.testing.assert_array_equal(Pg, oP)
        # prune of the GPU's own kNN graph: bit for bit with the oracle's
        # prune of that same graph
        Pgg = sg.sg_prune(nbr, R)
        np.testing.assert_array_equal(Pgg.cpu().numpy(), oracle.prune(g, R))
        graphs_gpu.append(Pgg)
    # merge of the oracle's pruned graphs: bit for bit, and the identity
    out, deg = sg.sg_merge(ooff, torch.from_numpy(omem).to(DEV),
                           torch.from_numpy(np.concatenate([oP, oP])).to(DEV), R, N, omega * R)
    oout, odeg = oracle.merge(ooff, omem, np.concatenate([oP, oP]), R, N, omega * R)
    np.testing.assert_array_equal(out.cpu().numpy(), oout)
    np.testing.assert_array_equal(deg.cpu().numpy(), odeg)
    np.testing.assert_array_equal(oout[:, :R], oP)
    # the all-GPU pipeline: its merge equals the oracle's merge of the same
    # (GPU-built) shard graphs bit for bit, and merging two equal shard
    # graphs reproduces the shard graph (both shards hold every row)
    G = torch.cat(graphs_gpu)
    gout, gdeg = sg.sg_merge(off.numpy(), mem, G, R, N, omega * R)
    Gh = G.cpu().numpy()
    oout2, odeg2 = oracle.merge(off.numpy(), mem.cpu().numpy(), Gh, R, N, omega * R)
    np.testing.assert_array_equal(gout.cpu().numpy(), oout2)
    np.testing.assert_array_equal(gdeg.cpu().numpy(), odeg2)
    np.testing.assert_array_equal(gout.cpu().numpy()[:, :R], Gh[:N])
    assert (gdeg.cpu().numpy() == R).all()
