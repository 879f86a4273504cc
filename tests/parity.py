"""Parity helpers shared by the GPU tests (comparison logic only).

kNN rows from the GPU are compared with the oracle's exact lists under the
tie rule for floating-point data: with tau = 1e-5, a GPU row passes when
  1. its ids are distinct and exclude the row itself,
  2. its distances are sorted,
  3. every GPU id outside the oracle's set has delta <= delta_K (1 + tau),
  4. every oracle id missing from the GPU set has delta >= delta_K (1 - tau),
  5. at every position j, |delta(gpu_j) - delta_oracle(j)| <= tau max(delta_oracle(j), floor),
where delta is the FP64 oracle distance, delta_K the oracle's K-th distance and
floor = 1e-6 x the median |delta_K|.  For IP the tolerance is relative to the IP
distance -x.y itself (an FP32 dot product resolves it to ~1e-7 relative; its
L2 form 2 + 2 delta is reported separately by l2_form_violations because an
FP32 dot product cannot resolve that form to 1e-5 for near-duplicate rows).
For integer-valued data the comparison is exact.
"""
import numpy as np

import oracle

TAU = 1e-5


def l2_form(d, metric):
    return d if metric == oracle.L2 else 2.0 + 2.0 * d


def _mag(d):
    return np.abs(d)


def check_rows(X64, rows, gpu_nbr, gpu_dist, ora_nbr, ora_dist, metric=oracle.L2, tau=TAU):
    rows = np.asarray(rows)
    K = ora_nbr.shape[1]
    od = ora_dist
    valid_k = np.isfinite(od[:, -1])
    floor = 1e-6 * (np.median(np.abs(od[valid_k, -1])) if valid_k.any() else 1.0)
    gd64 = oracle.pair_dist(X64, np.repeat(rows[:, None], K, 1), gpu_nbr, metric)
    bad = []
    for r, i in enumerate(rows):
        g = gpu_nbr[r]
        o = ora_nbr[r]
        gv = g[g >= 0]
        ov = o[o >= 0]
        if len(gv) != len(ov) or len(set(gv.tolist())) != len(gv) or i in gv:
            bad.append((int(i), "ids: count/distinct/self"))
            continue
        if gpu_dist is not None:
            gdist = gpu_dist[r][: len(gv)]
            if np.any(np.diff(gdist) < 0):
                bad.append((int(i), "gpu distances not sorted"))
                continue
        if len(ov) == 0:
            continue
        dK = od[r, len(ov) - 1]
        extra = set(gv.tolist()) - set(ov.tolist())
        missing = set(ov.tolist()) - set(gv.tolist())
        if extra:
            dx = gd64[r][[k for k, v in enumerate(g) if v in extra]]
            if np.any(dx > dK + tau * abs(dK) + floor):
                bad.append((int(i), "extra id beyond K-th"))
                continue
        if missing:
            dm = od[r][[k for k, v in enumerate(o) if v in missing]]
            if np.any(dm < dK - tau * abs(dK) - floor):
                bad.append((int(i), "missing id well inside K-th"))
                continue
        diff = np.abs(gd64[r][: len(ov)] - od[r][: len(ov)])
        if np.any(diff > tau * np.maximum(np.abs(od[r][: len(ov)]), floor)):
            bad.append((int(i), "position distance mismatch"))
    return bad


def recall(gpu_nbr, ora_nbr):
    """Mean |gpu set ∩ oracle set| / K over rows (valid ids only)."""
    hit = tot = 0
    for g, o in zip(gpu_nbr, ora_nbr):
        ov = set(o[o >= 0].tolist())
        hit += len(ov & set(g[g >= 0].tolist()))
        tot += len(ov)
    return hit / max(tot, 1)


def l2_form_violations(X64, rows, gpu_nbr, ora_dist, tau=TAU):
    """Rows of an IP result whose per-position distances differ from the
    oracle's by more than tau relative in the L2 form 2 + 2 delta."""
    rows = np.asarray(rows)
    K = ora_dist.shape[1]
    gd = oracle.pair_dist(X64, np.repeat(rows[:, None], K, 1), gpu_nbr, oracle.IP)
    a, b = 2 + 2 * gd, 2 + 2 * ora_dist
    ok = np.isfinite(b)
    floor = 1e-6 * np.median(b[ok])
    viol = (np.abs(a - b) > tau * np.maximum(b, floor)) & ok
    return np.nonzero(viol.any(1))[0]
