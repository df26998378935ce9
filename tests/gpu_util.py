"""Shared helpers for the GPU tests: device upload and oracle comparison."""
import numpy as np
import torch

import oracle


def to_dev(t):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(t.u).to(dev), torch.from_numpy(t.v).to(dev), torch.from_numpy(t.w).to(dev))


def gpu_dendrogram(t):
    import paper_2401_06089_amd as pd
    u, v, w = to_dev(t)
    ep, vp = pd.dendrogram(u, v, w, n=t.n)
    torch.cuda.synchronize()
    return ep.cpu().numpy(), vp.cpu().numpy()


def assert_matches_oracle(t, tag=""):
    ep, vp = gpu_dendrogram(t)
    oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    if not np.array_equal(vp, ovp):
        bad = np.flatnonzero(vp != ovp)
        raise AssertionError(f"{tag} vertex_parent differs at {len(bad)} of {t.n}: first {bad[:5]} "
                             f"gpu {vp[bad[:5]]} oracle {ovp[bad[:5]]}")
    if not np.array_equal(ep, oep):
        bad = np.flatnonzero(ep != oep)
        raise AssertionError(f"{tag} edge_parent differs at {len(bad)} of {t.m}: first {bad[:5]} "
                             f"gpu {ep[bad[:5]]} oracle {oep[bad[:5]]}")
    return ep, vp
