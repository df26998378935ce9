"""The largest accepted tree (about 1.07e9 vertices): the level tables' int32
ids reach their limit.  The oracle cannot run at this size, so a monotone
path is checked against its closed form and a random recursive tree built on
the device against properties that hold at any size."""
import pytest
import torch

pytestmark = pytest.mark.gpu

N_MAX = 1_073_700_000


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    pd.library()
    free, _ = torch.cuda.mem_get_info()
    if free < 180 * 2**30:
        pytest.skip("needs about 180 GB of free device memory")
    yield
    pd.release_workspaces()
    torch.cuda.empty_cache()


def weight_key(w):
    """Monotone int64 image of fp32 weights (-0.0 folded onto +0.0)."""
    b = w.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    b = torch.where(b == 0x80000000, torch.zeros_like(b), b)
    return torch.where(b >= 0x80000000, 0xFFFFFFFF - b, b | 0x80000000)


def test_largest_monotone_path_is_one_chain():
    import paper_2401_06089_amd as pd
    n = N_MAX
    dev = torch.device("cuda:0")
    u = torch.arange(0, n - 1, dtype=torch.int32, device=dev)
    v = u + 1
    w = torch.arange(0, n - 1, dtype=torch.float32, device=dev)   # ties above 2^24 fall to the id
    ep, vp = pd.dendrogram(u, v, w, n=n)
    assert pd.workspace_bytes(n) > 0
    assert int(ep[-1]) == -1
    assert torch.equal(ep[:-1], u[1:])                    # edge i hangs under edge i+1
    assert int(vp[0]) == 0
    assert torch.equal(vp[1:], u)                         # vertex x under edge x-1
    del u, v, w, ep, vp
    pd.release_workspaces()
    torch.cuda.empty_cache()


def test_largest_random_recursive_tree_properties():
    import paper_2401_06089_amd as pd
    n = N_MAX
    m = n - 1
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    i = torch.arange(1, n, dtype=torch.int64, device=dev)
    par = (torch.rand(m, generator=g, device=dev, dtype=torch.float64) * i).to(torch.int32)
    u = i.to(torch.int32)
    del i
    w = torch.rand(m, generator=g, device=dev, dtype=torch.float32)
    ep, vp = pd.dendrogram(u, par, w, n=n)

    ids = torch.arange(m, dtype=torch.int64, device=dev)
    assert m < 2**30
    key = (weight_key(w) << 30) | ids                    # the total order (w, id), below 2^62
    # exactly one root; every other edge hangs under a strictly heavier edge
    root = ep < 0
    assert int(root.sum()) == 1
    p = ep.clamp(min=0).to(torch.int64)
    assert bool((key[p] > key)[~root].all())
    # every edge node has exactly two children among edges and vertices
    kids = torch.bincount(p[~root], minlength=m) + torch.bincount(vp.to(torch.int64), minlength=m)
    assert bool((kids == 2).all())
    del p, kids, root
    # a vertex hangs under its lightest incident edge
    vpl = vp.to(torch.int64)
    assert bool(((u[vpl].to(torch.int64) == torch.arange(n, device=dev)) |
                 (par[vpl].to(torch.int64) == torch.arange(n, device=dev))).all())
    best = torch.full((n,), torch.iinfo(torch.int64).max, dtype=torch.int64, device=dev)
    best.scatter_reduce_(0, u.to(torch.int64), key, reduce="amin")
    best.scatter_reduce_(0, par.to(torch.int64), key, reduce="amin")
    assert torch.equal(best, key[vpl])
