"""GPU parity of user-mesh half-edges (Sec. 4.3, option 1) through the C
ABI: bit-exact against the oracle on organized meshes at their real sizes
(where it is also Alg. 2's HE from pl_mesh_opc), on shuffled and relabelled
meshes with fins, repeated and reversed triangles and degenerate edges, on
random soups over few points, and for ragged triangle counts."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
UNTOUCHED = -77


@pytest.fixture(scope="module")
def pl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2007_12065_amd as pl
    return pl


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def say(*a):
    print("[case]", *a, flush=True)


def gpu_he(pl, tris, n=None):
    import torch
    cap = len(tris)
    out = torch.full((max(3 * cap, 1),), UNTOUCHED, dtype=torch.int32, device="cuda:0")
    nd = None if n is None else torch.tensor([n], dtype=torch.int32, device="cuda:0")
    he = pl.pl_user_halfedges(to_dev(np.asarray(tris, dtype=np.int32).reshape(-1, 3)), nd, out=out)
    torch.cuda.synchronize()
    return he.cpu().numpy()


@pytest.mark.parametrize("kind", ["rgbd", "lidar", "lidar128"])
def test_organized_meshes(pl, orc, kind):
    import torch
    p = synth.make_frame(kind, 31)
    tri_map, T = orc.mesh(p)
    M, N = p.shape[:2]
    want = orc.halfedges(tri_map, M, N, len(T))
    say("user halfedges", kind, len(T))
    got = gpu_he(pl, T)
    assert np.array_equal(got, want)
    assert np.array_equal(got, oracle.user_halfedges(T))
    m = pl.pl_mesh_opc(to_dev(p))
    torch.cuda.synchronize()
    assert np.array_equal(got, m["halfedges"][:3 * len(T)].cpu().numpy())


def _messy_mesh(orc, rng):
    """An organized mesh shuffled and relabelled, with fins (third
    triangles on existing edges), repeated and reversed triangles and
    degenerate ones."""
    p = synth.random_grid(60, 90, 5, nan_frac=0.1)
    _, T = orc.mesh(p)
    relabel = rng.permutation(60 * 90).astype(np.int32)
    T = relabel[T]
    extra = []
    pick = rng.choice(len(T), 400, replace=False)
    for k, t in enumerate(pick):
        a, b, c = T[t]
        if k % 4 == 0:
            extra.append([b, a, 60 * 90 + k])         # a fin on edge a-b
        elif k % 4 == 1:
            extra.append([a, b, c])                   # repeated triangle
        elif k % 4 == 2:
            extra.append([a, c, b])                   # reversed triangle
        else:
            extra.append([a, a, b])                   # degenerate
    T = np.concatenate([T, np.array(extra, dtype=np.int32)])
    return T[rng.permutation(len(T))]


def test_non_manifold_and_shuffled(pl, orc):
    rng = np.random.default_rng(11)
    T = _messy_mesh(orc, rng)
    say("user halfedges messy", len(T))
    got = gpu_he(pl, T)
    want = oracle.user_halfedges(T)
    assert np.array_equal(got, want), np.count_nonzero(got != want)
    assert (want == -1).sum() > 1000


@pytest.mark.parametrize("seed,n,span", [(1, 5000, 40), (2, 100000, 300), (3, 3000, 6)])
def test_random_soups(pl, seed, n, span):
    rng = np.random.default_rng(seed)
    T = rng.integers(-span // 4, span, size=(n, 3)).astype(np.int32)
    say("user halfedges soup", n, span)
    got = gpu_he(pl, T)
    assert np.array_equal(got, oracle.user_halfedges(T))


def test_ragged_counts(pl, orc):
    p = synth.random_grid(20, 30, 9, nan_frac=0.2)
    _, T = orc.mesh(p)
    cap = len(T)
    for n in (cap, cap - 1, 1, 0, cap + 5, -2):
        say("user halfedges n", n, "cap", cap)
        got = gpu_he(pl, T, n)
        m = min(max(n, 0), cap)
        assert np.array_equal(got[:3 * m], oracle.user_halfedges(T[:m]))
        assert np.all(got[3 * m:3 * cap] == UNTOUCHED)


# The partitioned way's rare paths.  These tests know the library's bucket
# rule: 2^lg buckets, lg the least with 2^lg >= 3 cap / 2048, and a key's
# bucket the top lg bits of the 64-bit MurmurHash3 finaliser of
# (lo << 32 | hi), lo < hi as int32.

_M1, _M2, _MASK = 0xff51afd7ed558ccd, 0xc4ceb9fe1a85ec53, (1 << 64) - 1


def _mix(k):
    k ^= k >> 33
    k = (k * _M1) & _MASK
    k ^= k >> 33
    k = (k * _M2) & _MASK
    return k ^ (k >> 33)


def _unmix(v):
    """Inverse of _mix: x ^ (x >> 33) undoes itself, the products are
    undone by the inverses of the odd constants modulo 2^64."""
    v ^= v >> 33
    v = (v * pow(_M2, -1, 1 << 64)) & _MASK
    v ^= v >> 33
    v = (v * pow(_M1, -1, 1 << 64)) & _MASK
    return v ^ (v >> 33)


def _signed(u):
    return u - (1 << 32) if u >= 1 << 31 else u


def test_unmix_inverts_mix():
    rng = np.random.default_rng(5)
    for v in rng.integers(0, 1 << 63, size=100, dtype=np.int64):
        assert _mix(_unmix(int(v))) == int(v)


def test_overflowing_bucket(pl):
    """5000 triangles on one edge (0, 1), some reversed: the edge's bucket
    gets more entries than its region holds and reads the overflow list."""
    rng = np.random.default_rng(21)
    k = np.arange(2, 5002, dtype=np.int32)
    T = np.stack([np.zeros_like(k), np.ones_like(k), k], axis=1)
    flip = rng.random(len(T)) < 0.3
    T[flip, 0], T[flip, 1] = 1, 0
    T = T[rng.permutation(len(T))]
    say("user halfedges overflow", len(T))
    got = gpu_he(pl, T)
    want = oracle.user_halfedges(T)
    assert np.array_equal(got, want)
    assert (want >= 0).sum() > 0


def test_full_lds_table_falls_back(pl):
    """More distinct keys in one bucket than its LDS table has slots (keys
    built by inverting the hash): the global-table fallback redoes the mesh,
    with the same result as the oracle."""
    import torch
    cap, lg, n = 20000, 5, 4600
    assert (1 << lg) >= 3 * cap / 2048 > (1 << (lg - 1))
    rng = np.random.default_rng(8)
    edges = set()
    while len(edges) < n:
        v = int(rng.integers(0, 1 << (64 - lg)))        # top lg bits zero: bucket 0
        key = _unmix(v)
        lo, hi = _signed(key >> 32), _signed(key & 0xffffffff)
        if lo < hi:
            edges.add((lo, hi))
    E = np.array(sorted(edges), dtype=np.int64)
    third = rng.integers(-1000, 1000, size=len(E))
    T = np.zeros((cap, 3), dtype=np.int32)
    T[:n] = np.stack([E[:, 0], E[:, 1], third], axis=1).astype(np.int32)
    # a twin for every fifth crafted edge
    T[n:n + n // 5] = np.stack([E[::5, 1], E[::5, 0], third[::5] + 7], axis=1)[:n // 5].astype(np.int32)
    m = n + n // 5
    say("user halfedges lds fallback", m, "cap", cap)
    got = gpu_he(pl, T, m)
    want = oracle.user_halfedges(T[:m])
    assert np.array_equal(got[:3 * m], want)
    assert np.all(got[3 * m:] == UNTOUCHED)
    assert (want >= 0).sum() >= 2 * (n // 5)


def test_global_table_way(pl):
    """A capacity past the partitioned way's bound (more than 8192 buckets):
    the global table, on the first rows."""
    cap = 6_000_000
    assert 3 * cap / 2048 > 8192
    rng = np.random.default_rng(4)
    m = 60000
    T = np.zeros((cap, 3), dtype=np.int32)
    T[:m] = rng.integers(-500, 4000, size=(m, 3))
    say("user halfedges global table", m, "cap", cap)
    got = gpu_he(pl, T, m)
    assert np.array_equal(got[:3 * m], oracle.user_halfedges(T[:m]))
    assert np.all(got[3 * m:3 * m + 1000] == UNTOUCHED)
