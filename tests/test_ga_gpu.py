"""GPU parity of the Gaussian accumulator (Sec. 6.1, Alg. 3) through the C ABI.

Cell choice is an integer decided in float32, so with the same float32 cell
normals the kernel's cells and counts equal the oracle's brute force bit for
bit: random unit normals, normals on and between cells, near the cube-map
bin and face boundaries, lengths around the table's [0.5, 2] range, NaN and
infinite normals, float16 normals, strides and device-side counts, and the
smoothed normals of a synthetic frame.  The library's own icosahedron is
compared with the oracle's cell by cell."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def unit_rows(x):
    x = np.asarray(x, dtype=np.float64)
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def hard_normals(C, rng, n_random=40000):
    """Random directions plus the awkward ones: on cells, on midpoints of
    neighbouring cells, on cube-face edges and corners, on bin boundaries,
    and lengths just inside and outside [0.5, 2]."""
    c = C.astype(np.float64)
    parts = [unit_rows(rng.normal(size=(n_random, 3))), c]
    j = rng.integers(0, len(c), size=2000)
    k = np.argsort(-(c[j] @ c.T), axis=1)[:, 1]            # nearest other cell
    parts.append(unit_rows(c[j] + c[k]))                     # equidistant (up to rounding)
    parts.append(unit_rows(c[j] + c[k] + 1e-7 * rng.normal(size=(2000, 3))))
    e = rng.uniform(-1, 1, size=(3000, 3))
    e[:1000, 0] = e[:1000, 1]                                # |x| = |y|: face edges
    e[1000:2000] = np.sign(e[1000:2000])                     # cube corners
    g = 128
    e[2000:, 1] = np.round(e[2000:, 1] * g / 2) * 2 / g      # bin boundaries
    e[2000:, 0] = 1.0
    parts.append(unit_rows(e))
    base = np.concatenate(parts)
    scales = rng.choice([1.0, 0.5, 0.4999, 0.5001, 2.0, 1.9999, 2.0001, 0.3, 3.0, 1e-20],
                        size=len(base), p=[0.82] + [0.02] * 9)
    out = (base * scales[:, None]).astype(np.float32)
    out[:5] = [[np.nan, 0, 1], [0, np.inf, 0], [0, 0, 0], [-np.inf, 1, 1], [1, np.nan, np.nan]]
    return out


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_library_cells_equal_oracle_cells(pl, level):
    say("ga cells level", level)
    ga = pl.GaussianAccumulator(level)
    mine = ga.cells().cpu().numpy().astype(np.float64)
    _, _, ref = oracle.ga_icosahedron(level)
    ref = ref.astype(np.float64)
    assert mine.shape == ref.shape
    # a bijection: every library cell has one oracle cell within 1e-6 and
    # no two library cells share it
    nearest = np.empty(len(mine), dtype=np.int64)
    for s in range(0, len(mine), 2048):
        nearest[s:s + 2048] = np.argmax(mine[s:s + 2048] @ ref.T, axis=1)
    assert np.abs(mine - ref[nearest]).max() < 1e-6
    assert len(np.unique(nearest)) == len(mine)
    ga.close()


@pytest.mark.parametrize("level", [1, 3, 4, 5])
def test_integrate_parity_oracle_cells(pl, level):
    import torch
    _, _, C = oracle.ga_icosahedron(level)
    rng = np.random.default_rng(50 + level)
    N = hard_normals(C, rng)
    ga = pl.GaussianAccumulator(cells=C)
    for nd in (np.float32, np.float16):
        x = N.astype(nd)
        say("ga integrate level", level, nd.__name__, len(x))
        counts, cells = ga.integrate(to_dev(x), cell_out=True)
        torch.cuda.synchronize()
        want_idx, want_counts = oracle.ga_integrate(C, x.astype(np.float32))
        got_idx = cells.cpu().numpy()
        assert np.array_equal(got_idx, want_idx), np.count_nonzero(got_idx != want_idx)
        assert np.array_equal(counts.cpu().numpy(), want_counts)
    ga.close()


def test_integrate_stride_count_and_accumulation(pl):
    import torch
    _, _, C = oracle.ga_icosahedron(3)
    rng = np.random.default_rng(9)
    N = unit_rows(rng.normal(size=(10001, 3))).astype(np.float32)
    ga = pl.GaussianAccumulator(cells=C)
    xd = to_dev(N)
    for n, stride in ((10001, 1), (10001, 3), (9000, 8), (7, 8), (1, 1), (0, 1), (20000, 5), (-3, 2)):
        say("ga stride", stride, "n", n)
        nd = torch.tensor([n], dtype=torch.int32, device="cuda:0")
        counts, cells = ga.integrate(xd, n=nd, stride=stride, cell_out=True)
        torch.cuda.synchronize()
        m = min(max(n, 0), len(N))
        want_idx, want_counts = oracle.ga_integrate(C, N[:m], stride=stride)
        rows = len(want_idx)
        assert np.array_equal(cells.cpu().numpy()[:rows], want_idx)
        assert np.array_equal(counts.cpu().numpy(), want_counts)
    # counts are added to, not overwritten
    say("ga accumulation")
    counts, _ = ga.integrate(xd)
    counts, _ = ga.integrate(xd, counts=counts)
    torch.cuda.synchronize()
    _, once = oracle.ga_integrate(C, N)
    assert np.array_equal(counts.cpu().numpy(), 2 * once)
    ga.close()


def test_integrate_scene_normals(pl, orc):
    """The smoothed normals of a 480x640 frame (the oracle's, float32),
    sampled every 8th row, into a level-4 accumulator: identical to the
    oracle; the fullest cells are those nearest the scene's planes."""
    import torch
    k = synth.KINDS["rgbd"]
    p = synth.make_frame("rgbd", 1002)
    r = orc.pipeline(p, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                     k.sigma_angle, k.iters_bil, threads=8)
    nT = r["normals_T"].astype(np.float32)
    _, _, C = oracle.ga_icosahedron(4)
    ga = pl.GaussianAccumulator(cells=C)
    say("ga scene normals", len(nT))
    counts, cells = ga.integrate(to_dev(nT), stride=8, cell_out=True)
    torch.cuda.synchronize()
    want_idx, want_counts = oracle.ga_integrate(C, nT, stride=8)
    assert np.array_equal(cells.cpu().numpy(), want_idx)
    got = counts.cpu().numpy()
    assert np.array_equal(got, want_counts)
    # the fullest cell lies on a scene plane, and each plane (floor, two
    # walls) gathers a share of the samples in the cells within 5 deg of it
    planes = synth.scene_planes("rgbd", 1002).astype(np.float64)
    ang = np.degrees(np.arccos(np.clip(C.astype(np.float64) @ planes.T, -1, 1)))
    assert ang[int(np.argmax(got))].min() < 2.0
    share = [got[ang[:, j] < 5.0].sum() / got.sum() for j in range(len(planes))]
    assert min(share) > 0.03, share
    ga.close()


def test_library_level_matches_oracle_counts(pl):
    """Level 4 with the library's own cells: per-cell counts equal the
    oracle's (cells matched by normal) for directions whose nearest and
    second-nearest cells differ by more than 1e-6 in distance."""
    import torch
    ga = pl.GaussianAccumulator(4)
    mine = ga.cells().cpu().numpy().astype(np.float64)
    _, _, C = oracle.ga_icosahedron(4)
    ref = C.astype(np.float64)
    match = np.argmax(mine @ ref.T, axis=1)                 # library cell -> oracle cell
    rng = np.random.default_rng(77)
    N = unit_rows(rng.normal(size=(20000, 3))).astype(np.float32)
    say("ga library level 4")
    _, cells = ga.integrate(to_dev(N), cell_out=True)
    torch.cuda.synchronize()
    got = match[cells.cpu().numpy()]
    want, _ = oracle.ga_integrate(C, N)
    d = np.sort(np.linalg.norm(N.astype(np.float64)[:, None] - ref[None], axis=2), axis=1)
    clear = d[:, 1] - d[:, 0] > 1e-6
    assert clear.mean() > 0.99
    assert np.array_equal(got[clear], want[clear])
    ga.close()


def test_integrate_large_input(pl):
    """An input large enough for four rows per thread (the launch shape of a
    full frame's normals), level 3, float32 and float16: identical to the
    oracle."""
    import torch
    _, _, C = oracle.ga_icosahedron(3)
    rng = np.random.default_rng(123)
    N = np.concatenate([hard_normals(C, rng, n_random=300000)])
    ga = pl.GaussianAccumulator(cells=C)
    for nd in (np.float32, np.float16):
        x = N.astype(nd)
        say("ga large input", len(x), nd.__name__)
        counts, cells = ga.integrate(to_dev(x), cell_out=True)
        torch.cuda.synchronize()
        want_idx, want_counts = oracle.ga_integrate(C, x.astype(np.float32))
        assert np.array_equal(cells.cpu().numpy(), want_idx)
        assert np.array_equal(counts.cpu().numpy(), want_counts)
    ga.close()


@pytest.mark.parametrize("n_cells,seed", [(700, 1), (37, 2), (5000, 3)])
def test_arbitrary_cell_sets(pl, n_cells, seed):
    """The candidate tables hold for any unit cell set, not only icosahedra:
    random directions (uneven spacing), with near-duplicates and exact
    duplicates, against the oracle's brute force."""
    import torch
    rng = np.random.default_rng(seed)
    C = unit_rows(rng.normal(size=(n_cells, 3)))
    C[-3] = C[0]                                           # an exact duplicate
    C[-2] = unit_rows((C[1] + 1e-6 * rng.normal(size=3))[None])[0]   # a near-duplicate
    C = C.astype(np.float32)
    N = hard_normals(C, rng, n_random=30000)
    ga = pl.GaussianAccumulator(cells=C)
    say("ga arbitrary cells", n_cells)
    counts, cells = ga.integrate(to_dev(N), cell_out=True)
    torch.cuda.synchronize()
    want_idx, want_counts = oracle.ga_integrate(C, N)
    assert np.array_equal(cells.cpu().numpy(), want_idx)
    assert np.array_equal(counts.cpu().numpy(), want_counts)
    ga.close()
