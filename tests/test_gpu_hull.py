"""Both hoods from one read, and the convex hull: GPU against the oracle.

The plan flag UH_FLAG_BOTH_HOODS makes every tile wave compute the upper hood
and, on the mirrored points, the lower hood of its points; ``convex_hull``
joins the two.  Every result is compared index for index with the oracle
(whose lower hood and hull are pinned in test_oracle_hull.py).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1203_5004_amd as uh  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uh.load_library()


def _dev(xy):
    return torch.from_numpy(np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)).cuda()


def both_hoods(pts, off, strip=0, fan_in=0, flags=0, with_stats=False):
    flags |= uh.UH_FLAG_BOTH_HOODS
    plan = uh.upper_hull_plan_create(off, strip=strip, fan_in=fan_in, flags=flags)
    N, S = int(off[-1]), len(off) - 1
    out = torch.full((max(2 * N, 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((2 * S,), -7, dtype=torch.int32, device="cuda")
    stats = uh.new_stats(2 * S) if with_stats else None
    plan.run(_dev(pts), out, cnt, stats)
    torch.cuda.synchronize()
    res = (out.cpu().numpy(), cnt.cpu().numpy())
    plan.close()
    return res + ((stats.cpu().numpy(),) if with_stats else ())


def assert_both_equal(pts, off, out, cnt):
    N, S = int(off[-1]), len(off) - 1
    for half, ref_fn in ((0, oracle.upper_hull_batched), (1, oracle.lower_hull_batched)):
        ref_out, ref_cnt = ref_fn(pts, off)
        got_cnt = cnt[half * S:(half + 1) * S]
        assert np.array_equal(got_cnt, ref_cnt.astype(np.int32)), f"half {half}: counts differ"
        for s in range(S):
            a, c = int(off[s]), int(got_cnt[s])
            if not np.array_equal(out[half * N + a:half * N + a + c], ref_out[a:a + c]):
                raise AssertionError(f"half {half}, set {s}: indices differ")


def gpu_convex(xy):
    idx, cnt = uh.convex_hull(_dev(xy))
    torch.cuda.synchronize()
    c = int(cnt.item())
    return c, idx[:max(c, 0)].cpu().numpy()


def _mixed_sets(seed):
    rng = np.random.default_rng(seed)
    sets = [np.zeros((0, 2), np.float32), synth.lattice_points(1, 4, seed=seed),
            synth.lattice_points(3, 4, seed=seed + 1), synth.lattice_points(40, 8, seed=seed + 2)]
    for k in range(10):
        n = int(rng.integers(2, 9000))
        kind = k % 3
        if kind == 0:
            sets.append(synth.uniform(n, 20, seed=seed + 10 + k))
        elif kind == 1:
            sets.append(synth.arc(n, 20, 4, seed=seed + 10 + k))
        else:
            sets.append(synth.lattice_points(n, 64, seed=seed + 10 + k))
    return synth.concat_sets(sets)


# ------------------------------------------------------------- batched plan
@pytest.mark.parametrize("strip", [4, 8, 16, 32])
def test_both_hoods_mixed_sets_every_strip(strip):
    pts, off = _mixed_sets(100 + strip)
    out, cnt = both_hoods(pts, off, strip=strip)
    assert_both_equal(pts, off, out, cnt)


@pytest.mark.parametrize("fan_in", [2, 16, 256])
def test_both_hoods_fan_in(fan_in):
    pts, off = synth.concat_sets([synth.uniform(70001, 20, seed=5), synth.arc(50000, 20, 4, seed=6),
                                  synth.parabola(40000, 20, 1, seed=7)])
    out, cnt = both_hoods(pts, off, fan_in=fan_in)
    assert_both_equal(pts, off, out, cnt)


def test_both_hoods_single_set_several_tiles_and_ragged_tail():
    for n in (1, 2, 1023, 1024, 1025, 4097, 65536 + 17):
        pts = synth.uniform(n, 20, seed=n)
        off = np.array([0, n], np.int64)
        out, cnt = both_hoods(pts, off)
        assert_both_equal(pts, off, out, cnt)


def test_both_hoods_equal_x_runs_and_duplicates():
    # the 2^-27 grid forces runs of equal x; lattices add identical points
    pts, off = synth.concat_sets([synth.uniform_iid(300000, 27, seed=9),
                                  synth.lattice_points(5000, 16, seed=10),
                                  synth.lattice_points(3000, 4, seed=11)])
    out, cnt = both_hoods(pts, off)
    assert_both_equal(pts, off, out, cnt)


@pytest.mark.parametrize("strip", [8, 16, 32])
def test_upper_hood_of_convex_arms(strip):
    # a U-shaped set: the upper hood is a few corners, and most tiles lie on
    # a falling or rising convex arm (the tile kernel's chord test)
    u = synth.parabola(200000, 20, 1, seed=50)
    u[:, 1] = -u[:, 1]
    fall = u[:100000].copy()
    pts, off = synth.concat_sets([u, fall, u[100000:].copy()])
    out, cnt = both_hoods(pts, off, strip=strip)
    assert_both_equal(pts, off, out, cnt)


def test_upper_half_matches_the_upper_only_plan():
    pts, off = _mixed_sets(7)
    out, cnt = both_hoods(pts, off)
    plan = uh.upper_hull_plan_create(off)
    N, S = int(off[-1]), len(off) - 1
    o1 = torch.zeros(max(N, 1), dtype=torch.int32, device="cuda")
    c1 = torch.zeros(S, dtype=torch.int32, device="cuda")
    plan.run(_dev(pts), o1, c1)
    torch.cuda.synchronize()
    c1 = c1.cpu().numpy()
    assert np.array_equal(cnt[:S], c1)
    o1 = o1.cpu().numpy()
    for s in range(S):
        a = int(off[s])
        assert np.array_equal(out[a:a + c1[s]], o1[a:a + c1[s]])
    plan.close()


def test_both_hoods_force_fallback_and_stats():
    pts, off = synth.concat_sets([synth.arc(30000, 20, 4, seed=12), synth.parabola(20000, 20, 1, seed=13)])
    out, cnt, st = both_hoods(pts, off, with_stats=True)
    assert_both_equal(pts, off, out, cnt)
    assert np.all(st[:, 1] <= st[:, 0]) and st[:, 0].sum() > 0
    out2, cnt2, st2 = both_hoods(pts, off, flags=uh.UH_FLAG_FORCE_FALLBACK, with_stats=True)
    assert np.array_equal(cnt, cnt2) and np.array_equal(out, out2)
    assert np.array_equal(st2[:, 0], st2[:, 1])  # every test took the exact path


def test_both_hoods_data_errors_reach_both_halves():
    good = synth.uniform(5000, 20, seed=14)
    bad = good.copy()
    bad[2500, 0] = bad[10, 0]  # x decreases
    pts, off = synth.concat_sets([good, bad, good])
    out, cnt = both_hoods(pts, off)
    S = 3
    assert cnt[1] == uh.UH_ERR_UNSORTED and cnt[S + 1] == uh.UH_ERR_UNSORTED
    assert cnt[0] > 0 and cnt[S] > 0 and cnt[2] > 0 and cnt[S + 2] > 0


def test_both_hoods_graph_replays():
    pts, off = _mixed_sets(21)
    N, S = int(off[-1]), len(off) - 1
    plan = uh.upper_hull_plan_create(off, flags=uh.UH_FLAG_BOTH_HOODS | uh.UH_FLAG_GRAPH)
    d = _dev(pts)
    out = torch.zeros(2 * N, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(2 * S, dtype=torch.int32, device="cuda")
    for _ in range(3):
        out.fill_(-5)
        cnt.fill_(-5)
        torch.cuda.synchronize()
        plan.run(d, out, cnt)
        torch.cuda.synchronize()
        assert_both_equal(pts, off, out.cpu().numpy(), cnt.cpu().numpy())
    plan.close()


def test_both_hoods_buffers_too_small_are_rejected():
    off = np.array([0, 100], np.int64)
    plan = uh.upper_hull_plan_create(off, flags=uh.UH_FLAG_BOTH_HOODS)
    d = _dev(synth.uniform(100, 20, seed=1))
    with pytest.raises(ValueError):
        plan.run(d, torch.zeros(100, dtype=torch.int32, device="cuda"),
                 torch.zeros(2, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        plan.run(d, torch.zeros(200, dtype=torch.int32, device="cuda"),
                 torch.zeros(1, dtype=torch.int32, device="cuda"))
    plan.close()


# -------------------------------------------------------------- convex hull
def test_convex_hull_small_cases():
    cases = [np.zeros((0, 2)), [[0.5, 0.25]], [[0.25, 0.5], [0.75, -0.5]],
             [[0.5, 0.75], [0.5, -0.25]], [[0.5, 0.25]] * 3,
             [[0.0, 0.0], [0.0, 0.5], [1.0, 0.0]],
             [[0.0, 0.0], [0.0, 1.0], [0.5, 0.5], [1.0, -1.0], [1.0, 1.0]]]
    for xy in cases:
        xy = np.asarray(xy, np.float32).reshape(-1, 2)
        c, idx = gpu_convex(xy)
        ref = oracle.convex_hull(xy)
        assert c == len(ref) and list(idx) == list(ref), xy


def test_convex_hull_lattices():
    for seed in range(40):
        xy = synth.lattice_points(1 + seed % 30, (4, 8, 16, 32)[seed % 4], seed=300 + seed)
        c, idx = gpu_convex(xy)
        assert list(idx) == list(oracle.convex_hull(xy)), seed


@pytest.mark.parametrize("name", ["uniform", "arc", "parabola", "iid27"])
def test_convex_hull_workload_recipes(name):
    xy = {"uniform": lambda: synth.uniform(300000, 20, seed=31),
          "arc": lambda: synth.arc(200000, 24, 4, seed=32),
          "parabola": lambda: synth.parabola(150000, 20, 1, seed=33),
          "iid27": lambda: synth.uniform_iid(400000, 27, seed=34)}[name]()
    c, idx = gpu_convex(xy)
    ref = oracle.convex_hull(xy)
    assert c == len(ref)
    assert np.array_equal(idx, ref)


def test_convex_hull_data_error_and_reuse():
    xy = synth.uniform(3000, 20, seed=40)
    bad = xy.copy()
    bad[7, 1] = 3.0  # y out of range
    c, _ = gpu_convex(bad)
    assert c == uh.UH_ERR_RANGE
    c, idx = gpu_convex(xy)  # the cached plan is clean again
    assert np.array_equal(idx, oracle.convex_hull(xy))
