"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Every comparison is exact: corner indices are integers, so the bar is
bit-exact equality with the oracle (and, where noted, with brute force or
the definitions in oracle.bridge).  All calls go through the C ABI via the
thin Python binding.
"""
import ctypes
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import bridge as B
from oracle import invariants
from tests import golden_io

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


def gpu_hull(xy):
    idx, cnt = uh.upper_hull(_dev(xy))
    torch.cuda.synchronize()
    c = int(cnt.item())
    return c, idx[:max(c, 0)].cpu().numpy()


def gpu_batched(pts, off, strip=0, fan_in=0, flags=0, with_stats=False):
    plan = uh.upper_hull_plan_create(off, strip=strip, fan_in=fan_in, flags=flags)
    d = _dev(pts)
    S = len(off) - 1
    out = torch.full((max(int(off[-1]), 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((S,), -7, dtype=torch.int32, device="cuda")
    stats = uh.new_stats(S) if with_stats else None
    plan.run(d, out, cnt, stats)
    torch.cuda.synchronize()
    res = (out.cpu().numpy(), cnt.cpu().numpy())
    if with_stats:
        res = res + (stats.cpu().numpy(),)
    plan.close()
    return res


def assert_batched_equal(pts, off, out, cnt):
    ref_out, ref_cnt = oracle.upper_hull_batched(pts, off)
    assert np.array_equal(cnt, ref_cnt.astype(np.int32)), "counts differ"
    for s in range(len(off) - 1):
        a, c = int(off[s]), int(cnt[s])
        if not np.array_equal(out[a:a + c], ref_out[a:a + c]):
            raise AssertionError(f"set {s}: indices differ")


def assert_parity(xy):
    c, idx = gpu_hull(xy)
    ref = oracle.upper_hull(xy)
    assert c == len(ref), (c, len(ref))
    assert np.array_equal(idx, ref)


# ------------------------------------------------------------ small cases
@pytest.mark.parametrize("path", golden_io.all_fixtures(), ids=lambda p: p.split("/")[-1])
def test_golden_fixtures(path):
    xy, expect = golden_io.load(path)
    c, idx = gpu_hull(xy)
    assert list(idx) == list(expect)


def test_tiny_edge_cases():
    cases = [
        np.zeros((0, 2)), [[0.5, 0.25]], [[0.0, 0.0], [1.0, 0.0]],
        [[0.5, 0.0], [0.5, 0.25]], [[0.5, 0.25], [0.5, 0.0]],
        [[0.5, 0.25], [0.5, 0.25], [0.5, 0.25]],
        [[0.0, -1.0], [1.0, 1.0]], [[0.0, 1.0], [1.0, -1.0]],
    ]
    for xy in cases:
        xy = np.asarray(xy, np.float32).reshape(-1, 2)
        c, idx = gpu_hull(xy)
        assert c == len(oracle.upper_hull(xy))
        assert list(idx) == list(oracle.upper_hull(xy)), xy


def _lattice_sets():
    pts = [(x, y) for x in range(3) for y in range(3)]
    seen, sets = set(), []
    for n in range(1, 6):
        for combo in itertools.product(pts, repeat=n):
            seq = tuple(sorted(combo, key=lambda p: p[0]))
            if seq not in seen:
                seen.add(seq)
                sets.append(synth.from_integers([p[0] for p in seq], [p[1] for p in seq], 2))
    return sets


def test_exhaustive_lattices_batched():
    pts, off = synth.concat_sets(_lattice_sets())
    out, cnt = gpu_batched(pts, off)
    assert_batched_equal(pts, off, out, cnt)


@pytest.mark.parametrize("side", [4, 16, 256])
def test_random_lattices_batched(side):
    sets = [synth.lattice_points(1 + (k % 64), side, seed=k + 977 * side) for k in range(3000)]
    pts, off = synth.concat_sets(sets)
    out, cnt = gpu_batched(pts, off)
    assert_batched_equal(pts, off, out, cnt)


# ------------------------------------------------------------ tiles / rounds
TILE = 64 * 16  # points per tile of the default plan (64 lanes x strip 16)
GROUP = 256 * TILE  # points under one first-pass merge workgroup (fan-in 256)


@pytest.mark.parametrize("n", [TILE - 1, TILE, TILE + 1, 2 * TILE - 1, 2 * TILE + 1,
                               7 * TILE + 3, GROUP + 5, 2 * GROUP + 7])
def test_sizes_around_tiles(n):
    assert_parity(synth.uniform(n, 22, seed=n))
    assert_parity(synth.arc(min(n, 1 << 20), 20, 4, seed=n + 1))


def concave_chain(max_step=100, G=20):
    """A strictly concave chain whose every point is a corner: consecutive
    edge vectors are the primitive (dx, dy), 1 <= dx, |dy| <= max_step,
    in decreasing slope; all coordinates stay below 2^G (exact float32)."""
    from math import gcd
    vec = [(dx, dy) for dx in range(1, max_step + 1) for dy in range(-max_step, max_step + 1)
           if gcd(dx, abs(dy)) == 1]
    vec.sort(key=lambda v: -v[1] / v[0])
    X = np.concatenate([[0], np.cumsum([v[0] for v in vec])])
    Y = np.concatenate([[0], np.cumsum([v[1] for v in vec])])
    Y = Y - Y.min()
    assert X.max() < (1 << G) and Y.max() < (1 << G)
    return synth.from_integers(X, Y, G)


def test_concave_all_corners_global_path():
    # every point is a corner: tile hoods are full, merges exceed LDS
    xy = concave_chain()
    n = len(xy)
    assert n > 2 * TILE
    ref = oracle.upper_hull(xy)
    assert np.array_equal(ref, np.arange(n))
    c, idx = gpu_hull(xy)
    assert c == n and np.array_equal(idx, ref)
    # again with tiny tiles and fan-in 2: many global-memory rounds
    pts, off = synth.concat_sets([xy, xy[: n // 2 + 1]])
    out, cnt = gpu_batched(pts, off, strip=4, fan_in=2)
    assert_batched_equal(pts, off, out, cnt)


def test_equal_x_runs_across_tiles():
    n = 5 * TILE
    X = np.arange(n, dtype=np.int64)
    X[TILE - 300: 3 * TILE + 100] = TILE - 300  # one run spanning three tiles
    X = np.sort(X)
    rng = np.random.default_rng(4)
    Y = rng.integers(0, 1 << 20, n)
    Y[2 * TILE + 17] = (1 << 20) - 1  # the run's top sits mid-run
    Y[2 * TILE + 18] = (1 << 20) - 1  # an identical twin with a higher index
    xy = synth.from_integers(X, Y, 20)
    assert_parity(xy)
    assert_parity(synth.uniform_iid(1 << 20, 27, seed=9))


@pytest.mark.parametrize("strip", [4, 8, 16, 32])
@pytest.mark.parametrize("fan_in", [2, 16, 256])
def test_strip_and_fan_in_invariance(strip, fan_in):
    sets = [synth.uniform(50000, 20, seed=1), synth.arc(70001, 20, 4, seed=2),
            synth.parabola(40000, 20, 1, seed=3), synth.uniform_iid(30000, 27, seed=4)]
    pts, off = synth.concat_sets(sets)
    out, cnt = gpu_batched(pts, off, strip=strip, fan_in=fan_in)
    assert_batched_equal(pts, off, out, cnt)


def test_force_fallback_identical_and_stats():
    sets = [synth.parabola(1 << 16, 20, 1, seed=s) for s in range(4)]
    sets += [synth.uniform(1 << 15, 20, seed=11)]
    pts, off = synth.concat_sets(sets)
    out0, cnt0, st0 = gpu_batched(pts, off, with_stats=True)
    out1, cnt1, st1 = gpu_batched(pts, off, flags=uh.UH_FLAG_FORCE_FALLBACK, with_stats=True)
    assert_batched_equal(pts, off, out0, cnt0)
    assert np.array_equal(cnt0, cnt1) and np.array_equal(out0[:len(pts)], out1[:len(pts)])
    assert np.all(st0[:, 0] > 0) and np.all(st0[:, 1] <= st0[:, 0])
    assert np.array_equal(st1[:, 1], st1[:, 0])  # forced: every test falls back


def test_exact_path_rare_in_general_position():
    # Uniform sets on a fine grid have almost no ambiguous orientation
    # tests: the FP32 filter must decide nearly all of them (no test of a
    # corner against itself, which is an exact zero the filter cannot
    # certify, may reach the exact path).
    sets = [synth.uniform(200000, 22, seed=s) for s in range(4)]
    sets += [synth.uniform(3000, 22, seed=9)]
    pts, off = synth.concat_sets(sets)
    out, cnt, st = gpu_batched(pts, off, with_stats=True)
    assert_batched_equal(pts, off, out, cnt)
    evals, fb = int(st[:, 0].sum()), int(st[:, 1].sum())
    assert evals > 0 and fb <= 0.01 * evals, (evals, fb)


def test_determinism_repeated_runs():
    xy = synth.arc(300000, 20, 4, seed=12)
    c0, i0 = gpu_hull(xy)
    for _ in range(3):
        c1, i1 = gpu_hull(xy)
        assert c1 == c0 and np.array_equal(i0, i1)


def test_replicated_last_merge_repeated_runs():
    # A last merge pass of few items runs each item in several workgroups
    # that share the gathering of a large hood (here some 19 000 and 15 000
    # corners, merged over the workspace).  The replicas count themselves in
    # a word that must be back at zero for the next run, and the last of
    # them clears the set's group maxima: every run of one plan must match.
    a = synth.arc(1 << 20, 24, 4, seed=5)
    b = synth.arc(1 << 19, 24, 4, seed=6)
    u = synth.uniform(1 << 18, 24, seed=7)
    for sets, flags in (([a], 0), ([a, b, u], 0), ([b], uh.UH_FLAG_BOTH_HOODS)):
        pts, off = synth.concat_sets(sets)
        S, N = len(sets), int(off[-1])
        refs = [oracle.upper_hull_batched(pts, off)]
        if flags:
            refs.append(oracle.lower_hull_batched(pts, off))
        H = len(refs)
        plan = uh.upper_hull_plan_create(off, flags=flags)
        d = _dev(pts)
        for run in range(3):
            out = torch.full((H * N,), -7, dtype=torch.int32, device="cuda")
            cnt = torch.full((H * S,), -7, dtype=torch.int32, device="cuda")
            plan.run(d, out, cnt, None)
            torch.cuda.synchronize()
            o, c = out.cpu().numpy(), cnt.cpu().numpy()
            for h, (ref_out, ref_cnt) in enumerate(refs):
                assert np.array_equal(c[h * S:(h + 1) * S], ref_cnt.astype(np.int32)), (flags, run, h)
                for s in range(S):
                    a0, k = int(off[s]), int(c[h * S + s])
                    assert np.array_equal(o[h * N + a0:h * N + a0 + k], ref_out[a0:a0 + k]), \
                        (flags, run, h, s)
        plan.close()


# ------------------------------------------------------------ data errors
def test_data_errors_reported_per_set():
    good = synth.uniform(10000, 20, seed=3)
    unsorted = good.copy()
    unsorted[[5000, 5001]] = unsorted[[5001, 5000]]  # distinct x: now descends
    rng_bad = good.copy()
    rng_bad[7000, 1] = 1.5
    nan_bad = good.copy()
    nan_bad[100, 0] = np.nan
    grid_bad = good.copy()
    grid_bad[3, 1] = np.float32(2.0 ** -40)
    boundary = good.copy()  # descent exactly at a tile boundary
    boundary[TILE, 0] = boundary[TILE - 1, 0] - np.float32(2.0 ** -20)
    sets = [good, unsorted, rng_bad, nan_bad, grid_bad, good, boundary]
    pts, off = synth.concat_sets(sets)
    out, cnt = gpu_batched(pts, off)
    assert cnt[1] == uh.UH_ERR_UNSORTED
    assert cnt[0] == len(oracle.upper_hull(good)) and cnt[5] == cnt[0]
    assert cnt[2] == uh.UH_ERR_RANGE
    assert cnt[3] == uh.UH_ERR_RANGE
    assert cnt[4] == uh.UH_ERR_GRID
    assert cnt[6] == uh.UH_ERR_UNSORTED
    # single-set entry point reports on the stream too
    c, _ = gpu_hull(boundary)
    assert c == uh.UH_ERR_UNSORTED
    c, _ = gpu_hull(grid_bad[:50])
    assert c == uh.UH_ERR_GRID


def test_sets_whose_points_are_all_eliminated():
    # NaN heights fail every elimination test, so whole tiles, and whole
    # merge workgroups, end up with no surviving point: the merges must
    # still write consistent (empty) hoods and report the error, and the
    # valid sets around them must be unaffected.
    good = synth.uniform(300000, 22, seed=4)
    sets = []
    for n in (2 * TILE, 600000):
        bad = synth.uniform(n, 22, seed=n)
        bad[:, 1] = np.nan
        sets += [good, bad]
    half = good.copy()
    half[150000:, 1] = np.nan  # a valid left half, an eliminated right half
    sets += [half, good]
    pts, off = synth.concat_sets(sets)
    out, cnt = gpu_batched(pts, off)
    ref = oracle.upper_hull(good)
    for s in (0, 2, 5):
        assert cnt[s] == len(ref)
        assert np.array_equal(out[off[s]:off[s] + cnt[s]], ref)
    assert cnt[1] == uh.UH_ERR_RANGE and cnt[3] == uh.UH_ERR_RANGE
    assert cnt[4] == uh.UH_ERR_RANGE


def test_autotune_picks_a_candidate_with_identical_results():
    sets = [synth.uniform(150000, 20, seed=21), synth.arc(90001, 20, 4, seed=22),
            synth.uniform(777, 20, seed=23)]
    pts, off = synth.concat_sets(sets)
    cfg, ms = uh.upper_hull_autotune(_dev(pts), off, reps=2)
    assert cfg["strip"] in (8, 16, 32) and cfg["fan_in"] in (16, 32, 64, 128, 256)
    assert cfg["flags"] == 0 and ms > 0
    out, cnt = gpu_batched(pts, off, strip=cfg["strip"], fan_in=cfg["fan_in"])
    assert_batched_equal(pts, off, out, cnt)
    best = uh.upper_hull_config()
    assert uh.load_library().upper_hull_autotune(
        None, off.ctypes.data, len(off) - 1, 0, 0, ctypes.byref(best), None,
        None) == uh.UH_ERR_ARG  # reps < 1


def test_read_reference_times_a_read_and_checks_its_arguments():
    pts = _dev(synth.uniform(1 << 20, 20, seed=31))
    ms = uh.upper_hull_read_reference(pts, reps=3)
    assert 0 < ms < 100
    lib, out = uh.load_library(), ctypes.c_float(-1)
    base = pts.data_ptr()
    assert lib.upper_hull_read_reference(base + 8, 100, 1, ctypes.byref(out), None) \
        == uh.UH_ERR_ARG  # not 16-byte aligned
    assert lib.upper_hull_read_reference(base, 1, 1, ctypes.byref(out), None) == uh.UH_ERR_ARG
    assert lib.upper_hull_read_reference(base, 100, 0, ctypes.byref(out), None) == uh.UH_ERR_ARG


def test_argument_errors():
    with pytest.raises(RuntimeError):
        uh.upper_hull_plan_create([0, 5, 3])
    with pytest.raises(RuntimeError):
        uh.upper_hull_plan_create([0, 10], strip=5)
    with pytest.raises(RuntimeError):
        uh.upper_hull_plan_create([0, 10], fan_in=3)


# ------------------------------------------------------------ bridge entry
def _hood_pts(rng, n, x0, x1, concave):
    xs = np.sort(rng.choice(np.arange(x0, x1), size=n, replace=False))
    if concave:
        mid = (x0 + x1) / 2
        ys = (200000 - ((xs - mid) ** 2) // max(1, (x1 - x0) // 64)
              + rng.integers(-2, 3, n)).astype(np.int64)
    else:
        ys = rng.integers(0, 1 << 18, n)
    ys = np.clip(ys, 0, (1 << 20) - 1)
    xy = synth.from_integers(xs, ys, 20)
    h = oracle.upper_hull(xy)
    return xy[h]


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_bridge_entry_point(lanes):
    rng = np.random.default_rng(lanes)
    for trial in range(60):
        concave = trial % 3 != 0
        n1, n2 = rng.integers(1, 3000, 2)
        P = _hood_pts(rng, int(n1), 0, 1 << 19, concave)
        Q = _hood_pts(rng, int(n2), 1 << 19, 1 << 20, concave)
        ab = uh.upper_hull_bridge(_dev(P), _dev(Q), lanes=lanes).cpu().numpy()
        union = np.concatenate([P, Q])
        h = oracle.upper_hull(union)
        a = int(np.sum(h < len(P))) - 1
        b = int(h[a + 1] - len(P))
        assert (int(ab[0]), int(ab[1])) == (a, b), trial
        if len(P) * len(Q) <= 400:
            Pi = [tuple(v) for v in (P.astype(np.float64) * 2 ** 20).astype(np.int64)]
            Qi = [tuple(v) for v in (Q.astype(np.float64) * 2 ** 20).astype(np.int64)]
            assert B.bridge(Pi, Qi) == (a, b)


def test_bridge_collinear_ties():
    P = np.array([[0, 0], [2, 4], [4, 6]], np.float32) / 16
    Q = np.array([[6, 8], [8, 10], [10, 10]], np.float32) / 16
    for lanes in (1, 2, 4, 8, 16, 32, 64):
        ab = uh.upper_hull_bridge(_dev(P), _dev(Q), lanes=lanes).cpu().numpy()
        assert list(ab) == [1, 1]


# ------------------------------------------------------------ predicate
def _near_collinear_triples(rng, m, G):
    k = 1 << G
    a = rng.integers(0, k, (m, 2))
    b = rng.integers(0, k, (m, 2))
    t = rng.random(m)
    c = np.rint(a + (b - a) * t[:, None]).astype(np.int64) + rng.integers(-1, 2, (m, 2))
    c = np.clip(c, 0, k - 1)
    to = lambda v: synth.from_integers(v[:, 0], v[:, 1], G)
    return to(a), to(b), to(c)


@pytest.mark.parametrize("G", [8, 20, 24, 27, 30])
def test_orient_signs_exact(G):
    rng = np.random.default_rng(G)
    a, b, c = _near_collinear_triples(rng, 200000, G)
    ref = oracle.orient_signs(a, b, c)
    s, fb = uh.upper_hull_orient(_dev(a), _dev(b), _dev(c))
    s2, fb2 = uh.upper_hull_orient(_dev(a), _dev(b), _dev(c), force_fallback=True)
    s, s2, fb, fb2 = (v.cpu().numpy() for v in (s, s2, fb, fb2))
    assert np.array_equal(s, ref)
    assert np.array_equal(s2, ref)
    assert np.all(fb2 == 1)


def test_orient_exhaustive_small_grid():
    g = [(x, y) for x in range(4) for y in range(4)]
    trip = np.array(list(itertools.product(g, g, g)), dtype=np.int64)  # 4096 triples
    to = lambda v: synth.from_integers(v[:, 0], v[:, 1], 2)
    a, b, c = to(trip[:, 0]), to(trip[:, 1]), to(trip[:, 2])
    ref = oracle.orient_signs(a, b, c)
    s, _ = uh.upper_hull_orient(_dev(a), _dev(b), _dev(c))
    assert np.array_equal(s.cpu().numpy(), ref)


# ------------------------------------------------------------ graphs
def test_graph_replay_matches_eager():
    sets = [synth.uniform(20000 + 37 * k, 20, seed=k) for k in range(6)]
    sets += [synth.arc(50000, 20, 4, seed=99)]
    pts, off = synth.concat_sets(sets)
    eager_out, eager_cnt = gpu_batched(pts, off)
    assert_batched_equal(pts, off, eager_out, eager_cnt)
    plan = uh.upper_hull_plan_create(off, flags=uh.UH_FLAG_GRAPH)
    d = _dev(pts)
    out = torch.zeros(len(pts), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(len(sets), dtype=torch.int32, device="cuda")
    for rep in range(4):
        out.fill_(-1)
        cnt.fill_(-1)
        plan.run(d, out, cnt)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work in between
        torch.cuda.synchronize()
        assert np.array_equal(cnt.cpu().numpy(), eager_cnt)
        o = out.cpu().numpy()
        for s in range(len(sets)):
            a, c = int(off[s]), int(eager_cnt[s])
            assert np.array_equal(o[a:a + c], eager_out[a:a + c]), (rep, s)
        del junk
    plan.close()


def test_default_fan_in_takes_the_fewest_passes():
    # the default fan-in is 256 for every plan shape: one large set (16384
    # tiles: 64 first-level items), many sets, a small set; an explicit
    # fan-in is kept
    for off in ([0, 1 << 24], np.arange(0, 4097 * 5000, 5000), [0, 1 << 18]):
        plan = uh.upper_hull_plan_create(off)
        assert plan.config["fan_in"] == 256
        plan.close()
    assert uh.upper_hull_plan_create([0, 100], fan_in=16).config["fan_in"] == 16


@pytest.mark.parametrize("n", [6000, 7000, 9000, 12000, 20000])
def test_large_merges_every_point_a_corner(n):
    # a strictly concave chain: every point is a corner and the last merge
    # holds all n of them: in LDS (n <= 6144), positions in LDS with the
    # hoods in the workspace (6144 < n <= 9216), or all in the workspace
    xy = concave_chain(130, G=24)[:n]
    c, idx = gpu_hull(xy)
    assert c == n and np.array_equal(idx, np.arange(n))
    # the same inside a batch, next to a set that is not concave
    pts, off = synth.concat_sets([synth.uniform(5000, 20, seed=n), xy, xy[: n // 3]])
    for fan_in in (0, 4):
        out, cnt = gpu_batched(pts, off, fan_in=fan_in)
        assert_batched_equal(pts, off, out, cnt)


def test_work_per_point_stays_bounded():
    # The paper's work-optimal variant (its conclusions): serial strip hoods,
    # then merges with fewer lanes than corners by multi-level bracketing:
    # O(n) work.  Orientation tests per point must not grow with n, even when
    # every point is a corner (the concave chain) or on a noisy arc.
    per = {}
    for name, make in (("concave", lambda n: concave_chain(130, G=24)[:n]),
                       ("arc", lambda n: synth.arc(n, 24, 4, seed=n))):
        for n in (5000, 20000) if name == "concave" else (1 << 16, 1 << 20):
            xy = make(n)
            off = np.array([0, len(xy)], np.int64)
            out, cnt, st = gpu_batched(xy, off, with_stats=True)
            assert_batched_equal(xy, off, out, cnt)
            per[(name, n)] = st[0, 0] / len(xy)
    assert per[("concave", 20000)] <= 1.25 * per[("concave", 5000)] + 0.5, per
    assert per[("arc", 1 << 20)] <= 1.25 * per[("arc", 1 << 16)] + 0.5, per
    assert max(per.values()) < 16, per  # measured: about 11.3 (concave), 3.5 to 5 (arc)


def test_batched_call_without_a_plan():
    sets = [synth.uniform(9000, 20, seed=91), np.zeros((0, 2), np.float32),
            synth.arc(5000, 20, 4, seed=92), synth.lattice_points(30, 8, seed=93)]
    pts, off = synth.concat_sets(sets)
    d = _dev(pts)
    for _ in range(2):  # the second call reuses the cached plan
        out, cnt = uh.upper_hull_batched(d, off)
        torch.cuda.synchronize()
        assert_batched_equal(pts, off, out.cpu().numpy(), cnt.cpu().numpy())
    stats = uh.new_stats(len(off) - 1)
    out, cnt = uh.upper_hull_batched(d, off, stats=stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    assert np.all(st[:, 1] <= st[:, 0])
