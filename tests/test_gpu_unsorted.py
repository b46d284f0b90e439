"""Points in any order (UH_FLAG_UNSORTED): the device sort and the hoods
behind it, against the oracle.

The plan sorts every set by x on the device (stable, so ties keep input
order) and maps the corners back to input indices.  The sorted copy and the
permutation are checked against a stable host sort, and every hood against
``oracle.unsorted_hull``.
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


def _shuffled_sets(seed, sizes=None):
    rng = np.random.default_rng(seed)
    sets = []
    kinds = sizes or [0, 1, 3, 40, 4095, 4096, 4097, 9000, 30000]
    for k, n in enumerate(kinds):
        if n == 0:
            xy = np.zeros((0, 2), np.float32)
        elif k % 4 == 0:
            xy = synth.uniform(n, 20, seed=seed + k)
        elif k % 4 == 1:
            xy = synth.arc(n, 20, 4, seed=seed + k)
        elif k % 4 == 2:
            xy = synth.lattice_points(n, 16, seed=seed + k)  # duplicates and equal x
        else:
            xy = synth.uniform_iid(n, 27, seed=seed + k)    # runs of equal x
        sets.append(xy[rng.permutation(len(xy))])
    return sets


def run_plan(sets, flags, strip=0, fan_in=0):
    pts, off = synth.concat_sets(sets)
    H = 2 if flags & uh.UH_FLAG_BOTH_HOODS else 1
    N, S = int(off[-1]), len(off) - 1
    plan = uh.upper_hull_plan_create(off, strip=strip, fan_in=fan_in, flags=flags)
    out = torch.full((max(H * N, 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((H * S,), -7, dtype=torch.int32, device="cuda")
    plan.run(_dev(pts), out, cnt)
    torch.cuda.synchronize()
    return plan, pts, off, out.cpu().numpy(), cnt.cpu().numpy()


def check_hoods(sets, off, out, cnt, both):
    N, S = int(off[-1]), len(off) - 1
    for s, xy in enumerate(sets):
        for half, hood in enumerate(("upper", "lower")[:2 if both else 1]):
            rc, ref = oracle.unsorted_hull(xy, hood)
            c = int(cnt[half * S + s])
            assert (rc if rc else len(ref)) == c, (s, hood, c, len(ref))
            a = half * N + int(off[s])
            assert np.array_equal(out[a:a + c], ref), (s, hood)


def test_sort_matches_a_stable_host_sort():
    sets = _shuffled_sets(1)
    plan, pts, off, out, cnt = run_plan(sets, uh.UH_FLAG_UNSORTED)
    xy, perm = plan.sorted_view()
    for s, a in enumerate(sets):
        lo, hi = int(off[s]), int(off[s + 1])
        order = oracle.sort_order(a)
        assert np.array_equal(perm[lo:hi], order), s
        assert np.array_equal(xy[lo:hi].view(np.uint32), a[order].view(np.uint32)), s
    plan.close()


@pytest.mark.parametrize("strip", [8, 16, 32])
def test_upper_hood_of_shuffled_sets(strip):
    sets = _shuffled_sets(10 + strip)
    plan, pts, off, out, cnt = run_plan(sets, uh.UH_FLAG_UNSORTED, strip=strip)
    check_hoods(sets, off, out, cnt, both=False)
    plan.close()


def test_both_hoods_of_shuffled_sets():
    sets = _shuffled_sets(30)
    plan, pts, off, out, cnt = run_plan(sets, uh.UH_FLAG_UNSORTED | uh.UH_FLAG_BOTH_HOODS)
    check_hoods(sets, off, out, cnt, both=True)
    plan.close()


def test_sorted_input_gives_the_plain_result():
    sets = [synth.uniform(50000, 20, seed=4), synth.arc(20000, 20, 4, seed=5)]
    plan, pts, off, out, cnt = run_plan(sets, uh.UH_FLAG_UNSORTED)
    ref_out, ref_cnt = oracle.upper_hull_batched(pts, off)
    assert np.array_equal(cnt, ref_cnt.astype(np.int32))
    for s in range(len(sets)):
        a = int(off[s])
        assert np.array_equal(out[a:a + cnt[s]], ref_out[a:a + cnt[s]])
    plan.close()


def test_reversed_and_many_small_sets():
    sets = [synth.uniform(n, 20, seed=n)[::-1].copy() for n in (1, 2, 5, 64, 65, 700, 4100)]
    sets += _shuffled_sets(50, sizes=[7, 0, 33, 2048, 6000])
    plan, pts, off, out, cnt = run_plan(sets, uh.UH_FLAG_UNSORTED | uh.UH_FLAG_BOTH_HOODS,
                                        fan_in=16)
    check_hoods(sets, off, out, cnt, both=True)
    plan.close()


def test_data_error_in_unsorted_input():
    good = _shuffled_sets(60, sizes=[5000])[0]
    bad = good.copy()
    bad[123, 1] = 2.0  # y out of range
    plan, pts, off, out, cnt = run_plan([good, bad], uh.UH_FLAG_UNSORTED)
    assert cnt[0] > 0 and cnt[1] == uh.UH_ERR_RANGE
    plan.close()


def test_graph_replays_of_an_unsorted_plan():
    sets = _shuffled_sets(70, sizes=[3000, 12000, 1])
    pts, off = synth.concat_sets(sets)
    N, S = int(off[-1]), len(off) - 1
    plan = uh.upper_hull_plan_create(off, flags=uh.UH_FLAG_UNSORTED | uh.UH_FLAG_GRAPH)
    d = _dev(pts)
    out = torch.zeros(N, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(S, dtype=torch.int32, device="cuda")
    for _ in range(3):
        out.fill_(-5)
        cnt.fill_(-5)
        torch.cuda.synchronize()
        plan.run(d, out, cnt)
        torch.cuda.synchronize()
        check_hoods(sets, off, out.cpu().numpy(), cnt.cpu().numpy(), both=False)
    plan.close()


def test_sorted_view_needs_an_unsorted_plan():
    plan = uh.upper_hull_plan_create([0, 10])
    with pytest.raises(RuntimeError):
        plan.sorted_view()
    plan.close()


def test_unsorted_edge_values():
    good = _shuffled_sets(80, sizes=[3000])[0]
    # NaN and negative x are data errors wherever the sort puts them
    for v in (np.nan, -0.25, 1.5):
        bad = good.copy()
        bad[17, 0] = v
        plan, pts, off, out, cnt = run_plan([bad], uh.UH_FLAG_UNSORTED)
        assert cnt[0] == uh.UH_ERR_RANGE, v
        plan.close()
    # -0.0 is the same x as +0.0 (and sorts with it, in input order)
    z = good.copy()
    z[:40, 0] = 0.0
    z[5:40:3, 0] = -0.0
    plan, pts, off, out, cnt = run_plan([z], uh.UH_FLAG_UNSORTED | uh.UH_FLAG_BOTH_HOODS)
    check_hoods([z], off, out, cnt, both=True)
    plan.close()
